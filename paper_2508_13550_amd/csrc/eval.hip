// Evaluation of plans (paper §8, Algorithm 2 after the traversal):
//   gather weights -> [PP near field on a side stream] -> P2M (eq. PC proxy
//   weights of the leaves) -> M2M by levels (eq. upwardpass2, FP64 MFMA) ->
//   PC near field and CP+CC far field (tile engine) -> join -> per leaf: L2L
//   down its ancestors (eq. downward_2, two 1-D passes per level), L2P
//   (eq. downward_1), near field and the scatter to the caller's order.
//
// Every launch is a batch of up to kMaxBatch requests (a request is a plan
// with its own workspace, weights and output); block b works for the request
// r with prefix[r] <= b < prefix[r+1].  A single csfmm_eval is a batch of
// one, and every block's arithmetic depends only on its own request, so a
// request's result does not depend on what it is batched with.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <utility>

#include "common.h"
#include "dev_util.h"

namespace csfmm {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kMaxP1 = kMaxDegree + 1;

__device__ __forceinline__ double cheb(int k, int p) { return cos(double(k) * kPi / double(p)); }

__device__ __forceinline__ void locate(const Batch& b, int& r, int& local) {
    batch_locate(b, xcd_logical_block(blockIdx.x, gridDim.x), r, local);
}

// Orders a wave's LDS stores before its later loads (and the reverse) across
// its lanes; for LDS that one wave owns.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// e1: ws[k] = w[perm[k]]   (256 sorted sources per block)
__global__ __launch_bounds__(256) void k_gather_w(Batch b) {
    int r, local;
    locate(b, r, local);
    const ReqView& V = *b.v[r];
    const int64_t k = int64_t(local) * 256 + threadIdx.x;
    if (k < V.ns) V.ws[k] = b.w[r][V.s_perm[k]];
}

// psi = 0 for the request's output components (256 values per block)
__global__ __launch_bounds__(256) void k_zero_psi(Batch b) {
    int r, local;
    locate(b, r, local);
    const ReqView& V = *b.v[r];
    const int64_t k = int64_t(local) * 256 + threadIdx.x;
    if (k < int64_t(b.vd[r]) * V.psi_stride) V.psi[k] = 0.0;
}

__device__ __forceinline__ void cheb_setup(int p, double* s, double* beta) {
    for (int k = threadIdx.x; k <= p; k += blockDim.x) {
        s[k] = cheb(k, p);
        double bb = (k & 1) ? -1.0 : 1.0;
        if (k == 0 || k == p) bb *= 0.5;
        beta[k] = bb;
    }
}

// FP64 reciprocal: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Barycentric row L_0..L_{P1-1} at x in registers (§4, eq. barycentric);
// an exact node hit gives the Kronecker delta.
template <int P1>
__device__ __forceinline__ void bary_regs(const double* s, const double* beta, double x,
                                          double (&L)[P1]) {
    int hit = -1;
    double den = 0.0;
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        const double d = x - s[k];
        hit = (d == 0.0) ? k : hit;
        L[k] = beta[k] * rcp64(d);
        den += L[k];
    }
    const double inv = rcp64(den);
#pragma unroll
    for (int k = 0; k < P1; ++k) L[k] = hit >= 0 ? (k == hit ? 1.0 : 0.0) : L[k] * inv;
}

// e2 P2M: wbar_k(leaf) = sum_j L_k1(u_j) L_k2(v_j) w_j (eq. PC, §6), one wave
// per source leaf (p2m_waves per block: blocks of one wave made the launch
// wait on the rate at which workgroups are dispatched).  Each lane builds the
// rows of one point in registers and stores L1 and w L2 in its wave's LDS;
// then, as a matrix product over the points,
//   Wbar[k1][k2] = sum_j L1[j][k1] (w_j L2[j][k2]),
// runs on FP64 MFMA 16x16x4 (16-wide proxy-index tiles, 4 points per step).
template <int P1>
constexpr int p2m_waves() {
    return P1 <= 12 ? 4 : 2;  // the waves' LDS within 64 KB
}
template <int P1>
__global__ __launch_bounds__(64 * p2m_waves<P1>()) void k_p2m(Batch b) {
    constexpr int NT = (P1 + 15) / 16;
    constexpr int PW = p2m_waves<P1>();
    __shared__ double s[P1], beta[P1];
    __shared__ double Luw[PW][64][P1];
    __shared__ double Lww[PW][64][P1];
    const int lane = threadIdx.x & 63;
    int r, local;
    locate(b, r, local);
    const ReqView& V = *b.v[r];
    cheb_setup(P1 - 1, s, beta);
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    const int leaf = PW * local + wave;
    if (leaf >= V.nleaves_s) return;  // the whole wave leaves
    double(&Lu)[64][P1] = Luw[wave];
    double(&Lw)[64][P1] = Lww[wave];
    const int c = V.s_leaves[leaf];
    const int bgn = V.s_begin[c], m = V.s_count[c];
    const int KS = V.KS;
    double4_t acc[NT][NT];
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    const int kq = lane >> 4, l16 = lane & 15;
    for (int j0 = 0; j0 < m; j0 += 64) {
        const int j = j0 + lane;
        double L1[P1], L2[P1];
        double wj = 0.0;
        if (j < m) {
            bary_regs<P1>(s, beta, V.s_u[bgn + j], L1);
            bary_regs<P1>(s, beta, V.s_v[bgn + j], L2);
            wj = V.ws[bgn + j];
        } else {
#pragma unroll
            for (int k = 0; k < P1; ++k) L1[k] = L2[k] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < P1; ++k) {
            Lu[lane][k] = L1[k];
            Lw[lane][k] = wj * L2[k];
        }
        wave_lds_sync();
        const int steps = min(64, m - j0);
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int tj = 0; tj < NT; ++tj) {
                const int ka = ti * 16 + l16, kb = tj * 16 + l16;
                for (int kk = 0; kk < steps; kk += 4) {
                    const double av = ka < P1 ? Lu[kk + kq][ka] : 0.0;
                    const double bv = kb < P1 ? Lw[kk + kq][kb] : 0.0;
                    acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ti][tj], 0, 0, 0);
                }
            }
        wave_lds_sync();
    }
    double* wb = V.wbar + int64_t(c) * KS;
#pragma unroll
    for (int ti = 0; ti < NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k1 = ti * 16 + kq + 4 * i, k2 = tj * 16 + l16;
                if (k1 < P1 && k2 < P1) wb[k1 * P1 + k2] = acc[ti][tj][i];
            }
    for (int k = P1 * P1 + lane; k < KS; k += 64) wb[k] = 0.0;
}

// e3 M2M (eq. upwardpass2) at one tree level as batched small GEMMs on FP64
// MFMA (v_mfma_f64_16x16x4f64); request r's parents at the level are
// parents[a0[r] .. a0[r] + a1[r]).  Row = parent P; A = wbar of its 4
// children (4*KS contiguous values), B = bm2m [4KS][nb1], C = wbar(P).  One
// block per (16-row tile, 16-column tile); wave q takes the K-slice of child q
// (split-K) and the four partial tiles are summed in LDS.
// MFMA f64 16x16x4 operand layout: lane l holds A[l%16][l/16], B[l/16][l%16]
// and D[l/16 + 4*i][l%16], i = 0..3 (checked with a one-hot probe).
// Operand loads are issued kAhead MFMA steps ahead of their use.
__global__ __launch_bounds__(256) void k_m2m(Batch b) {
    constexpr int kAhead = 16;
    __shared__ double4_t part[3][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int r, local;
    locate(b, r, local);
    const ReqView& V = *b.v[r];
    const int32_t* rows = V.s_parents + b.a0[r];
    const int np = b.a1[r];
    const int KS = V.KS;
    const int nb = V.nb1;
    const int ntiles = nb / 16;
    const int rt = local / ntiles, tile = local % ntiles;
    const int r0 = rt * 16;
    if (r0 >= np) return;  // uniform over the block
    const int koff = wave * KS;  // K-slice of this wave: child `wave`
    const int ra = r0 + (lane & 15);
    const double* arow = ra < np ? V.wbar + int64_t(V.s_child0[rows[ra]]) * KS + koff : nullptr;
    const int kq = lane >> 4;
    const double* bcol = V.bm2m + int64_t(koff) * nb + tile * 16 + (lane & 15);
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < KS; kk += 4 * kAhead) {
        double av[kAhead], bv[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int k = kk + 4 * u + kq;
            const bool in = k < KS;
            av[u] = (arow && in) ? arow[k] : 0.0;
            bv[u] = in ? bcol[int64_t(k) * nb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (kk + 4 * u < KS)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    if (wave > 0) part[wave - 1][lane] = acc;
    __syncthreads();
    if (wave > 0) return;
    acc += part[0][lane];
    acc += part[1][lane];
    acc += part[2][lane];
    const int col = tile * 16 + (lane & 15);
    if (col < KS) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = r0 + kq + 4 * i;
            if (rr < np) V.wbar[int64_t(rows[rr]) * KS + col] = acc[i];
        }
    }
}

// The same product for levels of many parents (kM2mRowsMin or more), where
// the tiles above would read each parent's children once per column tile:
// one block per 32 parents and all nb1 columns: wave w takes the rows
// 16 (w >> 1) .. +15 and every other 16-column tile from w & 1.  K runs in
// chunks of 16: the block stages the chunk's A rows (32 x 16) and B rows
// (16 x nb1) in LDS, each thread holding its share of the next chunk in
// registers meanwhile, so the children's weights are read from HBM once and
// B (shared by every block) from L2 once a chunk.
// Measured on the 1/|x-y| workload's deepest level (24,576 parents, p = 10):
// that level 208 -> 78 us, the eval 8.48 -> 8.41 ms in FP64 and 4.41 -> 4.29
// ms in the FP32 form; on levels of a few thousand parents the 32-parent
// blocks leave most CUs idle, and the tiles above are faster.
constexpr int kM2mRows = 32;
constexpr int kM2mRowsMin = 8192;
constexpr int kM2mMaxNb = ((kMaxP1 * kMaxP1 + 3) / 4 * 4 + 15) / 16 * 16;
constexpr int kM2mMaxTiles = kM2mMaxNb / 16;
// LDS row stride of the B chunk (doubles): rows 1 and 3 of an MFMA step fall
// 128 bytes off rows 0 and 2, so a step's 64 lanes read in two conflict-free
// passes
__host__ __device__ constexpr int m2m_b_stride(int nb) { return nb % 32 == 0 ? nb + 16 : nb; }
__global__ __launch_bounds__(256) void k_m2m_rows(Batch b) {
    constexpr int kTW = (kM2mMaxTiles + 1) / 2;  // column tiles per wave
    __shared__ double As[kM2mRows][17];  // a row pad of one: an MFMA step's 16 rows in distinct banks
    __shared__ double Bs[16 * m2m_b_stride(kM2mMaxNb)];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int r, local;
    locate(b, r, local);
    const ReqView& V = *b.v[r];
    const int32_t* rows = V.s_parents + b.a0[r];
    const int np = b.a1[r];
    const int KS = V.KS, nb = V.nb1, K4 = 4 * KS;
    const int ntiles = nb / 16, SB = m2m_b_stride(nb);
    const int r0 = local * kM2mRows;
    if (r0 >= np) return;  // uniform over the block
    // A staging: thread t loads row t / 8, values 2 (t % 8) and 2 (t % 8) + 1
    const int ar = tid >> 3, ak = 2 * (tid & 7);
    const double* arow =
        r0 + ar < np ? V.wbar + int64_t(V.s_child0[rows[r0 + ar]]) * KS : nullptr;
    // B staging: thread t loads row t / 16 of the chunk, columns t % 16 + 16 j
    const int br = tid >> 4, bc = tid & 15;
    double a0 = 0.0, a1 = 0.0, bv[kM2mMaxTiles];
    auto fetch = [&](int kc) {
        if (arow) {
            a0 = arow[kc + ak];
            a1 = arow[kc + ak + 1];
        }
        const double* bsrc = V.bm2m + int64_t(kc + br) * nb + bc;
#pragma unroll
        for (int j = 0; j < kM2mMaxTiles; ++j) bv[j] = j < ntiles ? bsrc[16 * j] : 0.0;
    };
    const int rs = wave >> 1, ch = wave & 1;
    const int l16 = lane & 15, kq = lane >> 4;
    double4_t acc[kTW];
#pragma unroll
    for (int i = 0; i < kTW; ++i) acc[i] = double4_t{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int kc = 0; kc < K4; kc += 16) {
        __syncthreads();  // the previous chunk is consumed
        As[ar][ak] = a0;
        As[ar][ak + 1] = a1;
#pragma unroll
        for (int j = 0; j < kM2mMaxTiles; ++j)
            if (j < ntiles) Bs[br * SB + bc + 16 * j] = bv[j];
        __syncthreads();
        if (kc + 16 < K4) fetch(kc + 16);  // in flight while this chunk multiplies
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const double av = As[16 * rs + l16][4 * st + kq];
            const double* brow = Bs + (4 * st + kq) * SB + l16;
#pragma unroll
            for (int i = 0; i < kTW; ++i) {
                const int t = ch + 2 * i;
                if (t < ntiles) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, brow[16 * t], acc[i], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kTW; ++i) {
        const int col = 16 * (ch + 2 * i) + l16;
        if (ch + 2 * i < ntiles && col < KS) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rr = r0 + 16 * rs + kq + 4 * q;
                if (rr < np) V.wbar[int64_t(rows[rr]) * KS + col] = acc[i][q];
            }
        }
    }
}

// e3 M2M (eq. upwardpass2) of shrunk plans, one level: every parent has its
// own operator (the children's boxes differ), so instead of one GEMM a wave
// applies it to one parent (four per block) as two 1-D passes per child with
// the child's own factors A_xi, A_eta (A[m][k]: the parent's polynomial k at
// the child's node m):
//   t[k1][m2] = sum_m1 A_xi[m1][k1] wbar_c[m1][m2],
//   wbar_P[k1][k2] += sum_m2 A_eta[m2][k2] t[k1][m2].
template <int P1>
__global__ __launch_bounds__(256) void k_m2m_cells(Batch b) {
    constexpr int K = P1 * P1;
    constexpr int kRegs = (K + 63) / 64;
    __shared__ double wlds[4][4][K];  // per wave: child weights, t, A_xi, A_eta
    int r, local;
    locate(b, r, local);
    const ReqView& V = *b.v[r];
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    const int idx = 4 * local + wave;
    if (idx >= b.a1[r]) return;  // the whole wave leaves
    const int par = V.s_parents[b.a0[r] + idx];
    const int ch0 = V.s_child0[par];
    const int KS = V.KS;
    double* wc = wlds[wave][0];
    double* tb = wlds[wave][1];
    double* ax = wlds[wave][2];
    double* ay = wlds[wave][3];
    double out[kRegs];
#pragma unroll
    for (int i = 0; i < kRegs; ++i) out[i] = 0.0;
    for (int q = 0; q < 4; ++q) {
        const int c = ch0 + q;
        const double* src = V.wbar + int64_t(c) * KS;
        const double* op = V.s_ops + int64_t(c) * 2 * K;
        for (int k = lane; k < K; k += 64) {
            wc[k] = src[k];
            ax[k] = op[k];
            ay[k] = op[K + k];
        }
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < kRegs; ++i) {
            const int e = lane + 64 * i;
            if (e < K) {
                const int k1 = e / P1, m2 = e % P1;
                double t = 0.0;
#pragma unroll
                for (int m1 = 0; m1 < P1; ++m1) t = fma(ax[m1 * P1 + k1], wc[m1 * P1 + m2], t);
                tb[e] = t;
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < kRegs; ++i) {
            const int e = lane + 64 * i;
            if (e < K) {
                const int k1 = e / P1, k2 = e % P1;
                double t = out[i];
#pragma unroll
                for (int m2 = 0; m2 < P1; ++m2) t = fma(ay[m2 * P1 + k2], tb[k1 * P1 + m2], t);
                out[i] = t;
            }
        }
        wave_lds_sync();
    }
    double* wb = V.wbar + int64_t(par) * KS;
#pragma unroll
    for (int i = 0; i < kRegs; ++i) {
        const int e = lane + 64 * i;
        if (e < K) wb[e] = out[i];
    }
    for (int k = K + lane; k < KS; k += 64) wb[k] = 0.0;
}

// e6-e8: L2L (eq. downward_2) down the leaf's ancestors, L2P (eq.
// downward_1) at the leaf, near field (PP, PC) and scatter to the caller's
// order; one target leaf per wave (four per block: blocks of one wave made the
// launch wait on the rate at which workgroups are dispatched), one point per
// lane.
// The parent-to-child operator of eq. downward_2 is the Kronecker product of
// two 1-D factors A_bi (n1, m1) and A_bj (n2, m2), child q = 2 bi + bj, so
// each level is two 1-D passes over the (p+1) x (p+1) proxy array:
//   t[n1][m2] = sum_m1 A_bi[n1][m1] psi[m1][m2],
//   psi'[n1][n2] = own[n1][n2] + sum_m2 A_bj[n2][m2] t[n1][m2],
// starting from the root's own proxy potential.  The levels the block's
// leaves share (their common ancestors: all but the last for four sibling
// leaves) are computed once, by the whole block, one element a thread; each
// wave then walks the rest of its leaf's path (a table built with the plan;
// upper levels recomputed per block instead of one launch per level), loading
// each level's own proxy potential one level ahead.  Both follow the same
// order of operations, so the result does not depend on how the chain was
// split.  The accumulated proxy potential of the leaf is stored back into psi
// (no other wave reads a leaf's psi).
// The occupancy hint holds the scalar kernels of degree p <= 6 at 80 VGPRs
// (6 waves per SIMD, no spills): 6,144 leaves then fit the device at once.
template <int VD, int P1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(VD == 1 && P1 <= 7 ? 6 : 1))) void k_l2p(Batch b) {
    constexpr int K = P1 * P1;
    constexpr int kRegs = (VD * K + 63) / 64;  // elements per lane in the 1-D passes
    __shared__ double s[P1], beta[P1];
    __shared__ double A1[2][P1][P1];
    __shared__ double psw[4][VD][K], tbw[4][VD][K];
    __shared__ double opw[4][2][K];  // shrunk plans: the child's own factors
    __shared__ int ancw[4][kAncStride];
    __shared__ int ncom, wref;
    int r, local;
    locate(b, r, local);
    const ReqView& V = *b.v[r];
    double* out = b.out[r];
    // nodes, weights and 1-D factors, shared by the block's waves (one request)
    cheb_setup(P1 - 1, s, beta);
    for (int k = threadIdx.x; k < 2 * K; k += blockDim.x) (&A1[0][0][0])[k] = V.lag1d[k];
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    const int leaf = 4 * local + wave;
    const int tid = threadIdx.x & 63;
    int c = 0, bgn = 0, m = 0;
    if (leaf < V.nleaves_t) {
        c = V.t_leaves[leaf];
        bgn = V.t_begin[c];
        m = V.t_count[c];
    }
    const bool has = m > 0;  // uniform over the wave
    double(&ps)[VD][K] = psw[wave];
    double(&tb)[VD][K] = tbw[wave];
    int* anc = ancw[wave];
    const int KS = V.KS;
    if (has) {
        const int32_t* path = V.t_leaf_anc + int64_t(leaf) * kAncStride;
        for (int k = tid; k < kAncStride; k += 64) anc[k] = path[k];
    } else if (tid == 0) {
        anc[0] = 0;  // no path
    }
    __syncthreads();
    // the leading cells common to the paths of the block's leaves
    if (threadIdx.x == 0) {
        int lim = kAncStride, w0 = -1;
        for (int w = 0; w < 4; ++w)
            if (ancw[w][0] > 0) {
                lim = min(lim, ancw[w][0]);
                if (w0 < 0) w0 = w;
            }
        int n = 0;
        if (w0 >= 0)
            for (int l = 1; l <= lim; ++l) {
                bool same = true;
                for (int w = 0; w < 4; ++w)
                    if (ancw[w][0] > 0 && ancw[w][l] != ancw[w0][l]) same = false;
                if (!same) break;
                n = l;
            }
        ncom = n;
        wref = w0;
    }
    __syncthreads();
    const int nc = ncom;
    const int na = anc[0];  // anc[1] is the root, anc[na] the leaf
    auto own_at = [&](int cell, int k) {
        return V.psi[(k / K) * V.psi_stride + int64_t(cell) * KS + k % K];
    };
    // own proxy potential of a cell, this thread's elements (k = tid + 64 i)
    auto load_own = [&](int cell, double (&dst)[kRegs]) {
#pragma unroll
        for (int i = 0; i < kRegs; ++i) {
            const int k = tid + 64 * i;
            dst[i] = k < VD * K ? own_at(cell, k) : 0.0;
        }
    };
    double cur[kRegs], nxt[kRegs];
    const int l0 = nc >= 1 ? nc : 1;  // the wave's path goes on from its cell l0
    // the wave's first own level after the shared ones, in flight meanwhile
    if (has && na >= l0 + 1) load_own(anc[l0 + 1], nxt);
    if (nc >= 1) {
        // the shared levels, block-wide, in wave 0's arrays; each level's own
        // proxy potential is loaded one level ahead
        constexpr int kB = (VD * K + 255) / 256;
        const int* ac = ancw[wref];
        double(&bp)[VD][K] = psw[0];
        double(&bt)[VD][K] = tbw[0];
        double bown[kB];
        for (int k = threadIdx.x; k < VD * K; k += blockDim.x) bp[k / K][k % K] = own_at(ac[1], k);
        auto load_bown = [&](int cell) {
#pragma unroll
            for (int i = 0; i < kB; ++i) {
                const int k = int(threadIdx.x) + 256 * i;
                bown[i] = k < VD * K ? own_at(cell, k) : 0.0;
            }
        };
        if (nc >= 2) load_bown(ac[2]);
        __syncthreads();
        for (int l = 2; l <= nc; ++l) {
            const int ch = ac[l], par = ac[l - 1];
            const int q = ch - V.t_child0[par];
            const double* Ax = &A1[q >> 1][0][0];
            const double* Ay = &A1[q & 1][0][0];
            if (V.t_ops) {
                const double* src = V.t_ops + int64_t(ch) * 2 * K;
                for (int k = threadIdx.x; k < 2 * K; k += blockDim.x) (&opw[0][0][0])[k] = src[k];
                __syncthreads();
                Ax = &opw[0][0][0];
                Ay = &opw[0][1][0];
            }
            for (int k = threadIdx.x; k < VD * K; k += blockDim.x) {
                const int d = k / K, e = k % K, n1 = e / P1, m2 = e % P1;
                double t = 0.0;
#pragma unroll
                for (int m1 = 0; m1 < P1; ++m1) t = fma(Ax[n1 * P1 + m1], bp[d][m1 * P1 + m2], t);
                bt[d][e] = t;
            }
            __syncthreads();
            double own[kB];
#pragma unroll
            for (int i = 0; i < kB; ++i) own[i] = bown[i];
            if (l < nc) load_bown(ac[l + 1]);
#pragma unroll
            for (int i = 0; i < kB; ++i) {
                const int k = int(threadIdx.x) + 256 * i;
                if (k < VD * K) {
                    const int d = k / K, e = k % K, n1 = e / P1, n2 = e % P1;
                    double t = own[i];
#pragma unroll
                    for (int m2 = 0; m2 < P1; ++m2) t = fma(Ay[n2 * P1 + m2], bt[d][n1 * P1 + m2], t);
                    bp[d][e] = t;
                }
            }
            __syncthreads();
        }
        if (has && wave != 0)
            for (int k = tid; k < VD * K; k += 64) ps[k / K][k % K] = bp[k / K][k % K];
        __syncthreads();  // before wave 0 goes on in its arrays
    }
    if (!has) return;  // the whole wave leaves (no block barrier after this)
    if (nc == 0) {
        load_own(anc[1], cur);
#pragma unroll
        for (int i = 0; i < kRegs; ++i) {
            const int k = tid + 64 * i;
            if (k < VD * K) ps[k / K][k % K] = cur[i];
        }
    }
    wave_lds_sync();
    for (int l = l0 + 1; l <= na; ++l) {
        const int ch = anc[l], par = anc[l - 1];
        const int q = ch - V.t_child0[par];
        const int bi = q >> 1, bj = q & 1;
        // the 1-D factors of this level: fixed by the child's quadrant, or the
        // child's own (shrunk boxes)
        const double* Ax = &A1[bi][0][0];
        const double* Ay = &A1[bj][0][0];
        if (V.t_ops) {
            const double* src = V.t_ops + int64_t(ch) * 2 * K;
            for (int k = tid; k < 2 * K; k += 64) (&opw[wave][0][0])[k] = src[k];
            wave_lds_sync();
            Ax = &opw[wave][0][0];
            Ay = &opw[wave][1][0];
        }
#pragma unroll
        for (int i = 0; i < kRegs; ++i) cur[i] = nxt[i];
        if (l < na) load_own(anc[l + 1], nxt);  // one level ahead
#pragma unroll
        for (int i = 0; i < kRegs; ++i) {
            const int k = tid + 64 * i;
            if (k < VD * K) {
                const int d = k / K, e = k % K, n1 = e / P1, m2 = e % P1;
                double t = 0.0;
#pragma unroll
                for (int m1 = 0; m1 < P1; ++m1) t = fma(Ax[n1 * P1 + m1], ps[d][m1 * P1 + m2], t);
                tb[d][e] = t;
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < kRegs; ++i) {
            const int k = tid + 64 * i;
            if (k < VD * K) {
                const int d = k / K, e = k % K, n1 = e / P1, n2 = e % P1;
                double t = cur[i];
#pragma unroll
                for (int m2 = 0; m2 < P1; ++m2) t = fma(Ay[n2 * P1 + m2], tb[d][n1 * P1 + m2], t);
                ps[d][e] = t;
            }
        }
        wave_lds_sync();
    }
    for (int k = tid; k < K; k += 64)
#pragma unroll
        for (int d = 0; d < VD; ++d) V.psi[d * V.psi_stride + int64_t(c) * KS + k] = ps[d][k];
    for (int j0 = 0; j0 < m; j0 += 64) {
        const int jj = j0 + tid;
        if (jj >= m) continue;
        const int j = bgn + jj;
        double L1[P1], L2[P1];
        bary_regs<P1>(s, beta, V.t_u[j], L1);
        bary_regs<P1>(s, beta, V.t_v[j], L2);
        double acc[VD];
#pragma unroll
        for (int d = 0; d < VD; ++d) acc[d] = 0.0;
#pragma unroll 1
        for (int n1 = 0; n1 < P1; ++n1) {
            double inner[VD];
#pragma unroll
            for (int d = 0; d < VD; ++d) inner[d] = 0.0;
#pragma unroll
            for (int n2 = 0; n2 < P1; ++n2)
#pragma unroll
                for (int d = 0; d < VD; ++d) inner[d] = fma(ps[d][n1 * P1 + n2], L2[n2], inner[d]);
#pragma unroll
            for (int d = 0; d < VD; ++d) acc[d] = fma(L1[n1], inner[d], acc[d]);
        }
        const int64_t o = V.t_perm[j];
#pragma unroll
        for (int d = 0; d < VD; ++d)
            out[o * VD + d] = (V.phinear[d * V.nt + j] + V.phipc[d * V.nt + j]) + acc[d];
    }
}

// Degrees p = 1..16 as P1 = p + 1 template arguments.
#define CSFMM_P1_CASES(X) \
    X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17)

__global__ void k_scatter_near(const double* __restrict__ near, const double* __restrict__ pc,
                               int64_t nt, int vd, const int32_t* __restrict__ perm,
                               double* __restrict__ out) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const int64_t o = perm[k];
    for (int d = 0; d < vd; ++d) out[o * vd + d] = near[d * nt + k] + pc[d * nt + k];
}

// *p = v (a fill kernel rather than a memset node)
__global__ void k_set_i32(int32_t* p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Writes a request view to device memory (kernel argument instead of a copy,
// so that it is ordered on the caller's stream only).
__global__ void k_set_view(ReqView* dst, ReqView v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

inline unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }

using Timing = csfmm_plan_s::Timing;

// Adds the stage times of a finished slot to the sums.  Events of a slot:
// [0..4] on the eval stream (start, after P2M, after M2M, after PC + far,
// after L2L + L2P), [5, 6] around the PP launch on the side stream.
// With timing level 2 only the events around the two interaction launches
// are recorded: [2, 3] (PC + far field) and [5, 6] (PP).
bool event_recorded(int level, int k) {
    return level == 1 || k == 2 || k == 3 || k == 5 || k == 6 || k == 7;
}
int drain_slot(Timing& tm, int slot) {
    if (!tm.pending[slot]) return CSFMM_OK;
    hipEvent_t* e = &tm.ev[size_t(slot) * Timing::kEvents];
    const int level = tm.pending[slot];
    CSFMM_HIP_TRY(hipEventSynchronize(e[level == 1 ? Timing::kMain - 1 : 3]));
    CSFMM_HIP_TRY(hipEventSynchronize(e[Timing::kMain + 1]));
    CSFMM_HIP_TRY(hipEventSynchronize(e[Timing::kMain + 2]));
    static constexpr int from[Timing::kStages] = {0, 1, 5, 2, 3, 5};
    static constexpr int to[Timing::kStages] = {1, 2, 6, 3, 4, 7};
    for (int k = 0; k < Timing::kStages; ++k) {
        if (!event_recorded(level, from[k]) || !event_recorded(level, to[k])) continue;
        float ms = 0.f;
        CSFMM_HIP_TRY(hipEventElapsedTime(&ms, e[from[k]], e[to[k]]));
        tm.sum_ms[k] += ms;
    }
    tm.n += 1;
    tm.pending[slot] = 0;
    return CSFMM_OK;
}

// Launch helper: fills b.prefix from per-request block counts, skips empty launches.
template <class F>
int launch_batched(Batch& b, const int64_t* blocks, F&& launch) {
    int64_t tot = 0;
    for (int r = 0; r < b.n; ++r) {
        b.prefix[r] = int32_t(tot);
        tot += blocks[r];
    }
    b.prefix[b.n] = int32_t(tot);
    if (tot <= 0) return CSFMM_OK;
    if (tot > (int64_t(1) << 31) - 1) {
        set_error("batched launch too large");
        return CSFMM_E_INVALID;
    }
    launch(unsigned(tot));
    CSFMM_LAUNCH_CHECK();
    return CSFMM_OK;
}

int64_t mfma_tiles(int64_t nrows, int nb) { return ((nrows + 15) / 16) * (nb / 16); }

// Parents a level needs for the row-blocked M2M: kM2mRowsMin, or the value of
// the environment variable CSFMM_M2M_ROWS_MIN (read at each eval), which lets
// tests run that kernel on small trees; both kernels compute the same product.
int64_t m2m_rows_min() {
    const char* e = std::getenv("CSFMM_M2M_ROWS_MIN");
    if (!e || !*e) return kM2mRowsMin;
    char* end = nullptr;
    const long long v = std::strtoll(e, &end, 10);
    return (end && *end == 0 && v >= 0) ? int64_t(v) : int64_t(kM2mRowsMin);
}

#define RCX(x)                              \
    do {                                    \
        int rc_ = (x);                      \
        if (rc_ != CSFMM_OK) return rc_;    \
    } while (0)

// e1: sorted weights of every request of the batch
int launch_gather(Batch& b, const EvalReq* reqs, int n, hipStream_t s) {
    int64_t blk[kMaxBatch];
    for (int r = 0; r < n; ++r) blk[r] = (reqs[r].plan->ns + 255) / 256;
    return launch_batched(b, blk, [&](unsigned g) { k_gather_w<<<g, 256, 0, s>>>(b); });
}

// e2 P2M at the source leaves, grouped by degree (P1 is a template parameter)
int launch_p2m(Batch& b, const EvalReq* reqs, int n, hipStream_t s) {
    int64_t blk[kMaxBatch];
    for (int P1 = 2; P1 <= kMaxP1; ++P1) {
        bool any = false;
        for (int r = 0; r < n; ++r) {
            blk[r] = reqs[r].plan->p + 1 == P1 ? reqs[r].plan->st->nleaves : 0;
            any = any || blk[r] > 0;
        }
        if (!any) continue;
        switch (P1) {
#define X(Q)                                                                                   \
    case Q: {                                                                                  \
        constexpr int PW = p2m_waves<Q>();                                                     \
        for (int r = 0; r < n; ++r) blk[r] = (blk[r] + PW - 1) / PW;                           \
        RCX(launch_batched(b, blk, [&](unsigned g) { k_p2m<Q><<<g, 64 * PW, 0, s>>>(b); }));   \
    } break;
            CSFMM_P1_CASES(X)
#undef X
            default: break;
        }
    }
    return CSFMM_OK;
}

int max_source_depth(const EvalReq* reqs, int n) {
    int maxd = 0;
    for (int r = 0; r < n; ++r) maxd = std::max(maxd, int(reqs[r].plan->st->depth));
    return maxd;
}

// e3 M2M by levels, deepest parents first: parent levels lhi down to llo;
// plans with fixed operators in one MFMA launch per level, shrunk plans
// (per-cell operators) in one launch per level and degree
int launch_m2m(Batch& b, const EvalReq* reqs, int n, hipStream_t s, int lhi, int llo) {
    int64_t blk[kMaxBatch];
    bool any_shrunk = false;
    for (int r = 0; r < n; ++r) any_shrunk = any_shrunk || reqs[r].plan->st->ops != nullptr;
    const int64_t rows_min = m2m_rows_min();
    for (int l = lhi; l >= std::max(llo, 0); --l) {
        int64_t blk_rows[kMaxBatch];
        bool any_rows = false;
        for (int r = 0; r < n; ++r) {
            const Tree& S = *reqs[r].plan->st;
            const int np = l < S.depth ? S.parents_begin[l + 1] - S.parents_begin[l] : 0;
            b.a0[r] = l < S.depth ? S.parents_begin[l] : 0;
            b.a1[r] = np;
            blk[r] = (S.ops || np >= rows_min) ? 0 : mfma_tiles(np, reqs[r].plan->nb1);
            blk_rows[r] = (S.ops || np < rows_min) ? 0 : (int64_t(np) + kM2mRows - 1) / kM2mRows;
            any_rows = any_rows || blk_rows[r] > 0;
        }
        RCX(launch_batched(b, blk, [&](unsigned g) { k_m2m<<<g, 256, 0, s>>>(b); }));
        if (any_rows)
            RCX(launch_batched(b, blk_rows, [&](unsigned g) { k_m2m_rows<<<g, 256, 0, s>>>(b); }));
        if (!any_shrunk) continue;
        for (int P1 = 2; P1 <= kMaxP1; ++P1) {
            bool any = false;
            for (int r = 0; r < n; ++r) {
                const Tree& S = *reqs[r].plan->st;
                blk[r] = (S.ops && reqs[r].plan->p + 1 == P1) ? (int64_t(b.a1[r]) + 3) / 4 : 0;
                any = any || blk[r] > 0;
            }
            if (!any) continue;
            switch (P1) {
#define X(Q)                                                                                   \
    case Q:                                                                                    \
        RCX(launch_batched(b, blk, [&](unsigned g) { k_m2m_cells<Q><<<g, 256, 0, s>>>(b); })); \
        break;
                CSFMM_P1_CASES(X)
#undef X
                default: break;
            }
        }
    }
    return CSFMM_OK;
}

Batch batch_of(const EvalReq* reqs, int n) {
    Batch b{};
    b.n = n;
    for (int r = 0; r < n; ++r) {
        b.v[r] = reqs[r].ws->dview;
        b.w[r] = reqs[r].w;
        b.out[r] = reqs[r].out;
        b.vd[r] = reqs[r].kernel == CSFMM_K_BIOT_SAVART ? 3 : 1;
    }
    return b;
}

int run_chunk(const EvalReq* reqs, int n, hipStream_t s) {
    Batch b = batch_of(reqs, n);
    int64_t blk[kMaxBatch];
    // optional stage timing (single request)
    hipEvent_t* ev = nullptr;
    if (n == 1 && reqs[0].plan->timing.on) {
        Timing& tm = reqs[0].plan->timing;
        const int slot = tm.next;
        tm.next = (tm.next + 1) % Timing::kSlots;
        int rc = drain_slot(tm, slot);
        if (rc != CSFMM_OK) return rc;
        ev = &tm.ev[size_t(slot) * Timing::kEvents];
        tm.pending[slot] = tm.on;  // 1 every stage, 2 the two interaction launches
    }
    const int level = ev ? reqs[0].plan->timing.on : 0;
    // the PP near field runs on the first workspace's side stream
    csfmm_workspace_s* W0 = reqs[0].ws;
    hipStream_t side = W0->side;
    auto mark = [&](int k) -> int {
        if (ev && event_recorded(level, k))
            CSFMM_HIP_TRY(hipEventRecord(ev[k], (k < Timing::kMain || k == Timing::kMain + 2) ? s : side));
        return CSFMM_OK;
    };
    RCX(mark(0));
    // e1 gather
    RCX(launch_gather(b, reqs, n, s));
    // e4 PP near field on the side stream, concurrent with the upward pass
    // (all of it or its upper levels, see below), the zero fill and e5: it
    // needs the gathered weights only; one launch per (kernel, form) group
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int r = 0; r < n; ++r)
        groups[{reqs[r].kernel, (reqs[r].plan->flags & CSFMM_FP32_FORM) ? 1 : 0}].push_back(r);
    auto tile_group = [&](const std::vector<int>& idx, int mode, Batch& g) -> int {
        g = Batch{};
        g.n = int(idx.size());
        g.mode = mode;
        int64_t tn = 0, tf = 0;
        // a PP launch whose requests all take the one-wave-per-leaf path runs
        // k_tile_wave; k_tile takes the rest (far-field blocks on its block path,
        // near-field blocks of such requests on the one-wave-per-leaf path)
        g.wave_kernel = mode == kTileNearPP ? 1 : 0;
        for (int q = 0; q < g.n; ++q)
            if (!leaf_wave_path(reqs[idx[q]].plan->tt)) g.wave_kernel = 0;
        for (int q = 0; q < g.n; ++q) {
            const int r = idx[q];
            g.v[q] = b.v[r];
            g.w[q] = b.w[r];
            g.out[q] = b.out[r];
            g.vd[q] = b.vd[r];
            g.prefix[q] = int32_t(tn);
            g.prefix2[q] = int32_t(tf);
            // near-field blocks: four target leaves each (one a wave) on the
            // one-wave-per-leaf path, else one
            const Tree& tt = reqs[r].plan->tt;
            g.leaf_wave[q] = leaf_wave_path(tt) ? 1 : 0;
            // the symmetric PP path (a property of the request alone)
            g.sym[q] = (mode == kTileNearPP && sym_path(reqs[r].plan, reqs[r].kernel)) ? 1 : 0;
            tn += g.leaf_wave[q] ? (int64_t(tt.nleaves) + 3) / 4 : tt.nleaves;
            tf += mode == kTilePCFar ? reqs[r].plan->lists.n_far_targets : 0;
        }
        g.prefix[g.n] = int32_t(tn);
        g.prefix2[g.n] = int32_t(tf);
        if (tn + tf > (int64_t(1) << 31) - 1) {
            set_error("interaction launch too large");
            return CSFMM_E_INVALID;
        }
        return CSFMM_OK;
    };
    auto launch_pp = [&]() -> int {
        CSFMM_HIP_TRY(hipEventRecord(W0->fork, s));
        CSFMM_HIP_TRY(hipStreamWaitEvent(side, W0->fork, 0));
        RCX(mark(Timing::kMain));
        for (auto& kv : groups) {
            Batch g;
            RCX(tile_group(kv.second, kTileNearPP, g));
            RCX(launch_tile_batch(g, kv.first.first, kv.first.second != 0, side));
            // column sums of the symmetric pairs, once every pair is done
            bool any_sym = false;
            for (int q = 0; q < g.n; ++q) any_sym = any_sym || g.sym[q];
            if (any_sym) RCX(launch_sym_merge(g, kv.first.first, kv.first.second != 0, side));
        }
        RCX(mark(Timing::kMain + 1));
        CSFMM_HIP_TRY(hipEventRecord(W0->join, side));
        return CSFMM_OK;
    };
    // Where to fork: when the far field is light (PC + CP + CC evaluations
    // below kLateFork of the PP ones) the eval stream's critical path is the
    // latency-bound upward pass, so PP starts right after the gather; when it
    // is heavy, P2M and the deepest (largest) M2M level first run without PP
    // waves beside them and PP starts after them (measured on the Poisson
    // workload N = 393,216 in the FP32 form: p = 6 (ratio 0.28) early fork
    // 0.257 vs 0.262 ms; p = 8 (0.61) and p = 10 (1.19) the late fork).
    constexpr double kLateFork = 0.45;
    int64_t ev_pp = 0, ev_far = 0;
    for (int r = 0; r < n; ++r) {
        const Lists& Ls = reqs[r].plan->lists;
        ev_pp += Ls.evals[kPP];
        ev_far += Ls.evals[kPC] + Ls.evals[kCP] + Ls.evals[kCC];
    }
    const bool late = double(ev_far) > kLateFork * double(ev_pp);
    const int maxd = max_source_depth(reqs, n);
    if (!late) RCX(launch_pp());
    RCX(launch_p2m(b, reqs, n, s));
    RCX(mark(1));
    RCX(launch_m2m(b, reqs, n, s, maxd - 1, maxd - 1));
    if (late) RCX(launch_pp());
    RCX(launch_m2m(b, reqs, n, s, maxd - 2, 0));
    // zero the proxy potentials (CP + CC accumulate into them)
    for (int r = 0; r < n; ++r)
        blk[r] = (int64_t(b.vd[r]) * reqs[r].ws->dview_host.psi_stride + 255) / 256;
    RCX(launch_batched(b, blk, [&](unsigned g) { k_zero_psi<<<g, 256, 0, s>>>(b); }));
    RCX(mark(2));
    // e4+e5 PC at the target particles (into its own buffer) and CP + CC into
    // the proxy potentials, one launch per (kernel, form) group with the
    // near-field blocks first and the far-field blocks after them
    for (auto& kv : groups) {
        Batch g;
        RCX(tile_group(kv.second, kTilePCFar, g));
        RCX(launch_tile_batch(g, kv.first.first, kv.first.second != 0, s));
    }
    RCX(mark(3));
    // join the PP near field
    CSFMM_HIP_TRY(hipStreamWaitEvent(s, W0->join, 0));
    RCX(mark(Timing::kMain + 2));
    // e7+e8 L2P, near field and scatter to the caller's order; one launch per
    // number of output components (blocks of the other group are empty)
    for (int vdl : {1, 3})
        for (int P1 = 2; P1 <= kMaxP1; ++P1) {
            bool any = false;
            for (int r = 0; r < n; ++r) {
                blk[r] = (b.vd[r] == vdl && reqs[r].plan->p + 1 == P1)
                             ? (int64_t(reqs[r].plan->tt.nleaves) + 3) / 4
                             : 0;
                any = any || blk[r] > 0;
            }
            if (!any) continue;
            switch (P1) {
#define X(Q)                                                                                       \
    case Q:                                                                                        \
        if (vdl == 1)                                                                              \
            RCX(launch_batched(b, blk, [&](unsigned g) { k_l2p<1, Q><<<g, 256, 0, s>>>(b); })); \
        else                                                                                       \
            RCX(launch_batched(b, blk, [&](unsigned g) { k_l2p<3, Q><<<g, 256, 0, s>>>(b); })); \
        break;
                CSFMM_P1_CASES(X)
#undef X
                default: break;
            }
        }
    RCX(mark(4));
    return CSFMM_OK;
}

}  // namespace

int timing_enable(csfmm_plan_s* P, int on) {
    Timing& tm = P->timing;
    if (on && tm.ev.empty()) {
        tm.ev.assign(size_t(Timing::kSlots) * Timing::kEvents, nullptr);
        for (auto& e : tm.ev) CSFMM_HIP_TRY(hipEventCreate(&e));
        tm.pending.assign(Timing::kSlots, 0);
    }
    if (!tm.ev.empty()) {
        for (int s = 0; s < Timing::kSlots; ++s) {
            int rc = drain_slot(tm, s);
            if (rc != CSFMM_OK) return rc;
        }
    }
    for (double& v : tm.sum_ms) v = 0.0;
    tm.n = 0;
    tm.on = on;
    return CSFMM_OK;
}

int timing_collect(csfmm_plan_s* P) {
    Timing& tm = P->timing;
    for (int s = 0; s < int(tm.pending.size()); ++s) {
        int rc = drain_slot(tm, s);
        if (rc != CSFMM_OK) return rc;
    }
    return CSFMM_OK;
}

namespace {
std::mutex g_side_mu;
std::vector<hipStream_t> g_side_free[64];  // per device
}  // namespace

hipError_t acquire_side_stream(hipStream_t* s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < 64) {
        std::lock_guard<std::mutex> lk(g_side_mu);
        if (!g_side_free[dev].empty()) {
            *s = g_side_free[dev].back();
            g_side_free[dev].pop_back();
            return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

void release_side_stream(hipStream_t s) {
    int dev = -1;
    if (hipStreamGetDevice(s, &dev) == hipSuccess && dev >= 0 && dev < 64) {
        std::lock_guard<std::mutex> lk(g_side_mu);
        if (g_side_free[dev].size() < 64) {
            g_side_free[dev].push_back(s);
            return;
        }
    }
    (void)hipStreamDestroy(s);
}

int workspace_create(csfmm_plan_s* P, hipStream_t stream, csfmm_workspace_s** out) {
    *out = nullptr;
    csfmm_workspace_s* W = new (std::nothrow) csfmm_workspace_s();
    if (!W) {
        set_error("host allocation failed");
        return CSFMM_E_OOM;
    }
    W->plan = P;
    const Tree& T = P->tt;
    const Tree& S = *P->st;
    // one allocation (csfmm_workspace_bytes counts the same arrays)
    ArenaGroup G;
    char* sym = nullptr;
    G.add(&W->ws, P->ns);
    G.add(&W->wbar, int64_t(S.ncells) * P->KS);
    G.add(&W->psi, int64_t(3) * T.ncells * P->KS);
    G.add(&W->phinear, int64_t(3) * P->nt);
    G.add(&W->phipc, int64_t(3) * P->nt);
    if (sym_path_possible(P)) G.add(&sym, sym_value_bytes(P) * P->lists.sym.n_own * kWaveLeaf);
    G.add(&W->dview, 1);
    int rc = G.commit(W->arena);
    if (rc != CSFMM_OK) {
        delete W;
        return rc;
    }
    W->sym_col = sym;
    hipError_t se = acquire_side_stream(&W->side);
    if (se == hipSuccess) se = hipEventCreateWithFlags(&W->fork, hipEventDisableTiming);
    if (se == hipSuccess) se = hipEventCreateWithFlags(&W->join, hipEventDisableTiming);
    if (se != hipSuccess) {
        set_error("creating the side stream failed: %s", hipGetErrorString(se));
        delete W;
        return CSFMM_E_HIP;
    }
    ReqView& v = W->dview_host;
    v = ReqView{};
    v.t_begin = T.begin; v.t_count = T.count; v.t_child0 = T.child0; v.t_leaf_anc = T.leaf_anc;
    v.t_leaves = T.leaves;
    v.t_parents = T.parents; v.t_perm = T.perm;
    v.t_x = T.x; v.t_y = T.y; v.t_z = T.z; v.t_u = T.u; v.t_v = T.v;
    v.t_center = T.center; v.t_prox = T.prox;
    v.s_begin = S.begin; v.s_count = S.count; v.s_child0 = S.child0; v.s_leaves = S.leaves;
    v.s_parents = S.parents; v.s_perm = S.perm;
    v.s_x = S.x; v.s_y = S.y; v.s_z = S.z; v.s_u = S.u; v.s_v = S.v; v.s_prox = S.prox;
    for (int k = 0; k < 4; ++k) {
        v.off[k] = P->lists.off[k];
        v.src[k] = P->lists.src[k];
    }
    v.novl = P->lists.novl;
    v.ncl = P->lists.ncl;
    v.far_targets = P->lists.far_targets;
    v.bm2m = P->bm2m;
    v.lag1d = P->lag1d;
    v.t_ops = T.ops;
    v.s_ops = S.ops;
    v.ws = W->ws; v.wbar = W->wbar; v.psi = W->psi; v.phinear = W->phinear; v.phipc = W->phipc;
    v.nt = P->nt; v.ns = P->ns;
    v.psi_stride = int64_t(T.ncells) * P->KS;
    v.p = P->p; v.K = P->K; v.KS = P->KS; v.nb1 = P->nb1;
    v.nleaves_t = T.nleaves;
    v.nleaves_s = S.nleaves;
    const SymPP& Y = P->lists.sym;
    v.own_off = Y.own_off; v.own_src = Y.own_src; v.recv_off = Y.recv_off;
    v.recv_slot = Y.recv_slot; v.one_off = Y.one_off; v.one_src = Y.one_src;
    v.sym_col = W->sym_col;
    k_set_view<<<1, 64, 0, stream>>>(W->dview, v);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        set_error("writing the request view failed: %s", hipGetErrorString(e));
        delete W;
        return CSFMM_E_HIP;
    }
    *out = W;
    return CSFMM_OK;
}

int run_eval_batch(const EvalReq* reqs, int n, hipStream_t s) {
    for (int r0 = 0; r0 < n; r0 += kMaxBatch) {
        int rc = run_chunk(reqs + r0, std::min(kMaxBatch, n - r0), s);
        if (rc != CSFMM_OK) return rc;
    }
    return CSFMM_OK;
}

int run_eval(csfmm_plan_s* P, int kernel, const double* weights, double* out, double* wbar_out,
             double* psi_out, double* near_out, hipStream_t s) {
    EvalReq q{P, P->ws0, kernel, weights, out};
    int rc = run_eval_batch(&q, 1, s);
    if (rc != CSFMM_OK) return rc;
    const Tree& T = P->tt;
    const Tree& S = *P->st;
    const int vd = kernel == CSFMM_K_BIOT_SAVART ? 3 : 1;
    if (wbar_out)
        CSFMM_HIP_TRY(hipMemcpyAsync(wbar_out, P->ws0->wbar, sizeof(double) * S.ncells * P->KS,
                                     hipMemcpyDeviceToDevice, s));
    if (psi_out)
        CSFMM_HIP_TRY(hipMemcpyAsync(psi_out, P->ws0->psi,
                                     sizeof(double) * vd * int64_t(T.ncells) * P->KS,
                                     hipMemcpyDeviceToDevice, s));
    if (near_out) {
        k_scatter_near<<<nblk(P->nt), 256, 0, s>>>(P->ws0->phinear, P->ws0->phipc, P->nt, vd,
                                                   T.perm, near_out);
        CSFMM_LAUNCH_CHECK();
    }
    return CSFMM_OK;
}

int run_treecode(csfmm_plan_s* P, int kernel, const double* weights, double* out, hipStream_t s) {
    EvalReq q{P, P->ws0, kernel, weights, out};
    Batch b = batch_of(&q, 1);
    RCX(launch_gather(b, &q, 1, s));
    RCX(launch_p2m(b, &q, 1, s));
    RCX(launch_m2m(b, &q, 1, s, max_source_depth(&q, 1) - 1, 0));
    const Tree& T = P->tt;
    const Tree& S = *P->st;
    TcArgs a{};
    a.tx = T.x;
    a.ty = T.y;
    a.tz = T.z;
    a.tperm = T.perm;
    a.nt = P->nt;
    a.sbegin = S.begin;
    a.scount = S.count;
    a.schild0 = S.child0;
    a.scenter = S.center;
    a.sradius = S.radius;
    a.sx = S.x;
    a.sy = S.y;
    a.sz = S.z;
    a.sw = P->ws0->ws;
    a.sprox = S.prox;
    a.swbar = P->ws0->wbar;
    a.K = P->K;
    a.KS = P->KS;
    a.N0 = P->leaf;
    a.nroots = S.level_begin.size() > 1 ? S.level_begin[1] : 0;
    a.theta2 = P->theta * P->theta;
    a.out = out;
    if (!P->tc_status) RCX(P->arena.alloc(&P->tc_status, 1));
    a.status = P->tc_status;
    k_set_i32<<<1, 64, 0, s>>>(P->tc_status, 0);
    CSFMM_LAUNCH_CHECK();
    RCX(launch_treecode(a, kernel, s));
    int32_t st = 0;
    CSFMM_HIP_TRY(hipMemcpyAsync(&st, P->tc_status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CSFMM_HIP_TRY(hipStreamSynchronize(s));
    if (st != 0) {
        set_error("treecode: a traversal stack overflowed (result void)");
        return CSFMM_E_INTERNAL;
    }
    return CSFMM_OK;
}

}  // namespace csfmm
