// Evaluation of a plan (paper §8, Algorithm 2 lines 3, 5 and 7-21):
//   gather weights -> P2M (eq. PC proxy weights of the leaves) -> M2M by
//   levels (eq. upwardpass2, FP64 MFMA) -> near field PP+PC and far field
//   CP+CC (tile engine) -> L2L by levels (eq. downward_2, FP64 MFMA) ->
//   L2P at the leaves (eq. downward_1) fused with the scatter to the caller's
//   order.
#include "common.h"
#include "dev_util.h"

namespace csfmm {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kMaxP1 = kMaxDegree + 1;

__device__ __forceinline__ double cheb(int k, int p) { return cos(double(k) * kPi / double(p)); }

__global__ void k_gather_w(const double* __restrict__ w, const int32_t* __restrict__ perm, int64_t n,
                           double* __restrict__ ws) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) ws[k] = w[perm[k]];
}

__global__ void k_fill_zero(double* __restrict__ a, int64_t n) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) a[k] = 0.0;
}

// Barycentric values L_0..L_p at x (§4, eq. barycentric), exact hit -> delta.
__device__ __forceinline__ void bary_row(int p, const double* s, const double* beta, double x,
                                         double* L) {
    int hit = -1;
    double den = 0.0;
    for (int k = 0; k <= p; ++k) {
        const double d = x - s[k];
        if (d == 0.0) hit = k;
        L[k] = beta[k] / d;
        den += L[k];
    }
    if (hit >= 0) {
        for (int k = 0; k <= p; ++k) L[k] = (k == hit) ? 1.0 : 0.0;
    } else {
        const double inv = 1.0 / den;
        for (int k = 0; k <= p; ++k) L[k] *= inv;
    }
}

__device__ __forceinline__ void cheb_setup(int p, double* s, double* beta) {
    for (int k = threadIdx.x; k <= p; k += blockDim.x) {
        s[k] = cheb(k, p);
        double b = (k & 1) ? -1.0 : 1.0;
        if (k == 0 || k == p) b *= 0.5;
        beta[k] = b;
    }
}

// P2M: wbar_k(leaf) = sum_j L_k1(u_j) L_k2(v_j) w_j   (eq. PC, §6)
constexpr int kP2MThreads = 128;
__global__ __launch_bounds__(kP2MThreads) void k_p2m(const int32_t* __restrict__ leaves,
                                                     const int32_t* __restrict__ begin,
                                                     const int32_t* __restrict__ count,
                                                     const double* __restrict__ u,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ ws, int p, int KS,
                                                     double* __restrict__ wbar) {
    __shared__ double s[kMaxP1], beta[kMaxP1];
    __shared__ double Lu[kP2MThreads][kMaxP1 + 1];
    __shared__ double Lv[kP2MThreads][kMaxP1 + 1];
    __shared__ double wv[kP2MThreads];
    const int c = leaves[xcd_logical_block(blockIdx.x, gridDim.x)];
    const int b = begin[c], m = count[c];
    const int P1 = p + 1, K = P1 * P1;
    cheb_setup(p, s, beta);
    __syncthreads();
    double acc[3] = {0.0, 0.0, 0.0};  // K <= 3 * kP2MThreads
    for (int j0 = 0; j0 < m; j0 += kP2MThreads) {
        const int nj = min(kP2MThreads, m - j0);
        if (threadIdx.x < nj) {
            const int j = b + j0 + threadIdx.x;
            bary_row(p, s, beta, u[j], Lu[threadIdx.x]);
            bary_row(p, s, beta, v[j], Lv[threadIdx.x]);
            wv[threadIdx.x] = ws[j];
        }
        __syncthreads();
        for (int r = 0; r < 3; ++r) {
            const int k = threadIdx.x + r * kP2MThreads;
            if (k < K) {
                const int k1 = k / P1, k2 = k % P1;
                double a = acc[r];
                for (int j = 0; j < nj; ++j) a += Lu[j][k1] * Lv[j][k2] * wv[j];
                acc[r] = a;
            }
        }
        __syncthreads();
    }
    for (int r = 0; r < 3; ++r) {
        const int k = threadIdx.x + r * kP2MThreads;
        if (k < KS) wbar[int64_t(c) * KS + k] = (k < K) ? acc[r] : 0.0;
    }
}

// Batched small GEMM on FP64 MFMA (v_mfma_f64_16x16x4f64), 16 rows per block,
// the four waves share the 16-column tiles of the output.
//   MODE 0 (M2M, eq. upwardpass2): row = parent P;  A = wbar of its 4 children
//     (4*KS contiguous values), B = bm2m [4KS][nb], C = wbar(P) (KS columns, written)
//   MODE 1 (L2L, eq. downward_2):  row = (component, parent P); A = psi(P) (KS),
//     B = bl2l [KS][nb], C = psi of the 4 children (4*KS columns, accumulated)
// MFMA f64 16x16x4 operand layout: lane l holds A[l%16][l/16], B[l/16][l%16]
// and D[l/16 + 4*i][l%16], i = 0..3 (checked with a one-hot probe).
template <int MODE>
__global__ __launch_bounds__(256) void k_mfma_pass(const int32_t* __restrict__ rows, int np,
                                                   int ncomp, const int32_t* __restrict__ child0,
                                                   const double* __restrict__ Abase,
                                                   double* __restrict__ Cbase, int64_t comp_stride,
                                                   const double* __restrict__ B, int nb, int KS) {
    // MODE 0: one block per (16-row tile, 16-column tile); wave q takes the
    //   K-slice of child q (split-K) and the four partial tiles are summed in LDS.
    // MODE 1: one wave per (16-row tile, 16-column tile).
    // Operand loads are issued kAhead MFMA steps ahead of their use.
    constexpr int kAhead = 16;
    __shared__ double4_t part[MODE == 0 ? 3 : 1][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ntiles = nb / 16;
    const int gw = MODE == 0 ? int(blockIdx.x) : int(blockIdx.x) * 4 + wave;
    const int rt = gw / ntiles, tile = gw % ntiles;
    const int nrows = np * ncomp;
    const int r0 = rt * 16;
    if (r0 >= nrows) return;  // uniform over the block in MODE 0, over the wave in MODE 1
    const int Kd = KS;        // K-slice per wave: one child (MODE 0) or the parent (MODE 1)
    const int koff = MODE == 0 ? wave * KS : 0;
    const int Nw = MODE == 0 ? KS : 4 * KS;
    const int ra = r0 + (lane & 15);
    const double* arow = nullptr;
    if (ra < nrows) {
        const int comp = ra / np, P = rows[ra % np];
        const int cell = MODE == 0 ? child0[P] : P;
        arow = Abase + comp * comp_stride + int64_t(cell) * KS + koff;
    }
    const int kq = lane >> 4;
    const double* bcol = B + int64_t(koff) * nb + tile * 16 + (lane & 15);
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < Kd; kk += 4 * kAhead) {
        double av[kAhead], bv[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int k = kk + 4 * u + kq;
            const bool in = k < Kd;
            av[u] = (arow && in) ? arow[k] : 0.0;
            bv[u] = in ? bcol[int64_t(k) * nb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u)
            if (kk + 4 * u < Kd)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    if constexpr (MODE == 0) {
        if (wave > 0) part[wave - 1][lane] = acc;
        __syncthreads();
        if (wave > 0) return;
        acc += part[0][lane];
        acc += part[1][lane];
        acc += part[2][lane];
    }
    const int col = tile * 16 + (lane & 15);
    if (col < Nw) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + kq + 4 * i;
            if (r < nrows) {
                const int comp = r / np, P = rows[r % np];
                const int cell = MODE == 0 ? P : child0[P];
                double* crow = Cbase + comp * comp_stride + int64_t(cell) * KS;
                if (MODE == 0)
                    crow[col] = acc[i];
                else
                    crow[col] += acc[i];
            }
        }
    }
}

inline unsigned mfma_blocks(int mode, int64_t nrows, int nb) {
    const int64_t tiles = ((nrows + 15) / 16) * (nb / 16);
    return unsigned(mode == 0 ? tiles : (tiles + 3) / 4);
}

// L2P (eq. downward_1 at the leaves) + near field + scatter to caller order.
constexpr int kL2PThreads = 128;
template <int VD>
__global__ __launch_bounds__(kL2PThreads) void k_l2p(
    const int32_t* __restrict__ leaves, const int32_t* __restrict__ begin,
    const int32_t* __restrict__ count, const double* __restrict__ u, const double* __restrict__ v,
    const double* __restrict__ psi, int64_t psi_stride, const double* __restrict__ near,
    int64_t nt, const int32_t* __restrict__ perm, int p, int KS, double* __restrict__ out) {
    __shared__ double s[kMaxP1], beta[kMaxP1];
    __shared__ double ps[VD][(kMaxP1) * (kMaxP1) + 4];
    __shared__ double Lu[kL2PThreads][kMaxP1 + 1];
    __shared__ double Lv[kL2PThreads][kMaxP1 + 1];
    const int c = leaves[xcd_logical_block(blockIdx.x, gridDim.x)];
    const int b = begin[c], m = count[c];
    if (m == 0) return;
    const int P1 = p + 1, K = P1 * P1;
    cheb_setup(p, s, beta);
    for (int k = threadIdx.x; k < K; k += blockDim.x)
        for (int d = 0; d < VD; ++d) ps[d][k] = psi[d * psi_stride + int64_t(c) * KS + k];
    __syncthreads();
    for (int j0 = 0; j0 < m; j0 += kL2PThreads) {
        const int jj = j0 + threadIdx.x;
        if (jj < m) {
            const int j = b + jj;
            double* L1 = Lu[threadIdx.x];
            double* L2 = Lv[threadIdx.x];
            bary_row(p, s, beta, u[j], L1);
            bary_row(p, s, beta, v[j], L2);
            double acc[VD];
            for (int d = 0; d < VD; ++d) acc[d] = 0.0;
            for (int n1 = 0; n1 < P1; ++n1) {
                double inner[VD];
                for (int d = 0; d < VD; ++d) inner[d] = 0.0;
                for (int n2 = 0; n2 < P1; ++n2) {
                    const double l2 = L2[n2];
                    for (int d = 0; d < VD; ++d) inner[d] += ps[d][n1 * P1 + n2] * l2;
                }
                for (int d = 0; d < VD; ++d) acc[d] += L1[n1] * inner[d];
            }
            const int64_t o = perm[j];
            for (int d = 0; d < VD; ++d) out[o * VD + d] = near[d * nt + j] + acc[d];
        }
    }
}

__global__ void k_scatter_near(const double* __restrict__ near, int64_t nt, int vd,
                               const int32_t* __restrict__ perm, double* __restrict__ out) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const int64_t o = perm[k];
    for (int d = 0; d < vd; ++d) out[o * vd + d] = near[d * nt + k];
}

inline unsigned nblk(int64_t n, int t = 256) { return unsigned((n + t - 1) / t); }

using Timing = csfmm_plan_s::Timing;

// Adds the stage times of a finished slot to the sums.
int drain_slot(Timing& tm, int slot) {
    if (!tm.pending[slot]) return CSFMM_OK;
    hipEvent_t* e = &tm.ev[size_t(slot) * (Timing::kStages + 1)];
    CSFMM_HIP_TRY(hipEventSynchronize(e[Timing::kStages]));
    for (int k = 0; k < Timing::kStages; ++k) {
        float ms = 0.f;
        CSFMM_HIP_TRY(hipEventElapsedTime(&ms, e[k], e[k + 1]));
        tm.sum_ms[k] += ms;
    }
    tm.n += 1;
    tm.pending[slot] = 0;
    return CSFMM_OK;
}

}  // namespace

int timing_enable(csfmm_plan_s* P, bool on) {
    Timing& tm = P->timing;
    if (on && tm.ev.empty()) {
        tm.ev.assign(size_t(Timing::kSlots) * (Timing::kStages + 1), nullptr);
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

int run_eval(csfmm_plan_s* P, int kernel, const double* weights, double* out, double* wbar_out,
             double* psi_out, double* near_out, hipStream_t s) {
    Tree& T = P->tt;
    Tree& S = *P->st;
    const int vd = kernel == CSFMM_K_BIOT_SAVART ? 3 : 1;
    const int64_t psi_stride = int64_t(T.ncells) * P->KS;
    Timing& tm = P->timing;
    hipEvent_t* ev = nullptr;
    if (tm.on) {
        const int slot = tm.next;
        tm.next = (tm.next + 1) % Timing::kSlots;
        int rc = drain_slot(tm, slot);
        if (rc != CSFMM_OK) return rc;
        ev = &tm.ev[size_t(slot) * (Timing::kStages + 1)];
        tm.pending[slot] = 1;
    }
    auto mark = [&](int k) -> int {
        if (ev) CSFMM_HIP_TRY(hipEventRecord(ev[k], s));
        return CSFMM_OK;
    };
    int mrc = mark(0);
    if (mrc != CSFMM_OK) return mrc;

    // e1 gather weights into sorted order
    k_gather_w<<<nblk(P->ns), 256, 0, s>>>(weights, S.perm, P->ns, P->ws);
    CSFMM_LAUNCH_CHECK();
    // e2 P2M at the source leaves
    if (S.nleaves > 0) {
        k_p2m<<<S.nleaves, kP2MThreads, 0, s>>>(S.leaves, S.begin, S.count, S.u, S.v, P->ws, P->p,
                                                P->KS, P->wbar);
        CSFMM_LAUNCH_CHECK();
    }
    if ((mrc = mark(1)) != CSFMM_OK) return mrc;
    // e3 M2M, deepest parents first
    for (int l = S.depth - 1; l >= 0; --l) {
        const int pb = S.parents_begin[l], np = S.parents_begin[l + 1] - pb;
        if (np <= 0) continue;
        k_mfma_pass<0><<<mfma_blocks(0, np, P->nb1), 256, 0, s>>>(
            S.parents + pb, np, 1, S.child0, P->wbar, P->wbar, 0, P->bm2m, P->nb1, P->KS);
        CSFMM_LAUNCH_CHECK();
    }
    if ((mrc = mark(2)) != CSFMM_OK) return mrc;
    // e4 near field: PP + PC
    {
        int rc = launch_near(P, kernel, s);
        if (rc != CSFMM_OK) return rc;
    }
    if ((mrc = mark(3)) != CSFMM_OK) return mrc;
    // e5 far field: CP + CC into the accumulated proxy potentials
    k_fill_zero<<<nblk(vd * psi_stride), 256, 0, s>>>(P->psi, vd * psi_stride);
    CSFMM_LAUNCH_CHECK();
    {
        int rc = launch_far(P, kernel, s);
        if (rc != CSFMM_OK) return rc;
    }
    if ((mrc = mark(4)) != CSFMM_OK) return mrc;
    // e6 L2L, root level first
    for (int l = 0; l < T.depth; ++l) {
        const int pb = T.parents_begin[l], np = T.parents_begin[l + 1] - pb;
        if (np <= 0) continue;
        k_mfma_pass<1><<<mfma_blocks(1, int64_t(np) * vd, P->nb2), 256, 0, s>>>(
            T.parents + pb, np, vd, T.child0, P->psi, P->psi, psi_stride, P->bl2l, P->nb2, P->KS);
        CSFMM_LAUNCH_CHECK();
    }
    if ((mrc = mark(5)) != CSFMM_OK) return mrc;
    // e7+e8 L2P, near field and scatter to the caller's order
    if (T.nleaves > 0) {
        if (vd == 3)
            k_l2p<3><<<T.nleaves, kL2PThreads, 0, s>>>(T.leaves, T.begin, T.count, T.u, T.v, P->psi,
                                                       psi_stride, P->phinear, P->nt, T.perm, P->p,
                                                       P->KS, out);
        else
            k_l2p<1><<<T.nleaves, kL2PThreads, 0, s>>>(T.leaves, T.begin, T.count, T.u, T.v, P->psi,
                                                       psi_stride, P->phinear, P->nt, T.perm, P->p,
                                                       P->KS, out);
        CSFMM_LAUNCH_CHECK();
    }
    if ((mrc = mark(6)) != CSFMM_OK) return mrc;
    if (wbar_out)
        CSFMM_HIP_TRY(hipMemcpyAsync(wbar_out, P->wbar, sizeof(double) * S.ncells * P->KS,
                                     hipMemcpyDeviceToDevice, s));
    if (psi_out)
        CSFMM_HIP_TRY(hipMemcpyAsync(psi_out, P->psi, sizeof(double) * vd * psi_stride,
                                     hipMemcpyDeviceToDevice, s));
    if (near_out) {
        k_scatter_near<<<nblk(P->nt), 256, 0, s>>>(P->phinear, P->nt, vd, T.perm, near_out);
        CSFMM_LAUNCH_CHECK();
    }
    return CSFMM_OK;
}

}  // namespace csfmm
