// Plan construction on the GPU: face and Morton keys, sort, quadtree levels,
// cell geometry and proxy points, fixed interpolation operators and the dual
// tree traversal that produces the PP/PC/CP/CC lists.
//
// Paper passages: §3 (faces, quadtree of cubed-sphere cells, split when a
// cluster has more than N0 particles), §4 (Chebyshev points s_k = cos(k pi/n),
// barycentric weights, tensor-product proxies mapped affinely in the local
// angles), §6 eq. (upwardpass2) and §8.1 eq. (downward_2) (parent polynomials
// at child nodes), §8 Algorithm 2 and its MAC (r_t + r_s)/R < theta.
//
// Readings of the paper that this code fixes (the oracle takes the same ones):
//  * the face of a point is the axis of its largest |coordinate| (ties x, y, z);
//  * a level-l cell holds the points whose scaled angle t = (xi+pi/4)/(pi/2)
//    satisfies floor(2^l t) = cell index (half-open intervals);
//  * a split creates all four quadrants, also empty ones; leaf = no children;
//  * centre = image of the angle midpoint, radius = largest chord distance to
//    a corner, R = chord distance of the centres, MAC strict;
//  * recursion goes into the coarser-level cluster (tie: target), or into the
//    other one when that cluster is a leaf; both leaves -> PP even when
//    separated; separated and not both leaves -> PC / CP / CC exclusively.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace csfmm {
namespace {

constexpr int kT = 256;

inline unsigned nblk(int64_t n, int t = kT) { return unsigned((n + t - 1) / t); }

// --------------------------------------------------------------- geometry
// Face frames: (normal, e_a, e_b), right handed, for +x, +y, -x, -y, +z, -z.
// c = x.normal, a = x.e_a, b = x.e_b; the map back is v = normal + A e_a + B e_b.
__device__ __forceinline__ void face_coords(int f, double x, double y, double z, double& a,
                                            double& b, double& c) {
    switch (f) {
        case 0: c = x; a = y; b = z; break;
        case 1: c = y; a = -x; b = z; break;
        case 2: c = -x; a = -y; b = z; break;
        case 3: c = -y; a = x; b = z; break;
        case 4: c = z; a = y; b = -x; break;
        default: c = -z; a = y; b = x; break;
    }
}

__device__ __forceinline__ void gnomonic(int f, double xi, double eta, double* out) {
#pragma clang fp contract(off)
    const double A = tan(xi), B = tan(eta);
    double vx, vy, vz;
    switch (f) {
        case 0: vx = 1.0; vy = A; vz = B; break;
        case 1: vx = -A; vy = 1.0; vz = B; break;
        case 2: vx = -1.0; vy = -A; vz = B; break;
        case 3: vx = A; vy = -1.0; vz = B; break;
        case 4: vx = -B; vy = A; vz = 1.0; break;
        default: vx = B; vy = A; vz = -1.0; break;
    }
    const double r = sqrt(vx * vx + vy * vy + vz * vz);
    out[0] = vx / r;
    out[1] = vy / r;
    out[2] = vz / r;
}

__device__ __forceinline__ uint64_t spread_bits(uint32_t v) {
    uint64_t x = v & 0xFFFFFull;  // 20 bits
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// Morton prefix of cell (f, l, i, j): face bits above 2l interleaved bits (i high).
__device__ __forceinline__ uint64_t cell_prefix(int f, int l, uint32_t i, uint32_t j) {
    return (uint64_t(f) << (2 * l)) | (spread_bits(i) << 1) | spread_bits(j);
}

__global__ void k_check_points(const double* __restrict__ p, int64_t n, int* __restrict__ bad) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double x = p[3 * k], y = p[3 * k + 1], z = p[3 * k + 2];
    const double r = sqrt(x * x + y * y + z * z);
    const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && fabs(r - 1.0) <= 1e-12;
    if (!ok) atomicOr(bad, 1);
}

// §3: face of each point, local angles and the Morton key of its deepest cell.
__global__ void k_face_key(const double* __restrict__ p, int64_t n, uint64_t* __restrict__ keys,
                           int32_t* __restrict__ idx, double* __restrict__ xi_out,
                           double* __restrict__ eta_out) {
#pragma clang fp contract(off)
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double x = p[3 * k], y = p[3 * k + 1], z = p[3 * k + 2];
    const double ax = fabs(x), ay = fabs(y), az = fabs(z);
    int f;
    if (ax >= ay && ax >= az)
        f = x > 0 ? 0 : 2;
    else if (ay >= az)
        f = y > 0 ? 1 : 3;
    else
        f = z > 0 ? 4 : 5;
    double a, b, c;
    face_coords(f, x, y, z, a, b, c);
    const double xi = atan(a / c), eta = atan(b / c);
    const double scale = double(1u << kMaxLevel);
    const double ti = floor(((xi + kPi4) / kPi2) * scale);
    const double tj = floor(((eta + kPi4) / kPi2) * scale);
    const double top = double((1u << kMaxLevel) - 1);
    const uint32_t i = uint32_t(fmin(fmax(ti, 0.0), top));
    const uint32_t j = uint32_t(fmin(fmax(tj, 0.0), top));
    keys[k] = cell_prefix(f, kMaxLevel, i, j);
    idx[k] = int32_t(k);
    xi_out[k] = xi;
    eta_out[k] = eta;
}

__global__ void k_gather_points(const double* __restrict__ p, const int32_t* __restrict__ idx,
                                const double* __restrict__ xi, const double* __restrict__ eta,
                                int64_t n, double* __restrict__ x, double* __restrict__ y,
                                double* __restrict__ z, double* __restrict__ xs,
                                double* __restrict__ es) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t i = idx[k];
    x[k] = p[3 * i];
    y[k] = p[3 * i + 1];
    z[k] = p[3 * i + 2];
    xs[k] = xi[i];
    es[k] = eta[i];
}

__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* __restrict__ a, int64_t lo,
                                                   int64_t hi, uint64_t key) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ void k_roots(const uint64_t* __restrict__ keys, int64_t n, int32_t* face, int32_t* ci,
                        int32_t* cj, int32_t* begin, int32_t* count) {
    const int f = threadIdx.x;
    if (f >= 6) return;
    const uint64_t sh = 2 * kMaxLevel;
    const int64_t b = lower_bound_u64(keys, 0, n, uint64_t(f) << sh);
    const int64_t e = lower_bound_u64(keys, 0, n, uint64_t(f + 1) << sh);
    face[f] = f;
    ci[f] = 0;
    cj[f] = 0;
    begin[f] = int32_t(b);
    count[f] = int32_t(e - b);
}

__global__ void k_split_flags(const int32_t* __restrict__ count, int n, int N0, int level,
                              int32_t* __restrict__ flag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    flag[k] = (count[k] > N0 && level < kMaxLevel) ? 1 : 0;
}

// Children of the split cells of one level; child ranges by binary search of
// the sorted keys inside the parent's range.
__global__ void k_children(const uint64_t* __restrict__ keys, int n, int level,
                           const int32_t* __restrict__ flag, const int32_t* __restrict__ off,
                           const int32_t* __restrict__ pface, const int32_t* __restrict__ pci,
                           const int32_t* __restrict__ pcj, const int32_t* __restrict__ pbegin,
                           const int32_t* __restrict__ pcount, int32_t next_level_begin,
                           int32_t nchildren,
                           int32_t* __restrict__ pchild0, int32_t* __restrict__ cface,
                           int32_t* __restrict__ cci, int32_t* __restrict__ ccj,
                           int32_t* __restrict__ cbegin, int32_t* __restrict__ ccount) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (!flag[k]) {
        pchild0[k] = -1;
        return;
    }
    const int slot = 4 * off[k];
    if (slot + 4 > nchildren) {
        pchild0[k] = -1;
        return;
    }
    pchild0[k] = next_level_begin + slot;
    const int l = level + 1;
    const int f = pface[k];
    const int64_t b = pbegin[k], e = b + pcount[k];
    const int sh = 2 * (kMaxLevel - l);
    int64_t lo = b;
    for (int q = 0; q < 4; ++q) {
        const uint32_t i = 2u * uint32_t(pci[k]) + uint32_t(q >> 1);
        const uint32_t j = 2u * uint32_t(pcj[k]) + uint32_t(q & 1);
        const uint64_t pre = cell_prefix(f, l, i, j);
        const int64_t cb = lower_bound_u64(keys, lo, e, pre << sh);
        const int64_t ce = lower_bound_u64(keys, cb, e, (pre + 1) << sh);
        cface[slot + q] = f;
        cci[slot + q] = int32_t(i);
        ccj[slot + q] = int32_t(j);
        cbegin[slot + q] = int32_t(cb);
        ccount[slot + q] = int32_t(ce - cb);
        lo = ce;
    }
}

// The cell arrays of every level of the breadth-first build.
struct LevelArrays {
    int32_t nlev;
    int32_t first[kMaxLevel + 2];  // first cell of each level, then the end
    const int32_t* face[kMaxLevel + 1];
    const int32_t* ci[kMaxLevel + 1];
    const int32_t* cj[kMaxLevel + 1];
    const int32_t* begin[kMaxLevel + 1];
    const int32_t* count[kMaxLevel + 1];
    const int32_t* child0[kMaxLevel + 1];
};

// Concatenates the levels into the tree's cell arrays, with each cell's level,
// its parent (a cell writes the entries of its four children; roots get -1)
// and its leaf / parent flags for the compactions that follow.
__global__ void k_gather_levels(LevelArrays L, int nc, int32_t* __restrict__ level,
                                int32_t* __restrict__ face, int32_t* __restrict__ ci,
                                int32_t* __restrict__ cj, int32_t* __restrict__ begin,
                                int32_t* __restrict__ count, int32_t* __restrict__ child0,
                                int32_t* __restrict__ parent, int32_t* __restrict__ leaf_flag,
                                int32_t* __restrict__ parent_flag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nc) return;
    int l = 0;
    while (l + 1 < L.nlev && k >= L.first[l + 1]) ++l;
    const int j = k - L.first[l];
    const int c0 = L.child0[l][j];
    level[k] = l;
    face[k] = L.face[l][j];
    ci[k] = L.ci[l][j];
    cj[k] = L.cj[l][j];
    begin[k] = L.begin[l][j];
    count[k] = L.count[l][j];
    child0[k] = c0;
    if (l == 0) parent[k] = -1;
    if (c0 >= 0)
        for (int q = 0; q < 4; ++q) parent[c0 + q] = k;
    leaf_flag[k] = c0 < 0 ? 1 : 0;
    parent_flag[k] = c0 < 0 ? 0 : 1;
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
    if (int(threadIdx.x) < n) p[threadIdx.x] = 0ull;
}

// *a = *b = *c = 0 (the element past the entries of three kind arrays)
__global__ void k_zero_i32x3(int32_t* __restrict__ a, int32_t* __restrict__ b,
                             int32_t* __restrict__ c) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a = *b = *c = 0;
}

// Owner of the unordered pair of cells {t, s}, t != s: the smaller id when
// t + s is odd, else the larger, so that every cell owns about half of its
// symmetric pairs.
__device__ __forceinline__ int pair_owner(int t, int s) {
    return ((t + s) & 1) ? (t < s ? t : s) : (t < s ? s : t);
}

// Index of the entry of cell c whose source is x in the CSR lists, or -1.
__device__ __forceinline__ int pp_find(const int32_t* off, const int32_t* src, int c, int x) {
    for (int e = off[c]; e < off[c + 1]; ++e)
        if (src[e] == x) return e;
    return -1;
}

// Symmetric split of the PP entries of a same-set plan (see SymPP), per
// target cell: each entry past the overlapping head (the cell itself) is
// one-way (kind_one; every close entry, which keeps exact differences, and so
// stays first in the cell's one-way list), a symmetric pair the cell owns
// (kind_own) or one its partner owns (kind_recv, rev = the partner's entry of
// the pair).  One
// element past the entries stays 0, so exclusive scans of the kinds give the
// positions and, at off[t], the offsets of every cell.  One wave per target
// cell, a lane per entry.
__global__ void k_sym_kinds(int ncells, const int32_t* __restrict__ off,
                            const int32_t* __restrict__ src, const int32_t* __restrict__ novl,
                            const int32_t* __restrict__ ncl, int32_t* __restrict__ kind_own,
                            int32_t* __restrict__ kind_recv, int32_t* __restrict__ kind_one,
                            int32_t* __restrict__ rev) {
    const int t = int(blockIdx.x) * (blockDim.x / 64) + int(threadIdx.x / 64);
    if (t >= ncells) return;
    for (int e = off[t] + int(threadIdx.x % 64); e < off[t + 1]; e += 64) {
        int k = 0, r = -1;
        if (e >= off[t] + novl[t] + ncl[t]) {
            const int c = src[e];
            r = c != t ? pp_find(off, src, c, t) : -1;
            k = r < 0 ? 1 : (pair_owner(t, c) == t ? 2 : 3);
        } else if (e >= off[t] + novl[t]) {
            k = 1;
        }
        kind_own[e] = k == 2;
        kind_recv[e] = k == 3;
        kind_one[e] = k == 1;
        rev[e] = r;
    }
}

// Fills the SymPP arrays from the exclusive scans of the kinds (over the
// entries plus one): owned and one-way entries keep their list order; the
// slot of a received pair is the owned position of the partner's entry.
// Thread e writes entry e and, for e <= ncells, the offsets of cell e.
__global__ void k_sym_fill(int ncells, int64_t nent, const int32_t* __restrict__ off,
                           const int32_t* __restrict__ src, const int32_t* __restrict__ kind_own,
                           const int32_t* __restrict__ kind_recv,
                           const int32_t* __restrict__ kind_one, const int32_t* __restrict__ rev,
                           const int32_t* __restrict__ own_ex, const int32_t* __restrict__ recv_ex,
                           const int32_t* __restrict__ one_ex, int32_t* __restrict__ own_off,
                           int32_t* __restrict__ own_src, int32_t* __restrict__ recv_off,
                           int32_t* __restrict__ recv_slot, int32_t* __restrict__ one_off,
                           int32_t* __restrict__ one_src) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e <= ncells) {
        const int b = off[e];  // off[ncells] = nent
        own_off[e] = own_ex[b];
        recv_off[e] = recv_ex[b];
        one_off[e] = one_ex[b];
    }
    if (e >= nent) return;
    if (kind_own[e]) own_src[own_ex[e]] = src[e];
    if (kind_one[e]) one_src[one_ex[e]] = src[e];
    if (kind_recv[e]) recv_slot[recv_ex[e]] = own_ex[rev[e]];
}

// Largest point count over the leaves of a tree.
__global__ void k_max_leaf(const int32_t* __restrict__ leaves, int nleaves,
                           const int32_t* __restrict__ count, unsigned long long* __restrict__ mx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaves) return;
    atomicMax(mx, (unsigned long long)count[leaves[i]]);
}

// Kernel evaluations of list `kind` for target cell t: sum over its entries of
// (targets) x (sources), targets = particles (PP, PC) or K proxies (CP, CC),
// sources = particles (PP, CP) or K proxies (PC, CC); a same-set PP self entry
// omits the i = j pairs.  Integer sums, so the atomic total is exact.
__global__ void k_count_evals(int kind, const int32_t* __restrict__ off,
                              const int32_t* __restrict__ src, const int32_t* __restrict__ tcount,
                              const int32_t* __restrict__ scount, int ncells, int K, int same,
                              unsigned long long* __restrict__ total) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells) return;
    const bool tpart = kind == 0 || kind == 1, spart = kind == 0 || kind == 2;
    const long long nt = tpart ? tcount[t] : K;
    long long ev = 0;
    for (int e = off[t]; e < off[t + 1]; ++e) {
        const int sc = src[e];
        ev += nt * (spart ? scount[sc] : K);
        if (kind == 0 && same && sc == t) ev -= tcount[t];
    }
    if (ev) atomicAdd(total, (unsigned long long)ev);
}

// parent[c] = the cell whose four children include c; -1 for the roots
// Path from the root to every leaf (see Tree::leaf_anc).
__global__ void k_leaf_paths(const int32_t* __restrict__ leaves, int nleaves,
                             const int32_t* __restrict__ parent, int32_t* __restrict__ anc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaves) return;
    int32_t tmp[kMaxLevel + 1];
    int d = 0;
    for (int x = leaves[i]; x >= 0 && d <= kMaxLevel; x = parent[x]) tmp[d++] = x;
    int32_t* a = anc + int64_t(i) * kAncStride;
    a[0] = d;
    for (int k = 0; k < d; ++k) a[1 + k] = tmp[d - 1 - k];
}

__global__ void k_compact(const int32_t* __restrict__ flag, const int32_t* __restrict__ off, int n,
                          int32_t* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (flag[k]) out[off[k]] = k;
}

// §4: centre, radius (largest chord distance to a corner) and the (p+1)^2
// proxy points of every cell; proxies stored [cell][3][KS], zero padded.
// The box of every cell (xi_mid, eta_mid, half_xi, half_eta): its cell, or
// with shrinking (paper §3, the remark on nonuniform particles) the smallest
// (xi, eta) rectangle holding its points, each half width at least
// kShrinkFloor of the cell's.  One block per cell reduces its points' angles.
constexpr double kShrinkFloor = 1.0 / 1048576.0;  // 2^-20
__global__ __launch_bounds__(128) void k_cell_box(
    int n, const int32_t* __restrict__ level, const int32_t* __restrict__ ci,
    const int32_t* __restrict__ cj, const int32_t* __restrict__ begin,
    const int32_t* __restrict__ count, const double* __restrict__ xi,
    const double* __restrict__ eta, bool shrink, double* __restrict__ box) {
    __shared__ double red[4][128];
    const int c = blockIdx.x;
    if (c >= n) return;
    const double d = kPi2 / double(1u << level[c]);
    const double half = 0.5 * d;
    double xm = -kPi4 + (double(ci[c]) + 0.5) * d, ym = -kPi4 + (double(cj[c]) + 0.5) * d;
    double hx = half, hy = half;
    const int b = begin[c], m = count[c];
    if (shrink && m > 0) {
        double lo_x = xi[b], hi_x = xi[b], lo_y = eta[b], hi_y = eta[b];
        for (int k = threadIdx.x; k < m; k += blockDim.x) {
            lo_x = fmin(lo_x, xi[b + k]);
            hi_x = fmax(hi_x, xi[b + k]);
            lo_y = fmin(lo_y, eta[b + k]);
            hi_y = fmax(hi_y, eta[b + k]);
        }
        red[0][threadIdx.x] = lo_x;
        red[1][threadIdx.x] = hi_x;
        red[2][threadIdx.x] = lo_y;
        red[3][threadIdx.x] = hi_y;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w) {
                red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + w]);
                red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
                red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + w]);
                red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + w]);
            }
            __syncthreads();
        }
        xm = 0.5 * (red[0][0] + red[1][0]);
        hx = fmax(0.5 * (red[1][0] - red[0][0]), kShrinkFloor * half);
        ym = 0.5 * (red[2][0] + red[3][0]);
        hy = fmax(0.5 * (red[3][0] - red[2][0]), kShrinkFloor * half);
    }
    if (threadIdx.x == 0) {
        box[4 * int64_t(c)] = xm;
        box[4 * int64_t(c) + 1] = ym;
        box[4 * int64_t(c) + 2] = hx;
        box[4 * int64_t(c) + 3] = hy;
    }
}

__global__ void k_cell_geometry(int n, const int32_t* __restrict__ face,
                                const double* __restrict__ box, int p, int KS,
                                double* __restrict__ center, double* __restrict__ radius,
                                double* __restrict__ prox) {
#pragma clang fp contract(off)
    const int c = blockIdx.x;
    if (c >= n) return;
    const int f = face[c];
    const double xm = box[4 * int64_t(c)], ym = box[4 * int64_t(c) + 1];
    const double hx = box[4 * int64_t(c) + 2], hy = box[4 * int64_t(c) + 3];
    __shared__ double cen[3];
    if (threadIdx.x == 0) {
        gnomonic(f, xm, ym, cen);
        double r = 0.0;
        for (int q = 0; q < 4; ++q) {
            const double sx = (q >> 1) ? 1.0 : -1.0, sy = (q & 1) ? 1.0 : -1.0;
            double v[3];
            gnomonic(f, xm + hx * sx, ym + hy * sy, v);
            const double dx = v[0] - cen[0], dy = v[1] - cen[1], dz = v[2] - cen[2];
            r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz));
        }
        center[3 * c] = cen[0];
        center[3 * c + 1] = cen[1];
        center[3 * c + 2] = cen[2];
        radius[c] = r;
    }
    const int K = (p + 1) * (p + 1);
    double* pc = prox + int64_t(c) * 3 * KS;
    for (int k = threadIdx.x; k < KS; k += blockDim.x) {
        if (k < K) {
            const int k1 = k / (p + 1), k2 = k % (p + 1);
            const double s1 = cos(double(k1) * kPi / double(p));
            const double s2 = cos(double(k2) * kPi / double(p));
            double v[3];
            gnomonic(f, xm + hx * s1, ym + hy * s2, v);
            pc[k] = v[0];
            pc[KS + k] = v[1];
            pc[2 * KS + k] = v[2];
        } else {
            pc[k] = 0.0;
            pc[KS + k] = 0.0;
            pc[2 * KS + k] = 0.0;
        }
    }
}

// Local coordinates (u, v) in [-1,1]^2 of every point in its leaf's box (§4),
// and the leaf's gap: a lower bound on the geodesic distance from its points to
// the leaf's boundary.  The cell edges xi = const and eta = const are great
// circles; a point at angle xi on its face lies at sin-distance
// rho_a sin(xi - xi0) from the circle xi = xi0, rho_a^2 = (1 + A^2)/(1 + A^2 +
// B^2), A = tan xi, B = tan eta (and likewise for eta), and the geodesic
// distance is at least its sine.  Two points in leaves that do not overlap
// (cells are convex) are then at least gap_T + gap_S apart along the sphere.
__global__ void k_leaf_local(const int32_t* __restrict__ leaves, int nleaves,
                             const int32_t* __restrict__ level, const int32_t* __restrict__ ci,
                             const int32_t* __restrict__ cj, const int32_t* __restrict__ begin,
                             const int32_t* __restrict__ count, const double* __restrict__ xi,
                             const double* __restrict__ eta, const double* __restrict__ box,
                             double* __restrict__ u, double* __restrict__ v,
                             double* __restrict__ gap) {
    __shared__ unsigned gmin;
    const int L = blockIdx.x;
    if (L >= nleaves) return;
    if (threadIdx.x == 0) gmin = 0x7f800000u;  // +inf
    __syncthreads();
    const int c = leaves[L];
    const double d = kPi2 / double(1u << level[c]);
    const double half = 0.5 * d;
    const double xm = -kPi4 + (double(ci[c]) + 0.5) * d;
    const double ym = -kPi4 + (double(cj[c]) + 0.5) * d;
    const int b = begin[c], m = count[c];
    const double bxm = box[4 * int64_t(c)], bym = box[4 * int64_t(c) + 1];
    const double bhx = box[4 * int64_t(c) + 2], bhy = box[4 * int64_t(c) + 3];
    for (int k = threadIdx.x; k < m; k += blockDim.x) {
        // local coordinates in the box; the gap is to the cell's edges
        u[b + k] = (xi[b + k] - bxm) / bhx;
        v[b + k] = (eta[b + k] - bym) / bhy;
        const double uu = (xi[b + k] - xm) / half, vv = (eta[b + k] - ym) / half;
        const double A = tan(xi[b + k]), B = tan(eta[b + k]);
        const double q = 1.0 + A * A + B * B;
        const double ga = sqrt((1.0 + A * A) / q) * sin(fmax(0.0, 1.0 - fabs(uu)) * half);
        const double gb = sqrt((1.0 + B * B) / q) * sin(fmax(0.0, 1.0 - fabs(vv)) * half);
        // rounded down to FP32 (a lower bound); bits of non-negative floats order
        float g = float(fmax(0.0, fmin(ga, gb)));
        if (g > 0.f && double(g) > fmin(ga, gb)) g = __uint_as_float(__float_as_uint(g) - 1u);
        atomicMin(&gmin, __float_as_uint(g));
    }
    __syncthreads();
    if (threadIdx.x == 0) gap[c] = m > 0 ? double(__uint_as_float(gmin)) : 0.0;
}

// §4 barycentric Lagrange L_k(x) at the Chebyshev points, exact hit -> delta.
__device__ double lagrange1(int p, int k, double x) {
    double num = 0.0, den = 0.0;
    for (int m = 0; m <= p; ++m) {
        const double s = cos(double(m) * kPi / double(p));
        double b = (m & 1) ? -1.0 : 1.0;
        if (m == 0 || m == p) b *= 0.5;
        const double dx = x - s;
        if (dx == 0.0) return m == k ? 1.0 : 0.0;
        const double t = b / dx;
        den += t;
        if (m == k) num = t;
    }
    return num / den;
}

// Fixed operators of eq. (upwardpass2) and eq. (downward_2): with
// A_s[m][k] = L_k((s_m + s)/2) (parent polynomial k at child node m, s = -1, +1),
// child q = 2*bi + bj has T_q[k][m] = A_{2bi-1}[m1][k1] A_{2bj-1}[m2][k2].
//   A1d[bi][m][k] = A_{2bi-1}[m][k]  (the 1-D factors; L2L applies them as two
//                                     1-D passes in the leaf kernel)
//   bm2m[q*KS + m][k] = T_q[k][m]   (M2M: parent = rows of children x bm2m)
__global__ void k_build_ops(int p, int KS, int nb1, double* __restrict__ A1d,
                            double* __restrict__ bm2m) {
    const int P1 = p + 1, K = P1 * P1;
    for (int t = threadIdx.x; t < 2 * P1 * P1; t += blockDim.x) {
        const int sgn = t / (P1 * P1), r = t % (P1 * P1);
        const int m = r / P1, k = r % P1;
        const double s = cos(double(m) * kPi / double(p));
        A1d[t] = lagrange1(p, k, (s + (sgn ? 1.0 : -1.0)) * 0.5);
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < int64_t(4) * KS * nb1; t += blockDim.x) {
        const int row = int(t / nb1), k = int(t % nb1);
        const int q = row / KS, m = row % KS;
        double val = 0.0;
        if (m < K && k < K) {
            const int bi = q >> 1, bj = q & 1;
            val = A1d[bi * K + (m / P1) * P1 + (k / P1)] * A1d[bj * K + (m % P1) * P1 + (k % P1)];
        }
        bm2m[t] = val;
    }
}

// Shrinking: the 1-D factors of the parent-to-child operator of every cell
// below a root, A_c[dim][m][k] = L_k^P((mid_c + half_c s_m - mid_P)/half_P),
// the parent's polynomial k at the child's node m in the parent's box
// (dim 0: xi, 1: eta); the non-shrunk plans use the two fixed factors.
__global__ void k_cell_ops(int n, int p, const int32_t* __restrict__ parent,
                           const double* __restrict__ box, double* __restrict__ ops) {
    const int P1 = p + 1, K = P1 * P1;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= int64_t(n) * 2 * K) return;
    const int c = int(t / (2 * K)), r = int(t % (2 * K));
    const int dim = r / K, m = (r % K) / P1, k = r % P1;
    const int par = parent[c];
    double val = 0.0;
    if (par >= 0) {
        const double s = cos(double(m) * kPi / double(p));
        const double x = box[4 * int64_t(c) + dim] + box[4 * int64_t(c) + 2 + dim] * s;
        val = lagrange1(p, k, (x - box[4 * int64_t(par) + dim]) / box[4 * int64_t(par) + 2 + dim]);
    }
    ops[t] = val;
}

// ------------------------------------------------------------- traversal
// Action codes of one (T, S) pair.
enum { A_NONE = 0, A_PP = 1, A_PC = 2, A_CP = 3, A_CC = 4, A_SPLIT_T = 5, A_SPLIT_S = 6 };

struct TravTree {
    const int32_t *level, *count, *child0;
    const double *center, *radius;
};

__global__ void k_classify(const int32_t* __restrict__ ft, const int32_t* __restrict__ fs, int n,
                           TravTree T, TravTree S, double theta, int32_t* __restrict__ act,
                           int32_t* __restrict__ c0, int32_t* __restrict__ c1,
                           int32_t* __restrict__ c2, int32_t* __restrict__ c3,
                           int32_t* __restrict__ c4) {
#pragma clang fp contract(off)
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int t = ft[k], s = fs[k];
    int a = A_NONE;
    if (T.count[t] > 0 && S.count[s] > 0) {
        const bool lt = T.child0[t] < 0, ls = S.child0[s] < 0;
        const bool both = lt && ls;
        bool sep = false;
        if (!both) {
            const double rs = T.radius[t] + S.radius[s];
            const double dx = T.center[3 * t] - S.center[3 * s];
            const double dy = T.center[3 * t + 1] - S.center[3 * s + 1];
            const double dz = T.center[3 * t + 2] - S.center[3 * s + 2];
            const double R2 = dx * dx + dy * dy + dz * dz;
            sep = rs * rs < (theta * theta) * R2;
        }
        if (!both && sep)
            a = lt ? A_PC : (ls ? A_CP : A_CC);
        else if (!both)
            a = (!lt && (ls || T.level[t] <= S.level[s])) ? A_SPLIT_T : A_SPLIT_S;
        else
            a = A_PP;
    }
    act[k] = a;
    c0[k] = a == A_PP;
    c1[k] = a == A_PC;
    c2[k] = a == A_CP;
    c3[k] = a == A_CC;
    c4[k] = (a == A_SPLIT_T || a == A_SPLIT_S) ? 4 : 0;
}

struct Caps {
    int32_t c[5];
};

__global__ void k_emit(const int32_t* __restrict__ ft, const int32_t* __restrict__ fs, int n,
                       const int32_t* __restrict__ act, const int32_t* __restrict__ o0,
                       const int32_t* __restrict__ o1, const int32_t* __restrict__ o2,
                       const int32_t* __restrict__ o3, const int32_t* __restrict__ o4,
                       const int32_t* __restrict__ tchild0, const int32_t* __restrict__ schild0,
                       int32_t* __restrict__ l0t, int32_t* __restrict__ l0s,
                       int32_t* __restrict__ l1t, int32_t* __restrict__ l1s,
                       int32_t* __restrict__ l2t, int32_t* __restrict__ l2s,
                       int32_t* __restrict__ l3t, int32_t* __restrict__ l3s,
                       int32_t* __restrict__ nt, int32_t* __restrict__ ns, Caps cap) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int a = act[k];
    const int t = ft[k], s = fs[k];
    switch (a) {
        case A_PP: if (o0[k] < cap.c[0]) { l0t[o0[k]] = t; l0s[o0[k]] = s; } break;
        case A_PC: if (o1[k] < cap.c[1]) { l1t[o1[k]] = t; l1s[o1[k]] = s; } break;
        case A_CP: if (o2[k] < cap.c[2]) { l2t[o2[k]] = t; l2s[o2[k]] = s; } break;
        case A_CC: if (o3[k] < cap.c[3]) { l3t[o3[k]] = t; l3s[o3[k]] = s; } break;
        case A_SPLIT_T:
            if (o4[k] + 4 > cap.c[4]) break;
            for (int q = 0; q < 4; ++q) {
                nt[o4[k] + q] = tchild0[t] + q;
                ns[o4[k] + q] = s;
            }
            break;
        case A_SPLIT_S:
            if (o4[k] + 4 > cap.c[4]) break;
            for (int q = 0; q < 4; ++q) {
                nt[o4[k] + q] = t;
                ns[o4[k] + q] = schild0[s] + q;
            }
            break;
        default: break;
    }
}

__global__ void k_root_pairs(int32_t* ft, int32_t* fs) {
    const int k = threadIdx.x;
    if (k < 36) {
        ft[k] = k / 6;
        fs[k] = k % 6;
    }
}

struct CellIds {
    const int32_t *level, *face, *ci, *cj;
};

// Two cells overlap when one contains the other (same face, same ancestor at
// the coarser level); only then can they hold coincident points.
__device__ __forceinline__ bool cells_overlap(const CellIds& A, int a, const CellIds& B, int b) {
    if (A.face[a] != B.face[b]) return false;
    const int la = A.level[a], lb = B.level[b];
    const int l = la < lb ? la : lb;
    return (A.ci[a] >> (la - l)) == (B.ci[b] >> (lb - l)) &&
           (A.cj[a] >> (la - l)) == (B.cj[b] >> (lb - l));
}

// PP entries of non-overlapping leaves whose points may come close (FP32 form).
// The expanded squared distance |t|^2 + |s|^2 - 2 t.s of two points recentred
// at a cell centre errs by a few FP32 ulps of |t|^2 + |s|^2 =
// (|t + s|^2 + d^2)/2, d = |t - s|, and |t + s| <= 2 r + d for t in a cell of
// radius r about the centre: its relative error is a few ulps of
// (1 + (1 + 2 r/d)^2)/2.  With d at least the chord of gap_T + gap_S and r
// the larger radius (so that the class is the same for (T, S) and (S, T)),
// an entry is close when 2 r/d may exceed kCloseRatio, i.e. when the ratio
// may exceed 256 (a relative error of about 1e-4 of d^2 at most); such
// entries take exact differences.  Leaves of a uniform grid (points at least
// 1/8 of a half width from the edges) stay below it; random points do not.
constexpr double kCloseRatio = 21.6;
struct CloseGeom {
    const double *gap_t, *gap_s, *rad_t, *rad_s;
};
__device__ __forceinline__ bool pp_close(const CloseGeom& G, int t, int s) {
    const double dmin = 2.0 * sin(0.5 * fmin(G.gap_t[t] + G.gap_s[s], kPi));
    const double r = fmax(G.rad_t[t], G.rad_s[s]);
    return 2.0 * r > kCloseRatio * dmin;
}

// Sort key of a (target, source) entry: by target, then (PP only) the
// overlapping entries, the close ones (classify_close) and the others, then by
// source:  t*3ns + class*ns + s.
// Sort key of list entry k: base + target * 3 ns + class * ns + source (class
// 0 overlapping, 1 close, 2 other; only PP entries are classed); `base`
// places the four lists one after the other in one sort.
__global__ void k_pair_keys(const int32_t* __restrict__ t, const int32_t* __restrict__ s, int64_t n,
                            int64_t ns_cells, bool mark_overlap, bool classify_close, CellIds TC,
                            CellIds SC, CloseGeom G, uint64_t base, uint64_t* __restrict__ keys,
                            int32_t* __restrict__ vals) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const bool ovl = mark_overlap && cells_overlap(TC, t[k], SC, s[k]);
    const int cls = ovl ? 0 : ((classify_close && pp_close(G, t[k], s[k])) ? 1 : 2);
    keys[k] = base + uint64_t(t[k]) * uint64_t(3 * ns_cells) + uint64_t(cls) * uint64_t(ns_cells) +
              uint64_t(s[k]);
    vals[k] = int32_t(k);
}

// CSR of one list from its sorted keys (with the list's `base` removed: base
// is a multiple of 3 ns, so the source is the key mod ns as before)
__global__ void k_csr_from_keys(const uint64_t* __restrict__ keys, int64_t n, int64_t ns_cells,
                                int nt_cells, uint64_t base, int32_t* __restrict__ off,
                                int32_t* __restrict__ src, int32_t* __restrict__ novl,
                                int32_t* __restrict__ ncl) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t ns3 = uint64_t(3 * ns_cells), ns1 = uint64_t(ns_cells);
    if (k < n) src[k] = int32_t((keys[k] % ns3) % ns1);
    if (k <= nt_cells) {
        const int64_t b = lower_bound_u64(keys, 0, n, base + uint64_t(k) * ns3);
        off[k] = int32_t(b);
        if (novl && k < nt_cells) {
            const int64_t b1 = lower_bound_u64(keys, b, n, base + uint64_t(k) * ns3 + ns1);
            const int64_t b2 = lower_bound_u64(keys, b1, n, base + uint64_t(k) * ns3 + 2 * ns1);
            novl[k] = int32_t(b1 - b);
            ncl[k] = int32_t(b2 - b1);
        }
    }
}

// n_close += ncl[t] over the target cells
__global__ void k_sum_i32(const int32_t* __restrict__ a, int n, unsigned long long* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && a[k] != 0) atomicAdd(out, (unsigned long long)a[k]);
}

__global__ void k_far_flags(const int32_t* __restrict__ ocp, const int32_t* __restrict__ occ, int n,
                            int32_t* __restrict__ flag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    flag[k] = (ocp[k + 1] > ocp[k] || occ[k + 1] > occ[k]) ? 1 : 0;
}

// ------------------------------------------------------------- host helpers

#define RC(x)                              \
    do {                                   \
        int rc_ = (x);                     \
        if (rc_ != CSFMM_OK) return rc_;   \
    } while (0)

int read_i32(const int32_t* d, int32_t* h, hipStream_t s) {
    CSFMM_HIP_TRY(hipMemcpyAsync(h, d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CSFMM_HIP_TRY(hipStreamSynchronize(s));
    return CSFMM_OK;
}

// Build one tree over n points (device AoS coordinates).
int build_tree(csfmm_plan_s* P, Tree& T, const double* pts, int64_t n, hipStream_t s) {
    DevArena& A = P->arena;
    Scratch S(s);
    T.n = n;
    uint64_t* keys;
    int32_t* idx;
    double *xi0, *eta0, *xi, *eta;
    RC(S.get(&keys, n));
    RC(S.get(&idx, n));
    RC(S.get(&xi0, n));
    RC(S.get(&eta0, n));
    RC(S.get(&xi, n));
    RC(S.get(&eta, n));
    k_face_key<<<nblk(n), kT, 0, s>>>(pts, n, keys, idx, xi0, eta0);
    CSFMM_LAUNCH_CHECK();
    RC(radix_sort_u64(keys, idx, n, 3 + 2 * kMaxLevel, S, s));
    {
        ArenaGroup G;
        G.add(&T.x, n);
        G.add(&T.y, n);
        G.add(&T.z, n);
        G.add(&T.u, n);
        G.add(&T.v, n);
        G.add(&T.perm, n);
        RC(G.commit(A));
    }
    k_gather_points<<<nblk(n), kT, 0, s>>>(pts, idx, xi0, eta0, n, T.x, T.y, T.z, xi, eta);
    CSFMM_LAUNCH_CHECK();
    CSFMM_HIP_TRY(hipMemcpyAsync(T.perm, idx, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));

    // levels, breadth first
    struct Lev {
        int32_t n;
        int32_t *face, *ci, *cj, *begin, *count, *child0;
    };
    std::vector<Lev> levs;
    Lev L0{6};
    RC(S.get(&L0.face, 6));
    RC(S.get(&L0.ci, 6));
    RC(S.get(&L0.cj, 6));
    RC(S.get(&L0.begin, 6));
    RC(S.get(&L0.count, 6));
    RC(S.get(&L0.child0, 6));
    k_roots<<<1, 64, 0, s>>>(keys, n, L0.face, L0.ci, L0.cj, L0.begin, L0.count);
    CSFMM_LAUNCH_CHECK();
    levs.push_back(L0);
    int32_t* dtot;
    RC(S.get(&dtot, 1));
    int32_t total_cells = 6;
    for (int l = 0;; ++l) {
        Lev& cur = levs.back();
        int32_t *flag, *off;
        RC(S.get(&flag, cur.n));
        RC(S.get(&off, cur.n));
        k_split_flags<<<nblk(cur.n), kT, 0, s>>>(cur.count, cur.n, P->leaf, l, flag);
        CSFMM_LAUNCH_CHECK();
        RC(scan_exclusive_i32(flag, off, cur.n, dtot, S, s));
        int32_t nsplit = 0;
        RC(read_i32(dtot, &nsplit, s));
        Lev nx{4 * nsplit};
        if (nsplit > 0) {
            RC(S.get(&nx.face, nx.n));
            RC(S.get(&nx.ci, nx.n));
            RC(S.get(&nx.cj, nx.n));
            RC(S.get(&nx.begin, nx.n));
            RC(S.get(&nx.count, nx.n));
            RC(S.get(&nx.child0, nx.n));
        }
        k_children<<<nblk(cur.n), kT, 0, s>>>(keys, cur.n, l, flag, off, cur.face, cur.ci, cur.cj,
                                              cur.begin, cur.count, total_cells, nx.n, cur.child0,
                                              nx.face, nx.ci, nx.cj, nx.begin, nx.count);
        CSFMM_LAUNCH_CHECK();
        if (nsplit == 0) break;
        if (int64_t(total_cells) + nx.n > (int64_t(1) << 30)) {
            set_error("tree too large");
            return CSFMM_E_INVALID;
        }
        total_cells += nx.n;
        levs.push_back(nx);
    }
    T.depth = int32_t(levs.size()) - 1;
    T.ncells = total_cells;
    T.level_begin.assign(levs.size() + 1, 0);
    for (size_t l = 0; l < levs.size(); ++l) T.level_begin[l + 1] = T.level_begin[l] + levs[l].n;
    const int nc = T.ncells;
    const bool shrink = (P->flags & CSFMM_SHRINK) != 0;
    {
        ArenaGroup G;
        G.add(&T.level, nc);
        G.add(&T.face, nc);
        G.add(&T.ci, nc);
        G.add(&T.cj, nc);
        G.add(&T.begin, nc);
        G.add(&T.count, nc);
        G.add(&T.child0, nc);
        G.add(&T.parent, nc);
        G.add(&T.box, int64_t(4) * nc);
        G.add(&T.center, int64_t(3) * nc);
        G.add(&T.radius, nc);
        G.add(&T.prox, int64_t(3) * P->KS * nc);
        G.add(&T.gap, nc);
        if (shrink) G.add(&T.ops, int64_t(nc) * 2 * (P->p + 1) * (P->p + 1));
        RC(G.commit(A));
    }
    // cells of all levels in one array each; leaves and parents (non-leaf
    // cells, grouped by level)
    int32_t *lf, *pf, *lo, *po;
    RC(S.get(&lf, nc));
    RC(S.get(&pf, nc));
    RC(S.get(&lo, nc));
    RC(S.get(&po, nc));
    {
        if (levs.size() > size_t(kMaxLevel + 1)) {
            set_error("tree deeper than %d levels", kMaxLevel);
            return CSFMM_E_INTERNAL;
        }
        LevelArrays L{};
        L.nlev = int32_t(levs.size());
        for (size_t l = 0; l < levs.size(); ++l) {
            L.first[l] = T.level_begin[l];
            L.face[l] = levs[l].face;
            L.ci[l] = levs[l].ci;
            L.cj[l] = levs[l].cj;
            L.begin[l] = levs[l].begin;
            L.count[l] = levs[l].count;
            L.child0[l] = levs[l].child0;
        }
        L.first[levs.size()] = nc;
        k_gather_levels<<<nblk(nc), kT, 0, s>>>(L, nc, T.level, T.face, T.ci, T.cj, T.begin,
                                                T.count, T.child0, T.parent, lf, pf);
        CSFMM_LAUNCH_CHECK();
    }
    {
        const int32_t* fin[2] = {lf, pf};
        int32_t* fout[2] = {lo, po};
        RC(scan_exclusive_multi(fin, fout, 2, nc, dtot, S, s));
    }
    // the two totals and the parents' offset at each level start, in one read
    std::vector<int32_t> hpo(nc + 2);
    CSFMM_HIP_TRY(hipMemcpyAsync(hpo.data(), po, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    CSFMM_HIP_TRY(hipMemcpyAsync(hpo.data() + nc, dtot, sizeof(int32_t) * 2,
                                 hipMemcpyDeviceToHost, s));
    CSFMM_HIP_TRY(hipStreamSynchronize(s));
    const int32_t nleaves = hpo[nc], nparents = hpo[nc + 1];
    T.parents_begin.assign(levs.size() + 1, nparents);
    for (size_t l = 0; l < levs.size(); ++l) T.parents_begin[l] = hpo[T.level_begin[l]];
    T.nleaves = nleaves;
    {
        ArenaGroup G;
        G.add(&T.leaves, nleaves);
        G.add(&T.parents, nparents);
        G.add(&T.leaf_anc, int64_t(nleaves) * kAncStride);
        RC(G.commit(A));
    }
    k_compact<<<nblk(nc), kT, 0, s>>>(lf, lo, nc, T.leaves);
    k_compact<<<nblk(nc), kT, 0, s>>>(pf, po, nc, T.parents);
    CSFMM_LAUNCH_CHECK();
    k_leaf_paths<<<nblk(nleaves), kT, 0, s>>>(T.leaves, nleaves, T.parent, T.leaf_anc);
    CSFMM_LAUNCH_CHECK();

    // boxes (cells, or shrunk), geometry and proxies
    k_cell_box<<<nc, 128, 0, s>>>(nc, T.level, T.ci, T.cj, T.begin, T.count, xi, eta, shrink,
                                  T.box);
    CSFMM_LAUNCH_CHECK();
    k_cell_geometry<<<nc, 128, 0, s>>>(nc, T.face, T.box, P->p, P->KS, T.center, T.radius,
                                       T.prox);
    CSFMM_LAUNCH_CHECK();
    k_fill_f64<<<nblk(nc), kT, 0, s>>>(T.gap, nc, 0.0);
    k_leaf_local<<<nleaves, 128, 0, s>>>(T.leaves, nleaves, T.level, T.ci, T.cj, T.begin, T.count,
                                         xi, eta, T.box, T.u, T.v, T.gap);
    CSFMM_LAUNCH_CHECK();
    if (shrink) {
        const int64_t K = int64_t(P->p + 1) * (P->p + 1);
        k_cell_ops<<<nblk(int64_t(nc) * 2 * K), kT, 0, s>>>(nc, P->p, T.parent, T.box, T.ops);
        CSFMM_LAUNCH_CHECK();
    }
    return CSFMM_OK;
}

int build_lists(csfmm_plan_s* P, hipStream_t s) {
    Tree& T = P->tt;
    Tree& Sx = *P->st;
    DevArena& A = P->arena;
    Scratch S(s);
    TravTree tt{T.level, T.count, T.child0, T.center, T.radius};
    TravTree st{Sx.level, Sx.count, Sx.child0, Sx.center, Sx.radius};

    // the four lists grow in place: each traversal step appends its pairs of
    // each kind, and a full buffer moves to one of twice the size
    struct Grow {
        int32_t *t = nullptr, *s = nullptr;
        int64_t n = 0, cap = 0;
    };
    Grow out[4];
    const int64_t cap0 = 16 * int64_t(std::max(T.ncells, Sx.ncells)) + 1024;
    for (int k = 0; k < 4; ++k) {
        RC(S.get(&out[k].t, cap0));
        RC(S.get(&out[k].s, cap0));
        out[k].cap = cap0;
    }
    int32_t *ft, *fs;
    int32_t nf = 36;
    RC(S.get(&ft, nf));
    RC(S.get(&fs, nf));
    k_root_pairs<<<1, 64, 0, s>>>(ft, fs);
    CSFMM_LAUNCH_CHECK();
    int32_t* dtot;
    RC(S.get(&dtot, 8));
    for (int iter = 0; nf > 0; ++iter) {
        if (iter > 4 * kMaxLevel + 8) {
            set_error("traversal did not terminate");
            return CSFMM_E_HIP;
        }
        int32_t *act, *c[5], *o[5];
        RC(S.get(&act, nf));
        for (int k = 0; k < 5; ++k) {
            RC(S.get(&c[k], nf));
            RC(S.get(&o[k], nf));
        }
        k_classify<<<nblk(nf), kT, 0, s>>>(ft, fs, nf, tt, st, P->theta, act, c[0], c[1], c[2],
                                           c[3], c[4]);
        CSFMM_LAUNCH_CHECK();
        RC(scan_exclusive_multi(c, o, 5, nf, dtot, S, s));
        int32_t tot[5];
        CSFMM_HIP_TRY(hipMemcpyAsync(tot, dtot, sizeof(tot), hipMemcpyDeviceToHost, s));
        CSFMM_HIP_TRY(hipStreamSynchronize(s));
        for (int k = 0; k < 4; ++k) {
            Grow& g = out[k];
            if (g.n + tot[k] <= g.cap) continue;
            const int64_t cap = std::max<int64_t>(2 * g.cap, g.n + tot[k]);
            int32_t *t2, *s2;
            RC(S.get(&t2, cap));
            RC(S.get(&s2, cap));
            if (g.n > 0) {
                CSFMM_HIP_TRY(hipMemcpyAsync(t2, g.t, sizeof(int32_t) * g.n,
                                             hipMemcpyDeviceToDevice, s));
                CSFMM_HIP_TRY(hipMemcpyAsync(s2, g.s, sizeof(int32_t) * g.n,
                                             hipMemcpyDeviceToDevice, s));
            }
            g.t = t2;
            g.s = s2;
            g.cap = cap;
        }
        int32_t *nt, *ns;
        RC(S.get(&nt, tot[4]));
        RC(S.get(&ns, tot[4]));
        k_emit<<<nblk(nf), kT, 0, s>>>(ft, fs, nf, act, o[0], o[1], o[2], o[3], o[4], T.child0,
                                       Sx.child0, out[0].t + out[0].n, out[0].s + out[0].n,
                                       out[1].t + out[1].n, out[1].s + out[1].n,
                                       out[2].t + out[2].n, out[2].s + out[2].n,
                                       out[3].t + out[3].n, out[3].s + out[3].n, nt, ns,
                                       Caps{{tot[0], tot[1], tot[2], tot[3], tot[4]}});
        CSFMM_LAUNCH_CHECK();
        for (int k = 0; k < 4; ++k) out[k].n += tot[k];
        ft = nt;
        fs = ns;
        nf = tot[4];
    }

    // sort by (target, source), CSR by target cell
    const int64_t nsc = Sx.ncells;
    const int64_t maxkey = int64_t(T.ncells) * 3 * nsc;
    const CellIds tcid{T.level, T.face, T.ci, T.cj};
    const CellIds scid{Sx.level, Sx.face, Sx.ci, Sx.cj};
    const CloseGeom cg{T.gap, Sx.gap, T.radius, Sx.radius};
    const bool classify_close = (P->flags & CSFMM_FP32_FORM) != 0;
    {
        ArenaGroup G;
        G.add(&P->lists.novl, T.ncells);
        G.add(&P->lists.ncl, T.ncells);
        for (int k = 0; k < 4; ++k) {
            P->lists.cnt[k] = out[k].n;
            G.add(&P->lists.off[k], int64_t(T.ncells) + 1);
            G.add(&P->lists.src[k], out[k].n);
        }
        RC(G.commit(A));
    }
    // the four lists in one sort: list k's keys start at k * maxkey (a multiple
    // of 3 ns), so after the sort they are the run [first[k], first[k] + cnt[k])
    const bool one_sort = maxkey < (int64_t(1) << 60);
    int64_t first[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < 4; ++k) first[k + 1] = first[k] + out[k].n;
    const int64_t span = one_sort ? 4 * maxkey : maxkey;
    int bits = 1;
    while (bits < 63 && (int64_t(1) << bits) < span) ++bits;
    uint64_t* keys;
    int32_t* vals;
    RC(S.get(&keys, first[4]));
    RC(S.get(&vals, first[4]));
    for (int k = 0; k < 4; ++k) {
        const int64_t cnt = out[k].n;
        const uint64_t base = one_sort ? uint64_t(k) * uint64_t(maxkey) : 0;
        if (cnt > 0) {
            k_pair_keys<<<nblk(cnt), kT, 0, s>>>(out[k].t, out[k].s, cnt, nsc, k == kPP,
                                                 k == kPP && classify_close, tcid, scid, cg,
                                                 base, keys + first[k], vals + first[k]);
            CSFMM_LAUNCH_CHECK();
            if (!one_sort) RC(radix_sort_u64(keys + first[k], vals + first[k], cnt, bits, S, s));
        }
    }
    if (one_sort) RC(radix_sort_u64(keys, vals, first[4], bits, S, s));
    for (int k = 0; k < 4; ++k) {
        const int64_t cnt = out[k].n;
        const uint64_t base = one_sort ? uint64_t(k) * uint64_t(maxkey) : 0;
        const int64_t m = std::max<int64_t>(cnt, int64_t(T.ncells) + 1);
        k_csr_from_keys<<<nblk(m), kT, 0, s>>>(keys + first[k], cnt, nsc, T.ncells, base,
                                               P->lists.off[k], P->lists.src[k],
                                               k == kPP ? P->lists.novl : nullptr,
                                               k == kPP ? P->lists.ncl : nullptr);
        CSFMM_LAUNCH_CHECK();
    }
    // target cells with far-field (CP or CC) work
    int32_t *ff, *fo;
    RC(S.get(&ff, T.ncells));
    RC(S.get(&fo, T.ncells));
    k_far_flags<<<nblk(T.ncells), kT, 0, s>>>(P->lists.off[kCP], P->lists.off[kCC], T.ncells, ff);
    CSFMM_LAUNCH_CHECK();
    RC(scan_exclusive_i32(ff, fo, T.ncells, dtot, S, s));

    // evaluation counts of the four lists (integer sums on the device)
    unsigned long long* dev_ev;
    RC(S.get(&dev_ev, 6));
    k_zero_u64<<<1, 6, 0, s>>>(dev_ev, 6);
    k_sum_i32<<<nblk(T.ncells), kT, 0, s>>>(P->lists.ncl, T.ncells, dev_ev + 5);
    for (int k = 0; k < 4; ++k) {
        k_count_evals<<<nblk(T.ncells), kT, 0, s>>>(k, P->lists.off[k], P->lists.src[k], T.count,
                                                     Sx.count, T.ncells, P->K, P->same ? 1 : 0,
                                                     dev_ev + k);
    }
    // and the largest target leaf (selects the near-field tile path)
    k_max_leaf<<<nblk(T.nleaves), kT, 0, s>>>(T.leaves, T.nleaves, T.count, dev_ev + 4);
    CSFMM_LAUNCH_CHECK();

    // symmetric split of the PP entries (same-set plans): kinds and their
    // scans now, the fill after the read
    const bool sym = P->same;
    const int nc = T.ncells;
    const int64_t ne = P->lists.cnt[kPP];
    int32_t *ko = nullptr, *kr = nullptr, *k1 = nullptr, *rev = nullptr;
    int32_t *eo = nullptr, *er = nullptr, *e1 = nullptr;
    if (sym) {
        RC(S.get(&ko, ne + 1));
        RC(S.get(&kr, ne + 1));
        RC(S.get(&k1, ne + 1));
        RC(S.get(&rev, ne + 1));
        RC(S.get(&eo, ne + 1));
        RC(S.get(&er, ne + 1));
        RC(S.get(&e1, ne + 1));
        k_zero_i32x3<<<1, 1, 0, s>>>(ko + ne, kr + ne, k1 + ne);
        k_sym_kinds<<<nblk(int64_t(nc) * 64), kT, 0, s>>>(nc, P->lists.off[kPP], P->lists.src[kPP],
                                                          P->lists.novl, P->lists.ncl, ko, kr, k1,
                                                          rev);
        CSFMM_LAUNCH_CHECK();
        const int32_t* kin[3] = {ko, kr, k1};
        int32_t* kout[3] = {eo, er, e1};
        RC(scan_exclusive_multi(kin, kout, 3, ne + 1, dtot + 1, S, s));
    }

    // one read: far targets, the sym totals, the evaluation counts
    struct {
        int32_t tot[4];
        unsigned long long ev[6];
    } h;
    CSFMM_HIP_TRY(hipMemcpyAsync(h.tot, dtot, sizeof(h.tot), hipMemcpyDeviceToHost, s));
    CSFMM_HIP_TRY(hipMemcpyAsync(h.ev, dev_ev, sizeof(h.ev), hipMemcpyDeviceToHost, s));
    CSFMM_HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < 4; ++k) P->lists.evals[k] = int64_t(h.ev[k]);
    T.max_leaf = int32_t(h.ev[4]);
    P->lists.n_close = int64_t(h.ev[5]);
    const int32_t nfar = h.tot[0];
    P->lists.n_far_targets = nfar;
    SymPP& Y = P->lists.sym;
    {
        ArenaGroup G;
        G.add(&P->lists.far_targets, nfar);
        if (sym) {
            if (h.tot[1] != h.tot[2]) {
                set_error("symmetric PP pairs: %d owned but %d received", h.tot[1], h.tot[2]);
                return CSFMM_E_INTERNAL;
            }
            Y.n_own = h.tot[1];
            Y.n_one = h.tot[3];
            G.add(&Y.own_off, int64_t(nc) + 1);
            G.add(&Y.recv_off, int64_t(nc) + 1);
            G.add(&Y.one_off, int64_t(nc) + 1);
            G.add(&Y.own_src, Y.n_own);
            G.add(&Y.recv_slot, Y.n_own);
            G.add(&Y.one_src, Y.n_one);
        }
        RC(G.commit(A));
    }
    k_compact<<<nblk(T.ncells), kT, 0, s>>>(ff, fo, T.ncells, P->lists.far_targets);
    CSFMM_LAUNCH_CHECK();
    if (sym) {
        k_sym_fill<<<nblk(std::max<int64_t>(ne, int64_t(nc) + 1)), kT, 0, s>>>(
            nc, ne, P->lists.off[kPP], P->lists.src[kPP], ko, kr, k1, rev, eo, er, e1, Y.own_off,
            Y.own_src, Y.recv_off, Y.recv_slot, Y.one_off, Y.one_src);
        CSFMM_LAUNCH_CHECK();
        Y.on = true;
    }
    return CSFMM_OK;
}

}  // namespace

int build_plan(csfmm_plan_s* P, const double* targets, const double* sources, hipStream_t s) {
    DevArena& A = P->arena;
    {
        Scratch S(s);
        int* bad;
        RC(S.get(&bad, 1));
        CSFMM_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), s));
        k_check_points<<<nblk(P->nt), kT, 0, s>>>(targets, P->nt, bad);
        CSFMM_LAUNCH_CHECK();
        if (!P->same) {
            k_check_points<<<nblk(P->ns), kT, 0, s>>>(sources, P->ns, bad);
            CSFMM_LAUNCH_CHECK();
        }
        int hbad = 0;
        CSFMM_HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        CSFMM_HIP_TRY(hipStreamSynchronize(s));
        if (hbad) {
            set_error("a point is not finite or not on the unit sphere (| |x| - 1 | > 1e-12)");
            return CSFMM_E_NOT_ON_SPHERE;
        }
    }
    RC(build_tree(P, P->tt, targets, P->nt, s));
    if (P->same) {
        P->st = &P->tt;
    } else {
        RC(build_tree(P, P->st_own, sources, P->ns, s));
        P->st = &P->st_own;
    }
    // fixed interpolation operators
    P->nb1 = int(round_up(P->KS, 16));
    {
        ArenaGroup G;
        G.add(&P->lag1d, 2 * (P->p + 1) * (P->p + 1));
        G.add(&P->bm2m, int64_t(4) * P->KS * P->nb1);
        RC(G.commit(A));
    }
    k_build_ops<<<1, 256, 0, s>>>(P->p, P->KS, P->nb1, P->lag1d, P->bm2m);
    CSFMM_LAUNCH_CHECK();
    RC(build_lists(P, s));
    // the plan's own eval workspace
    RC(workspace_create(P, s, &P->ws0));
    CSFMM_HIP_TRY(hipStreamSynchronize(s));
    return CSFMM_OK;
}

}  // namespace csfmm
