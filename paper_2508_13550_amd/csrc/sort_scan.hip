// Device-wide exclusive scan and stable LSD radix sort for wave64 (gfx950).
//
// Scan: up to 65,536 values in one launch (one 1024-thread workgroup per
// array walks the array in tiles of 8,192, carrying the running sum), beyond
// that three passes (block sums, scan of the block sums in one workgroup,
// block scans plus offsets).  Plan building runs many short scans (cells of a
// level, traversal frontiers, digit counts), where the launches, not the
// bytes, are the cost.  Sort: 8-bit digits; per pass a digit histogram per
// tile, a scan of the [digit][tile] counts, and a stable scatter in which each
// wavefront ranks equal digits with eight ballots.
#include "common.h"

namespace csfmm {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Inclusive scan of one int over a 256-thread block (4 waves of 64).
__device__ int block_inclusive_scan(int v, int* lds_wave /*[4]*/) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    if (lane == 63) lds_wave[wave] = v;
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wave; ++w) off += lds_wave[w];
    __syncthreads();
    return v + off;
}

// Small scans: one workgroup per array, tiles of kSmallTile values.
constexpr int kSmallThreads = 1024;
constexpr int kSmallItems = 8;
constexpr int kSmallTile = kSmallThreads * kSmallItems;
constexpr int64_t kSmallMax = int64_t(kSmallTile) * 8;
constexpr int kMaxArrays = 8;

struct ScanArrays {
    const int32_t* in[kMaxArrays];
    int32_t* out[kMaxArrays];
};

// Each thread scans its own kSmallItems consecutive values and writes only
// them, after reading them, so in == out is safe.
__global__ __launch_bounds__(kSmallThreads) void k_scan_small(ScanArrays a, int64_t n,
                                                              int32_t* __restrict__ totals) {
    __shared__ int lw[kSmallThreads / 64];
    const int32_t* in = a.in[blockIdx.x];
    int32_t* out = a.out[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int carry = 0;
    for (int64_t t0 = 0; t0 < n; t0 += kSmallTile) {
        const int64_t base = t0 + int64_t(threadIdx.x) * kSmallItems;
        int v[kSmallItems];
        int s = 0;
#pragma unroll
        for (int k = 0; k < kSmallItems; ++k) {
            v[k] = (base + k < n) ? in[base + k] : 0;
            s += v[k];
        }
        int inc = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        if (lane == 63) lw[wave] = inc;
        __syncthreads();
        int off = 0, tile = 0;
        for (int w = 0; w < kSmallThreads / 64; ++w) {
            const int x = lw[w];
            off += (w < wave) ? x : 0;
            tile += x;
        }
        __syncthreads();
        int run = carry + off + inc - s;
#pragma unroll
        for (int k = 0; k < kSmallItems; ++k) {
            if (base + k < n) out[base + k] = run;
            run += v[k];
        }
        carry += tile;
    }
    if (threadIdx.x == 0 && totals) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* __restrict__ in,
                                                               int64_t n, int32_t* __restrict__ sums) {
    __shared__ int lw[4];
    const int64_t base = int64_t(blockIdx.x) * kScanTile;
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + int64_t(k) * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = block_inclusive_scan(s, lw);
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(int32_t* __restrict__ sums, int64_t nb,
                                                             int32_t* __restrict__ total) {
    __shared__ int lw[4];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        int64_t i = b0 + threadIdx.x;
        int v = (i < nb) ? sums[i] : 0;
        int inc = block_inclusive_scan(v, lw);
        int c = carry;
        if (i < nb) sums[i] = c + inc - v;
        __syncthreads();
        if (threadIdx.x == kScanThreads - 1) carry = c + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t* __restrict__ in,
                                                              int32_t* __restrict__ out, int64_t n,
                                                              const int32_t* __restrict__ sums) {
    __shared__ int lw[4];
    const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        s += v[k];
    }
    int inc = block_inclusive_scan(s, lw);
    int run = sums[blockIdx.x] + inc - s;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// ------------------------------------------------------------------ radix sort
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const uint64_t* __restrict__ keys,
                                                              int64_t n, int shift, int64_t nb,
                                                              int32_t* __restrict__ hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + int64_t(k) * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(
    const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    int32_t* __restrict__ vout, int64_t n, int shift, int64_t nb,
    const int32_t* __restrict__ offs) {
    __shared__ int running[256];
    __shared__ int wcnt[4][256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    running[threadIdx.x] = offs[int64_t(threadIdx.x) * nb + blockIdx.x];
    for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    const unsigned long long below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int k = 0; k < kSortItems; ++k) {
        const int64_t i = base + int64_t(k) * kSortThreads + threadIdx.x;
        const bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        int32_t val = valid ? vin[i] : 0;
        const unsigned d = unsigned(key >> shift) & 255u;
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const int rank = __popcll(m & below);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(m);
        __syncthreads();
        if (valid) {
            int pos = running[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            if (pos >= 0 && pos < n) {
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
        {
            const int t = threadIdx.x;
            running[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
            wcnt[0][t] = 0;
            wcnt[1][t] = 0;
            wcnt[2][t] = 0;
            wcnt[3][t] = 0;
        }
        __syncthreads();
    }
}

}  // namespace

int scan_exclusive_multi(const int32_t* const* in, int32_t* const* out, int m, int64_t n,
                         int32_t* d_totals, Scratch& S, hipStream_t s) {
    if (m < 1 || m > kMaxArrays) {
        set_error("scan of %d arrays (1..%d)", m, kMaxArrays);
        return CSFMM_E_INTERNAL;
    }
    if (n <= 0) {
        if (d_totals) CSFMM_HIP_TRY(hipMemsetAsync(d_totals, 0, sizeof(int32_t) * m, s));
        return CSFMM_OK;
    }
    if (n <= kSmallMax) {
        ScanArrays a{};
        for (int k = 0; k < m; ++k) {
            a.in[k] = in[k];
            a.out[k] = out[k];
        }
        k_scan_small<<<dim3(unsigned(m)), dim3(kSmallThreads), 0, s>>>(a, n, d_totals);
        CSFMM_LAUNCH_CHECK();
        return CSFMM_OK;
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    for (int k = 0; k < m; ++k) {
        int32_t* sums = nullptr;
        int rc = S.get(&sums, nb);
        if (rc != CSFMM_OK) return rc;
        k_scan_reduce<<<dim3(unsigned(nb)), dim3(kScanThreads), 0, s>>>(in[k], n, sums);
        k_scan_sums<<<1, kScanThreads, 0, s>>>(sums, nb, d_totals ? d_totals + k : nullptr);
        k_scan_apply<<<dim3(unsigned(nb)), dim3(kScanThreads), 0, s>>>(in[k], out[k], n, sums);
        CSFMM_LAUNCH_CHECK();
    }
    return CSFMM_OK;
}

int scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* d_total,
                       Scratch& S, hipStream_t s) {
    return scan_exclusive_multi(&in, &out, 1, n, d_total, S, s);
}

int radix_sort_u64(uint64_t* keys, int32_t* vals, int64_t n, int bits, Scratch& S,
                   hipStream_t s) {
    if (n <= 1) return CSFMM_OK;
    const int passes = (bits + 7) / 8;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    uint64_t* k2 = nullptr;
    int32_t* v2 = nullptr;
    int32_t* hist = nullptr;
    int rc = S.get(&k2, n);
    if (rc == CSFMM_OK) rc = S.get(&v2, n);
    if (rc == CSFMM_OK) rc = S.get(&hist, 256 * nb);
    if (rc != CSFMM_OK) return rc;
    uint64_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    for (int p = 0; p < passes && rc == CSFMM_OK; ++p) {
        const int shift = 8 * p;
        k_digit_hist<<<dim3(unsigned(nb)), dim3(kSortThreads), 0, s>>>(ka, n, shift, nb, hist);
        rc = scan_exclusive_i32(hist, hist, 256 * nb, nullptr, S, s);
        if (rc != CSFMM_OK) break;
        k_digit_scatter<<<dim3(unsigned(nb)), dim3(kSortThreads), 0, s>>>(ka, va, kb, vb, n, shift,
                                                                          nb, hist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            set_error("radix sort launch failed: %s", hipGetErrorString(e));
            rc = CSFMM_E_HIP;
        }
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (rc == CSFMM_OK && ka != keys) {
        hipError_t e1 = hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s);
        hipError_t e2 = hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            set_error("radix sort copy-back failed");
            rc = CSFMM_E_HIP;
        }
    }
    return rc;
}

}  // namespace csfmm
