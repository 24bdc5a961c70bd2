// Small device helpers shared by the kernels (wave64, 256-thread blocks).
#pragma once

#include <hip/hip_runtime.h>

namespace csfmm {

// Inclusive scan of one int over a 256-thread block (4 waves of 64 lanes).
__device__ __forceinline__ int block_scan_incl_256(int v, int* lds_wave /*[4]*/) {
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

// Workgroups are dispatched round robin over the 8 XCDs of an MI355X; this
// bijection gives each XCD a contiguous range of logical block ids, so that
// neighbouring (Morton-ordered) cells share one XCD's L2.
__device__ __forceinline__ int xcd_logical_block(int bid, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = bid & 7, k = bid >> 3;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// The same for a grid of two kinds of work, nf blocks of the first kind and
// nb - nf of the second: every XCD gets its share of each kind (a contiguous
// range of each), first-kind blocks first.  Sets `first` and returns the
// index within the kind.
__device__ __forceinline__ int xcd_split_block(int bid, int nb, int nf, bool& first) {
    const int q = nb >> 3, r = nb & 7;
    const int qf = nf >> 3, rf = nf & 7;
    const int x = bid & 7, k = bid >> 3;
    const int fx = qf + (x < rf ? 1 : 0);
    first = k < fx;
    if (first) return x * qf + min(x, rf) + k;
    return x * q + min(x, r) - (x * qf + min(x, rf)) + (k - fx);
}

}  // namespace csfmm
