// The walk of a sparse x's columns restricted to one block of rows (the
// bucket write-back of Section 4.2.2 without pair buffers): a workgroup
// owns rows [lo, hi) in LDS, groups of G lanes take x entries, and every
// entry of a selected column whose row falls in the block is handed to the
// caller's add(). Rows ascend within a CSC column, so a long column is cut
// to the block by two searches in which the group probes G points per step;
// short columns are read whole, G entries per step.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kWalkScan = 32;  // with G = 1 a thread reads columns up to this length whole
constexpr int kWalkU = 8;      // row indices a lane has in flight while it reads a column

// First position in [a, b) whose row is >= key (b if none), rows ascending:
// the G lanes of a group probe G interior points of the interval per step
// (G = 1 is the binary search). Every lane of the group gets the result;
// the group must be converged.
template <int G>
__device__ __forceinline__ int group_lower_bound(const int32_t* __restrict__ rows, int a, int b, int key) {
    const int lane = threadIdx.x % G;
    const int shift = (lane_id() / G) * G;  // the group's bits in the wave's ballot
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1);
    int lo = a, hi = b;
    while (lo < hi) {
        const int64_t span = hi - lo;
        const int p = lo + (int)((span * (lane + 1)) / (G + 1));  // in [lo, hi)
        const uint64_t m = (__ballot(rows[p] >= key) >> shift) & gmask;
        if (!m) {
            lo += (int)((span * G) / (G + 1)) + 1;  // every probe is below key
        } else {
            const int f = __ffsll((unsigned long long)m) - 1;
            const int lo0 = lo;
            hi = lo0 + (int)((span * (f + 1)) / (G + 1));
            if (f > 0) lo = lo0 + (int)((span * f) / (G + 1)) + 1;
        }
    }
    return lo;
}

// nthreads threads of the workgroup (threadIdx.x < nthreads, a multiple of
// G) walk the nnz_x entries of x; add(r - lo, k, x value) is called for
// every CSC position k of a selected column whose row r is in [lo, hi).
template <int DT, int G, typename Add>
__device__ __forceinline__ void walk_columns(int nthreads, int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                             const typename SR<DT>::X* __restrict__ x_val,
                                             const int32_t* __restrict__ col_ptr,
                                             const int32_t* __restrict__ row_idx, int lo, int hi,
                                             const Add& add) {
    using S = SR<DT>;
    constexpr int kScan = G == 1 ? kWalkScan : 4 * G;  // read whole up to this length
    const int lane = threadIdx.x % G;
    // the loop is uniform across each group of G lanes
    for (int e = threadIdx.x / G; e < nnz_x; e += nthreads / G) {
        const int j = x_idx[e];
        const typename S::X v = S::kVals ? x_val[e] : (typename S::X)1;
        int k0 = col_ptr[j], k1 = col_ptr[j + 1];
        if (k1 - k0 > kScan) {
            k0 = group_lower_bound<G>(row_idx, k0, k1, lo);
            k1 = group_lower_bound<G>(row_idx, k0, k1, hi);
        }
        // kWalkU row indices of a lane in flight at once (a lane's positions
        // past k1 read the column's last entry and are dropped), so a column
        // costs len / (G * kWalkU) round trips, not len / G
        for (int kb = k0 + lane; kb < k1; kb += G * kWalkU) {
            int r[kWalkU];
#pragma unroll
            for (int u = 0; u < kWalkU; ++u) r[u] = row_idx[min(kb + u * G, k1 - 1)];
#pragma unroll
            for (int u = 0; u < kWalkU; ++u) {
                const int k = kb + u * G;
                if (k < k1 && r[u] >= lo && r[u] < hi) add(r[u] - lo, k, v);
            }
        }
    }
}

}  // namespace spx
