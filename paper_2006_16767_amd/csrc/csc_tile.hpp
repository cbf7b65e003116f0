// Merge-path tiles over a sparse x and the effective entries of its
// columns (the load-balanced distribution of the column-major pattern).
//
// excl[0..nnz_x] is the exclusive prefix of the selected column lengths, so
// entry e of x owns effective positions [excl[e], excl[e+1]) and
// excl[nnz_x] = nnz_s. The merge of entry ends and positions is cut into
// tiles of kCscTile items; a tile stages the entries it touches in LDS and
// maps each of its positions back to (entry, CSC index) by a binary search
// in LDS.
#pragma once

#include "common.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kCscIpt = 8;
constexpr int kCscTile = kBlock * kCscIpt;


template <int DT>
struct CscTileLds {
    int32_t excl[kCscTile + 1];
    int32_t cs[kCscTile + 1];
    typename SR<DT>::X v[kCscTile + 1];
    int32_t bound[4];
};

struct CscTile {
    int e0, p0, e1, p1, ecount;
};

// Finds the tile's bounds and stages its entries. Ends with __syncthreads.
template <int DT>
__device__ __forceinline__ CscTile csc_tile_setup(int64_t tile, int32_t nnz_x, int64_t nnz_s,
                                                  const int32_t* __restrict__ x_idx,
                                                  const typename SR<DT>::X* __restrict__ x_val,
                                                  const int32_t* __restrict__ col_ptr,
                                                  const Excl excl, CscTileLds<DT>& L) {
    using S = SR<DT>;
    const int64_t total = (int64_t)nnz_x + nnz_s;
    const int64_t d0 = tile * kCscTile;
    const int64_t d1 = d0 + kCscTile < total ? d0 + kCscTile : total;
    auto ends = [&](int e) { return excl[e + 1]; };
    if (wave_id() < 2) {
        const int64_t d = wave_id() == 0 ? d0 : d1;
        const int e = merge_search_wave(ends, nnz_x, d);
        if (lane_id() == 0) {
            L.bound[wave_id() * 2 + 0] = e;
            L.bound[wave_id() * 2 + 1] = (int)(d - e);
        }
    }
    __syncthreads();
    CscTile t;
    t.e0 = L.bound[0];
    t.p0 = L.bound[1];
    t.e1 = L.bound[2];
    t.p1 = L.bound[3];
    const int elast = t.e1 < nnz_x - 1 ? t.e1 : nnz_x - 1;
    t.ecount = elast - t.e0 + 1;
    for (int u = threadIdx.x; u < t.ecount; u += kBlock) {
        const int e = t.e0 + u;
        L.excl[u] = excl[e];
        L.cs[u] = col_ptr[x_idx[e]];
        L.v[u] = S::kVals ? x_val[e] : (typename S::X)1;
    }
    __syncthreads();
    return t;
}

// Staged entry that owns position p (the last one whose prefix start <= p).
template <int DT>
__device__ __forceinline__ int csc_tile_locate(int p, const CscTile& t, const CscTileLds<DT>& L) {
    int lo = 0, hi = t.ecount - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.excl[mid] <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int DT>
struct EmitAtomic {
    typename SR<DT>::Y* y;
    __device__ void operator()(int r, typename SR<DT>::Acc v, int64_t) const {
        SR<DT>::atomic_add(&y[r], v);
    }
};

// excl[0..nnz_x]: exclusive prefix of the selected column lengths (excl[nnz_x]
// = nnz_s). Tiles are taken grid-stride until the merge length is covered.
template <int DT, typename Emit>
__device__ __forceinline__ void csc_merge_tile(int64_t tile, int32_t nnz_x, int64_t nnz_s,
                                               const int32_t* __restrict__ x_idx,
                                               const typename SR<DT>::X* __restrict__ x_val,
                                               const int32_t* __restrict__ col_ptr,
                                               const int32_t* __restrict__ row_idx,
                                               const typename SR<DT>::V* __restrict__ vals,
                                               const Excl excl, const Emit& emit, CscTileLds<DT>& L) {
    using S = SR<DT>;
    const CscTile t = csc_tile_setup<DT>(tile, nnz_x, nnz_s, x_idx, x_val, col_ptr, excl, L);
    for (int p = t.p0 + threadIdx.x; p < t.p1; p += kBlock) {
        const int u = csc_tile_locate<DT>(p, t, L);
        const int k = L.cs[u] + (p - L.excl[u]);
        emit(row_idx[k], S::mul(S::val(vals, k), L.v[u]), p);
    }
    __syncthreads();
}

// Direct distribution: a group of L lanes walks the column of entry e.
// excl (optional) gives each entry's prefix position for pair emission.
template <int DT, int L, typename Emit>
__device__ __forceinline__ void csc_direct_entry(int e, int g, const int32_t* __restrict__ x_idx,
                                                 const typename SR<DT>::X* __restrict__ x_val,
                                                 const int32_t* __restrict__ col_ptr,
                                                 const int32_t* __restrict__ row_idx,
                                                 const typename SR<DT>::V* __restrict__ vals,
                                                 const Excl excl, const Emit& emit) {
    using S = SR<DT>;
    const int j = x_idx[e];
    const typename S::X v = S::kVals ? x_val[e] : (typename S::X)1;
    const int c0 = col_ptr[j], c1 = col_ptr[j + 1];
    const int64_t pbase = excl ? (int64_t)excl[e] - c0 : 0;
    int k = c0 + g;
    for (; k + 3 * L < c1; k += 4 * L) {
        int r[4];
        typename S::V a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            r[u] = row_idx[k + u * L];
            a[u] = S::val(vals, k + u * L);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) emit(r[u], S::mul(a[u], v), pbase + k + u * L);
    }
    for (; k < c1; k += L) emit(row_idx[k], S::mul(S::val(vals, k), v), pbase + k);
}

}  // namespace spx
