// Merge-path tile of the row-major kernels (SpMV and bitvector-validated
// SpMSpV), shared by the single-vector kernel and the batched persistent
// kernel.
#pragma once

#include "common.hpp"

namespace spx {

// Workgroup b -> tile: each of the 8 XCDs (workgroups are dispatched to
// them round-robin) gets one contiguous range of tiles, so neighbouring
// tiles, which share x entries on matrices with locality, meet in the same
// L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
    constexpr int kXcd = 8;
    const int64_t x = b % kXcd, j = b / kXcd;
    const int64_t base = G / kXcd, rem = G % kXcd;
    return x * base + (x < rem ? x : rem) + j;
}

constexpr int kShortRow = 32;

// Products of the tile's nonzeros into LDS, written as straight-line phases
// so that every load of a phase is in flight before the first is used: all
// column indices, then (validation) all bitvector words, then the values
// and x entries, then the LDS stores. Items past Q use a clamped, valid
// index and are not stored. xf(c) returns x_c (a global load, or an LDS
// read for the columns a kernel keeps there).
template <int DT, bool VALID, int IPT, int NT, typename XF>
__device__ __forceinline__ void csr_stage_products(int k0, int Q, const int32_t* __restrict__ col_idx,
                                                   const typename SR<DT>::V* __restrict__ vals, XF xf,
                                                   const uint32_t* __restrict__ bits,
                                                   typename SR<DT>::Acc* __restrict__ prod) {
    using S = SR<DT>;
    int kk[IPT], c[IPT];
    bool on[IPT];
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int q = it * NT + threadIdx.x;
        on[it] = q < Q;
        kk[it] = k0 + (on[it] ? q : 0);
    }
    if (Q == 0) return;
#pragma unroll
    for (int it = 0; it < IPT; ++it) c[it] = col_idx[kk[it]];
    if constexpr (VALID) {
        uint32_t w[IPT];
#pragma unroll
        for (int it = 0; it < IPT; ++it) w[it] = bits[c[it] >> 5];
#pragma unroll
        for (int it = 0; it < IPT; ++it) on[it] = on[it] && ((w[it] >> (c[it] & 31)) & 1u);
        typename S::V a[IPT];
        typename S::X b[IPT];
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            a[it] = on[it] ? S::val(vals, kk[it]) : (typename S::V)0;
            b[it] = on[it] ? xf(c[it]) : (typename S::X)0;
        }
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            const int q = it * NT + threadIdx.x;
            if (q < Q) prod[q] = on[it] ? S::mul(a[it], b[it]) : S::zero();
        }
    } else {
        typename S::V a[IPT];
        typename S::X b[IPT];
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
            a[it] = S::val(vals, kk[it]);
            b[it] = xf(c[it]);
        }
#pragma unroll
        for (int it = 0; it < IPT; ++it)
            if (on[it]) prod[it * NT + threadIdx.x] = S::mul(a[it], b[it]);
    }
}

// A tile's LDS. A row longer than kShortRow within the tile takes more than
// kShortRow of its TILE items, so at most TILE / (kShortRow + 1) rows are
// long: lng needs no more (which keeps the tile at 16.4 KB for TILE = 2048
// and FP32, eight 256-thread workgroups per CU).
template <int DT, int TILE>
struct CsrTileLds {
    int32_t end[TILE + 1];
    typename SR<DT>::Acc prod[TILE];
    int32_t lng[TILE / (kShortRow + 1) + 1];
    int32_t nlong;
};

// One tile, NT threads: stage the products of its nonzeros in LDS (stage(k0,
// Q, prod) writes prod[q] for the tile's items q < Q in row order), then
// reduce every row whose end falls in the tile from LDS: short rows by one
// thread, rows longer than kShortRow by a whole wave. The row still open
// at the tile end leaves a carry for the fix-up pass (carry_row = -1 if
// none). Ends with __syncthreads.
template <int DT, int TILE, int NT, typename StageFn>
__device__ __forceinline__ void csr_merge_tile_core(int64_t tile, int32_t m, const int32_t* __restrict__ row_ptr,
                                                    typename SR<DT>::Y* __restrict__ y,
                                                    const int32_t* __restrict__ part, int32_t* __restrict__ carry_row,
                                                    typename SR<DT>::Acc* __restrict__ carry_val,
                                                    CsrTileLds<DT, TILE>& L, StageFn stage) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    constexpr int kWaves = NT / kWave;
    const int i0 = part[2 * tile], k0 = part[2 * tile + 1];
    const int i1 = part[2 * tile + 2], k1 = part[2 * tile + 3];
    const int R = i1 - i0;  // rows whose end lies in this tile
    const int Q = k1 - k0;  // nonzeros of this tile
    const bool open = i1 < m && k1 > row_ptr[i1];
    if (threadIdx.x == 0) L.nlong = 0;
    for (int r = threadIdx.x; r < R; r += NT) L.end[r] = row_ptr[i0 + 1 + r];
    stage(k0, Q, L.prod);
    __syncthreads();
    const int nrows = R + (open ? 1 : 0);
    for (int r = threadIdx.x; r < nrows; r += NT) {
        const int a = (r == 0 ? k0 : L.end[r - 1]) - k0;
        const int e = (r < R ? L.end[r] : k1) - k0;
        if (e - a <= kShortRow) {
            Acc acc = S::zero();
            for (int q = a; q < e; ++q) acc = S::add(acc, L.prod[q]);
            if (r < R) {
                y[i0 + r] = S::out(acc);
            } else {
                carry_row[tile] = i1;
                carry_val[tile] = acc;
            }
        } else {
            L.lng[atomicAdd(&L.nlong, 1)] = r;
        }
    }
    __syncthreads();
    const int nl = L.nlong;
    for (int li = wave_id(); li < nl; li += kWaves) {
        const int r = L.lng[li];
        const int a = (r == 0 ? k0 : L.end[r - 1]) - k0;
        const int e = (r < R ? L.end[r] : k1) - k0;
        Acc acc = S::zero();
        for (int q = a + lane_id(); q < e; q += kWave) acc = S::add(acc, L.prod[q]);
        acc = group_reduce<DT, kWave>(acc);
        if (lane_id() == 0) {
            if (r < R) {
                y[i0 + r] = S::out(acc);
            } else {
                carry_row[tile] = i1;
                carry_val[tile] = acc;
            }
        }
    }
    if (!open && threadIdx.x == 0) carry_row[tile] = -1;
    __syncthreads();
}

// The tile over the row-ordered entries, x read through xf.
template <int DT, bool VALID, int TILE, int NT, typename XF>
__device__ __forceinline__ void csr_merge_tile_nt(int64_t tile, int32_t m, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx,
                                                  const typename SR<DT>::V* __restrict__ vals, XF xf,
                                                  const uint32_t* __restrict__ bits,
                                                  typename SR<DT>::Y* __restrict__ y,
                                                  const int32_t* __restrict__ part, int32_t* __restrict__ carry_row,
                                                  typename SR<DT>::Acc* __restrict__ carry_val,
                                                  CsrTileLds<DT, TILE>& L) {
    csr_merge_tile_core<DT, TILE, NT>(tile, m, row_ptr, y, part, carry_row, carry_val, L,
                                      [&](int k0, int Q, typename SR<DT>::Acc* prod) {
                                          csr_stage_products<DT, VALID, TILE / NT, NT>(k0, Q, col_idx, vals, xf,
                                                                                       bits, prod);
                                      });
}

// Column-sorted tiles: inside each 2048-item merge tile the entries are
// ordered by column, so that the 64 gathers of a wave meet fewer cache
// lines, and each entry's word holds its column (low kTsColBits bits) and
// its position in the tile in row order (the bits above), where its product
// goes. The reduction then runs on row-ordered products as above.
constexpr int kTsColBits = 21;
constexpr uint32_t kTsColMask = (1u << kTsColBits) - 1u;
template <int DT, bool VALID, int IPT, int NT>
__device__ __forceinline__ void csr_stage_sorted(int k0, int Q, const uint32_t* __restrict__ pk,
                                                 const typename SR<DT>::V* __restrict__ vals,
                                                 const typename SR<DT>::X* __restrict__ x,
                                                 const uint32_t* __restrict__ bits,
                                                 typename SR<DT>::Acc* __restrict__ prod) {
    using S = SR<DT>;
    if (Q == 0) return;
    uint32_t w[IPT];
    int kk[IPT];
    bool on[IPT];
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int q = it * NT + threadIdx.x;
        on[it] = q < Q;
        kk[it] = k0 + (on[it] ? q : 0);
    }
#pragma unroll
    for (int it = 0; it < IPT; ++it) w[it] = pk[kk[it]];
    bool ok[IPT];
    if constexpr (VALID) {
        uint32_t bw[IPT];
#pragma unroll
        for (int it = 0; it < IPT; ++it) bw[it] = bits[(w[it] & kTsColMask) >> 5];
#pragma unroll
        for (int it = 0; it < IPT; ++it) ok[it] = (bw[it] >> (w[it] & 31u)) & 1u;
    } else {
#pragma unroll
        for (int it = 0; it < IPT; ++it) ok[it] = true;
    }
    typename S::V a[IPT];
    typename S::X b[IPT];
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        a[it] = ok[it] ? S::val(vals, kk[it]) : (typename S::V)0;
        b[it] = ok[it] ? S::xval(x, (int64_t)(w[it] & kTsColMask)) : (typename S::X)0;
    }
#pragma unroll
    for (int it = 0; it < IPT; ++it)
        if (on[it]) prod[w[it] >> kTsColBits] = ok[it] ? S::mul(a[it], b[it]) : S::zero();
}

// The tile with kBlock threads and x read from global memory.
template <int DT, bool VALID, int TILE>
__device__ __forceinline__ void csr_merge_tile(int64_t tile, int32_t m, const int32_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col_idx,
                                               const typename SR<DT>::V* __restrict__ vals,
                                               const typename SR<DT>::X* __restrict__ x,
                                               const uint32_t* __restrict__ bits,
                                               typename SR<DT>::Y* __restrict__ y,
                                               const int32_t* __restrict__ part, int32_t* __restrict__ carry_row,
                                               typename SR<DT>::Acc* __restrict__ carry_val,
                                               CsrTileLds<DT, TILE>& L) {
    csr_merge_tile_nt<DT, VALID, TILE, kBlock>(
        tile, m, row_ptr, col_idx, vals, [x](int c) { return SR<DT>::xval(x, c); }, bits, y, part, carry_row,
        carry_val, L);
}

// Carries of tiles whose last row continues, added in tile order by the
// first tile of each run of equal carry_row (deterministic). Threads of the
// calling group take tiles t = first, first + stride, ...
template <int DT>
__device__ __forceinline__ void csr_merge_fixup_range(int64_t first, int64_t stride, int64_t tiles,
                                                      const int32_t* __restrict__ carry_row,
                                                      const typename SR<DT>::Acc* __restrict__ carry_val,
                                                      typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    for (int64_t t = first; t < tiles; t += stride) {
        const int row = carry_row[t];
        if (row < 0) continue;
        if (t > 0 && carry_row[t - 1] == row) continue;
        typename S::Acc acc = S::zero();
        for (int64_t u = t; u < tiles && carry_row[u] == row; ++u) acc = S::add(acc, carry_val[u]);
        if constexpr (DT == SPX_BOOL) {
            if (acc) y[row] = 1;
        } else {
            y[row] = S::out(S::add((typename S::Acc)y[row], acc));
        }
    }
}

}  // namespace spx
