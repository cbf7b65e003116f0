// Row-major kernels (Section 4.1): SpMV, and SpMSpV with value validation
// against a bitvector of supp(x) (Section 6.1). Both with the two workload
// distributions of Section 4.2.1:
//
//  * direct   - a fixed group of L lanes per row (L = 1 is the classic
//               thread-per-row kernel; L = 64 a whole wave per row). The
//               group strides through the row, each lane keeps a partial sum
//               and the group reduces with cross-lane shuffles.
//  * balanced - merge-path tiles: the merge of row ends and nonzeros is cut
//               into equal pieces of kTile items, so every workgroup gets
//               the same amount of (rows + nonzeros) whatever the row-length
//               distribution. A tile stages its products in LDS with
//               coalesced loads; each thread then walks kIpt merge items,
//               partial sums that cross thread boundaries are combined with a
//               segmented scan, and a row that spans tiles is finished by a
//               small fix-up pass in tile order (deterministic).
//
// With validation (the CSR SpMSpV pattern) a product is formed only where
// bit(col) is set; x values are read from the scattered copy xd, so neither
// vals[k] nor xd[col] is touched for ineffective entries. For BOOL the
// product is the bit itself.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

// --------------------------------------------------------------- direct
template <int DT, int L, bool VALID>
__global__ __launch_bounds__(kBlock) void k_csr_direct(int32_t m, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx,
                                                       const typename SR<DT>::V* __restrict__ vals,
                                                       const typename SR<DT>::X* __restrict__ x,
                                                       const uint32_t* __restrict__ bits,
                                                       typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    constexpr int kRowsPerBlock = kBlock / L;
    const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / L;
    const int g = threadIdx.x % L;
    if (row >= m) return;  // whole groups leave together (L divides 64)
    const int k0 = row_ptr[row], k1 = row_ptr[row + 1];
    Acc acc = S::zero();
    int k = k0 + g;
    // four independent gathers in flight per lane
    for (; k + 3 * L < k1; k += 4 * L) {
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = col_idx[k + u * L];
        if constexpr (VALID) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (test_bit(bits, c[u])) acc = S::fma(S::val(vals, k + u * L), S::xval(x, c[u]), acc);
        } else {
            typename S::V a[4];
            typename S::X b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = S::val(vals, k + u * L);
                b[u] = S::xval(x, c[u]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = S::fma(a[u], b[u], acc);
        }
    }
    for (; k < k1; k += L) {
        const int c = col_idx[k];
        if constexpr (VALID) {
            if (test_bit(bits, c)) acc = S::fma(S::val(vals, k), S::xval(x, c), acc);
        } else {
            acc = S::fma(S::val(vals, k), S::xval(x, c), acc);
        }
    }
    acc = group_reduce<DT, L>(acc);
    if (g == 0) y[row] = S::out(acc);
}

// --------------------------------------------------------------- balanced
constexpr int kMergeIpt = 8;
constexpr int kMergeTile = kBlock * kMergeIpt;

template <int DT, bool VALID>
__global__ __launch_bounds__(kBlock) void k_csr_merge(int32_t m, int32_t nnz,
                                                      const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col_idx,
                                                      const typename SR<DT>::V* __restrict__ vals,
                                                      const typename SR<DT>::X* __restrict__ x,
                                                      const uint32_t* __restrict__ bits,
                                                      typename SR<DT>::Y* __restrict__ y,
                                                      int32_t* __restrict__ carry_row,
                                                      typename SR<DT>::Acc* __restrict__ carry_val) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    __shared__ int32_t s_end[kMergeTile + 1];  // row_ptr[i0 + 1 + r]
    __shared__ Acc s_prod[kMergeTile];
    __shared__ Acc s_row[kMergeTile];
    __shared__ int32_t s_key[kBlock];
    __shared__ Acc s_cv[kBlock];
    __shared__ int32_t s_bound[4];

    const int64_t total = (int64_t)m + nnz;
    const int64_t d0 = (int64_t)blockIdx.x * kMergeTile;
    const int64_t d1 = std::min<int64_t>(d0 + kMergeTile, total);
    auto ends = [&](int i) { return row_ptr[i + 1]; };
    if (wave_id() < 2) {
        const int64_t d = wave_id() == 0 ? d0 : d1;
        const int i = merge_search_wave(ends, m, d);
        if (lane_id() == 0) {
            s_bound[wave_id() * 2 + 0] = i;
            s_bound[wave_id() * 2 + 1] = (int)(d - i);
        }
    }
    __syncthreads();
    const int i0 = s_bound[0], k0 = s_bound[1], i1 = s_bound[2], k1 = s_bound[3];
    const int R = i1 - i0;   // rows whose end lies in this tile
    const int Q = k1 - k0;   // nonzeros consumed in this tile
    for (int r = threadIdx.x; r < R; r += kBlock) s_end[r] = row_ptr[i0 + 1 + r];
    for (int q = threadIdx.x; q < Q; q += kBlock) {
        const int k = k0 + q;
        const int c = col_idx[k];
        Acc p;
        if constexpr (VALID) {
            p = test_bit(bits, c) ? S::mul(S::val(vals, k), S::xval(x, c)) : S::zero();
        } else {
            p = S::mul(S::val(vals, k), S::xval(x, c));
        }
        s_prod[q] = p;
    }
    __syncthreads();

    // thread-level merge walk over kMergeIpt items
    const int tile_items = (int)(d1 - d0);
    const int dt = std::min((int)threadIdx.x * kMergeIpt, tile_items);
    const int dte = std::min(dt + kMergeIpt, tile_items);
    int r = merge_search_lds(s_end, R, dt, k0);
    int q = dt - r;
    const int r_start = r;
    Acc acc = S::zero();
    bool first_end = true;
    Acc first_val = S::zero();
    int first_row = -1;
    for (int it = dt; it < dte; ++it) {
        if (r < R && k0 + q >= s_end[r]) {
            if (first_end) {
                first_end = false;
                first_row = r;
                first_val = acc;
            } else {
                s_row[r] = acc;
            }
            acc = S::zero();
            ++r;
        } else {
            acc = S::add(acc, s_prod[q]);
            ++q;
        }
    }
    // carry-out: the partial sum of row r (still open at this thread's end)
    s_key[threadIdx.x] = r;
    s_cv[threadIdx.x] = acc;
    __syncthreads();
    // segmented inclusive scan of carries over threads (segments = equal key)
    for (int off = 1; off < kBlock; off <<= 1) {
        Acc add = S::zero();
        const int t = threadIdx.x;
        if (t >= off && s_key[t - off] == s_key[t]) add = s_cv[t - off];
        __syncthreads();
        s_cv[t] = S::add(s_cv[t], add);
        __syncthreads();
    }
    // carry-in of thread t = scanned carry of thread t-1 if it is open on the
    // row thread t started in (always true by continuity, unless t == 0)
    if (first_row >= 0) {
        Acc cin = S::zero();
        if (threadIdx.x > 0 && s_key[threadIdx.x - 1] == r_start) cin = s_cv[threadIdx.x - 1];
        s_row[first_row] = S::add(first_val, cin);
    }
    __syncthreads();
    for (int rr = threadIdx.x; rr < R; rr += kBlock) y[i0 + rr] = S::out(s_row[rr]);
    if (threadIdx.x == kBlock - 1) {
        // the row open at the tile end continues in the next tile
        const bool open = (i1 < m) && (k1 > row_ptr[i1]);
        carry_row[blockIdx.x] = open ? i1 : -1;
        carry_val[blockIdx.x] = open ? s_cv[kBlock - 1] : S::zero();
    }
}

// Adds the carries of tiles whose last row continues, in tile order. A row
// that spans several tiles appears as a run of equal carry_row; the first
// tile of the run sums the run and adds it to y (written by the tile that
// finished the row).
template <int DT>
__global__ __launch_bounds__(kBlock) void k_csr_merge_fixup(int32_t tiles,
                                                            const int32_t* __restrict__ carry_row,
                                                            const typename SR<DT>::Acc* __restrict__ carry_val,
                                                            typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= tiles) return;
    const int row = carry_row[t];
    if (row < 0) return;
    if (t > 0 && carry_row[t - 1] == row) return;
    typename S::Acc acc = S::zero();
    for (int u = t; u < tiles && carry_row[u] == row; ++u) acc = S::add(acc, carry_val[u]);
    if constexpr (DT == SPX_BOOL) {
        if (acc) y[row] = 1;
    } else {
        y[row] = S::out(S::add((typename S::Acc)y[row], acc));
    }
}

// --------------------------------------------------------------- launch
static int pick_lanes(int32_t m, int32_t nnz) {
    const double avg = m > 0 ? (double)nnz / m : 0.0;
    int L = 1;
    while (L < 64 && L < avg) L <<= 1;
    return L;
}

size_t spmv_csr_ws(int32_t m, int32_t nnz, const spx_plan* plan) {
    if (!plan || plan->distribution != SPX_DIST_BALANCED) return 0;
    const int64_t tiles = ceil_div((int64_t)m + nnz, kMergeTile);
    Sizer z;
    z.take<int32_t>(tiles);
    z.take<double>(tiles);
    return z.used;
}

template <int DT, bool VALID>
static spx_status launch_csr_t(const spx_csr* A, const void* x, const uint32_t* bits, void* y,
                               const spx_plan* plan, Arena& ws, hipStream_t s) {
    using S = SR<DT>;
    const auto* vals = (const typename S::V*)A->vals;
    const auto* xv = (const typename S::X*)x;
    auto* yv = (typename S::Y*)y;
    if (A->m == 0) return SPX_OK;
    if (plan->distribution == SPX_DIST_DIRECT) {
        int L = plan->lanes > 0 ? plan->lanes : pick_lanes(A->m, A->nnz);
        const int64_t blocks = ceil_div(A->m, kBlock / L);
        switch (L) {
#define SPX_L(LL)                                                                                   \
    case LL:                                                                                        \
        k_csr_direct<DT, LL, VALID><<<(unsigned)blocks, kBlock, 0, s>>>(A->m, A->row_ptr,           \
                                                                        A->col_idx, vals, xv, bits, yv); \
        break;
            SPX_L(1)
            SPX_L(2)
            SPX_L(4)
            SPX_L(8)
            SPX_L(16)
            SPX_L(32)
            SPX_L(64)
#undef SPX_L
            default:
                return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
        }
        SPX_HIP(hipGetLastError());
        return SPX_OK;
    }
    if (plan->distribution == SPX_DIST_BALANCED) {
        const int64_t tiles = ceil_div((int64_t)A->m + A->nnz, kMergeTile);
        int32_t* crow = ws.take<int32_t>(tiles);
        auto* cval = ws.take<typename S::Acc>(tiles);
        if (!crow || !cval) return fail(SPX_ERR_WORKSPACE, "spmv balanced: workspace too small");
        k_csr_merge<DT, VALID><<<(unsigned)tiles, kBlock, 0, s>>>(A->m, A->nnz, A->row_ptr, A->col_idx,
                                                                  vals, xv, bits, yv, crow, cval);
        SPX_HIP(hipGetLastError());
        k_csr_merge_fixup<DT><<<(unsigned)ceil_div(tiles, kBlock), kBlock, 0, s>>>((int32_t)tiles, crow,
                                                                                  cval, yv);
        SPX_HIP(hipGetLastError());
        return SPX_OK;
    }
    return fail(SPX_ERR_ARG, "unknown distribution");
}

spx_status launch_spmv_csr(const spx_csr* A, const void* x, const uint32_t* bits, void* y,
                           const spx_plan* plan, Arena& ws, hipStream_t s) {
    const bool valid = plan->pattern == SPX_PAT_CSR_SPMSPV;
    switch (A->dtype) {
#define SPX_DT(DT)                                                                            \
    case DT:                                                                                  \
        return valid ? launch_csr_t<DT, true>(A, x, bits, y, plan, ws, s)                     \
                     : launch_csr_t<DT, false>(A, x, bits, y, plan, ws, s);
        SPX_DT(SPX_F32)
        SPX_DT(SPX_F64)
        SPX_DT(SPX_I32)
        SPX_DT(SPX_BOOL)
#undef SPX_DT
    }
    return fail(SPX_ERR_DTYPE, "spmv: unknown dtype");
}

}  // namespace spx
