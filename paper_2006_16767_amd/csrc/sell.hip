// Sliced ELLPACK (SELL-C-sigma) and ELLPACK copies of A for the row-major
// SpMV: the storage formats beside CSR of the format pre-selection that the paper names
// as its extension (Section 8: choose the matrix format first, SMAT-style,
// then the kernel). The handle keeps the copy when the format tree
// (format_tree) prefers it.
//
// Layout: rows are sorted by descending length inside windows of
// kSellSigma = 4096 rows (stable), then cut into slices of C = 64 rows, one wave per slice,
// lane = row. A slice of width w (its longest row) stores its entries
// column-major: entry j of the row in lane l sits at slice_ptr[s] + 64 j + l,
// so each step of the wave reads 64 consecutive column indices and values
// (256 B each in FP32). Padding slots hold column -1. perm[slot] is the
// original row of a slot (-1 for the slots past m); src[slot] is the CSR
// position of its entry (-1 for padding), so a value refresh is one gather.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kSliceRows = 64;

// One thread per slot: the column indices and CSR positions of its row.
__global__ __launch_bounds__(kBlock) void k_sell_fill(int64_t slots, const int32_t* __restrict__ perm,
                                                      const int64_t* __restrict__ slice_ptr,
                                                      const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col_idx, int32_t* __restrict__ col,
                                                      int32_t* __restrict__ src) {
    const int64_t slot = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (slot >= slots) return;
    const int64_t s = slot / kSliceRows;
    const int lane = (int)(slot % kSliceRows);
    const int64_t base = slice_ptr[s];
    const int64_t w = (slice_ptr[s + 1] - base) / kSliceRows;
    const int row = perm[slot];
    const int32_t r0 = row >= 0 ? row_ptr[row] : 0;
    const int32_t len = row >= 0 ? row_ptr[row + 1] - r0 : 0;
    for (int64_t j = 0; j < w; ++j) {
        const int64_t pos = base + j * kSliceRows + lane;
        const bool on = j < len;
        col[pos] = on ? col_idx[r0 + j] : -1;
        src[pos] = on ? (int32_t)(r0 + j) : -1;
    }
}

// vals[pos] = csr_vals[src[pos]], 0 for padding.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sell_vals(int64_t total, const int32_t* __restrict__ src,
                                                      const T* __restrict__ csr_vals, T* __restrict__ vals) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < total; p += stride) {
        const int32_t k = src[p];
        vals[p] = k >= 0 ? csr_vals[k] : (T)0;
    }
}

// y = A x over the sliced copy: a wave per slice, a lane per row, the
// entries of a row accumulated in CSR order. Eight steps of the slice are
// loaded per round with the steps past the slice's width switched off, so
// a short slice (a stencil's 7) issues all its loads at once; the column
// and value loads of a round are independent.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_sell_spmv(int64_t nslices, const int64_t* __restrict__ slice_ptr,
                                                      const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ col,
                                                      const typename SR<DT>::V* __restrict__ vals,
                                                      const typename SR<DT>::X* __restrict__ x,
                                                      typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    constexpr int U = 8;
    const int64_t s = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (s >= nslices) return;
    const int lane = lane_id();
    const int64_t base = slice_ptr[s];
    const int w = (int)((slice_ptr[s + 1] - base) / kSliceRows);
    const int32_t* cp = col + base + lane;
    const int64_t vb = base + lane;
    ChunkedAcc<DT, U> acc;  // a partial sum per load slot: bounded chains on long rows
    for (int j = 0; j < w; j += U) {
        int c[U];
        typename S::V a[U];
        typename S::X b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = j + u < w ? cp[(int64_t)(j + u) * kSliceRows] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            a[u] = j + u < w ? S::val(vals, vb + (int64_t)(j + u) * kSliceRows) : (typename S::V)0;
#pragma unroll
        for (int u = 0; u < U; ++u) b[u] = c[u] >= 0 ? S::xval(x, c[u]) : (typename S::X)0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= 0) acc.part[u] = S::fma(a[u], b[u], acc.part[u]);
        acc.end_round();
    }
    const int row = perm[s * kSliceRows + lane];
    if (row >= 0) y[row] = S::out(acc.total());
}

SellPlanInfo sell_shape(const int32_t* row_ptr_host, int32_t m) {
    SellPlanInfo info;
    const int64_t ns = ceil_div((int64_t)m, kSliceRows);
    info.nslices = ns;
    info.perm.assign((size_t)(ns * kSliceRows), -1);
    info.slice_ptr.assign((size_t)ns + 1, 0);
    std::vector<int32_t> rows;
    for (int32_t w0 = 0; w0 < m; w0 += kSellSigma) {
        const int32_t w1 = std::min<int32_t>(m, w0 + kSellSigma);
        rows.resize((size_t)(w1 - w0));
        for (int32_t r = w0; r < w1; ++r) rows[(size_t)(r - w0)] = r;
        std::stable_sort(rows.begin(), rows.end(), [&](int32_t a, int32_t b) {
            return row_ptr_host[a + 1] - row_ptr_host[a] > row_ptr_host[b + 1] - row_ptr_host[b];
        });
        for (size_t i = 0; i < rows.size(); ++i) info.perm[(size_t)w0 + i] = rows[i];
    }
    for (int64_t s = 0; s < ns; ++s) {
        int32_t w = 0;
        for (int l = 0; l < kSliceRows; ++l) {
            const int32_t r = info.perm[(size_t)(s * kSliceRows + l)];
            if (r >= 0) w = std::max(w, row_ptr_host[r + 1] - row_ptr_host[r]);
        }
        info.slice_ptr[(size_t)s + 1] = info.slice_ptr[(size_t)s] + (int64_t)w * kSliceRows;
    }
    info.padded = info.slice_ptr[(size_t)ns];
    return info;
}

spx_status sell_build(const spx_csr& A, const SellPlanInfo& info, SellMat* out, hipStream_t s) {
    SellMat S;
    S.nslices = info.nslices;
    S.padded = info.padded;
    const int vs = value_size(A.dtype);
    const int64_t slots = info.nslices * kSliceRows;
    const size_t cells = (size_t)std::max<int64_t>(1, info.padded);
    if (hipMalloc((void**)&S.slice_ptr, info.slice_ptr.size() * 8) != hipSuccess ||
        hipMalloc((void**)&S.perm, (size_t)std::max<int64_t>(1, slots) * 4) != hipSuccess ||
        hipMalloc((void**)&S.col, cells * 4) != hipSuccess || hipMalloc((void**)&S.src, cells * 4) != hipSuccess ||
        (vs > 0 && hipMalloc(&S.vals, cells * vs) != hipSuccess)) {
        sell_free(&S);
        return fail(SPX_ERR_ALLOC, "sliced ELL allocation failed");
    }
    if (hipMemcpyAsync(S.slice_ptr, info.slice_ptr.data(), info.slice_ptr.size() * 8, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        (slots > 0 &&
         hipMemcpyAsync(S.perm, info.perm.data(), (size_t)slots * 4, hipMemcpyHostToDevice, s) != hipSuccess)) {
        sell_free(&S);
        return fail(SPX_ERR_HIP, "sliced ELL upload");
    }
    if (slots > 0) {
        k_sell_fill<<<(unsigned)ceil_div(slots, kBlock), kBlock, 0, s>>>(slots, S.perm, S.slice_ptr, A.row_ptr,
                                                                       A.col_idx, S.col, S.src);
        if (hipGetLastError() != hipSuccess) {
            sell_free(&S);
            return fail(SPX_ERR_HIP, "sliced ELL fill");
        }
    }
    // the host vectors above must stay alive until the uploads have run
    if (hipStreamSynchronize(s) != hipSuccess) {
        sell_free(&S);
        return fail(SPX_ERR_HIP, "sliced ELL build");
    }
    *out = S;
    return sell_refresh(*out, A, s);
}

spx_status sell_refresh(const SellMat& S, const spx_csr& A, hipStream_t s) {
    const int vs = value_size(A.dtype);
    if (vs == 0 || S.padded == 0) return SPX_OK;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(S.padded, kBlock), 8192));
    if (vs == 4)
        k_sell_vals<uint32_t><<<grid, kBlock, 0, s>>>(S.padded, S.src, (const uint32_t*)A.vals, (uint32_t*)S.vals);
    else
        k_sell_vals<uint64_t><<<grid, kBlock, 0, s>>>(S.padded, S.src, (const uint64_t*)A.vals, (uint64_t*)S.vals);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

void sell_free(SellMat* S) {
    void* ptrs[] = {S->slice_ptr, S->perm, S->col, S->src, S->vals};
    for (void* p : ptrs)
        if (p) hipFree(p);
    *S = SellMat{};
}

spx_status sell_spmv(const SellMat& S, int dtype, const void* x, void* y, hipStream_t s) {
    if (S.nslices == 0) return SPX_OK;
    const unsigned grid = (unsigned)ceil_div(S.nslices, kWavesPerBlock);
    switch (dtype) {
#define SPX_DT(DT)                                                                                              \
    case DT:                                                                                                    \
        k_sell_spmv<DT><<<grid, kBlock, 0, s>>>(S.nslices, S.slice_ptr, S.perm, S.col,                          \
                                                (const typename SR<DT>::V*)S.vals,                              \
                                                (const typename SR<DT>::X*)x, (typename SR<DT>::Y*)y);          \
        break;
        SPX_DT(SPX_F32)
        SPX_DT(SPX_F64)
        SPX_DT(SPX_I32)
        SPX_DT(SPX_BOOL)
        SPX_DT(SPX_F32_MINPLUS)
#undef SPX_DT
        default:
            return fail(SPX_ERR_DTYPE, "sliced ELL: unknown dtype");
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// ------------------------------------------------------------------ ELLPACK
// ELL copy of A: every row padded to the longest row w, stored column-major
// (entry j of row i at j * m + i, padding column -1), so that consecutive
// threads, one per row, read consecutive addresses at every step and y is
// written in row order. No row pointer is read. The third candidate of the
// format pre-selection, for matrices whose rows are nearly equal (the
// padding w * m / nnz stays close to 1).
__global__ __launch_bounds__(kBlock) void k_ell_fill(int32_t m, int32_t w, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx, int32_t* __restrict__ col,
                                                     int32_t* __restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const int32_t r0 = row_ptr[i], len = row_ptr[i + 1] - r0;
    for (int j = 0; j < w; ++j) {
        const int64_t pos = (int64_t)j * m + i;
        const bool on = j < len;
        col[pos] = on ? col_idx[r0 + j] : -1;
        src[pos] = on ? r0 + j : -1;
    }
}

// y = A x over the ELL copy: a thread per row, eight steps loaded per round
// (steps past w switched off), a partial sum per load slot.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_ell_spmv(int32_t m, int32_t w, const int32_t* __restrict__ col,
                                                     const typename SR<DT>::V* __restrict__ vals,
                                                     const typename SR<DT>::X* __restrict__ x,
                                                     typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    constexpr int U = 8;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    ChunkedAcc<DT, U> acc;
    for (int j = 0; j < w; j += U) {
        int c[U];
        typename S::V a[U];
        typename S::X b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) c[u] = j + u < w ? col[(int64_t)(j + u) * m + i] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u)
            a[u] = j + u < w ? S::val(vals, (int64_t)(j + u) * m + i) : (typename S::V)0;
#pragma unroll
        for (int u = 0; u < U; ++u) b[u] = c[u] >= 0 ? S::xval(x, c[u]) : (typename S::X)0;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (c[u] >= 0) acc.part[u] = S::fma(a[u], b[u], acc.part[u]);
        acc.end_round();
    }
    y[i] = S::out(acc.total());
}

spx_status ell_build(const spx_csr& A, int32_t w, EllMat* out, hipStream_t s) {
    EllMat E;
    E.m = A.m;
    E.width = w;
    E.cells = (int64_t)w * A.m;
    const int vs = value_size(A.dtype);
    const size_t cells = (size_t)std::max<int64_t>(1, E.cells);
    if (hipMalloc((void**)&E.col, cells * 4) != hipSuccess || hipMalloc((void**)&E.src, cells * 4) != hipSuccess ||
        (vs > 0 && hipMalloc(&E.vals, cells * vs) != hipSuccess)) {
        ell_free(&E);
        return fail(SPX_ERR_ALLOC, "ELL allocation failed");
    }
    if (A.m > 0 && w > 0) {
        k_ell_fill<<<(unsigned)ceil_div(A.m, kBlock), kBlock, 0, s>>>(A.m, w, A.row_ptr, A.col_idx, E.col, E.src);
        if (hipGetLastError() != hipSuccess) {
            ell_free(&E);
            return fail(SPX_ERR_HIP, "ELL fill");
        }
    }
    *out = E;
    return ell_refresh(*out, A, s);
}

spx_status ell_refresh(const EllMat& E, const spx_csr& A, hipStream_t s) {
    const int vs = value_size(A.dtype);
    if (vs == 0 || E.cells == 0) return SPX_OK;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(E.cells, kBlock), 8192));
    if (vs == 4)
        k_sell_vals<uint32_t><<<grid, kBlock, 0, s>>>(E.cells, E.src, (const uint32_t*)A.vals, (uint32_t*)E.vals);
    else
        k_sell_vals<uint64_t><<<grid, kBlock, 0, s>>>(E.cells, E.src, (const uint64_t*)A.vals, (uint64_t*)E.vals);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

void ell_free(EllMat* E) {
    void* ptrs[] = {E->col, E->src, E->vals};
    for (void* p : ptrs)
        if (p) hipFree(p);
    *E = EllMat{};
}

spx_status ell_spmv(const EllMat& E, int dtype, const void* x, void* y, hipStream_t s) {
    if (E.m == 0) return SPX_OK;
    const unsigned grid = (unsigned)ceil_div(E.m, kBlock);
    switch (dtype) {
#define SPX_DT(DT)                                                                                           \
    case DT:                                                                                                 \
        k_ell_spmv<DT><<<grid, kBlock, 0, s>>>(E.m, E.width, E.col, (const typename SR<DT>::V*)E.vals,       \
                                               (const typename SR<DT>::X*)x, (typename SR<DT>::Y*)y);        \
        break;
        SPX_DT(SPX_F32)
        SPX_DT(SPX_F64)
        SPX_DT(SPX_I32)
        SPX_DT(SPX_BOOL)
        SPX_DT(SPX_F32_MINPLUS)
#undef SPX_DT
        default:
            return fail(SPX_ERR_DTYPE, "ELL: unknown dtype");
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

}  // namespace spx
