// Diagonal (DIA) copy of A for the SpMV pattern: the entries of A lie on at
// most kDiaMax diagonals (offsets col - row), stored diagonal by diagonal
// (cell (d, i) at d * m + i, the entry of row i on diagonal d) with one
// presence bit per cell. A row's products then need no column index: the
// thread of row i reads its cells and x[i + offset] with both streams
// coalesced across the wave, and the copy moves values + bits + x + y where
// CSR moves values + column indices + x + y + row pointers.
//
// The copy exists when the offsets found in kDiaSampleRows rows spread over
// A, its first and last row included (at most kDiaMax of them), hold every
// entry, checked by one pass; cells
// without an entry (a diagonal's holes and its ends) have their bit clear
// and take no part in the sums, as in CSR.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kDiaSampleRows = 256;

// Offsets of the entries of row r_s = s (m - 1) / (kDiaSampleRows - 1),
// the first and the last row among them (at most kDiaMax per row; lens[s] =
// the row's length).
__global__ void k_dia_sample(int32_t m, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                             int32_t* __restrict__ offs, int32_t* __restrict__ lens) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= kDiaSampleRows) return;
    const int32_t r = m <= 1 ? 0 : (int32_t)((int64_t)s * (m - 1) / (kDiaSampleRows - 1));
    const int32_t k0 = row_ptr[r], k1 = row_ptr[r + 1];
    lens[s] = k1 - k0;
    for (int t = 0; t < kDiaMax && k0 + t < k1; ++t) offs[s * kDiaMax + t] = col_idx[k0 + t] - r;
}

// Position of offset o among the nd ascending offsets (-1 if absent).
__device__ __forceinline__ int dia_find(const int32_t* offs, int nd, int32_t o) {
    int lo = 0, hi = nd;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (offs[mid] < o)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < nd && offs[lo] == o ? lo : -1;
}

// *bad = 1 when some entry lies on none of the nd offsets.
__global__ __launch_bounds__(kBlock) void k_dia_check(int32_t m, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col_idx, int nd,
                                                      const int32_t* __restrict__ offs, int32_t* bad) {
    __shared__ int32_t s_off[kDiaMax];
    if (threadIdx.x < nd) s_off[threadIdx.x] = offs[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    bool ok = true;
    for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) ok = ok && dia_find(s_off, nd, col_idx[k] - (int32_t)i) >= 0;
    if (!ok) atomicOr(bad, 1);
}

// Cells and presence bits of the copy: the thread of row i places its
// entries; the wave's bits of each diagonal go out as two words (rows of
// a wave are 64 consecutive rows, 64-aligned).
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_dia_fill(int32_t m, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx,
                                                     const VT* __restrict__ vals, int nd,
                                                     const int32_t* __restrict__ offs, int64_t words,
                                                     VT* __restrict__ dvals, uint32_t* __restrict__ mask) {
    __shared__ int32_t s_off[kDiaMax];
    if (threadIdx.x < nd) s_off[threadIdx.x] = offs[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t has = 0;  // bit d: row i has an entry on diagonal d
    if (i < m) {
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const int d = dia_find(s_off, nd, col_idx[k] - (int32_t)i);
            if (d < 0) continue;  // excluded by the check
            has |= 1u << d;
            if (vals) dvals[(int64_t)d * m + i] = vals[k];
        }
    }
    const int64_t w0 = ((int64_t)blockIdx.x * kBlock + wave_id() * kWave) >> 5;
    for (int d = 0; d < nd; ++d) {
        const uint64_t b = __ballot((has >> d) & 1u);
        if (lane_id() == 0 && w0 < words) mask[(int64_t)d * words + w0] = (uint32_t)b;
        if (lane_id() == 32 && w0 + 1 < words) mask[(int64_t)d * words + w0 + 1] = (uint32_t)(b >> 32);
    }
}

// y = A x over the copy: a thread per row, eight diagonals per round, a
// partial sum per load slot. The bits, the cells and x (at an index clamped
// into [0, n)) are all loaded before any is used, so a row costs one round
// trip; a cell without its bit is then dropped by a select.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_dia_spmv(int32_t m, int32_t n, int nd, const int32_t* __restrict__ offs,
                                                     int64_t words, const typename SR<DT>::V* __restrict__ dvals,
                                                     const uint32_t* __restrict__ mask,
                                                     const typename SR<DT>::X* __restrict__ x,
                                                     typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    constexpr int U = 8;
    __shared__ int32_t s_off[kDiaMax];
    if (threadIdx.x < nd) s_off[threadIdx.x] = offs[threadIdx.x];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    ChunkedAcc<DT, U> acc;
    for (int d0 = 0; d0 < nd; d0 += U) {
        uint32_t w[U];
        typename S::V a[U];
        typename S::X b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (d0 + u < nd) {  // uniform
                const int64_t j = min(max(i + s_off[d0 + u], (int64_t)0), (int64_t)n - 1);
                w[u] = mask[(int64_t)(d0 + u) * words + (i >> 5)];
                a[u] = S::val(dvals, (int64_t)(d0 + u) * m + i);
                b[u] = S::xval(x, j);
            } else {
                w[u] = 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if ((w[u] >> (i & 31)) & 1u) acc.part[u] = S::fma(a[u], b[u], acc.part[u]);
        acc.end_round();
    }
    y[i] = S::out(acc.total());
}

// The same for 8-byte values, two consecutive rows per thread (one presence
// word): the wave has twice the bytes in flight, which paid in FP64 (34.7
// against 37.5 µs on Poisson 128^3) and not in FP32 (29.1 against 23.3).
template <int DT>
__global__ __launch_bounds__(kBlock) void k_dia_spmv2(int32_t m, int32_t n, int nd, const int32_t* __restrict__ offs,
                                                      int64_t words, const typename SR<DT>::V* __restrict__ dvals,
                                                      const uint32_t* __restrict__ mask,
                                                      const typename SR<DT>::X* __restrict__ x,
                                                      typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    constexpr int U = 8;
    constexpr int R = 2;
    __shared__ int32_t s_off[kDiaMax];
    if (threadIdx.x < nd) s_off[threadIdx.x] = offs[threadIdx.x];
    __syncthreads();
    const int64_t i0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * R;
    if (i0 >= m) return;
    typename S::Acc acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = S::zero();
    for (int d0 = 0; d0 < nd; d0 += U) {
        uint32_t w[U];
        typename S::V a[U][R];
        typename S::X b[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (d0 + u < nd) {  // uniform
                w[u] = mask[(int64_t)(d0 + u) * words + (i0 >> 5)];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t i = min(i0 + r, (int64_t)m - 1);
                    const int64_t j = min(max(i + s_off[d0 + u], (int64_t)0), (int64_t)n - 1);
                    a[u][r] = S::val(dvals, (int64_t)(d0 + u) * m + i);
                    b[u][r] = S::xval(x, j);
                }
            } else {
                w[u] = 0u;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r)
                if ((w[u] >> ((i0 + r) & 31)) & 1u) acc[r] = S::fma(a[u][r], b[u][r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (i0 + r < m) y[i0 + r] = S::out(acc[r]);
}

// ------------------------------------------------------------------ host side
void dia_free(DiaMat* D) {
    void* ptrs[] = {D->offs, D->vals, D->mask};
    for (void* p : ptrs)
        if (p) hipFree(p);
    *D = DiaMat{};
}

spx_status dia_try_build(const spx_csr& A, int32_t max_row, bool forced, DiaMat* out, hipStream_t s) {
    auto no = [&](const char* why) { return forced ? fail(SPX_ERR_UNSUPPORTED, why) : SPX_OK; };
    if (A.dtype == SPX_BOOL) return no("DIA: Boolean matrices keep the other formats");
    if (A.m == 0 || A.nnz == 0) return no("DIA: no entries");
    if (max_row > kDiaMax) return no("DIA: a row holds more than 32 entries");
    // offsets proposed by the sampled rows
    int32_t* tmp = nullptr;
    const size_t tmp_ints = (size_t)kDiaSampleRows * kDiaMax + kDiaSampleRows + 1 + kDiaMax;
    if (hipMalloc((void**)&tmp, tmp_ints * 4) != hipSuccess) return fail(SPX_ERR_ALLOC, "DIA: sample buffer");
    int32_t* d_offs = tmp;
    int32_t* d_lens = tmp + (size_t)kDiaSampleRows * kDiaMax;
    int32_t* d_bad = d_lens + kDiaSampleRows;
    int32_t* d_set = d_bad + 1;
    std::vector<int32_t> h_offs((size_t)kDiaSampleRows * kDiaMax), h_lens(kDiaSampleRows);
    k_dia_sample<<<1, kDiaSampleRows, 0, s>>>(A.m, A.row_ptr, A.col_idx, d_offs, d_lens);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h_offs.data(), d_offs, h_offs.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(h_lens.data(), d_lens, h_lens.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        hipFree(tmp);
        return fail(SPX_ERR_HIP, "DIA: sample read-back");
    }
    std::vector<int32_t> set;
    for (int r = 0; r < kDiaSampleRows; ++r)
        for (int t = 0; t < std::min(h_lens[r], kDiaMax); ++t) set.push_back(h_offs[(size_t)r * kDiaMax + t]);
    std::sort(set.begin(), set.end());
    set.erase(std::unique(set.begin(), set.end()), set.end());
    const int nd = (int)set.size();
    const int vs = value_size(A.dtype);
    const int64_t cells = (int64_t)nd * A.m;
    // fewer bytes than the CSR copy (values + column indices), with room
    const bool pays = (double)cells * (vs + 0.125) <= 0.8 * (double)A.nnz * (vs + 4);
    if (nd == 0 || nd > kDiaMax || (!forced && !pays) || (forced && cells > 4 * (int64_t)A.nnz + 65536)) {
        hipFree(tmp);
        return no("DIA: the entries lie on too many diagonals");
    }
    // every entry on one of them?
    int32_t bad = 0;
    const unsigned grid = (unsigned)ceil_div(A.m, kBlock);
    if (hipMemcpyAsync(d_set, set.data(), (size_t)nd * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(d_bad, 0, 4, s) != hipSuccess) {
        hipFree(tmp);
        return fail(SPX_ERR_HIP, "DIA: check set-up");
    }
    k_dia_check<<<grid, kBlock, 0, s>>>(A.m, A.row_ptr, A.col_idx, nd, d_set, d_bad);
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        hipFree(tmp);
        return fail(SPX_ERR_HIP, "DIA: check");
    }
    hipFree(tmp);
    if (bad) return no("DIA: some entry lies off the diagonals found in the sampled rows");
    DiaMat D;
    D.m = A.m;
    D.n = A.n;
    D.nd = nd;
    D.cells = cells;
    D.words = ceil_div(A.m, 32) + 1;  // the last wave writes its second word too
    if (hipMalloc((void**)&D.offs, (size_t)nd * 4) != hipSuccess ||
        hipMalloc(&D.vals, (size_t)cells * vs) != hipSuccess ||
        hipMalloc((void**)&D.mask, (size_t)nd * D.words * 4) != hipSuccess) {
        dia_free(&D);
        return fail(SPX_ERR_ALLOC, "DIA allocation failed");
    }
    // cells without an entry are read by the SpMV (and dropped): zero them once
    if (hipMemcpyAsync(D.offs, set.data(), (size_t)nd * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(D.vals, 0, (size_t)cells * vs, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        dia_free(&D);
        return fail(SPX_ERR_HIP, "DIA: offsets upload");
    }
    *out = D;
    const spx_status st = dia_refresh(*out, A, s);
    if (st != SPX_OK) dia_free(out);
    return st;
}

// Cells and bits from A's current values (also after values_updated).
spx_status dia_refresh(const DiaMat& D, const spx_csr& A, hipStream_t s) {
    if (D.m == 0) return SPX_OK;
    const unsigned grid = (unsigned)ceil_div(D.m, kBlock);
    if (value_size(A.dtype) == 4)
        k_dia_fill<uint32_t><<<grid, kBlock, 0, s>>>(D.m, A.row_ptr, A.col_idx, (const uint32_t*)A.vals, D.nd,
                                                     D.offs, D.words, (uint32_t*)D.vals, D.mask);
    else
        k_dia_fill<uint64_t><<<grid, kBlock, 0, s>>>(D.m, A.row_ptr, A.col_idx, (const uint64_t*)A.vals, D.nd,
                                                     D.offs, D.words, (uint64_t*)D.vals, D.mask);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status dia_spmv(const DiaMat& D, int dtype, const void* x, void* y, hipStream_t s) {
    if (D.m == 0) return SPX_OK;
    const unsigned grid = (unsigned)ceil_div(D.m, kBlock);
    switch (dtype) {
#define SPX_DT(DT)                                                                                          \
    case DT:                                                                                                \
        k_dia_spmv<DT><<<grid, kBlock, 0, s>>>(D.m, D.n, D.nd, D.offs, D.words, (const typename SR<DT>::V*)D.vals, \
                                               D.mask, (const typename SR<DT>::X*)x, (typename SR<DT>::Y*)y);  \
        break;
        SPX_DT(SPX_F32)
        SPX_DT(SPX_I32)
        SPX_DT(SPX_F32_MINPLUS)
#undef SPX_DT
        case SPX_F64:
            k_dia_spmv2<SPX_F64><<<(unsigned)ceil_div(D.m, kBlock * 2), kBlock, 0, s>>>(
                D.m, D.n, D.nd, D.offs, D.words, (const double*)D.vals, D.mask, (const double*)x, (double*)y);
            break;
        default:
            return fail(SPX_ERR_DTYPE, "DIA: dtype");
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

}  // namespace spx
