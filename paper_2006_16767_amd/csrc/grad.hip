// Backward of y_b = A(vals) x_b for a batch of B vectors, with G = dL/dY
// (B x m) and X (B x n):
//
//   dX[b, j]  = sum_i a_ij G[b, i]            (dX = G A, i.e. A^T g_b per b)
//   dvals_k   = sum_b G[b, row k] X[b, col k]  (a sampled dense-dense product)
//
// Both kernels read the matrix once for the whole batch and work on B-minor
// copies of the dense operands (G^T is m x B, X^T is n x B), so that the B
// values one stored entry needs are 4 * B contiguous bytes:
//
//  k_seg_gather one wave per column j of A (a row of A^T, read from the CSC
//               copy: a gather along the column, no atomics); lane b
//               accumulates sum_k vals[k] * G^T[row_k, b] (eight entries in
//               flight); a workgroup's 16 columns are turned through LDS so
//               that dX is stored B-major directly.
//  k_sddmm      one wave per row i of A, lane b = batch entry: sixteen stored
//               entries at a time, each lane forms its sixteen products
//               G^T[i, b] X^T[col_k, b] (coalesced 4B-per-lane rows), and a
//               butterfly over the wave folds the sixteen B-long sums with
//               17 shuffles.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

// out (cols x rows) = transpose of in (rows x cols), 32 x 32 tiles through LDS
template <typename T>
__global__ __launch_bounds__(kBlock) void k_transpose(int64_t rows, int64_t cols, const T* __restrict__ in,
                                                      T* __restrict__ out) {
    __shared__ T tile[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8
    for (int dy = ty; dy < 32; dy += 8) {
        const int64_t r = r0 + dy, c = c0 + tx;
        if (r < rows && c < cols) tile[dy][tx] = in[r * cols + c];
    }
    __syncthreads();
    for (int dy = ty; dy < 32; dy += 8) {
        const int64_t c = c0 + dy, r = r0 + tx;
        if (r < rows && c < cols) out[c * rows + r] = tile[tx][dy];
    }
}

template <typename T>
static spx_status transpose(int64_t rows, int64_t cols, const T* in, T* out, hipStream_t s) {
    if (rows == 0 || cols == 0) return SPX_OK;
    dim3 grid((unsigned)ceil_div(cols, 32), (unsigned)ceil_div(rows, 32));
    k_transpose<T><<<grid, kBlock, 0, s>>>(rows, cols, in, out);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// Segment gather over a batch, written B-major: out[b0 + b, j] = sum over
// the entries k of segment j of vals[k] * inT[idx[k], b0 + b], for b < nb.
// inT is B-minor (rows of B values), so a wave per segment reads the B
// values of one entry as one coalesced row (lane = batch entry). A
// workgroup takes kSegPerBlock consecutive segments, one wave each, and
// turns its kSegPerBlock x nb results through LDS so that every batch row
// is stored as kSegPerBlock consecutive values (no transpose pass). With
// the CSC (segments = columns, idx = rows, inT = G^T) it is dX = G A; with
// the CSR (segments = rows, idx = columns, inT = X^T) it is Y for
// y_b = A x_b.
constexpr int kSegPerBlock = 16;
constexpr int kSegThreads = kSegPerBlock * kWave;

template <typename T>
__global__ __launch_bounds__(kSegThreads) void k_seg_gather(int32_t nseg, int32_t B, int32_t b0, int32_t nb,
                                                            const int32_t* __restrict__ seg_ptr,
                                                            const int32_t* __restrict__ idx,
                                                            const T* __restrict__ vals, const T* __restrict__ inT,
                                                            T* __restrict__ out) {
    __shared__ T tile[kSegPerBlock][kWave + 1];
    const int w = __builtin_amdgcn_readfirstlane(wave_id());
    const int64_t j0 = (int64_t)blockIdx.x * kSegPerBlock;
    const int64_t j = j0 + w;
    const int lane = lane_id();
    if (j < nseg) {
        const bool on = lane < nb;
        const int c0 = seg_ptr[j], c1 = seg_ptr[j + 1];
        const T* g = inT + b0 + (on ? lane : 0);
        // a partial sum per load slot, folded every kFoldRounds rounds
        // (bounded chains on long segments)
        ChunkedAcc<sizeof(T) == 8 ? SPX_F64 : SPX_F32, 8> acc;
        int k = c0;
        for (; k + 7 < c1; k += 8) {
            int r[8];
            T v[8], gv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                r[u] = idx[k + u];
                v[u] = vals[k + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) gv[u] = g[(int64_t)r[u] * B];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc.part[u] = __builtin_fma(v[u], gv[u], acc.part[u]);
            acc.end_round();
        }
#pragma unroll
        for (int u = 0; u < 7; ++u)
            if (k + u < c1) acc.part[u] = __builtin_fma(vals[k + u], g[(int64_t)idx[k + u] * B], acc.part[u]);
        tile[w][lane] = acc.total();
    }
    __syncthreads();
    // thread t stores segment j0 + t % kSegPerBlock of batch row b0 + t / kSegPerBlock
    const int jj = threadIdx.x % kSegPerBlock;
    const int b = threadIdx.x / kSegPerBlock;
    if (b < nb && j0 + jj < nseg) out[(int64_t)(b0 + b) * nseg + j0 + jj] = tile[jj][b];
}

// Folds p[0..15] over the 64 lanes of a wave: lane l ends with the full sum
// of value (l >> 2) & 15. Each step halves the values a lane keeps and pairs
// it with the lane across one bit of the lane index.
template <typename T>
__device__ __forceinline__ T wave_fold16(T (&p)[16]) {
    const int lane = lane_id();
    T q[8], r[4], t[2];
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
    for (int v = 0; v < 8; ++v) q[v] = (h5 ? p[v + 8] : p[v]) + shfl_xor(h5 ? p[v] : p[v + 8], 32);
#pragma unroll
    for (int v = 0; v < 4; ++v) r[v] = (h4 ? q[v + 4] : q[v]) + shfl_xor(h4 ? q[v] : q[v + 4], 16);
#pragma unroll
    for (int v = 0; v < 2; ++v) t[v] = (h3 ? r[v + 2] : r[v]) + shfl_xor(h3 ? r[v] : r[v + 2], 8);
    T s = (h2 ? t[1] : t[0]) + shfl_xor(h2 ? t[0] : t[1], 4);
    s += shfl_xor(s, 2);
    s += shfl_xor(s, 1);
    return s;
}

// dvals[k] for the entries of row i: a wave per row, lane = batch entry
// (chunks of 64 for B > 64).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sddmm(int32_t m, int32_t B, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx, const T* __restrict__ GT,
                                                  const T* __restrict__ XT, T* __restrict__ dvals) {
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * kWavesPerBlock + wave_id());
    if (i >= m) return;
    const int lane = lane_id();
    const int k0 = row_ptr[i], k1 = row_ptr[i + 1];
    for (int k = k0; k < k1; k += 16) {
        int c[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) c[u] = col_idx[k + u < k1 ? k + u : k1 - 1];
        T p[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) p[u] = 0;
        for (int b0 = 0; b0 < B; b0 += 64) {
            const bool on = b0 + lane < B;
            const int b = b0 + (on ? lane : 0);
            const T gv = on ? GT[(int64_t)i * B + b] : (T)0;
            T xv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) xv[u] = XT[(int64_t)c[u] * B + b];
#pragma unroll
            for (int u = 0; u < 16; ++u) p[u] = __builtin_fma(gv, xv[u], p[u]);
        }
        const T s = wave_fold16(p);
        const int v = (lane >> 2) & 15;
        if ((lane & 3) == 0 && k + v < k1) dvals[k + v] = s;
    }
}

size_t grad_ws_bytes(int32_t m, int32_t n, int32_t B, int dtype) {
    const size_t es = dtype == SPX_F64 ? 8 : 4;
    Sizer z;
    z.take<char>((size_t)m * B * es);
    z.take<char>((size_t)n * B * es);
    return z.used;
}

// out (B x nseg, B-major) from a B-minor inT, 64 batch rows per launch
template <typename T>
static spx_status seg_gather(int32_t nseg, int32_t B, const int32_t* seg_ptr, const int32_t* idx, const T* vals,
                             const T* inT, T* out, hipStream_t s) {
    for (int32_t b0 = 0; b0 < B; b0 += kWave) {
        const int nb = std::min(kWave, B - b0);
        k_seg_gather<T><<<(unsigned)ceil_div(nseg, kSegPerBlock), kSegThreads, 0, s>>>(nseg, B, b0, nb, seg_ptr, idx,
                                                                                      vals, inT, out);
        SPX_HIP(hipGetLastError());
    }
    return SPX_OK;
}

template <typename T>
static spx_status dx_t(const int32_t* col_ptr, const int32_t* row_idx, const void* vals_csc, int32_t m, int32_t n,
                       int32_t B, const void* G, void* dX, Arena& ws, hipStream_t s) {
    T* GT = ws.take<T>((size_t)m * B);
    if (!GT) return fail(SPX_ERR_WORKSPACE, "dx: workspace too small");
    SPX_TRY(transpose<T>(B, m, (const T*)G, GT, s));
    return seg_gather<T>(n, B, col_ptr, row_idx, (const T*)vals_csc, GT, (T*)dX, s);
}

spx_status launch_dx(const int32_t* col_ptr, const int32_t* row_idx, const void* vals_csc, int32_t m, int32_t n,
                     int dtype, int32_t B, const void* G, void* dX, Arena& ws, hipStream_t s) {
    if (B == 0 || n == 0) return SPX_OK;
    if (m == 0) return fill_bytes(dX, 0, (size_t)B * n * (dtype == SPX_F64 ? 8 : 4), s);
    if (dtype == SPX_F32) return dx_t<float>(col_ptr, row_idx, vals_csc, m, n, B, G, dX, ws, s);
    if (dtype == SPX_F64) return dx_t<double>(col_ptr, row_idx, vals_csc, m, n, B, G, dX, ws, s);
    return fail(SPX_ERR_DTYPE, "dx: F32 or F64 only");
}

template <typename T>
static spx_status spmv_batch_t(const int32_t* row_ptr, const int32_t* col_idx, const void* vals, int32_t m,
                               int32_t n, int32_t B, const void* X, void* Y, Arena& ws, hipStream_t s) {
    T* XT = ws.take<T>((size_t)n * B);
    if (!XT) return fail(SPX_ERR_WORKSPACE, "spmv batch: workspace too small");
    SPX_TRY(transpose<T>(B, n, (const T*)X, XT, s));
    return seg_gather<T>(m, B, row_ptr, col_idx, (const T*)vals, XT, (T*)Y, s);
}

spx_status launch_spmv_batch(const int32_t* row_ptr, const int32_t* col_idx, const void* vals, int32_t m,
                             int32_t n, int dtype, int32_t B, const void* X, void* Y, Arena& ws, hipStream_t s) {
    if (B == 0 || m == 0) return SPX_OK;
    if (n == 0) return fill_bytes(Y, 0, (size_t)B * m * (dtype == SPX_F64 ? 8 : 4), s);
    if (dtype == SPX_F32) return spmv_batch_t<float>(row_ptr, col_idx, vals, m, n, B, X, Y, ws, s);
    if (dtype == SPX_F64) return spmv_batch_t<double>(row_ptr, col_idx, vals, m, n, B, X, Y, ws, s);
    return fail(SPX_ERR_DTYPE, "spmv batch: F32 or F64 only");
}

template <typename T>
static spx_status dvals_t(const int32_t* row_ptr, const int32_t* col_idx, int32_t m, int32_t n, int32_t nnz,
                          int32_t B, const void* G, const void* X, void* dvals, Arena& ws, hipStream_t s) {
    T* GT = ws.take<T>((size_t)m * B);
    T* XT = ws.take<T>((size_t)n * B);
    if (!GT || !XT) return fail(SPX_ERR_WORKSPACE, "dvals: workspace too small");
    SPX_TRY(transpose<T>(B, m, (const T*)G, GT, s));
    SPX_TRY(transpose<T>(B, n, (const T*)X, XT, s));
    (void)nnz;
    k_sddmm<T><<<(unsigned)ceil_div(m, kWavesPerBlock), kBlock, 0, s>>>(m, B, row_ptr, col_idx, GT, XT,
                                                                        (T*)dvals);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// dX = G A and dvals from one B-minor copy of G (and one of X): the two
// gradients of a backward pass, with the transposes they share made once.
template <typename T>
static spx_status backward_t(const int32_t* row_ptr, const int32_t* col_idx, const int32_t* col_ptr,
                             const int32_t* row_idx, const void* vals_csc, int32_t m, int32_t n, int32_t B,
                             const void* G, const void* X, void* dX, void* dvals, Arena& ws, hipStream_t s) {
    T* GT = ws.take<T>((size_t)m * B);
    T* XT = ws.take<T>((size_t)n * B);
    if (!GT || !XT) return fail(SPX_ERR_WORKSPACE, "backward: workspace too small");
    SPX_TRY(transpose<T>(B, m, (const T*)G, GT, s));
    if (dX) SPX_TRY(seg_gather<T>(n, B, col_ptr, row_idx, (const T*)vals_csc, GT, (T*)dX, s));
    if (dvals) {
        SPX_TRY(transpose<T>(B, n, (const T*)X, XT, s));
        k_sddmm<T><<<(unsigned)ceil_div(m, kWavesPerBlock), kBlock, 0, s>>>(m, B, row_ptr, col_idx, GT, XT,
                                                                            (T*)dvals);
        SPX_HIP(hipGetLastError());
    }
    return SPX_OK;
}

spx_status launch_backward(const int32_t* row_ptr, const int32_t* col_idx, const int32_t* col_ptr,
                           const int32_t* row_idx, const void* vals_csc, int32_t m, int32_t n, int32_t nnz, int dtype,
                           int32_t B, const void* G, const void* X, void* dX, void* dvals, Arena& ws, hipStream_t s) {
    const size_t es = dtype == SPX_F64 ? 8 : 4;
    if (B == 0) return dvals && nnz > 0 ? fill_bytes(dvals, 0, (size_t)nnz * es, s) : SPX_OK;
    if (m == 0 || nnz == 0) {
        if (dX && n > 0) SPX_TRY(fill_bytes(dX, 0, (size_t)B * n * es, s));
        return SPX_OK;
    }
    if (dtype == SPX_F32)
        return backward_t<float>(row_ptr, col_idx, col_ptr, row_idx, vals_csc, m, n, B, G, X, dX, dvals, ws, s);
    if (dtype == SPX_F64)
        return backward_t<double>(row_ptr, col_idx, col_ptr, row_idx, vals_csc, m, n, B, G, X, dX, dvals, ws, s);
    return fail(SPX_ERR_DTYPE, "backward: F32 or F64 only");
}

spx_status launch_dvals(const int32_t* row_ptr, const int32_t* col_idx, int32_t m, int32_t n, int32_t nnz,
                        int dtype, int32_t B, const void* G, const void* X, void* dvals, Arena& ws, hipStream_t s) {
    if (nnz == 0) return SPX_OK;
    if (B == 0) return fill_bytes(dvals, 0, (size_t)nnz * (dtype == SPX_F64 ? 8 : 4), s);
    if (dtype == SPX_F32) return dvals_t<float>(row_ptr, col_idx, m, n, nnz, B, G, X, dvals, ws, s);
    if (dtype == SPX_F64) return dvals_t<double>(row_ptr, col_idx, m, n, nnz, B, G, X, dvals, ws, s);
    return fail(SPX_ERR_DTYPE, "dvals: F32 or F64 only");
}

// ------------------------------------------------------------------ dense rows -> sparse vectors
// B dense rows of length n (x != 0 is a nonzero: -0.0 is zero, NaN is not)
// become CSR-of-vectors. Every row is cut into tiles of kRowTile entries so
// that a long row spreads over many workgroups: a count per tile, one
// exclusive scan over all tiles (row after row), then each tile compacts
// its entries in index order at its offset; the first tile of a row writes
// the row's start, the last tile of the last row the total.
constexpr int kRowTile = kBlock * 8;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_nnz(int32_t n, int32_t tpr, const T* __restrict__ X,
                                                     int32_t* __restrict__ cnt) {
    __shared__ int32_t s_tmp[kWavesPerBlock];
    const int64_t t = blockIdx.x;
    const int64_t b = t / tpr;
    const int64_t j0 = (t - b * tpr) * kRowTile;
    const T* x = X + b * n;
    int32_t c = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + u * kBlock + threadIdx.x;
        c += j < n && x[j] != (T)0;
    }
    int32_t tot;
    block_incl_scan(c, s_tmp, &tot);
    if (threadIdx.x == 0) cnt[t] = tot;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_compact(int32_t B, int32_t n, int32_t tpr, const T* __restrict__ X,
                                                         const int32_t* __restrict__ off,
                                                         int32_t* __restrict__ vec_ptr, int32_t* __restrict__ idx,
                                                         T* __restrict__ val) {
    __shared__ int32_t s_tmp[kWavesPerBlock];
    const int64_t t = blockIdx.x;
    const int64_t b = t / tpr;
    const int64_t tile = t - b * tpr;
    const int64_t j0 = tile * kRowTile + (int64_t)threadIdx.x * 8;  // 8 consecutive entries per thread
    const T* x = X + b * n;
    T v[8];
    uint32_t f = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + u;
        v[u] = j < n ? x[j] : (T)0;
        if (j < n && v[u] != (T)0) f |= 1u << u;
    }
    const int32_t c = __popc(f);
    int32_t tot;
    const int32_t incl = block_incl_scan(c, s_tmp, &tot);
    int32_t slot = off[t] + incl - c;
    while (f) {
        const int u = __ffs(f) - 1;
        f &= f - 1;
        idx[slot] = (int32_t)(j0 + u);
        if (val) val[slot] = v[u];
        ++slot;
    }
    if (threadIdx.x == 0) {
        if (tile == 0) vec_ptr[b] = off[t];
        if (t == (int64_t)B * tpr - 1) vec_ptr[B] = off[t] + tot;
    }
}

template <typename T>
static spx_status rows_to_sparse_t(int32_t B, int32_t n, const void* X, int32_t* vec_ptr, int32_t* idx, void* val,
                                   Arena& ws, hipStream_t s) {
    const int32_t tpr = (int32_t)std::max<int64_t>(1, ceil_div(n, kRowTile));
    const int64_t tiles = (int64_t)B * tpr;
    int32_t* off = ws.take<int32_t>((size_t)tiles + 1);
    int32_t* sws = ws.take<int32_t>(scan_ws_elems(tiles + 1));
    if (!off || !sws) return fail(SPX_ERR_WORKSPACE, "dense rows: workspace too small");
    SPX_TRY(fill_u32((uint32_t*)(off + tiles), 0u, 1, s));
    k_tile_nnz<T><<<(unsigned)tiles, kBlock, 0, s>>>(n, tpr, (const T*)X, off);
    SPX_HIP(hipGetLastError());
    SPX_TRY(scan_exclusive_i32(off, off, tiles + 1, nullptr, sws, s));
    k_tile_compact<T><<<(unsigned)tiles, kBlock, 0, s>>>(B, n, tpr, (const T*)X, off, vec_ptr, idx, (T*)val);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

size_t dense_rows_ws_bytes(int32_t B, int32_t n) {
    const int64_t tiles = (int64_t)B * std::max<int64_t>(1, ceil_div(n, kRowTile));
    Sizer z;
    z.take<int32_t>((size_t)tiles + 1);
    z.take<int32_t>(scan_ws_elems(tiles + 1));
    return z.used;
}

spx_status dense_rows_to_sparse(int32_t B, int32_t n, int dtype, const void* X, int32_t* vec_ptr, int32_t* idx,
                                void* val, Arena& ws, hipStream_t s) {
    if (B == 0) return fill_u32((uint32_t*)vec_ptr, 0, 1, s);
    if (n == 0) return fill_u32((uint32_t*)vec_ptr, 0, (size_t)B + 1, s);
    switch (dtype) {
        case SPX_F32: return rows_to_sparse_t<float>(B, n, X, vec_ptr, idx, val, ws, s);
        case SPX_F64: return rows_to_sparse_t<double>(B, n, X, vec_ptr, idx, val, ws, s);
        case SPX_I32: return rows_to_sparse_t<int32_t>(B, n, X, vec_ptr, idx, val, ws, s);
        case SPX_BOOL: return rows_to_sparse_t<uint8_t>(B, n, X, vec_ptr, idx, nullptr, ws, s);
    }
    return fail(SPX_ERR_DTYPE, "dense rows: dtype");
}

}  // namespace spx
