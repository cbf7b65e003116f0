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
//  k_spmm_csc   one wave per column j of A (a row of A^T, read from the CSC
//               copy: a gather along the column, no atomics); lane b
//               accumulates sum_k vals[k] * G^T[row_k, b].
//  k_sddmm      a group of lanes per row i of A; G^T[i, :] is staged in LDS
//               once per row; every lane takes one stored entry k and forms
//               the B-long dot product of G^T[i, :] and X^T[col_k, :].
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

// dX[b0 + lane, j] for lanes < nb; GT is m x B
template <typename T>
__global__ __launch_bounds__(kBlock) void k_spmm_csc(int32_t n, int32_t B, int32_t b0, int32_t nb,
                                                     const int32_t* __restrict__ col_ptr,
                                                     const int32_t* __restrict__ row_idx,
                                                     const T* __restrict__ vals, const T* __restrict__ GT,
                                                     T* __restrict__ dX) {
    const int64_t j = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (j >= n) return;
    const int lane = lane_id();
    const bool on = lane < nb;
    const int c0 = col_ptr[j], c1 = col_ptr[j + 1];
    const T* g = GT + b0 + (on ? lane : 0);
    T acc = 0;
    int k = c0;
    for (; k + 3 < c1; k += 4) {
        int r[4];
        T v[4], gv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            r[u] = row_idx[k + u];
            v[u] = vals[k + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) gv[u] = g[(int64_t)r[u] * B];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_fma(v[u], gv[u], acc);
    }
    for (; k < c1; ++k) acc = __builtin_fma(vals[k], g[(int64_t)row_idx[k] * B], acc);
    if (on) dX[(int64_t)(b0 + lane) * n + j] = acc;
}

// dvals[k] for the entries of row i; L lanes per row, B <= 64 per pass
template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_sddmm(int32_t m, int32_t B, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx, const T* __restrict__ GT,
                                                  const T* __restrict__ XT, T* __restrict__ dvals) {
    constexpr int kRows = kBlock / L;
    __shared__ T s_g[kRows][64];
    const int lr = threadIdx.x / L, g = threadIdx.x % L;
    const int64_t row = (int64_t)blockIdx.x * kRows + lr;
    const bool live = row < m;
    for (int b0 = 0; b0 < B; b0 += 64) {
        const int nb = std::min(64, B - b0);
        if (live)
            for (int b = g; b < nb; b += L) s_g[lr][b] = GT[row * B + b0 + b];
        __syncthreads();
        if (live) {
            const int k0 = row_ptr[row], k1 = row_ptr[row + 1];
            for (int k = k0 + g; k < k1; k += L) {
                const T* xr = XT + (int64_t)col_idx[k] * B + b0;
                T acc = 0;
                int b = 0;
                for (; b + 3 < nb; b += 4) {
                    const T x0 = xr[b], x1 = xr[b + 1], x2 = xr[b + 2], x3 = xr[b + 3];
                    acc = __builtin_fma(s_g[lr][b], x0, acc);
                    acc = __builtin_fma(s_g[lr][b + 1], x1, acc);
                    acc = __builtin_fma(s_g[lr][b + 2], x2, acc);
                    acc = __builtin_fma(s_g[lr][b + 3], x3, acc);
                }
                for (; b < nb; ++b) acc = __builtin_fma(s_g[lr][b], xr[b], acc);
                dvals[k] = b0 == 0 ? acc : dvals[k] + acc;
            }
        }
        __syncthreads();
    }
}

size_t grad_ws_bytes(int32_t m, int32_t n, int32_t B, int dtype) {
    const size_t es = dtype == SPX_F64 ? 8 : 4;
    Sizer z;
    z.take<char>((size_t)m * B * es);
    z.take<char>((size_t)n * B * es);
    return z.used;
}

template <typename T>
static spx_status dx_t(const int32_t* col_ptr, const int32_t* row_idx, const void* vals_csc, int32_t m, int32_t n,
                       int32_t B, const void* G, void* dX, Arena& ws, hipStream_t s) {
    T* GT = ws.take<T>((size_t)m * B);
    if (!GT) return fail(SPX_ERR_WORKSPACE, "dx: workspace too small");
    SPX_TRY(transpose<T>(B, m, (const T*)G, GT, s));
    for (int32_t b0 = 0; b0 < B; b0 += 64) {
        const int nb = std::min(64, B - b0);
        k_spmm_csc<T><<<(unsigned)ceil_div(n, kWavesPerBlock), kBlock, 0, s>>>(n, B, b0, nb, col_ptr, row_idx,
                                                                              (const T*)vals_csc, GT, (T*)dX);
        SPX_HIP(hipGetLastError());
    }
    return SPX_OK;
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
static spx_status dvals_t(const int32_t* row_ptr, const int32_t* col_idx, int32_t m, int32_t n, int32_t nnz,
                          int32_t B, const void* G, const void* X, void* dvals, Arena& ws, hipStream_t s) {
    T* GT = ws.take<T>((size_t)m * B);
    T* XT = ws.take<T>((size_t)n * B);
    if (!GT || !XT) return fail(SPX_ERR_WORKSPACE, "dvals: workspace too small");
    SPX_TRY(transpose<T>(B, m, (const T*)G, GT, s));
    SPX_TRY(transpose<T>(B, n, (const T*)X, XT, s));
    // at least 4 lanes per row keeps the per-row LDS copies of G^T within 32 KiB
    const double avg = (double)nnz / m;
    int L = 4;
    while (L < 64 && L < avg) L <<= 1;
    const int64_t blocks = ceil_div(m, kBlock / L);
    switch (L) {
#define SPX_L(LL)                                                                                               \
    case LL:                                                                                                    \
        k_sddmm<T, LL><<<(unsigned)blocks, kBlock, 0, s>>>(m, B, row_ptr, col_idx, GT, XT, (T*)dvals);          \
        break;
        SPX_L(4) SPX_L(8) SPX_L(16) SPX_L(32) SPX_L(64)
#undef SPX_L
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
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
// become CSR-of-vectors: counts per row, a prefix over rows, then each row
// compacted in index order by one workgroup.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_row_nnz(int32_t n, const T* __restrict__ X, int32_t* __restrict__ cnt) {
    __shared__ int32_t s_tmp[kWavesPerBlock];
    const T* x = X + (int64_t)blockIdx.x * n;
    int32_t c = 0;
    for (int j = threadIdx.x; j < n; j += kBlock) c += x[j] != (T)0;
    int32_t tot;
    block_incl_scan(c, s_tmp, &tot);
    if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_row_compact(int32_t n, const T* __restrict__ X,
                                                        const int32_t* __restrict__ vec_ptr, int32_t* __restrict__ idx,
                                                        T* __restrict__ val) {
    __shared__ int32_t s_tmp[kWavesPerBlock];
    const T* x = X + (int64_t)blockIdx.x * n;
    int32_t carry = vec_ptr[blockIdx.x];
    for (int j0 = 0; j0 < n; j0 += kBlock) {
        const int j = j0 + threadIdx.x;
        const T v = j < n ? x[j] : (T)0;
        const int32_t f = (j < n && v != (T)0) ? 1 : 0;
        int32_t tot;
        const int32_t incl = block_incl_scan(f, s_tmp, &tot);
        if (f) {
            idx[carry + incl - 1] = j;
            if (val) val[carry + incl - 1] = v;
        }
        carry += tot;
    }
}

template <typename T>
static spx_status rows_to_sparse_t(int32_t B, int32_t n, const void* X, int32_t* vec_ptr, int32_t* idx, void* val,
                                   int32_t* ws_i32, hipStream_t s) {
    k_row_nnz<T><<<B, kBlock, 0, s>>>(n, (const T*)X, vec_ptr);
    SPX_HIP(hipGetLastError());
    SPX_TRY(scan_exclusive_i32(vec_ptr, vec_ptr, (int64_t)B + 1, nullptr, ws_i32, s));
    k_row_compact<T><<<B, kBlock, 0, s>>>(n, (const T*)X, vec_ptr, idx, (T*)val);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status dense_rows_to_sparse(int32_t B, int32_t n, int dtype, const void* X, int32_t* vec_ptr, int32_t* idx,
                                void* val, int32_t* ws_i32, hipStream_t s) {
    if (B == 0) return fill_u32((uint32_t*)vec_ptr, 0, 1, s);
    // vec_ptr[B] must be 0 before the scan turns counts into offsets
    SPX_TRY(fill_u32((uint32_t*)(vec_ptr + B), 0, 1, s));
    switch (dtype) {
        case SPX_F32: return rows_to_sparse_t<float>(B, n, X, vec_ptr, idx, val, ws_i32, s);
        case SPX_F64: return rows_to_sparse_t<double>(B, n, X, vec_ptr, idx, val, ws_i32, s);
        case SPX_I32: return rows_to_sparse_t<int32_t>(B, n, X, vec_ptr, idx, val, ws_i32, s);
        case SPX_BOOL: return rows_to_sparse_t<uint8_t>(B, n, X, vec_ptr, idx, nullptr, ws_i32, s);
    }
    return fail(SPX_ERR_DTYPE, "dense rows: dtype");
}

}  // namespace spx
