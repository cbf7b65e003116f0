// Backward of y = A(vals) x with respect to the stored values:
//   dvals_k = sum_b G[b, row(k)] * X[b, col(k)]
// over the CSR pattern. A group of lanes walks each row, so row(k) is known
// without a search; G[b, row] is shared by the whole row.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

template <typename T, int L>
__global__ __launch_bounds__(kBlock) void k_dvals(int32_t m, int32_t n, const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx, int32_t B,
                                                  const T* __restrict__ G, const T* __restrict__ X,
                                                  T* __restrict__ dvals) {
    constexpr int kRows = kBlock / L;
    const int64_t row = (int64_t)blockIdx.x * kRows + threadIdx.x / L;
    if (row >= m) return;
    const int g = threadIdx.x % L;
    const int k0 = row_ptr[row], k1 = row_ptr[row + 1];
    for (int k = k0 + g; k < k1; k += L) {
        const int c = col_idx[k];
        T acc = 0;
        for (int b = 0; b < B; ++b) acc = __builtin_fma(G[(int64_t)b * m + row], X[(int64_t)b * n + c], acc);
        dvals[k] = acc;
    }
}

spx_status launch_dvals(const int32_t* row_ptr, const int32_t* col_idx, int32_t m, int32_t n, int32_t nnz,
                        int dtype, int32_t B, const void* G, const void* X, void* dvals, hipStream_t s) {
    if (m == 0 || nnz == 0) return SPX_OK;
    const double avg = (double)nnz / m;
    int L = 1;
    while (L < 64 && L < avg) L <<= 1;
    const int64_t blocks = ceil_div(m, kBlock / L);
#define SPX_L(T, LL)                                                                                \
    case LL:                                                                                        \
        k_dvals<T, LL><<<(unsigned)blocks, kBlock, 0, s>>>(m, n, row_ptr, col_idx, B, (const T*)G, \
                                                           (const T*)X, (T*)dvals);                 \
        break;
    if (dtype == SPX_F32) {
        switch (L) { SPX_L(float, 1) SPX_L(float, 2) SPX_L(float, 4) SPX_L(float, 8) SPX_L(float, 16)
                     SPX_L(float, 32) SPX_L(float, 64) }
    } else if (dtype == SPX_F64) {
        switch (L) { SPX_L(double, 1) SPX_L(double, 2) SPX_L(double, 4) SPX_L(double, 8) SPX_L(double, 16)
                     SPX_L(double, 32) SPX_L(double, 64) }
    } else {
        return fail(SPX_ERR_DTYPE, "dvals: F32 or F64 only");
    }
#undef SPX_L
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

}  // namespace spx
