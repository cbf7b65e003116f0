// Incremental PageRank driver (the second application the paper evaluates
// its kernels in, Section 7): residual push, where every round propagates
// only the vertices whose residual is above a threshold, so the product's
// input starts dense and thins out round by round, and run() follows it.
//
// Stored entry (i, j) is an edge j -> i of weight a_ij >= 0; the walk
// leaves j along (i, j) with probability a_ij / W_j, W_j = sum of column j.
// State: residual r (starts at (1 - d)/n) and rank p (starts at 0). A round
// (k_pr_select) folds the previous product into r (r += d y), moves every
// active residual (|r_v| > eps) into p_v, clears it, and appends the
// active vertices with W_v > 0 to the sparse input x_v = r_v / W_v of the
// next product y = A x.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "frontier.hpp"
#include "internal.hpp"

namespace spx {

// W_j = sum of column j over the CSC values; bad gets bit 0 if a weight is
// negative. Run once per value version of the handle.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pr_colsum(int32_t n, const int32_t* __restrict__ col_ptr,
                                                      const T* __restrict__ vals, T* __restrict__ W,
                                                      uint32_t* __restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
        T s = 0;
        bool neg = false;
        for (int32_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) {
            const T a = vals[k];
            neg |= a < (T)0;
            s += a;
        }
        W[j] = s;
        if (neg) atomicOr(bad, 1u);
    }
}

// r = r0 everywhere, p = 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pr_init(int32_t n, T r0, T* __restrict__ r, T* __restrict__ p) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        r[v] = r0;
        p[v] = (T)0;
    }
}

// One round. y = nullptr on the first round (no product yet). The counter
// gets {appended entries of x (low), their column lengths (high), i.e. the
// nnz_s of the next product}; count_clear is zeroed for the next round.
// r += d y is rounded as a product and then a sum (no fused multiply-add),
// the order the definition states.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pr_select(int32_t n, T d, T eps, const T* __restrict__ y,
                                                      T* __restrict__ r, T* __restrict__ p,
                                                      const T* __restrict__ W, const int32_t* __restrict__ col_ptr,
                                                      int32_t* __restrict__ x_idx, T* __restrict__ x_val,
                                                      Count* __restrict__ count, Count* __restrict__ count_clear) {
#pragma clang fp contract(off)
    __shared__ Count tmp[kWavesPerBlock];
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_clear = 0;
    for (int64_t base = (int64_t)blockIdx.x * kChunk; base < n; base += (int64_t)gridDim.x * kChunk) {
        const int64_t v0 = base + (int64_t)threadIdx.x * kVpt;
        uint32_t mask = 0, ns = 0;
        T xv[kVpt];
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            const int64_t v = v0 + j;
            xv[j] = (T)0;
            if (v < n) {
                T rv = r[v];
                if (y) {
                    const T dy = d * y[v];
                    rv = rv + dy;
                }
                if (rv > eps || rv < -eps) {
                    p[v] = p[v] + rv;
                    r[v] = (T)0;
                    const T w = W[v];
                    if (w > (T)0) {
                        mask |= 1u << j;
                        xv[j] = rv / w;
                        ns += (uint32_t)(col_ptr[v + 1] - col_ptr[v]);
                    }
                } else if (y) {
                    r[v] = rv;
                }
            }
        }
        block_append(mask, ns, count, tmp, [&](uint32_t slot, int j) {
            x_idx[slot] = (int32_t)(v0 + j);
            x_val[slot] = xv[j];
        });
    }
}

// r += d y (the product of the last round, when the rounds stop at the
// product limit).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pr_fold(int32_t n, T d, const T* __restrict__ y, T* __restrict__ r) {
#pragma clang fp contract(off)
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        const T dy = d * y[v];
        r[v] = r[v] + dy;
    }
}

static int flat_grid(int32_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kBlock), 4096)); }

template <typename T>
static spx_status pr_t(const PrArgs& a, hipStream_t s) {
    switch (a.stage) {
        case PR_COLSUM:
            k_pr_colsum<T><<<flat_grid(a.n), kBlock, 0, s>>>(a.n, a.col_ptr, (const T*)a.vals_csc, (T*)a.W, a.bad);
            break;
        case PR_INIT:
            k_pr_init<T><<<flat_grid(a.n), kBlock, 0, s>>>(a.n, (T)((1.0 - a.damping) / a.n), (T*)a.r, (T*)a.p);
            break;
        case PR_SELECT: {
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(a.n, kChunk), 2048));
            Count* c = (Count*)a.count;
            k_pr_select<T><<<grid, kBlock, 0, s>>>(a.n, (T)a.damping, (T)a.eps, (const T*)a.y, (T*)a.r, (T*)a.p,
                                                   (const T*)a.W, a.col_ptr, a.x_idx, (T*)a.x_val, c + (a.round & 1),
                                                   c + ((a.round - 1) & 1));
            break;
        }
        case PR_FOLD:
            k_pr_fold<T><<<flat_grid(a.n), kBlock, 0, s>>>(a.n, (T)a.damping, (const T*)a.y, (T*)a.r);
            break;
        default:
            return fail(SPX_ERR_ARG, "PageRank: unknown stage");
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status launch_pagerank(const PrArgs& a, hipStream_t s) {
    if (a.n <= 0) return SPX_OK;
    if (a.dtype == SPX_F32) return pr_t<float>(a, s);
    if (a.dtype == SPX_F64) return pr_t<double>(a, s);
    return fail(SPX_ERR_DTYPE, "PageRank supports F32 and F64");
}

}  // namespace spx
