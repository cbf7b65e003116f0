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
// next product y = A x, as a list and as a dense vector, so that no
// conversion runs before a row-major kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "frontier.hpp"
#include "internal.hpp"

namespace spx {

// bad gets bit 0 if a stored weight is negative (one atomic per wave that
// sees one). The column sums themselves are a product: W = A^T 1.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pr_negcheck(int64_t nnz, const T* __restrict__ vals,
                                                        uint32_t* __restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    bool neg = false;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz; k += stride) neg |= vals[k] < (T)0;
    if (__ballot(neg) && lane_id() == 0) atomicOr(bad, 1u);
}

// v = 1 everywhere (the x of W = A^T 1).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pr_ones(int32_t n, T* __restrict__ v) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) v[i] = (T)1;
}

// r = r0 everywhere, p = 0, and the dense x buffer of round 0 zeroed.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pr_init(int32_t n, T r0, T* __restrict__ r, T* __restrict__ p,
                                                    T* __restrict__ xd0) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride) {
        r[v] = r0;
        p[v] = (T)0;
        xd0[v] = (T)0;
    }
}

// Eight consecutive values from v0 (a multiple of 8; the array 16-byte
// aligned), as 16-byte loads; element by element at the tail.
template <typename T>
__device__ __forceinline__ void load8(const T* __restrict__ a, int64_t v0, int32_t n, T (&o)[kVpt]) {
    if (v0 + kVpt <= n) {
        constexpr int nv = kVpt * sizeof(T) / 16;
        const uint4* q = (const uint4*)(a + v0);
        uint4 w[nv];
#pragma unroll
        for (int u = 0; u < nv; ++u) w[u] = q[u];
        __builtin_memcpy(o, w, sizeof(o));
    } else {
#pragma unroll
        for (int j = 0; j < kVpt; ++j) o[j] = v0 + j < n ? a[v0 + j] : (T)0;
    }
}

template <typename T>
__device__ __forceinline__ void store8(T* __restrict__ a, int64_t v0, int32_t n, const T (&o)[kVpt]) {
    if (v0 + kVpt <= n) {
        constexpr int nv = kVpt * sizeof(T) / 16;
        uint4 w[nv];
        __builtin_memcpy(w, o, sizeof(o));
        uint4* q = (uint4*)(a + v0);
#pragma unroll
        for (int u = 0; u < nv; ++u) q[u] = w[u];
    } else {
#pragma unroll
        for (int j = 0; j < kVpt; ++j)
            if (v0 + j < n) a[v0 + j] = o[j];
    }
}

// One round. y = nullptr on the first round (no product yet). The counter
// gets {appended entries of x (low), their column lengths (high), i.e. the
// nnz_s of the next product}; count_clear is zeroed for the next round.
// Besides the list (x_idx, x_val), x goes dense into xd_fill at position
// map[v] (the column order of the row-major copy; v itself when map is
// null): xd_fill was zeroed by the previous round, and this round zeroes
// xd_clear for the next one (two buffers alternate, each zeroed while the
// other is in use). r += d y is rounded as a product and then a sum (no
// fused multiply-add), the order the definition states. r, p, y, W,
// col_ptr, map and xd_clear are 16-byte aligned.
template <typename T>
__global__ __launch_bounds__(kWideBlock) void k_pr_select(int32_t n, T d, T eps, const T* __restrict__ y,
                                                      T* __restrict__ r, T* __restrict__ p,
                                                      const T* __restrict__ W, const int32_t* __restrict__ col_ptr,
                                                      const int32_t* __restrict__ map, int32_t* __restrict__ x_idx,
                                                      T* __restrict__ x_val, T* __restrict__ xd_fill,
                                                      T* __restrict__ xd_clear, Count* __restrict__ count,
                                                      Count* __restrict__ count_clear) {
#pragma clang fp contract(off)
    __shared__ Count tmp[kWideBlock / kWave];
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_clear = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWideChunk; base < n; base += (int64_t)gridDim.x * kWideChunk) {
        const int64_t v0 = base + (int64_t)threadIdx.x * kVpt;
        // all loads of a phase are independent, so they are in flight together
        T rv[kVpt], wv[kVpt], xv[kVpt];
        load8(r, v0, n, rv);
        load8(W, v0, n, wv);
        if (y) {
            T yv[kVpt];
            load8(y, v0, n, yv);
#pragma unroll
            for (int j = 0; j < kVpt; ++j) {
                const T dy = d * yv[j];
                rv[j] = rv[j] + dy;
            }
        }
        uint32_t act = 0;
#pragma unroll
        for (int j = 0; j < kVpt; ++j)
            if (v0 + j < n && (rv[j] > eps || rv[j] < -eps)) act |= 1u << j;
        uint32_t mask = 0, ns = 0;
#pragma unroll
        for (int j = 0; j < kVpt; ++j) xv[j] = (T)0;
        if (act) {
            // the rank, the column pointers and the map of the thread's
            // vertices only when one of them is active
            T pv[kVpt];
            int32_t cp[kVpt], mp[kVpt];
            load8(p, v0, n, pv);
            load8(col_ptr, v0, n, cp);
            if (map) load8(map, v0, n, mp);
#pragma unroll
            for (int j = 0; j < kVpt; ++j) {
                if (!((act >> j) & 1u)) continue;
                pv[j] = pv[j] + rv[j];
                if (wv[j] > (T)0) {
                    mask |= 1u << j;
                    xv[j] = rv[j] / wv[j];
                    // end of column v0 + j (col_ptr has n + 1 entries)
                    const int32_t next = j + 1 < kVpt && v0 + j + 1 < n ? cp[j + 1] : col_ptr[v0 + j + 1];
                    ns += (uint32_t)(next - cp[j]);
                    xd_fill[map ? mp[j] : v0 + j] = xv[j];
                }
                rv[j] = (T)0;
            }
            store8(p, v0, n, pv);
        }
        if (y || act) store8(r, v0, n, rv);
        const T zero[kVpt] = {};
        store8(xd_clear, v0, n, zero);
        block_append<kWideBlock>(mask, ns, count, tmp, [&](uint32_t slot, int j) {
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
        case PR_NEGCHECK: {
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(a.nnz, kBlock), 4096));
            k_pr_negcheck<T><<<grid, kBlock, 0, s>>>(a.nnz, (const T*)a.vals_csc, a.bad);
            break;
        }
        case PR_ONES:
            k_pr_ones<T><<<flat_grid(a.n), kBlock, 0, s>>>(a.n, (T*)a.ones);
            break;
        case PR_INIT:
            k_pr_init<T><<<flat_grid(a.n), kBlock, 0, s>>>(a.n, (T)((1.0 - a.damping) / a.n), (T*)a.r, (T*)a.p,
                                                           (T*)a.xd[0]);
            break;
        case PR_SELECT: {
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(a.n, kWideChunk), 2048));
            Count* c = (Count*)a.count;
            k_pr_select<T><<<grid, kWideBlock, 0, s>>>(a.n, (T)a.damping, (T)a.eps, (const T*)a.y, (T*)a.r, (T*)a.p,
                                                   (const T*)a.W, a.col_ptr, a.map, a.x_idx, (T*)a.x_val,
                                                   (T*)a.xd[a.round & 1], (T*)a.xd[(a.round + 1) & 1],
                                                   c + (a.round & 1), c + ((a.round - 1) & 1));
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
