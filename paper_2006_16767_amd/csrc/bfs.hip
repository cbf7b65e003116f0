// Breadth-first search driver: every level is one adaptive (OR, AND)
// SpMSpV of the frontier (the application the paper evaluates its kernels
// in, Section 7), so the kernel follows the frontier's density from level
// to level. A level's product y = A (x) f marks every vertex with an edge
// from the frontier; the update kernel keeps the unvisited ones, labels
// them and appends them to the next frontier.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

__global__ __launch_bounds__(kBlock) void k_bfs_seed(int32_t n, int32_t source, int32_t* __restrict__ level,
                                                     int32_t* __restrict__ frontier, int32_t* __restrict__ count) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride)
        level[v] = v == source ? 0 : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        frontier[0] = source;
        *count = 0;
    }
}

// Vertices reached by the product and not labelled yet get level L and go
// to the next frontier; each wave reserves its slots with one atomic.
__global__ __launch_bounds__(kBlock) void k_bfs_update(int32_t n, const uint8_t* __restrict__ y, int32_t L,
                                                       int32_t* __restrict__ level, int32_t* __restrict__ next,
                                                       int32_t* __restrict__ count) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n; base += stride) {
        const int64_t v = base + threadIdx.x;
        const bool hit = v < n && y[v] && level[v] < 0;
        if (hit) level[v] = L;
        const uint64_t mask = __ballot(hit);
        const int lane = lane_id();
        int32_t slot = 0;
        if (lane == 0 && mask) slot = atomicAdd(count, (int32_t)__popcll(mask));
        slot = __shfl(slot, 0);
        if (hit) next[slot + __popcll(mask & ((1ull << lane) - 1))] = (int32_t)v;
    }
}

spx_status launch_bfs_seed(int32_t n, int32_t source, int32_t* level, int32_t* frontier, int32_t* count,
                           hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kBlock), 4096));
    k_bfs_seed<<<grid, kBlock, 0, s>>>(n, source, level, frontier, count);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status launch_bfs_update(int32_t n, const uint8_t* y, int32_t L, int32_t* level, int32_t* next, int32_t* count,
                             hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kBlock), 4096));
    k_bfs_update<<<grid, kBlock, 0, s>>>(n, y, L, level, next, count);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

}  // namespace spx
