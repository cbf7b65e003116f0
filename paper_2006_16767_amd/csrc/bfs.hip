// Breadth-first search driver: every level is one adaptive (OR, AND)
// SpMSpV of the frontier (the application the paper evaluates its kernels
// in, Section 7), so the kernel follows the frontier's density from level
// to level. A level's product y = A (x) f marks every vertex with an edge
// from the frontier; the update kernel keeps the unvisited ones, labels
// them and appends them to the next frontier. When the frontier's edges
// outweigh the unexplored ones, a level can instead run the masked pull
// kernel, which reads only the rows of unvisited vertices and stops each at
// its first frontier neighbour.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "frontier.hpp"
#include "internal.hpp"

namespace spx {

// Two counters alternate between levels: level L appends into count[L & 1]
// and clears the other one for level L + 1 (the host has read it before
// level L is enqueued, on the same stream).
//
// level = -1 except the source (0); the frontier is the source, as a list
// and as a bitvector; count[0] holds {1 vertex, out-degree of the source}
// and count[1] is cleared.
__global__ __launch_bounds__(kBlock) void k_bfs_seed(int32_t n, int32_t source, const int32_t* __restrict__ col_ptr,
                                                     int32_t* __restrict__ level, int32_t* __restrict__ frontier,
                                                     uint32_t* __restrict__ bits, Count* __restrict__ count) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += stride)
        level[v] = v == source ? 0 : -1;
    const int64_t words = ceil_div((int64_t)n, 32);
    for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < words; w += stride)
        bits[w] = w == source >> 5 ? 1u << (source & 31) : 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        frontier[0] = source;
        count[0] = ((Count)(uint32_t)(col_ptr[source + 1] - col_ptr[source]) << 32) | 1ull;
        count[1] = 0;
    }
}

// Vertices reached by the product and not labelled yet get level L and go
// to the next frontier. Thread t of a chunk owns its 8 consecutive vertices.
__global__ __launch_bounds__(kWideBlock) void k_bfs_update(int32_t n, const uint8_t* __restrict__ y, int32_t L,
                                                       const int32_t* __restrict__ col_ptr,
                                                       int32_t* __restrict__ level, int32_t* __restrict__ next,
                                                       uint32_t* __restrict__ next_bits,
                                                       Count* __restrict__ count, Count* __restrict__ count_clear) {
    __shared__ Count tmp[kWideBlock / kWave];
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_clear = 0;
    for (int64_t base = (int64_t)blockIdx.x * kWideChunk; base < n; base += (int64_t)gridDim.x * kWideChunk) {
        const int64_t v0 = base + (int64_t)threadIdx.x * kVpt;
        uint64_t yy = 0;
        if (v0 + kVpt <= n) {
            yy = *(const uint64_t*)(y + v0);  // y is 256-byte aligned and v0 a multiple of 8
        } else {
            for (int j = 0; v0 + j < n; ++j) yy |= (uint64_t)(y[v0 + j] != 0) << (8 * j);
        }
        uint32_t mask = 0, deg = 0;
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            if ((yy >> (8 * j)) & 0xffu) {
                const int64_t v = v0 + j;
                if (level[v] < 0) {
                    level[v] = L;
                    mask |= 1u << j;
                    deg += (uint32_t)(col_ptr[v + 1] - col_ptr[v]);
                }
            }
        }
        write_bits(mask, v0, n, next_bits);
        block_append<kWideBlock>(mask, v0, deg, next, count, tmp);
    }
}

// Masked pull (the row-major expansion restricted to the unvisited rows,
// with early exit). Row i of A lists the vertices with an edge into i; an
// unvisited i joins level L at its first entry in the frontier's
// bitvector (written by the previous level). Per chunk of kChunk rows:
//   A. each thread takes 8 rows strided by the workgroup size (coalesced)
//      and tests their first two entries, all loads independent;
//   B. the rows still open are listed in LDS and scanned by one wave each,
//      256 entries per step, stopping at the first hit;
//   C. each thread labels and appends its 8 consecutive rows' hits.
// Rows of visited vertices are not read.
__device__ __forceinline__ bool in_bits(const uint32_t* __restrict__ bits, int32_t c) {
    return (bits[c >> 5] >> (c & 31)) & 1u;
}

__global__ __launch_bounds__(kBlock) void k_bfs_pull(int32_t n, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx,
                                                     const uint32_t* __restrict__ bits, int32_t L,
                                                     const int32_t* __restrict__ col_ptr,
                                                     int32_t* __restrict__ level, int32_t* __restrict__ next,
                                                     uint32_t* __restrict__ next_bits,
                                                     Count* __restrict__ count, Count* __restrict__ count_clear) {
    __shared__ uint8_t hit[kChunk];
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_clear = 0;
    __shared__ int16_t open[kChunk];
    __shared__ int n_open;
    __shared__ Count tmp[kWavesPerBlock];
    for (int64_t base = (int64_t)blockIdx.x * kChunk; base < n; base += (int64_t)gridDim.x * kChunk) {
        if (threadIdx.x == 0) n_open = 0;
        __syncthreads();
        // A
        int32_t k0[kVpt], k1[kVpt];
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            const int64_t r = base + j * kBlock + threadIdx.x;
            k0[j] = k1[j] = 0;
            if (r < n && level[r] < 0) {
                k0[j] = row_ptr[r];
                k1[j] = row_ptr[r + 1];
            }
        }
        int32_t c0[kVpt], c1[kVpt];
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            c0[j] = k1[j] > k0[j] ? col_idx[k0[j]] : -1;
            c1[j] = k1[j] > k0[j] + 1 ? col_idx[k0[j] + 1] : -1;
        }
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            const bool h = (c0[j] >= 0 && in_bits(bits, c0[j])) || (c1[j] >= 0 && in_bits(bits, c1[j]));
            const int p = j * kBlock + threadIdx.x;
            hit[p] = h;
            if (!h && k1[j] > k0[j] + 2) open[atomicAdd(&n_open, 1)] = (int16_t)p;
        }
        __syncthreads();
        // B
        const int no = n_open, lane = lane_id();
        for (int q = wave_id(); q < no; q += kWavesPerBlock) {
            const int p = open[q];
            const int64_t r = base + p;
            const int32_t e = row_ptr[r + 1];
            bool found = false;
            for (int32_t kb = row_ptr[r] + 2; kb < e && !found; kb += 4 * kWave) {
                bool h = false;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t k = kb + u * kWave + lane;
                    h |= k < e && in_bits(bits, col_idx[k]);
                }
                found = __ballot(h) != 0;
            }
            if (found && lane == 0) hit[p] = 1;
        }
        __syncthreads();
        // C
        const int64_t v0 = base + (int64_t)threadIdx.x * kVpt;
        uint32_t mask = 0, deg = 0;
#pragma unroll
        for (int j = 0; j < kVpt; ++j) {
            if (hit[threadIdx.x * kVpt + j]) {
                const int64_t v = v0 + j;
                level[v] = L;
                mask |= 1u << j;
                deg += (uint32_t)(col_ptr[v + 1] - col_ptr[v]);
            }
        }
        write_bits(mask, v0, n, next_bits);
        block_append<kBlock>(mask, v0, deg, next, count, tmp);
    }
}

spx_status launch_bfs_seed(int32_t n, int32_t source, const int32_t* col_ptr, int32_t* level, int32_t* frontier,
                           uint32_t* bits, void* count, hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kBlock), 4096));
    k_bfs_seed<<<grid, kBlock, 0, s>>>(n, source, col_ptr, level, frontier, bits, (Count*)count);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status launch_bfs_update(int32_t n, const uint8_t* y, int32_t L, const int32_t* col_ptr, int32_t* level,
                             int32_t* next, uint32_t* next_bits, void* count, hipStream_t s) {
    if ((uintptr_t)y % 8) return fail(SPX_ERR_ARG, "breadth-first search: product buffer must be 8-byte aligned");
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kWideChunk), 2048));
    Count* c = (Count*)count;
    k_bfs_update<<<grid, kWideBlock, 0, s>>>(n, y, L, col_ptr, level, next, next_bits, c + (L & 1), c + ((L - 1) & 1));
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status launch_bfs_pull(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* bits,
                           int32_t L, const int32_t* col_ptr, int32_t* level, int32_t* next, uint32_t* next_bits,
                           void* count, hipStream_t s) {
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kChunk), 2048));
    Count* c = (Count*)count;
    k_bfs_pull<<<grid, kBlock, 0, s>>>(n, row_ptr, col_idx, bits, L, col_ptr, level, next, next_bits, c + (L & 1),
                                       c + ((L - 1) & 1));
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

}  // namespace spx
