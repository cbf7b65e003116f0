// Frontier appends shared by the graph drivers (breadth-first search and
// PageRank): a workgroup owns kChunk consecutive vertices, 8 per thread,
// and appends the ones it selects to an output list with one atomic on a
// packed counter.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace spx {

// A counter is one 64-bit word of two halves that are added together: the
// low half counts the vertices appended to the list, the high half holds a
// per-driver sum (both drivers: the column lengths of the appended
// vertices, i.e. nnz_s of the next product). Neither half can carry into the other (both stay below
// 2^31), so one atomic add updates both.
using Count = unsigned long long;

// Vertices per thread: a workgroup owns kChunk consecutive vertices and
// appends the ones it selects with a single atomic on the counter (one
// atomic per wave, all on the same word, costs more than the rest of a
// level on a large frontier).
constexpr int kVpt = 8;
constexpr int kChunk = kBlock * kVpt;

// Thread t holds the candidates v0 + j for the set bits j of mask, and
// high, its share of the counter's high half. The workgroup reserves one
// range of the list and calls emit(slot, j) for each candidate, slots
// ascending with the vertex. Contains __syncthreads; every thread of the
// workgroup must call it. tmp: kWavesPerBlock words of LDS.
template <typename Emit>
__device__ __forceinline__ void block_append(uint32_t mask, uint32_t high, Count* __restrict__ count, Count* tmp,
                                             Emit emit) {
    const Count mine = ((Count)high << 32) | (Count)__popc(mask);
    Count total;
    const Count incl = block_incl_scan<Count>(mine, tmp, &total);
    __shared__ Count base;
    if (threadIdx.x == 0) base = total ? atomicAdd(count, total) : 0ull;
    __syncthreads();
    uint32_t slot = (uint32_t)base + (uint32_t)(incl - mine);
    while (mask) {
        const int j = __ffs(mask) - 1;
        mask &= mask - 1;
        emit(slot++, j);
    }
    __syncthreads();  // base is reused by the next chunk
}

// The vertex list form: next[slot] = v0 + j.
__device__ __forceinline__ void block_append(uint32_t mask, int64_t v0, uint32_t high, int32_t* __restrict__ next,
                                             Count* __restrict__ count, Count* tmp) {
    block_append(mask, high, count, tmp, [&](uint32_t slot, int j) { next[slot] = (int32_t)(v0 + j); });
}

// Writes the next frontier's bitvector for the 8 consecutive vertices
// v0.. of every thread (v0 a multiple of 8): the four threads of one
// 32-bit word are neighbouring lanes. Every lane of the wave must call it.
__device__ __forceinline__ void write_bits(uint32_t mask8, int64_t v0, int32_t n, uint32_t* __restrict__ bits) {
    const uint32_t b1 = __shfl_down(mask8, 1, kWave), b2 = __shfl_down(mask8, 2, kWave),
                   b3 = __shfl_down(mask8, 3, kWave);
    if ((threadIdx.x & 3) == 0 && v0 < n) bits[v0 >> 5] = mask8 | b1 << 8 | b2 << 16 | b3 << 24;
}

}  // namespace spx
