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

// Vertices per thread: a workgroup owns NT * kVpt consecutive vertices and
// appends the ones it selects with a single atomic on the counter. Atomics
// on one word serialize (about 12 ns each on this GPU, so one per wave
// costs more than the rest of a level on a large frontier, and even one
// per 256-thread workgroup costs about 6 µs at n = 2^20): the streaming
// kernels therefore run 1024-thread workgroups (kWideBlock), the same
// threads in a quarter of the atomics.
constexpr int kVpt = 8;
constexpr int kChunk = kBlock * kVpt;
constexpr int kWideBlock = 1024;
constexpr int kWideChunk = kWideBlock * kVpt;

// Inclusive prefix sum across an NT-thread workgroup; tmp holds NT / 64
// elements of LDS; *total gets the workgroup total. Contains __syncthreads.
template <int NT, typename T>
__device__ __forceinline__ T block_scan_nt(T v, T* tmp, T* total) {
    constexpr int W = NT / kWave;
    T w = wave_incl_scan(v);
    if (lane_id() == kWave - 1) tmp[wave_id()] = w;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const T t = tmp[i];
        if (i < wave_id()) pre += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return w + pre;
}

// Thread t holds the candidates v0 + j for the set bits j of mask, and
// high, its share of the counter's high half. The workgroup (NT threads)
// reserves one range of the list and calls emit(slot, j) for each
// candidate, slots ascending with the vertex. Contains __syncthreads;
// every thread of the workgroup must call it. tmp: NT / 64 words of LDS.
template <int NT, typename Emit>
__device__ __forceinline__ void block_append(uint32_t mask, uint32_t high, Count* __restrict__ count, Count* tmp,
                                             Emit emit) {
    const Count mine = ((Count)high << 32) | (Count)__popc(mask);
    Count total;
    const Count incl = block_scan_nt<NT, Count>(mine, tmp, &total);
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
template <int NT>
__device__ __forceinline__ void block_append(uint32_t mask, int64_t v0, uint32_t high, int32_t* __restrict__ next,
                                             Count* __restrict__ count, Count* tmp) {
    block_append<NT>(mask, high, count, tmp, [&](uint32_t slot, int j) { next[slot] = (int32_t)(v0 + j); });
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
