// Shared device-side building blocks of libspx (gfx950, wave64).
//
// Semiring traits for the four value types, wave-level reductions and
// scans, and the merge-path search used by every load-balanced kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spx.h"

namespace spx {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup in every kernel
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------------------
// Semiring traits. V: stored matrix value, X: vector value, Acc: accumulator,
// Y: output element.
//   F32 / F64 : real (+, *)
//   I32       : (+, *) modulo 2^32 (unsigned accumulation, int32 output)
//   BOOL      : (OR, AND) over the pattern; x values and A values are not read
//   F32_MINPLUS: (min, +) over float32; zero +inf, absent x entries +inf
// ---------------------------------------------------------------------------
template <int DT>
struct SR;

template <>
struct SR<SPX_F32> {
    using V = float;
    using X = float;
    using Acc = float;
    using Y = float;
    static constexpr bool kVals = true;
    __device__ static Acc zero() { return 0.0f; }
    __device__ static V val(const V* __restrict__ v, int64_t k) { return v[k]; }
    __device__ static X xval(const X* __restrict__ x, int64_t j) { return x[j]; }
    __device__ static Acc mul(V a, X b) { return a * b; }
    __device__ static Acc fma(V a, X b, Acc c) { return __builtin_fmaf(a, b, c); }
    __device__ static Acc add(Acc a, Acc b) { return a + b; }
    __device__ static Y out(Acc a) { return a; }
    __device__ static bool nonzero(Acc a) { return a != 0.0f; }
    __device__ static bool present(X x) { return x != 0.0f; }
    __device__ static void atomic_add(Y* p, Acc v) { unsafeAtomicAdd(p, v); }
    __device__ static void lds_atomic_add(Acc* p, Acc v) { atomicAdd(p, v); }
};

// float32 minimum as integer atomics: non-negative floats order like their
// int bits, negative ones like their unsigned bits reversed.
__device__ __forceinline__ void atomic_min_f32(float* p, float v) {
    if (v >= 0.0f)
        atomicMin((int*)p, __float_as_int(v));
    else
        atomicMax((unsigned int*)p, __float_as_uint(v));
}

// (min, +) over float32: the zero is +inf, a product is a sum (one float32
// rounding), a sum is a minimum.
template <>
struct SR<SPX_F32_MINPLUS> {
    using V = float;
    using X = float;
    using Acc = float;
    using Y = float;
    static constexpr bool kVals = true;
    __device__ static Acc zero() { return __builtin_inff(); }
    __device__ static V val(const V* __restrict__ v, int64_t k) { return v[k]; }
    __device__ static X xval(const X* __restrict__ x, int64_t j) { return x[j]; }
    __device__ static Acc mul(V a, X b) { return a + b; }
    __device__ static Acc fma(V a, X b, Acc c) { return fminf(c, a + b); }
    __device__ static Acc add(Acc a, Acc b) { return fminf(a, b); }
    __device__ static Y out(Acc a) { return a; }
    __device__ static bool nonzero(Acc a) { return a != __builtin_inff(); }
    __device__ static bool present(X x) { return x != __builtin_inff(); }
    __device__ static void atomic_add(Y* p, Acc v) { atomic_min_f32(p, v); }
    __device__ static void lds_atomic_add(Acc* p, Acc v) { atomic_min_f32(p, v); }
};

template <>
struct SR<SPX_F64> {
    using V = double;
    using X = double;
    using Acc = double;
    using Y = double;
    static constexpr bool kVals = true;
    __device__ static Acc zero() { return 0.0; }
    __device__ static V val(const V* __restrict__ v, int64_t k) { return v[k]; }
    __device__ static X xval(const X* __restrict__ x, int64_t j) { return x[j]; }
    __device__ static Acc mul(V a, X b) { return a * b; }
    __device__ static Acc fma(V a, X b, Acc c) { return __builtin_fma(a, b, c); }
    __device__ static Acc add(Acc a, Acc b) { return a + b; }
    __device__ static Y out(Acc a) { return a; }
    __device__ static bool nonzero(Acc a) { return a != 0.0; }
    __device__ static bool present(X x) { return x != 0.0; }
    __device__ static void atomic_add(Y* p, Acc v) { unsafeAtomicAdd(p, v); }
    __device__ static void lds_atomic_add(Acc* p, Acc v) { atomicAdd(p, v); }
};

template <>
struct SR<SPX_I32> {
    using V = int32_t;
    using X = int32_t;
    using Acc = uint32_t;
    using Y = int32_t;
    static constexpr bool kVals = true;
    __device__ static Acc zero() { return 0u; }
    __device__ static V val(const V* __restrict__ v, int64_t k) { return v[k]; }
    __device__ static X xval(const X* __restrict__ x, int64_t j) { return x[j]; }
    __device__ static Acc mul(V a, X b) { return (uint32_t)a * (uint32_t)b; }
    __device__ static Acc fma(V a, X b, Acc c) { return c + (uint32_t)a * (uint32_t)b; }
    __device__ static Acc add(Acc a, Acc b) { return a + b; }
    __device__ static Y out(Acc a) { return (int32_t)a; }
    __device__ static bool nonzero(Acc a) { return a != 0u; }
    __device__ static bool present(X x) { return x != 0; }
    __device__ static void atomic_add(Y* p, Acc v) { atomicAdd((uint32_t*)p, v); }
    __device__ static void lds_atomic_add(Acc* p, Acc v) { atomicAdd(p, v); }
};

template <>
struct SR<SPX_BOOL> {
    using V = uint8_t;  // never read
    using X = uint8_t;  // dense x: 0/1 mask; sparse x: values never read
    using Acc = uint32_t;
    using Y = uint8_t;
    static constexpr bool kVals = false;
    __device__ static Acc zero() { return 0u; }
    __device__ static V val(const V* __restrict__, int64_t) { return 1; }
    __device__ static X xval(const X* __restrict__ x, int64_t j) { return x ? x[j] : (X)1; }
    __device__ static Acc mul(V, X b) { return b != 0; }
    __device__ static Acc fma(V, X b, Acc c) { return c | (Acc)(b != 0); }
    __device__ static Acc add(Acc a, Acc b) { return a | b; }
    __device__ static Y out(Acc a) { return a ? 1 : 0; }
    __device__ static bool nonzero(Acc a) { return a != 0u; }
    __device__ static bool present(X x) { return x != 0; }
    // OR is idempotent: racing writers store the same byte.
    __device__ static void atomic_add(Y* p, Acc v) {
        if (v) *p = 1;
    }
    __device__ static void lds_atomic_add(Acc* p, Acc v) {
        if (v) *p = 1u;
    }
};

// ---------------------------------------------------------------------------
// Bounded accumulation chains. A kernel that walks a long row (or column)
// keeps U independent partial sums, one per unrolled load slot, and every
// kFoldRounds rounds folds them pairwise into an outer sum. No single FP32
// accumulator then takes more than kFoldRounds + (length / (U * kFoldRounds))
// rounded additions, which keeps the error of a 10^5-entry row within the
// 1e-5 * sum |a_ij x_j| bound (a single serial chain over 2 * 10^5 positive
// terms exceeds it). Exact semirings are unaffected.
// ---------------------------------------------------------------------------
constexpr int kFoldRounds = 64;

template <int DT, int U>
struct ChunkedAcc {
    using Acc = typename SR<DT>::Acc;
    Acc part[U];
    Acc outer;
    int rounds;
    __device__ __forceinline__ ChunkedAcc() : outer(SR<DT>::zero()), rounds(0) {
#pragma unroll
        for (int u = 0; u < U; ++u) part[u] = SR<DT>::zero();
    }
    // pairwise sum of the U partials (U a power of two)
    __device__ __forceinline__ Acc tree() const {
        Acc t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = part[u];
#pragma unroll
        for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
            for (int u = 0; u < w; ++u) t[u] = SR<DT>::add(t[u], t[u + w]);
        return t[0];
    }
    // call once after every round of U slot updates
    __device__ __forceinline__ void end_round() {
        if (++rounds == kFoldRounds) {
            outer = SR<DT>::add(outer, tree());
#pragma unroll
            for (int u = 0; u < U; ++u) part[u] = SR<DT>::zero();
            rounds = 0;
        }
    }
    __device__ __forceinline__ Acc total() const { return SR<DT>::add(outer, tree()); }
};

// ---------------------------------------------------------------------------
// Wave primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int mask) {
    return __shfl_xor(v, mask, kWave);
}

template <typename T>
__device__ __forceinline__ T shfl_up(T v, int delta) {
    return __shfl_up(v, delta, kWave);
}

// Reduction across groups of L consecutive lanes (L a power of two <= 64):
// every lane of a group ends with the group total.
template <int DT, int L>
__device__ __forceinline__ typename SR<DT>::Acc group_reduce(typename SR<DT>::Acc a) {
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) a = SR<DT>::add(a, shfl_xor(a, off));
    return a;
}

// Inclusive prefix sum across the wave (int32 or int64).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = shfl_up(v, d);
        if (l >= d) v += o;
    }
    return v;
}

// Inclusive prefix sum across a 256-thread workgroup. `tmp` holds
// kWavesPerBlock elements of LDS. Returns the inclusive value; *total gets
// the workgroup total. Contains __syncthreads.
template <typename T>
__device__ __forceinline__ T block_incl_scan(T v, T* tmp, T* total) {
    T w = wave_incl_scan(v);
    if (lane_id() == kWave - 1) tmp[wave_id()] = w;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
        T t = tmp[i];
        if (i < wave_id()) pre += t;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return w + pre;
}

// ---------------------------------------------------------------------------
// Merge-path search (the load-balanced distribution).
//
// A sequence of R groups with inclusive end offsets ends[0..R-1] (for CSR:
// ends[i] = row_ptr[i+1]; for a sparse x over CSC: ends[e] = running total
// of the selected column lengths) is merged with its K = ends[R-1] items.
// Group i's end event happens after all of its items, so the merged order
// places it at step ends[i] + i. After d merge steps the number of finished
// groups is the first i with ends[i] + i >= d (R if none); d - that count
// items have been consumed.
//
// The whole wave cooperates: each round probes 64 positions and keeps the
// interval between the last false and the first true probe. Every lane
// returns the same result.
// ---------------------------------------------------------------------------
template <typename EndsFn>
__device__ __forceinline__ int merge_search_wave(EndsFn ends, int R, int64_t d) {
    int lo = 0, hi = R;
    const int l = lane_id();
    while (lo < hi) {
        const int64_t span = hi - lo;
        const int p = lo + (int)((span * l) / kWave);
        const bool pred = (p < hi) && ((int64_t)ends(p) + p >= d);
        const uint64_t mask = __ballot(pred);
        if (mask == 0) {
            const int plast = lo + (int)((span * (kWave - 1)) / kWave);
            lo = plast + 1;
        } else {
            const int f = __ffsll((unsigned long long)mask) - 1;
            const int pf = lo + (int)((span * f) / kWave);
            const int pprev = f > 0 ? lo + (int)((span * (f - 1)) / kWave) : lo - 1;
            hi = pf;
            lo = pprev + 1;
        }
    }
    return lo;
}

// Same search, one thread, over an LDS array.
template <typename T>
__device__ __forceinline__ int merge_search_lds(const T* ends, int R, int64_t d, int64_t base) {
    int lo = 0, hi = R;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((int64_t)ends[mid] - base + mid >= d)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ bool test_bit(const uint32_t* __restrict__ bits, int j) {
    return (bits[j >> 5] >> (j & 31)) & 1u;
}

}  // namespace spx
