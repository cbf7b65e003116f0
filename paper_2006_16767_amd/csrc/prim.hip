// Device primitives of libspx: fills, exclusive scan, stable LSD radix sort
// of (key, value) pairs, row expansion, permutation gather, vector format
// conversions (Section 6.3: done on the GPU with reduction, prefix sum and
// stream compaction) and the feature reductions of Table 1.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

// ------------------------------------------------------------------ fills
// A plain kernel (not hipMemsetAsync) so that the same code can be recorded
// into a HIP graph.
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v,
                                                     int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < n; i += stride) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_u8(uint8_t* __restrict__ p, uint8_t v,
                                                    int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < n; i += stride) p[i] = v;
}

static int fill_grid(int64_t n) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kBlock), 4096));
}

spx_status fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s) {
    if (count == 0) return SPX_OK;
    k_fill_u32<<<fill_grid(count), kBlock, 0, s>>>(p, v, (int64_t)count);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status fill_bytes(void* p, uint8_t v, size_t bytes, hipStream_t s) {
    if (bytes == 0) return SPX_OK;
    if (((uintptr_t)p & 3) == 0 && (bytes & 3) == 0) {
        uint32_t w = v * 0x01010101u;
        return fill_u32((uint32_t*)p, w, bytes / 4, s);
    }
    k_fill_u8<<<fill_grid(bytes), kBlock, 0, s>>>((uint8_t*)p, v, (int64_t)bytes);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// ------------------------------------------------------------------ streaming copy
// The achievable-bandwidth reference of the measurements: a plain copy with
// 16-byte loads and stores in which every workgroup copies its own
// contiguous 16 KiB (four loads in flight per thread, then four stores).
// On MI355X this one-chunk-per-workgroup shape streamed a 1 GiB copy at
// 5.8 TB/s, against 4.4-4.7 TB/s for grid-stride loops of the same loads
// (and 5.3 TB/s for the runtime's device-to-device copy).
constexpr int kCopyU = 4;
__global__ __launch_bounds__(kBlock) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                        int64_t n16) {
    const int64_t base = (int64_t)blockIdx.x * kBlock * kCopyU + threadIdx.x;
    uint4 a[kCopyU];
#pragma unroll
    for (int u = 0; u < kCopyU; ++u)
        if (base + u * kBlock < n16) a[u] = src[base + u * kBlock];
#pragma unroll
    for (int u = 0; u < kCopyU; ++u)
        if (base + u * kBlock < n16) dst[base + u * kBlock] = a[u];
}

}  // namespace spx

extern "C" spx_status spx_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
    using namespace spx;
    if (bytes == 0) return SPX_OK;
    if (!src || !dst) return fail(SPX_ERR_ARG, "stream copy: null pointer");
    if ((((uintptr_t)src | (uintptr_t)dst | bytes) & 15) != 0)
        return fail(SPX_ERR_ARG, "stream copy: pointers and size must be multiples of 16 bytes");
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t blocks = ceil_div(n16, (int64_t)kBlock * kCopyU);
    if (blocks > 0x7fffffff) return fail(SPX_ERR_ARG, "stream copy: more than 2^31 chunks of 16 KiB");
    k_stream_copy<<<(unsigned)blocks, kBlock, 0, (hipStream_t)stream>>>((const uint4*)src, (uint4*)dst, n16);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

namespace spx {

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of int32, reduce-then-scan over tiles of 2048.
constexpr int kScanIpt = 8;
constexpr int kScanTile = kBlock * kScanIpt;

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t* __restrict__ in,
                                                       int32_t* __restrict__ out, int64_t n,
                                                       int32_t* __restrict__ tile_sums,
                                                       int32_t* __restrict__ total) {
    __shared__ int32_t s_buf[kScanTile];
    __shared__ int32_t s_tmp[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int cnt = (int)std::min<int64_t>(kScanTile, n - base);
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) s_buf[i] = i < cnt ? in[base + i] : 0;
    __syncthreads();
    int32_t v[kScanIpt];
    int32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanIpt; ++i) {
        v[i] = s_buf[threadIdx.x * kScanIpt + i];
        sum += v[i];
    }
    int32_t tot;
    int32_t incl = block_incl_scan(sum, s_tmp, &tot);
    int32_t run = incl - sum;
#pragma unroll
    for (int i = 0; i < kScanIpt; ++i) {
        s_buf[threadIdx.x * kScanIpt + i] = run;
        run += v[i];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += kBlock) out[base + i] = s_buf[i];
    if (threadIdx.x == 0) {
        if (tile_sums) tile_sums[blockIdx.x] = tot;
        if (gridDim.x == 1 && total) *total = tot;
    }
}

// Single workgroup: exclusive scan of `count` values in place, total to *total.
__global__ __launch_bounds__(kBlock) void k_scan_single(int32_t* __restrict__ a, int64_t count,
                                                        int32_t* __restrict__ total) {
    __shared__ int32_t s_tmp[kWavesPerBlock];
    int32_t carry = 0;
    for (int64_t base = 0; base < count; base += kScanTile) {
        int32_t v[kScanIpt];
        int32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kScanIpt; ++i) {
            int64_t idx = base + threadIdx.x * kScanIpt + i;
            v[i] = idx < count ? a[idx] : 0;
            sum += v[i];
        }
        int32_t tot;
        int32_t incl = block_incl_scan(sum, s_tmp, &tot);
        int32_t run = carry + incl - sum;
#pragma unroll
        for (int i = 0; i < kScanIpt; ++i) {
            int64_t idx = base + threadIdx.x * kScanIpt + i;
            if (idx < count) a[idx] = run;
            run += v[i];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                     const int32_t* __restrict__ tile_pre) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int32_t add = tile_pre[blockIdx.x];
    if (add == 0) return;
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        int64_t idx = base + i;
        if (idx < n) out[idx] += add;
    }
}

size_t scan_ws_elems(int64_t n) { return (size_t)std::max<int64_t>(1, ceil_div(n, kScanTile)); }

spx_status scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev,
                              int32_t* ws, hipStream_t s) {
    if (n <= 0) {
        if (total_dev) SPX_TRY(fill_u32((uint32_t*)total_dev, 0, 1, s));
        return SPX_OK;
    }
    const int64_t tiles = ceil_div(n, kScanTile);
    k_scan_tiles<<<(unsigned)tiles, kBlock, 0, s>>>(in, out, n, ws, total_dev);
    SPX_HIP(hipGetLastError());
    if (tiles > 1) {
        k_scan_single<<<1, kBlock, 0, s>>>(ws, tiles, total_dev);
        SPX_HIP(hipGetLastError());
        k_scan_add<<<(unsigned)tiles, kBlock, 0, s>>>(out, n, ws);
        SPX_HIP(hipGetLastError());
    }
    return SPX_OK;
}

// ------------------------------------------------------------------ radix sort
// Stable LSD radix sort, 8-bit digits, tiles of 4096 pairs.
//  1. per-tile digit histograms, digit-major: H[d * tiles + t]
//  2. exclusive scan of H: global start of digit d for tile t
//  3. per tile: stable rank inside the tile (wave ballots per digit bit, waves
//     and rounds in index order), reorder in LDS by digit, write each digit
//     run to its global range (contiguous, so stores coalesce).
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kRadixIpt = 16;
constexpr int kRadixTile = kBlock * kRadixIpt;

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                       int64_t n, int shift, uint32_t dmask,
                                                       int32_t* __restrict__ H, int64_t tiles) {
    __shared__ int32_t s_h[kRadix];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int i = 0; i < kRadixIpt; ++i) {
        int64_t idx = base + i * kBlock + threadIdx.x;
        if (idx < n) atomicAdd(&s_h[(keys[idx] >> shift) & dmask], 1);
    }
    __syncthreads();
    H[(int64_t)threadIdx.x * tiles + blockIdx.x] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, uint32_t* __restrict__ okeys,
    uint32_t* __restrict__ ovals, int64_t n, int shift, int nbits, const int32_t* __restrict__ Hs,
    int64_t tiles) {
    __shared__ uint32_t s_k[kRadixTile];
    __shared__ uint32_t s_v[kRadixTile];
    __shared__ int32_t s_cnt[kRadix];
    __shared__ int32_t s_loc[kRadix];
    __shared__ int32_t s_base[kRadix];
    __shared__ int32_t s_run[kRadix];
    __shared__ int32_t s_w[kWavesPerBlock][kRadix];
    __shared__ int32_t s_tmp[kWavesPerBlock];

    const uint32_t dmask = (1u << nbits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    const int t = threadIdx.x;
    const int w = wave_id();
    const int l = lane_id();
    const uint64_t lt_mask = (l == 0) ? 0ull : (~0ull >> (kWave - l));

    uint32_t k[kRadixIpt], v[kRadixIpt];
    s_cnt[t] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRadixIpt; ++i) {
        int64_t idx = base + i * kBlock + t;
        if (idx < n) {
            k[i] = keys[idx];
            v[i] = vals[idx];
            atomicAdd(&s_cnt[(k[i] >> shift) & dmask], 1);
        }
    }
    __syncthreads();
    {
        int32_t c = s_cnt[t];
        int32_t tot;
        int32_t incl = block_incl_scan(c, s_tmp, &tot);
        s_loc[t] = incl - c;
        s_base[t] = Hs[(int64_t)t * tiles + blockIdx.x];
        s_run[t] = 0;
    }
    __syncthreads();

    for (int i = 0; i < kRadixIpt; ++i) {
        const int64_t idx = base + i * kBlock + t;
        const bool valid = idx < n;
        const uint32_t d = valid ? ((k[i] >> shift) & dmask) : 0u;
#pragma unroll
        for (int ww = 0; ww < kWavesPerBlock; ++ww) s_w[ww][t] = 0;
        __syncthreads();
        uint64_t match = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const int rank = __popcll(match & lt_mask);
        if (valid && rank == 0) s_w[w][d] = __popcll(match);
        __syncthreads();
        if (valid) {
            int pre = s_loc[d] + s_run[d] + rank;
            for (int ww = 0; ww < w; ++ww) pre += s_w[ww][d];
            s_k[pre] = k[i];
            s_v[pre] = v[i];
        }
        __syncthreads();
        {
            int32_t add = 0;
#pragma unroll
            for (int ww = 0; ww < kWavesPerBlock; ++ww) add += s_w[ww][t];
            s_run[t] += add;
        }
        __syncthreads();
    }
    const int cnt = (int)std::min<int64_t>(kRadixTile, n - base);
    for (int q = t; q < cnt; q += kBlock) {
        const uint32_t key = s_k[q];
        const uint32_t d = (key >> shift) & dmask;
        const int64_t g = (int64_t)s_base[d] + (q - s_loc[d]);
        okeys[g] = key;
        ovals[g] = s_v[q];
    }
}

size_t radix_ws_elems(int64_t n) {
    const int64_t tiles = std::max<int64_t>(1, ceil_div(n, kRadixTile));
    return (size_t)(tiles * kRadix) + scan_ws_elems(tiles * kRadix);
}

spx_status radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                            uint32_t* vals_alt, int64_t n, int bits, int32_t* ws, hipStream_t s,
                            bool* result_in_alt) {
    *result_in_alt = false;
    if (n <= 1 || bits <= 0) return SPX_OK;
    const int64_t tiles = ceil_div(n, kRadixTile);
    int32_t* H = ws;
    int32_t* scan_ws = ws + tiles * kRadix;
    uint32_t *ik = keys, *iv = vals, *ok = keys_alt, *ov = vals_alt;
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        const int nb = std::min(kRadixBits, bits - shift);
        const uint32_t dmask = (1u << nb) - 1u;
        k_radix_hist<<<(unsigned)tiles, kBlock, 0, s>>>(ik, n, shift, dmask, H, tiles);
        SPX_HIP(hipGetLastError());
        SPX_TRY(scan_exclusive_i32(H, H, tiles * kRadix, nullptr, scan_ws, s));
        k_radix_scatter<<<(unsigned)tiles, kBlock, 0, s>>>(ik, iv, ok, ov, n, shift, nb, H, tiles);
        SPX_HIP(hipGetLastError());
        std::swap(ik, ok);
        std::swap(iv, ov);
        *result_in_alt = !*result_in_alt;
    }
    return SPX_OK;
}

// ------------------------------------------------------------------ CSR helpers
// One wave per row writes the row id over the row's positions.
__global__ __launch_bounds__(kBlock) void k_expand_rows(const int32_t* __restrict__ row_ptr,
                                                        int32_t m, int32_t* __restrict__ rows) {
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    if (wave >= m) return;
    const int r = (int)wave;
    const int b = row_ptr[r], e = row_ptr[r + 1];
    for (int k = b + lane_id(); k < e; k += kWave) rows[k] = r;
}

spx_status expand_rows(const int32_t* row_ptr, int32_t m, int32_t* rows_out, hipStream_t s) {
    if (m <= 0) return SPX_OK;
    const int64_t blocks = ceil_div((int64_t)m * kWave, kBlock);
    k_expand_rows<<<(unsigned)blocks, kBlock, 0, s>>>(row_ptr, m, rows_out);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_perm(const T* __restrict__ in,
                                                        const int32_t* __restrict__ perm,
                                                        T* __restrict__ out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < n; i += stride) out[i] = in[perm[i]];
}

spx_status gather_perm(const void* in, const int32_t* perm, void* out, int64_t n, int esize,
                       hipStream_t s) {
    if (n <= 0) return SPX_OK;
    const int grid = (int)std::min<int64_t>(ceil_div(n, kBlock), 8192);
    if (esize == 4)
        k_gather_perm<uint32_t><<<grid, kBlock, 0, s>>>((const uint32_t*)in, perm, (uint32_t*)out, n);
    else if (esize == 8)
        k_gather_perm<uint64_t><<<grid, kBlock, 0, s>>>((const uint64_t*)in, perm, (uint64_t*)out, n);
    else
        return fail(SPX_ERR_DTYPE, "gather_perm: element size must be 4 or 8");
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// ------------------------------------------------------------------ conversions
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_bits(int32_t nnz_x, const int32_t* __restrict__ idx,
                                                         const T* __restrict__ val,
                                                         const int32_t* __restrict__ map,
                                                         uint32_t* __restrict__ bits,
                                                         T* __restrict__ xd) {
    int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= nnz_x) return;
    const int j = map ? map[idx[e]] : idx[e];
    atomicOr(&bits[j >> 5], 1u << (j & 31));
    if (xd) xd[j] = val[e];
}

spx_status sparse_to_bitvector(int32_t n, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                               int dtype, const int32_t* map, uint32_t* bits, void* xd, hipStream_t s,
                               bool clean) {
    if (!clean) SPX_TRY(fill_u32(bits, 0u, (size_t)ceil_div(n, 32), s));
    if (nnz_x <= 0) return SPX_OK;
    const unsigned g = (unsigned)ceil_div(nnz_x, kBlock);
    switch (value_size(dtype)) {
        case 0:
            k_scatter_bits<uint32_t><<<g, kBlock, 0, s>>>(nnz_x, x_idx, nullptr, map, bits, nullptr);
            break;
        case 4:
            k_scatter_bits<uint32_t><<<g, kBlock, 0, s>>>(nnz_x, x_idx, (const uint32_t*)x_val, map, bits,
                                                          (uint32_t*)xd);
            break;
        case 8:
            k_scatter_bits<uint64_t><<<g, kBlock, 0, s>>>(nnz_x, x_idx, (const uint64_t*)x_val, map, bits,
                                                          (uint64_t*)xd);
            break;
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_dense(int32_t nnz_x, const int32_t* __restrict__ idx,
                                                          const T* __restrict__ val, T one,
                                                          const int32_t* __restrict__ map,
                                                          T* __restrict__ xd) {
    int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= nnz_x) return;
    xd[map ? map[idx[e]] : idx[e]] = val ? val[e] : one;
}

spx_status sparse_to_dense(int32_t n, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                           int dtype, const int32_t* map, void* xd, hipStream_t s, bool clean) {
    // absent entries hold the semiring's zero (+inf for min-plus)
    if (clean)
        ;
    else if (zero_word(dtype))
        SPX_TRY(fill_u32((uint32_t*)xd, zero_word(dtype), (size_t)n, s));
    else
        SPX_TRY(fill_bytes(xd, 0, (size_t)n * std::max(1, value_size(dtype)), s));
    if (nnz_x <= 0) return SPX_OK;
    const unsigned g = (unsigned)ceil_div(nnz_x, kBlock);
    switch (value_size(dtype)) {
        case 0:
            k_scatter_dense<uint8_t><<<g, kBlock, 0, s>>>(nnz_x, x_idx, nullptr, (uint8_t)1, map, (uint8_t*)xd);
            break;
        case 4:
            k_scatter_dense<uint32_t><<<g, kBlock, 0, s>>>(nnz_x, x_idx, (const uint32_t*)x_val, 0u, map,
                                                           (uint32_t*)xd);
            break;
        case 8:
            k_scatter_dense<uint64_t><<<g, kBlock, 0, s>>>(nnz_x, x_idx, (const uint64_t*)x_val, 0ull, map,
                                                           (uint64_t*)xd);
            break;
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// xg[r] = x[order[r]] (a dense x in the renumbered column order) and, if
// bits is given, the bitvector of xg's nonzeros, one wave ballot per 64
// entries.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_permute_dense(int32_t n, const typename SR<DT>::X* __restrict__ x,
                                                          const int32_t* __restrict__ order,
                                                          typename SR<DT>::X* __restrict__ xg,
                                                          uint32_t* __restrict__ bits) {
    using T = typename SR<DT>::X;
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    T v = 0;
    if (r < n) {
        v = x[order[r]];
        xg[r] = v;
    }
    if (!bits) return;
    const uint64_t b = __ballot(r < n && SR<DT>::present(v));
    const int64_t base = r - lane_id();
    if (lane_id() == 0 && base < n) bits[base >> 5] = (uint32_t)b;
    if (lane_id() == 32 && base + 32 < n) bits[(base >> 5) + 1] = (uint32_t)(b >> 32);
}

spx_status permute_dense(int32_t n, const void* x, int dtype, const int32_t* order, void* xg, uint32_t* bits,
                         hipStream_t s) {
    if (n <= 0) return SPX_OK;
    const unsigned g = (unsigned)ceil_div(n, kBlock);
    switch (dtype) {
        case SPX_F32:
            k_permute_dense<SPX_F32><<<g, kBlock, 0, s>>>(n, (const float*)x, order, (float*)xg, bits);
            break;
        case SPX_F64:
            k_permute_dense<SPX_F64><<<g, kBlock, 0, s>>>(n, (const double*)x, order, (double*)xg, bits);
            break;
        case SPX_I32:
            k_permute_dense<SPX_I32><<<g, kBlock, 0, s>>>(n, (const int32_t*)x, order, (int32_t*)xg, bits);
            break;
        case SPX_BOOL:
            k_permute_dense<SPX_BOOL><<<g, kBlock, 0, s>>>(n, (const uint8_t*)x, order, (uint8_t*)xg, bits);
            break;
        case SPX_F32_MINPLUS:
            k_permute_dense<SPX_F32_MINPLUS><<<g, kBlock, 0, s>>>(n, (const float*)x, order, (float*)xg, bits);
            break;
        default:
            return fail(SPX_ERR_DTYPE, "permute_dense: dtype");
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// dense -> sparse: flag nonzeros (x != 0: -0.0 is zero, NaN is nonzero), scan,
// write (index, value) in index order.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_flag_nonzero(int32_t n, const typename SR<DT>::X* __restrict__ x,
                                                         int32_t* __restrict__ flags) {
    int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < n) flags[j] = SR<DT>::present(x[j]) ? 1 : 0;
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_compact(int32_t n, const typename SR<DT>::X* __restrict__ x,
                                                    const int32_t* __restrict__ pos,
                                                    int32_t* __restrict__ idx,
                                                    typename SR<DT>::X* __restrict__ val) {
    int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const typename SR<DT>::X v = x[j];
    if (SR<DT>::present(v)) {
        const int p = pos[j];
        idx[p] = j;
        if (val) val[p] = v;
    }
}

size_t compact_ws_elems(int32_t n) { return (size_t)n + scan_ws_elems(n) + 64; }

spx_status dense_to_sparse(int32_t n, const void* x, int dtype, int32_t* idx, void* val,
                           int32_t* nnz_dev, int32_t* ws, hipStream_t s) {
    if (n <= 0) return fill_u32((uint32_t*)nnz_dev, 0, 1, s);
    int32_t* flags = ws;
    int32_t* sws = ws + align_up(n, 64);
    const unsigned g = (unsigned)ceil_div(n, kBlock);
    switch (dtype) {
#define SPX_CASE(DT)                                                                              \
    case DT:                                                                                      \
        k_flag_nonzero<DT><<<g, kBlock, 0, s>>>(n, (const SR<DT>::X*)x, flags);                   \
        SPX_HIP(hipGetLastError());                                                               \
        SPX_TRY(scan_exclusive_i32(flags, flags, n, nnz_dev, sws, s));                            \
        k_compact<DT><<<g, kBlock, 0, s>>>(n, (const SR<DT>::X*)x, flags, idx, (SR<DT>::X*)val);  \
        break;
        SPX_CASE(SPX_F32)
        SPX_CASE(SPX_F64)
        SPX_CASE(SPX_I32)
        SPX_CASE(SPX_BOOL)
        SPX_CASE(SPX_F32_MINPLUS)
#undef SPX_CASE
        default:
            return fail(SPX_ERR_DTYPE, "dense_to_sparse: dtype");
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// ------------------------------------------------------------------ features
// Row-length reductions: max, min, sum, sum of squares (exact integers).
__global__ __launch_bounds__(kBlock) void k_row_stats(const int32_t* __restrict__ row_ptr, int32_t m,
                                                      unsigned long long* __restrict__ out) {
    // out[0] = max, out[1] = min, out[2] = sum, out[3] = sum of squares
    __shared__ unsigned long long s_red[4][kWavesPerBlock];
    unsigned long long mx = 0, mn = ~0ull, sm = 0, sq = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * kBlock) {
        unsigned long long L = (unsigned long long)(row_ptr[i + 1] - row_ptr[i]);
        mx = L > mx ? L : mx;
        mn = L < mn ? L : mn;
        sm += L;
        sq += L * L;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        unsigned long long a = __shfl_xor(mx, off, kWave), b = __shfl_xor(mn, off, kWave);
        mx = a > mx ? a : mx;
        mn = b < mn ? b : mn;
        sm += __shfl_xor(sm, off, kWave);
        sq += __shfl_xor(sq, off, kWave);
    }
    if (lane_id() == 0) {
        s_red[0][wave_id()] = mx;
        s_red[1][wave_id()] = mn;
        s_red[2][wave_id()] = sm;
        s_red[3][wave_id()] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kWavesPerBlock; ++i) {
            mx = s_red[0][i] > mx ? s_red[0][i] : mx;
            mn = s_red[1][i] < mn ? s_red[1][i] : mn;
            sm += s_red[2][i];
            sq += s_red[3][i];
        }
        atomicMax(&out[0], mx);
        atomicMin(&out[1], mn);
        atomicAdd(&out[2], sm);
        atomicAdd(&out[3], sq);
    }
}

// Histogram of row lengths; lengths below kLdsBins are counted in LDS first
// (most rows are short), longer ones go straight to global atomics.
constexpr int kLdsBins = 4096;
__global__ __launch_bounds__(kBlock) void k_len_hist(const int32_t* __restrict__ row_ptr, int32_t m, int32_t nbins,
                                                     int32_t* __restrict__ hist) {
    __shared__ int32_t s_h[kLdsBins];
    const int lb = nbins < kLdsBins ? nbins : kLdsBins;
    for (int i = threadIdx.x; i < lb; i += kBlock) s_h[i] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) {
        const int L = row_ptr[i + 1] - row_ptr[i];
        if (L < lb)
            atomicAdd(&s_h[L], 1);
        else
            atomicAdd(&hist[L], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < lb; i += kBlock)
        if (s_h[i]) atomicAdd(&hist[i], s_h[i]);
}

spx_status matrix_features_device(const int32_t* row_ptr, int32_t m, int32_t n, MatrixStats* out,
                                  hipStream_t s) {
    double* f = out->f;
    for (int i = 0; i < 9; ++i) f[i] = 0.0;
    f[0] = m;
    f[1] = n;
    if (m <= 0) return SPX_OK;
    unsigned long long* d_stats = nullptr;
    SPX_HIP(hipMallocAsync((void**)&d_stats, 4 * sizeof(unsigned long long), s));
    unsigned long long init[4] = {0ull, ~0ull, 0ull, 0ull};
    SPX_HIP(hipMemcpyAsync(d_stats, init, sizeof(init), hipMemcpyHostToDevice, s));
    const int grid = (int)std::min<int64_t>(ceil_div(m, kBlock), 1024);
    k_row_stats<<<grid, kBlock, 0, s>>>(row_ptr, m, d_stats);
    SPX_HIP(hipGetLastError());
    unsigned long long h[4];
    SPX_HIP(hipMemcpyAsync(h, d_stats, sizeof(h), hipMemcpyDeviceToHost, s));
    SPX_HIP(hipStreamSynchronize(s));
    SPX_HIP(hipFreeAsync(d_stats, s));
    const int64_t mx = (int64_t)h[0], mn = (int64_t)h[1], sum = (int64_t)h[2];
    const unsigned long long sq = h[3];
    // Gini from the histogram of row lengths: rows of length L occupy ranks
    // P_L + 1 .. P_L + c_L in ascending order, contributing
    // L * c_L * (2 P_L + c_L - m) to sum_i (2i - m - 1) r_(i).
    int32_t* d_hist = nullptr;
    SPX_HIP(hipMallocAsync((void**)&d_hist, (size_t)(mx + 1) * sizeof(int32_t), s));
    SPX_TRY(fill_u32((uint32_t*)d_hist, 0u, (size_t)(mx + 1), s));
    k_len_hist<<<grid, kBlock, 0, s>>>(row_ptr, m, (int32_t)(mx + 1), d_hist);
    SPX_HIP(hipGetLastError());
    std::vector<int32_t> hist((size_t)mx + 1);
    SPX_HIP(hipMemcpyAsync(hist.data(), d_hist, hist.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPX_HIP(hipStreamSynchronize(s));
    SPX_HIP(hipFreeAsync(d_hist, s));
    __int128 num = 0;
    int64_t P = 0;
    for (int64_t L = 0; L <= mx; ++L) {
        const int64_t c = hist[(size_t)L];
        if (c) num += (__int128)L * c * (2 * P + c - m);
        P += c;
    }
    f[2] = (double)sum;
    f[3] = (double)mx;
    f[4] = (double)mn;
    f[5] = (double)sum / (double)m;
    f[6] = n > 0 ? (double)(mx - mn) / (double)n : 0.0;
    // population variance = (m * sum L^2 - (sum L)^2) / m^2, exact in 128 bits
    const __int128 vnum = (__int128)m * (__int128)sq - (__int128)sum * (__int128)sum;
    f[7] = std::sqrt((double)vnum / ((double)m * (double)m));
    f[8] = sum > 0 ? (double)num / ((double)m * (double)sum) : 0.0;
    return SPX_OK;
}

// nnz_s = sum over supp(x) of column lengths; for a dense x also nnz_x.
__global__ __launch_bounds__(kBlock) void k_vec_feat_sparse(const int32_t* __restrict__ col_ptr,
                                                            int32_t nnz_x, const int32_t* __restrict__ idx,
                                                            unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s_red[kWavesPerBlock];
    unsigned long long acc = 0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz_x;
         e += (int64_t)gridDim.x * kBlock) {
        const int j = idx[e];
        acc += (unsigned long long)(col_ptr[j + 1] - col_ptr[j]);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane_id() == 0) s_red[wave_id()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kWavesPerBlock; ++i) acc += s_red[i];
        atomicAdd(&out[0], acc);
    }
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_vec_feat_dense(const int32_t* __restrict__ col_ptr, int32_t n,
                                                           const typename SR<DT>::X* __restrict__ x,
                                                           unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s_red[2][kWavesPerBlock];
    unsigned long long a = 0, c = 0;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * kBlock) {
        if (SR<DT>::present(x[j])) {
            a += (unsigned long long)(col_ptr[j + 1] - col_ptr[j]);
            c += 1;
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, kWave);
        c += __shfl_xor(c, off, kWave);
    }
    if (lane_id() == 0) {
        s_red[0][wave_id()] = a;
        s_red[1][wave_id()] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kWavesPerBlock; ++i) {
            a += s_red[0][i];
            c += s_red[1][i];
        }
        atomicAdd(&out[0], a);
        atomicAdd(&out[1], c);
    }
}

// The counts of run()'s lazy features in one launch: nnz_s (the column
// lengths summed over supp(x)) and, for a dense x, the number of its present
// entries. Every workgroup adds its partial sums into two device counters;
// the last to arrive (atomicInc wraps the ticket back to 0) takes the totals
// out of the counters (clearing them for the next call) and stores them to
// host-visible memory, so the host needs no copy command, only the stream
// synchronization. Counters and ticket are zero between calls.
template <int DT, bool DENSE>
__global__ __launch_bounds__(kBlock) void k_vec_counts(const int32_t* __restrict__ col_ptr, int32_t count,
                                                       const int32_t* __restrict__ idx,
                                                       const typename SR<DT>::X* __restrict__ x,
                                                       unsigned long long* __restrict__ acc2,
                                                       uint32_t* __restrict__ ticket, long long* __restrict__ host2) {
    __shared__ unsigned long long s_red[2][kWavesPerBlock];
    unsigned long long a = 0, c = 0;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < count; e += (int64_t)gridDim.x * kBlock) {
        if constexpr (DENSE) {
            if (SR<DT>::present(x[e])) {
                a += (unsigned long long)(col_ptr[e + 1] - col_ptr[e]);
                c += 1;
            }
        } else {
            const int j = idx[e];
            a += (unsigned long long)(col_ptr[j + 1] - col_ptr[j]);
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, kWave);
        c += __shfl_xor(c, off, kWave);
    }
    if (lane_id() == 0) {
        s_red[0][wave_id()] = a;
        s_red[1][wave_id()] = c;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < kWavesPerBlock; ++i) {
        a += s_red[0][i];
        c += s_red[1][i];
    }
    if (a) atomicAdd(&acc2[0], a);
    if (c) atomicAdd(&acc2[1], c);
    __threadfence();
    if (atomicInc(ticket, gridDim.x - 1) != gridDim.x - 1) return;
    __threadfence();
    const unsigned long long ta = atomicExch(&acc2[0], 0ull);
    const unsigned long long tc = atomicExch(&acc2[1], 0ull);
    __hip_atomic_store(&host2[0], (long long)ta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&host2[1], DENSE ? (long long)tc : (long long)count, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

spx_status vector_counts_to_host(const int32_t* col_ptr, int32_t n, const spx_vec* x, int dtype,
                                 unsigned long long* acc2, uint32_t* ticket, long long* host2, hipStream_t s) {
    const bool dense = x->kind != SPX_VEC_SPARSE;
    const int32_t count = dense ? n : x->nnz_x;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, kBlock * 4), 256));
    if (!dense) {
        k_vec_counts<SPX_F32, false><<<grid, kBlock, 0, s>>>(col_ptr, count, x->idx, nullptr, acc2, ticket, host2);
    } else {
        switch (dtype) {
#define SPX_DT(DT)                                                                                           \
    case DT:                                                                                                 \
        k_vec_counts<DT, true><<<grid, kBlock, 0, s>>>(col_ptr, count, nullptr,                              \
                                                       (const typename SR<DT>::X*)x->val, acc2, ticket, host2); \
        break;
            SPX_DT(SPX_F32) SPX_DT(SPX_F64) SPX_DT(SPX_I32) SPX_DT(SPX_BOOL) SPX_DT(SPX_F32_MINPLUS)
#undef SPX_DT
            default:
                return fail(SPX_ERR_DTYPE, "vector counts: dtype");
        }
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status vector_features_device(const int32_t* col_ptr, int32_t n, const spx_vec* x, int dtype,
                                  int64_t* out2_dev, hipStream_t s) {
    SPX_TRY(fill_u32((uint32_t*)out2_dev, 0u, 4, s));
    unsigned long long* o = (unsigned long long*)out2_dev;
    if (x->kind == SPX_VEC_SPARSE) {
        if (x->nnz_x > 0) {
            const int grid = (int)std::min<int64_t>(ceil_div(x->nnz_x, kBlock), 1024);
            k_vec_feat_sparse<<<grid, kBlock, 0, s>>>(col_ptr, x->nnz_x, x->idx, o);
        }
    } else {
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kBlock), 1024));
        switch (dtype) {
            case SPX_F32:
                k_vec_feat_dense<SPX_F32><<<grid, kBlock, 0, s>>>(col_ptr, n, (const float*)x->val, o);
                break;
            case SPX_F64:
                k_vec_feat_dense<SPX_F64><<<grid, kBlock, 0, s>>>(col_ptr, n, (const double*)x->val, o);
                break;
            case SPX_I32:
                k_vec_feat_dense<SPX_I32><<<grid, kBlock, 0, s>>>(col_ptr, n, (const int32_t*)x->val, o);
                break;
            case SPX_BOOL:
                k_vec_feat_dense<SPX_BOOL><<<grid, kBlock, 0, s>>>(col_ptr, n, (const uint8_t*)x->val, o);
                break;
            case SPX_F32_MINPLUS:
                k_vec_feat_dense<SPX_F32_MINPLUS><<<grid, kBlock, 0, s>>>(col_ptr, n, (const float*)x->val, o);
                break;
            default:
                return fail(SPX_ERR_DTYPE, "vector features: dtype");
        }
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

}  // namespace spx
