// Column-major, vector-driven SpMSpV (Section 4.1): for every entry (j, v)
// of the sparse x, column j of A is scaled by v and written back into y.
// Only effective nonzeros are read. Distributions (Section 4.2.1):
//
//  * direct   - a group of L lanes per x entry walks that column.
//  * balanced - merge-path tiles over (x entries + effective nonzeros): the
//               column lengths of supp(x) are prefix-summed, and every
//               workgroup takes kTile merge items, so a hub column is split
//               across workgroups and empty columns cost one item each.
//
// Write-backs (Section 4.2.2):
//  * atomic     - y is zero-filled, every product is added with a hardware
//                 atomic (global_atomic_add_f32/f64, integer add for I32,
//                 a plain byte store of 1 for BOOL since OR is idempotent).
//  * lds-atomic - each workgroup accumulates into its own copy of y in LDS
//                 and flushes the rows it touched with one atomic each
//                 (only when y fits in LDS).
//  * sort       - (row, value) pairs go to global memory at their prefix
//                 position, a stable radix sort orders them by row, and a
//                 reduce-by-key writes each row once; only runs that cross a
//                 tile boundary use an atomic.
//  * bucket     - see spmspv_bucket.hip.
#include <algorithm>

#include "common.hpp"
#include "csc_tile.hpp"
#include "csr_tile.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kLdsBytes = 65536;  // LDS budget of the privatized y copy

template <int DT>
struct EmitLds {
    typename SR<DT>::Acc* sy;
    __device__ void operator()(int r, typename SR<DT>::Acc v, int64_t) const {
        SR<DT>::lds_atomic_add(&sy[r], v);
    }
};

// pair at its global prefix position p; values stored as raw bits (4 bytes)
// or, for 8-byte values, in a separate array indexed by p
template <int DT>
struct EmitPairs {
    uint32_t* keys;
    uint32_t* vbits;                 // 4-byte value types (and BOOL: unused)
    typename SR<DT>::Acc* vwide;     // 8-byte value types
    __device__ void operator()(int r, typename SR<DT>::Acc v, int64_t p) const {
        keys[p] = (uint32_t)r;
        if constexpr (sizeof(typename SR<DT>::Acc) == 8) {
            vbits[p] = (uint32_t)p;
            vwide[p] = v;
        } else {
            uint32_t b;
            __builtin_memcpy(&b, &v, 4);
            vbits[p] = b;
        }
    }
};

template <int DT, int L>
__global__ __launch_bounds__(kBlock) void k_csc_direct_atomic(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                              const typename SR<DT>::X* __restrict__ x_val,
                                                              const int32_t* __restrict__ col_ptr,
                                                              const int32_t* __restrict__ row_idx,
                                                              const typename SR<DT>::V* __restrict__ vals,
                                                              typename SR<DT>::Y* __restrict__ y) {
    const int64_t e = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / L;
    if (e >= nnz_x) return;
    csc_direct_entry<DT, L>((int)e, threadIdx.x % L, x_idx, x_val, col_ptr, row_idx, vals, Excl{nullptr, nullptr},
                            EmitAtomic<DT>{y});
}

template <int DT, int L>
__global__ __launch_bounds__(kBlock) void k_csc_direct_pairs(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                             const typename SR<DT>::X* __restrict__ x_val,
                                                             const int32_t* __restrict__ col_ptr,
                                                             const int32_t* __restrict__ row_idx,
                                                             const typename SR<DT>::V* __restrict__ vals,
                                                             const Excl excl,
                                                             EmitPairs<DT> emit) {
    const int64_t e = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / L;
    if (e >= nnz_x) return;
    csc_direct_entry<DT, L>((int)e, threadIdx.x % L, x_idx, x_val, col_ptr, row_idx, vals, excl, emit);
}

// privatized: grid-stride over entries, y copy in LDS, flush touched rows
template <int DT, int L>
__global__ __launch_bounds__(kBlock) void k_csc_direct_lds(int32_t m, int32_t nnz_x,
                                                           const int32_t* __restrict__ x_idx,
                                                           const typename SR<DT>::X* __restrict__ x_val,
                                                           const int32_t* __restrict__ col_ptr,
                                                           const int32_t* __restrict__ row_idx,
                                                           const typename SR<DT>::V* __restrict__ vals,
                                                           typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    extern __shared__ __align__(16) char s_raw[];  // typed as the accumulator: 8-byte LDS ops need the alignment
    auto* sy = (typename S::Acc*)s_raw;
    for (int r = threadIdx.x; r < m; r += kBlock) sy[r] = S::zero();
    __syncthreads();
    const int groups = kBlock / L;
    for (int64_t e = (int64_t)blockIdx.x * groups + threadIdx.x / L; e < nnz_x;
         e += (int64_t)gridDim.x * groups)
        csc_direct_entry<DT, L>((int)e, threadIdx.x % L, x_idx, x_val, col_ptr, row_idx, vals,
                                Excl{nullptr, nullptr}, EmitLds<DT>{sy});
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += kBlock) {
        const typename S::Acc v = sy[r];
        if (S::nonzero(v)) S::atomic_add(&y[r], v);
    }
}

// --------------------------------------------------------------- prefix of lengths
__global__ __launch_bounds__(kBlock) void k_x_lengths(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                      const int32_t* __restrict__ col_ptr,
                                                      int32_t* __restrict__ len) {
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e > nnz_x) return;
    if (e == nnz_x) {
        len[e] = 0;
        return;
    }
    const int j = x_idx[e];
    len[e] = col_ptr[j + 1] - col_ptr[j];
}

// Prologue of the column-major kernels for a short x, in one launch:
// workgroup 0 writes excl (exclusive prefix of the selected column lengths,
// nnz_x + 1 entries, each thread a run of kProIpt consecutive entries);
// the other workgroups zero y (ywords 32-bit words, then ytail bytes).
constexpr int kProIpt = 32;
constexpr int kProMax = kBlock * kProIpt;  // nnz_x + 1 <= kProMax

__global__ __launch_bounds__(kBlock) void k_csc_prologue(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                         const int32_t* __restrict__ col_ptr,
                                                         int32_t* __restrict__ excl, uint32_t* __restrict__ y,
                                                         int64_t ywords, int ytail, uint32_t yfill) {
    if (blockIdx.x == 0) {
        __shared__ int32_t tmp[kWavesPerBlock];
        const int e0 = threadIdx.x * kProIpt;
        int j[kProIpt], len[kProIpt];
#pragma unroll
        for (int u = 0; u < kProIpt; ++u) j[u] = e0 + u < nnz_x ? x_idx[e0 + u] : -1;
#pragma unroll
        for (int u = 0; u < kProIpt; ++u) len[u] = j[u] >= 0 ? col_ptr[j[u] + 1] - col_ptr[j[u]] : 0;
        int sum = 0;
#pragma unroll
        for (int u = 0; u < kProIpt; ++u) sum += len[u];
        int total;
        int run = block_incl_scan<int32_t>(sum, tmp, &total) - sum;
#pragma unroll
        for (int u = 0; u < kProIpt; ++u) {
            if (e0 + u <= nnz_x) excl[e0 + u] = run;
            run += len[u];
        }
        return;
    }
    const int64_t stride = (int64_t)(gridDim.x - 1) * kBlock;
    for (int64_t i = (int64_t)(blockIdx.x - 1) * kBlock + threadIdx.x; i < ywords; i += stride) y[i] = yfill;
    if (blockIdx.x == 1 && (int)threadIdx.x < ytail) ((uint8_t*)(y + ywords))[threadIdx.x] = 0;
}

// The prefix of the selected column lengths over many workgroups, for x up
// to kLsMaxTiles runs of 256 entries, with the zero fill of y: workgroups
// [0, F) zero y; each of the T others writes the exclusive prefix of the
// lengths of its 256 entries (one per thread) to local and the run's total
// to sums. Readers add off[e >> 8], the exclusive prefix of the totals, to
// local[e] (Excl). off comes from a second one-workgroup launch, or, for
// up to kLsFenceTiles runs and a counter, from the last of the T workgroups
// to arrive (atomicInc wraps the counter back to 0, so it is zero again for
// the next call). No workgroup waits for another: the thread that writes a
// run total fences it before its workgroup arrives, and the last one fences
// before it reads the totals. Each fence writes back the XCD's L2, so the
// one-launch form is kept for few runs.
constexpr int kLsMaxTiles = 4096;  // nnz_x + 1 <= 2^20
constexpr int kLsFenceTiles = 32;
constexpr int kLsPer = kLsMaxTiles / kBlock;

// off[0..T) = exclusive prefix of sums[0..T), by one 256-thread workgroup
__device__ __forceinline__ void scan_run_totals(const int32_t* __restrict__ sums, int T, int32_t* __restrict__ off,
                                                int32_t* tmp) {
    const int i0 = threadIdx.x * kLsPer;
    int v[kLsPer];
    int run = 0;
#pragma unroll
    for (int u = 0; u < kLsPer; ++u) {
        v[u] = i0 + u < T ? sums[i0 + u] : 0;
        run += v[u];
    }
    int all;
    run = block_incl_scan<int32_t>(run, tmp, &all) - run;
#pragma unroll
    for (int u = 0; u < kLsPer; ++u) {
        if (i0 + u < T) off[i0 + u] = run;
        run += v[u];
    }
}

__global__ __launch_bounds__(kBlock) void k_csc_lengths_scan(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                             const int32_t* __restrict__ col_ptr,
                                                             int32_t* __restrict__ local, int32_t* __restrict__ sums,
                                                             int32_t* __restrict__ off, uint32_t* __restrict__ counter,
                                                             uint32_t* __restrict__ y, int64_t ywords, int ytail,
                                                             uint32_t yfill, int F) {
    if ((int)blockIdx.x < F) {
        const int64_t stride = (int64_t)F * kBlock;
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ywords; i += stride) y[i] = yfill;
        if (blockIdx.x == 0 && (int)threadIdx.x < ytail) ((uint8_t*)(y + ywords))[threadIdx.x] = 0;
        return;
    }
    __shared__ int32_t tmp[kWavesPerBlock];
    __shared__ int last;
    const int t = blockIdx.x - F;
    const int T = gridDim.x - F;
    const int e = t * kBlock + threadIdx.x;
    int len = 0;
    if (e < nnz_x) {
        const int j = x_idx[e];
        len = col_ptr[j + 1] - col_ptr[j];
    }
    int total;
    const int incl = block_incl_scan<int32_t>(len, tmp, &total);
    if (e <= nnz_x) local[e] = incl - len;
    if (!counter) {
        if (threadIdx.x == 0) sums[t] = total;
        return;
    }
    // only the run totals cross workgroups inside this kernel (local is read
    // by the next launch), so thread 0, which writes its total, fences it
    if (threadIdx.x == 0) {
        sums[t] = total;
        __threadfence();
        const bool l = atomicInc(counter, (unsigned)(T - 1)) == (unsigned)(T - 1);
        if (l) __threadfence();
        last = l;
    }
    __syncthreads();
    if (!last) return;
    scan_run_totals(sums, T, off, tmp);
}

__global__ __launch_bounds__(kBlock) void k_scan_run_totals(const int32_t* __restrict__ sums, int T,
                                                            int32_t* __restrict__ off) {
    __shared__ int32_t tmp[kWavesPerBlock];
    scan_run_totals(sums, T, off, tmp);
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_csc_merge_atomic(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                             const typename SR<DT>::X* __restrict__ x_val,
                                                             const int32_t* __restrict__ col_ptr,
                                                             const int32_t* __restrict__ row_idx,
                                                             const typename SR<DT>::V* __restrict__ vals,
                                                             const Excl excl,
                                                             typename SR<DT>::Y* __restrict__ y) {
    __shared__ CscTileLds<DT> L;
    const int64_t nnz_s = excl[nnz_x];
    const int64_t tiles = ceil_div((int64_t)nnz_x + nnz_s, kCscTile);
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x)
        csc_merge_tile<DT>(t, nnz_x, nnz_s, x_idx, x_val, col_ptr, row_idx, vals, excl, EmitAtomic<DT>{y}, L);
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_csc_merge_pairs(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                            const typename SR<DT>::X* __restrict__ x_val,
                                                            const int32_t* __restrict__ col_ptr,
                                                            const int32_t* __restrict__ row_idx,
                                                            const typename SR<DT>::V* __restrict__ vals,
                                                            const Excl excl,
                                                            EmitPairs<DT> emit) {
    __shared__ CscTileLds<DT> L;
    const int64_t nnz_s = excl[nnz_x];
    const int64_t tiles = ceil_div((int64_t)nnz_x + nnz_s, kCscTile);
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x)
        csc_merge_tile<DT>(t, nnz_x, nnz_s, x_idx, x_val, col_ptr, row_idx, vals, excl, emit, L);
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_csc_merge_lds(int32_t m, int32_t nnz_x,
                                                          const int32_t* __restrict__ x_idx,
                                                          const typename SR<DT>::X* __restrict__ x_val,
                                                          const int32_t* __restrict__ col_ptr,
                                                          const int32_t* __restrict__ row_idx,
                                                          const typename SR<DT>::V* __restrict__ vals,
                                                          const Excl excl,
                                                          typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    __shared__ CscTileLds<DT> L;
    extern __shared__ __align__(16) char s_raw[];  // typed as the accumulator: 8-byte LDS ops need the alignment
    auto* sy = (typename S::Acc*)s_raw;
    for (int r = threadIdx.x; r < m; r += kBlock) sy[r] = S::zero();
    __syncthreads();
    const int64_t nnz_s = excl[nnz_x];
    const int64_t tiles = ceil_div((int64_t)nnz_x + nnz_s, kCscTile);
    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x)
        csc_merge_tile<DT>(t, nnz_x, nnz_s, x_idx, x_val, col_ptr, row_idx, vals, excl, EmitLds<DT>{sy}, L);
    __syncthreads();
    for (int r = threadIdx.x; r < m; r += kBlock) {
        const typename S::Acc v = sy[r];
        if (S::nonzero(v)) S::atomic_add(&y[r], v);
    }
}

// --------------------------------------------------------------- reduce by key
// Sorted (row, value) pairs -> y. Tiles of kCscTile pairs; each thread sums
// kCscIpt consecutive pairs by run, a segmented scan over threads joins
// runs that cross threads, and each run is stored once. A run that
// continues into the next tile leaves its partial sum as the tile's carry
// instead; the tile where the run ends stores its own part, and a fix-up
// pass adds the carries in tile order (the same scheme as the balanced
// row-major kernels), so the result does not depend on scheduling.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_reduce_by_key(int64_t n, const uint32_t* __restrict__ keys,
                                                          const uint32_t* __restrict__ vbits,
                                                          const typename SR<DT>::Acc* __restrict__ vwide,
                                                          typename SR<DT>::Y* __restrict__ y,
                                                          int32_t* __restrict__ carry_row,
                                                          typename SR<DT>::Acc* __restrict__ carry_val) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    __shared__ uint32_t s_k[kCscTile + 2];
    __shared__ Acc s_val[kCscTile];
    __shared__ int32_t s_flag[kBlock];
    __shared__ Acc s_cv[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kCscTile;
    const int cnt = (int)std::min<int64_t>(kCscTile, n - base);
    // s_k[0] = key before the tile (or ~0), s_k[1 + i] = tile keys, s_k[1 + cnt] = key after
    for (int i = threadIdx.x; i < cnt; i += kBlock) {
        const uint32_t kk = keys[base + i];
        s_k[1 + i] = kk;
        Acc v;
        if constexpr (sizeof(Acc) == 8) {
            v = vwide[vbits[base + i]];
        } else if constexpr (DT == SPX_BOOL) {
            v = 1u;
        } else {
            const uint32_t b = vbits[base + i];
            __builtin_memcpy(&v, &b, 4);
        }
        s_val[i] = v;
    }
    if (threadIdx.x == 0) {
        s_k[0] = base > 0 ? keys[base - 1] : 0xffffffffu;
        s_k[1 + cnt] = base + cnt < n ? keys[base + cnt] : 0xffffffffu;
    }
    __syncthreads();
    const int i0 = threadIdx.x * kCscIpt;
    const int i1 = std::min(i0 + kCscIpt, cnt);
    // per-thread: running sum since the last run head inside the thread
    Acc acc = S::zero();
    bool has_head = false;
    for (int i = i0; i < i1; ++i) {
        if (i == 0 || s_k[1 + i] != s_k[i]) {
            has_head = true;
            acc = S::zero();
        }
        acc = S::add(acc, s_val[i]);
    }
    s_flag[threadIdx.x] = has_head ? 1 : 0;
    s_cv[threadIdx.x] = acc;
    __syncthreads();
    // inclusive segmented scan: (f1, v1) + (f2, v2) = (f1 | f2, f2 ? v2 : v1 + v2)
    for (int off = 1; off < kBlock; off <<= 1) {
        const int t = threadIdx.x;
        int f = s_flag[t];
        Acc v = s_cv[t];
        int fo = 0;
        Acc vo = S::zero();
        if (t >= off) {
            fo = s_flag[t - off];
            vo = s_cv[t - off];
        }
        __syncthreads();
        if (t >= off) {
            if (!f) v = S::add(vo, v);
            f |= fo;
        }
        s_flag[t] = f;
        s_cv[t] = v;
        __syncthreads();
    }
    Acc run = (threadIdx.x > 0 && i0 < cnt) ? s_cv[threadIdx.x - 1] : S::zero();
    for (int i = i0; i < i1; ++i) {
        if (i == 0 || s_k[1 + i] != s_k[i]) run = S::zero();
        run = S::add(run, s_val[i]);
        const bool tail = (i == cnt - 1) || (s_k[2 + i] != s_k[1 + i]);
        if (tail) {
            const uint32_t r = s_k[1 + i];
            const bool continues = i == cnt - 1 && s_k[1 + cnt] == r;
            if (continues) {
                carry_row[blockIdx.x] = (int32_t)r;
                carry_val[blockIdx.x] = run;
            } else {
                y[r] = S::out(run);
                if (i == cnt - 1) carry_row[blockIdx.x] = -1;
            }
        }
    }
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_rbk_fixup(int64_t tiles, const int32_t* __restrict__ carry_row,
                                                      const typename SR<DT>::Acc* __restrict__ carry_val,
                                                      typename SR<DT>::Y* __restrict__ y) {
    csr_merge_fixup_range<DT>((int64_t)blockIdx.x * kBlock + threadIdx.x, (int64_t)gridDim.x * kBlock, tiles,
                              carry_row, carry_val, y);
}

// --------------------------------------------------------------- launch
static int pick_col_lanes(int32_t n, int32_t nnz) {
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    int L = 1;
    while (L < 64 && L < avg) L <<= 1;
    return L;
}

static int key_bits(int32_t m) {
    int b = 0;
    while (b < 31 && (int64_t(1) << b) < m) ++b;
    return std::max(b, 1);
}

size_t spmspv_csc_ws(int32_t m, int32_t n, int32_t nnz, int32_t nnz_x, int dtype, const spx_plan* plan) {
    (void)n;
    Sizer z;
    const bool need_excl = plan->distribution == SPX_DIST_BALANCED || plan->writeback == SPX_WB_SORT ||
                           plan->writeback == SPX_WB_BUCKET || plan->writeback == SPX_WB_MERGE;
    if (need_excl) {
        z.take<int32_t>((size_t)nnz_x + 1);
        z.take<int32_t>(scan_ws_elems((int64_t)nnz_x + 1));
        z.take<int32_t>(kLsMaxTiles);
        z.take<int32_t>(kLsMaxTiles);
    }
    if (plan->writeback == SPX_WB_BUCKET) {
        const size_t b = csc_bucket_ws(m, nnz, nnz_x, dtype, plan);
        if (b == 0) return 0;
        z.used = align_up(z.used, 256) + b;
    }
    if (plan->writeback == SPX_WB_MERGE) {
        const size_t b = csc_merge_ws(m, nnz, nnz_x, dtype, plan);
        if (b == 0) return 0;
        z.used = align_up(z.used, 256) + b;
    }
    if (plan->writeback == SPX_WB_SORT) {
        const int64_t np = nnz;  // nnz_s <= nnz
        z.take<uint32_t>(np);    // keys
        z.take<uint32_t>(np);    // value bits
        z.take<uint32_t>(np);    // keys alt
        z.take<uint32_t>(np);    // value bits alt
        if (value_size(dtype) == 8) z.take<double>(np);
        z.take<int32_t>(radix_ws_elems(np));
        z.take<int32_t>(4);
        z.take<int32_t>(ceil_div(np, kCscTile));  // carries of the reduce-by-key tiles
        z.take<double>(ceil_div(np, kCscTile));
    }
    return z.used;
}

// y filled with the semiring's zero (0 bytes, or +inf words for min-plus)
static spx_status fill_y_zero(void* y, int dtype, size_t ybytes, hipStream_t s) {
    if (zero_word(dtype)) return fill_u32((uint32_t*)y, zero_word(dtype), ybytes / 4, s);
    return fill_bytes(y, 0, ybytes, s);
}

template <int DT>
static spx_status launch_csc_t(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val_v,
                               void* y_v, const spx_plan* plan, Arena& ws, hipStream_t s) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    const auto* x_val = (const typename S::X*)x_val_v;
    const auto* vals = (const typename S::V*)A.vals;
    auto* y = (typename S::Y*)y_v;
    const int wb = plan->writeback;
    const int dist = plan->distribution;
    const size_t ybytes = (size_t)A.m * sizeof(typename S::Y);
    if (A.m == 0) return SPX_OK;
    if (A.sparse && wb != SPX_WB_BUCKET) return fail(SPX_ERR_ARG, "sparse output needs the bucket write-back");
    if (A.sparse && nnz_x == 0) return SPX_OK;  // nothing reached; the caller zeroed the count
    if (nnz_x > 0 && csc_bucket_walks(A, nnz_x, plan)) return launch_csc_bucket_walk(A, nnz_x, x_idx, x_val_v, y_v, plan, s);
    const int L = plan->lanes > 0 ? plan->lanes : pick_col_lanes(A.n, A.nnz);
    const bool lds_ok = (int64_t)A.m * (int64_t)sizeof(Acc) <= kLdsBytes;
    if (wb == SPX_WB_LDS_ATOMIC && !lds_ok && nnz_x > 0)
        return fail(SPX_ERR_UNSUPPORTED, "lds-atomic write-back needs m * sizeof(acc) <= 64 KiB");
    // the bucket write-back writes every row itself (or, for a sparse
    // output, only the rows it lists)
    const bool writes_all_rows = wb == SPX_WB_BUCKET || wb == SPX_WB_MERGE;
    const bool fill_y = !A.sparse && (!writes_all_rows || nnz_x == 0);
    const bool need_excl =
        nnz_x > 0 && (dist == SPX_DIST_BALANCED || wb == SPX_WB_SORT || wb == SPX_WB_BUCKET || wb == SPX_WB_MERGE);
    int32_t* excl = nullptr;
    Excl ex{nullptr, nullptr};
    if (need_excl) {
        excl = ws.take<int32_t>((size_t)nnz_x + 1);
        int32_t* sws = ws.take<int32_t>(scan_ws_elems((int64_t)nnz_x + 1));
        if (!excl || !sws) return fail(SPX_ERR_WORKSPACE, "spmspv_csc: workspace too small");
        ex.local = excl;
        const int64_t T = ceil_div((int64_t)nnz_x + 1, kBlock);
        // the sort write-back reads nnz_s = excl[nnz_x] on the host: plain array
        if (T <= kLsMaxTiles && wb != SPX_WB_SORT && ((uintptr_t)y & 3) == 0) {
            int32_t* sums = ws.take<int32_t>(kLsMaxTiles);
            int32_t* off = ws.take<int32_t>(kLsMaxTiles);
            if (!sums || !off) return fail(SPX_ERR_WORKSPACE, "spmspv_csc: workspace too small");
            const int64_t ywords = fill_y ? (int64_t)(ybytes / 4) : 0;
            const int F = fill_y ? (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(ywords, kBlock), 2048)) : 0;
            uint32_t* counter = T <= kLsFenceTiles ? A.scan_counter : nullptr;
            k_csc_lengths_scan<<<(unsigned)(F + T), kBlock, 0, s>>>(nnz_x, x_idx, A.col_ptr, excl, sums, off,
                                                                   counter, (uint32_t*)y, ywords,
                                                                   fill_y ? (int)(ybytes & 3) : 0, zero_word(DT), F);
            SPX_HIP(hipGetLastError());
            if (!counter) {
                k_scan_run_totals<<<1, kBlock, 0, s>>>(sums, (int)T, off);
                SPX_HIP(hipGetLastError());
            }
            ex.off = off;
        } else if (nnz_x + 1 <= kProMax && ((uintptr_t)y & 3) == 0) {
            const int64_t ywords = fill_y ? (int64_t)(ybytes / 4) : 0;
            const int fill_blocks = fill_y ? (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(ywords, kBlock), 4096)) : 0;
            k_csc_prologue<<<1 + fill_blocks, kBlock, 0, s>>>(nnz_x, x_idx, A.col_ptr, excl, (uint32_t*)y, ywords,
                                                             fill_y ? (int)(ybytes & 3) : 0, zero_word(DT));
            SPX_HIP(hipGetLastError());
        } else {
            if (fill_y) SPX_TRY(fill_y_zero(y, DT, ybytes, s));
            k_x_lengths<<<(unsigned)ceil_div((int64_t)nnz_x + 1, kBlock), kBlock, 0, s>>>(nnz_x, x_idx, A.col_ptr,
                                                                                           excl);
            SPX_HIP(hipGetLastError());
            SPX_TRY(scan_exclusive_i32(excl, excl, (int64_t)nnz_x + 1, nullptr, sws, s));
        }
    } else if (fill_y) {
        SPX_TRY(fill_y_zero(y, DT, ybytes, s));
    }
    if (nnz_x == 0) return SPX_OK;
    // grid of the balanced kernels: enough tiles for the known or bounded work
    const int64_t ub = A.nnz_s_hint >= 0 ? A.nnz_s_hint : (int64_t)A.nnz;
    const int64_t merge_tiles = std::max<int64_t>(1, ceil_div((int64_t)nnz_x + ub, kCscTile));

    if (wb == SPX_WB_BUCKET) return launch_csc_bucket(A, nnz_x, x_idx, x_val_v, y_v, plan, ex, ws, s);
    if (wb == SPX_WB_MERGE) return launch_csc_merge(A, nnz_x, x_idx, x_val_v, y_v, plan, ex, ws, s);

    if (wb == SPX_WB_ATOMIC || wb == SPX_WB_LDS_ATOMIC) {
        if (dist == SPX_DIST_DIRECT) {
            if (wb == SPX_WB_ATOMIC) {
                const int64_t blocks = ceil_div((int64_t)nnz_x * L, kBlock);
                switch (L) {
#define SPX_L(LL)                                                                                       \
    case LL:                                                                                            \
        k_csc_direct_atomic<DT, LL><<<(unsigned)blocks, kBlock, 0, s>>>(nnz_x, x_idx, x_val, A.col_ptr, \
                                                                        A.row_idx, vals, y);            \
        break;
                    SPX_L(1) SPX_L(2) SPX_L(4) SPX_L(8) SPX_L(16) SPX_L(32) SPX_L(64)
#undef SPX_L
                    default:
                        return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
                }
            } else {
                const int64_t groups = kBlock / L;
                const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(nnz_x, groups), 64));
                const size_t lds = (size_t)A.m * sizeof(Acc);
                switch (L) {
#define SPX_L(LL)                                                                                              \
    case LL:                                                                                                   \
        k_csc_direct_lds<DT, LL><<<grid, kBlock, lds, s>>>(A.m, nnz_x, x_idx, x_val, A.col_ptr, A.row_idx, vals, \
                                                           y);                                                 \
        break;
                    SPX_L(1) SPX_L(2) SPX_L(4) SPX_L(8) SPX_L(16) SPX_L(32) SPX_L(64)
#undef SPX_L
                    default:
                        return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
                }
            }
        } else {
            if (wb == SPX_WB_ATOMIC) {
                const int grid = (int)std::min<int64_t>(merge_tiles, 8192);
                k_csc_merge_atomic<DT><<<grid, kBlock, 0, s>>>(nnz_x, x_idx, x_val, A.col_ptr, A.row_idx, vals,
                                                              ex, y);
            } else {
                const int grid = (int)std::min<int64_t>(merge_tiles, 64);
                k_csc_merge_lds<DT><<<grid, kBlock, (size_t)A.m * sizeof(Acc), s>>>(
                    A.m, nnz_x, x_idx, x_val, A.col_ptr, A.row_idx, vals, ex, y);
            }
        }
        SPX_HIP(hipGetLastError());
        return SPX_OK;
    }

    if (wb == SPX_WB_SORT) {
        // the sort needs the pair count on the host
        int64_t nnz_s = A.nnz_s_hint;
        if (nnz_s < 0) {
            int32_t h = 0;
            SPX_HIP(hipMemcpyAsync(&h, excl + nnz_x, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            SPX_HIP(hipStreamSynchronize(s));
            nnz_s = h;
        }
        if (nnz_s == 0) return SPX_OK;
        const int64_t np = A.nnz;
        uint32_t* keys = ws.take<uint32_t>(np);
        uint32_t* vb = ws.take<uint32_t>(np);
        uint32_t* keys2 = ws.take<uint32_t>(np);
        uint32_t* vb2 = ws.take<uint32_t>(np);
        Acc* vw = nullptr;
        if (sizeof(Acc) == 8) vw = ws.take<Acc>(np);
        int32_t* rws = ws.take<int32_t>(radix_ws_elems(np));
        ws.take<int32_t>(4);
        int32_t* crow = ws.take<int32_t>(ceil_div(np, kCscTile));
        Acc* cval = (Acc*)ws.take<double>(ceil_div(np, kCscTile));
        if (!keys || !vb || !keys2 || !vb2 || !rws || !crow || !cval || (sizeof(Acc) == 8 && !vw))
            return fail(SPX_ERR_WORKSPACE, "spmspv_csc sort: workspace too small");
        EmitPairs<DT> emit{keys, vb, vw};
        if (dist == SPX_DIST_DIRECT) {
            const int64_t blocks = ceil_div((int64_t)nnz_x * L, kBlock);
            switch (L) {
#define SPX_L(LL)                                                                                         \
    case LL:                                                                                              \
        k_csc_direct_pairs<DT, LL><<<(unsigned)blocks, kBlock, 0, s>>>(nnz_x, x_idx, x_val, A.col_ptr,    \
                                                                       A.row_idx, vals, ex, emit);        \
        break;
                SPX_L(1) SPX_L(2) SPX_L(4) SPX_L(8) SPX_L(16) SPX_L(32) SPX_L(64)
#undef SPX_L
                default:
                    return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
            }
        } else {
            const int grid = (int)std::min<int64_t>(ceil_div((int64_t)nnz_x + nnz_s, kCscTile), 8192);
            k_csc_merge_pairs<DT><<<grid, kBlock, 0, s>>>(nnz_x, x_idx, x_val, A.col_ptr, A.row_idx, vals, ex,
                                                         emit);
        }
        SPX_HIP(hipGetLastError());
        bool in_alt = false;
        SPX_TRY(radix_sort_pairs(keys, vb, keys2, vb2, nnz_s, key_bits(A.m), rws, s, &in_alt));
        const uint32_t* sk = in_alt ? keys2 : keys;
        const uint32_t* sv = in_alt ? vb2 : vb;
        const int64_t rtiles = ceil_div(nnz_s, kCscTile);
        k_reduce_by_key<DT><<<(unsigned)rtiles, kBlock, 0, s>>>(nnz_s, sk, sv, vw, y, crow, cval);
        SPX_HIP(hipGetLastError());
        k_rbk_fixup<DT><<<(unsigned)ceil_div(rtiles, kBlock), kBlock, 0, s>>>(rtiles, crow, cval, y);
        SPX_HIP(hipGetLastError());
        return SPX_OK;
    }
    return fail(SPX_ERR_UNSUPPORTED, "write-back not available for spmspv_csc");
}

spx_status launch_spmspv_csc(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                             void* y, const spx_plan* plan, Arena& ws, hipStream_t s) {
    switch (A.dtype) {
        case SPX_F32:
            return launch_csc_t<SPX_F32>(A, nnz_x, x_idx, x_val, y, plan, ws, s);
        case SPX_F64:
            return launch_csc_t<SPX_F64>(A, nnz_x, x_idx, x_val, y, plan, ws, s);
        case SPX_I32:
            return launch_csc_t<SPX_I32>(A, nnz_x, x_idx, x_val, y, plan, ws, s);
        case SPX_BOOL:
            return launch_csc_t<SPX_BOOL>(A, nnz_x, x_idx, x_val, y, plan, ws, s);
        case SPX_F32_MINPLUS:
            return launch_csc_t<SPX_F32_MINPLUS>(A, nnz_x, x_idx, x_val, y, plan, ws, s);
    }
    return fail(SPX_ERR_DTYPE, "spmspv_csc: unknown dtype");
}

}  // namespace spx
