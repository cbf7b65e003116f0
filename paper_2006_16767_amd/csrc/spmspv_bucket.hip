// Bucket write-back of the column-major SpMSpV.
//
// The rows of y are cut into NB buckets of R rows (R a power of two, R * acc
// size <= 64 KiB so a bucket's slice of y fits in LDS). Two kernels (a short
// x with the direct distribution takes the one-launch walk instead, see
// k_bucket_walk):
//
//  scatter     each workgroup takes a chunk of effective positions (one
//              merge-path tile for the balanced distribution, a contiguous
//              range of x entries for the direct one), counts its pairs per
//              bucket in LDS, prefix-sums the counts and writes every pair
//              (local row as uint16, product) into the chunk's own range of
//              the pair buffer, grouped by bucket. The chunk's range is its
//              range of prefix positions, so no global atomic and no count
//              pass are needed. Per (bucket, chunk) it records the offset and
//              count of that group, chunk-major (each chunk writes its own
//              contiguous row of the tables).
//  accumulate  one workgroup per bucket zeroes an LDS copy of its R rows,
//              adds the pairs of every chunk's group with LDS atomics, and
//              writes all R rows of y once (rows that received nothing get 0,
//              so y needs no zero fill).
//
// Traffic per effective entry: the CSC read (index + value) plus one pair
// write and one pair read (6 bytes for FP32 values), instead of a global
// atomic per entry.
#include <algorithm>

#include "common.hpp"
#include "csc_tile.hpp"
#include "csc_walk.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kMaxBuckets = 4096;
constexpr int kBucketLdsBytes = 65536;
constexpr int kDirectChunks = 1024;  // chunk count of the direct distribution

// exclusive scan of s_cnt[0..NB) into s_off[0..NB) by the whole workgroup
__device__ __forceinline__ void bucket_scan(const int32_t* s_cnt, int32_t* s_off, int NB, int32_t* s_tmp) {
    const int per = (NB + kBlock - 1) / kBlock;
    const int b0 = threadIdx.x * per;
    int32_t sum = 0;
    for (int b = b0; b < b0 + per && b < NB; ++b) sum += s_cnt[b];
    int32_t tot;
    const int32_t incl = block_incl_scan(sum, s_tmp, &tot);
    int32_t run = incl - sum;
    for (int b = b0; b < b0 + per && b < NB; ++b) {
        s_off[b] = run;
        run += s_cnt[b];
    }
}

template <int DT>
struct BucketOut {
    uint16_t* prow;
    typename SR<DT>::Acc* pval;  // unused for BOOL
    int32_t* moff;               // [NB][stride]
    int32_t* mcnt;               // [NB][stride]
    int32_t stride;
};

// ------------------------------------------------------------------ balanced scatter
// Chunk c = merge tile c. One pass: every thread forms the pairs of its
// kCscIpt positions in registers, takes each pair's rank within its bucket
// from the LDS counting atomic, and after the workgroup scan of the counts
// stores the pair at the chunk's start + the bucket's offset + that rank.
// The chunk's pairs fill a contiguous range, which the L2 assembles into
// whole lines.
template <int DT>
__global__ __launch_bounds__(kBlock) void k_bucket_scatter_merge(
    int32_t nnz_x, const int32_t* __restrict__ x_idx, const typename SR<DT>::X* __restrict__ x_val,
    const int32_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const typename SR<DT>::V* __restrict__ vals, const Excl excl, int logR, int NB,
    BucketOut<DT> out) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    __shared__ CscTileLds<DT> L;
    __shared__ int32_t s_tmp[kWavesPerBlock];
    extern __shared__ __align__(16) int32_t s_dyn[];  // counts and offsets, NB each
    int32_t* s_cnt = s_dyn;
    int32_t* s_off = s_dyn + NB;
    const int64_t nnz_s = excl[nnz_x];
    const int64_t tiles = ceil_div((int64_t)nnz_x + nnz_s, kCscTile);
    const int64_t chunk = blockIdx.x;
    if (chunk >= tiles) return;  // the accumulate pass reads only the chunks that exist
    const int rmask = (1 << logR) - 1;
    for (int b = threadIdx.x; b < NB; b += kBlock) s_cnt[b] = 0;
    const CscTile t = csc_tile_setup<DT>(chunk, nnz_x, nnz_s, x_idx, x_val, col_ptr, excl, L);
    int r[kCscIpt], slot[kCscIpt];
    Acc v[kCscIpt];
#pragma unroll
    for (int i = 0; i < kCscIpt; ++i) {
        const int p = t.p0 + threadIdx.x + i * kBlock;
        r[i] = -1;
        if (p < t.p1) {
            const int u = csc_tile_locate<DT>(p, t, L);
            const int k = L.cs[u] + (p - L.excl[u]);
            r[i] = row_idx[k];
            if constexpr (S::kVals) v[i] = S::mul(S::val(vals, k), L.v[u]);
        }
    }
#pragma unroll
    for (int i = 0; i < kCscIpt; ++i)
        if (r[i] >= 0) slot[i] = atomicAdd(&s_cnt[r[i] >> logR], 1);
    __syncthreads();
    bucket_scan(s_cnt, s_off, NB, s_tmp);
    __syncthreads();
    const int P0 = t.p0;
    for (int b = threadIdx.x; b < NB; b += kBlock) {
        const int64_t mi = chunk * NB + b;  // chunk-major: the chunk's table is one contiguous run
        out.moff[mi] = P0 + s_off[b];
        out.mcnt[mi] = s_cnt[b];
    }
#pragma unroll
    for (int i = 0; i < kCscIpt; ++i) {
        if (r[i] >= 0) {
            const int64_t pos = (int64_t)P0 + s_off[r[i] >> logR] + slot[i];
            out.prow[pos] = (uint16_t)(r[i] & rmask);
            if constexpr (S::kVals) out.pval[pos] = v[i];
        }
    }
}

// ------------------------------------------------------------------ direct scatter
// Chunk c = x entries [c * E, (c + 1) * E); a group of L lanes per entry walks
// the column twice: once to count per bucket, once to write.
template <int DT, int L>
__global__ __launch_bounds__(kBlock) void k_bucket_scatter_direct(
    int32_t nnz_x, int32_t E, const int32_t* __restrict__ x_idx, const typename SR<DT>::X* __restrict__ x_val,
    const int32_t* __restrict__ col_ptr, const int32_t* __restrict__ row_idx,
    const typename SR<DT>::V* __restrict__ vals, const Excl excl, int logR, int NB,
    BucketOut<DT> out) {
    using S = SR<DT>;
    __shared__ int32_t s_cnt[kMaxBuckets];
    __shared__ int32_t s_off[kMaxBuckets];
    __shared__ int32_t s_tmp[kWavesPerBlock];
    const int c = blockIdx.x;
    const int e_begin = (int)std::min<int64_t>((int64_t)c * E, nnz_x);
    const int e_end = (int)std::min<int64_t>((int64_t)(c + 1) * E, nnz_x);
    const int P0 = excl[e_begin];
    const int groups = kBlock / L;
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    for (int b = threadIdx.x; b < NB; b += kBlock) s_cnt[b] = 0;
    __syncthreads();
    for (int e = e_begin + g; e < e_end; e += groups) {
        const int j = x_idx[e];
        const int c0 = col_ptr[j], c1 = col_ptr[j + 1];
        for (int k = c0 + lane; k < c1; k += L) atomicAdd(&s_cnt[row_idx[k] >> logR], 1);
    }
    __syncthreads();
    bucket_scan(s_cnt, s_off, NB, s_tmp);
    __syncthreads();
    for (int b = threadIdx.x; b < NB; b += kBlock) {
        const int64_t mi = (int64_t)c * NB + b;
        out.moff[mi] = P0 + s_off[b];
        out.mcnt[mi] = s_cnt[b];
        s_cnt[b] = 0;  // becomes the write cursor
    }
    __syncthreads();
    for (int e = e_begin + g; e < e_end; e += groups) {
        const int j = x_idx[e];
        const typename S::X v = S::kVals ? x_val[e] : (typename S::X)1;
        const int c0 = col_ptr[j], c1 = col_ptr[j + 1];
        for (int k = c0 + lane; k < c1; k += L) {
            const int r = row_idx[k];
            const int b = r >> logR;
            const int64_t pos = (int64_t)P0 + s_off[b] + atomicAdd(&s_cnt[b], 1);
            out.prow[pos] = (uint16_t)(r & ((1 << logR) - 1));
            if constexpr (S::kVals) out.pval[pos] = S::mul(S::val(vals, k), v);
        }
    }
}

// ------------------------------------------------------------------ accumulate
// One 1024-thread workgroup per bucket. nch_fixed >= 0: number of chunks;
// otherwise derived from excl[nnz_x] and the tiles per chunk. The bucket's
// groups are taken kAccWin chunks at a time: their counts are prefix-summed
// in LDS, which flattens the window into one run of pairs that all threads
// stream through (each pair finds its chunk by a binary search in LDS), four
// independent pairs per thread per step.
constexpr int kAccThreads = 1024;
constexpr int kAccWin = 4096;

// Sparse output of one bucket (rows base .. base + R - 1): thread t lists
// its R / kAccThreads consecutive rows that were reached (touched bit, or a
// nonzero accumulator for the pattern semiring) and are not masked; one
// atomic per workgroup reserves their slots. Contains __syncthreads.
template <int DT>
__device__ __forceinline__ void bucket_emit_sparse(const typename SR<DT>::Acc* acc, const uint32_t* touched,
                                                   int64_t base, int R, int32_t m, const SparseOut& so) {
    using S = SR<DT>;
    constexpr int kWaves = kAccThreads / kWave;
    __shared__ int32_t s_w[kWaves];
    __shared__ int32_t s_base;
    const int per = R >= kAccThreads ? R / kAccThreads : 1;  // at most 16
    const int r0 = threadIdx.x * per;
    uint32_t keep = 0;
    if (r0 < R) {
        for (int j = 0; j < per; ++j) {
            const int r = r0 + j;
            const int64_t row = base + r;
            bool t;
            if constexpr (S::kVals)
                t = (touched[r >> 5] >> (r & 31)) & 1u;
            else
                t = acc[r] != 0u;
            if (t && row < m && !(so.mask && ((so.mask[row >> 5] >> (row & 31)) & 1u))) keep |= 1u << j;
        }
    }
    const int32_t cnt = __popc(keep);
    const int32_t incl = wave_incl_scan(cnt);
    if (lane_id() == kWave - 1) s_w[wave_id()] = incl;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int i = 0; i < kWaves; ++i) {
        const int32_t t = s_w[i];
        if (i < wave_id()) pre += t;
        tot += t;
    }
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(so.count, tot) : 0;
    __syncthreads();
    int32_t slot = s_base + pre + incl - cnt;
    auto* val = (typename S::Y*)so.val;
    while (keep) {
        const int j = __ffs(keep) - 1;
        keep &= keep - 1;
        so.idx[slot] = (int32_t)(base + r0 + j);
        if (val) val[slot] = S::out(acc[r0 + j]);
        ++slot;
    }
}

template <int DT, bool SPARSE>
__global__ __launch_bounds__(kAccThreads) void k_bucket_accumulate(int32_t m, int logR, int32_t nch_fixed,
                                                                   int32_t nnz_x,
                                                                   const Excl excl,
                                                                   const uint16_t* __restrict__ prow,
                                                                   const typename SR<DT>::Acc* __restrict__ pval,
                                                                   const int32_t* __restrict__ moff,
                                                                   const int32_t* __restrict__ mcnt, int32_t stride,
                                                                   typename SR<DT>::Y* __restrict__ y,
                                                                   const SparseOut so) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    constexpr int kWaves = kAccThreads / kWave;
    constexpr bool kTouch = SPARSE && S::kVals;  // a value can sum to 0: keep a touched bit per row
    extern __shared__ __align__(16) char s_raw[];  // typed as the accumulator: 8-byte LDS ops need the alignment
    Acc* acc = (Acc*)s_raw;
    __shared__ int32_t s_pre[kAccWin + 1];
    __shared__ int32_t s_off[kAccWin];
    __shared__ int32_t s_wsum[kWaves];
    const int R = 1 << logR;
    uint32_t* touched = (uint32_t*)(acc + R);
    const int b = blockIdx.x;
    for (int r = threadIdx.x; r < R; r += kAccThreads) acc[r] = S::zero();
    if constexpr (kTouch)
        for (int w = threadIdx.x; w < (R + 31) / 32; w += kAccThreads) touched[w] = 0u;
    int64_t nch = nch_fixed;
    if (nch < 0) nch = ceil_div((int64_t)nnz_x + excl[nnz_x], kCscTile);  // one chunk per merge tile
    // the tables are chunk-major (row c holds the chunk's NB groups): this
    // bucket's entries sit NB apart
    const int NB = (int)gridDim.x;
    (void)stride;
    constexpr int kPer = kAccWin / kAccThreads;
    for (int64_t w0 = 0; w0 < nch; w0 += kAccWin) {
        const int wn = (int)std::min<int64_t>(kAccWin, nch - w0);
        int32_t cnt[kPer];
        int32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int c = threadIdx.x * kPer + i;
            cnt[i] = c < wn ? mcnt[(w0 + c) * NB + b] : 0;
            if (c < wn) s_off[c] = moff[(w0 + c) * NB + b];
            sum += cnt[i];
        }
        // workgroup-wide exclusive scan of the per-thread sums
        const int32_t wincl = wave_incl_scan(sum);
        if (lane_id() == kWave - 1) s_wsum[wave_id()] = wincl;
        __syncthreads();
        int32_t pre = 0, tot = 0;
        for (int i = 0; i < kWaves; ++i) {
            const int32_t t = s_wsum[i];
            if (i < wave_id()) pre += t;
            tot += t;
        }
        int32_t run = pre + wincl - sum;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            s_pre[threadIdx.x * kPer + i] = run;
            run += cnt[i];
        }
        __syncthreads();
        auto locate = [&](int i) {
            int lo = 0, hi = wn - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pre[mid] <= i)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            return s_off[lo] + (i - s_pre[lo]);
        };
        int i = threadIdx.x;
        for (; i + 3 * kAccThreads < tot; i += 4 * kAccThreads) {
            int q[4];
            uint16_t r[4];
            Acc v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = locate(i + u * kAccThreads);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                r[u] = prow[q[u]];
                if constexpr (S::kVals) v[u] = pval[q[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if constexpr (S::kVals)
                    S::lds_atomic_add(&acc[r[u]], v[u]);
                else
                    acc[r[u]] = 1u;
                if constexpr (kTouch) atomicOr(&touched[r[u] >> 5], 1u << (r[u] & 31));
            }
        }
        for (; i < tot; i += kAccThreads) {
            const int q = locate(i);
            const int rq = prow[q];
            if constexpr (S::kVals)
                S::lds_atomic_add(&acc[rq], pval[q]);
            else
                acc[rq] = 1u;
            if constexpr (kTouch) atomicOr(&touched[rq >> 5], 1u << (rq & 31));
        }
        __syncthreads();
    }
    const int64_t base = (int64_t)b << logR;
    if constexpr (SPARSE) {
        bucket_emit_sparse<DT>(acc, touched, base, R, m, so);
    } else {
        for (int r = threadIdx.x; r < R; r += kAccThreads)
            if (base + r < m) y[base + r] = S::out(acc[r]);
    }
}

// ------------------------------------------------------------------ walk (short x)
// The direct bucket write-back for a short x, in one launch: one 1024-thread
// workgroup per bucket zeroes its R rows in LDS and walks the columns of x
// restricted to them (csc_walk.hpp: groups of G lanes per x entry, G = the
// plan's lanes, or the most that lets every entry of x go out in one
// round). Then the workgroup writes its rows of y once. No pair buffer, no
// prefix, no zero fill of y.
constexpr int kWalkMaxX = 2048;       // x entries of a walk
constexpr int64_t kWalkMaxS = 16384;  // estimated selected entries of a walk

template <int DT, bool SPARSE, int G>
__global__ __launch_bounds__(kAccThreads) void k_bucket_walk(int32_t m, int logR, int32_t nnz_x,
                                                             const int32_t* __restrict__ x_idx,
                                                             const typename SR<DT>::X* __restrict__ x_val,
                                                             const int32_t* __restrict__ col_ptr,
                                                             const int32_t* __restrict__ row_idx,
                                                             const typename SR<DT>::V* __restrict__ vals,
                                                             typename SR<DT>::Y* __restrict__ y,
                                                             const SparseOut so) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    constexpr bool kTouch = SPARSE && S::kVals;
    extern __shared__ __align__(16) char s_raw[];  // typed as the accumulator: 8-byte LDS ops need the alignment
    Acc* acc = (Acc*)s_raw;
    const int R = 1 << logR;
    uint32_t* touched = (uint32_t*)(acc + R);
    const int b = blockIdx.x;
    const int lo = b << logR, hi = lo + R;
    for (int r = threadIdx.x; r < R; r += kAccThreads) acc[r] = S::zero();
    if constexpr (kTouch)
        for (int w = threadIdx.x; w < (R + 31) / 32; w += kAccThreads) touched[w] = 0u;
    __syncthreads();
    walk_columns<DT, G>(kAccThreads, nnz_x, x_idx, x_val, col_ptr, row_idx, lo, hi,
                        [&](int r, int k, typename S::X v) {
                            if constexpr (S::kVals)
                                S::lds_atomic_add(&acc[r], S::mul(S::val(vals, k), v));
                            else
                                acc[r] = 1u;
                            if constexpr (kTouch) atomicOr(&touched[r >> 5], 1u << (r & 31));
                        });
    __syncthreads();
    if constexpr (SPARSE) {
        bucket_emit_sparse<DT>(acc, touched, lo, R, m, so);
    } else {
        for (int r = threadIdx.x; r < R; r += kAccThreads)
            if (lo + r < m) y[lo + r] = S::out(acc[r]);
    }
}

// ------------------------------------------------------------------ launch
struct BucketGeom {
    int logR, NB;
};

static bool bucket_geometry(int32_t m, int dtype, int bucket_rows, BucketGeom* g) {
    const int asz = dtype == SPX_F64 ? 8 : 4;
    const int rmax = kBucketLdsBytes / asz;
    int R;
    if (bucket_rows > 0) {
        R = bucket_rows;
    } else {
        R = 64;
        while (R < rmax && (int64_t)R * 256 < m) R <<= 1;
        while (R < rmax && ceil_div(m, R) > kMaxBuckets) R <<= 1;
    }
    if (R > rmax || R > 65536) return false;
    int logR = 0;
    while ((1 << logR) < R) ++logR;
    g->logR = logR;
    g->NB = (int)std::max<int64_t>(1, ceil_div(m, R));
    return g->NB <= kMaxBuckets;
}

static int64_t bucket_chunks(int32_t nnz_x, int64_t nnz_s_ub, const spx_plan* plan) {
    if (plan->distribution == SPX_DIST_BALANCED)
        return std::max<int64_t>(1, ceil_div((int64_t)nnz_x + nnz_s_ub, kCscTile));
    return std::max<int64_t>(1, std::min<int64_t>(nnz_x, kDirectChunks));
}

size_t csc_bucket_ws(int32_t m, int32_t nnz, int32_t nnz_x, int dtype, const spx_plan* plan) {
    BucketGeom g;
    if (!bucket_geometry(m, dtype, plan->bucket_rows, &g)) return 0;
    const int64_t ch = bucket_chunks(nnz_x, nnz, plan);
    Sizer z;
    z.take<uint16_t>((size_t)nnz + 1);
    if (dtype != SPX_BOOL) z.take<double>((size_t)nnz + 1);
    z.take<int32_t>((size_t)g.NB * ch);
    z.take<int32_t>((size_t)g.NB * ch);
    return z.used;
}

template <int DT>
static spx_status launch_bucket_t(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val_v,
                                  void* y_v, const spx_plan* plan, const Excl excl, Arena& ws, hipStream_t s) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    BucketGeom g;
    if (!bucket_geometry(A.m, DT, plan->bucket_rows, &g))
        return fail(SPX_ERR_UNSUPPORTED, "bucket write-back: rows per bucket must fit 64 KiB of LDS and at most 4096 buckets");
    const auto* x_val = (const typename S::X*)x_val_v;
    const auto* vals = (const typename S::V*)A.vals;
    auto* y = (typename S::Y*)y_v;
    const int64_t ub = A.nnz_s_hint >= 0 ? A.nnz_s_hint : (int64_t)A.nnz;
    const int64_t ch = bucket_chunks(nnz_x, ub, plan);
    BucketOut<DT> out;
    out.prow = ws.take<uint16_t>((size_t)ub + 1);
    out.pval = S::kVals ? ws.take<Acc>((size_t)ub + 1) : nullptr;
    out.moff = ws.take<int32_t>((size_t)g.NB * ch);
    out.mcnt = ws.take<int32_t>((size_t)g.NB * ch);
    out.stride = (int32_t)ch;
    if (!out.prow || (S::kVals && !out.pval) || !out.moff || !out.mcnt)
        return fail(SPX_ERR_WORKSPACE, "bucket write-back: workspace too small");
    int32_t nch_fixed = -1;
    if (plan->distribution == SPX_DIST_BALANCED) {
        k_bucket_scatter_merge<DT><<<(unsigned)ch, kBlock, (size_t)2 * g.NB * sizeof(int32_t), s>>>(
            nnz_x, x_idx, x_val, A.col_ptr, A.row_idx, vals, excl, g.logR, g.NB, out);
    } else {
        const int32_t E = (int32_t)ceil_div(nnz_x, ch);
        nch_fixed = (int32_t)ceil_div(nnz_x, E);
        const double avg = A.n > 0 ? (double)A.nnz / A.n : 0.0;
        int L = plan->lanes > 0 ? plan->lanes : 1;
        if (plan->lanes <= 0)
            while (L < 64 && L < avg) L <<= 1;
        switch (L) {
#define SPX_L(LL)                                                                                              \
    case LL:                                                                                                   \
        k_bucket_scatter_direct<DT, LL><<<(unsigned)nch_fixed, kBlock, 0, s>>>(nnz_x, E, x_idx, x_val, A.col_ptr, \
                                                                               A.row_idx, vals, excl, g.logR,  \
                                                                               g.NB, out);                     \
        break;
            SPX_L(1) SPX_L(2) SPX_L(4) SPX_L(8) SPX_L(16) SPX_L(32) SPX_L(64)
#undef SPX_L
            default:
                return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
        }
    }
    SPX_HIP(hipGetLastError());
    const size_t R = (size_t)1 << g.logR;
    if (A.sparse) {
        const size_t lds = R * sizeof(Acc) + (S::kVals ? ceil_div(R, 32) * 4 : 0);
        k_bucket_accumulate<DT, true><<<(unsigned)g.NB, kAccThreads, lds, s>>>(
            A.m, g.logR, nch_fixed, nnz_x, excl, out.prow, out.pval, out.moff, out.mcnt, out.stride, nullptr,
            *A.sparse);
    } else {
        k_bucket_accumulate<DT, false><<<(unsigned)g.NB, kAccThreads, R * sizeof(Acc), s>>>(
            A.m, g.logR, nch_fixed, nnz_x, excl, out.prow, out.pval, out.moff, out.mcnt, out.stride, y,
            SparseOut{});
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

// Every bucket's workgroup scans the short columns of x whole and cuts the
// long ones to its rows by binary search, so a walk's cost follows nnz_x
// and the average column length, not nnz_s (a hub column costs two
// searches per bucket). The test therefore uses nnz_x times the average
// column length whether or not the caller knows nnz_s.
bool csc_bucket_walks(const CscArgs& A, int32_t nnz_x, const spx_plan* plan) {
    if (plan->writeback != SPX_WB_BUCKET || plan->distribution != SPX_DIST_DIRECT) return false;
    const int64_t est = (int64_t)((double)nnz_x * (A.n > 0 ? (double)A.nnz / A.n : 0.0));
    return nnz_x <= kWalkMaxX && est <= kWalkMaxS;
}

template <int DT, bool SPARSE>
static void walk_launch(int G, unsigned grid, size_t lds, hipStream_t s, int32_t m, int logR, int32_t nnz_x,
                        const int32_t* x_idx, const void* x_val, const CscArgs& A, void* y, const SparseOut& so) {
    using S = SR<DT>;
    switch (G) {
#define SPX_G(GG)                                                                                          \
    case GG:                                                                                               \
        k_bucket_walk<DT, SPARSE, GG><<<grid, kAccThreads, lds, s>>>(                                     \
            m, logR, nnz_x, x_idx, (const typename S::X*)x_val, A.col_ptr, A.row_idx,                      \
            (const typename S::V*)A.vals, (typename S::Y*)y, so);                                          \
        break;
        SPX_G(1) SPX_G(2) SPX_G(4) SPX_G(8) SPX_G(16) SPX_G(32) SPX_G(64)
#undef SPX_G
    }
}

template <int DT>
static spx_status launch_walk_t(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val, void* y,
                                const spx_plan* plan, hipStream_t s) {
    using S = SR<DT>;
    BucketGeom g;
    if (!bucket_geometry(A.m, DT, plan->bucket_rows, &g))
        return fail(SPX_ERR_UNSUPPORTED, "bucket write-back: rows per bucket must fit 64 KiB of LDS and at most 4096 buckets");
    // lanes per x entry: the plan's, else the most that send every entry
    // out in one round of the workgroup
    int G = plan->lanes;
    if (G <= 0) {
        G = 64;
        while (G > 1 && (int64_t)nnz_x * G > kAccThreads) G >>= 1;
    }
    if (G > 64 || (G & (G - 1))) return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
    const size_t R = (size_t)1 << g.logR;
    if (A.sparse) {
        const size_t lds = R * sizeof(typename S::Acc) + (S::kVals ? ceil_div(R, 32) * 4 : 0);
        walk_launch<DT, true>(G, (unsigned)g.NB, lds, s, A.m, g.logR, nnz_x, x_idx, x_val, A, nullptr, *A.sparse);
    } else {
        walk_launch<DT, false>(G, (unsigned)g.NB, R * sizeof(typename S::Acc), s, A.m, g.logR, nnz_x, x_idx, x_val,
                               A, y, SparseOut{});
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status launch_csc_bucket_walk(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val, void* y,
                                  const spx_plan* plan, hipStream_t s) {
    switch (A.dtype) {
        case SPX_F32: return launch_walk_t<SPX_F32>(A, nnz_x, x_idx, x_val, y, plan, s);
        case SPX_F64: return launch_walk_t<SPX_F64>(A, nnz_x, x_idx, x_val, y, plan, s);
        case SPX_I32: return launch_walk_t<SPX_I32>(A, nnz_x, x_idx, x_val, y, plan, s);
        case SPX_BOOL: return launch_walk_t<SPX_BOOL>(A, nnz_x, x_idx, x_val, y, plan, s);
        case SPX_F32_MINPLUS: return launch_walk_t<SPX_F32_MINPLUS>(A, nnz_x, x_idx, x_val, y, plan, s);
    }
    return fail(SPX_ERR_DTYPE, "bucket: unknown dtype");
}

spx_status launch_csc_bucket(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val, void* y,
                             const spx_plan* plan, const Excl excl, Arena& ws, hipStream_t s) {
    switch (A.dtype) {
        case SPX_F32:
            return launch_bucket_t<SPX_F32>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_F64:
            return launch_bucket_t<SPX_F64>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_I32:
            return launch_bucket_t<SPX_I32>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_BOOL:
            return launch_bucket_t<SPX_BOOL>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_F32_MINPLUS:
            return launch_bucket_t<SPX_F32_MINPLUS>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
    }
    return fail(SPX_ERR_DTYPE, "bucket: unknown dtype");
}

}  // namespace spx
