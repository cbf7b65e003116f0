// Merge write-back of the column-major SpMSpV: each tile sorts its
// (row, product) pairs in LDS and reduces them to one partial sum per row;
// the sorted runs of all tiles are then merged per range of rows, and every
// row's partials are added in tile order. The sort-based write-back
// (Section 4.2.2) moves every pair through a global sort; here a pair is
// sorted inside its own tile, which also folds repeated rows (hub rows)
// before anything is written, and the merge reads each tile's run once.
// No atomics anywhere, so the result is the same bits on every call.
//
//  tile sort   (one 256-thread workgroup per tile of kCscTile pairs): the
//              pairs come from a merge-path tile over (x entries + effective
//              positions) for the balanced distribution, or from the
//              position range of the pair buffer that the direct emission
//              filled. Keys (row, slot) are sorted by a bitonic network in
//              LDS; a segmented scan over the sorted pairs sums each row;
//              the tile's run (ascending rows, one entry per row) is stored
//              at the tile's own range, with, per bucket of R rows, where
//              the bucket's part of the run starts and how long it is.
//  merge       (one 1024-thread workgroup per bucket): the bucket's parts of
//              consecutive tiles are gathered into windows of at most
//              kMergeWin pairs, each window is sorted by (row, position in
//              the window), which lists a row's partials in tile order, and
//              the first pair of each row adds the row's partials into the
//              bucket's accumulator in LDS (one writer per row). Every row
//              of the bucket, touched or not, is written once.
#include <algorithm>

#include "common.hpp"
#include "csc_tile.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kMergeThreads = 1024;
constexpr int kMergeWin = 2048;          // pairs per merge window (a tile's run fits)
// LDS of a bucket's accumulator: with the window's arrays the kernel stays
// within 64 KiB (FP64 windows take twice the bytes, so FP64 buckets are half
// as long)
constexpr int kMergeAccBytes = 32768;
constexpr int kMergeMaxBuckets = 4096;
constexpr int kMergeIpt = kCscIpt;       // pairs per thread in a tile

// Bitonic sort of s[0..N) ascending by the whole key, N a power of two
// >= 2, by NT threads. Contains __syncthreads.
template <typename K, int NT>
__device__ __forceinline__ void bitonic_sort_lds(K* s, int N) {
    for (int k = 2; k <= N; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < N; i += NT) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const K a = s[i], b = s[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        s[i] = b;
                        s[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ int pow2_at_least(int v) {
    int n = 2;
    while (n < v) n <<= 1;
    return n;
}

template <int DT>
struct MergeOut {
    uint16_t* prow;               // local row of each run entry
    typename SR<DT>::Acc* pval;   // its partial sum
    int32_t* moff;                // [NB][stride]: where bucket b's part of tile t's run starts
    int32_t* mcnt;                // [NB][stride]: its length
    int32_t stride;
};

template <int DT>
union MergeTileLds {
    CscTileLds<DT> csc;
    struct {
        uint64_t key[kCscTile];  // row << 32 | slot
        typename SR<DT>::Acc val[kCscTile];
        uint32_t urow[kCscTile];  // the run's rows, ascending
        typename SR<DT>::Acc cv[kBlock];
        int32_t flag[kBlock];
        int32_t tmp[kWavesPerBlock];
    } s;
};

// Pairs written by the direct emission at their prefix positions.
template <int DT>
struct EmitRowVal {
    int32_t* row;
    typename SR<DT>::Acc* val;
    __device__ void operator()(int r, typename SR<DT>::Acc v, int64_t p) const {
        row[p] = r;
        val[p] = v;
    }
};

template <int DT, int L>
__global__ __launch_bounds__(kBlock) void k_merge_emit_direct(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                              const typename SR<DT>::X* __restrict__ x_val,
                                                              const int32_t* __restrict__ col_ptr,
                                                              const int32_t* __restrict__ row_idx,
                                                              const typename SR<DT>::V* __restrict__ vals,
                                                              const Excl excl, EmitRowVal<DT> emit) {
    const int64_t e = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / L;
    if (e >= nnz_x) return;
    csc_direct_entry<DT, L>((int)e, threadIdx.x % L, x_idx, x_val, col_ptr, row_idx, vals, excl, emit);
}

// One tile: sort, reduce by row, store the run and the bucket table.
// FROM_PAIRS: the tile is positions [t * kCscTile, ...) of the emitted
// pairs (direct distribution); otherwise merge tile t over the CSC.
template <int DT, bool FROM_PAIRS>
__global__ __launch_bounds__(kBlock) void k_merge_tile_sort(int32_t nnz_x, const int32_t* __restrict__ x_idx,
                                                            const typename SR<DT>::X* __restrict__ x_val,
                                                            const int32_t* __restrict__ col_ptr,
                                                            const int32_t* __restrict__ row_idx,
                                                            const typename SR<DT>::V* __restrict__ vals,
                                                            const Excl excl, const int32_t* __restrict__ prow_in,
                                                            const typename SR<DT>::Acc* __restrict__ pval_in,
                                                            int logR, int NB, MergeOut<DT> out) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    __shared__ MergeTileLds<DT> L;
    const int64_t nnz_s = excl[nnz_x];
    const int64_t tiles = FROM_PAIRS ? ceil_div(nnz_s, kCscTile) : ceil_div((int64_t)nnz_x + nnz_s, kCscTile);
    const int64_t t = blockIdx.x;
    if (t >= tiles) return;  // the merge reads only the tiles that exist
    int r[kMergeIpt];
    Acc v[kMergeIpt];
    int count;
    if constexpr (FROM_PAIRS) {
        const int64_t p0 = t * kCscTile;
        count = (int)std::min<int64_t>(kCscTile, nnz_s - p0);
#pragma unroll
        for (int i = 0; i < kMergeIpt; ++i) {
            const int q = threadIdx.x + i * kBlock;
            r[i] = q < count ? prow_in[p0 + q] : -1;
            v[i] = q < count ? pval_in[p0 + q] : S::zero();
        }
    } else {
        const CscTile tl = csc_tile_setup<DT>(t, nnz_x, nnz_s, x_idx, x_val, col_ptr, excl, L.csc);
        count = tl.p1 - tl.p0;
#pragma unroll
        for (int i = 0; i < kMergeIpt; ++i) {
            const int p = tl.p0 + threadIdx.x + i * kBlock;
            r[i] = -1;
            v[i] = S::zero();
            if (p < tl.p1) {
                const int u = csc_tile_locate<DT>(p, tl, L.csc);
                const int k = L.csc.cs[u] + (p - L.csc.excl[u]);
                r[i] = row_idx[k];
                v[i] = S::mul(S::val(vals, k), L.csc.v[u]);
            }
        }
        __syncthreads();  // the staged entries are dead; the sort reuses their LDS
    }
    const int N = pow2_at_least(count);
#pragma unroll
    for (int i = 0; i < kMergeIpt; ++i) {
        const int q = threadIdx.x + i * kBlock;
        if (q < N) L.s.key[q] = q < count ? ((uint64_t)(uint32_t)r[i] << 32) | (uint32_t)q : ~0ull;
        if (q < count) L.s.val[q] = v[i];
    }
    __syncthreads();
    bitonic_sort_lds<uint64_t, kBlock>(L.s.key, N);
    // per thread kMergeIpt consecutive sorted pairs; a segmented scan over
    // the threads joins the runs that cross thread boundaries
    const int i0 = threadIdx.x * kMergeIpt;
    const int i1 = std::min(i0 + kMergeIpt, count);
    auto row_at = [&](int i) { return (uint32_t)(L.s.key[i] >> 32); };
    auto val_at = [&](int i) { return L.s.val[(uint32_t)L.s.key[i]]; };
    Acc acc = S::zero();
    bool head = false;
    for (int i = i0; i < i1; ++i) {
        if (i == 0 || row_at(i) != row_at(i - 1)) {
            head = true;
            acc = S::zero();
        }
        acc = S::add(acc, val_at(i));
    }
    L.s.flag[threadIdx.x] = head ? 1 : 0;
    L.s.cv[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int f = L.s.flag[threadIdx.x];
        Acc c = L.s.cv[threadIdx.x];
        int fo = 0;
        Acc co = S::zero();
        if ((int)threadIdx.x >= off) {
            fo = L.s.flag[threadIdx.x - off];
            co = L.s.cv[threadIdx.x - off];
        }
        __syncthreads();
        if ((int)threadIdx.x >= off) {
            if (!f) c = S::add(co, c);
            f |= fo;
        }
        L.s.flag[threadIdx.x] = f;
        L.s.cv[threadIdx.x] = c;
        __syncthreads();
    }
    // rank of each run among the tile's runs
    int tails = 0;
    for (int i = i0; i < i1; ++i) tails += (i == count - 1 || row_at(i + 1) != row_at(i)) ? 1 : 0;
    int total;
    const int rank0 = block_incl_scan<int32_t>(tails, L.s.tmp, &total) - tails;
    Acc run = (threadIdx.x > 0 && i0 < count) ? L.s.cv[threadIdx.x - 1] : S::zero();
    const int64_t base = t * kCscTile;
    const int rmask = (1 << logR) - 1;
    int rank = rank0;
    for (int i = i0; i < i1; ++i) {
        if (i == 0 || row_at(i) != row_at(i - 1)) run = S::zero();
        run = S::add(run, val_at(i));
        if (i == count - 1 || row_at(i + 1) != row_at(i)) {
            const uint32_t row = row_at(i);
            out.prow[base + rank] = (uint16_t)(row & (uint32_t)rmask);
            out.pval[base + rank] = run;
            L.s.urow[rank] = row;
            ++rank;
        }
    }
    __syncthreads();
    // bucket b's part of the run: rows in [b << logR, (b + 1) << logR)
    auto lower = [&](uint32_t key) {
        int lo = 0, hi = total;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (L.s.urow[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        return lo;
    };
    for (int b = threadIdx.x; b < NB; b += kBlock) {
        const int a = lower((uint32_t)b << logR);
        const int e = b + 1 < NB ? lower((uint32_t)(b + 1) << logR) : total;
        const int64_t mi = (int64_t)b * out.stride + t;
        out.moff[mi] = (int32_t)(base + a);
        out.mcnt[mi] = e - a;
    }
}

// One bucket: merge the parts of all tiles' runs in windows, add each row's
// partials in tile order, write the bucket's rows of y.
template <int DT, bool FROM_PAIRS>
__global__ __launch_bounds__(kMergeThreads) void k_merge_accumulate(int32_t m, int logR, int32_t nnz_x,
                                                                    const Excl excl,
                                                                    const uint16_t* __restrict__ prow,
                                                                    const typename SR<DT>::Acc* __restrict__ pval,
                                                                    const int32_t* __restrict__ moff,
                                                                    const int32_t* __restrict__ mcnt,
                                                                    int32_t stride, typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    constexpr int kWaves = kMergeThreads / kWave;
    extern __shared__ __align__(16) char s_raw[];  // typed as the accumulator: 8-byte LDS ops need the alignment
    Acc* acc = (Acc*)s_raw;
    __shared__ uint32_t s_key[kMergeWin];  // local row << 11 | position in the window
    __shared__ Acc s_val[kMergeWin];
    __shared__ int32_t s_pre[kMergeThreads + 1];
    __shared__ int32_t s_off[kMergeThreads];
    __shared__ int32_t s_w[kWaves];
    __shared__ int32_t s_take, s_total;
    const int R = 1 << logR;
    const int b = blockIdx.x;
    for (int r = threadIdx.x; r < R; r += kMergeThreads) acc[r] = S::zero();
    const int64_t nnz_s = excl[nnz_x];
    const int64_t tiles = FROM_PAIRS ? ceil_div(nnz_s, kCscTile) : ceil_div((int64_t)nnz_x + nnz_s, kCscTile);
    const int32_t* mo = moff + (int64_t)b * stride;
    const int32_t* mc = mcnt + (int64_t)b * stride;
    for (int64_t c0 = 0; c0 < tiles;) {
        // the longest run of tiles from c0 whose parts fit one window
        const int64_t c = c0 + threadIdx.x;
        const int32_t cnt = c < tiles ? mc[c] : 0;
        const int32_t incl = wave_incl_scan(cnt);
        if (lane_id() == kWave - 1) s_w[wave_id()] = incl;
        if (threadIdx.x == 0) {
            s_take = 0;
            s_total = 0;
        }
        __syncthreads();
        int32_t pre = 0;
        for (int i = 0; i < wave_id(); ++i) pre += s_w[i];
        const int32_t ipos = pre + incl;  // inclusive prefix over the tiles from c0
        const bool fits = c < tiles && ipos <= kMergeWin;
        // a prefix of the threads (the prefix grows); never empty, since
        // one tile's whole run fits a window
        const int take = __syncthreads_count(fits);
        if (fits) {
            s_pre[threadIdx.x] = ipos - cnt;
            s_off[threadIdx.x] = mo[c];
        }
        if ((int)threadIdx.x == take - 1) {
            s_total = ipos;
            s_take = take;
        }
        __syncthreads();
        const int total = s_total;
        const int ntake = s_take;
        // gather the window: pair q of tile j (in tile order) at position q
        for (int q = threadIdx.x; q < total; q += kMergeThreads) {
            int lo = 0, hi = ntake - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_pre[mid] <= q)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const int32_t src = s_off[lo] + (q - s_pre[lo]);
            s_key[q] = ((uint32_t)prow[src] << 11) | (uint32_t)q;
            s_val[q] = pval[src];
        }
        const int N = pow2_at_least(total);
        for (int q = total + threadIdx.x; q < N; q += kMergeThreads) s_key[q] = ~0u;
        __syncthreads();
        bitonic_sort_lds<uint32_t, kMergeThreads>(s_key, N);
        // the first pair of each row adds the row's partials (tile order)
        for (int q = threadIdx.x; q < total; q += kMergeThreads) {
            const uint32_t row = s_key[q] >> 11;
            if (q > 0 && (s_key[q - 1] >> 11) == row) continue;
            Acc sum = s_val[s_key[q] & 2047u];
            for (int u = q + 1; u < total && (s_key[u] >> 11) == row; ++u) sum = S::add(sum, s_val[s_key[u] & 2047u]);
            acc[row] = S::add(acc[row], sum);
        }
        __syncthreads();
        c0 += ntake > 0 ? ntake : 1;
    }
    const int64_t base = (int64_t)b << logR;
    for (int r = threadIdx.x; r < R; r += kMergeThreads)
        if (base + r < m) y[base + r] = S::out(acc[r]);
}

// ------------------------------------------------------------------ launch
struct MergeGeom {
    int logR, NB;
};

static bool merge_geometry(int32_t m, int dtype, int bucket_rows, MergeGeom* g) {
    const int asz = dtype == SPX_F64 ? 8 : 4;
    const int rmax = (dtype == SPX_F64 ? kMergeAccBytes / 2 : kMergeAccBytes) / asz;
    int R;
    if (bucket_rows > 0) {
        R = bucket_rows;
    } else {
        R = 64;
        while (R < rmax && (int64_t)R * 256 < m) R <<= 1;
        while (R < rmax && ceil_div(m, R) > kMergeMaxBuckets) R <<= 1;
    }
    if (R > rmax) return false;
    int logR = 0;
    while ((1 << logR) < R) ++logR;
    g->logR = logR;
    g->NB = (int)std::max<int64_t>(1, ceil_div(m, R));
    return g->NB <= kMergeMaxBuckets;
}

static int64_t merge_tiles_ub(int32_t nnz_x, int64_t nnz_s_ub, const spx_plan* plan) {
    if (plan->distribution == SPX_DIST_BALANCED)
        return std::max<int64_t>(1, ceil_div((int64_t)nnz_x + nnz_s_ub, kCscTile));
    return std::max<int64_t>(1, ceil_div(nnz_s_ub, kCscTile));
}

size_t csc_merge_ws(int32_t m, int32_t nnz, int32_t nnz_x, int dtype, const spx_plan* plan) {
    MergeGeom g;
    if (!merge_geometry(m, dtype, plan->bucket_rows, &g)) return 0;
    const int64_t tiles = merge_tiles_ub(nnz_x, nnz, plan);
    const int asz = dtype == SPX_F64 ? 8 : 4;
    Sizer z;
    if (plan->distribution != SPX_DIST_BALANCED) {
        z.take<int32_t>((size_t)nnz + 1);            // emitted rows
        z.take<char>(((size_t)nnz + 1) * asz);       // emitted products
    }
    z.take<uint16_t>((size_t)tiles * kCscTile);      // the tiles' runs
    z.take<char>((size_t)tiles * kCscTile * asz);
    z.take<int32_t>((size_t)g.NB * tiles);
    z.take<int32_t>((size_t)g.NB * tiles);
    return z.used;
}

template <int DT>
static spx_status launch_merge_t(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val_v, void* y_v,
                                 const spx_plan* plan, const Excl excl, Arena& ws, hipStream_t s) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    MergeGeom g;
    if (!merge_geometry(A.m, DT, plan->bucket_rows, &g))
        return fail(SPX_ERR_UNSUPPORTED, "merge write-back: rows per bucket must fit 32 KiB of LDS and at most 4096 buckets");
    const auto* x_val = (const typename S::X*)x_val_v;
    const auto* vals = (const typename S::V*)A.vals;
    auto* y = (typename S::Y*)y_v;
    const int64_t ub = A.nnz_s_hint >= 0 ? A.nnz_s_hint : (int64_t)A.nnz;
    const bool direct = plan->distribution != SPX_DIST_BALANCED;
    const int64_t tiles = merge_tiles_ub(nnz_x, ub, plan);
    int32_t* erow = nullptr;
    Acc* eval = nullptr;
    if (direct) {
        erow = ws.take<int32_t>((size_t)ub + 1);
        eval = (Acc*)ws.take<char>(((size_t)ub + 1) * sizeof(Acc));
    }
    MergeOut<DT> out;
    out.prow = ws.take<uint16_t>((size_t)tiles * kCscTile);
    out.pval = (Acc*)ws.take<char>((size_t)tiles * kCscTile * sizeof(Acc));
    out.moff = ws.take<int32_t>((size_t)g.NB * tiles);
    out.mcnt = ws.take<int32_t>((size_t)g.NB * tiles);
    out.stride = (int32_t)tiles;
    if ((direct && (!erow || !eval)) || !out.prow || !out.pval || !out.moff || !out.mcnt)
        return fail(SPX_ERR_WORKSPACE, "merge write-back: workspace too small");
    const size_t acc_lds = ((size_t)1 << g.logR) * sizeof(Acc);
    if (direct) {
        const double avg = A.n > 0 ? (double)A.nnz / A.n : 0.0;
        int L = plan->lanes > 0 ? plan->lanes : 1;
        if (plan->lanes <= 0)
            while (L < 64 && L < avg) L <<= 1;
        const int64_t blocks = ceil_div((int64_t)nnz_x * L, kBlock);
        const EmitRowVal<DT> emit{erow, eval};
        switch (L) {
#define SPX_L(LL)                                                                                              \
    case LL:                                                                                                   \
        k_merge_emit_direct<DT, LL><<<(unsigned)blocks, kBlock, 0, s>>>(nnz_x, x_idx, x_val, A.col_ptr, A.row_idx, \
                                                                        vals, excl, emit);                     \
        break;
            SPX_L(1) SPX_L(2) SPX_L(4) SPX_L(8) SPX_L(16) SPX_L(32) SPX_L(64)
#undef SPX_L
            default:
                return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
        }
        SPX_HIP(hipGetLastError());
        k_merge_tile_sort<DT, true><<<(unsigned)tiles, kBlock, 0, s>>>(nnz_x, x_idx, x_val, A.col_ptr, A.row_idx, vals,
                                                                        excl, erow, eval, g.logR, g.NB, out);
        SPX_HIP(hipGetLastError());
        k_merge_accumulate<DT, true><<<(unsigned)g.NB, kMergeThreads, acc_lds, s>>>(
            A.m, g.logR, nnz_x, excl, out.prow, out.pval, out.moff, out.mcnt, out.stride, y);
    } else {
        k_merge_tile_sort<DT, false><<<(unsigned)tiles, kBlock, 0, s>>>(nnz_x, x_idx, x_val, A.col_ptr, A.row_idx,
                                                                         vals, excl, nullptr, nullptr, g.logR, g.NB,
                                                                         out);
        SPX_HIP(hipGetLastError());
        k_merge_accumulate<DT, false><<<(unsigned)g.NB, kMergeThreads, acc_lds, s>>>(
            A.m, g.logR, nnz_x, excl, out.prow, out.pval, out.moff, out.mcnt, out.stride, y);
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status launch_csc_merge(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val, void* y,
                            const spx_plan* plan, const Excl excl, Arena& ws, hipStream_t s) {
    switch (A.dtype) {
        case SPX_F32: return launch_merge_t<SPX_F32>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_F64: return launch_merge_t<SPX_F64>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_I32: return launch_merge_t<SPX_I32>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_BOOL: return launch_merge_t<SPX_BOOL>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
        case SPX_F32_MINPLUS: return launch_merge_t<SPX_F32_MINPLUS>(A, nnz_x, x_idx, x_val, y, plan, excl, ws, s);
    }
    return fail(SPX_ERR_DTYPE, "merge: unknown dtype");
}

}  // namespace spx
