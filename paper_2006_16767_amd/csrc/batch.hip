// Batched SpMSpV: B sparse vectors of uneven sparsity in one graph launch,
// the plan of every vector chosen on the device.
//
//  k_batch_plan        one workgroup per vector: prefix sum of the lengths of
//                      the columns it selects (its nnz_s falls out), then the
//                      three decision trees evaluated on the Table 1 features
//                      (matrix features + nnz_x, x_sparsity, nnz_s,
//                      m_sparsity), and the vector's work-item counts for
//                      the three phases of its plan.
//  k_batch_scan        prefix sums of the counts: one ordered queue per
//                      phase; resets the queue heads.
//  k_batch_phase<A|B|C>  #CUs x 4 persistent workgroups pop the items of one
//                      phase until its queue is drained (every workgroup
//                      exits once the queue head passes the item count);
//                      beside B, on a branch of the graph of its own,
//                      k_batch_fused walks the work units of the fused
//                      groups (a queue per width, a wave per unit):
//                        A: row-major plans scatter x into the vector's
//                           bitvector / value slots; column-major plans zero
//                           the vector's row of Y
//                        B: one merge-path tile (or one row/entry chunk of the
//                           direct distribution) of the vector's kernel
//                        C: row-major balanced fix-up of tile carries, and the
//                           self-cleaning of the bitvector / value slots
//                      Items of one phase never wait for each other: the
//                      ordering between phases is the kernel boundary.
//
// Fused row-major groups: a vector whose plan is row-major (SpMV or CSR
// SpMSpV, any value type but BOOL), or whose entries reach
// kFusedMinXSparsity of n, joins a group that shares one pass over A: 128
// vectors of 4-byte values (two per lane), 64 of 8-byte ones. Its phase-A
// items scatter x into the group's dense slab X^T (n rows = columns of A,
// one slot per vector) and its phase-C items clear it again. k_batch_fused
// walks work units of A for each group (at most kFusedUnitNnz entries of at
// most kFusedUnitRows whole rows, or a piece of a longer row), a wave per
// unit; a last group of at most 64 vectors is walked one per lane. It is a
// kernel of its own (one per width) so that its registers set its
// occupancy, not those of the tile kernels. Pieces of split rows are added
// to Y with atomics (their rows of Y are zeroed by phase-A items of the
// group); every other row is written once. Non-support entries meet zeros
// in the slab, so the bitvector validation of CSR SpMSpV becomes a product
// with zero.
//
// The launches are captured once into a HIP graph by the caller and
// replayed. The per-vector bitvector and value slots are zero when a run
// starts and are cleared again by phase C, so no fill is recorded in the
// graph. Column-major plans write back with device atomics (the sort and
// bucket write-backs need per-vector pair buffers sized by nnz_s, which the
// host does not know without a sync).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "csc_tile.hpp"
#include "csr_tile.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kBatchTile = 2048;     // merge tile (row-major and column-major)
constexpr int kFillChunk = 65536;    // rows of Y zeroed per phase-A item
constexpr int kScatterChunk = 2048;  // x entries scattered / cleared per item
constexpr int kCscDirectEntries = 64;
constexpr int kCscDirectLanes = 4;
constexpr int kGroup = 64;                 // lanes of a fused group's wave

// vectors per lane of a full fused group: two 4-byte values (an 8-byte slab
// load per lane, 128 vectors per group and slab rows of 128 slots), one
// 8-byte value (64 per group). A last group of at most 64 vectors is walked
// one value per lane (32 entries per step instead of 16) over the first half
// of its slab rows.
template <int DT>
constexpr int group_vpl() {
    return sizeof(typename SR<DT>::X) == 4 ? 2 : 1;
}
// a column-major vector this dense joins a fused group: at 1 % two vectors
// could cost a whole pass over A, at 3 % too many products went to atomics
constexpr double kFusedMinXSparsity = 0.02;
constexpr int kSplitZeroRows = 64;  // split rows of Y zeroed per phase-A group item

struct BatchPlan {
    int32_t pattern, dist, wb, lanes;
    int32_t nnz_x, base;
    int32_t nA, nB, nC;
    int32_t gslot;  // slot in the fused row-major groups, or -1
    int64_t nnz_s;
};

struct BatchDev {
    int32_t m, n, nnz;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const void* vals;
    const int32_t* col_ptr;
    const int32_t* row_idx;
    const void* vals_csc;
    const int32_t* part;
    int64_t tiles_mat;
    int32_t B;
    int64_t cap_nnz_x;  // capacity of the per-entry arrays (host bound of vec_ptr[B])
    const int32_t* vec_ptr;
    const int32_t* idx;
    const void* val;
    void* Y;
    const DevSelector* sel;
    int32_t row_lanes;  // lanes per row of the row-major direct distribution
    // workspace
    BatchPlan* plans;
    int32_t* offs;    // 3 x (B + 1)
    int32_t* totals;  // 4
    int32_t* queue;   // queue heads: one per phase, [3] = err, [4, 5] and [6, 7] = the two fused walks' (64-bit)
    int32_t* err;
    int32_t* excl_all;  // cap_nnz_x + B
    uint32_t* bits_all;  // B x nwords
    void* xd_all;        // B x n values
    int32_t* carry_row_all;  // B x tiles_mat
    void* carry_val_all;     // B x tiles_mat accumulators
    int64_t nwords;
    // fused row-major groups
    const int4* units;        // {first row, end row, first entry, end entry}
    int32_t nunits;
    const int32_t* split_rows;  // rows cut into several units
    int32_t nsplit;
    int32_t* gcount;  // vectors in groups (reset per run)
    int32_t* gvec;    // slot -> vector
    void* xt_all;     // ceil(B / gsize) slabs of n x gsize values (self-cleaning)
    int32_t gsize;    // vectors per fused group and slots per slab row: 64 x group_vpl
};

__device__ __forceinline__ int dev_tree_eval(const DevTree& t, const double* f) {
    int i = 0;
    for (int guard = 0; guard < 64 && i >= 0 && i < t.n; ++guard) {
        if (t.cls[i] >= 0) return t.cls[i];
        const int fi = t.feat[i];
        i = (fi >= 0 && fi < F_COUNT && f[fi] <= t.thr[i]) ? t.left[i] : t.right[i];
    }
    return 0;
}

// ------------------------------------------------------------------ plan
template <int DT>
__global__ __launch_bounds__(kBlock) void k_batch_plan(BatchDev a) {
    __shared__ int32_t s_tmp[kWavesPerBlock];
    const int b = blockIdx.x;
    const int base = a.vec_ptr[b];
    const int nx = a.vec_ptr[b + 1] - base;
    if (base < 0 || nx < 0 || (int64_t)a.vec_ptr[a.B] > a.cap_nnz_x || nx > a.n) {
        // vec_ptr disagrees with the capacity the host sized: no work, flag it
        if (threadIdx.x == 0) {
            BatchPlan z{};
            a.plans[b] = z;
            atomicOr(a.err, 2);
        }
        return;
    }
    int32_t* excl = a.excl_all + base + b;
    const int32_t* idx = a.idx + base;
    const DevSelector& S = *a.sel;
    __shared__ int s_fuse;
    // host-known features first: a vector that joins a fused group needs no
    // prefix of its column lengths (unless the trees read nnz_s)
    if (threadIdx.x == 0) {
        int fuse = 0;
        if (DT != SPX_BOOL && a.units != nullptr && nx > 0 && !S.needs_nnz_s) {
            double f[F_COUNT];
            for (int i = 0; i < 9; ++i) f[i] = S.mfeat[i];
            f[9] = nx;
            f[10] = a.n > 0 ? (double)nx / a.n : 0.0;
            f[11] = f[12] = f[13] = 0.0;
            f[F_COUNTED] = 0.0;
            int pat = dev_tree_eval(S.t[0], f);
            if (pat < 0 || pat > 2) pat = 0;
            fuse = pat != SPX_PAT_CSC_SPMSPV || f[10] >= kFusedMinXSparsity;
        }
        s_fuse = fuse;
    }
    __syncthreads();
    if (s_fuse) {
        if (threadIdx.x == 0) {
            BatchPlan p{};
            p.pattern = SPX_PAT_SPMV;
            p.dist = SPX_DIST_BALANCED;
            p.wb = SPX_WB_NONE;
            p.lanes = a.row_lanes;
            p.nnz_x = nx;
            p.base = base;
            p.nnz_s = -1;
            p.gslot = atomicAdd(a.gcount, 1);
            a.gvec[p.gslot] = b;
            p.nA = (int32_t)ceil_div(nx, kScatterChunk);
            p.nB = 0;
            p.nC = (int32_t)ceil_div(nx, kScatterChunk);
            a.plans[b] = p;
        }
        return;
    }
    constexpr int kIpt = 8;
    int32_t carry = 0;
    for (int c0 = 0; c0 < nx; c0 += kBlock * kIpt) {
        int32_t len[kIpt];
        int32_t sum = 0;
#pragma unroll
        for (int i = 0; i < kIpt; ++i) {
            const int e = c0 + threadIdx.x * kIpt + i;
            len[i] = 0;
            if (e < nx) {
                const int j = idx[e];
                len[i] = a.col_ptr[j + 1] - a.col_ptr[j];
            }
            sum += len[i];
        }
        int32_t tot;
        const int32_t incl = block_incl_scan(sum, s_tmp, &tot);
        int32_t run = carry + incl - sum;
#pragma unroll
        for (int i = 0; i < kIpt; ++i) {
            const int e = c0 + threadIdx.x * kIpt + i;
            if (e < nx) excl[e] = run;
            run += len[i];
        }
        carry += tot;
    }
    if (threadIdx.x != 0) return;
    excl[nx] = carry;
    double f[F_COUNT];
    for (int i = 0; i < 9; ++i) f[i] = S.mfeat[i];
    f[9] = nx;
    f[10] = a.n > 0 ? (double)nx / a.n : 0.0;
    f[11] = carry;
    f[12] = a.nnz > 0 ? (double)carry / a.nnz : 0.0;
    f[13] = (double)carry / (double)(nx > 0 ? nx : 1);
    f[F_COUNTED] = 1.0;
    BatchPlan p;
    p.pattern = dev_tree_eval(S.t[0], f);
    if (p.pattern < 0 || p.pattern > 2) p.pattern = 0;
    p.gslot = -1;
    const bool fusable = DT != SPX_BOOL && a.units != nullptr && nx > 0;
    if (fusable && (p.pattern != SPX_PAT_CSC_SPMSPV || f[10] >= kFusedMinXSparsity)) {
        if (p.pattern == SPX_PAT_CSC_SPMSPV) p.pattern = SPX_PAT_SPMV;
        p.gslot = atomicAdd(a.gcount, 1);
        a.gvec[p.gslot] = b;
    }
    p.dist = dev_tree_eval(S.t[1 + p.pattern], f) == SPX_DIST_BALANCED ? SPX_DIST_BALANCED : SPX_DIST_DIRECT;
    p.wb = p.pattern == SPX_PAT_CSC_SPMSPV ? SPX_WB_ATOMIC : SPX_WB_NONE;
    p.lanes = a.row_lanes;
    p.nnz_x = nx;
    p.base = base;
    p.nnz_s = carry;
    if (p.gslot >= 0) {
        p.nA = (int32_t)ceil_div(nx, kScatterChunk);
        p.nB = 0;
        p.nC = (int32_t)ceil_div(nx, kScatterChunk);
    } else if (p.pattern == SPX_PAT_CSC_SPMSPV) {
        p.nA = (int32_t)ceil_div(a.m, kFillChunk);
        p.nB = p.dist == SPX_DIST_BALANCED ? (int32_t)ceil_div((int64_t)nx + carry, kBatchTile)
                                           : (int32_t)ceil_div(nx, kCscDirectEntries);
        p.nC = 0;
    } else {
        const int64_t rows_per_item = (int64_t)(kBlock / a.row_lanes) * 8;
        p.nA = (int32_t)ceil_div(nx, kScatterChunk);
        p.nB = p.dist == SPX_DIST_BALANCED ? (int32_t)a.tiles_mat : (int32_t)ceil_div(a.m, rows_per_item);
        p.nC = (p.dist == SPX_DIST_BALANCED ? 1 : 0) + (int32_t)ceil_div(nx, kScatterChunk);
    }
    a.plans[b] = p;
}

__global__ void k_batch_reset(int32_t* err, int32_t* gcount) {
    *err = 0;
    *gcount = 0;
}

// group items appended after the per-vector items of a phase (the groups'
// walk of A is k_batch_fused): phase A zeroes the split rows of the groups'
// vectors in Y, kSplitZeroRows rows per item (one item for all of them left
// a single workgroup with some 10^5 scattered stores, the tail of the phase)
__device__ __forceinline__ int32_t group_items(const BatchDev& a, int ph, int32_t G) {
    if (ph == 0) return G * (int32_t)ceil_div(a.nsplit, kSplitZeroRows);
    return 0;
}

// ------------------------------------------------------------------ queue
__global__ __launch_bounds__(kBlock) void k_batch_scan(BatchDev a) {
    __shared__ int32_t s_tmp[kWavesPerBlock];
    for (int ph = 0; ph < 3; ++ph) {
        int32_t* off = a.offs + ph * (a.B + 1);
        int32_t carry = 0;
        for (int c0 = 0; c0 < a.B; c0 += kBlock) {
            const int b = c0 + threadIdx.x;
            int32_t v = 0;
            if (b < a.B) v = ph == 0 ? a.plans[b].nA : (ph == 1 ? a.plans[b].nB : a.plans[b].nC);
            int32_t tot;
            const int32_t incl = block_incl_scan(v, s_tmp, &tot);
            if (b < a.B) off[b] = carry + incl - v;
            carry += tot;
        }
        if (threadIdx.x == 0) {
            off[a.B] = carry;
            const int32_t G = (int32_t)ceil_div(*a.gcount, a.gsize);
            a.totals[ph] = carry + group_items(a, ph, G);
        }
        __syncthreads();
    }
    if (threadIdx.x < 3 || (threadIdx.x >= 4 && threadIdx.x < 8)) a.queue[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ persistent
template <int DT>
union BatchLds {
    CsrTileLds<DT, kBatchTile> csr;
    CscTileLds<DT> csc;
};

// last b with off[b] <= item (off has B + 1 entries, non-decreasing)
__device__ __forceinline__ int find_vector(const int32_t* off, int B, int item) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <int DT, int L>
__device__ __forceinline__ void batch_rows_direct(const BatchDev& a, int64_t r0, int64_t r1, bool valid,
                                                  const typename SR<DT>::X* xd, const uint32_t* bits,
                                                  typename SR<DT>::Y* y) {
    using S = SR<DT>;
    const auto* vals = (const typename S::V*)a.vals;
    constexpr int G = kBlock / L;
    const int g = threadIdx.x / L, lane = threadIdx.x % L;
    for (int64_t row = r0 + g; row < r1; row += G) {
        const int k0 = a.row_ptr[row], k1 = a.row_ptr[row + 1];
        ChunkedAcc<DT, 4> acc;  // a partial sum per load slot: bounded chains on hub rows
        int k = k0 + lane;
        for (; k + 3 * L < k1; k += 4 * L) {
            int c[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = a.col_idx[k + u * L];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (!valid || test_bit(bits, c[u]))
                    acc.part[u] = S::fma(S::val(vals, k + u * L), S::xval(xd, c[u]), acc.part[u]);
            acc.end_round();
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int kk = k + u * L;
            if (kk < k1) {
                const int c = a.col_idx[kk];
                if (!valid || test_bit(bits, c)) acc.part[u] = S::fma(S::val(vals, kk), S::xval(xd, c), acc.part[u]);
            }
        }
        const typename S::Acc sum = group_reduce<DT, L>(acc.total());
        if (lane == 0) y[row] = S::out(sum);
    }
}

// Lane q's value, read into a scalar register (q uniform).
template <typename T>
__device__ __forceinline__ T lane_value(T v, int q) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, v), q));
    } else {
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)u, q);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(u >> 32), q);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Slab row `row` of a group (kSlots values), this lane's V slots (V
// consecutive values: one 4- or 8-byte load per lane). BUF: a buffer load with the row's byte
// offset in a scalar register and the lane's in a vector one (no 64-bit
// address per load); the group's slab is below 2 GiB then.
template <typename X, int V>
struct SlotVals {
    X v[V];
};

template <typename X, bool BUF, int V, int kSlots>
struct SlabRows {
    const X* base;  // the group's slab
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ SlabRows(const X* b, int64_t n) : base(b) {
        if constexpr (BUF)
            rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)b, (short)0, (int)(n * kSlots * (int64_t)sizeof(X)),
                                                     0x00020000);
    }
    __device__ __forceinline__ SlotVals<X, V> load(int row, int lane) const {
        static_assert(sizeof(X) * V == 4 || sizeof(X) * V == 8, "a lane loads 4 or 8 bytes");
        if constexpr (!BUF) {
            return *(const SlotVals<X, V>*)(base + (int64_t)row * kSlots + lane * V);
        } else if constexpr (sizeof(X) * V == 4) {
            return __builtin_bit_cast(SlotVals<X, V>, __builtin_amdgcn_raw_buffer_load_b32(
                                                          rsrc, lane * 4, row * (kSlots * (int)sizeof(X)), 0));
        } else {
            return __builtin_bit_cast(SlotVals<X, V>, __builtin_amdgcn_raw_buffer_load_b64(
                                                          rsrc, lane * 8, row * (kSlots * (int)sizeof(X)), 0));
        }
    }
};

constexpr int kStageRows = 16;  // rows of a fused unit staged in LDS before they are stored

// One work unit of A for the vectors of fused group g (at most 64 V of
// them; the group's slab rows hold kGroup x group_vpl slots): lane l holds
// slots V l .. V l + V - 1. The unit's entries stream 32 / V at a time (each a
// gather of the slab row X^T[col], V values per lane); a row's sums are
// staged when the stream passes its end, and every kStageRows / V rows the
// stage goes out as one run of consecutive rows per vector, not as 64 V
// scattered values per row. A piece of a split row adds its sums with
// atomics. st: the wave's kStageRows x 64 stage, sb: its 64 V vector ids
// (LDS).
template <int DT, bool BUF, int V>
__device__ __forceinline__ void batch_fused_unit(const BatchDev& a, int g, int32_t unit, typename SR<DT>::Acc* st,
                                                 int32_t* sb) {
    using S = SR<DT>;
    using X = typename S::X;
    using Acc = typename S::Acc;
    constexpr int SLOTS = kGroup * group_vpl<DT>();  // vectors per group, slots per slab row
    constexpr int GS = kGroup * V;                  // slots this walk covers
    constexpr int kRows = kStageRows / V;           // rows per stage
    constexpr int kPer = kWave / kRows;     // vectors per store of the stage
    const int4 u = a.units[unit];
    const int r0 = u.x, nrows = u.y - u.x, k0 = u.z, k1 = u.w;
    const int lane = lane_id();
    const int nvec = min(GS, *a.gcount - g * SLOTS);
    bool on[V];
    typename S::Y* y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int slot = lane * V + v;
        on[v] = slot < nvec;
        const int b = on[v] ? a.gvec[g * SLOTS + slot] : 0;
        y[v] = (typename S::Y*)a.Y + (int64_t)b * a.m;
        sb[slot] = b;
    }
    const SlabRows<X, BUF, V, SLOTS> xt((const X*)a.xt_all + (int64_t)g * a.n * SLOTS, a.n);
    const auto* vals = (const typename S::V*)a.vals;
    // lane i holds row_ptr[r0 + i], i <= nrows (nrows < 64)
    const int rp = lane <= nrows ? a.row_ptr[r0 + lane] : 0;
    const bool split = nrows == 1 && (k0 != lane_value(rp, 0) || k1 != lane_value(rp, 1));
    // rows [c0, c0 + cnt) of the stage to Y: lane = (row rr, vector t * kPer + lane / kRows)
    auto store_stage = [&](int c0, int cnt) {
        __builtin_amdgcn_wave_barrier();
        const int rr = lane & (kRows - 1);
#pragma unroll 4
        for (int t = 0; t < GS / kPer; ++t) {
            const int vs = t * kPer + lane / kRows;
            if (rr < cnt && vs < nvec)
                __builtin_nontemporal_store(S::out(st[rr * GS + vs]),
                                            (typename S::Y*)a.Y + (int64_t)sb[vs] * a.m + r0 + c0 + rr);
        }
        __builtin_amdgcn_wave_barrier();
    };
    Acc acc[V];
    auto flush = [&](int i) {
        if (split) {
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (on[v]) S::atomic_add(&y[v][r0 + i], acc[v]);
            return;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) st[(i & (kRows - 1)) * GS + lane * V + v] = acc[v];
        if ((i & (kRows - 1)) == kRows - 1) store_stage(i - (kRows - 1), kRows);
    };
    int i = 0;
    int end = lane_value(rp, 1);
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = S::zero();
    // kStep entries per step: lane q loads entry k + q (one coalesced load),
    // then all kStep slab rows are gathered before the first is used
    constexpr int kStep = 32 / V;
    for (int k = k0; k < k1; k += kStep) {
        const int kk = k + (lane & (kStep - 1));
        const bool in = kk < k1;
        // A streams through once per group: non-temporal, so that L2 keeps
        // the slab rows the gathers re-read
        const int cl = in ? __builtin_nontemporal_load(a.col_idx + kk) : 0;
        const typename S::V vl = in ? __builtin_nontemporal_load(vals + kk) : (typename S::V)0;
        // the step's slab rows into scalars first, with the whole wave
        // active; then only the group's lanes gather (a partial group moves
        // only its own bytes)
        int row[kStep];
#pragma unroll
        for (int q = 0; q < kStep; ++q) row[q] = lane_value(cl, q);
        SlotVals<X, V> xv[kStep];
        if (on[0]) {
#pragma unroll
            for (int q = 0; q < kStep; ++q) xv[q] = xt.load(row[q], lane);
        } else {
#pragma unroll
            for (int q = 0; q < kStep; ++q)
#pragma unroll
                for (int v = 0; v < V; ++v) xv[q].v[v] = (X)0;
        }
#pragma unroll
        for (int q = 0; q < kStep; ++q) {
            if (k + q >= k1) break;
            while (k + q >= end) {
                flush(i);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = S::zero();
                ++i;
                end = lane_value(rp, i + 1);
            }
            const typename S::V aq = lane_value(vl, q);
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = S::fma(aq, xv[q].v[v], acc[v]);
        }
    }
    for (; i < nrows; ++i) {
        flush(i);
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = S::zero();
    }
    if (!split && (nrows & (kRows - 1))) store_stage(nrows & ~(kRows - 1), nrows & (kRows - 1));
    __builtin_amdgcn_wave_barrier();
}

// The fused groups' work: item = group x unit, a wave per item, popped in
// order from a queue of its own (the kernel runs beside the phase-B tiles,
// so its workgroups become resident as the tiles' leave; every wave exits
// once the head passes the item count).
template <int DT, bool BUF, int V>
__global__ __launch_bounds__(kBlock) void k_batch_fused(BatchDev a) {
    if constexpr (DT != SPX_BOOL) {  // BOOL vectors never join a group
        using Acc = typename SR<DT>::Acc;
        constexpr int SLOTS = kGroup * group_vpl<DT>();
        __shared__ Acc s_stage[kWavesPerBlock][kStageRows * kGroup];
        __shared__ int32_t s_vec[kWavesPerBlock][kGroup * V];
        // groups of this walk: the two-wide one takes every group of more
        // than 64 vectors, the one-wide one the rest (a last partial group,
        // or all groups of 8-byte values); one kernel per width, so that
        // each has its own registers
        const int gcount = *a.gcount;
        const int64_t G = ceil_div(gcount, SLOTS);
        const int last = G > 0 ? gcount - (int)(G - 1) * SLOTS : 0;
        // groups 0 .. g_wide - 1 are wide
        const int64_t g_wide = (SLOTS > kGroup && G > 0) ? (last > kGroup ? G : G - 1) : 0;
        const int64_t g0 = V == 1 ? g_wide : 0;
        const int64_t ng = V == 1 ? G - g_wide : g_wide;
        const int64_t total = ng * a.nunits;
        if (total <= 0) return;  // nothing for this walk: no atomic on the head
        auto* head = (unsigned long long*)(a.queue + (V == 1 ? 6 : 4));
        for (;;) {
            unsigned long long got = 0;
            if (lane_id() == 0) got = atomicAdd(head, 1ull);
            // lane 0's value through scalar registers: the item (and so the
            // group's slab descriptor) is then known to be wave-uniform
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)got);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(got >> 32));
            const int64_t item = (int64_t)(((uint64_t)hi << 32) | lo);
            if (item >= total) break;
            batch_fused_unit<DT, BUF, V>(a, (int)(g0 + item / a.nunits), (int32_t)(item % a.nunits),
                                         s_stage[wave_id()], s_vec[wave_id()]);
        }
    }
}

template <int DT, int PH>
__global__ __launch_bounds__(kBlock) void k_batch_phase(BatchDev a) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    __shared__ BatchLds<DT> L;
    __shared__ int32_t s_item;
    // the phase's item offsets per vector, in LDS when they fit (the vector
    // of an item is found by a binary search over them)
    constexpr int kOffLds = 2048;
    __shared__ int32_t s_voff[kOffLds];
    const int32_t total = a.totals[PH];
    constexpr int ph = PH;
    const bool off_in_lds = a.B + 1 <= kOffLds;
    if (off_in_lds)
        for (int i = threadIdx.x; i <= a.B; i += kBlock) s_voff[i] = a.offs[ph * (a.B + 1) + i];
    const auto* vals = (const typename S::V*)a.vals;
    const auto* vals_csc = (const typename S::V*)a.vals_csc;
    const auto* xval_all = (const typename S::X*)a.val;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue + PH, 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int local = item;
        const int32_t* off = a.offs + ph * (a.B + 1);
        if (local >= off[a.B]) {
            // a fused group item (phase A: zero kSplitZeroRows split rows of
            // Y for the group's vectors)
            if constexpr (PH == 0) {
                const int gi = local - off[a.B];
                const int per = (int)ceil_div(a.nsplit, kSplitZeroRows);
                const int g = gi / per;
                const int s0 = (gi % per) * kSplitZeroRows;
                const int ns = min(kSplitZeroRows, a.nsplit - s0);
                const int gs = a.gsize;
                const int nvec = min(gs, *a.gcount - g * gs);
                for (int t = threadIdx.x; t < ns * nvec; t += kBlock) {
                    const int b = a.gvec[g * gs + t % nvec];
                    ((typename S::Y*)a.Y)[(int64_t)b * a.m + a.split_rows[s0 + t / nvec]] = (typename S::Y)0;
                }
            }
            continue;
        }
        const int b = find_vector(off_in_lds ? s_voff : off, a.B, local);
        const int j = local - off[b];
        const BatchPlan p = a.plans[b];
        auto* Yb = (typename S::Y*)a.Y + (int64_t)b * a.m;
        uint32_t* bits = a.bits_all + (int64_t)b * a.nwords;
        auto* xd = S::kVals ? (typename S::X*)a.xd_all + (int64_t)b * a.n : (typename S::X*)nullptr;
        const int32_t* idx = a.idx + p.base;
        const typename S::X* xv = S::kVals ? xval_all + p.base : nullptr;
        const bool csc = p.pattern == SPX_PAT_CSC_SPMSPV;
        if (p.gslot >= 0) {
            if constexpr (PH != 1) {
                if constexpr (S::kVals) {
                    // the chunk's kScatterChunk entries, eight per thread with
                    // every load of a step in flight before the stores
                    const int gs = a.gsize;
                    auto* xt = (typename S::X*)a.xt_all + (int64_t)(p.gslot / gs) * a.n * gs + p.gslot % gs;
                    const int e1 = std::min(p.nnz_x, (j + 1) * kScatterChunk);
                    constexpr int kPer = kScatterChunk / kBlock;
                    int c[kPer];
                    typename S::X v[kPer];
#pragma unroll
                    for (int q = 0; q < kPer; ++q) {
                        const int e = j * kScatterChunk + q * kBlock + threadIdx.x;
                        c[q] = e < e1 ? idx[e] : -1;
                        v[q] = (PH == 0 && e < e1) ? xv[e] : (typename S::X)0;
                    }
#pragma unroll
                    for (int q = 0; q < kPer; ++q)
                        if (c[q] >= 0) xt[(int64_t)c[q] * gs] = v[q];
                }
            }
            continue;
        }
        if constexpr (PH == 0) {
            if (csc) {
                const int64_t r0 = (int64_t)j * kFillChunk;
                const int64_t r1 = std::min<int64_t>(r0 + kFillChunk, a.m);
                for (int64_t r = r0 + threadIdx.x; r < r1; r += kBlock) Yb[r] = (typename S::Y)0;
            } else {
                const int e1 = std::min(p.nnz_x, (j + 1) * kScatterChunk);
                for (int e = j * kScatterChunk + threadIdx.x; e < e1; e += kBlock) {
                    const int c = idx[e];
                    atomicOr(&bits[c >> 5], 1u << (c & 31));
                    if constexpr (S::kVals) xd[c] = xv[e];
                }
            }
        } else if constexpr (PH == 1) {
            if (csc) {
                const int32_t* excl = a.excl_all + p.base + b;
                if (p.dist == SPX_DIST_BALANCED) {
                    csc_merge_tile<DT>(j, p.nnz_x, p.nnz_s, idx, xv, a.col_ptr, a.row_idx, vals_csc, Excl{excl, nullptr},
                                       EmitAtomic<DT>{Yb}, L.csc);
                } else {
                    const int e = j * kCscDirectEntries + threadIdx.x / kCscDirectLanes;
                    if (e < p.nnz_x)
                        csc_direct_entry<DT, kCscDirectLanes>(e, threadIdx.x % kCscDirectLanes, idx, xv, a.col_ptr,
                                                              a.row_idx, vals_csc, Excl{nullptr, nullptr},
                                                              EmitAtomic<DT>{Yb});
                }
            } else {
                const bool valid = p.pattern == SPX_PAT_CSR_SPMSPV || DT == SPX_BOOL;
                if (p.dist == SPX_DIST_BALANCED) {
                    int32_t* crow = a.carry_row_all + (int64_t)b * a.tiles_mat;
                    Acc* cval = (Acc*)a.carry_val_all + (int64_t)b * a.tiles_mat;
                    if (valid)
                        csr_merge_tile<DT, true, kBatchTile>(j, a.m, a.row_ptr, a.col_idx, vals, xd, bits, Yb, a.part,
                                                             crow, cval, L.csr);
                    else
                        csr_merge_tile<DT, false, kBatchTile>(j, a.m, a.row_ptr, a.col_idx, vals, xd, bits, Yb, a.part,
                                                              crow, cval, L.csr);
                } else {
                    const int64_t rpi = (int64_t)(kBlock / p.lanes) * 8;
                    const int64_t r0 = (int64_t)j * rpi, r1 = std::min<int64_t>(r0 + rpi, a.m);
                    switch (p.lanes) {
                        case 1: batch_rows_direct<DT, 1>(a, r0, r1, valid, xd, bits, Yb); break;
                        case 2: batch_rows_direct<DT, 2>(a, r0, r1, valid, xd, bits, Yb); break;
                        case 4: batch_rows_direct<DT, 4>(a, r0, r1, valid, xd, bits, Yb); break;
                        case 8: batch_rows_direct<DT, 8>(a, r0, r1, valid, xd, bits, Yb); break;
                        case 16: batch_rows_direct<DT, 16>(a, r0, r1, valid, xd, bits, Yb); break;
                        case 32: batch_rows_direct<DT, 32>(a, r0, r1, valid, xd, bits, Yb); break;
                        default: batch_rows_direct<DT, 64>(a, r0, r1, valid, xd, bits, Yb); break;
                    }
                }
            }
        } else {
            int jj = j;
            if (p.dist == SPX_DIST_BALANCED) {
                if (jj == 0) {
                    csr_merge_fixup_range<DT>(threadIdx.x, kBlock, a.tiles_mat, a.carry_row_all + (int64_t)b * a.tiles_mat,
                                              (const Acc*)a.carry_val_all + (int64_t)b * a.tiles_mat, Yb);
                }
                --jj;
            }
            if (jj >= 0) {
                const int e1 = std::min(p.nnz_x, (jj + 1) * kScatterChunk);
                for (int e = jj * kScatterChunk + threadIdx.x; e < e1; e += kBlock) {
                    const int c = idx[e];
                    bits[c >> 5] = 0u;
                    if constexpr (S::kVals) xd[c] = (typename S::X)0;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ host side
static void batch_layout(int32_t m, int32_t n, int dtype, int32_t B, int64_t cap_nnz_x, int64_t tiles_mat,
                         BatchDev* d, char* base, size_t* bytes) {
    Sizer z;
    size_t off[16];
    int k = 0;
    auto take = [&](size_t n_bytes) {
        z.used = align_up(z.used, 256);
        off[k++] = z.used;
        z.used += align_up(n_bytes, 256);
    };
    const int vs = std::max(1, value_size(dtype));
    const int as = dtype == SPX_F64 ? 8 : 4;
    const int64_t nwords = ceil_div(n, 32) + 1;
    take(sizeof(BatchPlan) * (size_t)B);                 // 0 plans
    take(4 * (size_t)3 * (B + 1));                       // 1 offs
    take(4 * 4);                                          // 2 totals
    take(4 * 8);                                          // 3 queue heads, err, two fused walk heads
    take(4);                                              // 4 group count
    take(4 * (size_t)(cap_nnz_x + B));                    // 5 excl
    take(4 * (size_t)B * nwords);                         // 6 bits (self-cleaning)
    take((size_t)vs * B * (size_t)n);                     // 7 xd (self-cleaning)
    take(4 * (size_t)B * tiles_mat);                      // 8 carry rows
    take((size_t)as * B * tiles_mat);                     // 9 carry values
    take(4 * (size_t)B);                                  // 10 group slot -> vector
    const int64_t gsize = (int64_t)kGroup * (vs == 4 ? 2 : 1);
    take((size_t)vs * ceil_div(B, gsize) * gsize * (size_t)n);  // 11 group slabs (self-cleaning)
    *bytes = z.used;
    if (!d || !base) return;
    d->plans = (BatchPlan*)(base + off[0]);
    d->offs = (int32_t*)(base + off[1]);
    d->totals = (int32_t*)(base + off[2]);
    d->queue = (int32_t*)(base + off[3]);
    d->err = d->queue + 3;
    d->excl_all = (int32_t*)(base + off[5]);
    d->bits_all = (uint32_t*)(base + off[6]);
    d->xd_all = base + off[7];
    d->carry_row_all = (int32_t*)(base + off[8]);
    d->carry_val_all = base + off[9];
    d->nwords = nwords;
    d->gcount = (int32_t*)(base + off[4]);
    d->gvec = (int32_t*)(base + off[10]);
    d->xt_all = base + off[11];
    d->gsize = (int32_t)gsize;
}

size_t batch_ws_size(int32_t m, int32_t n, int dtype, int32_t B, int64_t cap_nnz_x, int64_t tiles_mat,
                     size_t* zero_from, size_t* zero_bytes) {
    size_t bytes = 0;
    batch_layout(m, n, dtype, B, cap_nnz_x, tiles_mat, nullptr, nullptr, &bytes);
    // the whole workspace is zeroed at allocation; only the bitvector and
    // value slots rely on it (they are self-cleaning afterwards)
    if (zero_from) *zero_from = 0;
    if (zero_bytes) *zero_bytes = bytes;
    return bytes;
}

spx_status launch_batch(const BatchLaunch& L, void* ws, size_t ws_bytes, hipStream_t s, int32_t** err_dev) {
    BatchDev d{};
    d.m = L.csr.m;
    d.n = L.csr.n;
    d.nnz = L.csr.nnz;
    d.row_ptr = L.csr.row_ptr;
    d.col_idx = L.csr.col_idx;
    d.vals = L.csr.vals;
    d.col_ptr = L.col_ptr;
    d.row_idx = L.row_idx;
    d.vals_csc = L.vals_csc;
    d.part = L.part;
    d.tiles_mat = L.tiles_mat;
    d.B = L.B;
    d.cap_nnz_x = L.cap_nnz_x;
    d.vec_ptr = L.vec_ptr;
    d.idx = L.idx;
    d.val = L.val;
    d.Y = L.Y;
    d.sel = L.sel;
    d.row_lanes = L.row_lanes;
    d.units = (const int4*)L.units;
    d.nunits = L.nunits;
    d.split_rows = L.split_rows;
    d.nsplit = L.nsplit;
    size_t need = 0;
    batch_layout(d.m, d.n, L.csr.dtype, L.B, L.cap_nnz_x, L.tiles_mat, &d, (char*)ws, &need);
    if (need > ws_bytes) return fail(SPX_ERR_WORKSPACE, "run_batch: workspace too small");
    if (err_dev) *err_dev = d.err;
    if (L.B == 0) return SPX_OK;
    // a group's slab addressed by 32-bit buffer offsets when it fits
    const int vsz = std::max(1, value_size(L.csr.dtype));
    const bool slab_buf = (int64_t)d.n * d.gsize * vsz < ((int64_t)1 << 31);
    // the fused walk's items are dealt out by a grid stride, so its grid is
    // what stays resident at once (no late workgroup forms a tail)
    auto resident = [&](const void* fn) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        return (unsigned)std::max(1, L.persistent_grid / 4) * (unsigned)per_cu;
    };
    unsigned fused_grid = 1, fused_grid2 = 1;
    const bool fused = L.csr.dtype != SPX_BOOL && d.units && d.nunits > 0;
    const bool branch = L.side && L.fork && L.join;
    hipStream_t fs = branch ? L.side : s;
    switch (L.csr.dtype) {
#define SPX_DT(DT)                                                                                      \
    case DT:                                                                                            \
        fused_grid = slab_buf ? resident((const void*)k_batch_fused<DT, true, 1>)                       \
                              : resident((const void*)k_batch_fused<DT, false, 1>);                     \
        fused_grid2 = slab_buf ? resident((const void*)k_batch_fused<DT, true, group_vpl<DT>()>)        \
                               : resident((const void*)k_batch_fused<DT, false, group_vpl<DT>()>);      \
        break;
        SPX_DT(SPX_F32)
        SPX_DT(SPX_F64)
        SPX_DT(SPX_I32)
#undef SPX_DT
        default:
            break;
    }
    switch (L.csr.dtype) {
#define SPX_DT(DT)                                                            \
    case DT:                                                                  \
        k_batch_reset<<<1, 1, 0, s>>>(d.err, d.gcount);                       \
        k_batch_plan<DT><<<L.B, kBlock, 0, s>>>(d);                           \
        k_batch_scan<<<1, kBlock, 0, s>>>(d);                                 \
        k_batch_phase<DT, 0><<<L.persistent_grid, kBlock, 0, s>>>(d);         \
        if (fused) {                                                          \
            if (branch) {                                                     \
                SPX_HIP(hipEventRecord(L.fork, s));                           \
                SPX_HIP(hipStreamWaitEvent(L.side, L.fork, 0));               \
            }                                                                 \
            if (slab_buf) {                                                   \
                k_batch_fused<DT, true, 1><<<fused_grid, kBlock, 0, fs>>>(d); \
                if (d.gsize > kGroup)                                         \
                    k_batch_fused<DT, true, group_vpl<DT>()><<<fused_grid2, kBlock, 0, fs>>>(d); \
            } else {                                                          \
                k_batch_fused<DT, false, 1><<<fused_grid, kBlock, 0, fs>>>(d); \
                if (d.gsize > kGroup)                                         \
                    k_batch_fused<DT, false, group_vpl<DT>()><<<fused_grid2, kBlock, 0, fs>>>(d); \
            }                                                                 \
            if (branch) SPX_HIP(hipEventRecord(L.join, L.side));              \
        }                                                                     \
        k_batch_phase<DT, 1><<<L.persistent_grid, kBlock, 0, s>>>(d);         \
        if (fused && branch) SPX_HIP(hipStreamWaitEvent(s, L.join, 0));       \
        k_batch_phase<DT, 2><<<L.persistent_grid, kBlock, 0, s>>>(d);         \
        break;
        SPX_DT(SPX_F32)
        SPX_DT(SPX_F64)
        SPX_DT(SPX_I32)
        SPX_DT(SPX_BOOL)
#undef SPX_DT
        default:
            return fail(SPX_ERR_DTYPE, "run_batch: dtype");
    }
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

void upload_tree(const Tree& t, DevTree* out) {
    const int n = std::min<int>((int)t.cls.size(), kDevTreeNodes);
    out->n = n;
    for (int i = 0; i < n; ++i) {
        out->feat[i] = t.feat[i];
        out->thr[i] = t.thr[i];
        out->left[i] = t.left[i];
        out->right[i] = t.right[i];
        out->cls[i] = t.cls[i];
    }
}

}  // namespace spx
