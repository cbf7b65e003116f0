// C ABI of libspx: argument checks, the matrix handle (dual CSR + CSC
// storage, Section 6.1), lazy feature evaluation and the decision-tree
// cascade (Section 6.2-6.3), vector conversion on demand, and dispatch to
// the candidate kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "selector.hpp"

#define SPX_VERSION "spx 0.1 (gfx950)"

namespace spx {

static thread_local std::string g_err = "no error";

spx_status fail(spx_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

spx_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
    return SPX_ERR_HIP;
}

int value_size(int dtype) {
    switch (dtype) {
        case SPX_F32:
        case SPX_I32:
        case SPX_F32_MINPLUS:
            return 4;
        case SPX_F64:
            return 8;
        default:
            return 0;
    }
}

int out_size(int dtype) {
    switch (dtype) {
        case SPX_F32:
        case SPX_I32:
        case SPX_F32_MINPLUS:
            return 4;
        case SPX_F64:
            return 8;
        case SPX_BOOL:
            return 1;
        default:
            return 0;
    }
}

static bool valid_dtype(int dt) {
    return dt == SPX_F32 || dt == SPX_F64 || dt == SPX_I32 || dt == SPX_BOOL || dt == SPX_F32_MINPLUS;
}

// 32-bit word of the semiring's zero (the fill of a y that atomics update,
// and of an x that absent entries leave unwritten)
uint32_t zero_word(int dtype) { return dtype == SPX_F32_MINPLUS ? 0x7f800000u : 0u; }

static int key_bits_for(int32_t n) {
    int b = 0;
    while (b < 31 && (int64_t(1) << b) < n) ++b;
    return std::max(b, 1);
}

// ------------------------------------------------------------------ small kernels
__global__ __launch_bounds__(kBlock) void k_iota(uint32_t* __restrict__ p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * kBlock;
    for (; i < n; i += stride) p[i] = (uint32_t)i;
}

// col_ptr from column ids sorted ascending: position p starts every column
// in (key[p-1], key[p]].
__global__ __launch_bounds__(kBlock) void k_ptr_from_sorted(const uint32_t* __restrict__ keys, int64_t nnz,
                                                            int32_t n, int32_t* __restrict__ ptr) {
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p > nnz) return;
    const int64_t prev = p > 0 ? (int64_t)keys[p - 1] : -1;
    const int64_t cur = p < nnz ? (int64_t)keys[p] : (int64_t)n;
    for (int64_t j = prev + 1; j <= cur; ++j) ptr[j] = (int32_t)p;
}

// validation: row_ptr monotone with row_ptr[0] = 0 and row_ptr[m] = nnz,
// col_idx in range; sets bit 0 / bit 1 of *bad
__global__ __launch_bounds__(kBlock) void k_validate_csr(const int32_t* __restrict__ row_ptr, int32_t m,
                                                         const int32_t* __restrict__ col_idx, int32_t nnz,
                                                         int32_t n, uint32_t* __restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= m; i += stride) {
        const int32_t v = row_ptr[i];
        if ((i == 0 && v != 0) || (i == m && v != nnz) || (i > 0 && v < row_ptr[i - 1]) || v < 0 || v > nnz)
            atomicOr(bad, 1u);
    }
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz; k += stride) {
        const int32_t c = col_idx[k];
        if (c < 0 || c >= n) atomicOr(bad, 2u);
    }
}

// Entries of A listed column by column in rank order (rows ascending within
// a column): key = row, value = CSR position. rq[q] is the rank owning
// position q of that listing, gptr the prefix of column lengths by rank.
__global__ __launch_bounds__(kBlock) void k_rank_major(int64_t nnz, const int32_t* __restrict__ rq,
                                                       const int32_t* __restrict__ gptr,
                                                       const int32_t* __restrict__ gorder,
                                                       const int32_t* __restrict__ col_ptr,
                                                       const int32_t* __restrict__ row_idx,
                                                       const int32_t* __restrict__ perm,
                                                       uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < nnz; q += stride) {
        const int r = rq[q];
        const int64_t p = col_ptr[gorder[r]] + (q - gptr[r]);
        keys[q] = (uint32_t)row_idx[p];
        vals[q] = (uint32_t)perm[p];
    }
}

__global__ __launch_bounds__(kBlock) void k_renumber_cols(int64_t nnz, const int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ col_idx,
                                                          const int32_t* __restrict__ grank,
                                                          int32_t* __restrict__ gcol) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz; k += stride) gcol[k] = grank[col_idx[src[k]]];
}

// dense x -> bitvector of its nonzeros (x != 0): one element per lane
// (coalesced), the wave's ballot is its two words
template <int DT>
__global__ __launch_bounds__(kBlock) void k_dense_bits(int32_t n, const typename SR<DT>::X* __restrict__ x,
                                                       uint32_t* __restrict__ bits) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool nz = j < n && SR<DT>::present(x[j]);
    const uint64_t b = __ballot(nz);
    const int64_t j0 = j - lane_id();  // first element of the wave, a multiple of 64
    if (lane_id() == 0 && j0 < n) {
        bits[j0 >> 5] = (uint32_t)b;
        if (j0 + 32 < n) bits[(j0 >> 5) + 1] = (uint32_t)(b >> 32);
    }
}

static unsigned dense_bits_grid(int32_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kBlock)); }

}  // namespace spx

using namespace spx;

// ------------------------------------------------------------------ handle
struct spx_matrix {
    spx_csr csr{};  // borrowed arrays
    int device = 0;
    int32_t* col_ptr = nullptr;
    int32_t* row_idx = nullptr;
    int32_t* perm = nullptr;  // CSC position -> CSR position
    void* vals_csc = nullptr;
    // column renumbering of the row-major kernels (null when not used):
    // gorder[r] = original column of rank r, grank its inverse; gcsr is A
    // with renumbered columns (rows unchanged, entries of a row by rank),
    // gsrc[k] the CSR position of its entry k
    int32_t* gorder = nullptr;
    int32_t* grank = nullptr;
    int32_t* gcol = nullptr;
    int32_t* gsrc = nullptr;
    void* gvals = nullptr;
    spx_csr gcsr{};
    double feat[9] = {0};
    Selector sel;
    // conversion buffers (allocated on first use). *_clean: the buffer is
    // known to hold zeros (the semiring's zero for xd) once the work queued
    // so far has run, because the last balanced row-major product cleared
    // what its conversion scattered; the next sparse conversion then skips
    // its fill. Calls on one handle are ordered on one stream.
    uint32_t* bits = nullptr;
    void* xd = nullptr;
    bool bits_clean = false;
    bool xd_clean = false;
    // sliced ELLPACK copy of the row-major CSR (the renumbered one when
    // there is one), used by the SpMV pattern when present
    SellMat sell;
    double sell_ratio = 0.0;
    EllMat ell;
    DiaMat dia;
    Csr5Mat c5;
    // column-sorted copy of the renumbered CSR for the balanced SpMV with
    // 2048-item tiles (kept with the renumbered copy when n <= 2^21)
    TileSorted ts;
    int32_t* sp_idx = nullptr;
    void* sp_val = nullptr;
    int32_t* scratch_i32 = nullptr;  // compaction workspace
    int64_t* dev_scalars = nullptr;  // 4 x int64 (feature reductions, counts)
    // lazy counts of run(): two device counters and a ticket (zero between
    // calls) and the pinned host copy the counting kernel writes
    unsigned long long* cnt_dev = nullptr;
    long long* cnt_host = nullptr;
    uint32_t* scan_counter = nullptr;  // arrival counter of the one-launch length scan
    // merge-path partitions of the balanced row-major kernels, per tile size,
    // for A (index 0) and for A^T (index 1)
    int32_t* part[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    void* ws = nullptr;
    size_t ws_bytes = 0;
    spx_plan last_plan{};
    // batched path: device copy of the trees, workspace, captured graph
    DevSelector* dev_sel = nullptr;
    void* bws = nullptr;
    size_t bws_bytes = 0;
    int32_t bcap_B = 0;
    int64_t bcap_nnz = 0;
    int32_t* berr = nullptr;
    int32_t* units = nullptr;  // fused-group work units of A (4 ints each)
    int32_t nunits = 0;
    int32_t* split_rows = nullptr;
    int32_t nsplit = 0;
    // breadth-first search buffers (allocated on first use)
    int32_t* bfs_front[2] = {nullptr, nullptr};
    uint8_t* bfs_y = nullptr;
    int32_t* drv_count = nullptr;     // two packed counters of the graph drivers
    uint32_t* bfs_bits[2] = {nullptr, nullptr};
    int32_t* drv_host = nullptr;      // pinned copies of the counters (two slots of 16 bytes)
    hipEvent_t drv_ev[2] = {nullptr, nullptr};
    // trees for callers that know nnz_s without a device round trip (the
    // graph drivers); the host-feature trees otherwise
    Selector sel_known;
    bool has_sel_known = false;
    // lazy trees of run() and select_kernel() (they may test nnz_s at a
    // device round trip); the host-feature trees otherwise
    Selector sel_run;
    bool has_sel_run = false;
    // incremental PageRank: column sums (valid for the current values),
    // residual, product, sparse input, negative-weight flag
    void* pr_W = nullptr;
    void* pr_r = nullptr;
    void* pr_y = nullptr;
    int32_t* pr_xidx = nullptr;
    void* pr_xval = nullptr;
    void* pr_xd[2] = {nullptr, nullptr};
    void* pr_p = nullptr;  // rank, copied to the caller's array at the end
    uint32_t* pr_bad = nullptr;
    bool pr_W_valid = false;
    hipStream_t cap_stream = nullptr;
    hipStream_t cap_side = nullptr;  // a second branch of the captured graph (the fused walk)
    hipEvent_t cap_fork = nullptr, cap_join = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void* gkey[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    int32_t gkey_B = -1;
    // profiling
    int profiling = 0;
    double host_ms[2] = {0, 0};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_conv, ev_kern;
};

static spx_status ensure_ws(spx_matrix* H, size_t bytes) {
    if (bytes <= H->ws_bytes) return SPX_OK;
    if (H->ws) SPX_HIP(hipFree(H->ws));
    H->ws = nullptr;
    H->ws_bytes = 0;
    const size_t b = align_up(bytes, 1 << 20);
    if (hipMalloc(&H->ws, b) != hipSuccess) return fail(SPX_ERR_ALLOC, "workspace allocation failed");
    H->ws_bytes = b;
    return SPX_OK;
}

// Cached merge-path partition of the balanced row-major kernels.
static spx_status cached_part(spx_matrix* H, const spx_csr& A, int which, const spx_plan* p, hipStream_t s,
                              const int32_t** out) {
    *out = nullptr;
    if (p->distribution != SPX_DIST_BALANCED) return SPX_OK;
    const int tile = p->tile == 4096 ? 4096 : 2048;
    const int ti = tile == 4096 ? 1 : 0;
    if (!H->part[which][ti]) {
        const int64_t tiles = ceil_div((int64_t)A.m + A.nnz, tile);
        if (hipMalloc((void**)&H->part[which][ti], (size_t)(2 * (tiles + 1)) * 4) != hipSuccess)
            return fail(SPX_ERR_ALLOC, "partition allocation failed");
        SPX_TRY(merge_partition(A.m, A.nnz, A.row_ptr, tile, H->part[which][ti], s));
    }
    *out = H->part[which][ti];
    return SPX_OK;
}

static spx_status ensure_conv(spx_matrix* H) {
    if (H->dev_scalars) return SPX_OK;
    const int32_t n = H->csr.n;
    const size_t vs = std::max(1, value_size(H->csr.dtype));
    if (hipMalloc((void**)&H->bits, align_up((size_t)ceil_div(n, 32) * 4 + 4, 256)) != hipSuccess ||
        hipMalloc(&H->xd, align_up((size_t)n * vs + 8, 256)) != hipSuccess ||
        hipMalloc((void**)&H->sp_idx, align_up((size_t)n * 4 + 4, 256)) != hipSuccess ||
        hipMalloc(&H->sp_val, align_up((size_t)n * vs + 8, 256)) != hipSuccess ||
        hipMalloc((void**)&H->scratch_i32, compact_ws_elems(n) * 4 + 256) != hipSuccess ||
        hipMalloc((void**)&H->dev_scalars, 64) != hipSuccess)
        return fail(SPX_ERR_ALLOC, "conversion buffers: allocation failed");
    return SPX_OK;
}

static spx_csc handle_csc(const spx_matrix* H) {
    spx_csc c;
    c.m = H->csr.m;
    c.n = H->csr.n;
    c.nnz = H->csr.nnz;
    c.dtype = H->csr.dtype;
    c.col_ptr = H->col_ptr;
    c.row_idx = H->row_idx;
    c.vals = H->vals_csc;
    return c;
}

// The trees of a caller that knows nnz_s.
static const Selector& known_selector(const spx_matrix* H) { return H->has_sel_known ? H->sel_known : H->sel; }
// The trees of run() and select_kernel().
static const Selector& run_selector(const spx_matrix* H) { return H->has_sel_run ? H->sel_run : H->sel; }

// run_batch evaluates the host-feature trees on the device: with them a
// vector whose plan is row-major joins a fused group before any prefix of
// its column lengths is computed (trees that read nnz_s would need that
// prefix for every vector, which measured slower on the 512-vector batch).
static spx_status upload_selector(spx_matrix* H) {
    if (!H->dev_sel && hipMalloc((void**)&H->dev_sel, sizeof(DevSelector)) != hipSuccess)
        return fail(SPX_ERR_ALLOC, "device selector allocation failed");
    DevSelector* h = new (std::nothrow) DevSelector();
    if (!h) return fail(SPX_ERR_ALLOC, "selector staging");
    const Selector& S = H->sel;
    upload_tree(S.pattern, &h->t[0]);
    for (int p = 0; p < 3; ++p) upload_tree(S.distribution[p], &h->t[1 + p]);
    upload_tree(S.writeback, &h->t[4]);
    for (int i = 0; i < 9; ++i) h->mfeat[i] = H->feat[i];
    h->needs_nnz_s = S.reads_nnz_s() ? 1 : 0;
    hipError_t e = hipMemcpy(H->dev_sel, h, sizeof(DevSelector), hipMemcpyHostToDevice);
    delete h;
    if (e != hipSuccess) return hip_fail(e, "upload selector");
    return SPX_OK;
}

static Selector& global_selector() {
    static Selector s = builtin_selector();
    return s;
}

// Default trees that read nnz_s (first = loaded).
static std::pair<bool, Selector>& global_selector_known() {
    static std::pair<bool, Selector> s{false, Selector{}};
    return s;
}

// Default lazy trees of run() (first = loaded).
static std::pair<bool, Selector>& global_selector_run() {
    static std::pair<bool, Selector> s{false, Selector{}};
    return s;
}

// ------------------------------------------------------------------ checks
extern "C" spx_status spx_check_csr(const spx_csr* A) {
    if (!A) return fail(SPX_ERR_ARG, "matrix descriptor is null");
    if (!valid_dtype(A->dtype)) return fail(SPX_ERR_DTYPE, "unknown dtype");
    if (A->m < 0 || A->n < 0 || A->nnz < 0) return fail(SPX_ERR_SHAPE, "negative matrix size");
    if (!A->row_ptr) return fail(SPX_ERR_ARG, "row_ptr is null");
    if (A->nnz > 0 && !A->col_idx) return fail(SPX_ERR_ARG, "col_idx is null");
    if (A->nnz > 0 && A->dtype != SPX_BOOL && !A->vals) return fail(SPX_ERR_ARG, "vals is null");
    return SPX_OK;
}

spx_status spx::check_csc(const spx_csc* A) {
    if (!A) return fail(SPX_ERR_ARG, "matrix descriptor is null");
    if (!valid_dtype(A->dtype)) return fail(SPX_ERR_DTYPE, "unknown dtype");
    if (A->m < 0 || A->n < 0 || A->nnz < 0) return fail(SPX_ERR_SHAPE, "negative matrix size");
    if (!A->col_ptr) return fail(SPX_ERR_ARG, "col_ptr is null");
    if (A->nnz > 0 && !A->row_idx) return fail(SPX_ERR_ARG, "row_idx is null");
    if (A->nnz > 0 && A->dtype != SPX_BOOL && !A->vals) return fail(SPX_ERR_ARG, "vals is null");
    return SPX_OK;
}

extern "C" spx_status spx_check_plan(const spx_plan* p, int32_t dtype) {
    if (!p) return fail(SPX_ERR_ARG, "plan is null");
    if (!valid_dtype(dtype)) return fail(SPX_ERR_DTYPE, "unknown dtype");
    if (p->pattern < SPX_PAT_SPMV || p->pattern > SPX_PAT_CSC_SPMSPV) return fail(SPX_ERR_ARG, "bad pattern");
    if (p->distribution != SPX_DIST_DIRECT && p->distribution != SPX_DIST_BALANCED)
        return fail(SPX_ERR_ARG, "bad distribution");
    if (p->pattern == SPX_PAT_CSC_SPMSPV) {
        if (p->writeback < SPX_WB_ATOMIC || p->writeback > SPX_WB_MERGE)
            return fail(SPX_ERR_ARG, "column-major pattern needs a write-back");
    } else if (p->writeback != SPX_WB_NONE) {
        return fail(SPX_ERR_ARG, "row-major patterns take no write-back");
    }
    if (p->lanes != 0 && (p->lanes < 1 || p->lanes > 64 || (p->lanes & (p->lanes - 1))))
        return fail(SPX_ERR_ARG, "lanes must be 0 or a power of two in [1, 64]");
    if (p->bucket_rows != 0 && (p->bucket_rows < 64 || (p->bucket_rows & (p->bucket_rows - 1))))
        return fail(SPX_ERR_ARG, "bucket_rows must be 0 or a power of two >= 64");
    return SPX_OK;
}

extern "C" const char* spx_last_error(void) { return g_err.c_str(); }
extern "C" const char* spx_version(void) { return SPX_VERSION; }

// ------------------------------------------------------------------ workspace
static size_t ws_for(int32_t m, int32_t n, int32_t nnz, int32_t nnz_x, int32_t dtype, const spx_plan* p) {
    size_t b = 0;
    if (p->pattern == SPX_PAT_CSC_SPMSPV) {
        b = spmspv_csc_ws(m, n, nnz, nnz_x, dtype, p);
    } else {
        b = spmv_csr_ws(m, nnz, p);
        if (p->pattern == SPX_PAT_CSR_SPMSPV) {
            Sizer z;
            z.used = b;
            z.take<uint32_t>((size_t)ceil_div(n, 32) + 1);
            z.take<uint64_t>((size_t)n + 1);
            b = z.used;
        }
    }
    return b;
}

extern "C" size_t spx_workspace_size(int32_t m, int32_t n, int32_t nnz, int32_t nnz_x_max, int32_t dtype,
                                     const spx_plan* plan) {
    if (!plan || spx_check_plan(plan, dtype) != SPX_OK || m < 0 || n < 0 || nnz < 0 || nnz_x_max < 0) return 0;
    return ws_for(m, n, nnz, nnz_x_max, dtype, plan);
}

// ------------------------------------------------------------------ kernels by plan
extern "C" spx_status spmv_csr(const spx_csr* A, const void* x, void* y, const spx_plan* plan, void* workspace,
                               size_t ws_bytes, void* stream) {
    SPX_TRY(spx_check_csr(A));
    SPX_TRY(spx_check_plan(plan, A->dtype));
    if (plan->pattern != SPX_PAT_SPMV) return fail(SPX_ERR_ARG, "spmv_csr needs pattern SPX_PAT_SPMV");
    if ((A->n > 0 && !x) || (A->m > 0 && !y)) return fail(SPX_ERR_ARG, "x or y is null");
    Arena ws(workspace, ws_bytes);
    return launch_spmv_csr(A, x, nullptr, y, plan, nullptr, ws, (hipStream_t)stream);
}

extern "C" spx_status spmspv_csr(const spx_csr* A, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                                 void* y, const spx_plan* plan, void* workspace, size_t ws_bytes, void* stream) {
    SPX_TRY(spx_check_csr(A));
    SPX_TRY(spx_check_plan(plan, A->dtype));
    if (plan->pattern != SPX_PAT_CSR_SPMSPV) return fail(SPX_ERR_ARG, "spmspv_csr needs pattern SPX_PAT_CSR_SPMSPV");
    if (nnz_x < 0 || nnz_x > A->n) return fail(SPX_ERR_SHAPE, "nnz_x must be in [0, n]");
    if (nnz_x > 0 && (!x_idx || (A->dtype != SPX_BOOL && !x_val))) return fail(SPX_ERR_ARG, "x arrays are null");
    if (A->m > 0 && !y) return fail(SPX_ERR_ARG, "y is null");
    hipStream_t s = (hipStream_t)stream;
    Arena ws(workspace, ws_bytes);
    // the kernel's own workspace first, conversion buffers after it
    Arena probe = ws;
    const size_t kern = spmv_csr_ws(A->m, A->nnz, plan);
    probe.used = kern;
    uint32_t* bits = probe.take<uint32_t>((size_t)ceil_div(A->n, 32) + 1);
    void* xd = probe.take<uint64_t>((size_t)A->n + 1);
    if (!bits || !xd) return fail(SPX_ERR_WORKSPACE, "spmspv_csr: workspace too small");
    SPX_TRY(sparse_to_bitvector(A->n, nnz_x, x_idx, x_val, A->dtype, nullptr, bits,
                                A->dtype == SPX_BOOL ? nullptr : xd, s));
    return launch_spmv_csr(A, A->dtype == SPX_BOOL ? nullptr : xd, bits, y, plan, nullptr, ws, s);
}

extern "C" spx_status spmspv_csc(const spx_csc* A, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                                 void* y, const spx_plan* plan, void* workspace, size_t ws_bytes, void* stream) {
    SPX_TRY(check_csc(A));
    SPX_TRY(spx_check_plan(plan, A->dtype));
    if (plan->pattern != SPX_PAT_CSC_SPMSPV) return fail(SPX_ERR_ARG, "spmspv_csc needs pattern SPX_PAT_CSC_SPMSPV");
    if (nnz_x < 0 || nnz_x > A->n) return fail(SPX_ERR_SHAPE, "nnz_x must be in [0, n]");
    if (nnz_x > 0 && (!x_idx || (A->dtype != SPX_BOOL && !x_val))) return fail(SPX_ERR_ARG, "x arrays are null");
    if (A->m > 0 && !y) return fail(SPX_ERR_ARG, "y is null");
    CscArgs a{A->m, A->n, A->nnz, A->dtype, A->col_ptr, A->row_idx, A->vals, nullptr, nullptr, -1};
    Arena ws(workspace, ws_bytes);
    return launch_spmspv_csc(a, nnz_x, x_idx, x_val, y, plan, ws, (hipStream_t)stream);
}

// ------------------------------------------------------------------ handle
extern "C" spx_status spx_matrix_destroy(spx_matrix* H) {
    if (!H) return SPX_OK;
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(H->device);
    if (H->gexec) hipGraphExecDestroy(H->gexec);
    if (H->graph) hipGraphDestroy(H->graph);
    if (H->cap_stream) hipStreamDestroy(H->cap_stream);
    if (H->cap_side) hipStreamDestroy(H->cap_side);
    if (H->cap_fork) hipEventDestroy(H->cap_fork);
    if (H->cap_join) hipEventDestroy(H->cap_join);
    void* ptrs[] = {H->col_ptr, H->row_idx, H->perm, H->vals_csc, H->gorder, H->grank, H->gcol, H->gsrc,
                    H->gvals, H->bits, H->xd, H->sp_idx,
                    H->sp_val, H->scratch_i32, H->dev_scalars, H->scan_counter, H->ws,
                    H->part[0][0], H->part[0][1], H->part[1][0], H->part[1][1], H->dev_sel, H->bws,
                    H->units, H->split_rows, H->bfs_front[0], H->bfs_front[1], H->bfs_y, H->drv_count,
                    H->bfs_bits[0], H->bfs_bits[1], H->pr_W, H->pr_r, H->pr_y, H->pr_xidx, H->pr_xval,
                    H->pr_xd[0], H->pr_xd[1], H->pr_p, H->pr_bad, H->cnt_dev};
    for (void* p : ptrs)
        if (p) hipFree(p);
    sell_free(&H->sell);
    ell_free(&H->ell);
    dia_free(&H->dia);
    csr5_free(&H->c5);
    tile_sorted_free(&H->ts);
    if (H->drv_host) hipHostFree(H->drv_host);
    if (H->cnt_host) hipHostFree(H->cnt_host);
    for (auto& e : H->drv_ev)
        if (e) hipEventDestroy(e);
    for (auto& e : H->ev_conv) {
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    for (auto& e : H->ev_kern) {
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    hipSetDevice(cur);
    delete H;
    return SPX_OK;
}

static spx_status build_csc(spx_matrix* H, hipStream_t s) {
    const spx_csr& A = H->csr;
    const int64_t nnz = A.nnz;
    const int vs = value_size(A.dtype);
    if (hipMalloc((void**)&H->col_ptr, ((size_t)A.n + 1) * 4) != hipSuccess ||
        hipMalloc((void**)&H->row_idx, (size_t)std::max<int64_t>(nnz, 1) * 4) != hipSuccess ||
        hipMalloc((void**)&H->perm, (size_t)std::max<int64_t>(nnz, 1) * 4) != hipSuccess)
        return fail(SPX_ERR_ALLOC, "CSC allocation failed");
    if (vs > 0 && hipMalloc(&H->vals_csc, (size_t)std::max<int64_t>(nnz, 1) * vs) != hipSuccess)
        return fail(SPX_ERR_ALLOC, "CSC values allocation failed");
    if (nnz == 0) return fill_u32((uint32_t*)H->col_ptr, 0u, (size_t)A.n + 1, s);
    // stable radix sort of (column, CSR position): the permutation orders
    // entries by column and, within a column, by row
    uint32_t *keys = nullptr, *keys2 = nullptr, *vals2 = nullptr;
    int32_t* rws = nullptr;
    int32_t* rows = nullptr;
    const size_t rw = radix_ws_elems(nnz);
    if (hipMalloc((void**)&keys, nnz * 4) != hipSuccess || hipMalloc((void**)&keys2, nnz * 4) != hipSuccess ||
        hipMalloc((void**)&vals2, nnz * 4) != hipSuccess || hipMalloc((void**)&rws, rw * 4) != hipSuccess ||
        hipMalloc((void**)&rows, nnz * 4) != hipSuccess)
        return fail(SPX_ERR_ALLOC, "transpose temporaries: allocation failed");
    spx_status st = SPX_OK;
    do {
        if (hipMemcpyAsync(keys, A.col_idx, nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            st = fail(SPX_ERR_HIP, "copy col_idx");
            break;
        }
        const int grid = (int)std::min<int64_t>(ceil_div(nnz, kBlock), 8192);
        k_iota<<<grid, kBlock, 0, s>>>((uint32_t*)H->perm, nnz);
        bool alt = false;
        st = radix_sort_pairs(keys, (uint32_t*)H->perm, keys2, vals2, nnz, key_bits_for(A.n), rws, s, &alt);
        if (st) break;
        const uint32_t* sk = alt ? keys2 : keys;
        if (alt && hipMemcpyAsync(H->perm, vals2, nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            st = fail(SPX_ERR_HIP, "copy perm");
            break;
        }
        k_ptr_from_sorted<<<(unsigned)ceil_div(nnz + 1, kBlock), kBlock, 0, s>>>(sk, nnz, A.n, H->col_ptr);
        st = expand_rows(A.row_ptr, A.m, rows, s);
        if (st) break;
        st = gather_perm(rows, H->perm, H->row_idx, nnz, 4, s);
        if (st) break;
        if (vs > 0) st = gather_perm(A.vals, H->perm, H->vals_csc, nnz, vs, s);
        if (st) break;
        if (hipStreamSynchronize(s) != hipSuccess) st = fail(SPX_ERR_HIP, "transpose sync");
    } while (0);
    hipFree(keys);
    hipFree(keys2);
    hipFree(vals2);
    hipFree(rws);
    hipFree(rows);
    return st;
}

// Column renumbering for the row-major kernels. Their x (or bitvector)
// reads are gathers that run at the rate of the cache level holding the
// gathered lines; with columns ranked by descending length the most-read
// entries share lines that stay in the per-CU cache. Used by default when
// the kHotCols longest columns hold a share of the entries well above what
// uniform lengths would give them.
constexpr int32_t kHotCols = 16384;

static spx_status build_gcsr(spx_matrix* H, uint32_t flags, hipStream_t s) {
    const spx_csr& A = H->csr;
    const int64_t nnz = A.nnz;
    if ((flags & SPX_NO_RENUMBER) || A.n == 0 || nnz == 0) return SPX_OK;
    std::vector<int32_t> cp((size_t)A.n + 1);
    SPX_HIP(hipMemcpyAsync(cp.data(), H->col_ptr, cp.size() * 4, hipMemcpyDeviceToHost, s));
    SPX_HIP(hipStreamSynchronize(s));
    int32_t maxlen = 0;
    for (int32_t j = 0; j < A.n; ++j) maxlen = std::max(maxlen, cp[j + 1] - cp[j]);
    // stable counting sort of the columns by descending length
    std::vector<int64_t> start((size_t)maxlen + 2, 0);
    for (int32_t j = 0; j < A.n; ++j) ++start[(size_t)(maxlen - (cp[j + 1] - cp[j])) + 1];
    for (size_t b = 1; b < start.size(); ++b) start[b] += start[b - 1];
    std::vector<int32_t> order((size_t)A.n), rank((size_t)A.n), gptr((size_t)A.n + 1);
    for (int32_t j = 0; j < A.n; ++j) order[(size_t)start[(size_t)(maxlen - (cp[j + 1] - cp[j]))]++] = j;
    gptr[0] = 0;
    for (int32_t r = 0; r < A.n; ++r) {
        rank[(size_t)order[r]] = r;
        gptr[(size_t)r + 1] = gptr[r] + (cp[order[r] + 1] - cp[order[r]]);
    }
    if (!(flags & SPX_RENUMBER)) {
        const int32_t hot = std::min(kHotCols, A.n);
        const double share = (double)gptr[hot] / (double)nnz;
        const double uniform = (double)hot / A.n;
        if (A.n < 4 * kHotCols || share < std::max(0.3, 2.0 * uniform)) return SPX_OK;
    }
    const int vs = value_size(A.dtype);
    if (hipMalloc((void**)&H->gorder, (size_t)A.n * 4) != hipSuccess ||
        hipMalloc((void**)&H->grank, (size_t)A.n * 4) != hipSuccess ||
        hipMalloc((void**)&H->gcol, (size_t)nnz * 4) != hipSuccess ||
        (vs > 0 && hipMalloc(&H->gvals, (size_t)nnz * vs) != hipSuccess))
        return fail(SPX_ERR_ALLOC, "renumbered CSR allocation failed");
    uint32_t *keys = nullptr, *vals = nullptr, *keys2 = nullptr, *vals2 = nullptr;
    int32_t *rws = nullptr, *rq = nullptr, *dptr = nullptr;
    const size_t rw = radix_ws_elems(nnz);
    spx_status st = SPX_OK;
    do {
        if (hipMalloc((void**)&keys, nnz * 4) != hipSuccess || hipMalloc((void**)&vals, nnz * 4) != hipSuccess ||
            hipMalloc((void**)&keys2, nnz * 4) != hipSuccess || hipMalloc((void**)&vals2, nnz * 4) != hipSuccess ||
            hipMalloc((void**)&rws, rw * 4) != hipSuccess || hipMalloc((void**)&rq, nnz * 4) != hipSuccess ||
            hipMalloc((void**)&dptr, gptr.size() * 4) != hipSuccess) {
            st = fail(SPX_ERR_ALLOC, "renumbering temporaries: allocation failed");
            break;
        }
        if (hipMemcpyAsync(H->gorder, order.data(), order.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(H->grank, rank.data(), rank.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(dptr, gptr.data(), gptr.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) {
            st = fail(SPX_ERR_HIP, "renumbering upload");
            break;
        }
        if ((st = expand_rows(dptr, A.n, rq, s))) break;
        const int grid = (int)std::min<int64_t>(ceil_div(nnz, kBlock), 8192);
        k_rank_major<<<grid, kBlock, 0, s>>>(nnz, rq, dptr, H->gorder, H->col_ptr, H->row_idx, H->perm, keys, vals);
        bool alt = false;
        // stable by row: within a row the entries keep their rank order
        if ((st = radix_sort_pairs(keys, vals, keys2, vals2, nnz, key_bits_for(A.m), rws, s, &alt))) break;
        H->gsrc = (int32_t*)(alt ? vals2 : vals);
        (alt ? vals2 : vals) = nullptr;
        k_renumber_cols<<<grid, kBlock, 0, s>>>(nnz, H->gsrc, A.col_idx, H->grank, H->gcol);
        if (hipGetLastError() != hipSuccess) {
            st = fail(SPX_ERR_HIP, "renumbering kernels");
            break;
        }
        if (vs > 0 && (st = gather_perm(A.vals, H->gsrc, H->gvals, nnz, vs, s))) break;
        if (hipStreamSynchronize(s) != hipSuccess) st = fail(SPX_ERR_HIP, "renumbering sync");
    } while (0);
    for (void* p : {(void*)keys, (void*)vals, (void*)keys2, (void*)vals2, (void*)rws, (void*)rq, (void*)dptr})
        if (p) hipFree(p);
    if (st != SPX_OK) return st;
    H->gcsr = A;
    H->gcsr.col_idx = H->gcol;
    H->gcsr.vals = vs > 0 ? H->gvals : nullptr;
    // the column-sorted copy for the balanced SpMV (2048-item tiles)
    if (A.n <= (1 << 21)) {
        spx_plan bal{SPX_PAT_SPMV, SPX_DIST_BALANCED, SPX_WB_NONE, 0, 2048, 0};
        const int32_t* part = nullptr;
        SPX_TRY(cached_part(H, H->gcsr, 0, &bal, s, &part));
        SPX_TRY(tile_sorted_build(H->gcsr, part, H->gsrc, &H->ts, s));
    }
    return SPX_OK;
}

// Storage-format pre-selection: which copy beside CSR the SpMV pattern
// runs on (none, sliced ELLPACK, ELLPACK or CSR5). The tree reads the
// Table 1 features of A and the padding ratios (cells / nnz): the sliced
// copy's is computed from a host copy of row_ptr only when a node asks for
// it; the CSR5 copy is built from that host copy too.
constexpr int32_t kSellMaxRow = 4096;  // longest row the copy accepts (serial sums per lane)
constexpr double kSellMaxRatio = 3.0;  // most cells per entry it accepts, beyond a fixed allowance
constexpr int64_t kSellAllowance = 65536;  // cells any matrix may use (one partly filled slice)
constexpr int32_t kEllMaxRow = 4096;   // longest row the ELL copy accepts
constexpr double kEllMaxRatio = 1.5;   // most cells per entry it accepts, beyond the allowance
static spx_status choose_format(spx_matrix* H, uint32_t flags, hipStream_t s) {
    const spx_csr& A = H->gorder ? H->gcsr : H->csr;
    if ((flags & SPX_FORMAT_CSR) || A.m == 0) return SPX_OK;
    const int nforced = ((flags & SPX_FORMAT_SELL) ? 1 : 0) + ((flags & SPX_FORMAT_ELL) ? 1 : 0) +
                        ((flags & SPX_FORMAT_CSR5) ? 1 : 0) + ((flags & SPX_FORMAT_DIA) ? 1 : 0);
    if (nforced > 1)
        return fail(SPX_ERR_ARG, "SPX_FORMAT_SELL, SPX_FORMAT_ELL, SPX_FORMAT_CSR5 and SPX_FORMAT_DIA exclude each other");
    const bool forced = (flags & SPX_FORMAT_SELL) != 0;
    const bool forced_ell = (flags & SPX_FORMAT_ELL) != 0;
    const bool forced_c5 = (flags & SPX_FORMAT_CSR5) != 0;
    const bool forced_dia = (flags & SPX_FORMAT_DIA) != 0;
    // the DIA copy first: where it applies it moves fewer bytes than CSR
    // and than any padded copy (no column indices at all)
    if (forced_dia || nforced == 0) {
        SPX_TRY(dia_try_build(A, (int32_t)H->feat[3], forced_dia, &H->dia, s));
        if (H->dia.vals || forced_dia) return SPX_OK;
    }
    std::vector<int32_t> rp;
    SellPlanInfo info;
    bool fetched = false, shaped = false;
    spx_status st = SPX_OK;
    auto fetch = [&]() {
        if (fetched) return;
        fetched = true;
        rp.resize((size_t)A.m + 1);
        if (hipMemcpyAsync(rp.data(), A.row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = fail(SPX_ERR_HIP, "row_ptr read-back");
    };
    auto shape = [&]() {
        if (shaped) return;
        shaped = true;
        fetch();
        if (st == SPX_OK) info = sell_shape(rp.data(), A.m);
    };
    auto ratio = [&]() {
        shape();
        return (double)info.padded / (double)std::max<int64_t>(1, A.nnz);
    };
    const int choice = forced ? 1 : forced_ell ? 2 : forced_c5 ? 3 : format_choice(H->feat, ratio);
    if (st != SPX_OK || choice == 0) return st;
    if (choice == 3) {
        fetch();
        if (st != SPX_OK) return st;
        return csr5_build(A, rp.data(), &H->c5, s);
    }
    if (choice == 2) {
        const int32_t w = (int32_t)H->feat[3];
        const double cells = (double)w * (double)A.m;
        if (w > kEllMaxRow || cells > kEllMaxRatio * (double)A.nnz + (double)kSellAllowance) {
            if (forced_ell)
                return fail(SPX_ERR_UNSUPPORTED, "ELL: a row longer than 4096 or more than 1.5 nnz + 65536 cells");
            return SPX_OK;
        }
        return ell_build(A, w, &H->ell, s);
    }
    const double r = ratio();
    if (st != SPX_OK) return st;
    if (H->feat[3] > kSellMaxRow || (double)info.padded > kSellMaxRatio * (double)A.nnz + (double)kSellAllowance) {
        if (forced) return fail(SPX_ERR_UNSUPPORTED, "sliced ELL: a row longer than 4096 or more than 3 nnz + 65536 cells");
        return SPX_OK;
    }
    SPX_TRY(sell_build(A, info, &H->sell, s));
    H->sell_ratio = r;
    return SPX_OK;
}

extern "C" spx_status spx_matrix_create(const spx_csr* A, uint32_t flags, void* stream, spx_matrix** out) {
    if (!out) return fail(SPX_ERR_ARG, "out is null");
    *out = nullptr;
    SPX_TRY(spx_check_csr(A));
    hipStream_t s = (hipStream_t)stream;
    spx_matrix* H = new (std::nothrow) spx_matrix();
    if (!H) return fail(SPX_ERR_ALLOC, "handle allocation failed");
    H->csr = *A;
    hipGetDevice(&H->device);
    H->sel = global_selector();
    H->has_sel_known = global_selector_known().first;
    if (H->has_sel_known) H->sel_known = global_selector_known().second;
    H->has_sel_run = global_selector_run().first;
    if (H->has_sel_run) H->sel_run = global_selector_run().second;
    spx_status st = SPX_OK;
    if (flags & SPX_VALIDATE) {
        uint32_t* bad = nullptr;
        uint32_t hbad = 0;
        if (hipMalloc((void**)&bad, 4) != hipSuccess) {
            spx_matrix_destroy(H);
            return fail(SPX_ERR_ALLOC, "validation flag");
        }
        fill_u32(bad, 0, 1, s);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(std::max(A->nnz, A->m + 1), kBlock), 4096));
        k_validate_csr<<<grid, kBlock, 0, s>>>(A->row_ptr, A->m, A->col_idx, A->nnz, A->n, bad);
        hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s);
        hipStreamSynchronize(s);
        hipFree(bad);
        if (hbad) {
            spx_matrix_destroy(H);
            return fail(hbad & 1 ? SPX_ERR_SHAPE : SPX_ERR_INDEX,
                        hbad & 1 ? "row_ptr is not a valid CSR row pointer" : "a column index is out of range");
        }
    }
    if (hipMalloc((void**)&H->scan_counter, 256) != hipSuccess || hipMemset(H->scan_counter, 0, 256) != hipSuccess) {
        spx_matrix_destroy(H);
        return fail(SPX_ERR_ALLOC, "scan counter allocation failed");
    }
    st = build_csc(H, s);
    if (st == SPX_OK) st = build_gcsr(H, flags, s);
    if (st == SPX_OK) {
        MatrixStats ms;
        st = matrix_features_device(A->row_ptr, A->m, A->n, &ms, s);
        if (st == SPX_OK) std::memcpy(H->feat, ms.f, sizeof(H->feat));
    }
    if (st == SPX_OK) st = choose_format(H, flags, s);
    if (st == SPX_OK) st = upload_selector(H);
    if (st != SPX_OK) {
        std::string keep = g_err;
        spx_matrix_destroy(H);
        g_err = keep;
        return st;
    }
    *out = H;
    return SPX_OK;
}

extern "C" spx_status spx_matrix_csc(const spx_matrix* H, spx_csc* out) {
    if (!H || !out) return fail(SPX_ERR_ARG, "null argument");
    *out = handle_csc(H);
    return SPX_OK;
}

extern "C" spx_status spx_matrix_values_updated(spx_matrix* H, void* stream) {
    if (!H) return fail(SPX_ERR_ARG, "handle is null");
    const int vs = value_size(H->csr.dtype);
    H->pr_W_valid = false;
    if (vs == 0 || H->csr.nnz == 0) return SPX_OK;
    SPX_TRY(gather_perm(H->csr.vals, H->perm, H->vals_csc, H->csr.nnz, vs, (hipStream_t)stream));
    if (H->gsrc) SPX_TRY(gather_perm(H->csr.vals, H->gsrc, H->gvals, H->csr.nnz, vs, (hipStream_t)stream));
    if (H->sell.col) SPX_TRY(sell_refresh(H->sell, H->gorder ? H->gcsr : H->csr, (hipStream_t)stream));
    if (H->ell.col) SPX_TRY(ell_refresh(H->ell, H->gorder ? H->gcsr : H->csr, (hipStream_t)stream));
    if (H->dia.vals) SPX_TRY(dia_refresh(H->dia, H->gorder ? H->gcsr : H->csr, (hipStream_t)stream));
    if (H->c5.col) SPX_TRY(csr5_refresh(H->c5, H->gorder ? H->gcsr : H->csr, (hipStream_t)stream));
    if (H->ts.pk) SPX_TRY(gather_perm(H->csr.vals, H->ts.src, H->ts.vals, H->csr.nnz, vs, (hipStream_t)stream));
    return SPX_OK;
}

extern "C" spx_status spx_matrix_format(const spx_matrix* H, int32_t* format, double* padding_ratio) {
    if (!H || !format) return fail(SPX_ERR_ARG, "null argument");
    *format = H->sell.col ? 1 : H->ell.col ? 2 : H->c5.col ? 3 : H->dia.vals ? 4 : 0;
    if (padding_ratio)
        *padding_ratio = H->sell.col  ? H->sell_ratio
                         : H->dia.vals ? (double)H->dia.cells / (double)std::max<int32_t>(1, H->csr.nnz)
                         : H->ell.col ? (double)H->ell.cells / (double)std::max<int32_t>(1, H->csr.nnz)
                         : H->c5.col  ? (double)H->c5.cells / (double)std::max<int32_t>(1, H->csr.nnz)
                                      : 0.0;
    return SPX_OK;
}

extern "C" spx_status spx_matrix_column_order(const spx_matrix* H, int32_t* order, int32_t* renumbered,
                                              void* stream) {
    if (!H || !renumbered) return fail(SPX_ERR_ARG, "null argument");
    *renumbered = H->gorder ? 1 : 0;
    if (!H->gorder || !order || H->csr.n == 0) return SPX_OK;
    SPX_HIP(hipMemcpyAsync(order, H->gorder, (size_t)H->csr.n * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SPX_OK;
}

extern "C" spx_status spx_matrix_features(const spx_matrix* H, double* out9) {
    if (!H || !out9) return fail(SPX_ERR_ARG, "null argument");
    std::memcpy(out9, H->feat, sizeof(H->feat));
    return SPX_OK;
}

static spx_status check_vec(const spx_matrix* H, const spx_vec* x) {
    if (!x) return fail(SPX_ERR_ARG, "vector descriptor is null");
    if (x->n != H->csr.n) return fail(SPX_ERR_SHAPE, "vector length differs from n");
    if (x->kind == SPX_VEC_DENSE) {
        if (x->n > 0 && !x->val) return fail(SPX_ERR_ARG, "dense x is null");
    } else if (x->kind == SPX_VEC_SPARSE) {
        if (x->nnz_x < 0 || x->nnz_x > x->n) return fail(SPX_ERR_SHAPE, "nnz_x must be in [0, n]");
        if (x->nnz_x > 0 && (!x->idx || (H->csr.dtype != SPX_BOOL && !x->val)))
            return fail(SPX_ERR_ARG, "sparse x arrays are null");
    } else {
        return fail(SPX_ERR_ARG, "unknown vector kind");
    }
    return SPX_OK;
}

// device count of nnz_s (and nnz_x of a dense x): one launch that writes
// the totals to pinned host memory, then a stream synchronization
static spx_status device_vector_counts(spx_matrix* H, const spx_vec* x, hipStream_t s, int64_t* nnz_s,
                                       int64_t* nnz_x) {
    if (!H->cnt_dev) {
        if (hipMalloc((void**)&H->cnt_dev, 64) != hipSuccess) return fail(SPX_ERR_ALLOC, "count buffers");
        if (hipHostMalloc((void**)&H->cnt_host, 64, hipHostMallocCoherent) != hipSuccess) {
            hipFree(H->cnt_dev);
            H->cnt_dev = nullptr;
            return fail(SPX_ERR_ALLOC, "pinned count buffer");
        }
        SPX_HIP(hipMemset(H->cnt_dev, 0, 64));
        SPX_HIP(hipDeviceSynchronize());
    }
    volatile long long* h = H->cnt_host;
    h[0] = -1;
    h[1] = -1;
    SPX_TRY(vector_counts_to_host(H->col_ptr, H->csr.n, x, H->csr.dtype, H->cnt_dev, (uint32_t*)(H->cnt_dev + 2),
                                  H->cnt_host, s));
    // the kernel's last workgroup stores the totals to the pinned buffer:
    // poll it (a stream synchronization wakes the host about 10 us later),
    // and after a second without a result fall back to the synchronization,
    // which reports a failed launch
    const auto t0 = std::chrono::steady_clock::now();
    while ((h[0] < 0 || h[1] < 0) && std::chrono::steady_clock::now() - t0 < std::chrono::seconds(1)) {
    }
    if (h[0] < 0 || h[1] < 0) SPX_HIP(hipStreamSynchronize(s));
    if (h[0] < 0 || h[1] < 0) return fail(SPX_ERR_HIP, "vector counts: the counting kernel wrote no result");
    *nnz_s = h[0];
    *nnz_x = x->kind == SPX_VEC_SPARSE ? x->nnz_x : h[1];
    return SPX_OK;
}

extern "C" spx_status spx_vector_features(spx_matrix* H, const spx_vec* x, double* out4, void* stream) {
    if (!H || !out4) return fail(SPX_ERR_ARG, "null argument");
    SPX_TRY(check_vec(H, x));
    int64_t ns = 0, nx = 0;
    SPX_TRY(device_vector_counts(H, x, (hipStream_t)stream, &ns, &nx));
    out4[0] = (double)nx;
    out4[1] = H->csr.n > 0 ? (double)nx / H->csr.n : 0.0;
    out4[2] = (double)ns;
    out4[3] = H->csr.nnz > 0 ? (double)ns / H->csr.nnz : 0.0;
    return SPX_OK;
}

// ------------------------------------------------------------------ selection
struct LazyFeatures {
    spx_matrix* H;
    const spx_vec* x;
    hipStream_t s;
    bool no_sync;
    bool have_counts = false;
    int64_t nnz_s = -1, nnz_x = -1;
    bool synced = false;
    double count_ms = 0.0;  // host time spent on the device count and its round trip
    double get(int f) {
        const double* mf = H->feat;
        switch (f) {
            case F_M:
            case F_N:
            case F_NNZ:
            case F_MAX_ROW:
            case F_MIN_ROW:
            case F_AVG_ROW:
            case F_REL_RANGE:
            case F_VAR_ROW:
            case F_GINI:
                return mf[f];
            case F_NNZ_X:
                return (double)nx();
            case F_X_SPARSITY:
                return H->csr.n > 0 ? (double)nx() / H->csr.n : 0.0;
            case F_NNZ_S:
                return (double)ns();
            case F_M_SPARSITY:
                return H->csr.nnz > 0 ? (double)ns() / H->csr.nnz : 0.0;
            case F_S_PER_X:
                return (double)ns() / (double)std::max<int64_t>(1, nx());
            case F_COUNTED:
                return have_counts && synced ? 1.0 : 0.0;
        }
        return 0.0;
    }
    void counts() {
        if (have_counts) return;
        have_counts = true;
        if (no_sync || x->kind == SPX_VEC_DENSE) {
            // host-known fallback: a dense x counts as full, nnz_s is
            // estimated from the average column length
            nnz_x = x->kind == SPX_VEC_SPARSE ? x->nnz_x : H->csr.n;
            nnz_s = H->csr.n > 0 ? (int64_t)((double)H->csr.nnz / H->csr.n * nnz_x) : 0;
            return;
        }
        const auto t0 = std::chrono::steady_clock::now();
        if (device_vector_counts(H, x, s, &nnz_s, &nnz_x) != SPX_OK) {
            nnz_x = x->kind == SPX_VEC_SPARSE ? x->nnz_x : H->csr.n;
            nnz_s = H->csr.nnz;
        }
        count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        synced = true;
    }
    // A vector handed over dense is taken as dense (nnz_x = n): counting its
    // nonzeros would cost a device reduction and a sync on every call.
    int64_t nx() { return x->kind == SPX_VEC_SPARSE ? x->nnz_x : H->csr.n; }
    int64_t ns() {
        counts();
        return nnz_s;
    }
};

// Longest row (entries) for which run() still picks a write-back that sums a
// row in one serial FP32 chain: a serial chain over 2^17 products of one sign
// already comes within a factor two of the 1e-5 relative bound.
constexpr double kAtomicChainMax = 65536.0;

static spx_status select_impl(spx_matrix* H, const Selector& S, const spx_vec* x, uint32_t flags, spx_plan* out,
                              LazyFeatures& lf) {
    auto f = [&](int id) { return lf.get(id); };
    spx_plan p{};
    p.pattern = S.pattern.eval(f);
    if (p.pattern < 0 || p.pattern > 2) p.pattern = SPX_PAT_SPMV;
    // A vector handed over dense is taken as dense (nnz_x = n): the trees
    // were trained on vectors handed over as lists, for which a row-major
    // plan pays the scatter into a dense x; here the row-major plans read x
    // as it is, while a column-major plan would first compact it, with a
    // host round trip for its length. Such a vector takes the SpMV pattern.
    if (x->kind == SPX_VEC_DENSE && p.pattern == SPX_PAT_CSC_SPMSPV) p.pattern = SPX_PAT_SPMV;
    p.distribution = S.distribution[p.pattern].eval(f);
    if (p.distribution != SPX_DIST_BALANCED) p.distribution = SPX_DIST_DIRECT;
    p.writeback = SPX_WB_NONE;
    if (p.pattern == SPX_PAT_CSC_SPMSPV) {
        p.writeback = S.writeback.eval(f);
        if (p.writeback < SPX_WB_ATOMIC || p.writeback > SPX_WB_MERGE) p.writeback = SPX_WB_ATOMIC;
        if (p.writeback == SPX_WB_LDS_ATOMIC &&
            (int64_t)H->csr.m * std::max(4, value_size(H->csr.dtype)) > 65536)
            p.writeback = SPX_WB_SORT;
        // the atomic, LDS-atomic and bucket write-backs add a row's products
        // one at a time into one FP32 value; past kAtomicChainMax entries in
        // a row that chain can miss the FP32 error bound, so the row's sum
        // goes through the sort write-back's per-tile trees instead
        if (H->csr.dtype == SPX_F32 && H->feat[3] > kAtomicChainMax &&
            (p.writeback == SPX_WB_ATOMIC || p.writeback == SPX_WB_LDS_ATOMIC || p.writeback == SPX_WB_BUCKET))
            p.writeback = SPX_WB_SORT;
    }
    (void)flags;
    *out = p;
    return SPX_OK;
}

extern "C" spx_status select_kernel(spx_matrix* H, const spx_vec* x, uint32_t flags, spx_plan* out, void* stream) {
    if (!H || !out) return fail(SPX_ERR_ARG, "null argument");
    SPX_TRY(check_vec(H, x));
    LazyFeatures lf{H, x, (hipStream_t)stream, (flags & SPX_NO_SYNC) != 0};
    return select_impl(H, run_selector(H), x, flags, out, lf);
}

extern "C" spx_status spx_load_selector(spx_matrix* H, const char* json_path) {
    Selector s;
    if (!json_path) {
        s = builtin_selector();
    } else {
        std::ifstream in(json_path);
        if (!in) return fail(SPX_ERR_ARG, std::string("cannot open selector file ") + json_path);
        std::stringstream ss;
        ss << in.rdbuf();
        std::string err;
        if (!parse_selector_json(ss.str(), &s, &err)) return fail(SPX_ERR_ARG, "selector: " + err);
    }
    // host-feature trees replace every set (trees that test nnz_s, lazy or
    // not, load after them); lazy trees replace run()'s set only, other
    // trees that test nnz_s the drivers' set only
    const bool lazy = json_path && s.lazy;
    const bool known = json_path && !lazy && s.reads_nnz_s();
    if (!H) {
        if (lazy) {
            global_selector_run() = {true, s};
        } else if (known) {
            global_selector_known() = {true, s};
        } else {
            global_selector() = s;
            global_selector_known().first = false;
            global_selector_run().first = false;
        }
        return SPX_OK;
    }
    if (lazy) {
        H->sel_run = s;
        H->has_sel_run = true;
        return SPX_OK;
    }
    if (known) {
        H->sel_known = s;
        H->has_sel_known = true;
        return SPX_OK;
    }
    H->sel = s;
    H->has_sel_known = false;
    H->has_sel_run = false;
    return upload_selector(H);
}

// ------------------------------------------------------------------ execution
static void record(spx_matrix* H, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, bool start, hipStream_t s) {
    if (!H->profiling) return;
    if (start) {
        hipEvent_t a, b;
        hipEventCreate(&a);
        hipEventCreate(&b);
        v.emplace_back(a, b);
        hipEventRecord(a, s);
    } else {
        hipEventRecord(v.back().second, s);
    }
}

// Executes plan p for x. nnz_s_hint: exact nnz_s if known (else -1).
static spx_status exec_plan(spx_matrix* H, const spx_vec* x, void* y, const spx_plan* p, int64_t nnz_s_hint,
                            int64_t nnz_x_known, hipStream_t s) {
    // the row-major kernels read the renumbered copy when there is one
    const spx_csr& A = H->gorder && p->pattern != SPX_PAT_CSC_SPMSPV ? H->gcsr : H->csr;
    const int dt = A.dtype;
    SPX_TRY(spx_check_plan(p, dt));
    SPX_TRY(ensure_conv(H));
    if (p->pattern == SPX_PAT_SPMV) {
        const void* xd = x->val;
        Unscatter un;
        if (x->kind == SPX_VEC_SPARSE) {
            record(H, H->ev_conv, true, s);
            const bool clean = H->xd_clean;
            H->xd_clean = false;
            SPX_TRY(sparse_to_dense(A.n, x->nnz_x, x->idx, x->val, dt, H->grank, H->xd, s, clean));
            record(H, H->ev_conv, false, s);
            xd = H->xd;
            un = Unscatter{x->nnz_x, x->idx, H->grank, nullptr, H->xd, A.n};
        } else if (H->gorder) {
            record(H, H->ev_conv, true, s);
            H->xd_clean = false;
            SPX_TRY(permute_dense(A.n, x->val, dt, H->gorder, H->xd, nullptr, s));
            record(H, H->ev_conv, false, s);
            xd = H->xd;
        }
        SPX_TRY(ensure_ws(H, ws_for(A.m, A.n, A.nnz, 0, dt, p)));
        Arena ws(H->ws, H->ws_bytes);
        const int32_t* part = nullptr;
        SPX_TRY(cached_part(H, A, 0, p, s, &part));
        record(H, H->ev_kern, true, s);
        bool cleared = false;
        if (H->dia.vals)
            SPX_TRY(dia_spmv(H->dia, dt, xd, y, s));
        else if (H->sell.col)
            SPX_TRY(sell_spmv(H->sell, dt, xd, y, s));
        else if (H->ell.col)
            SPX_TRY(ell_spmv(H->ell, dt, xd, y, s));
        else if (H->c5.col)
            SPX_TRY(csr5_spmv(H->c5, dt, xd, y, s));
        else
            SPX_TRY(launch_spmv_csr(&A, xd, nullptr, y, p, part, ws, s, un.xd ? &un : nullptr, &cleared,
                                    H->gorder && H->ts.pk ? &H->ts : nullptr));
        record(H, H->ev_kern, false, s);
        if (un.xd) H->xd_clean = cleared;
        return SPX_OK;
    }
    if (p->pattern == SPX_PAT_CSR_SPMSPV) {
        const void* xd = nullptr;
        Unscatter un;
        record(H, H->ev_conv, true, s);
        if (x->kind == SPX_VEC_SPARSE) {
            // the values land in xd unfilled (the bitvector decides which
            // entries are read), so only the bitvector is cleared after
            const bool clean = H->bits_clean;
            H->bits_clean = false;
            if (dt != SPX_BOOL) H->xd_clean = false;
            SPX_TRY(sparse_to_bitvector(A.n, x->nnz_x, x->idx, x->val, dt, H->grank, H->bits,
                                        dt == SPX_BOOL ? nullptr : H->xd, s, clean));
            xd = dt == SPX_BOOL ? nullptr : H->xd;
            un = Unscatter{x->nnz_x, x->idx, H->grank, H->bits, nullptr, A.n};
        } else if (H->gorder) {
            H->bits_clean = false;
            H->xd_clean = false;
            SPX_TRY(permute_dense(A.n, x->val, dt, H->gorder, H->xd, H->bits, s));
            xd = dt == SPX_BOOL ? nullptr : H->xd;
        } else {
            H->bits_clean = false;
            const unsigned g = dense_bits_grid(A.n);
            switch (dt) {
                case SPX_F32: k_dense_bits<SPX_F32><<<g, kBlock, 0, s>>>(A.n, (const float*)x->val, H->bits); break;
                case SPX_F64: k_dense_bits<SPX_F64><<<g, kBlock, 0, s>>>(A.n, (const double*)x->val, H->bits); break;
                case SPX_I32: k_dense_bits<SPX_I32><<<g, kBlock, 0, s>>>(A.n, (const int32_t*)x->val, H->bits); break;
                case SPX_BOOL: k_dense_bits<SPX_BOOL><<<g, kBlock, 0, s>>>(A.n, (const uint8_t*)x->val, H->bits); break;
                case SPX_F32_MINPLUS:
                    k_dense_bits<SPX_F32_MINPLUS><<<g, kBlock, 0, s>>>(A.n, (const float*)x->val, H->bits);
                    break;
            }
            SPX_HIP(hipGetLastError());
            xd = dt == SPX_BOOL ? nullptr : x->val;
        }
        record(H, H->ev_conv, false, s);
        if (H->c5.col && p->distribution == SPX_DIST_BALANCED && p->tile == 0 && csr5_lds_fits(A.n)) {
            // the balanced bitvector SpMSpV over the CSR5 tiles the SpMV
            // reads, bitvector in LDS; it leaves the whole bitvector clean
            record(H, H->ev_kern, true, s);
            SPX_TRY(csr5_spmspv(H->c5, dt, A.n, xd, H->bits, y, s));
            record(H, H->ev_kern, false, s);
            H->bits_clean = true;
            return SPX_OK;
        }
        SPX_TRY(ensure_ws(H, ws_for(A.m, A.n, A.nnz, 0, dt, p)));
        Arena ws(H->ws, H->ws_bytes);
        const int32_t* part = nullptr;
        SPX_TRY(cached_part(H, A, 0, p, s, &part));
        record(H, H->ev_kern, true, s);
        bool cleared = false;
        SPX_TRY(launch_spmv_csr(&A, xd, H->bits, y, p, part, ws, s, un.bits ? &un : nullptr, &cleared,
                                H->gorder && H->ts.pk ? &H->ts : nullptr));
        record(H, H->ev_kern, false, s);
        if (un.bits) H->bits_clean = cleared;
        return SPX_OK;
    }
    // column-major: needs (idx, val)
    int32_t nnz_x = x->nnz_x;
    const int32_t* idx = x->idx;
    const void* val = x->val;
    if (x->kind == SPX_VEC_DENSE) {
        record(H, H->ev_conv, true, s);
        SPX_TRY(dense_to_sparse(A.n, x->val, dt, H->sp_idx, dt == SPX_BOOL ? nullptr : H->sp_val,
                                (int32_t*)(H->dev_scalars + 2), H->scratch_i32, s));
        record(H, H->ev_conv, false, s);
        if (nnz_x_known < 0) {
            int32_t h = 0;
            SPX_HIP(hipMemcpyAsync(&h, H->dev_scalars + 2, 4, hipMemcpyDeviceToHost, s));
            SPX_HIP(hipStreamSynchronize(s));
            nnz_x_known = h;
        }
        nnz_x = (int32_t)nnz_x_known;
        idx = H->sp_idx;
        val = H->sp_val;
    }
    SPX_TRY(ensure_ws(H, ws_for(A.m, A.n, A.nnz, nnz_x, dt, p)));
    Arena ws(H->ws, H->ws_bytes);
    CscArgs a{A.m, A.n, A.nnz, dt, H->col_ptr, H->row_idx, H->vals_csc, A.row_ptr, H->scan_counter, nnz_s_hint};
    record(H, H->ev_kern, true, s);
    SPX_TRY(launch_spmspv_csc(a, nnz_x, idx, val, y, p, ws, s));
    record(H, H->ev_kern, false, s);
    return SPX_OK;
}

extern "C" spx_status run(spx_matrix* H, const spx_vec* x, void* y, void* stream) {
    if (!H) return fail(SPX_ERR_ARG, "handle is null");
    SPX_TRY(check_vec(H, x));
    if (H->csr.m > 0 && !y) return fail(SPX_ERR_ARG, "y is null");
    hipStream_t s = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    LazyFeatures lf{H, x, s, false};
    spx_plan p;
    SPX_TRY(select_impl(H, run_selector(H), x, 0, &p, lf));
    auto t1 = std::chrono::steady_clock::now();
    if (H->profiling) {
        // features: the device count and its round trip when a tree asked
        // for nnz_s; model: the rest of the walk
        H->host_ms[0] += lf.count_ms;
        H->host_ms[1] += std::chrono::duration<double, std::milli>(t1 - t0).count() - lf.count_ms;
    }
    H->last_plan = p;
    return exec_plan(H, x, y, &p, lf.have_counts && lf.synced ? lf.nnz_s : -1,
                     lf.have_counts && lf.synced ? lf.nnz_x : -1, s);
}

// Selection for a sparse x whose nnz_s the caller knows (the graph drivers
// count it while they build x): the trees that read nnz_s decide, with no
// device round trip.
static spx_status select_counts(spx_matrix* H, const spx_vec* x, int64_t nnz_s, hipStream_t s, spx_plan* p) {
    LazyFeatures lf{H, x, s, false};
    lf.have_counts = true;
    lf.synced = true;
    lf.nnz_x = x->nnz_x;
    lf.nnz_s = nnz_s;
    SPX_TRY(select_impl(H, known_selector(H), x, 0, p, lf));
    H->last_plan = *p;
    return SPX_OK;
}

// run() for a sparse x with known nnz_s; the column-major kernels get the
// exact nnz_s too.
static spx_status run_counts(spx_matrix* H, const spx_vec* x, void* y, int64_t nnz_s, hipStream_t s) {
    spx_plan p;
    SPX_TRY(select_counts(H, x, nnz_s, s, &p));
    return exec_plan(H, x, y, &p, nnz_s, x->nnz_x, s);
}

// Executes plan p for a sparse x (F32/F64) that the caller has also written
// dense into xd, at grank[j] when the handle keeps the renumbered copy: the
// row-major kernels read xd with no conversion (the CSR SpMSpV takes its
// bitvector from the nonzeros of xd, which equals supp(x) up to entries
// whose value is exactly 0 and contribute nothing), the column-major ones
// read the list.
static spx_status exec_prepared(spx_matrix* H, const spx_vec* x, const void* xd, void* y, const spx_plan* p,
                                int64_t nnz_s, hipStream_t s) {
    if (p->pattern == SPX_PAT_CSC_SPMSPV) return exec_plan(H, x, y, p, nnz_s, x->nnz_x, s);
    const spx_csr& A = H->gorder ? H->gcsr : H->csr;
    const int dt = A.dtype;
    if (dt != SPX_F32 && dt != SPX_F64) return fail(SPX_ERR_DTYPE, "prepared x: F32 or F64 only");
    SPX_TRY(spx_check_plan(p, dt));
    SPX_TRY(ensure_conv(H));
    const uint32_t* bits = nullptr;
    if (p->pattern == SPX_PAT_CSR_SPMSPV) {
        record(H, H->ev_conv, true, s);
        H->bits_clean = false;
        if (dt == SPX_F32)
            k_dense_bits<SPX_F32><<<dense_bits_grid(A.n), kBlock, 0, s>>>(A.n, (const float*)xd, H->bits);
        else
            k_dense_bits<SPX_F64><<<dense_bits_grid(A.n), kBlock, 0, s>>>(A.n, (const double*)xd, H->bits);
        SPX_HIP(hipGetLastError());
        record(H, H->ev_conv, false, s);
        bits = H->bits;
    }
    SPX_TRY(ensure_ws(H, ws_for(A.m, A.n, A.nnz, 0, dt, p)));
    Arena ws(H->ws, H->ws_bytes);
    const int32_t* part = nullptr;
    SPX_TRY(cached_part(H, A, 0, p, s, &part));
    record(H, H->ev_kern, true, s);
    if (H->dia.vals && p->pattern == SPX_PAT_SPMV)
        SPX_TRY(dia_spmv(H->dia, dt, xd, y, s));
    else if (H->sell.col && p->pattern == SPX_PAT_SPMV)
        SPX_TRY(sell_spmv(H->sell, dt, xd, y, s));
    else if (H->ell.col && p->pattern == SPX_PAT_SPMV)
        SPX_TRY(ell_spmv(H->ell, dt, xd, y, s));
    else if (H->c5.col && p->pattern == SPX_PAT_SPMV)
        SPX_TRY(csr5_spmv(H->c5, dt, xd, y, s));
    else if (p->pattern == SPX_PAT_CSR_SPMSPV && p->distribution == SPX_DIST_BALANCED && p->tile == 0 && H->c5.col &&
             csr5_lds_fits(A.n)) {
        SPX_TRY(csr5_spmspv(H->c5, dt, A.n, xd, H->bits, y, s));
        H->bits_clean = true;
    } else
        SPX_TRY(launch_spmv_csr(&A, xd, bits, y, p, part, ws, s, nullptr, nullptr,
                                H->gorder && H->ts.pk ? &H->ts : nullptr));
    record(H, H->ev_kern, false, s);
    return SPX_OK;
}

extern "C" spx_status run_plan(spx_matrix* H, const spx_vec* x, void* y, const spx_plan* plan, void* stream) {
    if (!H || !plan) return fail(SPX_ERR_ARG, "null argument");
    SPX_TRY(check_vec(H, x));
    if (H->csr.m > 0 && !y) return fail(SPX_ERR_ARG, "y is null");
    H->last_plan = *plan;
    return exec_plan(H, x, y, plan, -1, -1, (hipStream_t)stream);
}

extern "C" spx_status spx_last_plan(const spx_matrix* H, spx_plan* out) {
    if (!H || !out) return fail(SPX_ERR_ARG, "null argument");
    *out = H->last_plan;
    return SPX_OK;
}

extern "C" spx_status spx_set_profiling(spx_matrix* H, int32_t on) {
    if (!H) return fail(SPX_ERR_ARG, "handle is null");
    H->profiling = on ? 1 : 0;
    return SPX_OK;
}

extern "C" spx_status spx_run_times(spx_matrix* H, double* out, int32_t cap, int32_t* count) {
    if (!H || !count || (cap > 0 && !out)) return fail(SPX_ERR_ARG, "null argument");
    int32_t i = 0;
    for (auto& e : H->ev_kern) {
        float ms = 0;
        hipEventSynchronize(e.second);
        hipEventElapsedTime(&ms, e.first, e.second);
        if (i < cap) out[i] = ms;
        ++i;
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    H->ev_kern.clear();
    *count = i;
    return SPX_OK;
}

extern "C" spx_status spx_stage_times(const spx_matrix* Hc, double* out4) {
    if (!Hc || !out4) return fail(SPX_ERR_ARG, "null argument");
    spx_matrix* H = const_cast<spx_matrix*>(Hc);
    // conversion events are consumed here; kernel events stay for
    // spx_run_times, which consumes them
    auto sum = [&](std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, bool consume) {
        double t = 0;
        for (auto& e : v) {
            float ms = 0;
            hipEventSynchronize(e.second);
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) t += ms;
            if (consume) {
                hipEventDestroy(e.first);
                hipEventDestroy(e.second);
            }
        }
        if (consume) v.clear();
        return t;
    };
    out4[0] = H->host_ms[0];
    out4[1] = H->host_ms[1];
    out4[2] = sum(H->ev_conv, true);
    out4[3] = sum(H->ev_kern, false);
    H->host_ms[0] = H->host_ms[1] = 0;
    return SPX_OK;
}

// ------------------------------------------------------------------ batch (device-side selection)
static int lanes_for(double avg) {
    int L = 1;
    while (L < 64 && L < avg) L <<= 1;
    return L;
}

// Work units of the fused row-major groups of run_batch: consecutive whole
// rows up to kFusedUnitNnz entries and kFusedUnitRows rows per unit; a longer
// row becomes pieces of kFusedUnitNnz entries (a split row).
static spx_status build_units(spx_matrix* H, hipStream_t s) {
    const spx_csr& A = H->csr;
    std::vector<int32_t> rp((size_t)A.m + 1);
    SPX_HIP(hipMemcpyAsync(rp.data(), A.row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, s));
    SPX_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> u;
    std::vector<int32_t> split;
    int32_t r = 0;
    while (r < A.m) {
        const int32_t len = rp[r + 1] - rp[r];
        if (len > kFusedUnitNnz) {
            for (int32_t k = rp[r]; k < rp[r + 1]; k += kFusedUnitNnz)
                u.insert(u.end(), {r, r + 1, k, std::min(k + kFusedUnitNnz, rp[r + 1])});
            split.push_back(r);
            ++r;
            continue;
        }
        const int32_t r0 = r;
        while (r < A.m && r - r0 < kFusedUnitRows && rp[r + 1] - rp[r0] <= kFusedUnitNnz) ++r;
        u.insert(u.end(), {r0, r, rp[r0], rp[r]});
    }
    H->nunits = (int32_t)(u.size() / 4);
    H->nsplit = (int32_t)split.size();
    if (hipMalloc((void**)&H->units, u.size() * 4) != hipSuccess ||
        hipMalloc((void**)&H->split_rows, std::max<size_t>(1, split.size()) * 4) != hipSuccess)
        return fail(SPX_ERR_ALLOC, "run_batch: work units allocation failed");
    SPX_HIP(hipMemcpy(H->units, u.data(), u.size() * 4, hipMemcpyHostToDevice));
    if (!split.empty()) SPX_HIP(hipMemcpy(H->split_rows, split.data(), split.size() * 4, hipMemcpyHostToDevice));
    return SPX_OK;
}

extern "C" spx_status run_batch(spx_matrix* H, int32_t B, int64_t total_nnz_x, const int32_t* vec_ptr,
                                const int32_t* idx, const void* val, void* Y, void* stream) {
    if (!H) return fail(SPX_ERR_ARG, "handle is null");
    if (B < 0 || total_nnz_x < 0) return fail(SPX_ERR_SHAPE, "B and total_nnz_x must be >= 0");
    if (H->csr.dtype == SPX_F32_MINPLUS) return fail(SPX_ERR_DTYPE, "the batched path has no min-plus kernels");
    if (B == 0) return SPX_OK;
    const spx_csr& A = H->csr;
    if (!vec_ptr || (total_nnz_x > 0 && (!idx || (A.dtype != SPX_BOOL && !val))) || (A.m > 0 && !Y))
        return fail(SPX_ERR_ARG, "run_batch: null array");
    if (total_nnz_x > (int64_t)B * A.n) return fail(SPX_ERR_SHAPE, "total_nnz_x exceeds B * n");
    hipStream_t s = (hipStream_t)stream;
    const spx_plan bal{SPX_PAT_SPMV, SPX_DIST_BALANCED, SPX_WB_NONE, 0, 0, 0};
    const int32_t* part = nullptr;
    SPX_TRY(cached_part(H, A, 0, &bal, s, &part));
    const int64_t tiles_mat = ceil_div((int64_t)A.m + A.nnz, 2048);
    if (!H->units && A.dtype != SPX_BOOL && A.m > 0) SPX_TRY(build_units(H, s));
    // capacity-bounded workspace, zeroed at allocation (the per-vector
    // bitvector and value slots and the group slabs are self-cleaning
    // afterwards)
    if (B > H->bcap_B || total_nnz_x > H->bcap_nnz) {
        const int32_t nb = std::max(B, H->bcap_B);
        const int64_t nn = std::max(total_nnz_x, H->bcap_nnz);
        size_t zf = 0, zb = 0;
        const size_t bytes = batch_ws_size(A.m, A.n, A.dtype, nb, nn, tiles_mat, &zf, &zb);
        SPX_HIP(hipStreamSynchronize(s));
        if (H->bws) SPX_HIP(hipFree(H->bws));
        H->bws = nullptr;
        if (hipMalloc(&H->bws, bytes) != hipSuccess) {
            H->bcap_B = 0;
            H->bcap_nnz = 0;
            return fail(SPX_ERR_ALLOC, "run_batch: workspace allocation failed");
        }
        SPX_HIP(hipMemset((char*)H->bws + zf, 0, zb));
        SPX_HIP(hipDeviceSynchronize());
        H->bws_bytes = bytes;
        H->bcap_B = nb;
        H->bcap_nnz = nn;
        H->gkey_B = -1;  // the captured graph points at the old workspace
    }
    BatchLaunch L{};
    L.csr = A;
    L.col_ptr = H->col_ptr;
    L.row_idx = H->row_idx;
    L.vals_csc = H->vals_csc;
    L.part = part;
    L.tiles_mat = tiles_mat;
    L.B = B;
    L.cap_nnz_x = H->bcap_nnz;
    L.vec_ptr = vec_ptr;
    L.idx = idx;
    L.val = val;
    L.Y = Y;
    L.sel = H->dev_sel;
    L.row_lanes = lanes_for(H->feat[5]);
    int dev = 0, cus = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    L.persistent_grid = std::max(1, cus) * 4;
    L.units = H->units;
    L.nunits = H->nunits;
    L.split_rows = H->split_rows;
    L.nsplit = H->nsplit;
    // the graph is keyed by everything its kernel arguments capture
    const void* key[5] = {vec_ptr, idx, val, Y, H->bws};
    const bool same = H->gexec && H->gkey_B == B && std::equal(key, key + 5, H->gkey);
    if (!same) {
        if (H->gexec) hipGraphExecDestroy(H->gexec);
        if (H->graph) hipGraphDestroy(H->graph);
        H->gexec = nullptr;
        H->graph = nullptr;
        if (!H->cap_stream) SPX_HIP(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
        if (!H->cap_side) SPX_HIP(hipStreamCreateWithFlags(&H->cap_side, hipStreamNonBlocking));
        if (!H->cap_fork) SPX_HIP(hipEventCreateWithFlags(&H->cap_fork, hipEventDisableTiming));
        if (!H->cap_join) SPX_HIP(hipEventCreateWithFlags(&H->cap_join, hipEventDisableTiming));
        L.side = H->cap_side;
        L.fork = H->cap_fork;
        L.join = H->cap_join;
        SPX_HIP(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
        spx_status st = launch_batch(L, H->bws, H->bws_bytes, H->cap_stream, &H->berr);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(H->cap_stream, &g);
        if (st != SPX_OK) {
            if (g) hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&H->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            return hip_fail(e, "hipGraphInstantiate");
        }
        H->graph = g;
        std::copy(key, key + 5, H->gkey);
        H->gkey_B = B;
    }
    SPX_HIP(hipGraphLaunch(H->gexec, s));
    return SPX_OK;
}

extern "C" spx_status spx_batch_status(spx_matrix* H, int32_t* flags, void* stream) {
    if (!H || !flags) return fail(SPX_ERR_ARG, "null argument");
    *flags = 0;
    if (!H->berr) return SPX_OK;
    SPX_HIP(hipMemcpyAsync(flags, H->berr, 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
    SPX_HIP(hipStreamSynchronize((hipStream_t)stream));
    return SPX_OK;
}

// ------------------------------------------------------------------ sparse output
extern "C" spx_status spmspv_sparse(spx_matrix* H, const spx_vec* x, const uint32_t* mask, const spx_plan* plan,
                                    int32_t* y_idx, void* y_val, int32_t* nnz_y, void* stream) {
    if (!H || !x || !nnz_y) return fail(SPX_ERR_ARG, "null argument");
    SPX_TRY(check_vec(H, x));
    if (x->kind != SPX_VEC_SPARSE) return fail(SPX_ERR_ARG, "the sparse-output product takes a sparse x");
    if (H->csr.m > 0 && !y_idx) return fail(SPX_ERR_ARG, "y_idx is null");
    *nnz_y = 0;
    const int dt = H->csr.dtype;
    hipStream_t s = (hipStream_t)stream;
    spx_plan p{};
    if (plan) {
        SPX_TRY(spx_check_plan(plan, dt));
        if (plan->pattern != SPX_PAT_CSC_SPMSPV || plan->writeback != SPX_WB_BUCKET)
            return fail(SPX_ERR_ARG, "the sparse-output product runs the column-major bucket plans");
        p = *plan;
    } else {
        // the column-major distribution tree decides; the write-back is the
        // bucket one, the only one that lists rows
        LazyFeatures lf{H, x, s, false};
        p.pattern = SPX_PAT_CSC_SPMSPV;
        p.distribution = H->sel.distribution[SPX_PAT_CSC_SPMSPV].eval([&](int f) { return lf.get(f); }) ==
                                 SPX_DIST_BALANCED
                             ? SPX_DIST_BALANCED
                             : SPX_DIST_DIRECT;
        p.writeback = SPX_WB_BUCKET;
    }
    // each bucket that lists rows takes one atomic on the shared count, and
    // atomics on one word serialize: the fewest, largest buckets that fit
    // LDS (a quarter of the default count at m = 2^20)
    if (p.bucket_rows <= 0) {
        const int asz = dt == SPX_F64 ? 8 : 4;
        int R = 64;
        while (R < 65536 / asz && R < H->csr.m) R <<= 1;
        p.bucket_rows = R;
    }
    H->last_plan = p;
    if (H->csr.m == 0 || x->nnz_x == 0) return SPX_OK;
    SPX_TRY(ensure_conv(H));
    int32_t* count = (int32_t*)(H->dev_scalars + 6);
    SPX_TRY(fill_u32((uint32_t*)count, 0u, 1, s));
    const SparseOut so{mask, y_idx, y_val, count};
    const spx_csr& A = H->csr;
    SPX_TRY(ensure_ws(H, ws_for(A.m, A.n, A.nnz, x->nnz_x, dt, &p)));
    Arena ws(H->ws, H->ws_bytes);
    CscArgs a{A.m, A.n, A.nnz, dt, H->col_ptr, H->row_idx, H->vals_csc, A.row_ptr, H->scan_counter, -1, &so};
    record(H, H->ev_kern, true, s);
    SPX_TRY(launch_spmspv_csc(a, x->nnz_x, x->idx, x->val, nullptr, &p, ws, s));
    record(H, H->ev_kern, false, s);
    int32_t h = 0;
    SPX_HIP(hipMemcpyAsync(&h, count, 4, hipMemcpyDeviceToHost, s));
    SPX_HIP(hipStreamSynchronize(s));
    *nnz_y = h;
    return SPX_OK;
}

// ------------------------------------------------------------------ graph drivers
static spx_status ensure_driver_counters(spx_matrix* H) {
    if (H->drv_host) return SPX_OK;
    if (!H->drv_count && hipMalloc((void**)&H->drv_count, 256) != hipSuccess)
        return fail(SPX_ERR_ALLOC, "driver counters: allocation failed");
    for (auto& e : H->drv_ev)
        if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            e = nullptr;
            return fail(SPX_ERR_HIP, "driver events: creation failed");
        }
    if (hipHostMalloc((void**)&H->drv_host, 64, hipHostMallocDefault) != hipSuccess) {
        H->drv_host = nullptr;
        return fail(SPX_ERR_ALLOC, "driver counters: pinned allocation failed");
    }
    return SPX_OK;
}

// Copies counter (round & 1) to the pinned host words drv_host[0..1] and
// waits for it.
static spx_status read_driver_counter(spx_matrix* H, int32_t round, hipStream_t s) {
    SPX_HIP(hipMemcpyAsync(H->drv_host, H->drv_count + 2 * (round & 1), 8, hipMemcpyDeviceToHost, s));
    SPX_HIP(hipStreamSynchronize(s));
    return SPX_OK;
}

// ------------------------------------------------------------------ breadth-first search
// Direction switch of the search (the direction-optimizing heuristic of
// breadth-first search, not part of the paper): pull once the frontier's
// out-edges exceed the unexplored edges / kPullAlpha, push again once the
// frontier holds fewer than n / kPushBeta vertices.
constexpr double kPullAlpha = 14.0;
constexpr double kPushBeta = 24.0;

extern "C" spx_status spx_bfs(spx_matrix* H, int32_t source, int32_t* level, int32_t max_levels,
                              const spx_plan* plan, uint32_t flags, int32_t* n_levels, spx_plan* plans,
                              int32_t plans_cap, void* stream) {
    if (!H || !n_levels || (plans_cap > 0 && !plans)) return fail(SPX_ERR_ARG, "null argument");
    const spx_csr& A = H->csr;
    if (A.m != A.n) return fail(SPX_ERR_SHAPE, "breadth-first search needs a square matrix");
    if (A.dtype != SPX_BOOL) return fail(SPX_ERR_DTYPE, "breadth-first search runs on a BOOL (pattern) handle");
    if (A.n == 0) {
        *n_levels = 0;
        return SPX_OK;
    }
    if (!level) return fail(SPX_ERR_ARG, "level is null");
    if (source < 0 || source >= A.n) return fail(SPX_ERR_INDEX, "source out of range");
    if (max_levels < 1) return fail(SPX_ERR_ARG, "max_levels must be >= 1");
    if (plan) SPX_TRY(spx_check_plan(plan, A.dtype));
    hipStream_t s = (hipStream_t)stream;
    SPX_TRY(ensure_conv(H));
    SPX_TRY(ensure_driver_counters(H));
    if (!H->bfs_y) {
        const size_t words = (size_t)ceil_div(A.n, 32) * 4;
        if (hipMalloc((void**)&H->bfs_front[0], (size_t)A.n * 4) != hipSuccess ||
            hipMalloc((void**)&H->bfs_front[1], (size_t)A.n * 4) != hipSuccess ||
            hipMalloc((void**)&H->bfs_bits[0], words) != hipSuccess ||
            hipMalloc((void**)&H->bfs_bits[1], words) != hipSuccess ||
            hipMalloc((void**)&H->bfs_y, (size_t)A.m) != hipSuccess)
            return fail(SPX_ERR_ALLOC, "breadth-first search buffers: allocation failed");
    }
    const bool may_pull = !plan && !(flags & SPX_BFS_PUSH_ONLY);
    SPX_TRY(launch_bfs_seed(A.n, source, H->col_ptr, level, H->bfs_front[0], H->bfs_bits[0], H->drv_count, s));
    auto read_count = [&](int32_t L) { return read_driver_counter(H, L, s); };
    SPX_TRY(read_count(0));
    int cur = 0;
    int32_t nf = H->drv_host[0];
    int64_t mf = H->drv_host[1];          // out-edges of the frontier
    int64_t mu = (int64_t)A.nnz - mf;     // out-edges of the unvisited vertices
    bool pull = false;
    int32_t depth = 1;  // levels labelled so far
    while (nf > 0 && depth < max_levels) {
        if (may_pull) {
            if (!pull && (double)mf > (double)mu / kPullAlpha)
                pull = true;
            else if (pull && (double)nf < (double)A.n / kPushBeta)
                pull = false;
        }
        spx_plan p{};
        if (pull) {
            SPX_TRY(launch_bfs_pull(A.n, A.row_ptr, A.col_idx, H->bfs_bits[cur], depth, H->col_ptr, level,
                                    H->bfs_front[cur ^ 1], H->bfs_bits[cur ^ 1], H->drv_count, s));
            p = spx_plan{SPX_PAT_CSR_SPMSPV, SPX_DIST_DIRECT, SPX_WB_NONE, -1, 0, 0};
        } else {
            spx_vec x{SPX_VEC_SPARSE, A.n, nf, H->bfs_front[cur], nullptr};
            if (plan) {
                SPX_TRY(run_plan(H, &x, H->bfs_y, plan, stream));
                p = *plan;
            } else {
                SPX_TRY(run_counts(H, &x, H->bfs_y, mf, s));
                p = H->last_plan;
            }
            SPX_TRY(launch_bfs_update(A.n, H->bfs_y, depth, H->col_ptr, level, H->bfs_front[cur ^ 1],
                                      H->bfs_bits[cur ^ 1], H->drv_count, s));
        }
        if (depth - 1 < plans_cap) plans[depth - 1] = p;
        SPX_TRY(read_count(depth));
        nf = H->drv_host[0];
        mf = H->drv_host[1];
        mu -= mf;
        cur ^= 1;
        if (nf > 0) ++depth;
    }
    *n_levels = depth;
    return SPX_OK;
}

// ------------------------------------------------------------------ incremental PageRank
extern "C" spx_status spx_pagerank(spx_matrix* H, double damping, double eps, int32_t max_iters,
                                   const spx_plan* plan, void* rank, void* residual, int32_t* n_iters,
                                   spx_plan* plans, int32_t plans_cap, void* stream) {
    if (!H || !n_iters || (plans_cap > 0 && !plans)) return fail(SPX_ERR_ARG, "null argument");
    const spx_csr& A = H->csr;
    if (A.m != A.n) return fail(SPX_ERR_SHAPE, "PageRank needs a square matrix");
    if (A.dtype != SPX_F32 && A.dtype != SPX_F64) return fail(SPX_ERR_DTYPE, "PageRank runs on an F32 or F64 handle");
    if (!(damping >= 0.0 && damping < 1.0)) return fail(SPX_ERR_ARG, "damping must lie in [0, 1)");
    if (!(eps >= 0.0)) return fail(SPX_ERR_ARG, "eps must be >= 0");
    if (max_iters < 0) return fail(SPX_ERR_ARG, "max_iters must be >= 0");
    *n_iters = 0;
    if (A.n == 0) return SPX_OK;
    if (!rank) return fail(SPX_ERR_ARG, "rank is null");
    if (plan) SPX_TRY(spx_check_plan(plan, A.dtype));
    hipStream_t s = (hipStream_t)stream;
    const size_t vbytes = (size_t)A.n * value_size(A.dtype);
    SPX_TRY(ensure_conv(H));
    SPX_TRY(ensure_driver_counters(H));
    if (!H->pr_r) {
        if (hipMalloc(&H->pr_W, vbytes) != hipSuccess || hipMalloc(&H->pr_r, vbytes) != hipSuccess ||
            hipMalloc(&H->pr_y, vbytes) != hipSuccess ||
            hipMalloc((void**)&H->pr_xidx, (size_t)A.n * 4) != hipSuccess ||
            hipMalloc(&H->pr_xval, vbytes) != hipSuccess || hipMalloc(&H->pr_xd[0], vbytes) != hipSuccess ||
            hipMalloc(&H->pr_xd[1], vbytes) != hipSuccess || hipMalloc(&H->pr_p, vbytes) != hipSuccess ||
            hipMalloc((void**)&H->pr_bad, 4) != hipSuccess) {
            H->pr_r = nullptr;
            return fail(SPX_ERR_ALLOC, "PageRank buffers: allocation failed");
        }
    }
    PrArgs a;
    a.dtype = A.dtype;
    a.n = A.n;
    a.damping = damping;
    a.eps = eps;
    a.col_ptr = H->col_ptr;
    a.vals_csc = H->vals_csc;
    a.bad = H->pr_bad;
    a.W = H->pr_W;
    a.r = H->pr_r;
    a.p = H->pr_p;
    a.x_idx = H->pr_xidx;
    a.x_val = H->pr_xval;
    a.xd[0] = H->pr_xd[0];
    a.xd[1] = H->pr_xd[1];
    a.map = H->gorder ? H->grank : nullptr;
    a.count = H->drv_count;
    if (!H->pr_W_valid) {
        SPX_TRY(fill_u32(H->pr_bad, 0u, 1, s));
        a.stage = PR_NEGCHECK;
        a.nnz = A.nnz;
        SPX_TRY(launch_pagerank(a, s));
        // W = A^T 1: the balanced row-major SpMV over the CSC arrays read as
        // the CSR of A^T (its merge partition cached as the handle's second
        // one), x = ones in the second dense buffer (zeroed again by round 0)
        a.stage = PR_ONES;
        a.ones = H->pr_xd[1];
        SPX_TRY(launch_pagerank(a, s));
        const spx_csr At{A.n, A.m, A.nnz, A.dtype, H->col_ptr, H->row_idx, H->vals_csc};
        const spx_plan bal{SPX_PAT_SPMV, SPX_DIST_BALANCED, SPX_WB_NONE, 0, 0, 0};
        const int32_t* part = nullptr;
        SPX_TRY(cached_part(H, At, 1, &bal, s, &part));
        SPX_TRY(ensure_ws(H, ws_for(At.m, At.n, At.nnz, 0, A.dtype, &bal)));
        Arena ws(H->ws, H->ws_bytes);
        SPX_TRY(launch_spmv_csr(&At, H->pr_xd[1], nullptr, H->pr_W, &bal, part, ws, s));
        SPX_HIP(hipMemcpyAsync(H->drv_host, H->pr_bad, 4, hipMemcpyDeviceToHost, s));
        SPX_HIP(hipStreamSynchronize(s));
        if (H->drv_host[0]) return fail(SPX_ERR_ARG, "PageRank needs nonnegative edge weights");
        H->pr_W_valid = true;
    }
    a.stage = PR_INIT;
    SPX_TRY(launch_pagerank(a, s));
    SPX_TRY(fill_u32((uint32_t*)H->drv_count, 0u, 4, s));
    // Round k's counter is copied to pinned slot k & 1 and marked by an
    // event, so the host can wait for a round's select without waiting for
    // the product queued behind it.
    auto enqueue_select = [&](int32_t round) -> spx_status {
        a.stage = PR_SELECT;
        a.round = round;
        a.y = round ? H->pr_y : nullptr;
        SPX_TRY(launch_pagerank(a, s));
        SPX_HIP(hipMemcpyAsync(H->drv_host + 4 * (round & 1), H->drv_count + 2 * (round & 1), 8,
                               hipMemcpyDeviceToHost, s));
        SPX_HIP(hipEventRecord(H->drv_ev[round & 1], s));
        return SPX_OK;
    };
    auto choose = [&](int32_t nx, int64_t ns, spx_plan* q) -> spx_status {
        if (plan) {
            *q = *plan;
            return SPX_OK;
        }
        spx_vec xs{SPX_VEC_SPARSE, A.n, nx, H->pr_xidx, H->pr_xval};
        return select_counts(H, &xs, ns, s, q);
    };
    // A row-major product reads the dense x and needs no count on the host,
    // so while the plans stay row-major the next round's product is queued
    // right behind its select, on the plan the last count chose, and the
    // GPU does not wait for the host between rounds. A column-major plan
    // needs the exact count: such a round waits for its select first.
    int32_t it = 0;
    bool pending = false;  // a product not yet folded into r
    bool spec = false;     // this round's product was queued before its count was read
    spx_plan spec_plan{};
    for (int32_t round = 0; it < max_iters;) {
        if (round == 0) SPX_TRY(enqueue_select(0));
        SPX_HIP(hipEventSynchronize(H->drv_ev[round & 1]));
        const int32_t nx = H->drv_host[4 * (round & 1)];
        const int64_t ns = H->drv_host[4 * (round & 1) + 1];  // column lengths of supp(x)
        spx_plan p{};
        if (spec) {
            // an empty x gave y = 0: nothing to count and nothing to fold
            if (nx == 0) {
                pending = false;
                break;
            }
            p = spec_plan;
        } else {
            pending = false;
            if (nx == 0) break;
            SPX_TRY(choose(nx, ns, &p));
            spx_vec x{SPX_VEC_SPARSE, A.n, nx, H->pr_xidx, H->pr_xval};
            SPX_TRY(exec_prepared(H, &x, H->pr_xd[round & 1], H->pr_y, &p, ns, s));
        }
        if (it < plans_cap) plans[it] = p;
        ++it;
        pending = true;
        if (it >= max_iters) break;
        ++round;
        SPX_TRY(enqueue_select(round));
        spec = false;
        if (p.pattern != SPX_PAT_CSC_SPMSPV) {
            spx_plan q{};
            SPX_TRY(choose(nx, ns, &q));
            if (q.pattern != SPX_PAT_CSC_SPMSPV) {
                spx_vec xd_only{SPX_VEC_SPARSE, A.n, 0, H->pr_xidx, H->pr_xval};
                SPX_TRY(exec_prepared(H, &xd_only, H->pr_xd[round & 1], H->pr_y, &q, -1, s));
                spec = true;
                spec_plan = q;
            }
        }
    }
    if (pending) {
        a.stage = PR_FOLD;
        a.y = H->pr_y;
        SPX_TRY(launch_pagerank(a, s));
    }
    SPX_HIP(hipMemcpyAsync(rank, H->pr_p, vbytes, hipMemcpyDeviceToDevice, s));
    if (residual) SPX_HIP(hipMemcpyAsync(residual, H->pr_r, vbytes, hipMemcpyDeviceToDevice, s));
    *n_iters = it;
    return SPX_OK;
}

// ------------------------------------------------------------------ backward
extern "C" spx_status spmv_csr_batch(spx_matrix* H, int32_t B, const void* X, void* Y, void* stream) {
    if (!H || (B > 0 && (!X || !Y))) return fail(SPX_ERR_ARG, "null argument");
    if (B < 0) return fail(SPX_ERR_SHAPE, "B must be >= 0");
    const int dt = H->csr.dtype;
    if (dt != SPX_F32 && dt != SPX_F64) return fail(SPX_ERR_DTYPE, "the fused batch SpMV supports F32 and F64");
    SPX_TRY(ensure_ws(H, grad_ws_bytes(H->csr.m, H->csr.n, B, dt)));
    Arena ws(H->ws, H->ws_bytes);
    return launch_spmv_batch(H->csr.row_ptr, H->csr.col_idx, H->csr.vals, H->csr.m, H->csr.n, dt, B, X, Y, ws,
                             (hipStream_t)stream);
}

extern "C" spx_status spmv_csr_transpose(spx_matrix* H, int32_t B, const void* G, void* dX, void* stream) {
    if (!H || (B > 0 && (!G || !dX))) return fail(SPX_ERR_ARG, "null argument");
    if (B < 0) return fail(SPX_ERR_SHAPE, "B must be >= 0");
    const int dt = H->csr.dtype;
    if (dt != SPX_F32 && dt != SPX_F64) return fail(SPX_ERR_DTYPE, "backward supports F32 and F64");
    SPX_TRY(ensure_ws(H, grad_ws_bytes(H->csr.m, H->csr.n, B, dt)));
    Arena ws(H->ws, H->ws_bytes);
    return launch_dx(H->col_ptr, H->row_idx, H->vals_csc, H->csr.m, H->csr.n, dt, B, G, dX, ws,
                     (hipStream_t)stream);
}

extern "C" spx_status dvals_pattern(spx_matrix* H, int32_t B, const void* G, const void* X, void* dvals,
                                    void* stream) {
    if (!H || (B > 0 && (!G || !X)) || (H->csr.nnz > 0 && !dvals)) return fail(SPX_ERR_ARG, "null argument");
    if (B < 0) return fail(SPX_ERR_SHAPE, "B must be >= 0");
    const int dt = H->csr.dtype;
    if (dt != SPX_F32 && dt != SPX_F64) return fail(SPX_ERR_DTYPE, "backward supports F32 and F64");
    SPX_TRY(ensure_ws(H, grad_ws_bytes(H->csr.m, H->csr.n, B, dt)));
    Arena ws(H->ws, H->ws_bytes);
    return launch_dvals(H->csr.row_ptr, H->csr.col_idx, H->csr.m, H->csr.n, H->csr.nnz, dt, B, G, X, dvals, ws,
                        (hipStream_t)stream);
}

extern "C" spx_status spx_backward(spx_matrix* H, int32_t B, const void* G, const void* X, void* dX, void* dvals,
                                   void* stream) {
    if (!H || (B > 0 && (!G || (dvals && !X))) || (!dX && !dvals)) return fail(SPX_ERR_ARG, "null argument");
    if (B < 0) return fail(SPX_ERR_SHAPE, "B must be >= 0");
    const int dt = H->csr.dtype;
    if (dt != SPX_F32 && dt != SPX_F64) return fail(SPX_ERR_DTYPE, "backward supports F32 and F64");
    SPX_TRY(ensure_ws(H, grad_ws_bytes(H->csr.m, H->csr.n, B, dt)));
    Arena ws(H->ws, H->ws_bytes);
    return launch_backward(H->csr.row_ptr, H->csr.col_idx, H->col_ptr, H->row_idx, H->vals_csc, H->csr.m, H->csr.n,
                           H->csr.nnz, dt, B, G, X, dX, dvals, ws, (hipStream_t)stream);
}

extern "C" spx_status spx_pack_mask(int32_t m, const uint8_t* rows, uint32_t* words, void* stream) {
    if (m < 0) return fail(SPX_ERR_SHAPE, "m must be >= 0");
    if (m == 0) return SPX_OK;
    if (!rows || !words) return fail(SPX_ERR_ARG, "null argument");
    k_dense_bits<SPX_BOOL><<<dense_bits_grid(m), kBlock, 0, (hipStream_t)stream>>>(m, rows, words);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

extern "C" spx_status spx_dense_rows_to_sparse(spx_matrix* H, int32_t B, const void* X, int32_t* vec_ptr,
                                               int32_t* idx, void* val, void* stream) {
    if (!H || (B > 0 && (!X || !vec_ptr || !idx || (H->csr.dtype != SPX_BOOL && !val))))
        return fail(SPX_ERR_ARG, "null argument");
    if (B < 0) return fail(SPX_ERR_SHAPE, "B must be >= 0");
    if (H->csr.dtype == SPX_F32_MINPLUS) return fail(SPX_ERR_DTYPE, "dense rows: the batched path has no min-plus");
    SPX_TRY(ensure_ws(H, dense_rows_ws_bytes(B, H->csr.n)));
    Arena ws(H->ws, H->ws_bytes);
    return dense_rows_to_sparse(B, H->csr.n, H->csr.dtype, X, vec_ptr, idx, val, ws, (hipStream_t)stream);
}
