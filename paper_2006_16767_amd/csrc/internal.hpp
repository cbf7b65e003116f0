// Host-side launchers shared between the translation units of libspx.
// Not part of the public ABI (include/spx.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/spx.h"
#include "selector.hpp"

namespace spx {

// Thread-local error message; returns code so call sites can `return fail(...)`.
spx_status fail(spx_status code, const std::string& msg);
spx_status hip_fail(hipError_t e, const char* what);

#define SPX_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

#define SPX_TRY(call)                     \
    do {                                  \
        spx_status s_ = (call);           \
        if (s_ != SPX_OK) return s_;      \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int value_size(int dtype);  // bytes per A / x value (0 for BOOL)
uint32_t zero_word(int dtype);  // the semiring's zero as a 32-bit word (+inf for min-plus, else 0)
int out_size(int dtype);    // bytes per y element (1 for BOOL)

// Bump allocator over a caller-provided workspace.
struct Arena {
    char* base;
    size_t size;
    size_t used = 0;
    Arena(void* b, size_t s) : base((char*)b), size(s) {}
    template <typename T>
    T* take(size_t count) {
        size_t off = align_up(used, 256);
        size_t need = off + align_up(count * sizeof(T), 256);
        if (!base || need > size) return nullptr;
        used = need;
        return (T*)(base + off);
    }
};
// Sizing twin of Arena: counts what a sequence of take() calls needs.
struct Sizer {
    size_t used = 0;
    template <typename T>
    void take(size_t count) {
        used = align_up(used, 256) + align_up(count * sizeof(T), 256);
    }
};

// ----------------------------------------------------------------- primitives
spx_status fill_bytes(void* p, uint8_t v, size_t bytes, hipStream_t s);
spx_status fill_u32(uint32_t* p, uint32_t v, size_t count, hipStream_t s);

// Exclusive scan of n int32 (in may equal out). Writes the total to
// *total_dev if not null. Workspace: scan_ws_elems(n) int32.
size_t scan_ws_elems(int64_t n);
spx_status scan_exclusive_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev,
                              int32_t* ws, hipStream_t s);

// Stable LSD radix sort of (key, value) uint32 pairs on the low `bits` bits
// of the key. keys/vals are sorted in place using the alternate buffers.
size_t radix_ws_elems(int64_t n);
spx_status radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                            uint32_t* vals_alt, int64_t n, int bits, int32_t* ws,
                            hipStream_t s, bool* result_in_alt);

// row id of every CSR position
spx_status expand_rows(const int32_t* row_ptr, int32_t m, int32_t* rows_out, hipStream_t s);
// out[p] = in[perm[p]] for element size esize (4 or 8)
spx_status gather_perm(const void* in, const int32_t* perm, void* out, int64_t n, int esize,
                       hipStream_t s);

// ------------------------------------------------------------------ kernels
// Positions a sparse x was scattered to (map[idx[e]], or idx[e] when map is
// null) in a bitvector and / or a dense x buffer. The balanced row-major
// launch clears them again in its fix-up pass, after the product has read
// them, so that the buffers are back at zero (the semiring's zero for xd)
// for the next conversion, which then needs no fill.
struct Unscatter {
    int32_t nnz_x = 0;
    const int32_t* idx = nullptr;
    const int32_t* map = nullptr;
    uint32_t* bits = nullptr;  // whole words are zeroed
    void* xd = nullptr;
    int32_t n = 0;  // length of x: past n / 16 entries the whole buffers are cleared with coalesced stores
};

// Column-sorted copy of a CSR for the balanced SpMV with 2048-item merge
// tiles (csr_tile.hpp: inside each tile the entries ordered by column, each
// word = column | position in the tile << 21; needs n <= 2^21).
struct TileSorted {
    uint32_t* pk = nullptr;  // [nnz]
    void* vals = nullptr;    // [nnz] (none for BOOL)
    int32_t* src = nullptr;  // [nnz] position in the original CSR (value refresh)
};

// part: merge-path partition of the balanced distribution (null: computed
// into the workspace on this call). un (optional): positions to clear after
// the product; *cleared (optional) tells whether they were (only the
// balanced distribution has the pass that does it). ts (optional): the
// column-sorted copy of A, which the balanced row-major kernels with
// 2048-item tiles (SpMV and the bitvector SpMSpV, LDS bitvector aside) then
// read instead of A's column indices and values.
spx_status launch_spmv_csr(const spx_csr* A, const void* x, const uint32_t* bits, void* y,
                           const spx_plan* plan, const int32_t* part, Arena& ws, hipStream_t s,
                           const Unscatter* un = nullptr, bool* cleared = nullptr,
                           const TileSorted* ts = nullptr);
// Builds ts for A (the partition of 2048-item tiles given); returns
// SPX_ERR_UNSUPPORTED when n > 2^21. Synchronizes the stream.
spx_status tile_sorted_build(const spx_csr& A, const int32_t* part, const int32_t* src_of_A, TileSorted* ts,
                             hipStream_t s);
void tile_sorted_free(TileSorted* ts);
spx_status merge_partition(int32_t m, int32_t nnz, const int32_t* row_ptr, int tile, int32_t* part,
                           hipStream_t s);
size_t spmv_csr_ws(int32_t m, int32_t nnz, const spx_plan* plan);

// Read-only view of excl[0..nnz_x]: either one array (off null), or the
// exclusive prefix within each run of 256 entries (local) plus the
// exclusive prefix of the run totals (off), as the one-launch length scan
// leaves it.
struct Excl {
    const int32_t* local;
    const int32_t* off;
    __device__ __forceinline__ int32_t operator[](int64_t e) const {
        return off ? local[e] + off[e >> 8] : local[e];
    }
    __host__ __device__ explicit operator bool() const { return local != nullptr; }
};

// Sparse output of the column-major SpMSpV (bucket write-back only): the
// rows that an effective entry reaches and whose bit in mask is clear
// (mask nullptr: none masked) go to idx / val (val may be nullptr;
// capacity m), ascending within each bucket of rows, buckets in any order;
// *count (device, zeroed by the caller) receives their number.
struct SparseOut {
    const uint32_t* mask;
    int32_t* idx;
    void* val;
    int32_t* count;
};
// host-side checks of a CSC descriptor (api.hip)
spx_status check_csc(const spx_csc* A);
struct CscArgs {
    int32_t m, n, nnz, dtype;
    const int32_t* col_ptr;
    const int32_t* row_idx;
    const void* vals;
    const int32_t* row_ptr;  // CSR row pointer of the same matrix (bucket layout); may be null
    uint32_t* scan_counter;  // handle-owned, zero between calls (the scan resets it); may be null
    int64_t nnz_s_hint;      // exact nnz_s if the host knows it, else -1
    const SparseOut* sparse = nullptr;  // sparse output instead of a dense y
};
spx_status launch_spmspv_csc(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx,
                             const void* x_val, void* y, const spx_plan* plan, Arena& ws,
                             hipStream_t s);
size_t spmspv_csc_ws(int32_t m, int32_t n, int32_t nnz, int32_t nnz_x, int dtype,
                     const spx_plan* plan);
// bucket write-back (spmspv_bucket.hip); excl = prefix of selected column lengths
// the direct bucket write-back for a short x: one launch, no prefix, no fill
bool csc_bucket_walks(const CscArgs& A, int32_t nnz_x, const spx_plan* plan);
spx_status launch_csc_bucket_walk(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val, void* y,
                                  const spx_plan* plan, hipStream_t s);
spx_status launch_csc_bucket(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                             void* y, const spx_plan* plan, const Excl excl, Arena& ws,
                             hipStream_t s);
size_t csc_bucket_ws(int32_t m, int32_t nnz, int32_t nnz_x, int dtype, const spx_plan* plan);
// merge write-back (spmspv_merge.hip); excl as for the bucket
spx_status launch_csc_merge(const CscArgs& A, int32_t nnz_x, const int32_t* x_idx, const void* x_val, void* y,
                            const spx_plan* plan, const Excl excl, Arena& ws, hipStream_t s);
size_t csc_merge_ws(int32_t m, int32_t nnz, int32_t nnz_x, int dtype, const spx_plan* plan);

// sparse x -> bitvector of supp(x) (cleared first unless `clean` says it
// is all zero already) + scattered values xd[n] (map, if given, renumbers
// the columns: entry j lands at map[j])
spx_status sparse_to_bitvector(int32_t n, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                               int dtype, const int32_t* map, uint32_t* bits, void* xd, hipStream_t s,
                               bool clean = false);
// sparse x -> dense x filled with the semiring's zero (skipped when `clean`
// says xd holds it already; map as above)
spx_status sparse_to_dense(int32_t n, int32_t nnz_x, const int32_t* x_idx, const void* x_val,
                           int dtype, const int32_t* map, void* xd, hipStream_t s, bool clean = false);
// dense x -> xg[r] = x[order[r]], plus the bitvector of xg's nonzeros if bits
spx_status permute_dense(int32_t n, const void* x, int dtype, const int32_t* order, void* xg, uint32_t* bits,
                         hipStream_t s);
// dense x -> (idx, val) of its nonzeros in index order; count to *nnz_dev
size_t compact_ws_elems(int32_t n);
spx_status dense_to_sparse(int32_t n, const void* x, int dtype, int32_t* idx, void* val,
                           int32_t* nnz_dev, int32_t* ws, hipStream_t s);

// features
struct MatrixStats {
    double f[9];
};
spx_status matrix_features_device(const int32_t* row_ptr, int32_t m, int32_t n,
                                  MatrixStats* out, hipStream_t s);
// nnz_s (and nnz_x for a dense x) on the device into out2[0..1] (int64)
// nnz_s (and a dense x's nonzero count) in one launch, written to host-visible
// host2[0..1]; acc2 (2 counters) and ticket must be zero and are left zero
spx_status vector_counts_to_host(const int32_t* col_ptr, int32_t n, const spx_vec* x, int dtype,
                                 unsigned long long* acc2, uint32_t* ticket, long long* host2, hipStream_t s);
spx_status vector_features_device(const int32_t* col_ptr, int32_t n, const spx_vec* x, int dtype,
                                  int64_t* out2_dev, hipStream_t s);

// batched SpMSpV (batch.hip)
constexpr int kDevTreeNodes = 512;
struct DevTree {
    int32_t n;
    int32_t feat[kDevTreeNodes], left[kDevTreeNodes], right[kDevTreeNodes], cls[kDevTreeNodes];
    double thr[kDevTreeNodes];
};
// t[0] pattern, t[1 + pattern] distribution, t[4] write-back; mfeat = the
// nine matrix features of Table 1
struct DevSelector {
    DevTree t[5];
    double mfeat[9];
    int32_t needs_nnz_s;  // a tree reads nnz_s, m_sparsity or s_per_x
};
void upload_tree(const Tree& t, DevTree* out);
struct BatchLaunch {
    spx_csr csr;
    const int32_t* col_ptr;
    const int32_t* row_idx;
    const void* vals_csc;
    const int32_t* part;  // merge-path partition of A at tile 2048
    int64_t tiles_mat;
    int32_t B;
    int64_t cap_nnz_x;
    const int32_t* vec_ptr;
    const int32_t* idx;
    const void* val;
    void* Y;
    const DevSelector* sel;
    int32_t row_lanes;
    int32_t persistent_grid;
    // work units of A for the fused row-major groups (null: no fusion): at
    // most kFusedUnitNnz entries of at most kFusedUnitRows whole rows, or a
    // piece of a row longer than kFusedUnitNnz
    const int32_t* units;  // 4 ints per unit
    int32_t nunits;
    const int32_t* split_rows;
    int32_t nsplit;
    // while the launches are captured: a second stream and two events that
    // put the fused groups' walk on a branch of its own, beside the
    // per-vector tiles (null: one stream)
    hipStream_t side;
    hipEvent_t fork, join;
};
constexpr int kFusedUnitNnz = 512;
constexpr int kFusedUnitRows = 63;
size_t batch_ws_size(int32_t m, int32_t n, int dtype, int32_t B, int64_t cap_nnz_x, int64_t tiles_mat,
                     size_t* zero_from, size_t* zero_bytes);
spx_status launch_batch(const BatchLaunch& L, void* ws, size_t ws_bytes, hipStream_t s, int32_t** err_dev);

// breadth-first search (bfs.hip). count points at two packed 64-bit
// frontier counters {vertices (low half), their out-degrees (high half)},
// read on the host as two int32 words (little-endian); level L appends
// into count[L & 1] and clears the other. The bitvectors hold
// ceil(n / 32) words.
spx_status launch_bfs_seed(int32_t n, int32_t source, const int32_t* col_ptr, int32_t* level, int32_t* frontier,
                           uint32_t* bits, void* count, hipStream_t s);
spx_status launch_bfs_update(int32_t n, const uint8_t* y, int32_t L, const int32_t* col_ptr, int32_t* level,
                             int32_t* next, uint32_t* next_bits, void* count, hipStream_t s);
spx_status launch_bfs_pull(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const uint32_t* bits,
                           int32_t L, const int32_t* col_ptr, int32_t* level, int32_t* next, uint32_t* next_bits,
                           void* count, hipStream_t s);

// incremental PageRank (pagerank.hip): one launch per stage. count: two
// packed counters as for breadth-first search, {entries appended to x,
// their column lengths}; round s appends into count[s & 1], clears the
// other.
enum PrStage { PR_NEGCHECK, PR_ONES, PR_INIT, PR_SELECT, PR_FOLD };
struct PrArgs {
    int stage = PR_INIT;
    int dtype = SPX_F32;
    int32_t n = 0;
    int32_t round = 0;
    double damping = 0.85, eps = 0.0;
    int64_t nnz = 0;
    const int32_t* col_ptr = nullptr;  // CSC column pointers
    const void* vals_csc = nullptr;    // NEGCHECK
    uint32_t* bad = nullptr;           // NEGCHECK: bit 0 = negative weight
    void* ones = nullptr;              // ONES: n values set to 1
    void* W = nullptr;                 // column sums
    void* r = nullptr;                 // residual
    void* p = nullptr;                 // rank
    const void* y = nullptr;           // last product (nullptr on round 0)
    int32_t* x_idx = nullptr;          // next product's input: list,
    void* x_val = nullptr;
    void* xd[2] = {nullptr, nullptr};  // dense (alternating, 16-byte aligned),
    const int32_t* map = nullptr;      // at map[v] (nullptr: v)
    void* count = nullptr;
};
spx_status launch_pagerank(const PrArgs& a, hipStream_t s);

// backward (grad.hip): workspace grad_ws_bytes(m, n, B, dtype)
size_t grad_ws_bytes(int32_t m, int32_t n, int32_t B, int dtype);
spx_status launch_spmv_batch(const int32_t* row_ptr, const int32_t* col_idx, const void* vals, int32_t m,
                             int32_t n, int dtype, int32_t B, const void* X, void* Y, Arena& ws, hipStream_t s);
spx_status launch_dx(const int32_t* col_ptr, const int32_t* row_idx, const void* vals_csc, int32_t m,
                     int32_t n, int dtype, int32_t B, const void* G, void* dX, Arena& ws, hipStream_t s);
spx_status launch_backward(const int32_t* row_ptr, const int32_t* col_idx, const int32_t* col_ptr,
                           const int32_t* row_idx, const void* vals_csc, int32_t m, int32_t n, int32_t nnz, int dtype,
                           int32_t B, const void* G, const void* X, void* dX, void* dvals, Arena& ws, hipStream_t s);
spx_status launch_dvals(const int32_t* row_ptr, const int32_t* col_idx, int32_t m, int32_t n,
                        int32_t nnz, int dtype, int32_t B, const void* G, const void* X,
                        void* dvals, Arena& ws, hipStream_t s);
// B dense rows of length n -> CSR-of-vectors (vec_ptr[B+1], idx, val);
// ws_i32: scan_ws_elems(B + 1) int32
spx_status dense_rows_to_sparse(int32_t B, int32_t n, int dtype, const void* X, int32_t* vec_ptr,
                                int32_t* idx, void* val, Arena& ws, hipStream_t s);
size_t dense_rows_ws_bytes(int32_t B, int32_t n);

// ------------------------------------------------------------------ sliced ELL
// SELL-C-sigma copy of A (C = 64 rows per slice, rows sorted by descending
// length inside windows of kSellSigma rows); see sell.hip for the layout.
constexpr int32_t kSellSigma = 4096;
struct SellMat {
    int64_t nslices = 0;
    int64_t padded = 0;           // stored cells, padding included
    int64_t* slice_ptr = nullptr;  // [nslices + 1], cells before each slice
    int32_t* perm = nullptr;       // [nslices * 64], row of each slot or -1
    int32_t* col = nullptr;        // [padded], -1 for padding
    int32_t* src = nullptr;        // [padded], CSR position or -1
    void* vals = nullptr;          // [padded] (none for BOOL)
};
// The slot order and slice widths, computed on the host from row_ptr.
struct SellPlanInfo {
    int64_t nslices = 0;
    int64_t padded = 0;
    std::vector<int32_t> perm;
    std::vector<int64_t> slice_ptr;
};
SellPlanInfo sell_shape(const int32_t* row_ptr_host, int32_t m);
spx_status sell_build(const spx_csr& A, const SellPlanInfo& info, SellMat* out, hipStream_t s);
spx_status sell_refresh(const SellMat& S, const spx_csr& A, hipStream_t s);
void sell_free(SellMat* S);
spx_status sell_spmv(const SellMat& S, int dtype, const void* x, void* y, hipStream_t s);

// ELL copy of A: rows padded to the longest, column-major (entry j of row i
// at j * m + i); see sell.hip.
struct EllMat {
    int32_t m = 0;
    int32_t width = 0;        // longest row
    int64_t cells = 0;        // width * m
    int32_t* col = nullptr;   // [cells], -1 for padding
    int32_t* src = nullptr;   // [cells], CSR position or -1
    void* vals = nullptr;     // [cells] (none for BOOL)
};
spx_status ell_build(const spx_csr& A, int32_t width, EllMat* out, hipStream_t s);
spx_status ell_refresh(const EllMat& E, const spx_csr& A, hipStream_t s);
void ell_free(EllMat* E);
spx_status ell_spmv(const EllMat& E, int dtype, const void* x, void* y, hipStream_t s);

// DIA copy of A: at most kDiaMax diagonals (ascending offsets col - row),
// cell (d, i) at d * m + i with a presence bit; see dia.hip.
constexpr int kDiaMax = 32;
struct DiaMat {
    int32_t m = 0, n = 0;
    int nd = 0;                // diagonals
    int64_t cells = 0;         // nd * m
    int64_t words = 0;         // presence words per diagonal
    int32_t* offs = nullptr;   // [nd]
    void* vals = nullptr;      // [cells]
    uint32_t* mask = nullptr;  // [nd * words]
};
// Builds the copy when A's entries lie on at most kDiaMax diagonals and it
// moves fewer bytes than CSR; otherwise leaves *out empty and returns
// SPX_OK (or, when forced, SPX_ERR_UNSUPPORTED).
spx_status dia_try_build(const spx_csr& A, int32_t max_row, bool forced, DiaMat* out, hipStream_t s);
spx_status dia_refresh(const DiaMat& D, const spx_csr& A, hipStream_t s);
void dia_free(DiaMat* D);
spx_status dia_spmv(const DiaMat& D, int dtype, const void* x, void* y, hipStream_t s);

// CSR5-style copy of A: tiles of 64 lanes x 16 consecutive entries stored
// transposed, with row-start bits per lane and the non-empty rows listed;
// see csr5.hip.
struct Csr5Mat {
    int32_t m = 0, nnz = 0;
    int64_t ntiles = 0;
    int64_t cells = 0;             // ntiles * tile size (the last tile padded)
    int32_t nonempty = 0, nempty = 0;
    int32_t* col = nullptr;        // [cells]
    void* vals = nullptr;          // [cells] (none for BOOL)
    uint32_t* flags = nullptr;     // [ntiles * 64] row-start bits per lane
    int32_t* tile_start = nullptr; // [ntiles + 1] ordinal of the tile's first row start
    int32_t* nz_rows = nullptr;    // [nonempty] ordinal -> row
    int32_t* empty_rows = nullptr; // [nempty]
    void* lead = nullptr;          // [ntiles] accumulators written by each call
    void* trail = nullptr;         // [ntiles]
};
int64_t csr5_cells(int32_t nnz);
spx_status csr5_build(const spx_csr& A, const int32_t* row_ptr_host, Csr5Mat* out, hipStream_t s);
spx_status csr5_refresh(const Csr5Mat& C, const spx_csr& A, hipStream_t s);
void csr5_free(Csr5Mat* C);
spx_status csr5_spmv(const Csr5Mat& C, int dtype, const void* x, void* y, hipStream_t s);
// The bitvector SpMSpV over the CSR5 tiles with the bitvector in LDS (n <=
// 2^20): x dense (read only where the bit is set), bits 16-byte aligned; the
// bitvector is all zero again after the call.
bool csr5_lds_fits(int32_t n);
spx_status csr5_spmspv(const Csr5Mat& C, int dtype, int32_t n, const void* x, uint32_t* bits, void* y,
                       hipStream_t s);

}  // namespace spx
