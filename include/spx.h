/*
 * spx: adaptive SpMV / SpMSpV for AMD MI355X (gfx950).
 *
 * C ABI of the library libspx.so. Plain C types and pointers only.
 *
 * The operation (Section 2 of Li, Ao, Yang, "Adaptive SpMV/SpMSpV on GPUs
 * for Input Vectors of Varied Sparsity"): A is an m-by-n sparse matrix
 * with nnz stored entries, x is a vector of length n, given either dense
 * (one array of n values) or sparse (nnz_x indices and nnz_x values), and
 * every entry point computes the dense output
 *
 *        y = A x        (y has length m and is overwritten, never added to)
 *
 * The library holds a family of kernels that differ along the paper's
 * axes (Section 4): computing pattern (row-major SpMV, row-major SpMSpV
 * with value validation, column-major SpMSpV), workload distribution
 * (direct or load-balanced) and, for the column-major pattern, write-back
 * (atomic, sort, plus an LDS-privatized atomic and a bucket write-back).
 * A three-step decision-tree cascade (Section 5, Section 6.2) picks one
 * per input vector at run time.
 *
 * Conventions for every entry point:
 *  - Pointers named dev_* or documented as "device" point to GPU memory
 *    that the caller allocated (e.g. with PyTorch) and still owns. The
 *    library never frees caller memory.
 *  - Indices are int32; nnz < 2^31. A CSR matrix has row_ptr[m+1]
 *    (row_ptr[0] = 0, non-decreasing) and col_idx[nnz] in [0, n); column
 *    indices within a row are unique (any order is accepted by every
 *    kernel). Sparse vectors have unique indices in [0, n), any order.
 *  - Value types (spx_dtype): F32 and F64 (real (+, *)), I32 ((+, *)
 *    modulo 2^32, bit-exact), BOOL ((OR, AND): A is its pattern and vals
 *    are ignored (may be NULL); a sparse x is the index set and x values
 *    are ignored (may be NULL); a dense x is uint8 0/1; y is uint8 0/1).
 *  - Explicit zeros stored in A or in a sparse x are structural: they are
 *    part of the pattern (an "effective nonzero" is any stored A entry in
 *    a column that x lists, Section 2).
 *  - Rows with no effective entry are written as exact +0 (0 for I32 and
 *    BOOL).
 *  - Every launch is enqueued on the caller's stream (a hipStream_t passed
 *    as void*; NULL is the default stream) and returns without waiting,
 *    except where a function says it synchronizes.
 *  - A handle's scratch (conversion buffers, workspace, driver state) is
 *    shared by all its calls, and it tracks what earlier calls left there
 *    (e.g. a conversion buffer cleared by the last product): calls on one
 *    handle must be ordered, on one stream or with the caller
 *    synchronizing between streams. Different handles are independent.
 *  - Every function returns an spx_status (0 on success, negative on
 *    error); nothing aborts and no C++ exception crosses the boundary.
 *    spx_last_error() returns a thread-local message for the last error.
 *    Faults inside a kernel surface at the next synchronizing call as
 *    SPX_ERR_HIP.
 *  - Floating-point results: FP32 kernels satisfy
 *    |y_i - exact_i| <= 1e-5 * sum_j |a_ij x_j|, FP64 kernels
 *    1e-12 * sum_j |a_ij x_j|; the order of accumulation is unspecified.
 *    The row-major patterns and the sort and merge write-backs give the
 *    same bits on every call; the atomic, LDS-atomic and bucket
 *    write-backs add a row's products in the order the hardware serves
 *    the atomics, so their last bits can differ between calls. Those three
 *    also sum a row in one serial FP32 chain: the bound holds for rows of
 *    up to about 2^16 entries (run() avoids them in FP32 beyond that).
 */
#ifndef SPX_H
#define SPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int spx_status;
#define SPX_OK 0
#define SPX_ERR_ARG (-1)          /* null pointer, negative size, bad enum value */
#define SPX_ERR_SHAPE (-2)        /* sizes that do not agree (e.g. x length != n) */
#define SPX_ERR_INDEX (-3)        /* an index out of range (validation mode only) */
#define SPX_ERR_DTYPE (-4)        /* dtype not supported by this entry point */
#define SPX_ERR_UNSUPPORTED (-5)  /* plan not available for these inputs */
#define SPX_ERR_ALLOC (-6)        /* device or host allocation failed */
#define SPX_ERR_HIP (-7)          /* a HIP runtime call failed */
#define SPX_ERR_WORKSPACE (-8)    /* workspace missing or smaller than required */

/* Value type and semiring of a handle. SPX_F32_MINPLUS is (min, +) over
 * float32 (the shortest-path relaxation; a semiring beyond the paper's):
 * y_i = min over the effective entries (i, j) of (a_ij + x_j), each sum one
 * float32 addition, +inf where none is effective; a dense x marks an absent
 * entry by +inf (the semiring's zero), a sparse x lists the present ones.
 * It runs the row- and column-major kernels of run()/run_plan() and the
 * sparse output; the batched path, the backward and the graph drivers
 * refuse it (SPX_ERR_DTYPE). */
typedef enum { SPX_F32 = 0, SPX_F64 = 1, SPX_BOOL = 2, SPX_I32 = 3, SPX_F32_MINPLUS = 4 } spx_dtype;

/* Computing pattern (Section 4.1). */
typedef enum {
    SPX_PAT_SPMV = 0,       /* row-major, matrix-driven, no validation: dense x */
    SPX_PAT_CSR_SPMSPV = 1, /* row-major, matrix-driven, validation by bitvector */
    SPX_PAT_CSC_SPMSPV = 2  /* column-major, vector-driven: visits effective entries only */
} spx_pattern;

/* Workload distribution (Section 4.2.1). Balanced tiles hold 2048 merge
 * items (tile = 0 or 2048) or 4096 (tile = 4096). For the balanced row-major
 * SpMSpV, tile = 1 keeps the bitvector of supp(x) in LDS instead (persistent
 * workgroups; n up to about 1.17M for FP32 or 1.1M for FP64, otherwise the
 * 2048 kernel); and through a handle whose SpMV format is CSR5 (n <=
 * 2^20), tile = 0 runs over the CSR5 tiles of 64 x 16 entries with the
 * bitvector in LDS, every wave of a persistent workgroup on its own tiles
 * with the next tile's indices in flight (tile = 2048 keeps the merge
 * tiles). */
typedef enum {
    SPX_DIST_DIRECT = 0,  /* a fixed group of `lanes` threads per row (per column for CSC) */
    SPX_DIST_BALANCED = 1 /* merge-path tiles with equal (rows + entries) per workgroup */
} spx_distribution;

/* Write-back of the column-major pattern (Section 4.2.2). NONE, SORT and
 * MERGE add each row's products in a fixed order, so a floating-point y
 * repeats bit for bit from call to call; ATOMIC, LDS_ATOMIC and BUCKET add
 * them in the order the hardware serves the atomics, so its last bits may
 * differ between calls (integer and Boolean results never do). */
typedef enum {
    SPX_WB_NONE = 0,       /* row-major patterns: each row written once, no conflict */
    SPX_WB_ATOMIC = 1,     /* zero y, then hardware atomic add per effective entry */
    SPX_WB_SORT = 2,       /* write (row, value) pairs, radix-sort by row, reduce by key */
    SPX_WB_LDS_ATOMIC = 3, /* per-workgroup copy of y in LDS, flushed with atomics (small m) */
    SPX_WB_BUCKET = 4,     /* bin pairs by row range, one workgroup per bucket sums in LDS */
    SPX_WB_MERGE = 5       /* sort each tile's pairs in LDS and sum them by row, then merge the
                              tiles' sorted runs per range of rows (no atomics) */
} spx_writeback;

/* One candidate kernel plus its launch parameters. Zero parameters mean
 * "choose automatically". */
typedef struct {
    int32_t pattern;      /* spx_pattern */
    int32_t distribution; /* spx_distribution */
    int32_t writeback;    /* spx_writeback; SPX_WB_NONE for row-major patterns */
    int32_t lanes;        /* direct: threads per row/column, power of two in [1, 64]; 0 = auto */
    int32_t tile;         /* balanced: items per 256-thread workgroup tile; 0 = auto */
    int32_t bucket_rows;  /* bucket write-back: rows per bucket, power of two; 0 = auto */
} spx_plan;

/* A CSR matrix (device arrays, caller-owned). */
typedef struct {
    int32_t m, n, nnz;
    int32_t dtype;          /* spx_dtype */
    const int32_t *row_ptr; /* device, m + 1 */
    const int32_t *col_idx; /* device, nnz */
    const void *vals;       /* device, nnz values of dtype; ignored for BOOL */
} spx_csr;

/* A CSC matrix (device arrays): col_ptr[n+1], row_idx[nnz], vals[nnz]. */
typedef struct {
    int32_t m, n, nnz;
    int32_t dtype;
    const int32_t *col_ptr;
    const int32_t *row_idx;
    const void *vals;
} spx_csc;

typedef enum { SPX_VEC_DENSE = 0, SPX_VEC_SPARSE = 1 } spx_vec_kind;

/* An input vector x of length n (Section 2: dense = one array of n values;
 * sparse = nnz_x indices plus nnz_x values). Device arrays, caller-owned. */
typedef struct {
    int32_t kind;        /* spx_vec_kind */
    int32_t n;
    int32_t nnz_x;       /* sparse: number of entries; dense: ignored (-1 ok) */
    const int32_t *idx;  /* sparse: device, nnz_x indices */
    const void *val;     /* dense: device, n values; sparse: device, nnz_x values */
} spx_vec;

typedef struct spx_matrix spx_matrix; /* opaque handle, see spx_matrix_create */

/* ---------------------------------------------------------------------
 * Candidate kernels, called directly with an explicit plan.
 * ------------------------------------------------------------------- */

/* Bytes of device workspace the given plan needs for a call on an m x n
 * matrix with nnz entries and at most nnz_x_max vector entries (dense x:
 * pass n). Returns 0 when none is needed. Host only. */
size_t spx_workspace_size(int32_t m, int32_t n, int32_t nnz, int32_t nnz_x_max, int32_t dtype,
                          const spx_plan *plan);

/* SpMV, row-major pattern (Section 4.1, the traditional SpMV): y = A x for a
 * dense x[n] (device, dtype; uint8 0/1 for BOOL). plan->pattern must be
 * SPX_PAT_SPMV; distribution DIRECT or BALANCED. BALANCED needs the
 * workspace of spx_workspace_size (carries between tiles). y: device, m
 * values (uint8 for BOOL). */
spx_status spmv_csr(const spx_csr *A, const void *x, void *y, const spx_plan *plan,
                    void *workspace, size_t ws_bytes, void *stream);

/* SpMSpV, row-major pattern with value validation (Section 4.1 and 6.1:
 * the SpMV skeleton skips entries whose column is not in supp(x), tested
 * with a bitvector of supp(x)). x is sparse: x_idx[nnz_x], x_val[nnz_x]
 * (device). The call converts x to a bitvector and a scattered value array
 * inside the workspace (spx_workspace_size with plan->pattern =
 * SPX_PAT_CSR_SPMSPV). */
spx_status spmspv_csr(const spx_csr *A, int32_t nnz_x, const int32_t *x_idx, const void *x_val,
                      void *y, const spx_plan *plan, void *workspace, size_t ws_bytes,
                      void *stream);

/* SpMSpV, column-major vector-driven pattern (Section 4.1): for every
 * (j, v) in x, column j of A is scaled by v and written back into y by the
 * plan's write-back (Section 4.2.2). A is CSC (see spx_matrix_csc for a
 * CSC built from a CSR). y is overwritten (zero rows included). The
 * workspace must hold spx_workspace_size(A->m, A->n, A->nnz, nnz_x, ...)
 * bytes; SPX_WB_BUCKET returns SPX_ERR_UNSUPPORTED when a bucket of rows
 * cannot fit 64 KiB of LDS within 4096 buckets. */
spx_status spmspv_csc(const spx_csc *A, int32_t nnz_x, const int32_t *x_idx, const void *x_val,
                      void *y, const spx_plan *plan, void *workspace, size_t ws_bytes,
                      void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * spmspv_csc with the workspace taken from a fixed scratch array inside the
 * library (64 MiB per device, reserved on every GPU the library runs on
 * until the process ends; spmspv_csc_noalloc_capacity() returns its size).
 * Same arguments and results as spmspv_csc minus the workspace; the calls
 * allocate nothing (no hipMalloc, no hipFree). Returns SPX_ERR_WORKSPACE
 * when spx_workspace_size(A->m, A->n, A->nnz, nnz_x, A->dtype, plan) is
 * larger than the scratch. The scratch is shared by every call on one GPU:
 * calls that overlap on one GPU (other streams, other threads) race and
 * must be ordered by the caller. The sort write-back reads a count on the
 * host and synchronizes the stream, as it does in spmspv_csc. */
spx_status spmspv_csc_noalloc(const spx_csc *A, int32_t nnz_x, const int32_t *x_idx, const void *x_val,
                              void *y, const spx_plan *plan, void *stream);
size_t spmspv_csc_noalloc_capacity(void);

/* ---------------------------------------------------------------------
 * Matrix handle: the dual CSR + CSC storage kept for the life of the
 * matrix (Section 6.1) and the matrix features computed once (Section 6.3).
 * ------------------------------------------------------------------- */

/* Builds the handle for the CSR matrix A. The handle BORROWS A's device
 * arrays (they must outlive it) and OWNS what it derives: the CSC copy
 * (stable counting-sort transpose on the device), the CSC-to-CSR
 * permutation, the matrix features and the workspace. Synchronizes the
 * stream (to read the column lengths and the matrix features). Host-side
 * checks only; pass flags & SPX_VALIDATE to also check row_ptr
 * monotonicity and index ranges on the device (one extra sync).
 *
 * Column renumbering (an implementation layout, not part of the paper's
 * method): when the 16384 longest columns hold at least max(0.3, twice the
 * uniform share) of the entries and n >= 65536, the handle also keeps a
 * copy of A whose columns are ranked by descending length (stable), with
 * the entries of each row ordered by rank; the row-major patterns run on
 * that copy and read x through the same renumbering (one gather of n
 * entries per call), so that the most-read x entries share cache lines.
 * Results are those of A up to the summation order within a row.
 * SPX_RENUMBER forces the copy, SPX_NO_RENUMBER forbids it. With it, for
 * n <= 2^21, the handle also keeps the copy's entries reordered by column
 * inside each 2048-item merge tile (each with its position in the tile),
 * which the balanced row-major kernels read, so that a wave's gathers of x
 * meet fewer cache lines; results are the same bits. Memory: 4 + value
 * size bytes per entry for the copy, 4 for its source positions, 8 per
 * column, and 8 + value size per entry for the reordered copy.
 *
 * Storage-format pre-selection (Section 8's extension: pick the matrix
 * format per matrix, before the kernel): besides CSR the handle can keep
 * one of four copies: a diagonal copy (DIA: at most 32 diagonals stored
 * one after another with a presence bit per cell, a thread per row, no
 * column indices read), a sliced ELLPACK copy (SELL-C-sigma: slices of 64
 * rows, one wave per slice and a lane per row, rows sorted by descending
 * length within windows of 4096 rows, padding to the longest row of each
 * slice), an ELLPACK copy (every row padded to the longest row of the
 * matrix, stored column-major, a thread per row, no row pointers read), or
 * a CSR5 copy (tiles of 64 lanes x 16 consecutive entries stored
 * transposed, a wave per tile, row starts marked by bits, rows that cross
 * lanes or tiles joined by segmented sums in a fixed order; no padding
 * beyond the last tile). When it does, every plan of the SpMV pattern runs
 * on that copy; the other patterns are unchanged. By default the DIA copy
 * is taken whenever it applies: the value types but BOOL, the offsets of
 * 256 rows spread over A (at most 32) hold every entry (one pass checks
 * it), and its cells move at most 0.8 x the bytes of CSR's values and
 * column indices; otherwise a small decision tree over the matrix features
 * and the padding ratios (cells / nnz; reading the sliced one copies
 * row_ptr to the host once) decides, trained on MI355X timings of the other
 * four formats. SPX_FORMAT_SELL forces the
 * sliced copy (SPX_ERR_UNSUPPORTED when a row is longer than 4096 entries or
 * the copy would take more than 3 nnz + 65536 cells), SPX_FORMAT_ELL the ELL
 * copy (SPX_ERR_UNSUPPORTED beyond 4096 entries per row or 1.5 nnz + 65536
 * cells), SPX_FORMAT_CSR5 the CSR5 copy (any matrix; building it copies
 * row_ptr to the host and synchronizes the stream), SPX_FORMAT_DIA the DIA
 * copy (SPX_ERR_UNSUPPORTED for BOOL, beyond 32 diagonals or 4 nnz + 65536
 * cells); two of these flags together are SPX_ERR_ARG. SPX_FORMAT_CSR
 * forbids every copy. Memory: 8 + value size bytes per cell (4 more per row
 * for the sliced copy; for CSR5, 4 per row and 4 + 16 per tile of 1024
 * cells; for DIA, value size + 1/8 per cell). */
#define SPX_VALIDATE 1u
#define SPX_RENUMBER 4u
#define SPX_NO_RENUMBER 8u
#define SPX_FORMAT_CSR 16u
#define SPX_FORMAT_SELL 32u
#define SPX_FORMAT_ELL 64u
#define SPX_FORMAT_CSR5 128u
#define SPX_FORMAT_DIA 256u
spx_status spx_matrix_create(const spx_csr *A, uint32_t flags, void *stream, spx_matrix **out);
spx_status spx_matrix_destroy(spx_matrix *H);

/* The handle's CSC copy (device pointers owned by the handle). */
spx_status spx_matrix_csc(const spx_matrix *H, spx_csc *out);

/* Re-derives the CSC values (and those of the renumbered, sliced ELL, ELL,
 * CSR5 and DIA copies) from the borrowed CSR values (gathers through the permutations);
 * call after the caller changed A's values in place. */
spx_status spx_matrix_values_updated(spx_matrix *H, void *stream);

/* *renumbered = 1 if the handle keeps the column-renumbered copy (see
 * spx_matrix_create), else 0. If so and order is not NULL, copies the
 * ranking to order (device, n int32: order[r] = the column of rank r),
 * asynchronously on stream. */
spx_status spx_matrix_column_order(const spx_matrix *H, int32_t *order, int32_t *renumbered, void *stream);

/* *format = 1 if the handle keeps the sliced ELLPACK copy, 2 if it keeps
 * the ELLPACK copy, 3 if it keeps the CSR5 copy, 4 if it keeps the DIA copy
 * (see spx_matrix_create), else 0; *padding_ratio (may be NULL) = that copy's cells / nnz (0 when
 * there is no copy). Host only. */
spx_status spx_matrix_format(const spx_matrix *H, int32_t *format, double *padding_ratio);

/* Matrix features of Table 1, out[9] = {m, n, nnz, max_row, min_row,
 * avg_row, relative_range = (max_row - min_row) / n, var_nnz_row
 * (population standard deviation of row lengths), Gini coefficient of
 * row lengths}. Host only (values computed at create). */
spx_status spx_matrix_features(const spx_matrix *H, double *out9);

/* Vector features of Table 1, out[4] = {nnz_x, x_sparsity = nnz_x / n,
 * nnz_s = stored entries in columns of supp(x), m_sparsity = nnz_s / nnz}.
 * Computed on the device (gather + reduction); synchronizes the stream. */
spx_status spx_vector_features(spx_matrix *H, const spx_vec *x, double *out4, void *stream);

/* ---------------------------------------------------------------------
 * Selection and adaptive execution (Sections 5 and 6).
 * ------------------------------------------------------------------- */

/* Loads the three decision trees (pattern, distribution, write-back) from
 * a JSON file written by the tuner; json_path NULL means the built-in
 * trees. A handle holds three sets of trees:
 *  - the host-feature trees, which test only features the host knows
 *    (Table 1 minus nnz_s and m_sparsity); run_batch evaluates them on the
 *    device, and run() and select_kernel() use them until lazy trees load;
 *  - lazy trees (the file has "lazy": true) decide run() and
 *    select_kernel(): they may test nnz_s, m_sparsity or s_per_x (nnz_s /
 *    max(1, nnz_x)), which are computed on the device, with one stream
 *    synchronization, only when the walk reaches such a node (Section 6.3:
 *    features evaluated lazily, cheap rules first; the tuner trains them
 *    with that round trip charged to every vector that takes it);
 *  - trees that test nnz_s without "lazy" serve the callers that know it
 *    for free: the graph drivers (spx_bfs, spx_pagerank count it while
 *    building x). Until such trees are loaded, they use the host-feature
 *    trees.
 * Host-feature trees (a file that tests no count feature, or NULL) replace
 * all three sets; load the others after them. With H NULL the trees become
 * the default of handles created afterwards; otherwise they replace H's
 * only (for example trees trained for the BOOL semiring on a BOOL
 * handle). */
spx_status spx_load_selector(spx_matrix *H, const char *json_path);

/* Walks the cascade of run()'s trees: pattern tree, then distribution
 * tree, then (column-major only) write-back tree (Section 6.2). Features
 * are evaluated lazily (Section 6.3): the only device work is the nnz_s
 * reduction, made when a node tests nnz_s, m_sparsity or s_per_x; it
 * synchronizes the stream, and flags & SPX_NO_SYNC forbids it (such nodes
 * then read nnz_s as nnz_x times the average column length). A vector
 * handed over dense counts as dense (nnz_x = n) and never takes the
 * column-major pattern (it would need a compaction and a host round trip
 * first): where the pattern tree says column-major, it takes SpMV. */
#define SPX_NO_SYNC 2u
spx_status select_kernel(spx_matrix *H, const spx_vec *x, uint32_t flags, spx_plan *out,
                         void *stream);

/* Adaptive y = A x: select_kernel, convert x to the format the chosen
 * kernel reads if it differs (Section 6.3: conversion only on change),
 * launch. y: device, m values of the matrix dtype (uint8 for BOOL). */
spx_status run(spx_matrix *H, const spx_vec *x, void *y, void *stream);

/* y = A x with a given plan through the handle (its CSC and workspace). */
spx_status run_plan(spx_matrix *H, const spx_vec *x, void *y, const spx_plan *plan, void *stream);

/* The plan the last run() chose, and per-stage times in milliseconds of
 * the run() calls since the last spx_stage_times, while profiling is on
 * (Section 7's overhead breakdown): out[0] features (host time, including
 * any device reduction and its synchronization), out[1] model evaluation
 * (host time), out[2] vector conversion and out[3] kernel(s) (HIP events on
 * the caller's stream; synchronizes on them). Resets the feature, model and
 * conversion totals; the kernel events stay until spx_run_times reads
 * them. */
spx_status spx_last_plan(const spx_matrix *H, spx_plan *out);
spx_status spx_set_profiling(spx_matrix *H, int32_t on);
spx_status spx_stage_times(const spx_matrix *H, double *out4);

/* Kernel time (ms, HIP events on the caller's stream around the launches of
 * the chosen kernel) of each run()/run_plan() since the last call, in call
 * order, while profiling is on. Writes min(count, cap) values to out and
 * the number of runs to *count, then forgets them. Synchronizes on the
 * recorded events. */
spx_status spx_run_times(spx_matrix *H, double *out, int32_t cap, int32_t *count);

/* ---------------------------------------------------------------------
 * Batched SpMSpV: B sparse vectors in one launch sequence.
 * X is CSR-of-vectors: vec_ptr[B+1] (device), idx[total] and val[total]
 * (device); Y is B x m row-major (device), each vector's y contiguous.
 * The plan of every vector is chosen on the device: the trees run() uses
 * (see spx_load_selector), evaluated by a device kernel on the matrix
 * features and the vector's nnz_x; a vector's nnz_s (the prefix of its
 * column lengths) is computed on the device when its plan is column-major,
 * or for every vector when the loaded trees test nnz_s. Vectors whose plan
 * is row-major, or that hold at least 2 % of n, share passes over A in
 * groups of 64 (not for BOOL). The calls are a plan kernel, a queue scan,
 * three persistent phase kernels and, on a parallel branch beside the
 * second, the groups' walk of A, captured once into a HIP graph and
 * replayed while the arrays and B stay the same; nothing synchronizes
 * except a workspace reallocation.
 * total_nnz_x (host) is an upper bound of vec_ptr[B] used to size the
 * workspace. Column-major plans write back with device atomics in this
 * path. Vector indices must be unique within a vector.
 * ------------------------------------------------------------------- */
spx_status run_batch(spx_matrix *H, int32_t B, int64_t total_nnz_x, const int32_t *vec_ptr,
                     const int32_t *idx, const void *val, void *Y, void *stream);

/* Status of the last run_batch on H: *flags = 0 when every work item ran;
 * bit 1 (value 2) is set when vec_ptr disagreed with the capacity the host
 * sized (vec_ptr[B] above total_nnz_x, a negative or decreasing entry, or a
 * vector longer than n): such vectors are skipped and their rows of Y are
 * not valid. No other bit is used. Synchronizes the stream. */
spx_status spx_batch_status(spx_matrix *H, int32_t *flags, void *stream);

/* Y[b] = A X[b] for the B rows of a dense X (B x n -> Y B x m, device,
 * row-major): the row-major SpMV of Section 4.1 applied to all B vectors
 * in one pass over A (a wave per row, lane = batch entry, entries of x
 * gathered from a B-minor copy of X in the workspace). Reads A once where
 * B separate calls read it B times; meant for dense batches such as layer
 * activations. One wave walks a whole row, so rows far longer than the
 * average (hub rows) serialize. F32 and F64 only. */
spx_status spmv_csr_batch(spx_matrix *H, int32_t B, const void *X, void *Y, void *stream);

/* Sparse-output SpMSpV with a complement mask (the frontier form of the
 * product, Section 7; the bucket write-back of Section 4.2.2 listing rows
 * instead of writing a dense y): for a sparse x, the rows i that an
 * effective entry reaches (a stored entry in a column of supp(x), however
 * its products sum) and whose bit in mask is clear (mask: device bitvector
 * of ceil(m / 32) words, bit i of word i / 32; NULL masks nothing) go to
 * y_idx[k] (device int32) with y_val[k] = (A x)_i (device, the handle's
 * value type; NULL to skip the values; for BOOL all 1), k < *nnz_y (host).
 * Rows ascend within each bucket of rows; the buckets come in any order.
 * y_idx / y_val must hold the rows that can be listed (m at most). No
 * dense y is written, so the cost follows nnz_x and nnz_s, not m.
 * plan: a column-major plan with the bucket write-back (its distribution,
 * lanes and bucket rows are used), or NULL to let the column-major
 * distribution tree choose. Synchronizes the stream (the count). */
spx_status spmspv_sparse(spx_matrix *H, const spx_vec *x, const uint32_t *mask, const spx_plan *plan,
                         int32_t *y_idx, void *y_val, int32_t *nnz_y, void *stream);

/* The complement mask of spmspv_sparse from one byte per row: bit i of
 * words[i / 32] = (rows[i] != 0) for i < m; the unused high bits of the last
 * word are cleared. rows: device, m bytes; words: device, ceil(m / 32)
 * words, written. One wave ballot per 64 rows. */
spx_status spx_pack_mask(int32_t m, const uint8_t *rows, uint32_t *words, void *stream);

/* Breadth-first search over the graph of a square BOOL handle (stored entry
 * (i, j) = edge j -> i, so a column lists a vertex's out-edges): level[v] =
 * fewest edges from source, -1 if unreachable (level: device int32[n]).
 * A level is one (OR, AND) SpMSpV of the frontier, through run() (the
 * kernel chosen per level, as the frontier's density changes; Section 7)
 * or through run_plan() with the given plan, followed by a kernel that
 * keeps the unvisited vertices, labels them and appends them to the next
 * frontier. Without a plan and without SPX_BFS_PUSH_ONLY, a level whose
 * frontier's out-edges exceed the unexplored ones / 14 runs instead as a
 * masked pull (only the rows of unvisited vertices, each stopped at its
 * first frontier neighbour), until the frontier falls below n / 24
 * vertices (the direction-optimizing heuristic; not part of the paper).
 * At most max_levels levels are labelled. *n_levels = the number of levels
 * labelled (1 + the largest level). If plans is given, plans[l] receives
 * the plan of expansion l for l < plans_cap; a masked pull is reported as
 * {SPX_PAT_CSR_SPMSPV, SPX_DIST_DIRECT, SPX_WB_NONE, lanes = -1}.
 * Synchronizes the stream once per level (the frontier size decides the
 * next call). The frontier lists and bitvectors, the product buffer and
 * a pinned counter belong to the handle (allocated on the first call). */
#define SPX_BFS_PUSH_ONLY 1u
spx_status spx_bfs(spx_matrix *H, int32_t source, int32_t *level, int32_t max_levels, const spx_plan *plan,
                   uint32_t flags, int32_t *n_levels, spx_plan *plans, int32_t plans_cap, void *stream);

/* Incremental (residual-push) PageRank over the graph of a square F32 or
 * F64 handle (the second application of Section 7): stored entry (i, j) is
 * an edge j -> i of weight a_ij >= 0 (SPX_ERR_ARG on a negative weight);
 * the walk leaves j along (i, j) with probability a_ij / W_j, W_j = sum of
 * column j, and a vertex with W_j = 0 is dangling (its mass leaves the
 * graph). The fixed point p solves p = (1 - d)/n + d A diag(1/W) p.
 * Residual r starts at (1 - d)/n, p at 0. Each round moves every residual
 * with |r_v| > eps into p_v and clears it; the active vertices that are not
 * dangling form the sparse input x_v = r_v / W_v of one product y = A x
 * (through run(), or run_plan() with the given plan), and r += d y. The
 * rounds stop when no active vertex can propagate, or after max_iters
 * products (then the last product is folded into r too). At any stop
 * p + (I - d A diag(1/W))^-1 r is the fixed point.
 * damping in [0, 1), eps >= 0, max_iters >= 0. rank (required) and
 * residual (optional): device arrays of n values of the handle's type,
 * written by the call. *n_iters = the number of products; plans[k]
 * receives the plan of product k for k < plans_cap. Synchronizes the
 * stream once per round. The column sums are computed on the first call
 * and again after spx_matrix_values_updated; the work buffers belong to
 * the handle. */
spx_status spx_pagerank(spx_matrix *H, double damping, double eps, int32_t max_iters, const spx_plan *plan,
                        void *rank, void *residual, int32_t *n_iters, spx_plan *plans, int32_t plans_cap,
                        void *stream);

/* ---------------------------------------------------------------------
 * Backward of Y[b] = A(vals) X[b] for a loss L(Y), with G = dL/dY
 * (B x m) and X (B x n), both dense, row-major, on the device:
 *   dX[b] = A^T G[b]                       (spmv_csr_transpose: the CSC copy
 *                                           read as rows of A^T, a gather
 *                                           along columns, no atomics)
 *   dvals_k = sum_b G[b, row k] X[b, col k]  over the CSR pattern
 * Both read the matrix once for the whole batch. F32 and F64 only. The
 * handle's workspace holds B-minor copies of G (and X); dX is stored
 * B-major directly by the gather kernel (a workgroup's 16 columns turned
 * through LDS).
 * ------------------------------------------------------------------- */

/* dX[b] = A^T G[b] for b < B: G is B x m, dX is B x n (device, row-major). */
spx_status spmv_csr_transpose(spx_matrix *H, int32_t B, const void *G, void *dX, void *stream);

/* dvals[k] = sum_{b<B} G[b, row(k)] * X[b, col(k)], k over CSR positions.
 * G is B x m and X is B x n dense (device, row-major). */
spx_status dvals_pattern(spx_matrix *H, int32_t B, const void *G, const void *X, void *dvals,
                         void *stream);

/* Both gradients of one backward pass: dX = G A (as spmv_csr_transpose)
 * and dvals (as dvals_pattern), computed from one B-minor copy of G, which
 * the two separate calls would each make. dX or dvals may be NULL to skip
 * it (not both); X may be NULL when dvals is. Same layouts and dtypes as
 * the separate calls. */
spx_status spx_backward(spx_matrix *H, int32_t B, const void *G, const void *X, void *dX, void *dvals,
                        void *stream);

/* Vector format conversion for a batch (Section 6.3): the B dense rows of
 * X (B x n, matrix dtype; uint8 for BOOL) become sparse vectors in
 * CSR-of-vectors form, ready for run_batch: vec_ptr[B+1], idx[], val[]
 * (caller-owned device arrays with room for B * n entries). x != 0 marks a
 * nonzero (-0.0 is zero, NaN is not). */
spx_status spx_dense_rows_to_sparse(spx_matrix *H, int32_t B, const void *X, int32_t *vec_ptr,
                                    int32_t *idx, void *val, void *stream);

/* Measurement helper: copies bytes from src to dst (device pointers, both
 * 16-byte aligned, bytes a multiple of 16; SPX_ERR_ARG otherwise) with a
 * plain streaming kernel (16-byte loads and stores). Its rate is the
 * achievable HBM bandwidth that the kernels' effective bandwidth is set
 * against, beside the published peak. */
spx_status spx_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* ---------------------------------------------------------------------
 * Host-only helpers.
 * ------------------------------------------------------------------- */

/* Checks the host-visible fields of a CSR descriptor (no device access). */
spx_status spx_check_csr(const spx_csr *A);
/* Checks that a plan is a legal kernel for the given dtype (no device access). */
spx_status spx_check_plan(const spx_plan *plan, int32_t dtype);
/* Thread-local message describing the last error (never NULL). */
const char *spx_last_error(void);
/* Library version string. */
const char *spx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPX_H */
