/*
 * CPU oracle for adaptive SpMV / SpMSpV (Li, Ao, Yang, "Adaptive SpMV/SpMSpV
 * on GPUs for Input Vectors of Varied Sparsity").
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do. It shares no code and no header with the HIP
 * library.
 *
 * Every routine is the plain definition of what the method computes,
 * written as a single slow loop nest:
 *   - floating-point inputs arrive as double (FP32 inputs are widened
 *     exactly, so every product of two FP32 numbers is exact in double)
 *     and sums are Neumaier-compensated in double;
 *   - the boolean (OR, AND) and the integer (+, x) mod 2^32 semirings are
 *     exact by construction;
 *   - alongside every real-valued sum the routines return
 *     S_i = sum |a_ij x_j| over the same terms, which scales the error
 *     tolerance of a faster implementation.
 *
 * Parity status: every function here is pinned by the CPU tests (dense
 * brute force, a library routine, closed forms, invariants, finite
 * differences, an edge-list BFS step); none is "parity unpinned".
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no -ffast-math:
 * compensation relies on IEEE rounding).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OK 0
#define ERR_ALLOC (-1)
#define ERR_ARG (-2)

/* Neumaier (improved Kahan-Babuska) summation: running sum s and running
 * correction c; the result is s + c. */
static void nadd(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

/* ---------------------------------------------------------------------
 * O1: SpMV over CSR (Section 2: y = A x, A m-by-n with nnz entries, x a
 * dense vector of length n; the row-major matrix-driven pattern without
 * value validation is the traditional SpMV of Section 4.1).
 *   y[i] = sum_{k = row_ptr[i]}^{row_ptr[i+1]-1} vals[k] * x[col_idx[k]]
 *   s[i] = sum of |vals[k] * x[col_idx[k]]| over the same k
 * ------------------------------------------------------------------- */
int oracle_spmv(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                const double *vals, const double *x, double *y, double *s)
{
    if (m < 0 || n < 0)
        return ERR_ARG;
    for (int32_t i = 0; i < m; ++i) {
        double acc = 0.0, cor = 0.0, mag = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double p = vals[k] * x[col_idx[k]];
            nadd(&acc, &cor, p);
            mag += fabs(p);
        }
        y[i] = acc + cor;
        if (s)
            s[i] = mag;
    }
    return OK;
}

/* ---------------------------------------------------------------------
 * O2a: the oracle's own CSR -> CSC conversion (Section 2: CSC gives O(1)
 * access to a column; Section 6.1: both formats are stored up front).
 * Counting sort by column, stable in row order, so row_idx is ascending
 * within each column. perm[p] is the CSR position of CSC position p.
 * vals / vals_csc may be NULL (pattern only).
 * ------------------------------------------------------------------- */
int oracle_transpose(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *vals, int32_t *col_ptr, int32_t *row_idx, int32_t *perm,
                     double *vals_csc)
{
    int32_t nnz = row_ptr[m];
    int64_t *next = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!next)
        return ERR_ALLOC;
    for (int32_t k = 0; k < nnz; ++k)
        next[col_idx[k] + 1] += 1;
    for (int32_t j = 0; j < n; ++j)
        next[j + 1] += next[j];
    for (int32_t j = 0; j <= n; ++j)
        col_ptr[j] = (int32_t)next[j];
    for (int32_t i = 0; i < m; ++i) {
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int64_t p = next[col_idx[k]]++;
            row_idx[p] = i;
            if (perm)
                perm[p] = k;
            if (vals && vals_csc)
                vals_csc[p] = vals[k];
        }
    }
    free(next);
    return OK;
}

/* ---------------------------------------------------------------------
 * O2b: SpMSpV, vector-driven column-major (Section 4.1, the pattern the
 * paper tags (2,8)): for every nonzero (j, v) of the sparse x, scatter
 * column j of A into a dense accumulator y of length m. Only the
 * effective nonzeros (entries in columns j in supp(x), Section 2) are
 * touched. Rows that receive nothing stay exactly +0.
 * ------------------------------------------------------------------- */
int oracle_spmspv_csc(int32_t m, int32_t n, const int32_t *col_ptr, const int32_t *row_idx,
                      const double *vals_csc, int32_t nnz_x, const int32_t *x_idx,
                      const double *x_val, double *y, double *s)
{
    double *cor = (double *)calloc((size_t)m + 1, sizeof(double));
    if (!cor)
        return ERR_ALLOC;
    for (int32_t i = 0; i < m; ++i) {
        y[i] = 0.0;
        if (s)
            s[i] = 0.0;
    }
    for (int32_t t = 0; t < nnz_x; ++t) {
        int32_t j = x_idx[t];
        if (j < 0 || j >= n) {
            free(cor);
            return ERR_ARG;
        }
        double v = x_val[t];
        for (int32_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k) {
            int32_t i = row_idx[k];
            double p = vals_csc[k] * v;
            nadd(&y[i], &cor[i], p);
            if (s)
                s[i] += fabs(p);
        }
    }
    for (int32_t i = 0; i < m; ++i)
        y[i] += cor[i];
    free(cor);
    return OK;
}

/* ---------------------------------------------------------------------
 * O2c: the same column scatter, restricted to the output rows [r0, r1).
 * Row i of y receives exactly the terms O2b adds to it, in the same order
 * (x entries in order, each column top to bottom), so the result equals
 * O2b's bit for bit. Rows ascend within a column of the oracle's own
 * transpose (O2a is a stable counting sort), so a column's entries in
 * [r0, r1) form one contiguous run, found by two binary searches.
 * O2d runs disjoint row ranges of O2c on the host's cores (OpenMP); it is
 * the multi-core leg of the CPU baseline, pinned equal to O2b.
 * ------------------------------------------------------------------- */
static int32_t lower_row(const int32_t *row_idx, int32_t a, int32_t b, int32_t key)
{
    while (a < b) {
        int32_t mid = a + (b - a) / 2;
        if (row_idx[mid] < key)
            a = mid + 1;
        else
            b = mid;
    }
    return a;
}

int oracle_spmspv_csc_rows(int32_t m, int32_t n, const int32_t *col_ptr, const int32_t *row_idx,
                           const double *vals_csc, int32_t nnz_x, const int32_t *x_idx,
                           const double *x_val, int32_t r0, int32_t r1, double *y, double *s)
{
    if (r0 < 0 || r1 > m || r0 > r1)
        return ERR_ARG;
    double *cor = (double *)calloc((size_t)(r1 - r0) + 1, sizeof(double));
    if (!cor)
        return ERR_ALLOC;
    for (int32_t i = r0; i < r1; ++i) {
        y[i] = 0.0;
        if (s)
            s[i] = 0.0;
    }
    for (int32_t t = 0; t < nnz_x; ++t) {
        int32_t j = x_idx[t];
        if (j < 0 || j >= n) {
            free(cor);
            return ERR_ARG;
        }
        double v = x_val[t];
        int32_t k0 = lower_row(row_idx, col_ptr[j], col_ptr[j + 1], r0);
        int32_t k1 = lower_row(row_idx, k0, col_ptr[j + 1], r1);
        for (int32_t k = k0; k < k1; ++k) {
            int32_t i = row_idx[k];
            double p = vals_csc[k] * v;
            nadd(&y[i], &cor[i - r0], p);
            if (s)
                s[i] += fabs(p);
        }
    }
    for (int32_t i = r0; i < r1; ++i)
        y[i] += cor[i - r0];
    free(cor);
    return OK;
}

int oracle_spmspv_csc_omp(int32_t m, int32_t n, const int32_t *col_ptr, const int32_t *row_idx,
                          const double *vals_csc, int32_t nnz_x, const int32_t *x_idx,
                          const double *x_val, double *y, double *s)
{
    const int32_t blocks = 256;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(|: bad)
    for (int32_t b = 0; b < blocks; ++b) {
        int32_t r0 = (int32_t)((int64_t)m * b / blocks), r1 = (int32_t)((int64_t)m * (b + 1) / blocks);
        if (oracle_spmspv_csc_rows(m, n, col_ptr, row_idx, vals_csc, nnz_x, x_idx, x_val, r0, r1, y, s) != OK)
            bad = 1;
    }
    return bad ? ERR_ARG : OK;
}

/* threads the OpenMP leg runs on */
int oracle_omp_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------
 * O3: boolean (OR, AND) SpMSpV. A is a pattern; x is a set of indices.
 *   y[i] = OR over stored (i, j) of [j in supp(x)]
 * Written row by row from the definition (a membership mark per column).
 * ------------------------------------------------------------------- */
int oracle_bool_spmspv(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                       int32_t nnz_x, const int32_t *x_idx, uint8_t *y)
{
    uint8_t *mark = (uint8_t *)calloc((size_t)n + 1, 1);
    if (!mark)
        return ERR_ALLOC;
    for (int32_t t = 0; t < nnz_x; ++t) {
        if (x_idx[t] < 0 || x_idx[t] >= n) {
            free(mark);
            return ERR_ARG;
        }
        mark[x_idx[t]] = 1;
    }
    for (int32_t i = 0; i < m; ++i) {
        uint8_t any = 0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            any = (uint8_t)(any | mark[col_idx[k]]);
        y[i] = any;
    }
    free(mark);
    return OK;
}

/* ---------------------------------------------------------------------
 * Min-plus semiring over float32 (shortest-path relaxation):
 * y_i = min over the stored entries (i, j) with x_j present of
 * (a_ij + x_j), each sum one float32 addition (correctly rounded, so the
 * result does not depend on the order of the minimum); +inf when no entry
 * is effective. A dense x marks an absent entry by +inf; a sparse x lists
 * the present ones (any other index is absent).
 * ------------------------------------------------------------------- */
int oracle_minplus_spmv(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        const float *vals, const float *x, float *y)
{
    (void)n;
    for (int32_t i = 0; i < m; ++i) {
        float best = INFINITY;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const float xj = x[col_idx[k]];
            if (xj == INFINITY)
                continue;
            const volatile float sum = vals[k] + xj; /* one float32 rounding */
            if (sum < best)
                best = sum;
        }
        y[i] = best;
    }
    return OK;
}

/* ---------------------------------------------------------------------
 * O4: integer (+, x) semiring modulo 2^32, reinterpreted as int32.
 * Unsigned arithmetic, so wrap-around is defined.
 * SpMV over CSR, and SpMSpV as the column scatter of O2b.
 * ------------------------------------------------------------------- */
int oracle_int_spmv(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                    const int32_t *vals, const int32_t *x, int32_t *y)
{
    (void)n;
    for (int32_t i = 0; i < m; ++i) {
        uint32_t acc = 0u;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            acc += (uint32_t)vals[k] * (uint32_t)x[col_idx[k]];
        y[i] = (int32_t)acc;
    }
    return OK;
}

int oracle_int_spmspv_csc(int32_t m, int32_t n, const int32_t *col_ptr, const int32_t *row_idx,
                          const int32_t *vals_csc, int32_t nnz_x, const int32_t *x_idx,
                          const int32_t *x_val, int32_t *y)
{
    uint32_t *acc = (uint32_t *)calloc((size_t)m + 1, sizeof(uint32_t));
    if (!acc)
        return ERR_ALLOC;
    for (int32_t t = 0; t < nnz_x; ++t) {
        int32_t j = x_idx[t];
        if (j < 0 || j >= n) {
            free(acc);
            return ERR_ARG;
        }
        for (int32_t k = col_ptr[j]; k < col_ptr[j + 1]; ++k)
            acc[row_idx[k]] += (uint32_t)vals_csc[k] * (uint32_t)x_val[t];
    }
    for (int32_t i = 0; i < m; ++i)
        y[i] = (int32_t)acc[i];
    free(acc);
    return OK;
}

/* ---------------------------------------------------------------------
 * O6: gradients of L = sum_b <g_b, A x_b> for a batch of B vectors.
 *   dx_b[j]  = sum_i a_ij g_b[i]            (A^T g_b), written as a scatter
 *                                             along CSR rows, the opposite
 *                                             traversal of a CSC gather
 *   sdx_b[j] = sum_i |a_ij g_b[i]|
 *   dvals[k] = sum_b g_b[row(k)] * x_b[col(k)]   over the CSR pattern
 * G is B-by-m and X is B-by-n, row-major; dX and sdX are B-by-n.
 * Any of dX / sdX / dvals may be NULL.
 * ------------------------------------------------------------------- */
int oracle_grad(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                const double *vals, int32_t B, const double *G, const double *X,
                double *dX, double *sdX, double *dvals)
{
    if (dX) {
        double *cor = (double *)calloc((size_t)n + 1, sizeof(double));
        if (!cor)
            return ERR_ALLOC;
        for (int32_t b = 0; b < B; ++b) {
            double *d = dX + (size_t)b * n;
            double *sd = sdX ? sdX + (size_t)b * n : NULL;
            const double *g = G + (size_t)b * m;
            memset(cor, 0, sizeof(double) * (size_t)n);
            for (int32_t j = 0; j < n; ++j) {
                d[j] = 0.0;
                if (sd)
                    sd[j] = 0.0;
            }
            for (int32_t i = 0; i < m; ++i) {
                for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                    int32_t j = col_idx[k];
                    double p = vals[k] * g[i];
                    nadd(&d[j], &cor[j], p);
                    if (sd)
                        sd[j] += fabs(p);
                }
            }
            for (int32_t j = 0; j < n; ++j)
                d[j] += cor[j];
        }
        free(cor);
    }
    if (dvals) {
        for (int32_t i = 0; i < m; ++i) {
            for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                int32_t j = col_idx[k];
                double acc = 0.0, cor = 0.0;
                for (int32_t b = 0; b < B; ++b)
                    nadd(&acc, &cor, G[(size_t)b * m + i] * X[(size_t)b * n + j]);
                dvals[k] = acc + cor;
            }
        }
    }
    return OK;
}

/* ---------------------------------------------------------------------
 * O5: the features of Table 1.
 * Matrix part, out[0..8]:
 *   m, n, nnz, max_row, min_row, avg_row = nnz/m,
 *   relative_range = (max_row - min_row) / n   (the table's formula),
 *   var_nnz_row = population standard deviation of row lengths,
 *   Gini = sum_{i=1..m} (2i - m - 1) r_(i) / (m sum r), r ascending,
 *          0 when sum r = 0.
 * Vector part, out[0..3]:
 *   nnz_x, x_sparsity = nnz_x / n,
 *   nnz_s = number of stored entries in columns j in supp(x)
 *           (effective nonzeros, Section 2, counted structurally),
 *   m_sparsity = nnz_s / nnz.
 * ------------------------------------------------------------------- */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

int oracle_matrix_features(int32_t m, int32_t n, const int32_t *row_ptr, double *out)
{
    int32_t *len = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
    if (!len)
        return ERR_ALLOC;
    int64_t total = 0;
    int32_t mx = 0, mn = 0;
    for (int32_t i = 0; i < m; ++i) {
        len[i] = row_ptr[i + 1] - row_ptr[i];
        total += len[i];
        if (i == 0 || len[i] > mx)
            mx = len[i];
        if (i == 0 || len[i] < mn)
            mn = len[i];
    }
    double avg = m > 0 ? (double)total / (double)m : 0.0;
    double var = 0.0, cor = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        double d = (double)len[i] - avg;
        nadd(&var, &cor, d * d);
    }
    var = m > 0 ? (var + cor) / (double)m : 0.0;
    qsort(len, (size_t)m, sizeof(int32_t), cmp_i32);
    int64_t num = 0;
    for (int32_t i = 0; i < m; ++i)
        num += (int64_t)(2 * (int64_t)(i + 1) - m - 1) * (int64_t)len[i];
    double gini = total > 0 ? (double)num / ((double)m * (double)total) : 0.0;
    free(len);
    out[0] = m;
    out[1] = n;
    out[2] = (double)total;
    out[3] = mx;
    out[4] = mn;
    out[5] = avg;
    out[6] = n > 0 ? (double)(mx - mn) / (double)n : 0.0;
    out[7] = sqrt(var);
    out[8] = gini;
    return OK;
}

int oracle_vector_features(int32_t n, int32_t nnz, const int32_t *col_ptr, int32_t nnz_x,
                           const int32_t *x_idx, double *out)
{
    int64_t nnz_s = 0;
    for (int32_t t = 0; t < nnz_x; ++t) {
        int32_t j = x_idx[t];
        if (j < 0 || j >= n)
            return ERR_ARG;
        nnz_s += col_ptr[j + 1] - col_ptr[j];
    }
    out[0] = nnz_x;
    out[1] = n > 0 ? (double)nnz_x / (double)n : 0.0;
    out[2] = (double)nnz_s;
    out[3] = nnz > 0 ? (double)nnz_s / (double)nnz : 0.0;
    return OK;
}

/* ---------------------------------------------------------------------
 * O7: one breadth-first-search frontier expansion over an edge list
 * (the vector is the set of active vertices, Section 1): the next
 * frontier is every target of an edge whose source is active. No visited
 * mask. Sources index [0, n), targets [0, m).
 * ------------------------------------------------------------------- */
int oracle_bfs_step(int64_t n_edges, const int32_t *src, const int32_t *dst, int32_t n,
                    const uint8_t *active, int32_t m, uint8_t *next)
{
    memset(next, 0, (size_t)m);
    for (int64_t e = 0; e < n_edges; ++e) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= m)
            return ERR_ARG;
        if (active[src[e]])
            next[dst[e]] = 1;
    }
    return OK;
}

/* ---------------------------------------------------------------------
 * Breadth-first search levels over a directed edge list src[e] -> dst[e]
 * of n vertices (the traversal the paper runs its kernels in, Section 7):
 * level[v] = fewest edges on a path from source, -1 if v is unreachable.
 * Textbook queue order: out-edges grouped by their source vertex, a FIFO of
 * discovered vertices, each vertex labelled when first discovered.
 * ------------------------------------------------------------------- */
int oracle_bfs_levels(int64_t n_edges, const int32_t *src, const int32_t *dst, int32_t n, int32_t source,
                      int32_t *level)
{
    if (n < 0 || (n > 0 && (source < 0 || source >= n)))
        return ERR_ARG;
    int64_t *start = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *out = (int32_t *)malloc((size_t)(n_edges > 0 ? n_edges : 1) * sizeof(int32_t));
    int32_t *queue = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!start || !out || !queue) {
        free(start);
        free(out);
        free(queue);
        return ERR_ALLOC;
    }
    for (int64_t e = 0; e < n_edges; ++e) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) {
            free(start);
            free(out);
            free(queue);
            return ERR_ARG;
        }
        start[src[e] + 1] += 1;
    }
    for (int32_t v = 0; v < n; ++v)
        start[v + 1] += start[v];
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!fill) {
        free(start);
        free(out);
        free(queue);
        return ERR_ALLOC;
    }
    for (int32_t v = 0; v < n; ++v)
        fill[v] = start[v];
    for (int64_t e = 0; e < n_edges; ++e)
        out[fill[src[e]]++] = dst[e];
    free(fill);
    for (int32_t v = 0; v < n; ++v)
        level[v] = -1;
    if (n > 0) {
        int32_t head = 0, tail = 0;
        level[source] = 0;
        queue[tail++] = source;
        while (head < tail) {
            int32_t u = queue[head++];
            for (int64_t e = start[u]; e < start[u + 1]; ++e) {
                int32_t v = out[e];
                if (level[v] < 0) {
                    level[v] = level[u] + 1;
                    queue[tail++] = v;
                }
            }
        }
    }
    free(start);
    free(out);
    free(queue);
    return OK;
}
