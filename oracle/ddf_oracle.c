/*
 * Plain FP64 CPU oracle for the DDF hot path.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load this code.  It
 * shares no source, header, table or helper with the library; the two meet only in the
 * canonical plan tables, which each side writes out by itself.
 *
 * Values (sparse matrix-vector multiply, forward substitution, their adjoints, levels) are the
 * plain row-by-row definitions: the DDF executor only reorganises loads, so its result must
 * equal these up to rounding order (paper, Sec. II and Sec. V: the sequential CSR codes are
 * the baseline every executor is compared against).
 *
 * The plan is the inspector of the paper's Algorithm 1 (Sec. IV-A) taken step by step:
 *   computeAccessFunctions -> findDependencies -> partitionIterationSpace (level sets),
 *   then per partition: GetConsecutiveIterations (windows of t rows), and per window the
 *   three strategies BLAS_first / PSCI_first / PSCII_first, each costed with Eq. (1), the
 *   cheapest kept (min_cost) and appended to the codelet list.
 * Candidate codelets are classified from the first order partial differences (FOPD) of the
 * three access functions evaluated on their explicit iteration space (Sec. III-D), with the
 * class definitions of Sec. III-B (all three strided = BLAS, two = PSC I, one = PSC II).
 * Where the paper is silent the readings are: window t = 64 by default; whole rows per
 * codelet; a ragged (non-rectangular) space makes the value and column accesses non-strided;
 * Eq. (1)'s m is the number of access functions (3) and a strided function costs no table;
 * an irregular column table may be stored as runs (start, length) when that is smaller;
 * ties in min_cost go BLAS_first, PSCI_first, PSCII_first; dependence groups are ASAP level
 * sets.
 *
 * Compiled with -O2 -ffp-contract=off: IEEE binary64, round to nearest even, no FMA.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ----------------------------------------------------------------------------------------
 * Values
 * -------------------------------------------------------------------------------------- */

/* Y = A X.  X is (n_cols, k) row-major, Y is (n_rows, k) row-major. */
void orc_spmv(int32_t n_rows, const int32_t *rp, const int32_t *ci, const double *v,
              int32_t k, const double *X, double *Y) {
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t r = 0; r < k; r++) {
            double acc = 0.0;
            for (int64_t e = rp[i]; e < rp[i + 1]; e++)
                acc += v[e] * X[(int64_t)ci[e] * k + r];
            Y[i * k + r] = acc;
        }
    }
}

/* Forward substitution L X = B, L lower triangular with its diagonal last in each row.
 * B and X may be the same buffer. */
void orc_sptrsv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t k,
                const double *B, double *X) {
    for (int64_t i = 0; i < n; i++) {
        int64_t d = rp[i + 1] - 1;
        for (int64_t r = 0; r < k; r++) {
            double acc = B[i * k + r];
            for (int64_t e = rp[i]; e < d; e++)
                acc -= v[e] * X[(int64_t)ci[e] * k + r];
            X[i * k + r] = acc / v[d];
        }
    }
}

/* Adjoint of Y = A X for upstream G = dLoss/dY:
 *   GX = A^T G  (n_cols, k)      GV[e] = sum_r G[i,r] * X[col_e, r]   (dLoss/dA_ij = g_i x_j) */
void orc_spmv_adj(int32_t n_rows, int32_t n_cols, const int32_t *rp, const int32_t *ci,
                  const double *v, int32_t k, const double *X, const double *G, double *GX,
                  double *GV) {
    if (GX)
        for (int64_t j = 0; j < (int64_t)n_cols * k; j++) GX[j] = 0.0;
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int64_t c = ci[e];
            if (GX)
                for (int64_t r = 0; r < k; r++) GX[c * k + r] += v[e] * G[i * k + r];
            if (GV) {
                double s = 0.0;
                for (int64_t r = 0; r < k; r++) s += G[i * k + r] * X[c * k + r];
                GV[e] = s;
            }
        }
    }
}

/* Adjoint of L X = B for upstream G = dLoss/dX: solve L^T Lam = G (backward substitution,
 * column-oriented over L's rows), GB = Lam, GV[e] = -sum_r Lam[i,r] * X[col_e,r] for every
 * stored entry (i, col_e) including the diagonal (dLoss/dL_ij = -lam_i x_j).
 * work is caller scratch of n*k doubles. */
void orc_sptrsv_adj(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t k,
                    const double *X, const double *G, double *GB, double *GV, double *work) {
    for (int64_t j = 0; j < (int64_t)n * k; j++) work[j] = G[j];
    for (int64_t i = n - 1; i >= 0; i--) {
        int64_t d = rp[i + 1] - 1;
        for (int64_t r = 0; r < k; r++) {
            double lam = work[i * k + r] / v[d];
            GB[i * k + r] = lam;
            for (int64_t e = rp[i]; e < d; e++)
                work[(int64_t)ci[e] * k + r] -= v[e] * lam;
        }
    }
    if (GV) {
        for (int64_t i = 0; i < n; i++) {
            for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
                double s = 0.0;
                for (int64_t r = 0; r < k; r++) s += GB[i * k + r] * X[(int64_t)ci[e] * k + r];
                GV[e] = -s;
            }
        }
    }
}

/* ASAP levels of the dependence DAG of forward substitution: lev[i] = 0 without
 * off-diagonals, else 1 + max over off-diagonal columns.  Returns the number of levels. */
int64_t orc_levels(int32_t n, const int32_t *rp, const int32_t *ci, int64_t *lev) {
    int64_t nlev = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t l = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int64_t c = ci[e];
            if (c == i) continue;
            if (lev[c] + 1 > l) l = lev[c] + 1;
        }
        lev[i] = l;
        if (l + 1 > nlev) nlev = l + 1;
    }
    return n > 0 ? nlev : 0;
}

/* ----------------------------------------------------------------------------------------
 * Input validation (kinds: 0 = SpMV, 1 = lower triangular with diagonal last,
 * 2 = upper triangular with diagonal first, the transpose of kind 1)
 * Returns 0 when valid, else a positive code naming the first violation.
 * -------------------------------------------------------------------------------------- */
int32_t orc_validate(int32_t kind, int32_t n_rows, int32_t n_cols, const int32_t *rp,
                     const int32_t *ci) {
    if (n_rows < 0 || n_cols < 0) return 1;
    if (rp[0] != 0) return 2;
    for (int64_t i = 0; i < n_rows; i++)
        if (rp[i + 1] < rp[i]) return 2;
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            if (ci[e] < 0 || ci[e] >= n_cols) return 3;
            if (e > rp[i] && ci[e] <= ci[e - 1]) return 4;
        }
    }
    if (kind == 1 || kind == 2) {
        if (n_rows != n_cols) return 5;
        for (int64_t i = 0; i < n_rows; i++) {
            if (rp[i + 1] == rp[i]) return 6;
            if (kind == 1 && ci[rp[i + 1] - 1] != i) return 6;
            if (kind == 2 && ci[rp[i]] != i) return 6;
        }
    }
    return 0;
}

/* Transpose by a stable counting sort on column; perm[eT] = e (position in A). */
void orc_transpose(int32_t n_rows, int32_t n_cols, const int32_t *rp, const int32_t *ci,
                   const double *v, int32_t *rpT, int32_t *ciT, double *vT, int64_t *perm) {
    int64_t nnz = rp[n_rows];
    for (int64_t j = 0; j <= n_cols; j++) rpT[j] = 0;
    for (int64_t e = 0; e < nnz; e++) rpT[ci[e] + 1]++;
    for (int64_t j = 0; j < n_cols; j++) rpT[j + 1] += rpT[j];
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (n_cols + 1));
    for (int64_t j = 0; j < n_cols; j++) next[j] = rpT[j];
    for (int64_t i = 0; i < n_rows; i++) {
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int64_t p = next[ci[e]]++;
            ciT[p] = (int32_t)i;
            if (vT) vT[p] = v[e];
            perm[p] = e;
        }
    }
    free(next);
}

/* ----------------------------------------------------------------------------------------
 * Inspector (Algorithm 1)
 * -------------------------------------------------------------------------------------- */

#define F_S0 1
#define F_S1 2
#define F_S2 4
#define F_SEP 8
#define F_RECT 16
#define F_RUNS 32

#define NREG 8  /* part, pos0, T, first_codelet, chosen_strategy, cost[3] */
#define NCOD 18 /* type, flags, part, region, u, m, nn, P, row0, row_step, op0, op_step,
                   col0, sigma0, sigma1, aux_off, aux_len, cost */

typedef struct {
    int64_t header[9]; /* kind, n_rows, n_cols, nnz, t, n_parts, n_regions, n_codelets, aux_len */
    int64_t *part_ptr;
    int64_t *part_rows;
    int64_t *regions;
    int64_t *codelets;
    int32_t *aux;
} orc_plan;

/* The kernel's statement, in the notation of Sec. III-A: iteration i0 is an outer
 * iteration (row q), i1 its operation index; the three access functions are
 *   f0(i0)     = q                   (output: y for SpMV, x for the solve)
 *   f1(i0, i1) = opstart(q) + i1     (matrix values)
 *   f2(i0, i1) = col[f1(i0, i1)]     (input vector)
 * For the triangular kinds the diagonal is not an operation: the executor divides by it. */
typedef struct {
    int32_t kind;
    const int32_t *rp;
    const int32_t *ci;
} kernel_t;

static int64_t opstart(const kernel_t *K, int64_t q) {
    return K->kind == 2 ? (int64_t)K->rp[q] + 1 : (int64_t)K->rp[q];
}
static int64_t nops(const kernel_t *K, int64_t q) {
    int64_t len = (int64_t)K->rp[q + 1] - K->rp[q];
    return K->kind == 0 ? len : len - 1;
}
static int64_t f1(const kernel_t *K, int64_t q, int64_t i1) { return opstart(K, q) + i1; }
static int64_t f2(const kernel_t *K, int64_t q, int64_t i1) { return K->ci[f1(K, q, i1)]; }

/* Classification of the candidate rows q[0..m-1] (Sec. III-B, III-D). */
typedef struct {
    int rect, s0, s1, sep, s2;
    int64_t nn;
} cls_t;

static cls_t classify(const kernel_t *K, const int64_t *q, int64_t m) {
    cls_t c;
    /* the iteration space is rectangular when every row has the same op count */
    c.nn = nops(K, q[0]);
    c.rect = 1;
    for (int64_t a = 1; a < m; a++)
        if (nops(K, q[a]) != c.nn) c.rect = 0;
    /* f0 strided: all FOPD_i0 of f0 equal */
    c.s0 = 1;
    for (int64_t a = 1; a + 1 < m; a++)
        if (q[a + 1] - q[a] != q[1] - q[0]) c.s0 = 0;
    c.s1 = c.sep = c.s2 = 0;
    if (!c.rect) return c;
    /* f1 strided: FOPD_i1 of f1 is always 1; all FOPD_i0 of f1 equal */
    c.s1 = 1;
    if (c.nn > 0) {
        int64_t d0 = m > 1 ? f1(K, q[1], 0) - f1(K, q[0], 0) : 0;
        for (int64_t a = 0; a + 1 < m; a++)
            for (int64_t b = 0; b < c.nn; b++)
                if (f1(K, q[a + 1], b) - f1(K, q[a], b) != d0) c.s1 = 0;
    }
    /* f2: FOPD_i0 all equal (separable), then also FOPD_i1 all equal (strided) */
    c.sep = 1;
    if (c.nn > 0 && m > 1) {
        int64_t d0 = f2(K, q[1], 0) - f2(K, q[0], 0);
        for (int64_t a = 0; a + 1 < m; a++)
            for (int64_t b = 0; b < c.nn; b++)
                if (f2(K, q[a + 1], b) - f2(K, q[a], b) != d0) c.sep = 0;
    }
    c.s2 = c.sep;
    if (c.sep && c.nn > 1) {
        int64_t d1 = f2(K, q[0], 1) - f2(K, q[0], 0);
        for (int64_t a = 0; a < m; a++)
            for (int64_t b = 0; b + 1 < c.nn; b++)
                if (f2(K, q[a], b + 1) - f2(K, q[a], b) != d1) c.s2 = 0;
    }
    return c;
}

static int strided_count(cls_t c) { return c.s0 + c.s1 + c.s2; }

/* number of maximal runs of consecutive columns within row q */
static int64_t row_runs(const kernel_t *K, int64_t q) {
    int64_t n = nops(K, q), r = 0;
    for (int64_t b = 0; b < n; b++)
        if (b == 0 || f2(K, q, b) != f2(K, q, b - 1) + 1) r++;
    return r;
}

/* A codelet over candidate rows q[0..m-1]: its record fields, table sizes and Eq. (1) cost. */
typedef struct {
    cls_t c;
    int64_t m, P, xtab_len, aux_len, cost;
    int runs;
} codelet_t;

static codelet_t make_codelet(const kernel_t *K, const int64_t *q, int64_t m) {
    codelet_t d;
    d.c = classify(K, q, m);
    d.m = m;
    d.P = 0;
    for (int64_t a = 0; a < m; a++) d.P += nops(K, q[a]);
    d.runs = 0;
    d.xtab_len = 0;
    if (!d.c.s2) {
        int64_t plain, R;
        if (d.c.sep) { /* one offset pattern shared by every row */
            plain = d.c.nn;
            R = row_runs(K, q[0]);
        } else { /* every column listed */
            plain = d.P;
            R = 0;
            for (int64_t a = 0; a < m; a++) R += row_runs(K, q[a]);
        }
        if (2 * R < plain) {
            d.runs = 1;
            d.xtab_len = 2 * R;
        } else {
            d.xtab_len = plain;
        }
    }
    int64_t s0 = d.c.s0 ? 0 : m, s1 = d.c.s1 ? 0 : m, cnt = d.c.rect ? 0 : m;
    d.aux_len = s0 + s1 + cnt + d.xtab_len;
    /* Eq. (1): c = |p| + (number of access functions) + sum of table sizes; row counts of a
       ragged codelet are loop bounds, not accesses, and are not costed */
    d.cost = d.P + 3 + s0 + s1 + d.xtab_len;
    return d;
}

/* Longest run of rows from position u of the window (T rows at q) that keeps at least
 * `need` strided access functions; 0 if the single row already has fewer. */
static int64_t longest(const kernel_t *K, const int64_t *q, int64_t T, int64_t u, int need) {
    int64_t best = 0;
    for (int64_t m = 1; u + m <= T; m++) {
        if (strided_count(classify(K, q + u, m)) < need) break;
        best = m;
    }
    return best;
}

/* One strategy over the window; returns its total cost; if emit, writes codelet starts/sizes */
static int64_t strategy(const kernel_t *K, const int64_t *q, int64_t T, int s, int64_t *us,
                        int64_t *ms, int64_t *count) {
    int64_t u = 0, total = 0, nc = 0;
    while (u < T) {
        int64_t m;
        if (s == 0) { /* BLAS_first: all three strided if possible, then two */
            m = longest(K, q, T, u, 3);
            if (m < 1) m = longest(K, q, T, u, 2);
        } else if (s == 1) { /* PSCI_first */
            m = longest(K, q, T, u, 2);
        } else { /* PSCII_first */
            m = longest(K, q, T, u, 1);
        }
        total += make_codelet(K, q + u, m).cost;
        if (us) { us[nc] = u; ms[nc] = m; }
        nc++;
        u += m;
    }
    if (count) *count = nc;
    return total;
}

typedef struct {
    int64_t *v;
    int64_t n, cap;
} vec64;
typedef struct {
    int32_t *v;
    int64_t n, cap;
} vec32;
static void push64(vec64 *a, int64_t x) {
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 1024;
        a->v = (int64_t *)realloc(a->v, sizeof(int64_t) * a->cap);
    }
    a->v[a->n++] = x;
}
static void push32(vec32 *a, int64_t x) {
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 1024;
        a->v = (int32_t *)realloc(a->v, sizeof(int32_t) * a->cap);
    }
    a->v[a->n++] = (int32_t)x;
}

/* Append a codelet's record and tables in the canonical layout. */
static void emit(const kernel_t *K, const int64_t *q, int64_t m, int64_t part, int64_t region,
                 int64_t u, vec64 *cod, vec32 *aux) {
    codelet_t d = make_codelet(K, q, m);
    int flags = (d.c.s0 ? F_S0 : 0) | (d.c.s1 ? F_S1 : 0) | (d.c.s2 ? F_S2 : 0) |
                (d.c.sep ? F_SEP : 0) | (d.c.rect ? F_RECT : 0) | (d.runs ? F_RUNS : 0);
    int64_t col0 = nops(K, q[0]) > 0 ? f2(K, q[0], 0) : 0;
    int64_t aux_off = aux->n;
    int64_t type = strided_count(d.c) == 3 ? 0 : (strided_count(d.c) == 2 ? 1 : 2);
    push64(cod, type);
    push64(cod, flags);
    push64(cod, part);
    push64(cod, region);
    push64(cod, u);
    push64(cod, m);
    push64(cod, d.c.rect ? d.c.nn : -1);
    push64(cod, d.P);
    push64(cod, q[0]);
    push64(cod, (d.c.s0 && m >= 2) ? q[1] - q[0] : 0);
    push64(cod, opstart(K, q[0]));
    push64(cod, (d.c.s1 && m >= 2) ? opstart(K, q[1]) - opstart(K, q[0]) : 0);
    push64(cod, col0);
    push64(cod, (d.c.sep && m >= 2 && d.c.nn > 0) ? f2(K, q[1], 0) - f2(K, q[0], 0) : 0);
    push64(cod, (d.c.s2 && d.c.nn >= 2) ? f2(K, q[0], 1) - f2(K, q[0], 0) : 0);
    push64(cod, aux_off);
    push64(cod, d.aux_len);
    push64(cod, d.cost);
    if (!d.c.s0)
        for (int64_t a = 0; a < m; a++) push32(aux, q[a]);
    if (!d.c.s1)
        for (int64_t a = 0; a < m; a++) push32(aux, opstart(K, q[a]));
    if (!d.c.rect)
        for (int64_t a = 0; a < m; a++) push32(aux, nops(K, q[a]));
    if (!d.c.s2) {
        int64_t last = d.c.sep ? 1 : m; /* a shared pattern is stored once */
        for (int64_t a = 0; a < last; a++) {
            int64_t n = nops(K, q[a]);
            int64_t base = d.c.sep ? col0 : 0;
            if (!d.runs) {
                for (int64_t b = 0; b < n; b++) push32(aux, f2(K, q[a], b) - base);
            } else {
                int64_t b = 0;
                while (b < n) {
                    int64_t e = b + 1;
                    while (e < n && f2(K, q[a], e) == f2(K, q[a], e - 1) + 1) e++;
                    push32(aux, f2(K, q[a], b) - base);
                    push32(aux, e - b);
                    b = e;
                }
            }
        }
    }
}

/* ----------------------------------------------------------------------------------------
 * The BLAS-only cover of a window: the ablation of Sec. V-A and V-B, where every codelet is
 * a BLAS codelet (all three access functions strided, Sec. III-B).  Rows whose columns do
 * not keep one stride cannot be whole BLAS codelets, so codelets become column slices
 * (Sec. III-C, the three-BLAS cover of the worked example): a codelet covers ops
 * [a, a + w) of m consecutive rows of the window.
 *   1. Each row's ops are cut into slices from left to right; a slice starts at the first op
 *      not yet cut and takes the following ops while the column difference stays the one
 *      between its first two ops (a slice of one op has stride 0).
 *   2. Slices are taken row by row (window order), left to right; an unused slice starts a
 *      codelet, which grows down to the next row of the window while that row has an unused
 *      slice at the same op offset with the same width and column stride, and the row
 *      number, value index and first column still move by the steps of the first two rows.
 * Rows without ops get no codelet.  Each codelet costs |p| + 3 by Eq. (1) (no tables).
 * -------------------------------------------------------------------------------------- */
typedef struct {
    int64_t a, w, s1;
    int used;
} slice_t;

static void emit_slice(const kernel_t *K, const int64_t *q, int64_t m, int64_t a, int64_t w, int64_t s1,
                       int64_t part, int64_t region, int64_t u, vec64 *cod) {
    int64_t op0 = opstart(K, q[0]) + a;
    push64(cod, 0); /* BLAS */
    push64(cod, F_S0 | F_S1 | F_S2 | F_SEP | F_RECT);
    push64(cod, part);
    push64(cod, region);
    push64(cod, u);
    push64(cod, m);
    push64(cod, w);
    push64(cod, m * w);
    push64(cod, q[0]);
    push64(cod, m >= 2 ? q[1] - q[0] : 0);
    push64(cod, op0);
    push64(cod, m >= 2 ? opstart(K, q[1]) - opstart(K, q[0]) : 0);
    push64(cod, K->ci[op0]);
    push64(cod, m >= 2 ? f2(K, q[1], a) - f2(K, q[0], a) : 0);
    push64(cod, w >= 2 ? s1 : 0);
    push64(cod, 0); /* aux_off: no tables */
    push64(cod, 0);
    push64(cod, m * w + 3);
}

/* Emits the window's BLAS-only codelets; returns their total Eq. (1) cost. */
static int64_t blas_only_window(const kernel_t *K, const int64_t *q, int64_t T, int64_t part, int64_t region,
                                vec64 *cod) {
    slice_t **sl = (slice_t **)calloc(T, sizeof(slice_t *));
    int64_t *ns = (int64_t *)calloc(T, sizeof(int64_t));
    for (int64_t u = 0; u < T; u++) {
        int64_t n = nops(K, q[u]);
        sl[u] = (slice_t *)calloc(n > 0 ? n : 1, sizeof(slice_t));
        int64_t a = 0;
        while (a < n) {
            int64_t w = 1, s1 = 0;
            if (a + 1 < n) {
                s1 = f2(K, q[u], a + 1) - f2(K, q[u], a);
                w = 2;
                while (a + w < n && f2(K, q[u], a + w) - f2(K, q[u], a + w - 1) == s1) w++;
            }
            slice_t s = {a, w, s1, 0};
            sl[u][ns[u]++] = s;
            a += w;
        }
    }
    int64_t total = 0;
    for (int64_t u = 0; u < T; u++) {
        for (int64_t j = 0; j < ns[u]; j++) {
            slice_t *s = &sl[u][j];
            if (s->used) continue;
            s->used = 1;
            int64_t m = 1;
            while (u + m < T) {
                /* the next row's slice at the same op offset, unused, of the same shape */
                slice_t *nx = NULL;
                for (int64_t jj = 0; jj < ns[u + m]; jj++)
                    if (sl[u + m][jj].a == s->a) nx = &sl[u + m][jj];
                if (!nx || nx->used || nx->w != s->w || nx->s1 != s->s1) break;
                /* the steps of the first two rows hold for rows, value starts and first columns */
                if (m >= 2) {
                    const int64_t *r = q + u;
                    if (r[m] - r[m - 1] != r[1] - r[0]) break;
                    if (opstart(K, r[m]) - opstart(K, r[m - 1]) != opstart(K, r[1]) - opstart(K, r[0])) break;
                    if (f2(K, r[m], s->a) - f2(K, r[m - 1], s->a) != f2(K, r[1], s->a) - f2(K, r[0], s->a)) break;
                }
                nx->used = 1;
                m++;
            }
            emit_slice(K, q + u, m, s->a, s->w, s->s1, part, region, u, cod);
            total += m * s->w + 3;
        }
    }
    for (int64_t u = 0; u < T; u++) free(sl[u]);
    free(sl);
    free(ns);
    return total;
}

/* Inspector.  kind: 0 SpMV, 1 lower solve (diagonal last), 2 transposed solve (upper,
 * diagonal first; levels run from the last row).  t: window.  sample: mine only windows
 * w with w % sample == 0 or w the last one (1 = all); unmined windows get chosen = -1.
 * only_blas: every window takes its BLAS-only cover (chosen = 3, costs [total, 0, 0]). */
orc_plan *orc_inspect_ex(int32_t kind, int32_t n_rows, int32_t n_cols, const int32_t *rp,
                         const int32_t *ci, int32_t t, int32_t sample, int32_t only_blas) {
    kernel_t K = {kind, rp, ci};
    orc_plan *p = (orc_plan *)calloc(1, sizeof(orc_plan));
    int64_t n = n_rows;
    /* 1) grouping independent iterations: dependences and partitions */
    int64_t *grp = (int64_t *)calloc(n > 0 ? n : 1, sizeof(int64_t));
    int64_t nparts = 0;
    if (kind == 0) {
        nparts = n > 0 ? 1 : 0; /* no dependences: one group of all rows */
    } else if (kind == 1) {
        nparts = orc_levels(n_rows, rp, ci, grp);
    } else { /* reverse levels over the upper-triangular rows */
        for (int64_t i = n - 1; i >= 0; i--) {
            int64_t l = 0;
            for (int64_t e = rp[i] + 1; e < rp[i + 1]; e++)
                if (grp[ci[e]] + 1 > l) l = grp[ci[e]] + 1;
            grp[i] = l;
            if (l + 1 > nparts) nparts = l + 1;
        }
    }
    p->part_ptr = (int64_t *)calloc(nparts + 1, sizeof(int64_t));
    p->part_rows = (int64_t *)calloc(n > 0 ? n : 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) p->part_ptr[grp[i] + 1]++;
    for (int64_t l = 0; l < nparts; l++) p->part_ptr[l + 1] += p->part_ptr[l];
    {
        int64_t *fill = (int64_t *)calloc(nparts + 1, sizeof(int64_t));
        for (int64_t i = 0; i < n; i++) p->part_rows[p->part_ptr[grp[i]] + fill[grp[i]]++] = i;
        free(fill);
    }
    free(grp);
    /* 2) codelet creation: windows of t consecutive iterations of each group */
    vec64 reg = {0}, cod = {0};
    vec32 aux = {0};
    int64_t nreg = 0, w = 0, total_w = 0;
    for (int64_t l = 0; l < nparts; l++)
        total_w += (p->part_ptr[l + 1] - p->part_ptr[l] + t - 1) / t;
    int64_t *us = (int64_t *)malloc(sizeof(int64_t) * (t + 1));
    int64_t *ms = (int64_t *)malloc(sizeof(int64_t) * (t + 1));
    for (int64_t l = 0; l < nparts; l++) {
        int64_t size = p->part_ptr[l + 1] - p->part_ptr[l];
        for (int64_t pos0 = 0; pos0 < size; pos0 += t, w++) {
            int64_t T = size - pos0 < t ? size - pos0 : t;
            const int64_t *q = p->part_rows + p->part_ptr[l] + pos0;
            push64(&reg, l);
            push64(&reg, pos0);
            push64(&reg, T);
            if (!(sample <= 1 || w % sample == 0 || w == total_w - 1)) {
                for (int z = 0; z < 5; z++) push64(&reg, -1);
                nreg++;
                continue;
            }
            if (only_blas) {
                push64(&reg, cod.n / NCOD);
                push64(&reg, 3);
                int64_t at = reg.n;
                for (int s = 0; s < 3; s++) push64(&reg, 0);
                reg.v[at] = blas_only_window(&K, q, T, l, nreg, &cod);
                nreg++;
                continue;
            }
            int64_t cost[3];
            for (int s = 0; s < 3; s++) cost[s] = strategy(&K, q, T, s, NULL, NULL, NULL);
            int best = 0;
            for (int s = 1; s < 3; s++)
                if (cost[s] < cost[best]) best = s;
            int64_t nc = 0;
            strategy(&K, q, T, best, us, ms, &nc);
            push64(&reg, cod.n / NCOD);
            push64(&reg, best);
            for (int s = 0; s < 3; s++) push64(&reg, cost[s]);
            for (int64_t c = 0; c < nc; c++) emit(&K, q + us[c], ms[c], l, nreg, us[c], &cod, &aux);
            nreg++;
        }
    }
    free(us);
    free(ms);
    p->regions = reg.v;
    p->codelets = cod.v;
    p->aux = aux.v;
    p->header[0] = kind;
    p->header[1] = n_rows;
    p->header[2] = n_cols;
    p->header[3] = rp[n_rows];
    p->header[4] = t;
    p->header[5] = nparts;
    p->header[6] = nreg;
    p->header[7] = cod.n / NCOD;
    p->header[8] = aux.n;
    return p;
}

orc_plan *orc_inspect(int32_t kind, int32_t n_rows, int32_t n_cols, const int32_t *rp,
                      const int32_t *ci, int32_t t, int32_t sample) {
    return orc_inspect_ex(kind, n_rows, n_cols, rp, ci, t, sample, 0);
}

/* Debug view used by the tests: the strided-function count k(u, m) of rows q[0..m-1] of a
 * kind, and its flag word. */
int32_t orc_classify(int32_t kind, const int32_t *rp, const int32_t *ci, const int64_t *q,
                     int64_t m, int64_t *nn_out) {
    kernel_t K = {kind, rp, ci};
    cls_t c = classify(&K, q, m);
    if (nn_out) *nn_out = c.nn;
    return (c.s0 ? F_S0 : 0) | (c.s1 ? F_S1 : 0) | (c.s2 ? F_S2 : 0) | (c.sep ? F_SEP : 0) |
           (c.rect ? F_RECT : 0);
}

void orc_plan_free(orc_plan *p) {
    if (!p) return;
    free(p->part_ptr);
    free(p->part_rows);
    free(p->regions);
    free(p->codelets);
    free(p->aux);
    free(p);
}
