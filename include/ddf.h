/*
 * libddf — DDF inspector/executor for sparse matrix-vector multiply (SpMV) and the sparse
 * lower-triangular solve (SpTRSV) on AMD Instinct MI355X (gfx950), FP64.
 *
 * The method is the DDF framework of "Vectorizing Sparse Matrix Codes with Dependency
 * Driven Trace Analysis" (Cetinic, Cheshmi, Mehri Dehnavi): an inspector (Algorithm 1,
 * Sec. IV-A) mines a CSR pattern into partially strided codelets (Sec. III: BLAS, PSC I and
 * PSC II, classified by the first order partial differences of the three access functions
 * and chosen per window by the cost model of Eq. (1)), grouped into partitions of
 * independent rows (dependence levels for the solve); an executor (Sec. IV-B) runs the
 * codelets partition by partition.  Here the executor is a set of HIP kernels; the solve
 * runs in one persistent dataflow kernel (a row waits only for the solution values it reads;
 * no level barriers), in one single-block kernel when every level fits one block (one
 * right-hand side), or in one launch per level, as set by the options or the autotuner.
 *
 * Conventions for every call below:
 *  - Host arrays are read during the call only; nothing keeps a pointer to them.
 *  - Device pointers are plain HIP device addresses owned by the caller.  Dense vectors
 *    are row-major (rows, nrhs): element (i, r) at [i * nrhs + r].
 *  - Outputs are overwritten (y = A x, never y += A x).
 *  - Execution calls are asynchronous on `stream` (a hipStream_t, NULL = default stream),
 *    allocate nothing, and copy nothing synchronously, so they may be captured in a graph.
 *    Per plan, one forward call (SpMV, solve) and one adjoint call (ddf_spmv_adjoint,
 *    ddf_sptrsv_adjoint, ddf_sptrsv_value_grad) may be in flight at a time, on any
 *    streams: the solves' scratch (the dataflow kernel's counters, per-call streams, the
 *    values in transposed order) is per direction.
 *  - Arguments are validated before any launch.  On an error no kernel is launched,
 *    outputs are untouched, and ddf_last_error() holds a message (thread-local).
 *  - A zero diagonal is not an error: it gives inf/nan by IEEE rules.  The dataflow and
 *    one-launch-per-level solves compute (b_i - sum) / L_ii as forward substitution does, so
 *    every entry has the substitution's IEEE class (+inf, -inf, nan); the single-block solve
 *    divides each value of a row by L_ii before summing, so the same entries are non-finite
 *    but some that substitution makes +-inf come out nan.
 */
#ifndef DDF_H
#define DDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddf_plan_s *ddf_plan_t;
typedef struct ddf_graph_s *ddf_graph_t;
typedef void *ddf_stream_t; /* hipStream_t */

typedef enum {
    DDF_SPMV = 0,         /* y = A x; A any n_rows x n_cols CSR                         */
    DDF_SPTRSV_LOWER = 1, /* L x = b; L square, lower, diagonal stored last in each row */
} ddf_kind;

typedef enum {
    DDF_OK = 0,
    DDF_E_ARG = 1,         /* bad argument (null pointer, nrhs outside 1..32, aliasing ...) */
    DDF_E_CSR = 2,         /* malformed CSR: row_ptr not monotone / columns unsorted,
                              repeated or out of range                                      */
    DDF_E_NOT_LOWER = 3,   /* SpTRSV: an entry above the diagonal                          */
    DDF_E_NO_DIAG = 4,     /* SpTRSV: a row without its diagonal as last entry             */
    DDF_E_KIND = 5,        /* call does not match the plan's kind (or batch vs single)     */
    DDF_E_NOMEM = 6,       /* host or device allocation failed                             */
    DDF_E_HIP = 7,         /* a HIP runtime call failed                                    */
    DDF_E_DEVICE = 8,      /* a kernel raised the plan's device error flag (level-wait
                              watchdog); reported by ddf_plan_sync_status                  */
    DDF_E_UNSUPPORTED = 9, /* e.g. execution on a host-only plan, no adjoint plan built    */
} ddf_status;

typedef struct {
    int32_t window;        /* t: rows per inspection window (Alg. 1, GetConsecutiveIterations);
                              default 64, range 1..1024                                     */
    int32_t build_adjoint; /* 1: also build the transposed plan (A^T, or L^T on reverse
                              levels) used by the adjoint calls; default 1                  */
    int32_t host_only;     /* 1: inspect on the host only; no device tables are made; the
                              plan can be exported and queried but not executed            */
    int32_t threads;       /* host threads for the inspector; 0 = hardware concurrency     */
    int32_t ops_per_lane;  /* schedule: target operations per lane (lanes per row =
                              next power of two of row length / this); 0 = default 4       */
    int32_t rows_passes;   /* schedule: row passes per wavefront task; 0 = default 2       */
    int32_t xcd_remap;     /* schedule: give each XCD a contiguous block range; -1 default */
    int32_t solve_blocks;  /* schedule (solve): 256-thread blocks of the persistent dataflow
                              kernel; 0 = every block the device keeps resident at once     */
    int32_t solve_path;    /* solve kernel: 0 auto (single-block when every level fits one
                              1024-lane pass, else the dataflow kernel; batches: the
                              dataflow kernel), 1 the dataflow kernel (one persistent
                              launch, batches too), 2 single-block when possible, 3 one
                              launch per level (batches: over all matrices, one op per
                              lane, one row pass)                                          */
    int32_t thin_helpers;  /* single-block solve: helper blocks that pull the next levels'
                              tables into the solver's L2; -1 default (4), 0 none, max 8  */
    int32_t thin_ahead;    /* single-block solve: levels the helpers run ahead; 0 default
                              (24), at least 8                                              */
    int32_t thin_ring;     /* single-block solve: LDS ring of recent solutions, in rows; a
                              power of two in 256..16384; 0 default (16384)                */
    int32_t thin_lanes;    /* single-block solve: most lanes a level may use; a level with
                              more is cut into consecutive sub-levels (its rows are
                              independent, so any cut keeps the order); a multiple of 64 in
                              64..1024; 0 default: chosen by a cost model (each level costs a
                              fixed latency plus the issue time of the waves sharing a SIMD),
                              and a level wider than 1024 lanes rules the single-block solve
                              out                                                           */
    int32_t only_blas;     /* 1: the BLAS-only ablation (Sec. V-A, V-B): every window covered by
                              BLAS codelets only, as column slices of rows (a codelet is ops
                              [a, a + w) of m rows, all three access functions strided);
                              rows are then shared by several codelets, whose partial sums
                              the executor combines with FP64 atomic adds (results are not
                              bitwise reproducible run to run).  Such a plan runs ddf_spmv(_v)
                              and ddf_sptrsv(_v) (one launch per level) and exports its
                              tables; the adjoint calls and ddf_autotune return
                              DDF_E_UNSUPPORTED, and so does a batch.  Default 0          */
} ddf_opts;

typedef struct {
    int32_t n_rows, n_cols;
    const int32_t *row_ptr; /* [n_rows + 1], row_ptr[0] = 0, non-decreasing              */
    const int32_t *col_idx; /* [nnz], strictly increasing within a row, in [0, n_cols)   */
    const double *values;   /* [nnz]; may be NULL for a pattern-only plan (then every
                               call needs explicit values: the _v forms)                 */
} ddf_csr_host;

/* Canonical plan tables (host memory owned by the plan, valid until ddf_plan_destroy).
 * Layout of the paper's codelet list cList, one fixed-width int64 record per item:
 *   header[9]   kind, n_rows, n_cols, nnz, t, n_parts, n_regions, n_codelets, aux_len
 *   part_ptr    [n_parts + 1]  partitions (levels) as ranges of part_rows
 *   part_rows   [n_rows]       rows of each partition, ascending
 *   regions     [n_regions][8] part, pos0, T, first_codelet, chosen_strategy, cost[3]
 *   codelets    [n_codelets][18] type (0 BLAS, 1 PSC I, 2 PSC II), flags (S0 1, S1 2,
 *               S2 4, SEP 8, RECT 16, RUNS 32), part, region, u, m, nn (-1 if ragged), P,
 *               row0, row_step, op0, op_step, col0, sigma0, sigma1, aux_off, aux_len, cost
 *   aux         [aux_len] int32: per codelet ROWS (if !S0), OPSTART (if !S1), COUNTS
 *               (if !RECT), then the column table (if !S2): shared offsets, shared runs
 *               (offset, len), full columns, or full runs (start, len) per row.
 * `which` selects the forward plan (0) or the transposed/adjoint plan (1); for a batch
 * plan `mat` selects the member matrix.  perm (adjoint plan only) maps each entry of the
 * transposed CSR to the forward value it reads. */
typedef struct {
    const int64_t *header;
    const int64_t *part_ptr;
    const int64_t *part_rows;
    const int64_t *regions;
    const int64_t *codelets;
    const int32_t *aux;
    const int32_t *perm; /* NULL for the forward plan */
} ddf_plan_tables_t;

typedef struct {
    int32_t kind, nmat;
    int32_t n_rows, n_cols; /* totals over a batch */
    int64_t nnz;
    int64_t n_parts, n_regions, n_codelets, aux_len; /* forward plan(s), summed */
    int64_t codelets_by_type[3];                     /* BLAS, PSC I, PSC II */
    int64_t ops_by_type[3];
    int64_t n_tasks, n_tasks_adjoint;
    int64_t dev_plan_bytes;     /* forward device tables: records + aux + tasks (solve schedules: + one 64-byte codelet copy per task) */
    int64_t dev_plan_bytes_adj; /* adjoint-pass device tables (0 if none)            */
    int32_t has_adjoint;
    int32_t max_levels;
    double inspect_seconds;     /* wall time of the host inspector                   */
    uint64_t hash;              /* FNV-1a over the canonical tables                  */
    int32_t ops_per_lane, rows_passes, xcd_remap;
    int32_t solve_path;         /* kernel the solve uses: 1 multi-block, 2 single-block,
                                   3 one launch per level                                */
    int32_t solve_path_adj;     /* same for the adjoint solve (0 for SpMV plans)          */
    int32_t reserved;
    double phase_seconds[5];    /* wall time of ddf_inspect's phases: [0] Alg. 1 on the
                                   forward pattern(s) (inspect_seconds minus [1]), [1] the
                                   transposition and the adjoint plan's Alg. 1, [2] device
                                   records and tables (packing), [3] single-block solve
                                   records, [4] schedules, uploads and the rest            */
} ddf_plan_info_t;

typedef enum {
    DDF_OP_SPMV = 0,
    DDF_OP_SPMV_ADJ = 1,
    DDF_OP_SPTRSV = 2,
    DDF_OP_SPTRSV_ADJ = 3,
    DDF_OP_SPTRSV_T = 4, /* the transposed solve alone (ddf_sptrsv_adjoint with d_gvals = NULL) */
    /* ddf_plan_traffic only: the bytes of a call's main kernel (the one ddf_plan_time_kernels
     * times): the product kernel of ddf_spmv_adjoint, the solve kernel of a transposed solve */
    DDF_OP_SPMV_ADJ_KERNEL = 5,
    DDF_OP_SPTRSV_ADJ_KERNEL = 6,
} ddf_op;

/* Defaults for ddf_opts (window 64, adjoint plan on). */
void ddf_opts_default(ddf_opts *o);

/* Inspector (Alg. 1) on a host CSR, then packing and upload of the device tables (unless
 * host_only).  Synchronous.  On success *out owns everything it made; on error *out = NULL.
 * Errors: DDF_E_ARG, DDF_E_CSR, DDF_E_NOT_LOWER, DDF_E_NO_DIAG, DDF_E_NOMEM, DDF_E_HIP. */
ddf_status ddf_inspect(ddf_kind kind, const ddf_csr_host *A, const ddf_opts *opts,
                       ddf_plan_t *out);

/* A batch of lower-triangular matrices solved in one launch, matrix b with nrhs[b] right
 * hand sides (1..32).  Each member gets its own plan (identical to ddf_inspect's);
 * execution concatenates them.  Packed layouts: values of matrix b follow those of b-1;
 * vector blocks (n_b, nrhs_b) row-major follow each other in b order. */
ddf_status ddf_inspect_batch(ddf_kind kind, int32_t nmat, const ddf_csr_host *mats,
                             const int32_t *nrhs, const ddf_opts *opts, ddf_plan_t *out);

/* Frees host tables, device tables, device copies of values and scratch.  NULL is a no-op.
 * The caller must make sure no execution on the plan is still in flight. */
ddf_status ddf_plan_destroy(ddf_plan_t plan);

/* SpMV executor (Listing 3 of the paper, one launch): Y = A X with the values captured at
 * inspect time.  d_x (n_cols, nrhs), d_y (n_rows, nrhs); they must not overlap. */
ddf_status ddf_spmv(ddf_plan_t plan, const double *d_x, double *d_y, int32_t nrhs,
                    ddf_stream_t stream);
/* Same with explicit device values d_vals[nnz] in the CSR order given at inspect time. */
ddf_status ddf_spmv_v(ddf_plan_t plan, const double *d_vals, const double *d_x, double *d_y,
                      int32_t nrhs, ddf_stream_t stream);

/* SpTRSV executor: L X = B on the plan's solve path: by default the single-block kernel when
 * eligible (one right-hand side, every level within one block), else the persistent dataflow
 * kernel (one launch: the output is first marked unsolved, then each row is solved once the
 * solution values it reads are there); solve_path 3: one launch per level.  d_b and d_x are
 * (n, nrhs); d_b == d_x (in place) is allowed (the dataflow path then takes one launch per
 * level); partial overlap is not. */
ddf_status ddf_sptrsv(ddf_plan_t plan, const double *d_b, double *d_x, int32_t nrhs,
                      ddf_stream_t stream);
ddf_status ddf_sptrsv_v(ddf_plan_t plan, const double *d_vals, const double *d_b, double *d_x,
                        int32_t nrhs, ddf_stream_t stream);

/* SpMV adjoint for upstream d_gy = dLoss/dY (n_rows, nrhs):
 *   d_gx    (n_cols, nrhs) = A^T G   (transposed plan, deterministic, no atomics)
 *   d_gvals [nnz]          = sum_r G[i,r] X[col,r]  (dLoss/dA_ij = g_i x_j)
 * Either output may be NULL.  Two launches: the value gradient, then the transposed product.
 * The value gradient runs over the forward plan's codelets (every op once, in the product's
 * lane layout) when nrhs is 2, 4, 8, 16 or 32 and d_gy, d_x are 16-byte aligned, otherwise
 * over the CSR pattern.  Needs build_adjoint. */
ddf_status ddf_spmv_adjoint(ddf_plan_t plan, const double *d_vals, const double *d_x,
                            const double *d_gy, double *d_gx, double *d_gvals, int32_t nrhs,
                            ddf_stream_t stream);

/* SpTRSV adjoint for upstream d_gx = dLoss/dX, given the forward solution d_x:
 *   d_gb    (n, nrhs) = Lam with L^T Lam = G   (reverse-level plan of L^T)
 *   d_gvals [nnz]     = -sum_r Lam[i,r] X[col,r] for every stored entry incl. the diagonal
 * d_gvals may be NULL (then d_x is not read).  The transposed solve, then the value gradient
 * over the CSR pattern of L.  Needs build_adjoint. */
ddf_status ddf_sptrsv_adjoint(ddf_plan_t plan, const double *d_vals, const double *d_x,
                              const double *d_gx, double *d_gb, double *d_gvals, int32_t nrhs,
                              ddf_stream_t stream);

/* The value gradient of the SpTRSV adjoint alone (the second half of ddf_sptrsv_adjoint),
 * from d_gb = Lam (n, nrhs) and the forward solution d_x (n, nrhs):
 *   d_gvals [nnz] = -sum_r Lam[i,r] X[col,r] for every stored entry of L incl. the diagonal.
 * With ddf_sptrsv_adjoint(..., d_gvals = NULL) before it, the adjoint's transposed solve no
 * longer depends on the forward solve, so the two can run on different streams.  Single
 * plans (not batches) built with build_adjoint; d_gvals must not overlap d_gb or d_x. */
ddf_status ddf_sptrsv_value_grad(ddf_plan_t plan, const double *d_x, const double *d_gb, double *d_gvals,
                                 int32_t nrhs, ddf_stream_t stream);

/* ddf_sptrsv_adjoint for callers that cannot allocate device memory, with the same arguments,
 * outputs and errors.  Its scratch (the values of L in the order of L^T, and the dataflow
 * solve's four counter lines) lives in one static device array of the library, 32 MiB + 512 B
 * per GPU, held until the process ends, instead of in the plan's own allocations: the call
 * makes no allocation and no library routine it calls does.  The transposed solve always runs
 * the dataflow kernel (in place, gb == gx: one launch per level).  Limits: at most 4194304
 * stored values in L (larger plans get DDF_E_ARG before any launch).  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (on different streams, or two
 * plans at once) race and give wrong results; run them one after another.  The counters start
 * from zero at each call (cleared by a kernel, not a memset); a watchdog trip is reported by
 * ddf_plan_sync_status on the plan. */
ddf_status ddf_sptrsv_adjoint_noalloc(ddf_plan_t plan, const double *d_vals, const double *d_x,
                                      const double *d_gx, double *d_gb, double *d_gvals, int32_t nrhs,
                                      ddf_stream_t stream);

/* Batched forms (plan from ddf_inspect_batch; nrhs per matrix fixed at inspect time).
 * d_vals_packed may be NULL to use the values captured at inspect time. */
ddf_status ddf_sptrsv_batch(ddf_plan_t plan, const double *d_vals_packed,
                            const double *d_b_packed, double *d_x_packed, ddf_stream_t stream);
ddf_status ddf_sptrsv_batch_adjoint(ddf_plan_t plan, const double *d_vals_packed,
                                    const double *d_x_packed, const double *d_gx_packed,
                                    double *d_gb_packed, double *d_gvals_packed,
                                    ddf_stream_t stream);

/* hipGraph of one batched solve (forward, or adjoint when adjoint = 1) on fixed buffers:
 * captured once, replayed by ddf_graph_launch on any stream.  ddf_autotune replaces the
 * plan's schedule buffers: a graph captured before it (this one, or any capture of the
 * execution calls) would read freed memory, so ddf_graph_launch refuses it with DDF_E_ARG;
 * capture again after tuning.  Destroy a plan's graphs before the plan. */
ddf_status ddf_graph_create_batch(ddf_plan_t plan, int32_t adjoint, const double *d_vals_packed,
                                  const double *d_in_packed, const double *d_x_packed,
                                  double *d_out_packed, double *d_gvals_packed,
                                  ddf_graph_t *out);
ddf_status ddf_graph_launch(ddf_graph_t graph, ddf_stream_t stream);
ddf_status ddf_graph_destroy(ddf_graph_t graph);

/* Plain GPU comparators on the same device CSR the plan holds (no codelets):
 * CSR-vector SpMV; one launch per level for the solve; FP64-atomic SpMV adjoint; one launch
 * per reverse level for the solve adjoint.  Same argument rules as the DDF forms. */
ddf_status ddf_plain_spmv(ddf_plan_t plan, const double *d_vals, const double *d_x, double *d_y,
                          int32_t nrhs, ddf_stream_t stream);
ddf_status ddf_plain_sptrsv(ddf_plan_t plan, const double *d_vals, const double *d_b,
                            double *d_x, int32_t nrhs, ddf_stream_t stream);
ddf_status ddf_plain_spmv_adjoint(ddf_plan_t plan, const double *d_vals, const double *d_x,
                                  const double *d_gy, double *d_gx, double *d_gvals,
                                  int32_t nrhs, ddf_stream_t stream);
ddf_status ddf_plain_sptrsv_adjoint(ddf_plan_t plan, const double *d_vals, const double *d_x,
                                    const double *d_gx, double *d_gb, double *d_gvals,
                                    int32_t nrhs, ddf_stream_t stream);
/* Per-matrix launches of the single-matrix persistent solve over a batch plan. */
ddf_status ddf_sptrsv_batch_per_matrix(ddf_plan_t plan, const double *d_vals_packed,
                                       const double *d_b_packed, double *d_x_packed,
                                       ddf_stream_t stream);

/* Autotuner: times schedule candidates (SpMV: ops per lane, row passes, XCD remap; solves:
 * single-block helper settings, one launch per level, dataflow grid sizes) for `op` with nrhs
 * right-hand sides on scratch buffers, keeps the fastest in the plan.  Results are cached by
 * plan hash (in memory, and in the JSON file named by DDF_TUNE_CACHE if set).  Synchronises
 * `stream`; allocates its scratch and frees it.  It replaces the plan's schedule buffers, so
 * graphs captured earlier on the plan must be captured again (see ddf_graph_create_batch).
 * budget_ms bounds the total timing time (<= 0: no bound). */
ddf_status ddf_autotune(ddf_plan_t plan, ddf_op op, int32_t nrhs, ddf_stream_t stream,
                        double budget_ms);

/* Introspection. */
ddf_status ddf_plan_info(ddf_plan_t plan, ddf_plan_info_t *out);
ddf_status ddf_plan_export(ddf_plan_t plan, int32_t which, int32_t mat, ddf_plan_tables_t *out);
/* Algorithmic HBM bytes of one call (values, plan tables, perm, vectors read once and
 * written once), the CSR-equivalent bytes, and flops. */
ddf_status ddf_plan_traffic(ddf_plan_t plan, ddf_op op, int32_t nrhs, int64_t *bytes_alg,
                            int64_t *bytes_csr, int64_t *flops);

/* Host copies of the tables the kernels read (also built for host-only plans), for
 * inspection and testing.  which: 0 forward pass, 1 adjoint pass, 2 per-matrix batch
 * schedule.  Valid until the next ddf_autotune or ddf_plan_destroy.
 *   cods   [n_cods][16]  flags, m, nn, row0, row_step, op0, op_step, col0, sigma0, sigma1,
 *                        rows_off, ops_off, cnt_off, xt_off, xp_off, mat
 *   tasks  [n_tasks][4]  codelet, first row, end row, meta (log2 lanes per row |
 *                        streamed << 10 | row ranges << 11 | long row << 12 | row list << 13);
 *                        for SpMV the list used with one right-hand side; for the solve the
 *                        one-launch-per-level schedule, in level order
 *   sync   [n_tasks][4]  solve: the level order of that schedule as a counter protocol (the
 *                        counter of the level before, its task count, the task's own level
 *                        counter; checked by the CPU replay), then the level the launch
 *                        groups by (-1 for the value-gradient tasks of a batch adjoint)
 *   tasksN [n_tasksN][4] SpMV: the list used with several right-hand sides */
typedef struct {
    const int32_t *cods, *aux, *tasks, *sync, *tasksN;
    int64_t n_cods, aux_len, n_tasks, n_counters, n_tasksN;
    const int32_t *thin_rec; /* single-block solve: [n_thin_rec][21] per lane slot: row, value
                                index of the diagonal, ops, placeholder flag (levels start on
                                64-record boundaries), value indices[5], columns[5],
                                operand codes[5]: INT32_MIN empty; >= 0 solve-order index of
                                a row read from global memory; -(1 + thin_ring_size) the
                                row's right-hand-side term (value index -1, column the row);
                                -(1 + e) with e >= thin_ring_size + 2 a pinned LDS entry e
                                (a global operand past the lane's first two global slots);
                                else -(1 + ring slot); then 0, or 1 / 2 for the first /
                                second half of a row of 2G lanes; then, in a row's first
                                lane, the second LDS entry its solution is written to (its
                                ring slot, or its pinned entry), -1 in other lanes          */
    const int32_t *thin_lvl; /* [n][4] first record, lane slots in use, first solve-order
                                index, rows of 2G lanes, per level, then empty levels up to a
                                multiple of 4 plus 4 (absent: n = 0)                        */
    const int32_t *thin_rows; /* [n_rows] row of each solve-order index (absent: NULL)      */
    int64_t n_thin_rec, n_thin_lvl;
    int32_t thin_lg;          /* log2 lane slots per row                                       */
    int32_t thin_ring_size;   /* operand codes < 0: slot = -(code + 1) = solve-order index of
                                 the row mod thin_ring_size                                    */
    int32_t thin_reserved;
    int32_t thin_ngs;         /* op slots per lane (the lowest) that may read global memory   */
    int32_t thin_block;       /* threads of the solving block                                  */
    int32_t reserved;
    const int32_t *rowlist;   /* SpMV, one RHS: rows of the row-list tasks (tasks with bit 13:
                                 list entries [i0b, i0e), one lane per row, run from the CSR
                                 pattern)                                                      */
    int64_t n_rowlist;
    const int32_t *df_tasks;  /* solve, persistent dataflow kernel: [n_df_tasks][4] codelet, first
                                 row, end row (at most 8 rows of at most 16 ops), 0; in level
                                 order over all matrices (which = 2: matrix after matrix).
                                 Rows of more than 16 ops go in wide-row tasks, first in their
                                 level: codelet, first row, offset of the rows' columns in
                                 df_lcols, (1 << 14) | (rows << 16), 1 to 8 consecutive rows  */
    int64_t n_df_tasks;
    const int64_t *df_ptr;    /* [n_df_ptr] task ranges: 0, n_df_tasks (which = 2: per matrix) */
    int64_t n_df_ptr;
    const int32_t *df_lcols;  /* [n_df_lcols] columns of the wide-row tasks' ops: row after row,
                                 each in op order                                              */
    int64_t n_df_lcols;
    int32_t df_group;         /* 8: every level and every wide-row task starts a group of 8
                                 tasks (empty tasks fill the gaps); 1: no padding, and a
                                 level's rows of at most 16 ops go 8 to a mixed task (codelet
                                 of its first row, first slot, end slot, 1 << 15) whatever
                                 their codelets (batches)                                      */
    int32_t df_reserved;
    const int32_t *df_slots;  /* [n_df_slots][2] (codelet, row within it) of each mixed-task row */
    int64_t n_df_slots;
} ddf_device_tables_t;
ddf_status ddf_plan_device_tables(ddf_plan_t plan, int32_t which, ddf_device_tables_t *out);

/* Kernel timing for measurement.  With enable = 1, every later execution call on the plan
 * (up to 256 calls) records a pair of HIP events on its stream around its main kernel: the
 * solve kernel of a solve or transposed solve (one launch per level: from the first level's
 * launch to the last's), the product kernel of ddf_spmv or ddf_spmv_adjoint; enable = 0 stops
 * it.  Either call forgets the calls timed so far.  Events are created on the first enable
 * (the only allocation); execution calls still allocate nothing.
 * ddf_plan_kernel_time synchronises those events and returns the total time of the timed
 * kernels in ms, the number of timed calls and the number of kernel launches they made. */
ddf_status ddf_plan_time_kernels(ddf_plan_t plan, int32_t enable);
ddf_status ddf_plan_kernel_time(ddf_plan_t plan, double *ms, int64_t *calls, int64_t *launches);

/* Synchronises `stream`, then reads and clears the plan's device error flag. */
ddf_status ddf_plan_sync_status(ddf_plan_t plan, ddf_stream_t stream);
/* Test hook: spin limit of the dataflow solve's waits (0 = default): a wait that exceeds it
 * raises the plan's error flag (DDF_E_DEVICE from ddf_plan_sync_status) and stops. */
ddf_status ddf_plan_set_spin_limit(ddf_plan_t plan, int64_t limit);

const char *ddf_status_string(ddf_status s);
const char *ddf_last_error(void);
const char *ddf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DDF_H */
