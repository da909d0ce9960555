// Kernel argument blocks and launchers (device code in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "ddf_internal.hpp"

namespace ddf {

struct SpmvArgs {
    const DCod *cods;
    const int32_t *aux;
    const Task *tasks;
    int32_t ntasks;
    int32_t k;     // right-hand sides (row stride of x, y)
    int32_t remap; // XCD-contiguous block order
    const double *vals;
    const int32_t *perm; // values through perm (transposed plan)
    const int32_t *rp, *ci; // CSR pattern of the pass (TASK_CSR and TASK_ROWS tasks)
    const int32_t *rows;    // row list of TASK_ROWS tasks
    const double *x;
    double *y;
};

// Single-block solve of a matrix whose every level fits one 1024-thread pass; G lanes per row,
// THIN_SLOTS op slots per lane.  Static record per lane slot and level, THIN_REC int32:
//   [0] row, [1] value index of the diagonal, [2] ops in the lane, [3] placeholder flag,
//   [4..8] value index of each op slot, [9..13] its column,
//   [14..18] its operand code: THIN_UNUSED for an empty slot; >= 0 the solve-order index of a
//   row solved at least THIN_HORIZON levels before, read from global memory (only in the first
//   `ngs` slots); otherwise -(1 + ring slot) of the LDS ring that keeps the solutions of the
//   last `ring` rows solved, ring slot = solve-order index mod ring; -(1 + ring) is the row's
//   right-hand-side term (value index THIN_VIDX_B, column the row): its operand, the entry one
//   past the ring, holds -1;
//   [19] 0 for a row of G lanes; a "wide" row takes 2G lanes (its first G flagged 1, the
//   others 2) and comes before the other rows of its level;
//   [20] in the row's first lane (its writer), the LDS entry that receives its solution besides
//   the ring slot: the ring slot itself, or a pinned entry past the ring's two constants that
//   keeps the solution to the end of the solve, for readers too far ahead for the ring whose
//   lanes already use THIN_PIN_SLOTS global slots (-1 in the other lanes).
// Every level's records start on a 64-record boundary; placeholder records (flag 1, no ops)
// fill the gap.  The solve order numbers rows level by level, wide rows first.  Per call, a
// stream is gathered in record order, structure-of-arrays per 64 records: four 16-byte fields
// (codes 0..3; v0 v1; v2 v3; v4 and code 4) of 64 records each, each value divided by the row's
// diagonal (the right-hand-side term's value is b / diagonal), so that a row's solution is
// minus the sum of its slots; then one chunk of empty records, read by lanes with no record at
// a level.  A stream code is the byte offset in LDS of the slot's operand: a ring slot, the
// entry past the ring (-1, right-hand-side terms) or the one after it (0, empty slots); in the
// first `ngs` slots a global operand is coded -(1 + its solve-order index) instead, and the
// other codes there also gather the zero kept past the solutions; a pinned operand's code is
// its pinned entry's offset.  The fourth word of the last field holds the writer lane's second
// LDS entry (its byte offset).  The codes and the empty
// chunk do not change between calls: they are written once, when the tables are uploaded, from
// the records, which are then released.  Per call only the values are gathered, driven by a
// compact index table of THIN_GIDX int32 per record, per 64-record chunk the value indices of
// slots 0-3 (an int4 per record), then slot 4's and the diagonal's (an int2 per record); a slot
// index is the value index, THIN_UNUSED for an empty slot, or -(2 + row) for the
// right-hand-side term.  The solve writes solutions in solve order, and a scatter puts them in
// row order.  One right-hand side.
constexpr int THIN_SLOTS = 5;
constexpr int THIN_SW = 8;                  // stream doubles per record
constexpr int THIN_PIN = 2048;              // pinned LDS entries
constexpr int THIN_PIN_SLOTS = 2;           // global slots a lane may use when pins are available
constexpr int32_t THIN_VIDX_B = -1;         // value index of the right-hand-side term
constexpr int THIN_THREADS = 1024;
constexpr int THIN_KT_MAX = 1;              // right-hand sides the single-block kernel takes
constexpr int THIN_RING_MAX = 16384;       // LDS ring of solutions, plan positions (128 KiB); then
                                           // -1, 0 and the pinned entries
constexpr double THIN_SIMD_FIXED = 3.5;   // per-level fixed cost over one wave's issue time
constexpr int THIN_HORIZON = 3;           // a global operand's row was solved this many levels before
constexpr int32_t THIN_UNUSED = (int32_t)0x80000000;
struct ThinArgs {
    const int32_t *rec;  // records (only while the codes are written at upload)
    const int32_t *gidx; // gather index table, THIN_GIDX int32 per record
    int32_t remap;       // XCD-contiguous record ranges in the gather
    const int4 *lvl; // per level: first record, lanes in use, first solve index, wide rows
                     // (padded with empty levels)
    const int32_t *rows; // row of each solve-order index
    int32_t nlev;     // levels
    int32_t nlev_pad; // levels rounded up to a multiple of 4 (the table holds 4 more)
    int32_t lg;       // log2 lanes per row
    int32_t k;        // right-hand sides (at most the kernel's KT)
    int32_t kt;       // the kernel's KT (stride of xs)
    int32_t ring;     // LDS ring size in plan positions (a power of two); two more entries hold -1, 0
    int32_t ngs;      // op slots per lane that may hold a global operand
    int32_t pins;     // the plan uses pinned LDS entries (writers store their solution twice)
    int32_t helpers;  // blocks that pull upcoming levels into the solver's L2
    int32_t ahead;    // levels the helpers may run ahead of the solver
    int32_t n;        // rows
    int32_t block;    // threads of the solving block
    int64_t n_rec;    // records (a multiple of 64; the stream holds one more chunk)
    const double *vals;
    const double *b;
    double *x;
    double *stream;     // THIN_SW doubles per record, gathered before the solve
    double *xs;         // solutions in solve order, kt per row, then one zero
    unsigned *progress; // levels the solver has finished (read by the helpers)
    unsigned *sink;     // helpers' discard word (never read)
};

constexpr int CTR_STRIDE = 32; // uint32 per counter line (128 bytes)
enum : int32_t { TASK_STREAM = 1 << 10,   // SpMV: one-RHS task streamed element by element
                 TASK_CSR = 1 << 11,      // SpMV, one RHS: rows [i0b, i0e) of the CSR pattern
                 TASK_LONG = 1 << 12,     // with TASK_CSR: one row longer than a stream task
                 TASK_ROWS = 1 << 13 };   // SpMV, one RHS: rows list[i0b, i0e) (<= 64), a lane each
constexpr int ROWS_MAX_LEN = 8;          // longest row a TASK_ROWS lane takes
constexpr int STREAM_ELEMS = 64 * 8;     // elements of a stream task (64 lanes x 8)

struct SolveArgs {
    const DCod *cods;  // the solve's plan
    const int32_t *aux;
    const Task *tasks;
    const DCod *tcods; // the codelet of each task, in task order (loaded beside the task), or null
    const int4 *sync; // per task: counter to wait on (-1 none), count to wait for, counter to signal
    int32_t ntasks;
    int32_t backoff_max;
    const MatInfo *mats;
    const double *vals;
    const int32_t *perm; // adjoint: U's entries -> L's values (per matrix, local); the per-level
                         // kernel of a single-matrix call reads vals in U's order instead
    const double *b;     // right-hand side (adjoint: upstream gradient)
    double *x;           // solution (adjoint: lambda)
    unsigned *ctr;       // dataflow solve: lines of CTR_STRIDE: ticket, error flag, check-in count, mode
    unsigned *err;       // the error flag the dataflow solve raises (null: ctr's second line)
    int64_t spin_limit;
    int32_t k_override; // > 0: right-hand sides of a single-matrix call
    int32_t npass;      // dataflow solve: wave passes (each 64 / KR rows, DF_RG rows per task)
    const int32_t *lcols; // dataflow solve: columns of the wide-row tasks (offset in the task's i0e)
    const int2 *slots;    // dataflow solve: (codelet, row) of the mixed tasks' row slots
    const int4 *mdesc;    // dataflow solve: the same slots' descriptors (NULL: read the codelets)
    const int32_t *mcols; // dataflow solve: the mixed rows' operand elements
};
constexpr int WAVE_LANES = 64;
constexpr int DF_RG = 8;  // dataflow solve: rows per task (one codelet's)
constexpr int DF_PASS_MAX = 8; // dataflow solve: most tasks one wave pass takes (one right-hand side)
constexpr int DF_U = 16;  // dataflow solve: ops per lane loaded before a wait
// Dataflow solve: rows of more than DF_U ops (more than one chunk of a lane) run as wide-row
// tasks (meta DF_LONG | rows << 16): up to 8 consecutive rows of one codelet, from row i0b,
// their columns one after the other at lcols[i0e...].  Such a task has a wave pass to itself:
// its rows split the 64 lanes, and each row's lanes split its ops as well as its right-hand
// sides.  In a list for several right-hand-side counts a task of this kind sits at a multiple
// of DF_PASS_MAX, followed by empty tasks up to the next multiple.
constexpr int32_t DF_LONG = 1 << 14;
constexpr int DF_LONG_ROWS_SHIFT = 16;
// Dataflow solve of a batch (8 lanes per row, one task per pass): a mixed task (meta DF_MIXED)
// holds up to DF_RG rows of any codelets of one level, row slots[s] for s in [i0b, i0e).
constexpr int32_t DF_MIXED = 1 << 15;

struct PlainArgs {
    const int32_t *rp;
    const int32_t *ci;
    const double *vals;
    const int32_t *perm;
    const int32_t *rows;
    const double *x; // input vector (solve: right-hand side)
    double *y;       // output vector (solve: solution; atomic adjoint: gx)
    const double *g; // adjoint upstream (or lambda for GV)
    double *gv;
    int64_t n, lo, hi;
    int32_t k, lg, upper;
};

enum PlainKind { PLAIN_SPMV, PLAIN_LEVEL, PLAIN_SPMV_ADJ, PLAIN_GV };

// Value gradient over a CSR pattern: gv[e] = sign * sum_r g[row, r] x[col, r] for every stored
// entry e = (row, col), rows of k values (row-major, stride k).
struct GvArgs {
    const int32_t *rp;
    const int32_t *ci;
    const double *g;
    const double *x;
    double *gv;
    double sign;
    int64_t n; // rows
    int32_t k;
    int32_t lg; // log2 lanes per row
    const int2 *chunks; // (row, first entry) of the chunks of rows longer than GV_LONG_ROW
    int64_t n_chunks;
};
// Value gradient of the SpMV adjoint through the forward plan's several-right-hand-side tasks.
struct GvPlanArgs {
    const DCod *cods;
    const int32_t *aux;
    const Task *tasks;
    int32_t ntasks;
    int32_t k;
    int32_t remap;
    const double *g;
    const double *x;
    double *gv;
    double sign;
};
// Value gradient of a batch adjoint, one launch per class of right-hand-side counts (k up to
// KT, a power of two): the class's rows are its matrices' rows, matrix after matrix; row q of
// the class is row q - mstart[j] of matrix mids[j] (mstart ascending, one more entry at the
// end).  Rows longer than GV_LONG_ROW run as chunks {matrix, row, first entry, 0}.
struct GvBatchArgs {
    const int32_t *rp;   // packed row pointers (batch-wide entry indices)
    const int32_t *ci;   // packed columns (local to each matrix)
    const double *g;     // lambda, packed vectors (n_b, k_b) per matrix
    const double *x;     // forward solution, packed the same way
    double *gv;          // value gradient, packed values
    const MatInfo *mats;
    const int32_t *mids;
    const int32_t *mstart;
    int32_t nm;          // matrices of the class
    int64_t n;           // rows of the class
    int32_t lg;          // log2 lanes per row
    const int4 *chunks;
    int64_t n_chunks;
    int32_t aligned;     // g and x 16-byte aligned
};
constexpr int GV_LONG_ROW = 256;  // rows longer than this run in chunks of GV_CHUNK entries
constexpr int GV_CHUNK = 512;

// Column-slice (BLAS-only) plans: SpMV adds each slice's partial sums into y (zeroed by the
// init kernel); the solve adds them into per-row accumulators and tallies, and the contributor
// completing a row's tally writes its solution (init: zeroes both, solves rows without ops).
struct SliceArgs {
    const DCod *cods;
    const Task *tasks; // rows [i0b, i0e) of a codelet, meta = log2 lanes per row
    int32_t ntasks;
    int32_t k;            // right-hand sides (row stride of x, y, b, xs)
    const double *vals;
    const double *x;      // operand vector (solve: the solution being built, = xs)
    double *y;            // SpMV: the output; solve: per-row accumulators
    const double *b;      // solve: right-hand side
    double *xs;           // solve: solution
    unsigned *cnt;        // solve: slices added per row
    const int32_t *need;  // solve: slices per row (null for SpMV)
    const int32_t *rp;    // solve: row pointers of L (diagonal last)
    int64_t n;            // rows
};
hipError_t launch_slices_init(const SliceArgs &a, hipStream_t s);
hipError_t launch_slices(const SliceArgs &a, hipStream_t s);

int kt_for(int k);
hipError_t init_device_info();
hipError_t launch_spmv(const SpmvArgs &a, bool vperm, hipStream_t s);
int kr_for(int k);
int df_lanes(int k); // lanes per row of the dataflow solve for k right-hand sides
hipError_t launch_df_reset(unsigned *ctr, hipStream_t s);
hipError_t launch_solve_df(const SolveArgs &a, bool adj, bool vperm, int kr, int blocks, double *fill, int64_t nfill,
                           hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_solve_range(const SolveArgs &a, bool adj, int kt, hipStream_t s);
int num_cu();
int resident_solve_blocks(); // 256-thread blocks of the dataflow solve the device keeps resident
// The static scratch of the no-allocation entry point on the current device: its address
// (taken once per device) and its size in doubles; the first NOALLOC_CTR_WORDS / 2 doubles
// hold the dataflow solve's counter lines, the rest the gathered values.
constexpr int64_t NOALLOC_VALUES = int64_t(1) << 22; // values the scratch holds (32 MiB)
constexpr int64_t NOALLOC_CTR_WORDS = 4 * CTR_STRIDE; // uint32 words of the counter lines
hipError_t noalloc_scratch(double **ptr);
hipError_t launch_reset(unsigned *ctr, int64_t n, hipStream_t s);
// ev0 / ev1 (nullable): events recorded on the stream around the solve kernel itself
hipError_t launch_solve_thin(const ThinArgs &a, int ngs, hipStream_t s, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);
hipError_t launch_thin_codes(const ThinArgs &a, hipStream_t s);
hipError_t launch_fill(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_gather(double *dst, const double *src, const int32_t *idx, int64_t n, hipStream_t s);
hipError_t launch_plain(PlainKind which, PlainArgs a, double avg_row, int kt, hipStream_t s);
hipError_t launch_gv(GvArgs a, double avg_short_row, hipStream_t s);
// k in {2, 4, 8, 16, 32} and g, x 16-byte aligned
bool gv_plan_fits(int32_t k, const double *g, const double *x);
hipError_t launch_gv_plan(const GvPlanArgs &a, hipStream_t s);
hipError_t launch_gv_batch_class(GvBatchArgs a, int kt, double avg_short_row, hipStream_t s);

} // namespace ddf
