// Internal data structures of libddf (host side).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ddf.h"

namespace ddf {

// canonical flag bits (the codelet record's `flags` field)
enum : int32_t { FS0 = 1, FS1 = 2, FS2 = 4, FSEP = 8, FRECT = 16, FRUNS = 32 };
// device-only bits
enum : int32_t { DOPS = 64, DCONTIG = 128, DXPTR = 256, DRPTR = 512 };

enum : int { NREG = 8, NCOD = 18 };
enum CodField : int {
    C_TYPE, C_FLAGS, C_PART, C_REGION, C_U, C_M, C_NN, C_P, C_ROW0, C_ROWSTEP, C_OP0,
    C_OPSTEP, C_COL0, C_SIG0, C_SIG1, C_AUXOFF, C_AUXLEN, C_COST
};

// Which access functions a kernel kind reads.  kind 0: SpMV (all entries are ops);
// kind 1: lower solve, diagonal last (not an op); kind 2: transposed solve on U = L^T,
// diagonal first (not an op), dependence levels counted from the last row.
struct Pattern {
    int kind = 0;
    int32_t n_rows = 0, n_cols = 0;
    const int32_t *rp = nullptr;
    const int32_t *ci = nullptr;
    int64_t opstart(int64_t q) const { return kind == 2 ? (int64_t)rp[q] + 1 : (int64_t)rp[q]; }
    int64_t nops(int64_t q) const {
        int64_t len = (int64_t)rp[q + 1] - rp[q];
        return kind == 0 ? len : len - 1;
    }
};

// The canonical tables of one inspected matrix.
struct Canon {
    int64_t header[9] = {0};
    std::vector<int64_t> part_ptr, part_rows, regions, codelets;
    std::vector<int32_t> aux;
    std::vector<int32_t> perm; // adjoint plan: transposed entry -> forward value index
    bool sliced = false;       // BLAS-only cover: codelets are column slices, rows shared
    int64_t n_parts() const { return header[5]; }
    int64_t n_codelets() const { return header[7]; }
};

// Single-block solve: int32 per lane-slot record, and per record of the gather index.
constexpr int THIN_REC = 21;
constexpr int THIN_GIDX = 6;

// Device codelet record: 16 x int32 = 64 bytes.
struct DCod {
    int32_t flags, m, nn, row0, row_step, op0, op_step, col0;
    int32_t sigma0, sigma1, rows_off, ops_off, cnt_off, xt_off, xp_off, mat;
};
static_assert(sizeof(DCod) == 64, "DCod layout");

// A wavefront's work item: rows [i0b, i0e) of one codelet; meta = log2(lanes per row) and
// the task-kind bits of the schedule that holds it.
struct Task {
    int32_t cod, i0b, i0e, meta;
};

// Per-matrix bases of a batch (single plans have one entry of zeros and k = nrhs).
struct MatInfo {
    int64_t row_base; // first packed row
    int64_t val_base; // first packed value
    int64_t vec_base; // first element of the (n_b, k_b) packed vector block
    int32_t k;        // right-hand sides of this matrix
    int32_t n;
};

struct SchedParams {
    int32_t ops_per_lane = 4;
    int32_t passes = 2;
    int32_t remap = 1;
    int32_t blocks = 0;   // solve: persistent grid in 256-thread blocks (0 = all resident)
    int32_t backoff = 4;  // dataflow solve: longest sleep between polls (units of 64 cycles)
    int32_t path = 0;     // solve: 0 auto, 1 multi-block, 2 single-block
    int32_t helpers = 4;  // single-block solve: L2 prefetch blocks on the solver's XCD
    int32_t ahead = 24;   // single-block solve: levels the prefetch runs ahead (>= 8)
};

// Device-resident tables of one plan pass (forward or adjoint).
struct DevTables {
    std::vector<DCod> cods;
    std::vector<int32_t> aux;          // canonical aux followed by device supplements
    std::vector<Task> tasks;           // solve; SpMV with one right-hand side
    std::vector<Task> tasksN;          // SpMV with several right-hand sides
    std::vector<int32_t> sync;         // solve: 4 int32 per task (wait counter, count, signal counter, level)
    std::vector<Task> df_tasks;        // dataflow solve: up to DF_RG rows of one codelet, in level order
    std::vector<int64_t> df_ptr;       // per-matrix ranges of df_tasks (per-matrix schedules only)
    std::vector<int32_t> df_lcols;     // columns of the dataflow solve's wide-row tasks
    int32_t *d_df_lcols = nullptr;
    std::vector<int32_t> df_slots;     // (codelet, row) of the dataflow solve's mixed-task row slots
    int32_t *d_df_slots = nullptr;
    // device-only form of a batch's mixed-task row slots: per slot four int32 (first value
    // index | (k - 1) << 27, first element of the row in x, offset in df_mcols | ops << 27, the
    // matrix's first value index) and the rows' operand elements (vector base + column * k)
    std::vector<int32_t> df_mdesc, df_mcols;
    int32_t *d_df_mdesc = nullptr, *d_df_mcols = nullptr;
    int64_t n_counters = 0;            // solve: level counters of the sync protocol (CPU replay)
    int64_t csr_rows = 0, csr_nnz = 0; // SpMV, one right-hand side: rows run from the CSR pattern
    int64_t table_bytes1 = 0;          // plan bytes a one-RHS SpMV launch reads
    std::vector<int32_t> cod_aux;      // aux words of each codelet
    std::vector<uint8_t> csr_cod;      // SpMV, one right-hand side: codelet run from the CSR pattern
                                       // (1: in row ranges, 2: in the row list)
    std::vector<int32_t> rowlist;      // SpMV, one right-hand side: rows of TASK_ROWS tasks
    int32_t *d_rowlist = nullptr;
    std::vector<int32_t> thin_rec;     // single-block solve records (empty if not eligible)
    std::vector<int32_t> thin_lvl;     // per level: first record, lanes, first solve index, wide rows
    std::vector<int32_t> thin_rows;    // row of each solve-order index
    int32_t thin_lg = 0;
    int32_t thin_ring = 0;             // LDS ring size in plan positions
    int32_t thin_nlev = 0;             // levels of the single-block solve (sub-levels included)
    int32_t thin_nlev_pad = 0;         // levels rounded up to a multiple of 4
    int32_t thin_ngs = 0;              // op slots per lane that may hold a global operand
    int32_t thin_pins = 0;             // pinned LDS entries in use
    int32_t thin_block = 64;           // threads of the solving block (widest level, rounded to 64)
    double *d_thin_xs = nullptr;       // solutions in solve order
    int32_t *d_thin_gidx = nullptr;    // per-call gather index (the records stay on the host)
    int32_t *d_thin_lvl = nullptr;
    int32_t *d_thin_rows = nullptr;
    double *d_thin_stream = nullptr;   // per-call stream, THIN_SW doubles per record
    DCod *d_cods = nullptr;
    int32_t *d_aux = nullptr;
    Task *d_tasks = nullptr;
    DCod *d_tcods = nullptr;           // solve: the codelet record of each task, in task order
    Task *d_df_tasks = nullptr;
    DCod *d_df_tcods = nullptr;        // the codelet record of each dataflow task
    Task *d_tasksN = nullptr;
    int32_t *d_sync = nullptr;
    // device bytes of the tables (solve schedules add the per-task codelet copy)
    int64_t bytes() const {
        return (int64_t)cods.size() * sizeof(DCod) + (int64_t)aux.size() * 4 +
               (int64_t)tasks.size() * (sizeof(Task) + (sync.empty() ? 0 : sizeof(DCod))) + (int64_t)sync.size() * 4 +
               (int64_t)df_tasks.size() * (sizeof(Task) + sizeof(DCod)) +
               (int64_t)(df_lcols.size() + df_slots.size()) * 4;
    }
    // plan bytes a one-launch-per-level solve reads: each task, its codelet copy and its sync
    // entry, and aux
    int64_t solve_read_bytes() const {
        return (int64_t)aux.size() * 4 + (int64_t)tasks.size() * (sizeof(Task) + sizeof(DCod)) +
               (int64_t)sync.size() * 4;
    }
    // plan bytes the dataflow solve reads: each task and its codelet copy, and aux
    int64_t df_read_bytes() const {
        return (int64_t)aux.size() * 4 + (int64_t)df_tasks.size() * (sizeof(Task) + sizeof(DCod)) +
               (int64_t)(df_lcols.size() + (df_mdesc.empty() ? df_slots.size() : df_mdesc.size() + df_mcols.size())) * 4;
    }
    // plan bytes a single-block solve reads per call: gather index, level table, rows
    int64_t thin_bytes() const {
        return ((int64_t)thin_rec.size() / THIN_REC * THIN_GIDX + (int64_t)thin_lvl.size() +
                (int64_t)thin_rows.size()) * 4;
    }
    // bytes a launch reads: records and aux (upper bound) plus its own task list
    int64_t launch_bytes(bool many_rhs) const {
        return (int64_t)cods.size() * sizeof(DCod) + (int64_t)aux.size() * 4 +
               (int64_t)(many_rhs ? tasksN.size() : tasks.size()) * sizeof(Task) + (int64_t)sync.size() * 4;
    }
};

std::string &last_error();
ddf_status fail(ddf_status s, const std::string &msg);

// inspector.cpp
ddf_status validate(int kind, const ddf_csr_host &A);
void inspect(const Pattern &P, int32_t t, int threads, Canon &out, bool only_blas = false);
void transpose(int32_t n_rows, int32_t n_cols, const int32_t *rp, const int32_t *ci,
               std::vector<int32_t> &rpT, std::vector<int32_t> &ciT, std::vector<int32_t> &perm, int threads = 0);
uint64_t hash_canon(const Canon &c, uint64_t h);

} // namespace ddf
