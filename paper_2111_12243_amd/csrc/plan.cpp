// libddf host side: plan object, device packing, schedule, and the C ABI of include/ddf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <thread>
#include <sstream>
#include <string>

#include "ddf_internal.hpp"
#include "kernels.hpp"

using namespace ddf;

namespace ddf {
std::string &last_error() {
    static thread_local std::string s;
    return s;
}
ddf_status fail(ddf_status s, const std::string &msg) {
    last_error() = msg;
    return s;
}
} // namespace ddf

struct ddf_plan_s {
    int kind = 0;
    int nmat = 1;
    bool batch = false;
    ddf_opts opts{};
    bool host_only = false, has_adj = false;
    std::vector<Canon> fwd, adj;
    std::vector<MatInfo> mats;
    std::vector<int32_t> hrp, hci; // single-matrix host pattern (plain comparators)
    std::vector<int32_t> hrpT;     // row pointers of the transposed pattern (single matrix)
    int64_t n_rows = 0, n_cols = 0, nnz = 0, vec_total = 0;
    SchedParams sp_f, sp_a;
    DevTables F, T, Fpm;
    int64_t n_solve_tasks_adj = 0;    // adjoint: tasks of the one-launch-per-level transposed solve
    int64_t ctr_words_f = 0;          // counter words of the forward solves
    int64_t ctr_words_a = 0;          // and of the adjoint's (after them, in the same allocation)
    int64_t n_gx_tasks = 0;           // SpMV adjoint: tasks before the GV pass (one RHS)
    int64_t n_gx_tasksN = 0;          // same, several right-hand sides
    std::vector<int32_t> gv_chunks;   // value gradient: (row, first entry) per chunk of a long row
    int32_t *d_gv_chunks = nullptr;
    double gv_avg_short = 1.0;        // mean length of the other rows
    // batch adjoint's value gradient, per class of right-hand-side counts (k up to 1, 2, 4, ..., 32):
    // its matrices (offset in gvb_mids), its rows, its long-row chunks (offset in gvb_chunks, int4
    // each) and the mean length of its other rows
    struct GvClass {
        int32_t kt, nm;
        int64_t mid_off, nrows, chunk_off, nchunks;
        double avg;
    };
    std::vector<GvClass> gvb;
    int32_t *d_gvb_mids = nullptr;   // per class: matrix ids, then row starts (nm + 1)
    int32_t *d_gvb_chunks = nullptr;
    double *d_vals = nullptr;
    double *d_valsT = nullptr; // single-matrix SpTRSV adjoint: values in transposed order, per call
    int32_t *d_perm = nullptr, *d_rp = nullptr, *d_ci = nullptr, *d_rpT = nullptr, *d_ciT = nullptr;
    int32_t *d_rows = nullptr, *d_rrows = nullptr;
    MatInfo *d_mats = nullptr;
    unsigned *d_ctr = nullptr;        // forward solves' counters, progress words and error flag
    unsigned *d_ctr_adj = nullptr;    // the adjoint's own (a forward and an adjoint may overlap)
    int64_t spin_limit = int64_t(1) << 26;
    double inspect_seconds = 0;
    double phase_seconds[5] = {0, 0, 0, 0, 0}; // ddf_inspect's phases (ddf_plan_info_t)
    uint64_t hash = 0;
    int max_levels = 0;
    std::vector<void *> allocs;
    uint64_t generation = 0; // bumped whenever the schedule's device buffers are replaced
    // BLAS-only (column-slice) plans: slice tasks level by level (solve: task range of each
    // level in sl_lvl), slices per row, and per-call accumulators and tallies
    bool sliced = false;
    std::vector<int64_t> sl_lvl;
    int32_t *d_need = nullptr;
    double *d_acc = nullptr;
    int64_t acc_words = 0;
    unsigned *d_tally = nullptr;
    // kernel timing (ddf_plan_time_kernels): event pairs around the main kernel of each call
    std::vector<hipEvent_t> tev;
    int32_t tev_used = 0;
    int64_t tev_launches = 0;
    bool timing = false;
};

namespace {
constexpr int TIMED_CALLS = 256;
// The next event pair for a timed call (null when timing is off or the pairs are used up).
std::pair<hipEvent_t, hipEvent_t> next_timer(ddf_plan_t p, int64_t launches) {
    if (!p->timing || p->tev_used >= TIMED_CALLS) return {nullptr, nullptr};
    const int i = p->tev_used++;
    p->tev_launches += launches;
    return {p->tev[2 * i], p->tev[2 * i + 1]};
}
} // namespace

struct ddf_graph_s {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ddf_plan_t plan = nullptr;
    uint64_t generation = 0; // the plan's schedule generation the graph captured
};

namespace {

#define HIPCHK(x)                                                                                  \
    do {                                                                                           \
        hipError_t _e = (x);                                                                       \
        if (_e != hipSuccess)                                                                      \
            return fail(DDF_E_HIP, std::string(#x) + ": " + hipGetErrorString(_e));                \
    } while (0)

int g_alloc_count = 0;

ddf_status dalloc(ddf_plan_t p, void **ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 8;
    if (const char *s = getenv("DDF_TEST_FAIL_ALLOC")) {
        int n = atoi(s);
        if (n > 0 && ++g_alloc_count == n) return fail(DDF_E_NOMEM, "device allocation failed (test hook)");
    }
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? DDF_E_NOMEM : DDF_E_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    p->allocs.push_back(*ptr);
    return DDF_OK;
}

template <class T>
ddf_status upload(ddf_plan_t p, T **dst, const T *src, size_t n) {
    ddf_status s = dalloc(p, (void **)dst, n * sizeof(T));
    if (s) return s;
    if (n) HIPCHK(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return DDF_OK;
}

int xmode_host(int fl) {
    if (fl & FS2) return 0;
    if (fl & FSEP) return (fl & FRUNS) ? 2 : 1;
    return (fl & FRUNS) ? 4 : 3;
}

// Full column tables stored as runs stay runs on the device only when runs are long on
// average; shorter ones are decoded faster from a plain column list.
constexpr double RUNS_MIN_AVG = 3.0;

// Device tables of one matrix's codelets: per codelet, exactly the tables its kernel path
// reads (the canonical tables' information, re-encoded for the GPU):
//   ROWS (!S0), OPSTART (!S1, or when S1 holds only because rows have no operations and a
//   solve still needs each row's diagonal position), COUNTS (!RECT), and the column table:
//   shared offsets (SEP; runs expanded), full runs with a per-row run index, or full
//   columns with a per-row offset when rows are neither rectangular nor contiguous.
void pack(const Canon &c, const Pattern &P, int mat, DevTables &D) {
    const int64_t ncod = c.header[7];
    const size_t first = D.cods.size();
    D.cods.resize(first + ncod);
    std::vector<int64_t> rows, opst, nops;
    D.cod_aux.resize(first + ncod);
    for (int64_t i = 0; i < ncod; i++) {
        const int64_t *r = &c.codelets[i * NCOD];
        const int32_t fl = (int32_t)r[C_FLAGS];
        const int32_t m = (int32_t)r[C_M];
        const size_t aux0 = D.aux.size();
        DCod d;
        d.m = m;
        d.nn = (int32_t)r[C_NN];
        d.row0 = (int32_t)r[C_ROW0];
        d.row_step = (int32_t)r[C_ROWSTEP];
        d.op0 = (int32_t)r[C_OP0];
        d.op_step = (int32_t)r[C_OPSTEP];
        d.col0 = (int32_t)r[C_COL0];
        d.sigma0 = (int32_t)r[C_SIG0];
        d.sigma1 = (int32_t)r[C_SIG1];
        d.rows_off = d.ops_off = d.cnt_off = d.xt_off = d.xp_off = -1;
        d.mat = mat;
        int32_t dfl = fl & ~FRUNS;
        // rows of the codelet: canonical ROWS table or the strided formula
        rows.resize(m);
        opst.resize(m);
        nops.resize(m);
        int64_t ap = r[C_AUXOFF];
        for (int32_t a = 0; a < m; a++)
            rows[a] = (fl & FS0) ? (int64_t)d.row0 + (int64_t)a * d.row_step : c.aux[ap + a];
        for (int32_t a = 0; a < m; a++) {
            // a column slice covers ops [op0 - opstart, + nn) of each row; a whole-row
            // codelet all of them
            opst[a] = c.sliced ? (int64_t)d.op0 + (int64_t)a * d.op_step : P.opstart(rows[a]);
            nops[a] = c.sliced ? (int64_t)d.nn : P.nops(rows[a]);
        }
        if (!(fl & FS0)) {
            d.rows_off = (int32_t)D.aux.size();
            for (int32_t a = 0; a < m; a++) D.aux.push_back((int32_t)rows[a]);
        }
        bool need_ops = !(fl & FS1);
        if (!need_ops && P.kind >= 1 && m >= 2)
            for (int32_t a = 0; a < m; a++)
                if (opst[a] != (int64_t)d.op0 + (int64_t)a * d.op_step) need_ops = true;
        if (need_ops) {
            d.ops_off = (int32_t)D.aux.size();
            dfl |= DOPS;
            for (int32_t a = 0; a < m; a++) D.aux.push_back((int32_t)opst[a]);
        }
        if (!(fl & FRECT)) {
            d.cnt_off = (int32_t)D.aux.size();
            for (int32_t a = 0; a < m; a++) D.aux.push_back((int32_t)nops[a]);
        }
        if (!(fl & FS2)) {
            if (fl & FSEP) {
                d.xt_off = (int32_t)D.aux.size();
                for (int64_t b = 0; b < nops[0]; b++) D.aux.push_back(P.ci[opst[0] + b] - d.col0);
            } else {
                int64_t Ptot = 0, R = 0;
                for (int32_t a = 0; a < m; a++) {
                    Ptot += nops[a];
                    for (int64_t b = 0; b < nops[a]; b++)
                        if (b == 0 || P.ci[opst[a] + b] != P.ci[opst[a] + b - 1] + 1) R++;
                }
                const bool keep_runs = (fl & FRUNS) && (double)Ptot >= RUNS_MIN_AVG * (double)R;
                if (keep_runs) {
                    dfl |= FRUNS | DRPTR;
                    d.xt_off = (int32_t)D.aux.size();
                    std::vector<int32_t> rptr(m);
                    int64_t j = 0;
                    for (int32_t a = 0; a < m; a++) {
                        rptr[a] = (int32_t)j;
                        int64_t b = 0;
                        while (b < nops[a]) {
                            int64_t e = b + 1;
                            while (e < nops[a] && P.ci[opst[a] + e] == P.ci[opst[a] + e - 1] + 1) e++;
                            D.aux.push_back(P.ci[opst[a] + b]);
                            D.aux.push_back((int32_t)(e - b));
                            j++;
                            b = e;
                        }
                    }
                    // per row its first run, then one past the last row's runs
                    rptr.push_back((int32_t)j);
                    d.xp_off = (int32_t)D.aux.size();
                    D.aux.insert(D.aux.end(), rptr.begin(), rptr.end());
                } else {
                    d.xt_off = (int32_t)D.aux.size();
                    for (int32_t a = 0; a < m; a++)
                        for (int64_t b = 0; b < nops[a]; b++) D.aux.push_back(P.ci[opst[a] + b]);
                    if (!(fl & FRECT)) {
                        bool contig = true;
                        for (int32_t a = 0; a + 1 < m; a++)
                            if (opst[a + 1] != opst[a] + nops[a]) contig = false;
                        if (contig) {
                            dfl |= DCONTIG;
                        } else {
                            dfl |= DXPTR;
                            d.xp_off = (int32_t)D.aux.size();
                            int64_t s = 0;
                            for (int32_t a = 0; a < m; a++) {
                                D.aux.push_back((int32_t)s);
                                s += nops[a];
                            }
                        }
                    }
                }
            }
        }
        d.flags = dfl;
        D.cods[first + i] = d;
        D.cod_aux[first + i] = (int32_t)(D.aux.size() - aux0);
    }
}

int lg_of(int64_t n, int opl) {
    int lg = 0;
    while (lg < 6 && (int64_t(1) << lg) * opl < n) lg++;
    return lg;
}

// Tasks of one codelet: rows grouped so that a task's lanes-per-row fits its rows.
void codelet_tasks(const DCod &d, const std::vector<int32_t> &aux, int32_t cod_index, const SchedParams &sp,
                   std::vector<Task> &out) {
    const int32_t m = d.m;
    auto nops_of = [&](int32_t a) -> int64_t { return (d.flags & FRECT) ? d.nn : aux[d.cnt_off + a]; };
    int32_t a = 0;
    while (a < m) {
        int lg = lg_of(nops_of(a), sp.ops_per_lane);
        int32_t b = a + 1;
        while (b < m) {
            int lgb = lg_of(nops_of(b), sp.ops_per_lane);
            int lgn = std::max(lg, lgb);
            if (lgb + 2 < lg || lgb > lg + 1) break;
            if ((b - a + 1) > (64 >> lgn) * sp.passes) break;
            lg = lgn;
            b++;
        }
        out.push_back({cod_index, a, b, lg});
        a = b;
    }
}

// SpMV tasks of one codelet for one right-hand side: rectangular codelets whose values
// (and full column table) are contiguous are streamed element by element, STREAM_ELEMS per
// task; others get lanes-per-row tasks.
// A rectangular codelet whose rows fit one stream task runs element-streamed.
bool stream_cod(const DCod &d) {
    const int mode = xmode_host(d.flags);
    return (d.flags & FRECT) && d.nn >= 1 && d.nn <= STREAM_ELEMS && (mode == 0 || mode == 1 || mode == 3) &&
           !(d.flags & DOPS) && (d.m == 1 || d.op_step == d.nn);
}

void spmv1_tasks(const DCod &d, const std::vector<int32_t> &aux, int32_t cod_index, const SchedParams &sp,
                 std::vector<Task> &out) {
    const bool stream = stream_cod(d);
    if (!stream) {
        codelet_tasks(d, aux, cod_index, sp, out);
        return;
    }
    // the kernel sums one row per lane: at most 64 rows, and at most STREAM_ELEMS elements
    const int32_t rows = std::min<int32_t>(STREAM_ELEMS / d.nn, 64);
    for (int32_t a = 0; a < d.m; a += rows) out.push_back({cod_index, a, std::min(d.m, a + rows), TASK_STREAM});
}

// Ops of a device codelet.
int64_t cod_ops(const DCod &d, const std::vector<int32_t> &aux) {
    if (d.flags & FRECT) return (int64_t)d.m * d.nn;
    int64_t s = 0;
    for (int32_t a = 0; a < d.m; a++) s += aux[d.cnt_off + a];
    return s;
}

// Rows of a device codelet.
void cod_rows(const DCod &d, const std::vector<int32_t> &aux, std::vector<int32_t> &out) {
    for (int32_t a = 0; a < d.m; a++) out.push_back((d.flags & FS0) ? d.row0 + a * d.row_step : aux[d.rows_off + a]);
}

// Codelets with fewer ops than this run as packed row ranges of the CSR pattern (one wave per
// up to STREAM_ELEMS elements or 64 rows; a longer row gets a wave of its own).
constexpr int64_t TINY_OPS = 128;

// Splits a plan pass between codelet tasks and rows run from the CSR pattern: a codelet with
// fewer than TINY_OPS ops runs as row ranges when all its rows lie in runs of at least CSR_RUN
// consecutive such rows, else in the row list (one lane per row, 64 rows to a wave) when none
// of its rows is longer than ROWS_MAX_LEN; a codelet that does not stream and whose rows all
// hold more than LONG_ROW entries runs as row ranges too (a wave per row beyond STREAM_ELEMS,
// in chunks with every lane's loads in flight); the others keep their own tasks.
constexpr int64_t CSR_RUN = 16;
constexpr int64_t LONG_ROW = 256;

void split_tiny(const DevTables &D, int64_t n_rows, const std::vector<int32_t> &rp, std::vector<uint8_t> &csr_cod,
                std::vector<int32_t> &rows, std::vector<int32_t> &listrows) {
    std::vector<uint8_t> tiny_row(n_rows, 0);
    std::vector<int32_t> tmp;
    csr_cod.assign(D.cods.size(), 0);
    for (size_t c = 0; c < D.cods.size(); c++)
        if (cod_ops(D.cods[c], D.aux) < TINY_OPS) {
            tmp.clear();
            cod_rows(D.cods[c], D.aux, tmp);
            for (int32_t r : tmp) tiny_row[r] = 1;
        }
    // length of the run of tiny rows through each row
    std::vector<int32_t> run(n_rows, 0);
    for (int64_t r = 0; r < n_rows;) {
        if (!tiny_row[r]) {
            r++;
            continue;
        }
        int64_t e = r;
        while (e < n_rows && tiny_row[e]) e++;
        for (int64_t q = r; q < e; q++) run[q] = (int32_t)std::min<int64_t>(e - r, INT32_MAX);
        r = e;
    }
    rows.clear();
    listrows.clear();
    for (size_t c = 0; c < D.cods.size(); c++) {
        if (!stream_cod(D.cods[c])) {
            tmp.clear();
            cod_rows(D.cods[c], D.aux, tmp);
            bool longrows = !tmp.empty();
            for (int32_t r : tmp) longrows = longrows && rp[r + 1] - rp[r] > LONG_ROW;
            if (longrows) {
                csr_cod[c] = 1;
                rows.insert(rows.end(), tmp.begin(), tmp.end());
                continue;
            }
        }
        if (cod_ops(D.cods[c], D.aux) >= TINY_OPS) continue;
        tmp.clear();
        cod_rows(D.cods[c], D.aux, tmp);
        bool ok = true, fits = true;
        for (int32_t r : tmp) {
            ok = ok && run[r] >= CSR_RUN;
            fits = fits && rp[r + 1] - rp[r] <= ROWS_MAX_LEN;
        }
        if (ok) {
            csr_cod[c] = 1;
            rows.insert(rows.end(), tmp.begin(), tmp.end());
        } else if (fits) {
            csr_cod[c] = 2;
            listrows.insert(listrows.end(), tmp.begin(), tmp.end());
        }
    }
}

// Row-list tasks: rows sorted by length (lanes of a wave then loop about equally long), 64 to
// a task.  The sorted list is kept for the device.
void rows_tasks(std::vector<int32_t> &listrows, const std::vector<int32_t> &rp, std::vector<Task> &out) {
    std::sort(listrows.begin(), listrows.end(), [&](int32_t a, int32_t b) {
        const int32_t la = rp[a + 1] - rp[a], lb = rp[b + 1] - rp[b];
        return la != lb ? la < lb : a < b;
    });
    for (size_t i = 0; i < listrows.size(); i += 64)
        out.push_back({-1, (int32_t)i, (int32_t)std::min(listrows.size(), i + 64), TASK_ROWS});
}

void csr_tasks(std::vector<int32_t> &rows, const std::vector<int32_t> &rp, std::vector<Task> &out) {
    std::sort(rows.begin(), rows.end());
    size_t i = 0;
    while (i < rows.size()) {
        const int32_t r0 = rows[i];
        const int64_t len0 = rp[r0 + 1] - rp[r0];
        if (len0 > STREAM_ELEMS) {
            out.push_back({-1, r0, r0 + 1, TASK_CSR | TASK_LONG});
            i++;
            continue;
        }
        size_t j = i + 1;
        while (j < rows.size() && rows[j] == rows[j - 1] + 1 && j - i < 64 &&
               (int64_t)rp[rows[j] + 1] - rp[r0] <= STREAM_ELEMS)
            j++;
        out.push_back({-1, r0, rows[j - 1] + 1, TASK_CSR});
        i = j;
    }
}

// Plan bytes a one-RHS SpMV launch reads: records and aux of the codelets it runs as codelets,
// its task list, and the CSR columns and row pointers of the rows it runs from the pattern.
int64_t spmv1_table_bytes(const DevTables &D) {
    int64_t b = (int64_t)D.tasks.size() * sizeof(Task) + 4 * D.csr_nnz + 8 * D.csr_rows + 4 * (int64_t)D.rowlist.size();
    for (size_t c = 0; c < D.cods.size(); c++)
        if (!D.csr_cod[c]) b += (int64_t)sizeof(DCod) + 4 * (int64_t)D.cod_aux[c];
    return b;
}

// SpMV tasks for several right-hand sides: fixed row blocks (right-hand sides across lanes).
void spmvN_tasks(const DCod &d, int32_t cod_index, const SchedParams &sp, std::vector<Task> &out) {
    const int32_t rows = 16 * std::max(1, sp.passes);
    for (int32_t a = 0; a < d.m; a += rows) out.push_back({cod_index, a, std::min(d.m, a + rows), 0});
}

// Persistent-solve schedule of several matrices.  Tasks are ordered by (level, matrix);
// every level of every matrix gets a completion counter (ids from counter_base on).  A task
// of level l > 0 waits until counter (b, l-1) reaches that level's task count and signals
// counter (b, l).  Returns per matrix the (counter id, task count) of its last level.
std::vector<std::pair<int64_t, int64_t>> build_solve(const DevTables &D, const std::vector<int64_t> &cod_begin,
                                                     const std::vector<std::vector<int32_t>> &levels,
                                                     const SchedParams &sp, std::vector<Task> &tasks,
                                                     std::vector<int32_t> &sync, int64_t &counter_base) {
    const int nm = (int)cod_begin.size() - 1;
    std::vector<std::vector<std::vector<Task>>> per(nm);
    std::vector<int64_t> base(nm);
    int32_t maxl = 0;
    for (int b = 0; b < nm; b++) {
        int32_t nl = 0;
        for (int32_t l : levels[b]) nl = std::max(nl, l + 1);
        per[b].resize(nl);
        maxl = std::max(maxl, nl);
        for (int64_t c = cod_begin[b]; c < cod_begin[b + 1]; c++)
            codelet_tasks(D.cods[c], D.aux, (int32_t)c, sp, per[b][levels[b][c - cod_begin[b]]]);
        base[b] = counter_base;
        counter_base += nl;
    }
    for (int32_t l = 0; l < maxl; l++)
        for (int b = 0; b < nm; b++) {
            if (l >= (int32_t)per[b].size()) continue;
            for (const Task &t : per[b][l]) {
                tasks.push_back(t);
                const int32_t sy[4] = {l > 0 ? (int32_t)(base[b] + l - 1) : -1,
                                       l > 0 ? (int32_t)per[b][l - 1].size() : 0, (int32_t)(base[b] + l), l};
                sync.insert(sync.end(), sy, sy + 4);
            }
        }
    std::vector<std::pair<int64_t, int64_t>> last(nm, {-1, 0});
    for (int b = 0; b < nm; b++)
        if (!per[b].empty()) last[b] = {base[b] + (int64_t)per[b].size() - 1, (int64_t)per[b].back().size()};
    return last;
}

// A device codelet's row i0 (row, first value index, ops) and its ops' columns, decoded on the
// host the way the kernels read the records.
struct HostRow {
    int64_t row, opst, nops;
};

HostRow host_row(const DCod &d, const std::vector<int32_t> &aux, int32_t i0) {
    HostRow r;
    r.row = (d.flags & FS0) ? (int64_t)d.row0 + (int64_t)i0 * d.row_step : aux[d.rows_off + i0];
    r.opst = (d.flags & DOPS) ? aux[d.ops_off + i0] : (int64_t)d.op0 + (int64_t)i0 * d.op_step;
    r.nops = (d.flags & FRECT) ? d.nn : aux[d.cnt_off + i0];
    return r;
}

void host_cols(const DCod &d, const std::vector<int32_t> &aux, int32_t i0, const HostRow &r,
               std::vector<int32_t> &out) {
    const int mode = xmode_host(d.flags);
    const int64_t base = (int64_t)d.col0 + (int64_t)i0 * d.sigma0;
    if (mode == 0) {
        for (int64_t b = 0; b < r.nops; b++) out.push_back((int32_t)(base + b * d.sigma1));
    } else if (mode == 1) {
        for (int64_t b = 0; b < r.nops; b++) out.push_back((int32_t)(base + aux[d.xt_off + b]));
    } else if (mode == 3) {
        const int64_t off = (d.flags & FRECT) ? (int64_t)i0 * d.nn
                            : (d.flags & DCONTIG) ? r.opst - d.op0
                                                  : aux[d.xp_off + i0];
        for (int64_t b = 0; b < r.nops; b++) out.push_back(aux[d.xt_off + off + b]);
    } else {
        // runs: (start, length) pairs; shared (mode 2) from the table's head, full (mode 4)
        // from the row's first run
        int64_t j = mode == 2 ? 0 : aux[d.xp_off + i0];
        const int64_t b0 = mode == 2 ? base : 0;
        int64_t got = 0;
        while (got < r.nops) {
            const int64_t st = aux[d.xt_off + 2 * j], ln = aux[d.xt_off + 2 * j + 1];
            for (int64_t q = 0; q < ln && got < r.nops; q++, got++) out.push_back((int32_t)(b0 + st + q));
            j++;
        }
    }
}

// Rows a wide-row task of the dataflow solve may hold: the most R of 8, 4, 2 whose lanes per
// row (64 / R) still split, after the right-hand-side lanes, into enough groups for the longest
// row's ops to take one chunk of DF_U per group; else 1.
int wide_rows_for(int64_t nops, int32_t k) {
    int kr = 1;
    while (kr < k && kr < WAVE_LANES) kr <<= 1;
    for (int R = DF_RG; R > 1; R >>= 1) {
        const int lanes = WAVE_LANES / R, kl = std::min(kr, lanes);
        if ((int64_t)(lanes / kl) * DF_U >= nops) return R;
    }
    return 1;
}

// Dataflow-solve tasks: level by level over all matrices (a topological order of every
// matrix's dependences).  Rows of at most DF_U ops go in groups of up to DF_RG consecutive rows
// of one codelet; longer rows go in wide-row tasks of consecutive long rows (as many as
// wide_rows_for allows for the task's longest row and the matrix's right-hand-side count, 8
// where that count is a per-call argument), first in their level, with their columns appended
// to lcols.  A wave pass takes 1, 2, 4 or 8 consecutive tasks, starting at a multiple of that
// count, and its rows must not depend on each other; with group = DF_PASS_MAX (lists for any
// right-hand-side count) every level is padded with empty tasks to a multiple of 8 and every
// wide-row task starts a group of 8 that it fills with empty tasks.  With group = 1 (batches,
// whose passes take one task of up to 8 rows) nothing is padded, and the short rows of a level
// go 8 to a mixed task whatever their codelets (small codelets would otherwise leave most of a
// pass idle), each row slot a (codelet, row) pair in slots.  by_matrix: matrix after matrix
// instead (per-matrix launches), with each matrix's range in ptr.
void build_df(const DevTables &D, const std::vector<int64_t> &cod_begin, const std::vector<std::vector<int32_t>> &levels,
              bool by_matrix, int group, const std::vector<MatInfo> *mats, std::vector<Task> &out,
              std::vector<int64_t> &ptr, std::vector<int32_t> &lcols, std::vector<int32_t> &slots) {
    const int nm = (int)cod_begin.size() - 1;
    out.clear();
    lcols.clear();
    slots.clear();
    ptr.assign(1, 0);
    std::vector<Task> shortt, widet;
    std::vector<int64_t> nops;
    auto split = [&](int64_t c) {
        const DCod &d = D.cods[c];
        const int32_t k = mats ? (*mats)[d.mat].k : 8;
        nops.resize(d.m);
        for (int32_t a = 0; a < d.m; a++) nops[a] = host_row(d, D.aux, a).nops;
        int32_t a = 0;
        while (a < d.m) {
            int32_t e = a;
            if (nops[a] <= DF_U) {
                while (e < d.m && nops[e] <= DF_U && e - a < DF_RG) e++;
                shortt.push_back({(int32_t)c, a, e, 0});
            } else {
                int R = wide_rows_for(nops[a], k);
                e = a + 1;
                while (e < d.m && nops[e] > DF_U && e - a < std::min(R, wide_rows_for(nops[e], k))) {
                    R = std::min(R, wide_rows_for(nops[e], k));
                    e++;
                }
                widet.push_back({(int32_t)c, a, e, DF_LONG});
            }
            a = e;
        }
    };
    auto pad = [&]() {
        while (out.size() % group) out.push_back({out.back().cod, 0, 0, 0});
    };
    // wide-row tasks first (they take longest), then the others
    auto flush = [&]() {
        for (const Task &t : widet) {
            const DCod &d = D.cods[t.cod];
            out.push_back({t.cod, t.i0b, (int32_t)lcols.size(), DF_LONG | ((t.i0e - t.i0b) << DF_LONG_ROWS_SHIFT)});
            for (int32_t a = t.i0b; a < t.i0e; a++) host_cols(d, D.aux, a, host_row(d, D.aux, a), lcols);
            pad();
        }
        if (group == 1) {
            int32_t n = 0, first = 0;
            for (const Task &t : shortt)
                for (int32_t a = t.i0b; a < t.i0e; a++) {
                    if (n == 0) first = t.cod;
                    slots.push_back(t.cod);
                    slots.push_back(a);
                    if (++n == DF_RG) {
                        const int32_t e = (int32_t)(slots.size() / 2);
                        out.push_back({first, e - n, e, DF_MIXED});
                        n = 0;
                    }
                }
            if (n) {
                const int32_t e = (int32_t)(slots.size() / 2);
                out.push_back({first, e - n, e, DF_MIXED});
            }
        } else {
            out.insert(out.end(), shortt.begin(), shortt.end());
        }
        if (!out.empty()) pad();
        shortt.clear();
        widet.clear();
    };
    // codelets of a matrix come in level order: per matrix, the first codelet of each level
    std::vector<std::vector<int64_t>> lvl_begin(nm);
    int32_t maxl = 0;
    for (int b = 0; b < nm; b++) {
        int32_t nl = 0;
        for (int32_t l : levels[b]) nl = std::max(nl, l + 1);
        maxl = std::max(maxl, nl);
        lvl_begin[b].assign(nl + 1, cod_begin[b + 1]);
        for (int64_t c = cod_begin[b + 1] - 1; c >= cod_begin[b]; c--) lvl_begin[b][levels[b][c - cod_begin[b]]] = c;
        for (int32_t l = nl - 1; l >= 0; l--) lvl_begin[b][l] = std::min(lvl_begin[b][l], lvl_begin[b][l + 1]);
    }
    if (by_matrix) {
        for (int b = 0; b < nm; b++) {
            for (int32_t l = 0; l + 1 < (int32_t)lvl_begin[b].size(); l++) {
                for (int64_t c = lvl_begin[b][l]; c < lvl_begin[b][l + 1]; c++) split(c);
                flush();
            }
            ptr.push_back((int64_t)out.size());
        }
        return;
    }
    for (int32_t l = 0; l < maxl; l++) {
        for (int b = 0; b < nm; b++)
            if (l + 1 < (int32_t)lvl_begin[b].size())
                for (int64_t c = lvl_begin[b][l]; c < lvl_begin[b][l + 1]; c++) split(c);
        flush();
    }
    ptr.push_back((int64_t)out.size());
}

void drop_alloc(ddf_plan_t p, void *ptr) {
    if (!ptr) return;
    auto it = std::find(p->allocs.begin(), p->allocs.end(), ptr);
    if (it != p->allocs.end()) p->allocs.erase(it);
    (void)hipFree(ptr);
}

// The device-only descriptors of a batch's mixed-task row slots (DevTables::df_mdesc), so that
// a mixed pass reads each row's value range, output position and operand list from one record
// instead of its codelet record, the matrix's bases and the codelet's column tables.  Left
// empty (the kernel then reads the codelets) when a field does not fit its bits.
void mixed_desc(const std::vector<DCod> &cods, const std::vector<int32_t> &aux, const std::vector<int32_t> &slots,
                const std::vector<MatInfo> &mats, std::vector<int32_t> &desc, std::vector<int32_t> &mcols) {
    desc.clear();
    mcols.clear();
    constexpr int64_t M27 = int64_t(1) << 27;
    std::vector<int32_t> cols;
    for (size_t q = 0; q + 1 < slots.size(); q += 2) {
        const DCod &d = cods[slots[q]];
        const int32_t i0 = slots[q + 1];
        const HostRow r = host_row(d, aux, i0);
        const MatInfo &mi = mats[d.mat];
        const int64_t e = mi.val_base + r.opst, coff = (int64_t)mcols.size();
        const int64_t rowel = mi.vec_base + r.row * mi.k;
        if (e >= M27 || coff + r.nops >= M27 || r.nops > DF_U || mi.k < 1 || mi.k > 32 || rowel >= (int64_t(1) << 31) ||
            mi.val_base >= (int64_t(1) << 31)) {
            desc.clear();
            mcols.clear();
            return;
        }
        cols.clear();
        host_cols(d, aux, i0, r, cols);
        for (int32_t c : cols) {
            const int64_t el = mi.vec_base + (int64_t)c * mi.k;
            if (el >= (int64_t(1) << 31)) {
                desc.clear();
                mcols.clear();
                return;
            }
            mcols.push_back((int32_t)el);
        }
        desc.push_back((int32_t)(e | ((int64_t)(mi.k - 1) << 27)));
        desc.push_back((int32_t)rowel);
        desc.push_back((int32_t)(coff | (r.nops << 27)));
        desc.push_back((int32_t)mi.val_base);
    }
}

ddf_status upload_tasks(ddf_plan_t p, DevTables &D) {
    if (p->host_only) return DDF_OK;
    p->generation++; // graphs captured before now read the buffers freed below
    // schedule buffers are replaced when the schedule changes (autotune)
    drop_alloc(p, D.d_tasks);
    drop_alloc(p, D.d_tasksN);
    drop_alloc(p, D.d_sync);
    drop_alloc(p, D.d_rowlist);
    drop_alloc(p, D.d_tcods);
    drop_alloc(p, D.d_df_tasks);
    drop_alloc(p, D.d_df_tcods);
    drop_alloc(p, D.d_df_lcols);
    drop_alloc(p, D.d_df_slots);
    drop_alloc(p, D.d_df_mdesc);
    drop_alloc(p, D.d_df_mcols);
    D.d_df_mdesc = nullptr;
    D.d_df_mcols = nullptr;
    D.d_df_tasks = nullptr;
    D.d_df_tcods = nullptr;
    D.d_df_lcols = nullptr;
    D.d_df_slots = nullptr;
    D.d_tasks = nullptr;
    D.d_tasksN = nullptr;
    D.d_sync = nullptr;
    D.d_rowlist = nullptr;
    D.d_tcods = nullptr;
    ddf_status s = upload(p, &D.d_tasks, D.tasks.data(), D.tasks.size());
    if (!s && !D.sync.empty() && !D.tasks.empty()) {
        // solve schedules: each task's codelet record in task order, so that a wave loads its
        // task and its codelet side by side
        const std::vector<DCod> &cods = &D == &p->T ? p->T.cods : p->F.cods;
        std::vector<DCod> tc(D.tasks.size());
        for (size_t i = 0; i < D.tasks.size(); i++) tc[i] = cods[D.tasks[i].cod];
        s = upload(p, &D.d_tcods, tc.data(), tc.size());
    }
    if (!s && !D.df_tasks.empty()) {
        const std::vector<DCod> &cods = &D == &p->T ? p->T.cods : p->F.cods;
        std::vector<DCod> tc(D.df_tasks.size());
        for (size_t i = 0; i < D.df_tasks.size(); i++) tc[i] = cods[D.df_tasks[i].cod];
        s = upload(p, &D.d_df_tasks, D.df_tasks.data(), D.df_tasks.size());
        if (!s) s = upload(p, &D.d_df_tcods, tc.data(), tc.size());
        if (!s && !D.df_lcols.empty()) s = upload(p, &D.d_df_lcols, D.df_lcols.data(), D.df_lcols.size());
        if (!s && !D.df_slots.empty()) s = upload(p, &D.d_df_slots, D.df_slots.data(), D.df_slots.size());
        D.df_mdesc.clear();
        D.df_mcols.clear();
        if (p->batch && !D.df_slots.empty())
            mixed_desc(cods, &D == &p->T ? p->T.aux : p->F.aux, D.df_slots, p->mats, D.df_mdesc, D.df_mcols);
        if (!s && !D.df_mdesc.empty()) s = upload(p, &D.d_df_mdesc, D.df_mdesc.data(), D.df_mdesc.size());
        if (!s && !D.df_mcols.empty()) s = upload(p, &D.d_df_mcols, D.df_mcols.data(), D.df_mcols.size());
    }
    if (!s && !D.rowlist.empty()) s = upload(p, &D.d_rowlist, D.rowlist.data(), D.rowlist.size());
    if (!s && !D.tasksN.empty()) s = upload(p, &D.d_tasksN, D.tasksN.data(), D.tasksN.size());
    if (!s && !D.sync.empty()) s = upload(p, &D.d_sync, D.sync.data(), D.sync.size());
    return s;
}

// Records of the single-block solve, built from a matrix's codelets level by level (rows in
// plan order).  Every row takes its ops plus one right-hand-side term; eligible when that fits 64 * THIN_SLOTS slots per row and (without a lane cap)
// every level fits one 1024-lane pass; value indices go through perm for the transposed solve.
void build_thin(const Canon &c, const Pattern &P, const std::vector<int32_t> *perm, int32_t ring, int32_t lane_cap,
                DevTables &D) {
    D.thin_rec.clear();
    D.thin_lvl.clear();
    D.thin_rows.clear();
    D.thin_block = 64;
    const int64_t n = P.n_rows;
    // rows of G lanes, and "wide" rows of 2G lanes
    std::vector<int64_t> hist;
    int64_t maxn = 0;
    for (int64_t r = 0; r < n; r++) {
        const int64_t no = P.nops(r) + 1; // ops and the right-hand-side term
        maxn = std::max(maxn, no);
        if ((int64_t)hist.size() <= no) hist.resize(no + 1, 0);
        hist[no]++;
    }
    // G: the fewest lanes over all rows, a row taking G lanes when its slots fit, else 2G
    // (counted as 3G: the extra combining step makes wide rows worth it only where they are few)
    int lg = -1;
    int64_t best = 0;
    for (int t = 0; t <= 5; t++) {
        const int64_t cap1 = int64_t(THIN_SLOTS) << t;
        if (2 * cap1 < maxn) continue;
        int64_t lanes = 0;
        for (int64_t no = 0; no < (int64_t)hist.size(); no++) lanes += hist[no] * (no <= cap1 ? 1 : 3) << t;
        if (lg < 0 || lanes < best) {
            best = lanes;
            lg = t;
        }
    }
    if (lg < 0) return;
    const int G = 1 << lg;
    // lanes per row: 2G ("wide") when its ops do not fit G lanes, or when its operands from
    // global memory would need more than one slot per lane
    std::vector<uint8_t> wide(n, 0);
    for (int64_t r = 0; r < n; r++) wide[r] = P.nops(r) + 1 > (int64_t)G * THIN_SLOTS;
    auto lanes_of = [&](int64_t row) -> int { return wide[row] ? 2 * G : G; };
    const int64_t ncl = c.header[5];
    // codelets of each level, in plan order
    std::vector<std::vector<int64_t>> by_level(ncl);
    for (int64_t i = 0; i < c.header[7]; i++) by_level[c.codelets[i * NCOD + C_PART]].push_back(i);
    std::vector<int32_t> lev(n, -1);
    // the solve's levels: each level's rows in plan order, wide rows first (so they start on
    // 2G-lane boundaries), cut into consecutive sub-levels of at most `lane_cap` lanes (rows of
    // one level are independent, so any cut keeps the dependences)
    std::vector<std::vector<int64_t>> rows_of;
    std::vector<int32_t> nwide;
    // solve order of a row: its index in plan order (levels in turn, wide rows first in each);
    // lvl_end: one past a level's last solve-order index; R: widest level in G-lane groups
    std::vector<int64_t> plan_pos(n, -1), lvl_end;
    int64_t R = 1, nl = 0;
    // lane cap: given, or the one that minimises a cost model of the solve: every level costs a
    // fixed latency plus the instruction issue of the waves that share a SIMD (four SIMDs per
    // compute unit; idle waves issue as much as busy ones); THIN_SIMD_FIXED is the fixed part
    // in units of one wave's issue
    int64_t cap = lane_cap;
    if (cap <= 0) {
        std::vector<int64_t> lanes(ncl, 0);
        int64_t maxl = 0;
        for (int64_t l0 = 0; l0 < ncl; l0++) {
            for (int64_t ci : by_level[l0]) {
                const int64_t *r = &c.codelets[ci * NCOD];
                const int32_t fl = (int32_t)r[C_FLAGS];
                for (int64_t a = 0; a < r[C_M]; a++)
                    lanes[l0] += lanes_of((fl & FS0) ? r[C_ROW0] + a * r[C_ROWSTEP] : c.aux[r[C_AUXOFF] + a]);
            }
            maxl = std::max(maxl, lanes[l0]);
        }
        if (maxl > THIN_THREADS) return;
        double best = 0;
        for (int64_t cc = 64; cc <= THIN_THREADS; cc += 64) {
            int64_t subs = 0;
            for (int64_t v : lanes) subs += (v + cc - 1) / cc;
            const int64_t waves = (std::min(cc, maxl) + 63) / 64;
            const double cost = (double)subs * (THIN_SIMD_FIXED + (double)((waves + 3) / 4));
            if (cap <= 0 || cost < best) {
                best = cost;
                cap = cc;
            }
        }
    }
    auto layout = [&]() {
        R = 1;
        int64_t q = 0;
        rows_of.clear();
        nwide.clear();
        lvl_end.clear();
        for (int64_t l0 = 0; l0 < ncl; l0++) {
            std::vector<int64_t> wrows, narrow;
            for (int64_t ci : by_level[l0]) {
                const int64_t *r = &c.codelets[ci * NCOD];
                const int32_t fl = (int32_t)r[C_FLAGS];
                for (int64_t a = 0; a < r[C_M]; a++) {
                    const int64_t row = (fl & FS0) ? r[C_ROW0] + a * r[C_ROWSTEP] : c.aux[r[C_AUXOFF] + a];
                    (wide[row] ? wrows : narrow).push_back(row);
                }
            }
            wrows.insert(wrows.end(), narrow.begin(), narrow.end());
            size_t i = 0;
            while (i < wrows.size()) {
                std::vector<int64_t> sub;
                int64_t lanes = 0;
                int32_t nw = 0;
                while (i < wrows.size() && (sub.empty() || lanes + lanes_of(wrows[i]) <= cap)) {
                    lanes += lanes_of(wrows[i]);
                    nw += wide[wrows[i]];
                    sub.push_back(wrows[i++]);
                }
                const int64_t l = (int64_t)rows_of.size();
                int64_t groups = 0;
                for (int64_t row : sub) {
                    lev[row] = (int32_t)l;
                    plan_pos[row] = q++;
                    groups += lanes_of(row) / G;
                }
                lvl_end.push_back(q);
                nwide.push_back(nw);
                rows_of.push_back(std::move(sub));
                R = std::max(R, groups);
            }
        }
        nl = (int64_t)rows_of.size();
    };
    // an operand is read from the LDS ring unless a position written up to the reading level
    // has overwritten its slot
    auto is_global = [&](int64_t col, int64_t l) { return plan_pos[col] < lvl_end[l] - ring; };
    layout();
    const std::vector<uint8_t> wide_ops = wide;
    // rows whose operands from global memory would need more than `per_lane` slots per lane
    // (and whose slots fit 2G lanes) take 2G lanes
    auto mark = [&](int per_lane) {
        bool changed = false;
        for (int64_t l = 0; l < nl; l++)
            for (int64_t row : rows_of[l]) {
                if (wide_ops[row]) continue;
                const int64_t op = P.opstart(row), no = P.nops(row);
                int64_t ng = 0;
                for (int64_t i = 0; i < no; i++) ng += is_global(P.ci[op + i], l);
                const uint8_t w = ng > (int64_t)per_lane * G && 2 * G * THIN_SLOTS >= no + 1;
                if (w != wide[row]) {
                    wide[row] = w;
                    changed = true;
                }
            }
        if (changed) layout();
    };
    mark(1);
    if (R * G > THIN_THREADS) return;
    auto vidx = [&](int64_t e) -> int32_t { return perm ? (*perm)[e] : (int32_t)e; };
    // Records, level by level.  With pins, a global operand past the first THIN_PIN_SLOTS
    // slots of its lane is read from a pinned LDS entry instead (past the ring's two constants),
    // written by its row when that row is solved; a lane then needs at most THIN_PIN_SLOTS
    // global slots.  Returns false when the matrix needs more than THIN_PIN entries.
    int ngs = 0;
    std::vector<int32_t> slot_vi, slot_col, slot_code;
    std::vector<int64_t> head(n, -1);  // record of each row's writer lane
    std::vector<int32_t> pin_of(n, -1); // pinned LDS entry of a row
    std::vector<char> pinned_op;
    auto emit = [&](bool pins) -> bool {
        ngs = 0;
        D.thin_rec.clear();
        D.thin_lvl.clear();
        D.thin_block = 64;
        std::fill(head.begin(), head.end(), -1);
        std::fill(pin_of.begin(), pin_of.end(), -1);
        int32_t npin = 0;
        for (int64_t l = 0; l < nl; l++) {
            const int64_t first = (int64_t)D.thin_rec.size() / THIN_REC;
            for (int64_t row : rows_of[l]) {
                const int64_t op = P.opstart(row), no = P.nops(row);
                const int64_t dpos = P.kind == 2 ? op - 1 : op + no;
                // slot s = j * NL + g (op slot j of lane g of the row's NL lanes): operands from
                // global memory first, so that they sit in the lowest slot indices of every lane
                const int NL = lanes_of(row);
                const int S = NL * THIN_SLOTS;
                slot_vi.assign(S, vidx(dpos));
                slot_col.assign(S, (int32_t)row);
                slot_code.assign(S, THIN_UNUSED);
                // globals in op order: the ones past the lanes' pinned-slot bound go to LDS
                // entries of their own
                pinned_op.assign(no, 0);
                for (int64_t i = 0, ng = 0; i < no; i++)
                    if (is_global(P.ci[op + i], l)) pinned_op[i] = pins && ng++ >= THIN_PIN_SLOTS * NL;
                int next = 0;
                for (int pass = 0; pass < 2; pass++)
                    for (int64_t i = 0; i < no; i++) {
                        const int32_t col = P.ci[op + i];
                        const int64_t m = lev[col];
                        const bool pinned = pinned_op[i] != 0;
                        const bool global = is_global(col, l) && !pinned;
                        if (global && m > l - THIN_HORIZON) { // ring too small for this matrix
                            D.thin_rec.clear();
                            D.thin_lvl.clear();
                            return true;
                        }
                        if (global != (pass == 0)) continue;
                        slot_vi[next] = vidx(op + i);
                        slot_col[next] = col;
                        if (pinned) {
                            if (pin_of[col] < 0) {
                                if (npin == THIN_PIN) return false;
                                pin_of[col] = npin++;
                                D.thin_rec[(size_t)head[col] * THIN_REC + THIN_REC - 1] = ring + 2 + pin_of[col];
                            }
                            slot_code[next] = -(1 + ring + 2 + pin_of[col]);
                        } else {
                            slot_code[next] = global ? (int32_t)plan_pos[col]
                                                     : -(1 + (int32_t)(plan_pos[col] & (ring - 1)));
                        }
                        if (global) ngs = std::max(ngs, next / NL + 1);
                        next++;
                    }
                // the right-hand-side term: operand -1 read from the slot one past the ring, value
                // b[row] (scaled by 1 / diagonal with the ops when the stream is gathered)
                slot_vi[next] = THIN_VIDX_B;
                slot_col[next] = (int32_t)row;
                slot_code[next] = -(1 + ring);
                head[row] = (int64_t)D.thin_rec.size() / THIN_REC;
                for (int g = 0; g < NL; g++) {
                    int32_t rec[THIN_REC] = {(int32_t)row, vidx(dpos), 0, 0};
                    rec[THIN_REC - 2] = NL == G ? 0 : g < G ? 1 : 2;
                    // the writer lane's second LDS entry: its own ring slot until a pin is given
                    rec[THIN_REC - 1] = g == 0 ? (int32_t)(plan_pos[row] & (ring - 1)) : -1;
                    int cnt = 0;
                    for (int j = 0; j < THIN_SLOTS; j++) {
                        const int sl = j * NL + g;
                        rec[4 + j] = slot_vi[sl];
                        rec[4 + THIN_SLOTS + j] = slot_col[sl];
                        rec[4 + 2 * THIN_SLOTS + j] = slot_code[sl];
                        cnt += slot_code[sl] != THIN_UNUSED;
                    }
                    rec[2] = cnt;
                    D.thin_rec.insert(D.thin_rec.end(), rec, rec + THIN_REC);
                }
            }
            const int64_t lanes = (int64_t)D.thin_rec.size() / THIN_REC - first;
            // placeholders up to the next 64-record boundary: the level's first row, flag 1, no ops
            while (((int64_t)D.thin_rec.size() / THIN_REC) % 64) {
                int32_t rec[THIN_REC];
                std::copy(&D.thin_rec[first * THIN_REC], &D.thin_rec[first * THIN_REC] + THIN_REC, rec);
                rec[2] = 0;
                rec[3] = 1;
                rec[THIN_REC - 2] = 0;
                rec[THIN_REC - 1] = -1;
                for (int j = 0; j < THIN_SLOTS; j++) rec[4 + 2 * THIN_SLOTS + j] = THIN_UNUSED;
                D.thin_rec.insert(D.thin_rec.end(), rec, rec + THIN_REC);
            }
            D.thin_lvl.push_back((int32_t)first);
            D.thin_lvl.push_back((int32_t)lanes);
            D.thin_lvl.push_back((int32_t)(lvl_end[l] - (int64_t)rows_of[l].size()));
            D.thin_lvl.push_back(nwide[l]);
            D.thin_block = std::max<int32_t>(D.thin_block, (int32_t)((lanes + 63) / 64 * 64));
        }
        D.thin_pins = npin;
        return true;
    };
    if (!emit(true)) emit(false);
    if (!D.thin_rec.empty() && ngs == THIN_PIN_SLOTS) {
        // every lane gathers two slots anyway: rows with up to two global operands per lane
        // stay at G lanes (fewer lanes per level), unless that needs more global slots
        const int ngs1 = ngs;
        mark(THIN_PIN_SLOTS);
        bool ok = R * G <= THIN_THREADS;
        if (ok) {
            if (!emit(true)) emit(false);
            ok = !D.thin_rec.empty() && ngs <= ngs1;
        }
        if (!ok) {
            mark(1);
            if (R * G > THIN_THREADS) {
                D.thin_rec.clear();
                D.thin_lvl.clear();
                return;
            }
            if (!emit(true)) emit(false);
        }
    }
    if (D.thin_rec.empty()) return;
    // empty levels up to a multiple of four, and four more for the kernel's fetches ahead
    const int64_t pad = (nl + 3) / 4 * 4;
    for (int64_t l = nl; l < pad + 4; l++) {
        D.thin_lvl.push_back(0);
        D.thin_lvl.push_back(0);
        D.thin_lvl.push_back((int32_t)n);
        D.thin_lvl.push_back(0);
    }
    // row of each solve-order index
    D.thin_rows.assign(n, 0);
    for (int64_t r = 0; r < n; r++) D.thin_rows[plan_pos[r]] = (int32_t)r;
    D.thin_ngs = ngs == 4 ? THIN_SLOTS : ngs;
    D.thin_lg = lg;
    D.thin_ring = ring;
    D.thin_nlev = (int32_t)nl;
    D.thin_nlev_pad = (int32_t)pad;
}

// Counter lines of the persistent solve: ticket, error flag, one per level of the largest
// schedule.  Grown (never shrunk) when a schedule needs more.
ddf_status ensure_counters(ddf_plan_t p) {
    if (p->host_only || p->kind == DDF_SPMV) return DDF_OK;
    const int64_t nf = std::max<int64_t>(p->ctr_words_f, 4 * CTR_STRIDE);
    const int64_t na = std::max<int64_t>(p->ctr_words_a, 4 * CTR_STRIDE);
    if (p->d_ctr && nf <= p->ctr_words_f && na <= p->ctr_words_a) return DDF_OK;
    drop_alloc(p, p->d_ctr);
    p->d_ctr = p->d_ctr_adj = nullptr;
    if (ddf_status s = dalloc(p, (void **)&p->d_ctr, (nf + na) * sizeof(unsigned))) return s;
    if (hipError_t e = hipMemset(p->d_ctr, 0, (nf + na) * sizeof(unsigned)))
        return fail(DDF_E_HIP, std::string("hipMemset: ") + hipGetErrorString(e));
    p->d_ctr_adj = p->d_ctr + nf;
    p->ctr_words_f = nf;
    p->ctr_words_a = na;
    return DDF_OK;
}

std::vector<int32_t> codelet_levels(const Canon &c) {
    std::vector<int32_t> lv(c.header[7]);
    for (int64_t i = 0; i < c.header[7]; i++) lv[i] = (int32_t)c.codelets[i * NCOD + C_PART];
    return lv;
}

// Schedule of a column-slice plan (forward only): the slice tasks of every codelet, in codelet
// order, which is level order; for the solve, the task range of each level and the slices
// per row.
ddf_status build_slices(ddf_plan_t p) {
    DevTables &D = p->F;
    D.tasks.clear();
    p->sl_lvl.assign(1, 0);
    const Canon &c = p->fwd[0];
    std::vector<int32_t> need(p->n_rows, 0), rows;
    for (size_t i = 0; i < D.cods.size(); i++) {
        const int64_t lev = c.codelets[i * NCOD + C_PART];
        while ((int64_t)p->sl_lvl.size() <= lev) p->sl_lvl.push_back((int64_t)D.tasks.size());
        codelet_tasks(D.cods[i], D.aux, (int32_t)i, p->sp_f, D.tasks);
        rows.clear();
        cod_rows(D.cods[i], D.aux, rows);
        for (int32_t r : rows) need[r]++;
    }
    p->sl_lvl.push_back((int64_t)D.tasks.size());
    if (p->host_only) return DDF_OK;
    if (ddf_status s = upload_tasks(p, D)) return s;
    if (p->kind == DDF_SPTRSV_LOWER && !p->d_need) {
        if (ddf_status s = upload(p, &p->d_need, need.data(), need.size())) return s;
        if (ddf_status s = dalloc(p, (void **)&p->d_tally, (size_t)p->n_rows * sizeof(unsigned))) return s;
    }
    return DDF_OK;
}

// (Re)build every task list of the plan from its schedule parameters.
ddf_status build_schedule(ddf_plan_t p, bool fwd, bool adjp) {
    if (p->sliced) return fwd ? build_slices(p) : DDF_OK;
    if (p->kind == DDF_SPMV) {
        if (fwd) {
            p->F.tasks.clear();
            p->F.tasksN.clear();
            std::vector<int32_t> tiny, listrows;
            std::vector<uint8_t> csr_cod;
            split_tiny(p->F, p->n_rows, p->hrp, csr_cod, tiny, listrows);
            for (size_t c = 0; c < p->F.cods.size(); c++) {
                if (!csr_cod[c]) spmv1_tasks(p->F.cods[c], p->F.aux, (int32_t)c, p->sp_f, p->F.tasks);
                spmvN_tasks(p->F.cods[c], (int32_t)c, p->sp_f, p->F.tasksN);
            }
            p->F.csr_cod = csr_cod;
            p->F.csr_rows = (int64_t)(tiny.size() + listrows.size());
            p->F.csr_nnz = 0;
            for (int32_t r : tiny) p->F.csr_nnz += p->hrp[r + 1] - p->hrp[r];
            for (int32_t r : listrows) p->F.csr_nnz += p->hrp[r + 1] - p->hrp[r];
            csr_tasks(tiny, p->hrp, p->F.tasks);
            rows_tasks(listrows, p->hrp, p->F.tasks);
            p->F.rowlist = listrows;
            p->F.table_bytes1 = spmv1_table_bytes(p->F);
            if (ddf_status s = upload_tasks(p, p->F)) return s;
        }
        if (adjp && p->has_adj) {
            p->T.tasks.clear();
            p->T.tasksN.clear();
            std::vector<int32_t> tiny, listrows;
            std::vector<uint8_t> csr_cod;
            split_tiny(p->T, p->n_cols, p->hrpT, csr_cod, tiny, listrows);
            for (size_t c = 0; c < p->T.cods.size(); c++) {
                if (!csr_cod[c]) spmv1_tasks(p->T.cods[c], p->T.aux, (int32_t)c, p->sp_a, p->T.tasks);
                spmvN_tasks(p->T.cods[c], (int32_t)c, p->sp_a, p->T.tasksN);
            }
            p->T.csr_cod = csr_cod;
            p->T.csr_rows = (int64_t)(tiny.size() + listrows.size());
            p->T.csr_nnz = 0;
            for (int32_t r : tiny) p->T.csr_nnz += p->hrpT[r + 1] - p->hrpT[r];
            for (int32_t r : listrows) p->T.csr_nnz += p->hrpT[r + 1] - p->hrpT[r];
            csr_tasks(tiny, p->hrpT, p->T.tasks);
            rows_tasks(listrows, p->hrpT, p->T.tasks);
            p->T.rowlist = listrows;
            p->T.table_bytes1 = spmv1_table_bytes(p->T);
            // the value gradient runs over the CSR pattern, apart from these tasks
            p->n_gx_tasks = (int64_t)p->T.tasks.size();
            p->n_gx_tasksN = (int64_t)p->T.tasksN.size();
            if (ddf_status s = upload_tasks(p, p->T)) return s;
        }
        return DDF_OK;
    }
    std::vector<int64_t> cb(p->nmat + 1, 0);
    for (int b = 0; b < p->nmat; b++) cb[b + 1] = cb[b] + p->fwd[b].header[7];
    std::vector<std::vector<int32_t>> lv(p->nmat);
    for (int b = 0; b < p->nmat; b++) lv[b] = codelet_levels(p->fwd[b]);
    // a batch's dataflow passes take one task each (8 lanes per row), and its matrices' right-
    // hand-side counts are known; a single matrix's count is a per-call argument
    const int df_group = p->batch ? 1 : DF_PASS_MAX;
    const std::vector<MatInfo> *df_mats = p->batch ? &p->mats : nullptr;
    if (fwd) {
        p->F.tasks.clear();
        p->F.sync.clear();
        p->F.n_counters = 0;
        build_solve(p->F, cb, lv, p->sp_f, p->F.tasks, p->F.sync, p->F.n_counters);
        build_df(p->F, cb, lv, false, df_group, df_mats, p->F.df_tasks, p->F.df_ptr, p->F.df_lcols, p->F.df_slots);
        if (ddf_status s = upload_tasks(p, p->F)) return s;
        if (p->batch) {
            // per-matrix dataflow schedules for the one-launch-per-matrix comparator
            build_df(p->F, cb, lv, true, df_group, df_mats, p->Fpm.df_tasks, p->Fpm.df_ptr, p->Fpm.df_lcols,
                     p->Fpm.df_slots);
            if (ddf_status s = upload_tasks(p, p->Fpm)) return s;
        }
    }
    if (adjp && p->has_adj) {
        std::vector<int64_t> cba(p->nmat + 1, 0);
        std::vector<std::vector<int32_t>> lva(p->nmat);
        for (int b = 0; b < p->nmat; b++) {
            cba[b + 1] = cba[b] + p->adj[b].header[7];
            lva[b] = codelet_levels(p->adj[b]);
        }
        p->T.tasks.clear();
        p->T.sync.clear();
        p->T.n_counters = 0;
        build_solve(p->T, cba, lva, p->sp_a, p->T.tasks, p->T.sync, p->T.n_counters);
        build_df(p->T, cba, lva, false, df_group, df_mats, p->T.df_tasks, p->T.df_ptr, p->T.df_lcols,
                 p->T.df_slots);
        p->n_solve_tasks_adj = (int64_t)p->T.tasks.size();
        if (ddf_status s = upload_tasks(p, p->T)) return s;
    }
    return ensure_counters(p);
}

ddf_status upload_tables(ddf_plan_t p, DevTables &D) {
    if (ddf_status s = upload(p, &D.d_cods, D.cods.data(), D.cods.size())) return s;
    if (!D.thin_rec.empty()) {
        const int64_t n_rec = (int64_t)D.thin_rec.size() / THIN_REC; // a multiple of 64
        // gather index: per 64-record chunk, slots 0-3 (int4 per record), then slot 4 and the
        // diagonal (int2 per record); a slot holds its value index, THIN_UNUSED, or -(2 + row)
        // for the right-hand-side term
        std::vector<int32_t> gidx((size_t)n_rec * THIN_GIDX);
        for (int64_t q = 0; q < n_rec; q++) {
            const int32_t *r = &D.thin_rec[(size_t)q * THIN_REC];
            int32_t *g = &gidx[(size_t)(q / 64) * 64 * THIN_GIDX];
            const int l = (int)(q % 64);
            for (int j = 0; j < THIN_SLOTS; j++) {
                const int32_t code = r[4 + 2 * THIN_SLOTS + j], vi = r[4 + j];
                const int32_t e = code == THIN_UNUSED ? THIN_UNUSED : vi == THIN_VIDX_B ? -2 - r[0] : vi;
                if (j < 4) g[l * 4 + j] = e;
                else g[64 * 4 + l * 2] = e;
            }
            g[64 * 4 + l * 2 + 1] = r[1];
        }
        if (ddf_status s = upload(p, &D.d_thin_gidx, gidx.data(), gidx.size())) return s;
        if (ddf_status s = upload(p, &D.d_thin_lvl, D.thin_lvl.data(), D.thin_lvl.size())) return s;
        if (ddf_status s = upload(p, &D.d_thin_rows, D.thin_rows.data(), D.thin_rows.size())) return s;
        if (ddf_status s = dalloc(p, (void **)&D.d_thin_stream, (n_rec + 64) * THIN_SW * sizeof(double))) return s;
        // solutions in solve order, and one zero that gathers of slots without a global operand read
        if (ddf_status s = dalloc(p, (void **)&D.d_thin_xs, (D.thin_rows.size() + 1) * sizeof(double))) return s;
        // the stream's codes, written once from the records (on the null stream, then released)
        int32_t *d_rec = nullptr;
        if (ddf_status s = upload(p, &d_rec, D.thin_rec.data(), D.thin_rec.size())) return s;
        ThinArgs t{};
        t.rec = d_rec;
        t.n_rec = n_rec;
        t.ring = D.thin_ring;
        t.stream = D.d_thin_stream;
        hipError_t e = launch_thin_codes(t, nullptr);
        if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
        drop_alloc(p, d_rec);
        HIPCHK(e);
    }
    return upload(p, &D.d_aux, D.aux.data(), D.aux.size());
}

// the single-block kernel takes up to THIN_KT_MAX right-hand sides
bool use_thin(const DevTables &D, const SchedParams &sp, int32_t k) {
    return !D.thin_rec.empty() && (sp.path == 0 || sp.path == 2) && k <= THIN_KT_MAX;
}

ddf_status thin_launch(ddf_plan_t p, const DevTables &D, const SchedParams &sp, int nlev, const double *vals,
                       const double *b, double *x, int32_t k, hipStream_t s) {
    ThinArgs t{};
    t.gidx = D.d_thin_gidx;
    t.remap = &D == &p->T ? 1 : 0; // the transposed plan's value gathers reuse lines across nearby records
    t.lvl = reinterpret_cast<const int4 *>(D.d_thin_lvl);
    t.rows = D.d_thin_rows;
    t.nlev = nlev;
    t.nlev_pad = D.thin_nlev_pad;
    t.lg = D.thin_lg;
    t.k = k;
    t.kt = 1;
    t.ring = D.thin_ring;
    t.ngs = D.thin_ngs;
    t.pins = D.thin_pins > 0 ? 1 : 0;
    t.n = (int32_t)D.thin_rows.size();
    t.block = D.thin_block;
    t.xs = D.d_thin_xs;
    t.helpers = std::max(0, std::min(sp.helpers, 8));
    t.ahead = std::max(8, sp.ahead);
    t.n_rec = (int64_t)D.thin_rec.size() / THIN_REC;
    t.vals = vals;
    t.b = b;
    t.x = x;
    t.stream = D.d_thin_stream;
    unsigned *ctr = &D == &p->T ? p->d_ctr_adj : p->d_ctr;
    t.progress = ctr + CTR_STRIDE + 16; // second counter line: error flag, then these
    t.sink = ctr + CTR_STRIDE + 17;
    const auto tm = next_timer(p, 1);
    HIPCHK(launch_solve_thin(t, D.thin_ngs, s, tm.first, tm.second));
    return DDF_OK;
}

void free_plan(ddf_plan_t p) {
    if (!p) return;
    for (hipEvent_t e : p->tev) (void)hipEventDestroy(e);
    for (void *ptr : p->allocs) (void)hipFree(ptr);
    delete p;
}

void apply_opts(ddf_opts &o, const ddf_opts *in) {
    ddf_opts_default(&o);
    if (!in) return;
    o = *in;
    if (o.window <= 0) o.window = 64;
    if (o.ops_per_lane <= 0) o.ops_per_lane = 4;
    if (o.rows_passes <= 0) o.rows_passes = 2;
}

// Shared body of ddf_inspect / ddf_inspect_batch.
double seconds_since(std::chrono::steady_clock::time_point t) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t).count();
}

ddf_status make_plan(ddf_kind kind, int32_t nmat, const ddf_csr_host *mats, const int32_t *nrhs,
                     const ddf_opts *opts, bool batch, ddf_plan_t *out) {
    *out = nullptr;
    if (kind != DDF_SPMV && kind != DDF_SPTRSV_LOWER) return fail(DDF_E_KIND, "unknown kind");
    if (nmat < 1 || !mats) return fail(DDF_E_ARG, "no matrices");
    if (batch && kind != DDF_SPTRSV_LOWER) return fail(DDF_E_KIND, "batches are lower-triangular solves");
    ddf_opts o;
    apply_opts(o, opts);
    if (o.thin_ring != 0 && (o.thin_ring < 256 || o.thin_ring > THIN_RING_MAX || (o.thin_ring & (o.thin_ring - 1))))
        return fail(DDF_E_ARG, "thin_ring must be 0 or a power of two in 256..16384");
    if (o.thin_lanes != 0 && (o.thin_lanes < 64 || o.thin_lanes > THIN_THREADS || o.thin_lanes % 64))
        return fail(DDF_E_ARG, "thin_lanes must be 0 or a multiple of 64 in 64..1024");
    if (o.window < 1 || o.window > 1024) return fail(DDF_E_ARG, "window must be in 1..1024");
    if (o.only_blas && batch) return fail(DDF_E_UNSUPPORTED, "BLAS-only plans are single-matrix plans");
    for (int b = 0; b < nmat; b++) {
        if (ddf_status s = validate(kind, mats[b])) return s;
        if (batch && (!nrhs || nrhs[b] < 1 || nrhs[b] > 32)) return fail(DDF_E_ARG, "nrhs must be in 1..32");
    }
    auto t0 = std::chrono::steady_clock::now();
    ddf_plan_t p = new (std::nothrow) ddf_plan_s();
    if (!p) return fail(DDF_E_NOMEM, "host allocation failed");
    p->kind = kind;
    p->nmat = nmat;
    p->batch = batch;
    p->opts = o;
    p->host_only = o.host_only != 0;
    p->has_adj = o.build_adjoint != 0;
    p->sliced = o.only_blas != 0;
    p->sp_f.ops_per_lane = p->sp_a.ops_per_lane = o.ops_per_lane;
    p->sp_f.passes = p->sp_a.passes = o.rows_passes;
    p->sp_f.remap = p->sp_a.remap = o.xcd_remap < 0 ? 1 : o.xcd_remap;
    p->sp_f.blocks = p->sp_a.blocks = o.solve_blocks > 0 ? o.solve_blocks : 0;
    p->fwd.resize(nmat);
    if (p->has_adj) p->adj.resize(nmat);
    p->mats.resize(nmat);
    std::vector<std::vector<int32_t>> rpT(nmat), ciT(nmat), perm(nmat);
    for (int b = 0; b < nmat; b++) {
        const ddf_csr_host &A = mats[b];
        Pattern P{kind, A.n_rows, A.n_cols, A.row_ptr, A.col_idx};
        inspect(P, o.window, o.threads, p->fwd[b], o.only_blas != 0);
        if (p->has_adj) {
            const auto ta = std::chrono::steady_clock::now();
            transpose(A.n_rows, A.n_cols, A.row_ptr, A.col_idx, rpT[b], ciT[b], perm[b], o.threads);
            Pattern PT{kind == DDF_SPMV ? 0 : 2, A.n_cols, A.n_rows, rpT[b].data(), ciT[b].data()};
            inspect(PT, o.window, o.threads, p->adj[b], o.only_blas != 0);
            p->adj[b].perm = std::move(perm[b]);
            p->phase_seconds[1] += seconds_since(ta);
        }
        MatInfo &mi = p->mats[b];
        mi.row_base = p->n_rows;
        mi.val_base = p->nnz;
        mi.vec_base = p->vec_total;
        mi.k = batch ? nrhs[b] : 0;
        mi.n = A.n_rows;
        p->n_rows += A.n_rows;
        p->n_cols += A.n_cols;
        p->nnz += A.row_ptr[A.n_rows];
        p->vec_total += (int64_t)A.n_rows * (batch ? nrhs[b] : 1);
        p->max_levels = std::max<int>(p->max_levels, (int)p->fwd[b].header[5]);
    }
    p->inspect_seconds = seconds_since(t0);
    p->phase_seconds[0] = p->inspect_seconds - p->phase_seconds[1];
    uint64_t h = 1469598103934665603ull;
    for (auto &c : p->fwd) h = hash_canon(c, h);
    p->hash = h;
    if (!batch) {
        p->hrp.assign(mats[0].row_ptr, mats[0].row_ptr + mats[0].n_rows + 1);
        p->hci.assign(mats[0].col_idx, mats[0].col_idx + p->nnz);
        if (p->has_adj) p->hrpT = rpT[0];
    }
    // device tables (built on the host for every plan; uploaded unless host_only)
    if (!p->host_only) {
        if (hipError_t e = init_device_info()) {
            free_plan(p);
            return fail(DDF_E_HIP, std::string("device query: ") + hipGetErrorString(e));
        }
    }
    auto tph = std::chrono::steady_clock::now();
    for (int b = 0; b < nmat; b++) {
        Pattern P{kind, mats[b].n_rows, mats[b].n_cols, mats[b].row_ptr, mats[b].col_idx};
        pack(p->fwd[b], P, b, p->F);
        if (p->has_adj) {
            Pattern PT{kind == DDF_SPMV ? 0 : 2, mats[b].n_cols, mats[b].n_rows, rpT[b].data(), ciT[b].data()};
            pack(p->adj[b], PT, b, p->T);
        }
    }
    p->phase_seconds[2] = seconds_since(tph);
    tph = std::chrono::steady_clock::now();
    if (kind == DDF_SPTRSV_LOWER && !batch && !p->sliced) {
        const int32_t ring = o.thin_ring > 0 ? o.thin_ring : THIN_RING_MAX;
        Pattern P{kind, mats[0].n_rows, mats[0].n_cols, mats[0].row_ptr, mats[0].col_idx};
        // the transposed plan's records on a second host thread (the two are independent)
        std::thread adj_thin;
        if (p->has_adj) {
            Pattern PT{2, mats[0].n_cols, mats[0].n_rows, rpT[0].data(), ciT[0].data()};
            adj_thin = std::thread([&, PT]() { build_thin(p->adj[0], PT, &p->adj[0].perm, ring, o.thin_lanes, p->T); });
        }
        build_thin(p->fwd[0], P, nullptr, ring, o.thin_lanes, p->F);
        if (adj_thin.joinable()) adj_thin.join();
    }
    p->phase_seconds[3] = seconds_since(tph);
    p->sp_f.path = p->sp_a.path = o.solve_path;
    if (batch) {
        // batches: the dataflow kernel by default; the one-launch-per-level tasks (solve_path 3,
        // and the adjoint's value-gradient pass) take one op per lane and one row pass
        if (o.solve_path == 0) p->sp_f.path = p->sp_a.path = 1;
        p->sp_f.ops_per_lane = p->sp_a.ops_per_lane = 1;
        p->sp_f.passes = p->sp_a.passes = 1;
    }
    p->sp_f.helpers = p->sp_a.helpers = o.thin_helpers < 0 ? 4 : std::min(o.thin_helpers, 8);
    p->sp_f.ahead = p->sp_a.ahead = o.thin_ahead <= 0 ? 24 : std::max(o.thin_ahead, 8);
    if (p->host_only) {
        tph = std::chrono::steady_clock::now();
        ddf_status st = build_schedule(p, true, true);
        if (st) {
            free_plan(p);
            return st;
        }
        p->phase_seconds[4] = seconds_since(tph);
        *out = p;
        return DDF_OK;
    }
    ddf_status s = DDF_OK;
    tph = std::chrono::steady_clock::now();
    auto fin = [&](ddf_status st) {
        if (st) {
            free_plan(p);
            return st;
        }
        p->phase_seconds[4] = seconds_since(tph);
        *out = p;
        return DDF_OK;
    };
    if ((s = upload_tables(p, p->F))) return fin(s);
    if (p->has_adj && (s = upload_tables(p, p->T))) return fin(s);
    if ((s = build_schedule(p, true, true))) return fin(s);
    if ((s = upload(p, &p->d_mats, p->mats.data(), p->mats.size()))) return fin(s);
    // values captured at inspect time (packed over a batch)
    bool have_vals = true;
    for (int b = 0; b < nmat; b++)
        if (!mats[b].values && mats[b].row_ptr[mats[b].n_rows] > 0) have_vals = false;
    if (have_vals && p->nnz > 0) {
        if ((s = dalloc(p, (void **)&p->d_vals, p->nnz * sizeof(double)))) return fin(s);
        for (int b = 0; b < nmat; b++) {
            int64_t n = mats[b].row_ptr[mats[b].n_rows];
            if (n)
                if (hipError_t e = hipMemcpy(p->d_vals + p->mats[b].val_base, mats[b].values, n * 8, hipMemcpyHostToDevice))
                    return fin(fail(DDF_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e)));
        }
    }
    if (p->has_adj) {
        std::vector<int32_t> pall;
        for (int b = 0; b < nmat; b++) pall.insert(pall.end(), p->adj[b].perm.begin(), p->adj[b].perm.end());
        if ((s = upload(p, &p->d_perm, pall.data(), pall.size()))) return fin(s);
        // the per-level transposed solve of one matrix reads its values gathered in transposed
        // order (one pass per call) instead of through perm in every level
        if (!batch && kind == DDF_SPTRSV_LOWER && (s = dalloc(p, (void **)&p->d_valsT, (size_t)p->nnz * 8)))
            return fin(s);
    }
    if (batch && p->has_adj) {
        // the batch adjoint's value gradient: every matrix's CSR pattern, packed, with row
        // pointers that hold batch-wide entry indices; matrices grouped by right-hand-side
        // count class, one launch per class; rows longer than GV_LONG_ROW go in chunks
        if (p->nnz > INT32_MAX || p->n_rows > INT32_MAX)
            return fin(fail(DDF_E_ARG, "a batch with an adjoint holds at most 2^31 - 1 entries"));
        std::vector<int32_t> rp(p->n_rows + 1), ci((size_t)p->nnz), mids, chunks;
        for (int b = 0; b < nmat; b++) {
            const ddf_csr_host &A = mats[b];
            const MatInfo &mi = p->mats[b];
            for (int32_t r = 0; r < A.n_rows; r++) rp[mi.row_base + r] = (int32_t)(mi.val_base + A.row_ptr[r]);
            std::copy(A.col_idx, A.col_idx + A.row_ptr[A.n_rows], ci.begin() + mi.val_base);
        }
        rp[p->n_rows] = (int32_t)p->nnz;
        for (int kt = 1; kt <= 32; kt <<= 1) {
            ddf_plan_s::GvClass c{kt, 0, (int64_t)mids.size(), 0, (int64_t)chunks.size() / 4, 0, 1.0};
            std::vector<int32_t> starts;
            int64_t short_rows = 0, short_nnz = 0;
            for (int b = 0; b < nmat; b++) {
                const int32_t k = p->mats[b].k;
                if (k > kt || (kt > 1 && k <= kt / 2)) continue;
                const ddf_csr_host &A = mats[b];
                mids.push_back(b);
                starts.push_back((int32_t)c.nrows);
                c.nrows += A.n_rows;
                for (int32_t r = 0; r < A.n_rows; r++) {
                    const int32_t b0 = A.row_ptr[r], len = A.row_ptr[r + 1] - b0;
                    if (len > GV_LONG_ROW) {
                        for (int32_t e = b0; e < b0 + len; e += GV_CHUNK) {
                            const int32_t q[4] = {b, r, (int32_t)(p->mats[b].val_base + e), 0};
                            chunks.insert(chunks.end(), q, q + 4);
                        }
                    } else {
                        short_rows++;
                        short_nnz += len;
                    }
                }
            }
            c.nm = (int32_t)starts.size();
            if (c.nm == 0) {
                continue;
            }
            starts.push_back((int32_t)c.nrows);
            mids.insert(mids.end(), starts.begin(), starts.end());
            c.nchunks = (int64_t)chunks.size() / 4 - c.chunk_off;
            c.avg = short_rows ? std::max(1.0, (double)short_nnz / (double)short_rows) : 1.0;
            p->gvb.push_back(c);
        }
        if ((s = upload(p, &p->d_rp, rp.data(), rp.size()))) return fin(s);
        if ((s = upload(p, &p->d_ci, ci.data(), ci.size()))) return fin(s);
        if ((s = upload(p, &p->d_gvb_mids, mids.data(), mids.size()))) return fin(s);
        if (!chunks.empty() && (s = upload(p, &p->d_gvb_chunks, chunks.data(), chunks.size()))) return fin(s);
    }
    if (!batch) {
        // CSR copies for the plain comparators and the adjoints' value gradient
        if ((s = upload(p, &p->d_rp, p->hrp.data(), p->hrp.size()))) return fin(s);
        if ((s = upload(p, &p->d_ci, p->hci.data(), p->hci.size()))) return fin(s);
        if (p->has_adj) {
            // value gradient: rows longer than GV_LONG_ROW go in chunks of GV_CHUNK entries
            int64_t short_rows = 0, short_nnz = 0;
            for (int64_t r = 0; r < p->n_rows; r++) {
                const int32_t b0 = p->hrp[r], len = p->hrp[r + 1] - b0;
                if (len > GV_LONG_ROW) {
                    for (int32_t e = b0; e < b0 + len; e += GV_CHUNK) {
                        p->gv_chunks.push_back((int32_t)r);
                        p->gv_chunks.push_back(e);
                    }
                } else {
                    short_rows++;
                    short_nnz += len;
                }
            }
            p->gv_avg_short = short_rows ? std::max(1.0, (double)short_nnz / (double)short_rows) : 1.0;
            if (!p->gv_chunks.empty() && (s = upload(p, &p->d_gv_chunks, p->gv_chunks.data(), p->gv_chunks.size())))
                return fin(s);
            if ((s = upload(p, &p->d_rpT, rpT[0].data(), rpT[0].size()))) return fin(s);
            if ((s = upload(p, &p->d_ciT, ciT[0].data(), ciT[0].size()))) return fin(s);
        }
        if (kind == DDF_SPTRSV_LOWER) {
            std::vector<int32_t> rows(p->fwd[0].part_rows.begin(), p->fwd[0].part_rows.end());
            if ((s = upload(p, &p->d_rows, rows.data(), rows.size()))) return fin(s);
            if (p->has_adj) {
                std::vector<int32_t> rr(p->adj[0].part_rows.begin(), p->adj[0].part_rows.end());
                if ((s = upload(p, &p->d_rrows, rr.data(), rr.size()))) return fin(s);
            }
        }
    }
    return fin(DDF_OK);
}

bool overlap(const void *a, int64_t na, const void *b, int64_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

ddf_status need_device(ddf_plan_t p) {
    if (!p) return fail(DDF_E_ARG, "plan is NULL");
    if (p->host_only) return fail(DDF_E_UNSUPPORTED, "plan was inspected host-only");
    return DDF_OK;
}

ddf_status check_nrhs(int32_t k) {
    if (k < 1 || k > 32) return fail(DDF_E_ARG, "nrhs must be in 1..32");
    return DDF_OK;
}

const double *vals_or_own(ddf_plan_t p, const double *v) { return v ? v : p->d_vals; }

// One solve (adj: the transposed solve) over a schedule: tasks [t0, t0 + ntasks) of the
// one-launch-per-level lists.  Every path but 3 runs the dataflow tasks of D instead (matrix
// `mat` of a per-matrix schedule, or all).  An in-place call (b == x) takes one launch per
// level: the dataflow solve marks the output as not yet solved before it starts.
// Where a solve call keeps its scratch: the values in transposed order and the dataflow
// solve's counter lines (null: the plan's own), and the error flag it raises.
struct SolveScratch {
    double *valsT = nullptr;
    unsigned *ctr = nullptr;
    unsigned *err = nullptr;
};

ddf_status solve_launch(ddf_plan_t p, const DevTables &D, int64_t t0, int64_t ntasks, bool adj, const double *vals,
                        const double *b, double *x, int32_t k_override, int kt,
                        hipStream_t s, int mat = -1, const SolveScratch &scr = SolveScratch()) {
    const SchedParams &sp = adj ? p->sp_a : p->sp_f;
    SolveArgs a{};
    a.cods = adj ? p->T.d_cods : p->F.d_cods;
    a.aux = adj ? p->T.d_aux : p->F.d_aux;
    a.tasks = D.d_tasks + t0;
    a.tcods = D.d_tcods ? D.d_tcods + t0 : nullptr;
    a.sync = D.d_sync ? reinterpret_cast<const int4 *>(D.d_sync) + t0 : nullptr;
    a.ntasks = (int32_t)ntasks;
    a.backoff_max = sp.backoff > 0 ? sp.backoff : 16;
    a.mats = p->d_mats;
    a.vals = vals;
    a.perm = p->d_perm;
    a.b = b;
    a.x = x;
    a.ctr = scr.ctr ? scr.ctr : adj ? p->d_ctr_adj : p->d_ctr;
    a.err = scr.err;
    a.spin_limit = p->spin_limit;
    a.k_override = k_override;
    const bool single = k_override > 0;
    // the transposed solve of one matrix gathers its values in transposed order first, so that
    // no task reads them through perm (one matrix: 0.37 ms of gather against 0.56 ms more in
    // the dataflow solve on the 170^3 stencil)
    double *valsT = scr.valsT ? scr.valsT : p->d_valsT;
    if (adj && single && valsT && p->nnz) {
        HIPCHK(launch_gather(valsT, vals, p->d_perm, p->nnz, s));
        a.vals = valsT;
    }
    if (sp.path != 3 && b != x && !D.df_tasks.empty()) {
        const int64_t d0 = mat >= 0 ? D.df_ptr[mat] : 0;
        const int64_t d1 = mat >= 0 ? D.df_ptr[mat + 1] : (int64_t)D.df_tasks.size();
        SolveArgs df = a;
        df.tasks = D.d_df_tasks + d0;
        df.tcods = D.d_df_tcods + d0;
        df.lcols = D.d_df_lcols;
        df.slots = reinterpret_cast<const int2 *>(D.d_df_slots);
        df.mdesc = reinterpret_cast<const int4 *>(D.d_df_mdesc);
        df.mcols = D.d_df_mcols;
        df.ntasks = (int32_t)(d1 - d0);
        const int kr = single ? df_lanes(k_override) : 8;
        const int per_pass = WAVE_LANES / kr / DF_RG;
        df.npass = (int32_t)((df.ntasks + per_pass - 1) / per_pass);
        // the output block the tasks write: marked not yet solved before the launch
        double *fill = x;
        int64_t nfill = single ? p->n_rows * (int64_t)k_override : p->vec_total;
        if (mat >= 0) {
            fill = x + p->mats[mat].vec_base;
            nfill = (int64_t)p->mats[mat].n * p->mats[mat].k;
        }
        if (df.ntasks > 0) {
            HIPCHK(launch_df_reset(df.ctr, s));
            const auto tm = next_timer(p, 1);
            HIPCHK(launch_solve_df(df, adj, adj && !single, kr, sp.blocks, fill, nfill, s, tm.first, tm.second));
        }
        return DDF_OK;
    }
    // one launch per level (task ranges of equal level, over all matrices of a batch)
    const Task *tk = a.tasks;
    const DCod *tc = a.tcods;
    const int4 *sy = a.sync;
    int64_t nlaunch = 0;
    for (int64_t i = 0; i < ntasks; i++)
        if (i == 0 || D.sync[(t0 + i) * 4 + 3] != D.sync[(t0 + i - 1) * 4 + 3]) nlaunch++;
    const auto tm = next_timer(p, nlaunch);
    if (tm.first) (void)hipEventRecord(tm.first, s);
    int64_t i = 0;
    while (i < ntasks) {
        const int32_t lev = D.sync[(t0 + i) * 4 + 3];
        int64_t j = i + 1;
        while (j < ntasks && D.sync[(t0 + j) * 4 + 3] == lev) j++;
        a.tasks = tk + i;
        a.tcods = tc ? tc + i : nullptr;
        a.sync = sy + i;
        a.ntasks = (int32_t)(j - i);
        HIPCHK(launch_solve_range(a, adj, kt, s));
        i = j;
    }
    if (tm.second) (void)hipEventRecord(tm.second, s);
    return DDF_OK;
}

// Value gradient over the plan's CSR pattern (the forward matrix, diagonal included for a
// triangular plan): gv[e] = sign * <g[row], x[col]>.
hipError_t launch_gv_pass(ddf_plan_t p, const double *g, const double *x, double *gv, double sign, int32_t k,
                          hipStream_t s) {
    GvArgs a{};
    a.rp = p->d_rp;
    a.ci = p->d_ci;
    a.g = g;
    a.x = x;
    a.gv = gv;
    a.sign = sign;
    a.n = p->n_rows;
    a.k = k;
    a.chunks = reinterpret_cast<const int2 *>(p->d_gv_chunks);
    a.n_chunks = (int64_t)p->gv_chunks.size() / 2;
    return launch_gv(a, p->gv_avg_short, s);
}

// The batch adjoint's value gradient, gv[e] = -<lambda[row], x[col]> over every entry of every
// L_b (diagonal included): one pass over the packed CSR patterns per class of right-hand-side
// counts.
hipError_t launch_gv_batch(ddf_plan_t p, const double *lam, const double *x, double *gv, hipStream_t s) {
    for (const auto &c : p->gvb) {
        GvBatchArgs a{};
        a.rp = p->d_rp;
        a.ci = p->d_ci;
        a.g = lam;
        a.x = x;
        a.gv = gv;
        a.mats = p->d_mats;
        a.mids = p->d_gvb_mids + c.mid_off;
        a.mstart = a.mids + c.nm;
        a.nm = c.nm;
        a.n = c.nrows;
        a.chunks = reinterpret_cast<const int4 *>(p->d_gvb_chunks) + c.chunk_off;
        a.n_chunks = c.nchunks;
        if (hipError_t e = launch_gv_batch_class(a, c.kt, c.avg, s)) return e;
    }
    return hipSuccess;
}

// Column-slice plans: SpMV is one init launch (y = 0) and one launch of every slice task; the
// solve is one init launch (accumulators and tallies zeroed, rows without ops solved) and one
// launch per level that holds slices (the launch boundary orders the levels).
ddf_status sliced_run(ddf_plan_t p, const double *vals, const double *x_or_b, double *out, int32_t k,
                      hipStream_t s) {
    const bool solve = p->kind == DDF_SPTRSV_LOWER;
    SliceArgs a{};
    a.cods = p->F.d_cods;
    a.tasks = p->F.d_tasks;
    a.k = k;
    a.vals = vals;
    a.n = p->n_rows;
    if (solve) {
        const int64_t words = p->n_rows * (int64_t)k;
        if (words > p->acc_words) {
            drop_alloc(p, p->d_acc);
            p->d_acc = nullptr;
            p->acc_words = 0;
            if (ddf_status st = dalloc(p, (void **)&p->d_acc, (size_t)words * 8)) return st;
            p->acc_words = words;
        }
        a.x = out;
        a.y = p->d_acc;
        a.b = x_or_b;
        a.xs = out;
        a.cnt = p->d_tally;
        a.need = p->d_need;
        a.rp = p->d_rp;
    } else {
        a.x = x_or_b;
        a.y = out;
    }
    int64_t nlaunch = 1;
    if (solve) {
        for (size_t l = 0; l + 1 < p->sl_lvl.size(); l++) nlaunch += p->sl_lvl[l + 1] > p->sl_lvl[l];
    } else {
        nlaunch += !p->F.tasks.empty();
    }
    const auto tm = next_timer(p, nlaunch);
    if (tm.first) (void)hipEventRecord(tm.first, s);
    HIPCHK(launch_slices_init(a, s));
    if (solve) {
        for (size_t l = 0; l + 1 < p->sl_lvl.size(); l++) {
            if (p->sl_lvl[l + 1] == p->sl_lvl[l]) continue;
            a.tasks = p->F.d_tasks + p->sl_lvl[l];
            a.ntasks = (int32_t)(p->sl_lvl[l + 1] - p->sl_lvl[l]);
            HIPCHK(launch_slices(a, s));
        }
    } else {
        a.ntasks = (int32_t)p->F.tasks.size();
        HIPCHK(launch_slices(a, s));
    }
    if (tm.second) (void)hipEventRecord(tm.second, s);
    return DDF_OK;
}

ddf_status refuse_sliced(ddf_plan_t p) {
    if (p && p->sliced) return fail(DDF_E_UNSUPPORTED, "BLAS-only plans run the forward SpMV and solve only");
    return DDF_OK;
}

} // namespace

// =================================================================================================
// C ABI
// =================================================================================================
extern "C" {

void ddf_opts_default(ddf_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->window = 64;
    o->build_adjoint = 1;
    o->ops_per_lane = 4;
    o->rows_passes = 2;
    o->xcd_remap = -1;
    o->solve_blocks = 0;
    o->thin_helpers = -1;
    o->thin_ahead = 0;
}

const char *ddf_version(void) { return "ddf-mi355x 0.1"; }

const char *ddf_status_string(ddf_status s) {
    switch (s) {
    case DDF_OK: return "DDF_OK";
    case DDF_E_ARG: return "DDF_E_ARG";
    case DDF_E_CSR: return "DDF_E_CSR";
    case DDF_E_NOT_LOWER: return "DDF_E_NOT_LOWER";
    case DDF_E_NO_DIAG: return "DDF_E_NO_DIAG";
    case DDF_E_KIND: return "DDF_E_KIND";
    case DDF_E_NOMEM: return "DDF_E_NOMEM";
    case DDF_E_HIP: return "DDF_E_HIP";
    case DDF_E_DEVICE: return "DDF_E_DEVICE";
    case DDF_E_UNSUPPORTED: return "DDF_E_UNSUPPORTED";
    }
    return "DDF_E_UNKNOWN";
}

const char *ddf_last_error(void) { return last_error().c_str(); }

ddf_status ddf_inspect(ddf_kind kind, const ddf_csr_host *A, const ddf_opts *opts, ddf_plan_t *out) {
    if (!out) return fail(DDF_E_ARG, "out is NULL");
    *out = nullptr;
    if (!A) return fail(DDF_E_ARG, "matrix is NULL");
    try {
        return make_plan(kind, 1, A, nullptr, opts, false, out);
    } catch (const std::bad_alloc &) {
        return fail(DDF_E_NOMEM, "host allocation failed");
    }
}

ddf_status ddf_inspect_batch(ddf_kind kind, int32_t nmat, const ddf_csr_host *mats, const int32_t *nrhs,
                             const ddf_opts *opts, ddf_plan_t *out) {
    if (!out) return fail(DDF_E_ARG, "out is NULL");
    *out = nullptr;
    try {
        return make_plan(kind, nmat, mats, nrhs, opts, true, out);
    } catch (const std::bad_alloc &) {
        return fail(DDF_E_NOMEM, "host allocation failed");
    }
}

ddf_status ddf_plan_destroy(ddf_plan_t plan) {
    free_plan(plan);
    return DDF_OK;
}

ddf_status ddf_spmv_v(ddf_plan_t p, const double *d_vals, const double *d_x, double *d_y, int32_t nrhs,
                      ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (p->kind != DDF_SPMV) return fail(DDF_E_KIND, "plan is not an SpMV plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    if ((!d_vals && p->nnz) || (!d_x && p->n_cols) || (!d_y && p->n_rows)) return fail(DDF_E_ARG, "NULL buffer");
    if (overlap(d_x, p->n_cols * nrhs * 8, d_y, p->n_rows * nrhs * 8)) return fail(DDF_E_ARG, "x and y overlap");
    hipStream_t s = (hipStream_t)stream;
    if (p->n_rows == 0) return DDF_OK;
    if (p->sliced) return sliced_run(p, d_vals, d_x, d_y, nrhs, s);
    SpmvArgs a{};
    a.cods = p->F.d_cods;
    a.aux = p->F.d_aux;
    a.rp = p->d_rp;
    a.ci = p->d_ci;
    a.rows = p->F.d_rowlist;
    const bool many = nrhs > 1;
    a.tasks = many ? p->F.d_tasksN : p->F.d_tasks;
    a.ntasks = (int32_t)(many ? p->F.tasksN.size() : p->F.tasks.size());
    a.k = nrhs;
    a.remap = p->sp_f.remap;
    a.vals = d_vals;
    a.x = d_x;
    a.y = d_y;
    const auto tm = next_timer(p, 1);
    if (tm.first) (void)hipEventRecord(tm.first, s);
    HIPCHK(launch_spmv(a, false, s));
    if (tm.second) (void)hipEventRecord(tm.second, s);
    return DDF_OK;
}

ddf_status ddf_spmv(ddf_plan_t p, const double *d_x, double *d_y, int32_t nrhs, ddf_stream_t stream) {
    if (p && !p->d_vals && p->nnz) return fail(DDF_E_ARG, "plan holds no values: use ddf_spmv_v");
    return ddf_spmv_v(p, nullptr, d_x, d_y, nrhs, stream);
}

ddf_status ddf_sptrsv_v(ddf_plan_t p, const double *d_vals, const double *d_b, double *d_x, int32_t nrhs,
                        ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (p->kind != DDF_SPTRSV_LOWER || p->batch) return fail(DDF_E_KIND, "plan is not a single-matrix SpTRSV plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    int64_t nb = p->n_rows * nrhs * 8;
    if ((!d_vals && p->nnz) || (!d_b && p->n_rows) || (!d_x && p->n_rows)) return fail(DDF_E_ARG, "NULL buffer");
    if (d_b != d_x && overlap(d_b, nb, d_x, nb)) return fail(DDF_E_ARG, "b and x partially overlap");
    if (p->n_rows == 0) return DDF_OK;
    if (p->sliced) return sliced_run(p, d_vals, d_b, d_x, nrhs, (hipStream_t)stream);
    if (use_thin(p->F, p->sp_f, nrhs))
        return thin_launch(p, p->F, p->sp_f, p->F.thin_nlev, d_vals, d_b, d_x, nrhs, (hipStream_t)stream);
    // the single matrix's right-hand-side count is a per-call argument (k_override)
    return solve_launch(p, p->F, 0, (int64_t)p->F.tasks.size(), false, d_vals, d_b, d_x, nrhs,
                        kt_for(nrhs), (hipStream_t)stream);
}

ddf_status ddf_sptrsv(ddf_plan_t p, const double *d_b, double *d_x, int32_t nrhs, ddf_stream_t stream) {
    if (p && !p->d_vals && p->nnz) return fail(DDF_E_ARG, "plan holds no values: use ddf_sptrsv_v");
    return ddf_sptrsv_v(p, nullptr, d_b, d_x, nrhs, stream);
}

ddf_status ddf_spmv_adjoint(ddf_plan_t p, const double *d_vals, const double *d_x, const double *d_gy,
                            double *d_gx, double *d_gvals, int32_t nrhs, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (ddf_status s = refuse_sliced(p)) return s;
    if (p->kind != DDF_SPMV) return fail(DDF_E_KIND, "plan is not an SpMV plan");
    if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    if ((!d_vals && p->nnz) || (!d_gy && p->n_rows) || (d_gvals && !d_x && p->n_cols))
        return fail(DDF_E_ARG, "NULL buffer");
    if (d_gx && (overlap(d_gx, p->n_cols * nrhs * 8, d_gy, p->n_rows * nrhs * 8) ||
                 overlap(d_gx, p->n_cols * nrhs * 8, d_x, p->n_cols * nrhs * 8)))
        return fail(DDF_E_ARG, "gx overlaps an input");
    if (d_gvals && (overlap(d_gvals, p->nnz * 8, d_gy, p->n_rows * nrhs * 8) ||
                    overlap(d_gvals, p->nnz * 8, d_x, p->n_cols * nrhs * 8) ||
                    overlap(d_gvals, p->nnz * 8, d_gx, p->n_cols * nrhs * 8)))
        return fail(DDF_E_ARG, "gvals overlaps another buffer");
    hipStream_t s = (hipStream_t)stream;
    const bool many = nrhs > 1;
    const int64_t ngx = many ? p->n_gx_tasksN : p->n_gx_tasks;
    if (d_gvals && many && gv_plan_fits(nrhs, d_gy, d_x)) {
        GvPlanArgs g{};
        g.cods = p->F.d_cods;
        g.aux = p->F.d_aux;
        g.tasks = p->F.d_tasksN;
        g.ntasks = (int32_t)p->F.tasksN.size();
        g.k = nrhs;
        g.remap = p->sp_f.remap;
        g.g = d_gy;
        g.x = d_x;
        g.gv = d_gvals;
        g.sign = 1.0;
        HIPCHK(launch_gv_plan(g, s));
    } else if (d_gvals) {
        HIPCHK(launch_gv_pass(p, d_gy, d_x, d_gvals, 1.0, nrhs, s));
    }
    if (!d_gx || ngx == 0) return DDF_OK;
    SpmvArgs a{};
    a.cods = p->T.d_cods;
    a.aux = p->T.d_aux;
    a.rp = p->d_rpT;
    a.ci = p->d_ciT;
    a.rows = p->T.d_rowlist;
    a.tasks = many ? p->T.d_tasksN : p->T.d_tasks;
    a.ntasks = (int32_t)ngx;
    a.k = nrhs;
    a.remap = p->sp_a.remap;
    a.vals = d_vals;
    a.perm = p->d_perm;
    a.x = d_gy;
    a.y = d_gx;
    const auto tm = next_timer(p, 1);
    if (tm.first) (void)hipEventRecord(tm.first, s);
    HIPCHK(launch_spmv(a, true, s));
    if (tm.second) (void)hipEventRecord(tm.second, s);
    return DDF_OK;
}

ddf_status ddf_sptrsv_adjoint(ddf_plan_t p, const double *d_vals, const double *d_x, const double *d_gx,
                              double *d_gb, double *d_gvals, int32_t nrhs, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (ddf_status s = refuse_sliced(p)) return s;
    if (p->kind != DDF_SPTRSV_LOWER || p->batch) return fail(DDF_E_KIND, "plan is not a single-matrix SpTRSV plan");
    if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    int64_t nb = p->n_rows * nrhs * 8;
    if ((!d_vals && p->nnz) || (!d_gx && p->n_rows) || (!d_gb && p->n_rows) || (d_gvals && !d_x))
        return fail(DDF_E_ARG, "NULL buffer");
    if (d_gb != d_gx && overlap(d_gb, nb, d_gx, nb)) return fail(DDF_E_ARG, "gb and gx partially overlap");
    if (overlap(d_gb, nb, d_x, nb)) return fail(DDF_E_ARG, "gb overlaps x");
    if (d_gvals && (overlap(d_gvals, p->nnz * 8, d_gb, nb) || overlap(d_gvals, p->nnz * 8, d_x, nb)))
        return fail(DDF_E_ARG, "gvals overlaps another buffer");
    if (p->n_rows == 0) return DDF_OK;
    // the transposed solve for lambda, then the value gradient -lambda[row] x[col] of every entry
    // of L (diagonal included), in value order
    hipStream_t s = (hipStream_t)stream;
    if (use_thin(p->T, p->sp_a, nrhs)) {
        if (ddf_status st = thin_launch(p, p->T, p->sp_a, p->T.thin_nlev, d_vals, d_gx, d_gb, nrhs, s)) return st;
    } else if (ddf_status st = solve_launch(p, p->T, 0, p->n_solve_tasks_adj, true, d_vals, d_gx, d_gb,
                                            nrhs, kt_for(nrhs), s)) {
        return st;
    }
    if (d_gvals) HIPCHK(launch_gv_pass(p, d_gb, d_x, d_gvals, -1.0, nrhs, s));
    return DDF_OK;
}

ddf_status ddf_sptrsv_value_grad(ddf_plan_t p, const double *d_x, const double *d_gb, double *d_gvals,
                                 int32_t nrhs, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (p->kind != DDF_SPTRSV_LOWER || p->batch) return fail(DDF_E_KIND, "plan is not a single-matrix SpTRSV plan");
    if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    const int64_t nb = p->n_rows * nrhs * 8;
    if ((!d_x || !d_gb || !d_gvals) && p->n_rows) return fail(DDF_E_ARG, "NULL buffer");
    if (overlap(d_gvals, p->nnz * 8, d_gb, nb) || overlap(d_gvals, p->nnz * 8, d_x, nb))
        return fail(DDF_E_ARG, "gvals overlaps another buffer");
    if (p->n_rows == 0) return DDF_OK;
    HIPCHK(launch_gv_pass(p, d_gb, d_x, d_gvals, -1.0, nrhs, (hipStream_t)stream));
    return DDF_OK;
}

ddf_status ddf_sptrsv_adjoint_noalloc(ddf_plan_t p, const double *d_vals, const double *d_x, const double *d_gx,
                                      double *d_gb, double *d_gvals, int32_t nrhs, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (ddf_status s = refuse_sliced(p)) return s;
    if (p->kind != DDF_SPTRSV_LOWER || p->batch) return fail(DDF_E_KIND, "plan is not a single-matrix SpTRSV plan");
    if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    int64_t nb = p->n_rows * nrhs * 8;
    if ((!d_vals && p->nnz) || (!d_gx && p->n_rows) || (!d_gb && p->n_rows) || (d_gvals && !d_x))
        return fail(DDF_E_ARG, "NULL buffer");
    if (d_gb != d_gx && overlap(d_gb, nb, d_gx, nb)) return fail(DDF_E_ARG, "gb and gx partially overlap");
    if (overlap(d_gb, nb, d_x, nb)) return fail(DDF_E_ARG, "gb overlaps x");
    if (d_gvals && (overlap(d_gvals, p->nnz * 8, d_gb, nb) || overlap(d_gvals, p->nnz * 8, d_x, nb)))
        return fail(DDF_E_ARG, "gvals overlaps another buffer");
    if (p->nnz > NOALLOC_VALUES)
        return fail(DDF_E_ARG, "ddf_sptrsv_adjoint_noalloc: " + std::to_string(p->nnz) +
                                   " values exceed its static scratch of " + std::to_string(NOALLOC_VALUES));
    if (p->n_rows == 0) return DDF_OK;
    double *scr = nullptr;
    HIPCHK(noalloc_scratch(&scr));
    SolveScratch ss;
    ss.ctr = reinterpret_cast<unsigned *>(scr);
    ss.valsT = scr + NOALLOC_CTR_WORDS / 2;
    ss.err = p->d_ctr_adj + CTR_STRIDE; // reported by ddf_plan_sync_status like the other calls
    hipStream_t s = (hipStream_t)stream;
    // the dataflow transposed solve (in place: one launch per level), whatever path the plan
    // takes otherwise, then the value gradient
    const int32_t path = p->sp_a.path;
    p->sp_a.path = d_gb == d_gx ? 3 : 1;
    ddf_status st = solve_launch(p, p->T, 0, p->n_solve_tasks_adj, true, d_vals, d_gx, d_gb, nrhs,
                                 kt_for(nrhs), s, -1, ss);
    p->sp_a.path = path;
    if (st) return st;
    if (d_gvals) HIPCHK(launch_gv_pass(p, d_gb, d_x, d_gvals, -1.0, nrhs, s));
    return DDF_OK;
}

static int batch_kt(ddf_plan_t p) {
    int mk = 1;
    for (auto &m : p->mats) mk = std::max(mk, m.k);
    return kt_for(mk);
}

ddf_status ddf_sptrsv_batch(ddf_plan_t p, const double *d_vals, const double *d_b, double *d_x,
                            ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (!p->batch) return fail(DDF_E_KIND, "plan is not a batch plan");
    d_vals = vals_or_own(p, d_vals);
    int64_t nb = p->vec_total * 8;
    if ((!d_vals && p->nnz) || !d_b || !d_x) return fail(DDF_E_ARG, "NULL buffer");
    if (d_b != d_x && overlap(d_b, nb, d_x, nb)) return fail(DDF_E_ARG, "b and x partially overlap");
    return solve_launch(p, p->F, 0, (int64_t)p->F.tasks.size(), false, d_vals, d_b, d_x, 0,
                        batch_kt(p), (hipStream_t)stream);
}

ddf_status ddf_sptrsv_batch_adjoint(ddf_plan_t p, const double *d_vals, const double *d_x, const double *d_gx,
                                    double *d_gb, double *d_gvals, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (!p->batch) return fail(DDF_E_KIND, "plan is not a batch plan");
    if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    d_vals = vals_or_own(p, d_vals);
    int64_t nb = p->vec_total * 8;
    if ((!d_vals && p->nnz) || !d_gx || !d_gb || (d_gvals && !d_x)) return fail(DDF_E_ARG, "NULL buffer");
    if (d_gb != d_gx && overlap(d_gb, nb, d_gx, nb)) return fail(DDF_E_ARG, "gb and gx partially overlap");
    if (overlap(d_gb, nb, d_x, nb)) return fail(DDF_E_ARG, "gb overlaps x");
    hipStream_t s = (hipStream_t)stream;
    if (ddf_status st = solve_launch(p, p->T, 0, p->n_solve_tasks_adj, true, d_vals, d_gx, d_gb, 0, batch_kt(p), s))
        return st;
    if (d_gvals) HIPCHK(launch_gv_batch(p, d_gb, d_x, d_gvals, s));
    return DDF_OK;
}

ddf_status ddf_sptrsv_batch_per_matrix(ddf_plan_t p, const double *d_vals, const double *d_b, double *d_x,
                                       ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (!p->batch) return fail(DDF_E_KIND, "plan is not a batch plan");
    d_vals = vals_or_own(p, d_vals);
    if ((!d_vals && p->nnz) || !d_b || !d_x) return fail(DDF_E_ARG, "NULL buffer");
    if (d_b == d_x) return fail(DDF_E_ARG, "the per-matrix comparator does not run in place");
    // matrix after matrix: one dataflow launch each (the batch schedule's per-matrix lists)
    const int path = p->sp_f.path;
    p->sp_f.path = 1;
    ddf_status st = DDF_OK;
    for (int b = 0; b < p->nmat && !st; b++)
        st = solve_launch(p, p->Fpm, 0, 0, false, d_vals, d_b, d_x, 0, kt_for(p->mats[b].k),
                          (hipStream_t)stream, b);
    p->sp_f.path = path;
    return st;
    return DDF_OK;
}

ddf_status ddf_graph_create_batch(ddf_plan_t p, int32_t adjoint, const double *d_vals, const double *d_in,
                                  const double *d_x, double *d_out, double *d_gvals, ddf_graph_t *out) {
    if (!out) return fail(DDF_E_ARG, "out is NULL");
    *out = nullptr;
    if (ddf_status s = need_device(p)) return s;
    if (!p->batch) return fail(DDF_E_KIND, "plan is not a batch plan");
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    ddf_graph_s *g = new ddf_graph_s();
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    ddf_status st = DDF_OK;
    if (e == hipSuccess) {
        st = adjoint ? ddf_sptrsv_batch_adjoint(p, d_vals, d_x, d_in, d_out, d_gvals, s)
                     : ddf_sptrsv_batch(p, d_vals, d_in, d_out, s);
        hipError_t e2 = hipStreamEndCapture(s, &g->g);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess && st == DDF_OK) e = hipGraphInstantiate(&g->e, g->g, nullptr, nullptr, 0);
    g->plan = p;
    g->generation = p->generation;
    (void)hipStreamDestroy(s);
    if (st != DDF_OK || e != hipSuccess) {
        if (g->e) (void)hipGraphExecDestroy(g->e);
        if (g->g) (void)hipGraphDestroy(g->g);
        delete g;
        if (st != DDF_OK) return st;
        return fail(DDF_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *out = g;
    return DDF_OK;
}

ddf_status ddf_graph_launch(ddf_graph_t g, ddf_stream_t stream) {
    if (!g || !g->e) return fail(DDF_E_ARG, "graph is NULL");
    if (g->plan->generation != g->generation)
        return fail(DDF_E_ARG, "the plan's schedule changed (ddf_autotune) after this graph was captured: "
                               "capture it again");
    HIPCHK(hipGraphLaunch(g->e, (hipStream_t)stream));
    return DDF_OK;
}

ddf_status ddf_graph_destroy(ddf_graph_t g) {
    if (!g) return DDF_OK;
    if (g->e) (void)hipGraphExecDestroy(g->e);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
    return DDF_OK;
}

// ---------------------------------------------------------------- plain comparators

ddf_status ddf_plain_spmv(ddf_plan_t p, const double *d_vals, const double *d_x, double *d_y, int32_t nrhs,
                          ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (p->kind != DDF_SPMV) return fail(DDF_E_KIND, "plan is not an SpMV plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    if ((!d_vals && p->nnz) || !d_x || !d_y) return fail(DDF_E_ARG, "NULL buffer");
    if (overlap(d_x, p->n_cols * nrhs * 8, d_y, p->n_rows * nrhs * 8)) return fail(DDF_E_ARG, "x and y overlap");
    PlainArgs a{};
    a.rp = p->d_rp;
    a.ci = p->d_ci;
    a.vals = d_vals;
    a.x = d_x;
    a.y = d_y;
    a.n = p->n_rows;
    a.k = nrhs;
    HIPCHK(launch_plain(PLAIN_SPMV, a, p->n_rows ? (double)p->nnz / p->n_rows : 1.0, kt_for(nrhs),
                        (hipStream_t)stream));
    return DDF_OK;
}

ddf_status ddf_plain_sptrsv(ddf_plan_t p, const double *d_vals, const double *d_b, double *d_x, int32_t nrhs,
                            ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (p->kind != DDF_SPTRSV_LOWER || p->batch) return fail(DDF_E_KIND, "plan is not a single-matrix SpTRSV plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    int64_t nb = p->n_rows * nrhs * 8;
    if ((!d_vals && p->nnz) || !d_b || !d_x) return fail(DDF_E_ARG, "NULL buffer");
    if (d_b != d_x && overlap(d_b, nb, d_x, nb)) return fail(DDF_E_ARG, "b and x partially overlap");
    PlainArgs a{};
    a.rp = p->d_rp;
    a.ci = p->d_ci;
    a.vals = d_vals;
    a.rows = p->d_rows;
    a.x = d_b;
    a.y = d_x;
    a.k = nrhs;
    a.upper = 0;
    const Canon &c = p->fwd[0];
    double avg = p->n_rows ? (double)(p->nnz - p->n_rows) / p->n_rows : 1.0;
    for (int64_t l = 0; l < c.header[5]; l++) {
        a.lo = c.part_ptr[l];
        a.hi = c.part_ptr[l + 1];
        HIPCHK(launch_plain(PLAIN_LEVEL, a, avg, kt_for(nrhs), (hipStream_t)stream));
    }
    return DDF_OK;
}

ddf_status ddf_plain_spmv_adjoint(ddf_plan_t p, const double *d_vals, const double *d_x, const double *d_gy,
                                  double *d_gx, double *d_gvals, int32_t nrhs, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (p->kind != DDF_SPMV) return fail(DDF_E_KIND, "plan is not an SpMV plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    if ((!d_vals && p->nnz) || !d_x || !d_gy) return fail(DDF_E_ARG, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    if (d_gx) HIPCHK(launch_fill(d_gx, p->n_cols * nrhs, 0.0, s));
    PlainArgs a{};
    a.rp = p->d_rp;
    a.ci = p->d_ci;
    a.vals = d_vals;
    a.x = d_x;
    a.g = d_gy;
    a.y = d_gx;
    a.gv = d_gvals;
    a.n = p->n_rows;
    a.k = nrhs;
    HIPCHK(launch_plain(PLAIN_SPMV_ADJ, a, p->n_rows ? (double)p->nnz / p->n_rows : 1.0, 1, s));
    return DDF_OK;
}

ddf_status ddf_plain_sptrsv_adjoint(ddf_plan_t p, const double *d_vals, const double *d_x, const double *d_gx,
                                    double *d_gb, double *d_gvals, int32_t nrhs, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    if (p->kind != DDF_SPTRSV_LOWER || p->batch) return fail(DDF_E_KIND, "plan is not a single-matrix SpTRSV plan");
    if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    if (ddf_status s = check_nrhs(nrhs)) return s;
    d_vals = vals_or_own(p, d_vals);
    if ((!d_vals && p->nnz) || !d_gx || !d_gb || (d_gvals && !d_x)) return fail(DDF_E_ARG, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    PlainArgs a{};
    a.rp = p->d_rpT;
    a.ci = p->d_ciT;
    a.vals = d_vals;
    a.perm = p->d_perm;
    a.rows = p->d_rrows;
    a.x = d_gx;
    a.y = d_gb;
    a.k = nrhs;
    a.upper = 1;
    const Canon &c = p->adj[0];
    double avg = p->n_rows ? (double)(p->nnz - p->n_rows) / p->n_rows : 1.0;
    for (int64_t l = 0; l < c.header[5]; l++) {
        a.lo = c.part_ptr[l];
        a.hi = c.part_ptr[l + 1];
        HIPCHK(launch_plain(PLAIN_LEVEL, a, avg, kt_for(nrhs), s));
    }
    if (d_gvals) {
        PlainArgs g{};
        g.rp = p->d_rp;
        g.ci = p->d_ci;
        g.g = d_gb;
        g.x = d_x;
        g.gv = d_gvals;
        g.n = p->n_rows;
        g.k = nrhs;
        HIPCHK(launch_plain(PLAIN_GV, g, p->n_rows ? (double)p->nnz / p->n_rows : 1.0, 1, s));
    }
    return DDF_OK;
}

// ---------------------------------------------------------------- introspection

ddf_status ddf_plan_info(ddf_plan_t p, ddf_plan_info_t *o) {
    if (!p || !o) return fail(DDF_E_ARG, "NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->kind = p->kind;
    o->nmat = p->nmat;
    o->n_rows = (int32_t)p->n_rows;
    o->n_cols = (int32_t)p->n_cols;
    o->nnz = p->nnz;
    for (auto &c : p->fwd) {
        o->n_parts += c.header[5];
        o->n_regions += c.header[6];
        o->n_codelets += c.header[7];
        o->aux_len += c.header[8];
        for (int64_t i = 0; i < c.header[7]; i++) {
            const int64_t *r = &c.codelets[i * NCOD];
            o->codelets_by_type[r[C_TYPE]]++;
            o->ops_by_type[r[C_TYPE]] += r[C_P];
        }
    }
    o->n_tasks = (int64_t)p->F.tasks.size();
    o->n_tasks_adjoint = (int64_t)p->T.tasks.size();
    o->dev_plan_bytes = p->F.bytes();
    o->dev_plan_bytes_adj = p->has_adj ? p->T.bytes() : 0;
    o->has_adjoint = p->has_adj;
    o->max_levels = p->max_levels;
    o->inspect_seconds = p->inspect_seconds;
    for (int i = 0; i < 5; i++) o->phase_seconds[i] = p->phase_seconds[i];
    o->hash = p->hash;
    o->ops_per_lane = p->sp_f.ops_per_lane;
    o->rows_passes = p->sp_f.passes;
    o->xcd_remap = p->sp_f.remap;
    if (p->kind != 0) {
        o->solve_path = use_thin(p->F, p->sp_f, 1) ? 2 : p->sp_f.path == 3 ? 3 : 1;
        o->solve_path_adj = p->has_adj ? (use_thin(p->T, p->sp_a, 1) ? 2 : p->sp_a.path == 3 ? 3 : 1) : 0;
    }
    return DDF_OK;
}

ddf_status ddf_plan_export(ddf_plan_t p, int32_t which, int32_t mat, ddf_plan_tables_t *o) {
    if (!p || !o) return fail(DDF_E_ARG, "NULL argument");
    if (mat < 0 || mat >= p->nmat) return fail(DDF_E_ARG, "matrix index out of range");
    if (which != 0 && which != 1) return fail(DDF_E_ARG, "which must be 0 or 1");
    if (which == 1 && !p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    const Canon &c = which ? p->adj[mat] : p->fwd[mat];
    o->header = c.header;
    o->part_ptr = c.part_ptr.data();
    o->part_rows = c.part_rows.data();
    o->regions = c.regions.data();
    o->codelets = c.codelets.data();
    o->aux = c.aux.data();
    o->perm = which ? c.perm.data() : nullptr;
    return DDF_OK;
}

ddf_status ddf_plan_device_tables(ddf_plan_t p, int32_t which, ddf_device_tables_t *o) {
    if (!p || !o) return fail(DDF_E_ARG, "NULL argument");
    const DevTables *D = which == 0 ? &p->F : which == 1 ? &p->T : which == 2 ? &p->Fpm : nullptr;
    if (!D) return fail(DDF_E_ARG, "which must be 0, 1 or 2");
    if (which == 1 && !p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    const DevTables &S = which == 2 ? p->F : *D; // per-matrix schedules share F's records
    o->cods = reinterpret_cast<const int32_t *>(S.cods.data());
    o->aux = S.aux.data();
    o->tasks = reinterpret_cast<const int32_t *>(D->tasks.data());
    o->sync = D->sync.data();
    o->n_cods = (int64_t)S.cods.size();
    o->aux_len = (int64_t)S.aux.size();
    o->n_tasks = (int64_t)D->tasks.size();
    o->n_counters = D->n_counters;
    o->tasksN = reinterpret_cast<const int32_t *>(D->tasksN.data());
    o->n_tasksN = (int64_t)D->tasksN.size();
    o->thin_rec = D->thin_rec.data();
    o->thin_lvl = D->thin_lvl.data();
    o->n_thin_rec = (int64_t)D->thin_rec.size() / THIN_REC;
    o->n_thin_lvl = (int64_t)D->thin_lvl.size() / 4;
    o->thin_rows = D->thin_rows.data();
    o->thin_lg = D->thin_lg;
    o->thin_ring_size = D->thin_ring;
    o->thin_ngs = D->thin_ngs;
    o->thin_block = D->thin_block;
    o->rowlist = D->rowlist.data();
    o->n_rowlist = (int64_t)D->rowlist.size();
    o->df_tasks = reinterpret_cast<const int32_t *>(D->df_tasks.data());
    o->n_df_tasks = (int64_t)D->df_tasks.size();
    o->df_ptr = D->df_ptr.data();
    o->n_df_ptr = (int64_t)D->df_ptr.size();
    o->df_lcols = D->df_lcols.data();
    o->n_df_lcols = (int64_t)D->df_lcols.size();
    o->df_group = p->batch ? 1 : DF_PASS_MAX;
    o->df_slots = D->df_slots.data();
    o->n_df_slots = (int64_t)D->df_slots.size() / 2;
    o->df_reserved = 0;
    return DDF_OK;
}

ddf_status ddf_plan_traffic(ddf_plan_t p, ddf_op op, int32_t nrhs, int64_t *bytes_alg, int64_t *bytes_csr,
                            int64_t *flops) {
    if (!p) return fail(DDF_E_ARG, "plan is NULL");
    int64_t nnz = p->nnz, n = p->n_rows, nc = p->n_cols;
    int64_t vk = p->batch ? p->vec_total : n * nrhs;      // sum of n_b k_b
    int64_t ck = p->batch ? p->vec_total : nc * nrhs;
    int64_t kf = p->batch ? 0 : nrhs;
    const bool many = !p->batch && nrhs > 1;
    int64_t ba = 0, bc = 0, fl = 0;
    switch (op) {
    case DDF_OP_SPMV:
        ba = 8 * nnz + (many ? p->F.launch_bytes(true) : p->F.table_bytes1) + 8 * ck + 8 * vk;
        bc = 12 * nnz + 4 * (n + 1) + 8 * ck + 8 * vk;
        fl = 2 * nnz * nrhs;
        break;
    case DDF_OP_SPMV_ADJ:
        // transposed product: values through perm; value gradient over the CSR pattern, or with
        // 2, 4, 8, 16 or 32 right-hand sides over the forward plan's tasks
        if (many && (nrhs & (nrhs - 1)) == 0 && nrhs <= 32)
            ba = 20 * nnz + (p->has_adj ? p->T.launch_bytes(true) : 0) + p->F.launch_bytes(true) + 16 * vk + 16 * ck;
        else
            ba = 24 * nnz + (p->has_adj ? (many ? p->T.launch_bytes(true) : p->T.table_bytes1) : 0) + 4 * (n + 1) +
                 16 * vk + 16 * ck;
        bc = 20 * nnz + 4 * (n + 1) + 8 * vk + 16 * ck;
        fl = 2 * nnz * nrhs + nnz * (2 * nrhs - 1);
        break;
    case DDF_OP_SPTRSV:
        ba = 8 * nnz +
             (!p->batch && use_thin(p->F, p->sp_f, nrhs) ? p->F.thin_bytes()
              : p->sp_f.path != 3                        ? p->F.df_read_bytes()
                                                         : p->F.solve_read_bytes()) +
             16 * vk;
        bc = 12 * nnz + 4 * (n + 1) + 16 * vk;
        if (p->batch) {
            for (size_t b = 0; b < p->mats.size(); b++) {
                int64_t nz = p->fwd[b].header[3], nb = p->mats[b].n;
                fl += (int64_t)p->mats[b].k * (2 * (nz - nb) + nb);
            }
        } else {
            fl = kf * (2 * (nnz - n) + n);
        }
        break;
    case DDF_OP_SPTRSV_ADJ:
        // transposed solve, then the value gradient over the CSR pattern (columns and row pointers)
        // (batches: the solve reads the values through perm; one matrix: the values are first
        // copied in transposed order, written and read back)
        if (p->has_adj && !p->batch && use_thin(p->T, p->sp_a, nrhs))
            ba = 20 * nnz + p->T.thin_bytes() + 4 * (n + 1) + 24 * vk;
        else if (p->batch)
            ba = 24 * nnz + (p->has_adj ? (p->sp_a.path != 3 ? p->T.df_read_bytes() : p->T.solve_read_bytes()) : 0) +
                 4 * (n + 1) + 32 * vk;
        else
            ba = 24 * nnz + (p->has_adj ? (p->sp_a.path != 3 ? p->T.df_read_bytes() : p->T.solve_read_bytes()) : 0) +
                 4 * (n + 1) + 32 * vk + 16 * nnz;
        bc = 20 * nnz + 4 * (n + 1) + 24 * vk;
        if (p->batch) {
            for (size_t b = 0; b < p->mats.size(); b++) {
                int64_t nz = p->fwd[b].header[3], nb = p->mats[b].n, k = p->mats[b].k;
                fl += k * (2 * (nz - nb) + nb) + nz * (2 * k - 1);
            }
        } else {
            fl = kf * (2 * (nnz - n) + n) + nnz * (2 * kf - 1);
        }
        break;
    case DDF_OP_SPTRSV_T:
        if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
        if (!p->batch && use_thin(p->T, p->sp_a, nrhs))
            ba = 8 * nnz + p->T.thin_bytes() + 16 * vk;
        else
            ba = 8 * nnz +
                 (p->sp_a.path != 3 ? p->T.df_read_bytes()
                                    : (int64_t)p->T.aux.size() * 4 +
                                          p->n_solve_tasks_adj * (int64_t)(sizeof(Task) + sizeof(DCod) + 16)) +
                 16 * vk + (!p->batch ? 16 * nnz : 0);
        bc = 12 * nnz + 4 * (n + 1) + 16 * vk;
        fl = p->batch ? 0 : kf * (2 * (nnz - n) + n);
        break;
    case DDF_OP_SPMV_ADJ_KERNEL:
        // the transposed product alone: values through perm, the transposed plan's tables, g
        // read, gx written
        if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
        ba = 12 * nnz + (many ? p->T.launch_bytes(true) : p->T.table_bytes1) + 8 * vk + 8 * ck;
        bc = 12 * nnz + 4 * (nc + 1) + 8 * vk + 8 * ck;
        fl = 2 * nnz * nrhs;
        break;
    case DDF_OP_SPTRSV_ADJ_KERNEL:
        // the transposed solve kernel alone: values (already in U's order for one matrix,
        // through perm for a batch), tables, g read, lambda written
        if (!p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
        if (!p->batch && use_thin(p->T, p->sp_a, nrhs))
            ba = 8 * nnz + p->T.thin_bytes() + 16 * vk;
        else
            ba = (p->batch ? 12 : 8) * nnz + (p->sp_a.path != 3 ? p->T.df_read_bytes() : p->T.solve_read_bytes()) +
                 16 * vk;
        bc = 12 * nnz + 4 * (n + 1) + 16 * vk;
        fl = p->batch ? 0 : kf * (2 * (nnz - n) + n);
        break;
    default: return fail(DDF_E_ARG, "unknown op");
    }
    if (bytes_alg) *bytes_alg = ba;
    if (bytes_csr) *bytes_csr = bc;
    if (flops) *flops = fl;
    return DDF_OK;
}

ddf_status ddf_plan_sync_status(ddf_plan_t p, ddf_stream_t stream) {
    if (ddf_status s = need_device(p)) return s;
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    if (!p->d_ctr) return DDF_OK;
    bool tripped = false;
    for (unsigned *c : {p->d_ctr, p->d_ctr_adj}) {
        unsigned flag = 0;
        HIPCHK(hipMemcpy(&flag, c + CTR_STRIDE, sizeof(unsigned), hipMemcpyDeviceToHost));
        if (flag) {
            unsigned z = 0;
            HIPCHK(hipMemcpy(c + CTR_STRIDE, &z, sizeof(unsigned), hipMemcpyHostToDevice));
            tripped = true;
        }
    }
    if (tripped) return fail(DDF_E_DEVICE, "a level wait exceeded its spin limit");
    return DDF_OK;
}

ddf_status ddf_plan_time_kernels(ddf_plan_t p, int32_t enable) {
    if (ddf_status s = need_device(p)) return s;
    if (enable && p->tev.empty()) {
        p->tev.resize(2 * TIMED_CALLS, nullptr);
        for (hipEvent_t &e : p->tev) HIPCHK(hipEventCreate(&e));
    }
    p->timing = enable != 0;
    p->tev_used = 0;
    p->tev_launches = 0;
    return DDF_OK;
}

ddf_status ddf_plan_kernel_time(ddf_plan_t p, double *ms, int64_t *calls, int64_t *launches) {
    if (ddf_status s = need_device(p)) return s;
    if (!ms || !calls || !launches) return fail(DDF_E_ARG, "NULL argument");
    double total = 0;
    for (int i = 0; i < p->tev_used; i++) {
        HIPCHK(hipEventSynchronize(p->tev[2 * i + 1]));
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, p->tev[2 * i], p->tev[2 * i + 1]));
        total += t;
    }
    *ms = total;
    *calls = p->tev_used;
    *launches = p->tev_launches;
    return DDF_OK;
}

ddf_status ddf_plan_set_spin_limit(ddf_plan_t p, int64_t limit) {
    if (!p) return fail(DDF_E_ARG, "plan is NULL");
    p->spin_limit = limit > 0 ? limit : (int64_t(1) << 26);
    return DDF_OK;
}

} // extern "C"

// ---------------------------------------------------------------- autotuner

namespace {

std::mutex g_tune_mu;
std::map<std::string, SchedParams> g_tune_cache;

std::string tune_key(ddf_plan_t p, ddf_op op, int32_t nrhs) {
    std::ostringstream os;
    os << std::hex << p->hash << std::dec << ":" << (int)op << ":" << nrhs;
    return os.str();
}

void load_tune_file() {
    const char *path = getenv("DDF_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // one entry per line: "key": [ops_per_lane, passes, remap, blocks, path, helpers, ahead],
        size_t q1 = line.find('"'), q2 = line.find('"', q1 + 1), b = line.find('[');
        if (q1 == std::string::npos || q2 == std::string::npos || b == std::string::npos) continue;
        SchedParams sp;
        if (sscanf(line.c_str() + b, "[%d, %d, %d, %d, %d, %d, %d]", &sp.ops_per_lane, &sp.passes, &sp.remap,
                   &sp.blocks, &sp.path, &sp.helpers, &sp.ahead) == 7)
            g_tune_cache[line.substr(q1 + 1, q2 - q1 - 1)] = sp;
    }
}

void save_tune_file() {
    const char *path = getenv("DDF_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path);
    f << "{\n";
    size_t i = 0;
    for (auto &kv : g_tune_cache)
        f << "  \"" << kv.first << "\": [" << kv.second.ops_per_lane << ", " << kv.second.passes << ", "
          << kv.second.remap << ", " << kv.second.blocks << ", " << kv.second.path << ", " << kv.second.helpers
          << ", " << kv.second.ahead << "]"
          << (++i < g_tune_cache.size() ? "," : "") << "\n";
    f << "}\n";
}

} // namespace

extern "C" ddf_status ddf_autotune(ddf_plan_t p, ddf_op op, int32_t nrhs, ddf_stream_t stream, double budget_ms) {
    if (ddf_status s = need_device(p)) return s;
    if (ddf_status s = refuse_sliced(p)) return s;
    if (p->batch) nrhs = 1;
    else if (ddf_status s = check_nrhs(nrhs)) return s;
    if (op < DDF_OP_SPMV || op > DDF_OP_SPTRSV_ADJ) return fail(DDF_E_ARG, "autotune takes the four executor ops");
    bool is_spmv = op == DDF_OP_SPMV || op == DDF_OP_SPMV_ADJ;
    if (is_spmv != (p->kind == DDF_SPMV)) return fail(DDF_E_KIND, "op does not match the plan kind");
    bool adjop = op == DDF_OP_SPMV_ADJ || op == DDF_OP_SPTRSV_ADJ;
    if (adjop && !p->has_adj) return fail(DDF_E_UNSUPPORTED, "plan was built without its adjoint plan");
    if (!p->d_vals && p->nnz) return fail(DDF_E_ARG, "autotune needs values captured at inspect time");
    SchedParams &target = adjop ? p->sp_a : p->sp_f;
    const std::string key = tune_key(p, op, nrhs);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        static bool loaded = false;
        if (!loaded) {
            load_tune_file();
            loaded = true;
        }
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            target = it->second;
            return build_schedule(p, !adjop, adjop);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    int64_t nvec = p->batch ? p->vec_total : std::max(p->n_rows, p->n_cols) * nrhs;
    double *buf = nullptr;
    HIPCHK(hipMalloc(&buf, (3 * nvec + p->nnz + 1) * sizeof(double)));
    double *x = buf, *y = buf + nvec, *z = buf + 2 * nvec, *gv = buf + 3 * nvec;
    ddf_status st = launch_fill(x, 3 * nvec, 0.5, s) == hipSuccess ? DDF_OK : DDF_E_HIP;
    auto run = [&]() -> ddf_status {
        switch (op) {
        case DDF_OP_SPMV: return ddf_spmv_v(p, nullptr, x, y, nrhs, s);
        case DDF_OP_SPMV_ADJ: return ddf_spmv_adjoint(p, nullptr, x, z, y, gv, nrhs, s);
        case DDF_OP_SPTRSV:
            return p->batch ? ddf_sptrsv_batch(p, nullptr, x, y, s) : ddf_sptrsv_v(p, nullptr, x, y, nrhs, s);
        default:
            return p->batch ? ddf_sptrsv_batch_adjoint(p, nullptr, x, z, y, gv, s)
                            : ddf_sptrsv_adjoint(p, nullptr, x, z, y, gv, nrhs, s);
        }
    };
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    SchedParams best = target;
    float best_ms = 1e30f;
    double spent = 0;
    // candidates: SpMV varies lanes per row, row passes and XCD block order; the solve
    // varies lanes per row, row passes and whether small levels run as THIN ranges
    struct Cand {
        int opl, ps, rm, blocks, path, helpers, ahead;
    };
    std::vector<Cand> cands;
    cands.push_back({target.ops_per_lane, target.passes, target.remap, target.blocks, target.path, target.helpers,
                     target.ahead}); // current first
    if (is_spmv) {
        for (int rm : {1, 0})
            for (int opl : {1, 2, 4, 8, 16})
                for (int ps : {1, 2, 4}) cands.push_back({opl, ps, rm, 0, 0, target.helpers, target.ahead});
    } else {
        const DevTables &D = adjop ? p->T : p->F;
        if (!D.thin_rec.empty() && nrhs <= THIN_KT_MAX)
            for (int hp : {4, 2, 0})
                for (int ah : {24, 32, 64}) cands.push_back({target.ops_per_lane, target.passes, target.remap, 0, 2, hp, ah});
        if (!p->batch)
            for (int opl : {2, 1, 4})
                for (int ps : {1, 2}) cands.push_back({opl, ps, target.remap, 0, 3, target.helpers, target.ahead});
        // the dataflow solve: every resident block, or fewer waves polling ahead of the frontier
        const int full = resident_solve_blocks();
        for (int blocks : {0, full / 2, full / 4})
            cands.push_back({target.ops_per_lane, target.passes, target.remap, blocks, 1, target.helpers, target.ahead});
    }
    for (const Cand &cd : cands) {
        if (st || (budget_ms > 0 && spent > budget_ms)) break;
        target.ops_per_lane = cd.opl;
        target.passes = cd.ps;
        target.remap = cd.rm;
        target.blocks = cd.blocks;
        target.path = cd.path;
        target.helpers = cd.helpers;
        target.ahead = cd.ahead;
        if ((st = build_schedule(p, !adjop, adjop))) break;
        if ((st = run())) break;
        (void)hipEventRecord(e0, s);
        const int reps = 3;
        for (int r = 0; r < reps && !st; r++) st = run();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        spent += ms * (reps + 1);
        ms /= reps;
        if (ms < best_ms) {
            best_ms = ms;
            best = target;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    target = best;
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
        save_tune_file();
    }
    return build_schedule(p, !adjop, adjop);
}
