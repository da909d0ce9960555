// DDF inspector (the paper's Algorithm 1, Sec. IV-A), optimised host implementation.
//
// Steps: validate the CSR; group independent rows (one group for SpMV, ASAP dependence
// levels for the solves); cut each group into windows of t consecutive rows
// (GetConsecutiveIterations); in every window run the three strategies BLAS_first,
// PSCI_first and PSCII_first, cost their codelet lists with Eq. (1) and keep the cheapest
// (ties: BLAS_first, PSCI_first, PSCII_first).
//
// A candidate codelet is a run of rows of one window.  Its class comes from the first order
// partial differences (Sec. III-D) of the access functions f0 (output row), f1 (value index)
// and f2 (input column): a function is strided when all of its FOPDs over the iteration
// space are equal (BLAS: three strided, PSC I: two, PSC II: one; Sec. III-B).  Each flag
// holds for a run iff it holds for every prefix of it, so the inspector tracks, per start
// row, the first run length at which each flag fails, extending runs one row at a time and
// resuming where an earlier query stopped (the memoisation of mined runs that Sec. IV-A
// describes).  The work per window is linear in its operations.  Windows are mined in
// parallel and concatenated in order, so the tables do not depend on the thread count.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>
#include <thread>

#include "ddf_internal.hpp"

namespace ddf {

ddf_status validate(int kind, const ddf_csr_host &A) {
    if (A.n_rows < 0 || A.n_cols < 0) return fail(DDF_E_ARG, "negative dimensions");
    if (!A.row_ptr) return fail(DDF_E_ARG, "row_ptr is NULL");
    if (A.row_ptr[0] != 0) return fail(DDF_E_CSR, "row_ptr[0] != 0");
    for (int64_t i = 0; i < A.n_rows; i++)
        if (A.row_ptr[i + 1] < A.row_ptr[i])
            return fail(DDF_E_CSR, "row_ptr decreases at row " + std::to_string(i));
    int64_t nnz = A.row_ptr[A.n_rows];
    if (nnz > 0 && !A.col_idx) return fail(DDF_E_ARG, "col_idx is NULL");
    for (int64_t i = 0; i < A.n_rows; i++) {
        for (int64_t e = A.row_ptr[i]; e < A.row_ptr[i + 1]; e++) {
            int32_t c = A.col_idx[e];
            if (c < 0 || c >= A.n_cols)
                return fail(DDF_E_CSR, "column out of range in row " + std::to_string(i));
            if (e > A.row_ptr[i] && c <= A.col_idx[e - 1])
                return fail(DDF_E_CSR, "columns not strictly increasing in row " + std::to_string(i));
        }
    }
    if (kind == DDF_SPTRSV_LOWER) {
        if (A.n_rows != A.n_cols) return fail(DDF_E_ARG, "triangular matrix must be square");
        for (int64_t i = 0; i < A.n_rows; i++) {
            int64_t b = A.row_ptr[i], e = A.row_ptr[i + 1];
            if (e == b) return fail(DDF_E_NO_DIAG, "row " + std::to_string(i) + " is empty");
            int32_t last = A.col_idx[e - 1];
            if (last > i) return fail(DDF_E_NOT_LOWER, "entry above the diagonal in row " + std::to_string(i));
            if (last != i) return fail(DDF_E_NO_DIAG, "row " + std::to_string(i) + " has no diagonal");
        }
    }
    return DDF_OK;
}

void transpose(int32_t n_rows, int32_t n_cols, const int32_t *rp, const int32_t *ci,
               std::vector<int32_t> &rpT, std::vector<int32_t> &ciT, std::vector<int32_t> &perm, int threads) {
    const int64_t nnz = rp[n_rows];
    rpT.assign((size_t)n_cols + 1, 0);
    ciT.resize(nnz);
    perm.resize(nnz);
    // row chunks on host threads: each counts its entries per column, the chunks' counts are
    // laid out column by column in chunk order, then each chunk scatters its own entries, so
    // a column's entries come in ascending row order as in the serial counting sort
    int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = (int)std::min<int64_t>({nt, 16, std::max<int64_t>(1, nnz / (int64_t(1) << 20))});
    std::vector<int64_t> rb(nt + 1);
    for (int t = 0; t <= nt; t++) {
        // chunk boundaries at rows that split the entries evenly
        const int64_t target = nnz * t / nt;
        rb[t] = std::lower_bound(rp, rp + n_rows + 1, (int32_t)target) - rp;
    }
    rb[nt] = n_rows;
    std::vector<std::vector<int32_t>> cnt(nt, std::vector<int32_t>((size_t)n_cols, 0));
    auto run = [&](auto &&f) {
        std::vector<std::thread> pool;
        for (int t = 1; t < nt; t++) pool.emplace_back(f, t);
        f(0);
        for (auto &th : pool) th.join();
    };
    run([&](int t) {
        int32_t *c = cnt[t].data();
        for (int64_t e = rp[rb[t]]; e < rp[rb[t + 1]]; e++) c[ci[e]]++;
    });
    // column starts, then each chunk's first slot in each column
    int64_t acc = 0;
    for (int64_t j = 0; j < n_cols; j++) {
        rpT[j] = (int32_t)acc;
        for (int t = 0; t < nt; t++) {
            const int32_t v = cnt[t][j];
            cnt[t][j] = (int32_t)acc;
            acc += v;
        }
    }
    rpT[n_cols] = (int32_t)acc;
    run([&](int t) {
        int32_t *next = cnt[t].data();
        for (int64_t i = rb[t]; i < rb[t + 1]; i++)
            for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
                const int32_t q = next[ci[e]]++;
                ciT[q] = (int32_t)i;
                perm[q] = (int32_t)e;
            }
    });
}

uint64_t hash_canon(const Canon &c, uint64_t h) {
    auto mix = [&h](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < n; i++) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    mix(c.header, sizeof(c.header));
    mix(c.part_ptr.data(), c.part_ptr.size() * 8);
    mix(c.codelets.data(), c.codelets.size() * 8);
    mix(c.aux.data(), c.aux.size() * 4);
    return h;
}

namespace {

constexpr int32_t NEVER = INT32_MAX;

// Everything known about one window: its rows and per-row facts.
struct Window {
    const Pattern *P;
    const int64_t *q; // rows of the window (positions pos0 .. pos0+T-1 of the partition)
    int32_t T;
    std::vector<int64_t> nops, opst, runs; // per position
    std::vector<uint8_t> arith;            // row's columns form one arithmetic progression
    std::vector<int64_t> pre_ops, pre_runs;

    void load(const Pattern &pat, const int64_t *rows, int32_t t) {
        P = &pat;
        q = rows;
        T = t;
        nops.resize(T);
        opst.resize(T);
        runs.resize(T);
        arith.resize(T);
        pre_ops.assign(T + 1, 0);
        pre_runs.assign(T + 1, 0);
        for (int32_t a = 0; a < T; a++) {
            int64_t r = q[a], o = pat.opstart(r), n = pat.nops(r);
            nops[a] = n;
            opst[a] = o;
            int64_t R = 0;
            bool ar = true;
            for (int64_t b = 0; b < n; b++) {
                if (b == 0 || pat.ci[o + b] != pat.ci[o + b - 1] + 1) R++;
                if (b >= 2 && pat.ci[o + b] - pat.ci[o + b - 1] != pat.ci[o + 1] - pat.ci[o]) ar = false;
            }
            runs[a] = R;
            arith[a] = ar;
            pre_ops[a + 1] = pre_ops[a] + n;
            pre_runs[a + 1] = pre_runs[a] + R;
        }
    }
    int64_t col(int32_t a, int64_t b) const { return P->ci[opst[a] + b]; }
};

// First run length at which each flag fails, for runs starting at position u.
struct Scan {
    int32_t m_done = 0;
    int32_t dRECT = NEVER, dS0 = NEVER, dS1 = NEVER, dSEP = NEVER, dS2 = NEVER;
    int64_t nn = 0, drow = 0, dop = 0, sig0 = 0;
    bool s2ok = false; // nn <= 1 or the first row is an arithmetic progression

    void start(const Window &W, int32_t u) {
        m_done = 1;
        dRECT = dS0 = dS1 = dSEP = NEVER;
        nn = W.nops[u];
        s2ok = nn <= 1 || W.arith[u];
        dS2 = s2ok ? NEVER : 1;
    }
    // flags of the run of length m (m <= m_done)
    int32_t flags(int32_t m) const {
        return (m < dS0 ? FS0 : 0) | (m < dS1 ? FS1 : 0) | (m < dS2 ? FS2 : 0) |
               (m < dSEP ? FSEP : 0) | (m < dRECT ? FRECT : 0);
    }
    // the need-th largest failure point of S0, S1, S2 (runs shorter than it keep `need`)
    int32_t limit(int need) const {
        int32_t d[3] = {dS0, dS1, dS2};
        std::sort(d, d + 3, [](int32_t a, int32_t b) { return a > b; });
        return d[need - 1];
    }
    void extend(const Window &W, int32_t u) {
        int32_t m = m_done + 1;
        int32_t a = u + m - 1; // the new row
        if (dRECT == NEVER && W.nops[a] != nn) dRECT = m;
        if (m == 2) {
            drow = W.q[u + 1] - W.q[u];
            dop = W.opst[u + 1] - W.opst[u];
        } else if (dS0 == NEVER && W.q[a] - W.q[a - 1] != drow) {
            dS0 = m;
        }
        if (dRECT != NEVER) {
            if (dS1 == NEVER) dS1 = dRECT;
            if (dSEP == NEVER) dSEP = dRECT;
        } else if (nn > 0) {
            if (dS1 == NEVER && W.opst[a] - W.opst[a - 1] != dop) dS1 = m;
            if (dSEP == NEVER) {
                if (m == 2) sig0 = W.col(u + 1, 0) - W.col(u, 0);
                for (int64_t b = 0; b < nn; b++)
                    if (W.col(a, b) - W.col(a - 1, b) != sig0) {
                        dSEP = m;
                        break;
                    }
            }
        }
        if (s2ok) dS2 = dSEP;
        m_done = m;
    }
    // L_need(u): longest run from u keeping at least `need` strided functions (0 if none)
    int32_t longest(const Window &W, int32_t u, int need) {
        int32_t cap = W.T - u;
        while (limit(need) > m_done && m_done < cap) extend(W, u);
        int32_t L = limit(need) - 1;
        return L < cap ? L : cap;
    }
};

struct CodeletDesc {
    int32_t flags; // canonical, RUNS included
    int64_t P, xtab, aux_len, cost;
};

CodeletDesc describe(const Window &W, const Scan &S, int32_t u, int32_t m) {
    CodeletDesc d;
    int32_t f = S.flags(m);
    d.P = W.pre_ops[u + m] - W.pre_ops[u];
    d.xtab = 0;
    if (!(f & FS2)) {
        int64_t plain, R;
        if (f & FSEP) {
            plain = W.nops[u];
            R = W.runs[u];
        } else {
            plain = d.P;
            R = W.pre_runs[u + m] - W.pre_runs[u];
        }
        if (2 * R < plain) {
            f |= FRUNS;
            d.xtab = 2 * R;
        } else {
            d.xtab = plain;
        }
    }
    int64_t s0 = (f & FS0) ? 0 : m, s1 = (f & FS1) ? 0 : m, cnt = (f & FRECT) ? 0 : m;
    d.flags = f;
    d.aux_len = s0 + s1 + cnt + d.xtab;
    d.cost = d.P + 3 + s0 + s1 + d.xtab;
    return d;
}

struct BlockOut {
    std::vector<int64_t> reg, cod;
    std::vector<int32_t> aux;
};

void emit(const Window &W, const Scan &S, int32_t u, int32_t m, int64_t part, int64_t region,
          BlockOut &out) {
    CodeletDesc d = describe(W, S, u, m);
    int32_t f = d.flags;
    int k = ((f & FS0) != 0) + ((f & FS1) != 0) + ((f & FS2) != 0);
    int64_t col0 = W.nops[u] > 0 ? W.col(u, 0) : 0;
    int64_t rec[NCOD];
    rec[C_TYPE] = 3 - k;
    rec[C_FLAGS] = f;
    rec[C_PART] = part;
    rec[C_REGION] = region;
    rec[C_U] = u;
    rec[C_M] = m;
    rec[C_NN] = (f & FRECT) ? W.nops[u] : -1;
    rec[C_P] = d.P;
    rec[C_ROW0] = W.q[u];
    rec[C_ROWSTEP] = ((f & FS0) && m >= 2) ? W.q[u + 1] - W.q[u] : 0;
    rec[C_OP0] = W.opst[u];
    rec[C_OPSTEP] = ((f & FS1) && m >= 2) ? W.opst[u + 1] - W.opst[u] : 0;
    rec[C_COL0] = col0;
    rec[C_SIG0] = ((f & FSEP) && m >= 2 && W.nops[u] > 0) ? W.col(u + 1, 0) - W.col(u, 0) : 0;
    rec[C_SIG1] = ((f & FS2) && W.nops[u] >= 2) ? W.col(u, 1) - W.col(u, 0) : 0;
    rec[C_AUXOFF] = (int64_t)out.aux.size(); // block-local, fixed at merge
    rec[C_AUXLEN] = d.aux_len;
    rec[C_COST] = d.cost;
    out.cod.insert(out.cod.end(), rec, rec + NCOD);
    if (!(f & FS0))
        for (int32_t a = u; a < u + m; a++) out.aux.push_back((int32_t)W.q[a]);
    if (!(f & FS1))
        for (int32_t a = u; a < u + m; a++) out.aux.push_back((int32_t)W.opst[a]);
    if (!(f & FRECT))
        for (int32_t a = u; a < u + m; a++) out.aux.push_back((int32_t)W.nops[a]);
    if (!(f & FS2)) {
        int32_t last = (f & FSEP) ? u + 1 : u + m;
        int64_t base = (f & FSEP) ? col0 : 0;
        for (int32_t a = u; a < last; a++) {
            int64_t n = W.nops[a];
            if (!(f & FRUNS)) {
                for (int64_t b = 0; b < n; b++) out.aux.push_back((int32_t)(W.col(a, b) - base));
            } else {
                int64_t b = 0;
                while (b < n) {
                    int64_t e = b + 1;
                    while (e < n && W.col(a, e) == W.col(a, e - 1) + 1) e++;
                    out.aux.push_back((int32_t)(W.col(a, b) - base));
                    out.aux.push_back((int32_t)(e - b));
                    b = e;
                }
            }
        }
    }
}

// The BLAS-only cover of a window (the ablation of Sec. V-A/V-B, every codelet BLAS): each
// row's ops cut greedily into column slices of one stride, then slices of consecutive rows
// with the same op offset, width and stride stacked while the row number, value start and
// first column keep the steps of the first two rows.  A codelet is ops [a, a + w) of m rows;
// rows without ops get none.  Region record: chosen strategy 3, costs (total, 0, 0).
struct Cut {
    int32_t a, w;
    int64_t s1;
};

void cover_blas_only(const Pattern &P, const int64_t *q, int32_t T, int64_t part, int64_t pos0, int64_t region,
                     Window &W, BlockOut &out) {
    W.load(P, q, T);
    std::vector<std::vector<Cut>> cuts(T);
    std::vector<std::vector<uint8_t>> taken(T);
    for (int32_t u = 0; u < T; u++) {
        const int64_t n = W.nops[u];
        for (int64_t a = 0; a < n;) {
            int64_t w = 1, s1 = 0;
            if (a + 1 < n) {
                s1 = W.col(u, a + 1) - W.col(u, a);
                for (w = 2; a + w < n && W.col(u, a + w) - W.col(u, a + w - 1) == s1; w++) {
                }
            }
            cuts[u].push_back({(int32_t)a, (int32_t)w, s1});
            a += w;
        }
        taken[u].assign(cuts[u].size(), 0);
    }
    // index of row u's cut that starts at op a, or -1
    auto find = [&](int32_t u, int32_t a) -> int64_t {
        auto it = std::lower_bound(cuts[u].begin(), cuts[u].end(), a,
                                   [](const Cut &c, int32_t v) { return c.a < v; });
        return (it != cuts[u].end() && it->a == a) ? it - cuts[u].begin() : -1;
    };
    const int64_t first = (int64_t)(out.cod.size() / NCOD);
    int64_t total = 0;
    for (int32_t u = 0; u < T; u++) {
        for (size_t j = 0; j < cuts[u].size(); j++) {
            if (taken[u][j]) continue;
            taken[u][j] = 1;
            const Cut c = cuts[u][j];
            int32_t m = 1;
            for (; u + m < T; m++) {
                const int64_t jj = find(u + m, c.a);
                if (jj < 0 || taken[u + m][jj] || cuts[u + m][jj].w != c.w || cuts[u + m][jj].s1 != c.s1) break;
                if (m >= 2 && (q[u + m] - q[u + m - 1] != q[u + 1] - q[u] ||
                               W.opst[u + m] - W.opst[u + m - 1] != W.opst[u + 1] - W.opst[u] ||
                               W.col(u + m, c.a) - W.col(u + m - 1, c.a) != W.col(u + 1, c.a) - W.col(u, c.a)))
                    break;
                taken[u + m][jj] = 1;
            }
            int64_t rec[NCOD];
            rec[C_TYPE] = 0;
            rec[C_FLAGS] = FS0 | FS1 | FS2 | FSEP | FRECT;
            rec[C_PART] = part;
            rec[C_REGION] = region;
            rec[C_U] = u;
            rec[C_M] = m;
            rec[C_NN] = c.w;
            rec[C_P] = (int64_t)m * c.w;
            rec[C_ROW0] = q[u];
            rec[C_ROWSTEP] = m >= 2 ? q[u + 1] - q[u] : 0;
            rec[C_OP0] = W.opst[u] + c.a;
            rec[C_OPSTEP] = m >= 2 ? W.opst[u + 1] - W.opst[u] : 0;
            rec[C_COL0] = W.col(u, c.a);
            rec[C_SIG0] = m >= 2 ? W.col(u + 1, c.a) - W.col(u, c.a) : 0;
            rec[C_SIG1] = c.w >= 2 ? c.s1 : 0;
            rec[C_AUXOFF] = 0; // no tables
            rec[C_AUXLEN] = 0;
            rec[C_COST] = (int64_t)m * c.w + 3;
            total += rec[C_COST];
            out.cod.insert(out.cod.end(), rec, rec + NCOD);
        }
    }
    const int64_t reg[NREG] = {part, pos0, T, first, 3, total, 0, 0};
    out.reg.insert(out.reg.end(), reg, reg + NREG);
}

// Mines one window; appends its region record and chosen codelets.
void mine_window(const Pattern &P, const int64_t *q, int32_t T, int64_t part, int64_t pos0,
                 int64_t region, Window &W, std::vector<Scan> &scans, BlockOut &out) {
    W.load(P, q, T);
    scans.resize(T);
    std::vector<uint8_t> started(T, 0);
    auto scan = [&](int32_t u) -> Scan & {
        if (!started[u]) {
            scans[u].start(W, u);
            started[u] = 1;
        }
        return scans[u];
    };
    auto run = [&](int s, bool doemit) -> int64_t {
        int64_t total = 0;
        int32_t u = 0;
        while (u < T) {
            Scan &S = scan(u);
            int32_t m;
            if (s == 0) {
                m = S.longest(W, u, 3);
                if (m < 1) m = S.longest(W, u, 2);
            } else if (s == 1) {
                m = S.longest(W, u, 2);
            } else {
                m = S.longest(W, u, 1);
            }
            if (doemit)
                emit(W, S, u, m, part, region, out);
            else
                total += describe(W, S, u, m).cost;
            u += m;
        }
        return total;
    };
    int64_t cost[3];
    for (int s = 0; s < 3; s++) cost[s] = run(s, false);
    int best = 0;
    for (int s = 1; s < 3; s++)
        if (cost[s] < cost[best]) best = s;
    int64_t rec[NREG] = {part, pos0, T, (int64_t)(out.cod.size() / NCOD), best, cost[0], cost[1], cost[2]};
    out.reg.insert(out.reg.end(), rec, rec + NREG);
    run(best, true);
}

} // namespace

void inspect(const Pattern &P, int32_t t, int threads, Canon &C, bool only_blas) {
    const int64_t n = P.n_rows;
    C.sliced = only_blas;
    // 1) grouping independent rows
    std::vector<int32_t> grp((size_t)std::max<int64_t>(n, 1), 0);
    int64_t nparts = 0;
    if (P.kind == 0) {
        nparts = n > 0 ? 1 : 0;
    } else if (P.kind == 1) {
        for (int64_t i = 0; i < n; i++) {
            int32_t l = 0;
            for (int64_t e = P.rp[i]; e < P.rp[i + 1] - 1; e++) l = std::max(l, grp[P.ci[e]] + 1);
            grp[i] = l;
            nparts = std::max<int64_t>(nparts, l + 1);
        }
    } else {
        for (int64_t i = n - 1; i >= 0; i--) {
            int32_t l = 0;
            for (int64_t e = P.rp[i] + 1; e < P.rp[i + 1]; e++) l = std::max(l, grp[P.ci[e]] + 1);
            grp[i] = l;
            nparts = std::max<int64_t>(nparts, l + 1);
        }
    }
    C.part_ptr.assign(nparts + 1, 0);
    C.part_rows.assign(n, 0);
    for (int64_t i = 0; i < n; i++) C.part_ptr[grp[i] + 1]++;
    for (int64_t l = 0; l < nparts; l++) C.part_ptr[l + 1] += C.part_ptr[l];
    {
        std::vector<int64_t> fill(C.part_ptr.begin(), C.part_ptr.end() - 1);
        for (int64_t i = 0; i < n; i++) C.part_rows[fill[grp[i]]++] = i;
    }
    // 2) windows
    struct Win {
        int64_t part, pos0;
        int32_t T;
    };
    std::vector<Win> wins;
    for (int64_t l = 0; l < nparts; l++) {
        int64_t size = C.part_ptr[l + 1] - C.part_ptr[l];
        for (int64_t p0 = 0; p0 < size; p0 += t) wins.push_back({l, p0, (int32_t)std::min<int64_t>(t, size - p0)});
    }
    const int64_t nw = (int64_t)wins.size();
    const int64_t BLK = 2048;
    const int64_t nblk = (nw + BLK - 1) / BLK;
    std::vector<BlockOut> blocks(nblk);
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        Window W;
        std::vector<Scan> scans;
        for (;;) {
            int64_t b = next.fetch_add(1);
            if (b >= nblk) break;
            BlockOut &out = blocks[b];
            for (int64_t w = b * BLK; w < std::min(nw, (b + 1) * BLK); w++) {
                const Win &wi = wins[w];
                const int64_t *q = C.part_rows.data() + C.part_ptr[wi.part] + wi.pos0;
                if (only_blas)
                    cover_blas_only(P, q, wi.T, wi.part, wi.pos0, w, W, out);
                else
                    mine_window(P, q, wi.T, wi.part, wi.pos0, w, W, scans, out);
            }
        }
    };
    int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = (int)std::min<int64_t>(nt, std::max<int64_t>(nblk, 1));
    if (nt <= 1) {
        worker();
    } else {
        std::vector<std::thread> pool;
        for (int i = 0; i < nt; i++) pool.emplace_back(worker);
        for (auto &th : pool) th.join();
    }
    // 3) concatenate blocks in window order
    int64_t ncod = 0, naux = 0;
    for (auto &b : blocks) {
        ncod += (int64_t)b.cod.size() / NCOD;
        naux += (int64_t)b.aux.size();
    }
    C.regions.resize((size_t)nw * NREG);
    C.codelets.resize((size_t)ncod * NCOD);
    C.aux.resize(naux);
    int64_t cbase = 0, abase = 0, rpos = 0;
    for (auto &b : blocks) {
        int64_t nc = (int64_t)b.cod.size() / NCOD;
        for (size_t r = 0; r < b.reg.size(); r += NREG) {
            for (int z = 0; z < NREG; z++) C.regions[rpos + z] = b.reg[r + z];
            C.regions[rpos + 3] += cbase;
            rpos += NREG;
        }
        for (int64_t c = 0; c < nc; c++) {
            int64_t *dst = &C.codelets[(cbase + c) * NCOD];
            std::memcpy(dst, &b.cod[c * NCOD], NCOD * 8);
            if (!only_blas) dst[C_AUXOFF] += abase;
        }
        std::memcpy(C.aux.data() + abase, b.aux.data(), b.aux.size() * 4);
        cbase += nc;
        abase += (int64_t)b.aux.size();
        b = BlockOut();
    }
    C.header[0] = P.kind;
    C.header[1] = P.n_rows;
    C.header[2] = P.n_cols;
    C.header[3] = P.rp[P.n_rows];
    C.header[4] = t;
    C.header[5] = nparts;
    C.header[6] = nw;
    C.header[7] = ncod;
    C.header[8] = naux;
}

} // namespace ddf
