"""Test helper: replays the kernels' indexing over the device tables on the CPU.

It reads the tables exactly as the HIP kernels do (record fields, flag bits, aux offsets,
tasks, groups, thin-level bounds), asserts that every table, value and column index stays
in bounds, that groups only read solution entries written by earlier groups, and returns the
results so they can be compared with the oracle.  It shares nothing with the library but
the published table layout.
"""
import numpy as np

FS0, FS1, FS2, FSEP, FRECT, FRUNS = 1, 2, 4, 8, 16, 32
DOPS, DCONTIG, DXPTR, DRPTR = 64, 128, 256, 512
TASK_STREAM = 1 << 10
TASK_CSR = 1 << 11
TASK_LONG = 1 << 12
TASK_ROWS = 1 << 13
ROWS_MAX_LEN = 8
STREAM_ELEMS = 512
F = {n: i for i, n in enumerate(["flags", "m", "nn", "row0", "row_step", "op0", "op_step", "col0", "sigma0",
                                 "sigma1", "rows_off", "ops_off", "cnt_off", "xt_off", "xp_off", "mat"])}


def xmode(fl):
    if fl & FS2:
        return 0
    if fl & FSEP:
        return 2 if fl & FRUNS else 1
    return 4 if fl & FRUNS else 3


class Tables:
    def __init__(self, t):
        self.cods, self.aux, self.tasks = t["cods"], t["aux"], t["tasks"]

    def a(self, i):
        assert 0 <= i < self.aux.size, f"aux index {i} out of [0, {self.aux.size})"
        return int(self.aux[i])

    def row_info(self, c, i0):
        fl = int(c[F["flags"]])
        assert 0 <= i0 < c[F["m"]]
        row = int(c[F["row0"]] + i0 * c[F["row_step"]]) if fl & FS0 else self.a(c[F["rows_off"]] + i0)
        opst = self.a(c[F["ops_off"]] + i0) if fl & DOPS else int(c[F["op0"]] + i0 * c[F["op_step"]])
        nops = int(c[F["nn"]]) if fl & FRECT else self.a(c[F["cnt_off"]] + i0)
        return row, opst, nops

    def cols(self, c, i0, opst, nops):
        fl = int(c[F["flags"]])
        mode = xmode(fl)
        out = []
        if mode == 0:
            base = int(c[F["col0"]] + i0 * c[F["sigma0"]])
            out = [base + i1 * int(c[F["sigma1"]]) for i1 in range(nops)]
        elif mode == 1:
            base = int(c[F["col0"]] + i0 * c[F["sigma0"]])
            out = [base + self.a(c[F["xt_off"]] + i1) for i1 in range(nops)]
        elif mode == 3:
            if fl & FRECT:
                off = i0 * int(c[F["nn"]])
            elif fl & DCONTIG:
                off = opst - int(c[F["op0"]])
            else:
                off = self.a(c[F["xp_off"]] + i0)
            out = [self.a(c[F["xt_off"]] + off + i1) for i1 in range(nops)]
        else:
            if mode == 2:
                rt, base = int(c[F["xt_off"]]), int(c[F["col0"]] + i0 * c[F["sigma0"]])
            else:
                rt, base = int(c[F["xt_off"]]) + 2 * self.a(c[F["xp_off"]] + i0), 0
            j, cum, ln, st = -1, 0, 0, 0
            for i1 in range(nops):
                while i1 >= cum + ln:
                    cum += ln
                    j += 1
                    st, ln = self.a(rt + 2 * j), self.a(rt + 2 * j + 1)
                out.append(base + st + (i1 - cum))
        return out

    def task_rows(self, t):
        """[(row, value indices, columns)] of task t, with the codelet record."""
        cod, i0b, i0e, meta = (int(v) for v in self.tasks[t])
        c = self.cods[cod]
        lg = meta & 7
        assert 0 <= i0b < i0e <= c[F["m"]]
        out = []
        for i0 in range(i0b, i0e):
            row, opst, nops = self.row_info(c, i0)
            out.append((row, opst, nops, self.cols(c, i0, opst, nops)))
        if meta & TASK_STREAM:
            # the stream kernel's own indexing: contiguous values from op0 + i0b*nn, and for a
            # full table contiguous columns from xt_off + i0b*nn
            fl, nn = int(c[F["flags"]]), int(c[F["nn"]])
            assert fl & FRECT and 1 <= nn and (i0e - i0b) * nn <= STREAM_ELEMS and not fl & DOPS
            assert i0e - i0b <= 64  # one row per lane sums the products
            assert c[F["m"]] == 1 or c[F["op_step"]] == nn
            mode = xmode(fl)
            assert mode in (0, 1, 3)
            ebase = int(c[F["op0"]]) + i0b * nn
            magic = (0xFFFFFFFF // nn + 1) & 0xFFFFFFFFFFFFFFFF  # the kernel's 64-bit divisor
            for e in range((i0e - i0b) * nn):
                assert (e * magic) >> 32 == e // nn
            for q, (row, opst, nops, cols) in enumerate(out):
                i0 = i0b + q
                assert opst == ebase + q * nn and row == (int(c[F["row0"]] + i0 * c[F["row_step"]]) if fl & FS0
                                                          else self.a(c[F["rows_off"]] + i0))
                for i1 in range(nn):
                    if mode == 0:
                        col = int(c[F["col0"]] + i0 * c[F["sigma0"]] + i1 * c[F["sigma1"]])
                    elif mode == 1:
                        col = int(c[F["col0"]] + i0 * c[F["sigma0"]]) + self.a(c[F["xt_off"]] + i1)
                    else:
                        col = self.a(c[F["xt_off"]] + i0b * nn + q * nn + i1)
                    assert col == cols[i1]
        return c, meta, out


def spmv(tabs, A, X, vals=None, perm=None, tasks=None, many=False):
    """Y = A X replayed over SpMV tasks (values through perm for the transposed plan); many
    selects the task list of several right-hand sides."""
    T = Tables(dict(tabs, tasks=tabs["tasksN"]) if many else tabs)
    v = A.values if vals is None else vals
    k = X.shape[1]
    Y = np.full((A.n_rows, k), np.nan)
    seen = np.zeros(A.n_rows, int)
    for t in (range(T.tasks.shape[0]) if tasks is None else tasks):
        meta = int(T.tasks[t][3])
        assert (meta >> 8) & 1 == 0  # every task computes rows
        if meta & TASK_CSR:
            # rows [i0b, i0e) straight from the CSR pattern (at most 64 rows and STREAM_ELEMS
            # elements, or one longer row)
            r0, r1 = int(T.tasks[t][1]), int(T.tasks[t][2])
            assert int(T.tasks[t][0]) == -1 and 0 <= r0 < r1 <= A.n_rows
            ne = int(A.row_ptr[r1]) - int(A.row_ptr[r0])
            if meta & TASK_LONG:
                assert r1 == r0 + 1 and ne > STREAM_ELEMS
            else:
                assert r1 - r0 <= 64 and ne <= STREAM_ELEMS
            rows = [(r, int(A.row_ptr[r]), int(A.row_ptr[r + 1] - A.row_ptr[r]),
                     A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]) for r in range(r0, r1)]
        elif meta & TASK_ROWS:
            # rows list[i0b, i0e) of the row list, one lane each, from the CSR pattern
            i0b, i0e = int(T.tasks[t][1]), int(T.tasks[t][2])
            lst = tabs["rowlist"]
            assert int(T.tasks[t][0]) == -1 and 0 <= i0b < i0e <= lst.size and i0e - i0b <= 64
            rows = []
            for r in lst[i0b:i0e]:
                r = int(r)
                assert 0 <= r < A.n_rows and A.row_ptr[r + 1] - A.row_ptr[r] <= ROWS_MAX_LEN
                rows.append((r, int(A.row_ptr[r]), int(A.row_ptr[r + 1] - A.row_ptr[r]),
                             A.col_idx[A.row_ptr[r]:A.row_ptr[r + 1]]))
        else:
            c, meta, rows = T.task_rows(t)
        for row, opst, nops, cols in rows:
            assert 0 <= row < A.n_rows
            seen[row] += 1
            acc = np.zeros(k)
            for i1, col in enumerate(cols):
                e = opst + i1
                assert 0 <= e < int(A.row_ptr[-1]) and 0 <= col < X.shape[0]
                acc += (v[perm[e]] if perm is not None else v[e]) * X[col]
            Y[row] = acc
    assert np.all(seen == 1), "rows not covered exactly once"
    return Y


def solve(tabs, L, B, kind=1, vals=None, perm=None, only_mat=None):
    """Replays the persistent solve task by task in ticket order.  kind 1: L X = B on L's
    plan; kind 2: U Lam = B with U = L^T, values through perm.  Checks the counter protocol:
    each task's wait is already satisfied by earlier tickets, every count waited for equals
    the number of tasks signalling that counter, and every solution entry a task reads was
    written by a task whose counter the wait covers."""
    T = Tables(tabs)
    sync = tabs["sync"]
    v = L.values if vals is None else vals
    n, k = B.shape
    X = np.full((n, k), np.nan)
    writer = np.full(n, -2)  # signal counter of the task that wrote each row

    def mat_of(t):
        return int(T.cods[int(T.tasks[t][0])][F["mat"]])

    # one launch covers the tasks of `only_mat` (per-matrix schedules reuse counter ids)
    mine = [t for t in range(T.tasks.shape[0]) if only_mat is None or mat_of(t) == only_mat]
    sigs = np.array([int(sync[t][2]) for t in mine], dtype=np.int64)
    nsig = np.bincount(sigs[sigs >= 0], minlength=max(1, int(tabs["n_counters"])))
    done = np.zeros_like(nsig)
    for t in mine:
        w, cnt, sig, _ = (int(x) for x in sync[t])
        if w >= 0:
            assert nsig[w] == cnt, "count waited for differs from the tasks signalling the counter"
            assert done[w] >= cnt, "wait not satisfied by earlier tickets"
        assert (int(T.tasks[t][3]) >> 8) & 1 == 0  # every task solves rows
        assert sig >= 0 and (w == -1 or w == sig - 1)
        c, _, rows = T.task_rows(t)
        pending = []
        for row, opst, nops, cols in rows:
            acc = np.zeros(k)
            for i1, col in enumerate(cols):
                e = opst + i1
                assert writer[col] >= 0 and writer[col] <= w, f"row {row} reads x[{col}] not covered by its wait"
                acc += (v[perm[e]] if kind == 2 else v[e]) * X[col]
            d = opst - 1 if kind == 2 else opst + nops
            diag = v[perm[d]] if kind == 2 else v[d]
            pending.append((row, (B[row] - acc) / diag))
        for row, val in pending:
            assert writer[row] == -2
            X[row] = val
            writer[row] = sig
        done[sig] += 1
    assert (writer >= 0).all()
    return X


DF_RG = 8
DF_PASS_MAX = 8
DF_U = 16  # ops of a lane's chunk: longer rows go in wide-row tasks
DF_LONG = 1 << 14  # a wide-row task: rows i0b, i0b + 1, ... (count in bits 16+), columns at df_lcols[i0e:]
DF_MIXED = 1 << 15  # a mixed task (batches): rows df_slots[i0b:i0e], each (codelet, row)


def df_solve(tabs, L, B, kind=1, vals=None, perm=None, only_mat=None):
    """Replays the dataflow solve's tasks in list order (kind 1: L X = B; kind 2: U Lam = B
    with U = L^T, values through perm).  Checks that a task holds at most DF_RG rows of one
    codelet, of at most DF_U ops each, or is a wide-row task of 1..8 consecutive rows of more
    than DF_U ops whose column list matches the codelet's columns, alone in its group of
    df_group tasks; that every solution entry a row reads was written by a task of an earlier
    group (so the list is a topological order, and the earliest unfinished task never waits);
    and exact cover."""
    T = Tables(dict(tabs, tasks=tabs["df_tasks"]))
    grp = tabs.get("df_group", DF_PASS_MAX)
    assert grp in (1, DF_PASS_MAX)
    v = L.values if vals is None else vals
    n, k = B.shape
    X = np.full((n, k), np.nan)
    written = np.full(n, -1)  # task that wrote each row
    ptr = tabs["df_ptr"]
    per_matrix = only_mat is not None and ptr.size > 2  # matrix after matrix, ranges in ptr
    lo, hi = (int(ptr[only_mat]), int(ptr[only_mat + 1])) if per_matrix else (0, T.tasks.shape[0])
    assert lo % grp == 0 and hi % grp == 0
    lcols = tabs.get("df_lcols", np.zeros(0, np.int32))
    slots = tabs.get("df_slots", np.zeros((0, 2), np.int32))
    wide_group = -1  # the group a wide-row task holds alone
    for t in range(lo, hi):
        cod, i0b, i0e, meta = (int(x) for x in T.tasks[t])
        assert 0 <= cod < T.cods.shape[0]
        c = T.cods[cod]
        if meta & DF_LONG:
            assert meta & 0xFFFF == DF_LONG and t % grp == 0
            nrow = meta >> 16
            assert 1 <= nrow <= DF_RG and i0b + nrow <= c[F["m"]]
            rows, off = [], i0e
            for i0 in range(i0b, i0b + nrow):
                row, opst, nops = T.row_info(c, i0)
                assert nops > DF_U and 0 <= off and off + nops <= lcols.size
                cols = [int(q) for q in lcols[off:off + nops]]
                assert cols == [int(q) for q in T.cols(c, i0, opst, nops)]
                rows.append((row, opst, nops, cols))
                off += nops
            wide_group = t // grp
        elif meta == DF_MIXED:
            # a batch's mixed task: up to DF_RG rows of any codelets (of one matrix here or not)
            assert grp == 1 and 1 <= i0e - i0b <= DF_RG and i0e <= slots.shape[0]
            rows = []
            for sc, si in slots[i0b:i0e]:
                sc, si = int(sc), int(si)
                assert 0 <= sc < T.cods.shape[0] and 0 <= si < T.cods[sc][F["m"]]
                row, opst, nops = T.row_info(T.cods[sc], si)
                assert nops <= DF_U
                if only_mat is None or int(T.cods[sc][F["mat"]]) == only_mat:
                    rows.append((row, opst, nops, T.cols(T.cods[sc], si, opst, nops)))
                else:
                    assert not per_matrix
        else:
            assert meta == 0 and 0 <= i0e - i0b <= DF_RG
            if i0e == i0b:
                continue  # padding: a wave pass never spans two levels
            assert t // grp != wide_group, "a wide-row task shares its group"
            _, _, rows = T.task_rows(t)
            assert all(nops <= DF_U for _, _, nops, _ in rows)
        if meta != DF_MIXED and only_mat is not None and int(c[F["mat"]]) != only_mat:
            assert not per_matrix
            continue
        for row, opst, nops, cols in rows:
            acc = np.zeros(k)
            for i1, col in enumerate(cols):
                e = opst + i1
                # written by a task of an earlier group (a wave pass takes up to a group's
                # consecutive tasks, all at once)
                assert 0 <= written[col] and written[col] // grp < t // grp, \
                    f"row {row} reads x[{col}] before an earlier pass wrote it"
                acc += (v[perm[e]] if kind == 2 else v[e]) * X[col]
            d = opst - 1 if kind == 2 else opst + nops
            diag = v[perm[d]] if kind == 2 else v[d]
            assert written[row] == -1
            X[row] = (B[row] - acc) / diag
            written[row] = t
    assert (written >= 0).all()
    return X


THIN_UNUSED = -(1 << 31)
THIN_VIDX_B = -1  # value index of a row's right-hand-side term
THIN_PIN = 2048  # pinned LDS entries past the ring's two constants


def thin_solve(tabs, L, B, vals=None, Xf=None):
    """Replays the single-block solve: level by level, G lanes per row (2G for wide rows),
    operands by their codes.  Checks that every ring operand finds its row in the LDS ring (its
    slot, solve-order index mod ring size, not overwritten by a row solved up to and including
    the reading level), that every global operand sits in one of the first thin_ngs slots of
    its lane, names the solve-order index of its column and was solved at least
    THIN_HORIZON levels before (so the gather two levels ahead sees it final), that a pinned
    operand's entry (past the ring's two constants) was written by its row, by that row alone,
    that empty slots carry no op, and that every row is solved once.  With Xf (transposed solve), also returns
    the value gradient of the follow-up pass: -<x[col], Xf[row]> at each op's value index and
    -<x[row], Xf[row]> at the diagonal."""
    rec, lvl, lg = tabs["thin_rec"], tabs["thin_lvl"], tabs["thin_lg"]
    M, ngs, rows_of = tabs["thin_ring_size"], tabs["thin_ngs"], tabs["thin_rows"]
    S = 5  # op slots per lane
    assert M > 0 and M & (M - 1) == 0 and ngs in (0, 1, 2, 3, 5) and rec.shape[1] == 21
    assert lvl.shape[0] % 4 == 0 and lvl.shape[1] == 4 and (lvl[-4:, 1] == 0).all()
    assert rec.shape[0] % 64 == 0 and tabs["thin_block"] >= lvl[:, 1].max()
    assert B.shape[1] == 1 and sorted(rows_of.tolist()) == list(range(B.shape[0]))
    v = L.values if vals is None else vals
    n, k = B.shape
    G = 1 << lg
    X = np.full((n, k), np.nan)
    gv = np.full(v.shape[0], np.nan) if Xf is not None else None
    level_of = np.full(n, -1)
    ring, pinned, pin_w = {}, {}, {}
    so_next = 0
    for l, (first, lanes, so0, nw) in enumerate(lvl):
        if lanes == 0:
            continue
        assert 0 < lanes <= 1024 and lanes % G == 0 and first % 64 == 0 and so0 == so_next
        nxt = first + (lanes + 63) // 64 * 64
        assert (rec[first:first + lanes, 3] == 0).all() and (rec[first + lanes:nxt, 3] == 1).all()
        assert (rec[first + lanes:nxt, 4 + 2 * S:4 + 3 * S] == THIN_UNUSED).all()
        acc, diag, dpos, slot = {}, {}, {}, {}
        reads, bterm = {}, set()
        rank = 0
        for s in range(lanes):
            r = rec[first + s]
            row, dp, cnt, wide = int(r[0]), int(r[1]), int(r[2]), int(r[19])
            assert wide in (0, 1, 2)
            if s % G == 0 and wide != 2:
                # head of a row of G lanes (wide = 0) or of 2G lanes (wide = 1, 2G-aligned; all
                # wide rows of a level come first)
                assert row not in acc and (wide == 0 or s % (2 * G) == 0)
                assert (wide == 1) == (rank < nw)
                so = so0 + rank
                assert rows_of[so] == row
                rank += 1
                acc[row] = np.zeros(k)
                diag[row], dpos[row] = v[dp], dp
                slot[row] = so % M
                # the writer's second LDS entry: its ring slot, or a pinned entry
                pin_w[row] = int(r[20])
                assert pin_w[row] == so % M or M + 2 <= pin_w[row] < M + 2 + THIN_PIN
            else:
                assert row in acc and int(r[20]) == -1
                prev = rec[first + s - (s % G if wide != 2 or s % G else G)]
                assert int(prev[0]) == row and (wide == int(prev[19]) or (wide == 2 and int(prev[19]) == 1))
            assert cnt == sum(int(c) != THIN_UNUSED for c in r[4 + 2 * S:4 + 3 * S])
            for j in range(S):
                vi, col, code = int(r[4 + j]), int(r[4 + S + j]), int(r[4 + 2 * S + j])
                if code == THIN_UNUSED:
                    continue
                if code == -(1 + M):
                    # the row's right-hand-side term (its operand is the entry past the ring)
                    assert vi == THIN_VIDX_B and col == row and row not in bterm
                    bterm.add(row)
                    continue
                m = level_of[col]
                assert 0 <= m < l, f"row {row} reads x[{col}] not solved in an earlier level"
                if code >= 0:
                    assert j < ngs and rows_of[code] == col and m <= l - 3
                elif -code - 1 >= M + 2:
                    assert pinned.get(-code - 1) == col, f"row {row} reads pinned entry {-code - 1}"
                else:
                    assert ring.get(-code - 1) == col
                    reads[-code - 1] = col
                acc[row] += v[vi] * X[col]
                if gv is not None:
                    assert np.isnan(gv[vi])
                    gv[vi] = -np.dot(X[col], Xf[row])
        so_next = so0 + rank
        # waves of one level may write before others read: no slot read here is written here
        assert not (set(slot.values()) & set(reads)), "a ring slot is read and overwritten in one level"
        assert bterm == set(acc), "every row has one right-hand-side term"
        for row, a in acc.items():
            assert level_of[row] == -1
            X[row] = (B[row] - a) / diag[row]
            level_of[row] = l
            ring[slot[row]] = row
            if pin_w[row] >= M + 2:
                assert pin_w[row] not in pinned, "a pinned entry is written twice"
                pinned[pin_w[row]] = row
            if gv is not None:
                gv[dpos[row]] = -np.dot(X[row], Xf[row])
    assert (level_of >= 0).all()
    return X if gv is None else (X, gv)
