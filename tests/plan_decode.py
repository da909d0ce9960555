"""Test helper: decode canonical plan tables back into (row, value index, column) triples.

Independent of both inspectors: it only reads the published table layout.
"""
import numpy as np

F_S0, F_S1, F_S2, F_SEP, F_RECT, F_RUNS = 1, 2, 4, 8, 16, 32
C = {name: i for i, name in enumerate(
    ["type", "flags", "part", "region", "u", "m", "nn", "P", "row0", "row_step", "op0",
     "op_step", "col0", "sigma0", "sigma1", "aux_off", "aux_len", "cost"])}


def decode_codelet(rec, aux):
    """Returns (rows[m], opstart[m], counts[m], list of per-row column arrays)."""
    m, nn, fl = int(rec[C["m"]]), int(rec[C["nn"]]), int(rec[C["flags"]])
    p = int(rec[C["aux_off"]])
    end = p + int(rec[C["aux_len"]])
    if fl & F_S0:
        rows = rec[C["row0"]] + np.arange(m, dtype=np.int64) * rec[C["row_step"]]
    else:
        rows = aux[p:p + m].astype(np.int64)
        p += m
    if fl & F_S1:
        ops = rec[C["op0"]] + np.arange(m, dtype=np.int64) * rec[C["op_step"]]
    else:
        ops = aux[p:p + m].astype(np.int64)
        p += m
    if fl & F_RECT:
        cnt = np.full(m, nn, dtype=np.int64)
    else:
        cnt = aux[p:p + m].astype(np.int64)
        p += m
    col0, s0, s1 = int(rec[C["col0"]]), int(rec[C["sigma0"]]), int(rec[C["sigma1"]])
    cols = []
    if fl & F_S2:
        for a in range(m):
            cols.append(col0 + a * s0 + np.arange(cnt[a], dtype=np.int64) * s1)
    elif fl & F_SEP:
        if fl & F_RUNS:
            tab = aux[p:end].reshape(-1, 2)
            s = np.concatenate([o + np.arange(l) for o, l in tab]) if tab.size else np.zeros(0)
        else:
            s = aux[p:end].astype(np.int64)
        for a in range(m):
            cols.append(col0 + a * s0 + s.astype(np.int64))
    else:
        if fl & F_RUNS:
            tab = aux[p:end].reshape(-1, 2).astype(np.int64)
            j = 0
            for a in range(m):
                got = []
                tot = 0
                while tot < cnt[a]:
                    st, ln = tab[j]
                    got.append(st + np.arange(ln))
                    tot += ln
                    j += 1
                assert tot == cnt[a]
                cols.append(np.concatenate(got) if got else np.zeros(0, np.int64))
            assert j == tab.shape[0]
        else:
            flat = aux[p:end].astype(np.int64)
            o = 0
            for a in range(m):
                cols.append(flat[o:o + cnt[a]])
                o += cnt[a]
            assert o == flat.size
    return rows, ops, cnt, cols


def decode_plan(plan):
    """All (row, value index, column) triples of the plan, sorted by value index."""
    out = []
    for rec in plan["codelets"]:
        rows, ops, cnt, cols = decode_codelet(rec, plan["aux"])
        for a in range(len(rows)):
            n = int(cnt[a])
            if n:
                out.append(np.stack([np.full(n, rows[a]), ops[a] + np.arange(n), cols[a]], 1))
    if not out:
        return np.zeros((0, 3), dtype=np.int64)
    t = np.concatenate(out).astype(np.int64)
    return t[np.argsort(t[:, 1], kind="stable")]


def expected_triples(kind, A):
    rp = A.row_ptr.astype(np.int64)
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(rp))
    e = np.arange(rp[-1], dtype=np.int64)
    col = A.col_idx.astype(np.int64)
    if kind == 0:
        keep = np.ones(e.size, bool)
    elif kind == 1:
        keep = e != (rp[1:] - 1)[rows]
    else:
        keep = e != rp[:-1][rows]
    return np.stack([rows[keep], e[keep], col[keep]], 1)


def codelet_rows(plan):
    """Rows covered by each codelet, concatenated in codelet order."""
    out = []
    for rec in plan["codelets"]:
        rows, _, _, _ = decode_codelet(rec, plan["aux"])
        out.append(rows)
    return np.concatenate(out) if out else np.zeros(0, np.int64)
