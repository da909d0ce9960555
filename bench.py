"""Benchmark of the DDF hot path on one MI355X.

One step = SpMV forward, SpMV adjoint (A^T g and dA), SpTRSV forward and SpTRSV adjoint
(L^T lambda = g and dL) on one synthetic workload, FP64, inputs resident in HBM.  The
adjoint's transposed solve does not need the forward solution, and the SpMV calls need
neither solve, so the step runs on three streams: the forward solve, the transposed solve
(then its value gradient, once the forward solve is done), and the two SpMV calls.  The
serial step time is reported too.  The value is
whole-step effective HBM bandwidth: the algorithmic bytes of the four calls (values, plan
tables, vectors read once and written once; see ddf_plan_traffic) divided by the step time.
The plain GPU comparators (CSR-vector SpMV, FP64-atomic adjoint, one launch per level) are
timed the same way, and the CPU oracle on a bounded sample of the same step.

    python bench.py [--steps K] [--warmup W] [--workload c2|c5|c1|c3|c4]

With --workload c4 (256 triangular matrices with 1..32 right-hand sides each) a step is the
batched solve and its adjoint, one launch each; the comparator is one launch per matrix.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBPS = 8000.0  # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--op-reps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-op", default="", help="run only this op K times (for rocprofv3)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernels_sha():
    """Digest of the library's sources (kernels and the schedules that drive them)."""
    d = os.path.join(ROOT, "paper_2111_12243_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:12]


def traffic_from_profiles(op, workload):
    """HBM bytes per call (every kernel the call launches) from a committed rocprofv3 counter
    summary, when it was taken on the current library sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{op}_{workload}.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"sources_sha:\s*(\w+)", txt)
    m_b = re.search(r"hbm_bytes_per_call:\s*([0-9.eE+]+)", txt)
    if not m_sha or not m_b or m_sha.group(1) != kernels_sha():
        return None
    return float(m_b.group(1))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "of this path is a design note, not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2111_12243_amd import ddf
    from paper_2111_12243_amd import inputs as I

    if not os.path.exists(ddf.LIB_PATH):
        from paper_2111_12243_amd import build as B
        B.build()
    dev = torch.device("cuda:0")
    if args.workload == "c4":
        return bench_batch(args, np, torch, ddf, I, dev)
    t0 = time.time()
    w = I.workload(args.workload)
    log(f"[bench] workload {w.name} generated in {time.time() - t0:.1f}s")
    k = w.k
    A, L = w.A, w.L

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    t0 = time.time()
    pA = ddf.ddf_inspect(ddf.DDF_SPMV, A)
    tA = time.time() - t0
    t0 = time.time()
    pL = ddf.ddf_inspect(ddf.DDF_SPTRSV_LOWER, L) if L is not None else None
    tL = time.time() - t0
    log(f"[bench] inspect: A {tA:.2f}s, L {tL:.2f}s")
    vA, X, Gy = d(A.values), d(w.X), d(w.Gy)
    Y = torch.empty((A.n_rows, k), dtype=torch.float64, device=dev)
    GX = torch.empty((A.n_cols, k), dtype=torch.float64, device=dev)
    GVA = torch.empty(A.nnz, dtype=torch.float64, device=dev)
    if pL is not None:
        vL, Bv, Gx = d(L.values), d(w.B), d(w.Gx)
        Xs = torch.empty_like(Bv)
        GB = torch.empty_like(Bv)
        GVL = torch.empty(L.nnz, dtype=torch.float64, device=dev)

    ops = {
        "spmv": lambda: ddf.ddf_spmv_v(pA, vA, X, Y, k),
        "spmv_adj": lambda: ddf.ddf_spmv_adjoint(pA, vA, X, Gy, GX, GVA, k),
    }
    plain = {
        "spmv": lambda: ddf.ddf_plain_spmv(pA, vA, X, Y, k),
        "spmv_adj": lambda: ddf.ddf_plain_spmv_adjoint(pA, vA, X, Gy, GX, GVA, k),
    }
    if pL is not None:
        ops["sptrsv"] = lambda: ddf.ddf_sptrsv_v(pL, vL, Bv, Xs, k)
        ops["sptrsv_adj"] = lambda: ddf.ddf_sptrsv_adjoint(pL, vL, Xs, Gx, GB, GVL, k)
        plain["sptrsv"] = lambda: ddf.ddf_plain_sptrsv(pL, vL, Bv, Xs, k)
        plain["sptrsv_adj"] = lambda: ddf.ddf_plain_sptrsv_adjoint(pL, vL, Xs, Gx, GB, GVL, k)

    if not args.no_tune:
        t0 = time.time()
        ddf.ddf_autotune(pA, ddf.DDF_OP_SPMV, k, budget_ms=1500)
        ddf.ddf_autotune(pA, ddf.DDF_OP_SPMV_ADJ, k, budget_ms=1500)
        if pL is not None:
            ddf.ddf_autotune(pL, ddf.DDF_OP_SPTRSV, k, budget_ms=3000)
            ddf.ddf_autotune(pL, ddf.DDF_OP_SPTRSV_ADJ, k, budget_ms=3000)
        torch.cuda.synchronize()
        log(f"[bench] autotune {time.time() - t0:.1f}s")

    # algorithmic bytes per call, for the schedules the tuner settled on
    traffic = {"spmv": ddf.ddf_plan_traffic(pA, ddf.DDF_OP_SPMV, k),
               "spmv_adj": ddf.ddf_plan_traffic(pA, ddf.DDF_OP_SPMV_ADJ, k)}
    if pL is not None:
        traffic["sptrsv"] = ddf.ddf_plan_traffic(pL, ddf.DDF_OP_SPTRSV, k)
        traffic["sptrsv_adj"] = ddf.ddf_plan_traffic(pL, ddf.DDF_OP_SPTRSV_ADJ, k)

    if args.profile_op:
        # a leg per name, each run --steps times (rocprofv3 counter and trace runs); "copy" is
        # an elementwise copy of 64 Mi doubles (512 MiB read, 512 MiB written) to scale counters.
        # A one-element fill ends each leg, so that a trace splits into legs at its fill kernels.
        mark = torch.zeros(1, dtype=torch.float64, device=dev)
        for leg, name in enumerate(args.profile_op.split(",")):
            if name == "copy":
                src = torch.rand(1 << 26, dtype=torch.float64, device=dev)
                dst = torch.empty_like(src)
                fn = lambda: torch.mul(src, 1.0, out=dst)  # noqa: E731
            else:
                fn = ops[name]
            for _ in range(args.steps):
                fn()
            mark.fill_(float(leg))
            torch.cuda.synchronize()
            log(f"[bench] ran {name} x{args.steps}")
        return

    def step(table):
        for f in table.values():
            f()

    def time_steps(table, n, warm, per_op=None):
        """Average ms per step over n steps; with per_op, also each call's average from HIP
        events recorded around it on the stream the calls launch on."""
        for _ in range(warm):
            step(table)
        torch.cuda.synchronize()
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        e0, e1 = ev(), ev()
        marks = {name: [] for name in table} if per_op is not None else None
        e0.record()
        for _ in range(n):
            for name, f in table.items():
                if marks is None:
                    f()
                else:
                    a, b = ev(), ev()
                    a.record()
                    f()
                    b.record()
                    marks[name].append((a, b))
        e1.record()
        torch.cuda.synchronize()
        if marks is not None:
            for name, m in marks.items():
                per_op[name] = sum(a.elapsed_time(b) for a, b in m) / len(m)
        return e0.elapsed_time(e1) / n

    def time_op(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # Each call's own duration: serial steps, each call bracketed by HIP events on the stream
    # it launches on (overlapped calls would share the GPU and read slower one by one).
    op_ms = {}
    ms_serial = time_steps(ops, args.steps, args.warmup, op_ms)
    if pL is not None:
        # timed region: K whole steps on three streams: the forward solve, the adjoint's
        # transposed solve, and the two SpMV calls (which depend on neither solve)
        s_adj, s_mv = torch.cuda.Stream(), torch.cuda.Stream()
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

        def ddf_step():
            s0 = torch.cuda.current_stream()
            s_adj.wait_stream(s0)
            s_mv.wait_stream(s0)
            with torch.cuda.stream(s_adj):
                ddf.ddf_sptrsv_adjoint(pL, vL, None, Gx, GB, None, k)
            with torch.cuda.stream(s_mv):
                ops["spmv"]()
                ops["spmv_adj"]()
            ops["sptrsv"]()
            fwd = torch.cuda.Event()
            fwd.record(s0)
            s_adj.wait_event(fwd)
            with torch.cuda.stream(s_adj):
                ddf.ddf_sptrsv_value_grad(pL, Xs, GB, GVL, k)
            s0.wait_stream(s_adj)
            s0.wait_stream(s_mv)

        for _ in range(args.warmup):
            ddf_step()
        torch.cuda.synchronize()
        e0, e1 = ev(), ev()
        e0.record()
        for _ in range(args.steps):
            ddf_step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        log(f"[bench] DDF step {ms:.3f} ms on three streams, {ms_serial:.3f} ms serial")
    else:
        ms = ms_serial
    if pL is not None:
        ddf.ddf_plan_sync_status(pL)
    log(f"[bench] DDF step {ms:.3f} ms")
    ms_plain = time_steps(plain, max(3, args.steps // 4), 1)
    log(f"[bench] plain step {ms_plain:.3f} ms")
    per_op = {}
    for name in ops:
        t = op_ms[name]
        tp = time_op(plain[name], max(2, args.op_reps // 2))
        ba, bc, fl = traffic[name]
        per_op[name] = {"ms": round(t, 4), "gbps_alg": round(ba / t / 1e6, 1), "pct_peak": round(100 * ba / t / 1e6 / PEAK_GBPS, 2),
                        "gbps_csr_equiv": round(bc / t / 1e6, 1), "gflops": round(fl / t / 1e6, 2),
                        "plain_ms": round(tp, 4), "speedup_vs_plain": round(tp / t, 3)}
        log(f"[bench] {name}: {per_op[name]}")

    # parity spot check against the oracle (outside the timed region)
    import oracle as O
    parity = {}
    step(ops)
    torch.cuda.synchronize()
    yref = O.spmv(A, w.X)
    parity["spmv_max_abs_err"] = float(np.max(np.abs(Y.cpu().numpy() - yref)))
    if pL is not None:
        xref = O.sptrsv(L, w.B)
        parity["sptrsv_rel_err"] = float(np.max(np.abs(Xs.cpu().numpy() - xref)) / np.max(np.abs(xref)))

    bytes_step = sum(t[0] for t in traffic.values())
    value = bytes_step / (ms / 1e3) / 1e9
    value_plain = bytes_step / (ms_plain / 1e3) / 1e9
    # the dominant kernel: each call of the step is one main launch (the solves add a small
    # counter reset on the multi-block path)
    info_L = ddf.ddf_plan_info(pL) if pL is not None else {}
    info_A = ddf.ddf_plan_info(pA)
    kernel_of = {"spmv": "k_spmv1" if k == 1 else "k_spmvN", "spmv_adj": "k_spmv1" if k == 1 else "k_spmvN"}
    if pL is not None:
        names = {1: "k_solve", 2: "k_solve_thin", 3: "k_solve_range"}
        kernel_of["sptrsv"] = names[info_L["solve_path"]]
        kernel_of["sptrsv_adj"] = names[info_L["solve_path_adj"]]
    dom = max(per_op, key=lambda n: per_op[n]["ms"])
    kname = kernel_of[dom]
    ach = traffic[dom][0] / (per_op[dom]["ms"] / 1e3) / 1e9
    hbm = traffic_from_profiles(dom, args.workload)
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / PEAK_GBPS, 4),
                "traffic": hbm, "kernel": f"{dom} call (main kernel {kname})", "bytes_alg_per_call": traffic[dom][0]}

    cpu = None
    if not args.no_cpu:
        # the oracle as it stands, single-threaded, on whole steps until ~cpu_seconds elapse
        t0 = time.time()
        nsteps = 0
        while True:
            O.spmv(A, w.X)
            O.spmv_adj(A, w.X, w.Gy)
            if L is not None:
                xr = O.sptrsv(L, w.B)
                O.sptrsv_adj(L, xr, w.Gx)
            nsteps += 1
            if time.time() - t0 > args.cpu_seconds:
                break
        cpu_s = (time.time() - t0) / nsteps
        cpu = {"value": round(bytes_step / cpu_s / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{nsteps} whole steps of {w.name} (SpMV fwd+adj, SpTRSV fwd+adj), "
                         f"{cpu_s * 1e3:.1f} ms/step, single-threaded plain C loops"}
        log(f"[bench] cpu oracle {cpu_s * 1e3:.1f} ms/step")

    out = {
        "metric": "SpMV/SpTRSV fwd+adjoint effective HBM GB/s and % of peak vs plain, FP64",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic", "ms_per_step_serial": round(ms_serial, 4),
        "config": {"workload": w.name, "n": A.n_rows, "nnz_A": A.nnz, "nnz_L": L.nnz if L is not None else 0,
                   "levels": info_L.get("n_parts", 0), "nrhs": k,
                   "solve_kernel": {"fwd": kernel_of.get("sptrsv"), "adj": kernel_of.get("sptrsv_adj")},
                   "codelets_A_by_type": info_A["codelets_by_type"], "ops_A_by_type": info_A["ops_by_type"],
                   "codelets_L_by_type": info_L.get("codelets_by_type"),
                   "inspect_s": {"A": round(tA, 3), "L": round(tL, 3)}},
        "pct_of_peak": round(100 * value / PEAK_GBPS, 2),
        # the plain calls run one after the other: compared with the DDF calls run the same way
        "plain": {"ms_per_step": round(ms_plain, 4), "value": round(value_plain, 2),
                  "speedup_vs_plain": round(ms_plain / ms_serial, 3), "serial": True},
        "per_op": per_op, "bytes_alg_per_step": bytes_step, "parity": parity,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_batch(args, np, torch, ddf, I, dev):
    """The batched solve and its adjoint on C4, one persistent launch each."""
    import oracle as O
    t0 = time.time()
    w = I.workload("c4")
    mats = [m["L"] for m in w.batch]
    ks = [m["k"] for m in w.batch]
    log(f"[bench] workload {w.name} generated in {time.time() - t0:.1f}s")
    t0 = time.time()
    p = ddf.ddf_inspect_batch(ddf.DDF_SPTRSV_LOWER, mats, ks)
    t_insp = time.time() - t0
    log(f"[bench] inspect {t_insp:.2f}s")

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    vals = d(np.concatenate([m.values for m in mats]))
    B = d(np.concatenate([m["B"].ravel() for m in w.batch]))
    G = d(np.concatenate([m["G"].ravel() for m in w.batch]))
    X, GB, GV = torch.empty_like(B), torch.empty_like(B), torch.empty_like(vals)
    ops = {"sptrsv_batch": lambda: ddf.ddf_sptrsv_batch(p, vals, B, X),
           "sptrsv_batch_adj": lambda: ddf.ddf_sptrsv_batch_adjoint(p, vals, X, G, GB, GV)}
    if args.profile_op:
        for name in args.profile_op.split(","):
            for _ in range(args.steps):
                ops[name]()
            torch.cuda.synchronize()
            log(f"[bench] ran {name} x{args.steps}")
        return

    def ev():
        return torch.cuda.Event(enable_timing=True)

    for _ in range(args.warmup):
        for f in ops.values():
            f()
    torch.cuda.synchronize()
    marks = {n: [] for n in ops}
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(args.steps):
        for n, f in ops.items():
            a, b = ev(), ev()
            a.record()
            f()
            b.record()
            marks[n].append((a, b))
    e1.record()
    torch.cuda.synchronize()
    ddf.ddf_plan_sync_status(p)
    ms = e0.elapsed_time(e1) / args.steps
    op_ms = {n: sum(a.elapsed_time(b) for a, b in m) / len(m) for n, m in marks.items()}
    log(f"[bench] batch step {ms:.3f} ms {op_ms}")
    # comparator: the same solve, one launch per matrix
    ddf.ddf_sptrsv_batch_per_matrix(p, vals, B, X)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    for _ in range(2):
        ddf.ddf_sptrsv_batch_per_matrix(p, vals, B, X)
    b.record()
    torch.cuda.synchronize()
    per_matrix_ms = a.elapsed_time(b) / 2
    # graph replay of the forward launch
    g = ddf.ddf_graph_create_batch(p, 0, vals, B, None, X, None)
    ddf.ddf_graph_launch(g)
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    for _ in range(3):
        ddf.ddf_graph_launch(g)
    b.record()
    torch.cuda.synchronize()
    graph_ms = a.elapsed_time(b) / 3
    ddf.ddf_graph_destroy(g)

    traffic = {"sptrsv_batch": ddf.ddf_plan_traffic(p, ddf.DDF_OP_SPTRSV, 1),
               "sptrsv_batch_adj": ddf.ddf_plan_traffic(p, ddf.DDF_OP_SPTRSV_ADJ, 1)}
    bytes_step = sum(t[0] for t in traffic.values())
    value = bytes_step / (ms / 1e3) / 1e9
    per_op = {n: {"ms": round(op_ms[n], 4), "gbps_alg": round(traffic[n][0] / op_ms[n] / 1e6, 1),
                  "pct_peak": round(100 * traffic[n][0] / op_ms[n] / 1e6 / PEAK_GBPS, 2)} for n in ops}
    per_op["sptrsv_batch"]["plain_ms"] = round(per_matrix_ms, 4)
    per_op["sptrsv_batch"]["speedup_vs_plain"] = round(per_matrix_ms / op_ms["sptrsv_batch"], 3)
    per_op["sptrsv_batch"]["graph_replay_ms"] = round(graph_ms, 4)

    # parity spot check: a few matrices against the oracle
    ddf.ddf_sptrsv_batch(p, vals, B, X)
    torch.cuda.synchronize()
    xh = X.cpu().numpy()
    rel, off = 0.0, 0
    for m in w.batch:
        n, k = m["L"].n_rows, m["k"]
        if len(mats) < 8 or m is w.batch[0] or m is w.batch[-1]:
            ref = O.sptrsv(m["L"], m["B"])
            got = xh[off:off + n * k].reshape(n, k)
            rel = max(rel, float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300)))
        off += n * k
    dom = max(per_op, key=lambda n: per_op[n]["ms"])
    ach = traffic[dom][0] / (op_ms[dom] / 1e3) / 1e9
    binfo = ddf.ddf_plan_info(p)
    bkey = "solve_path_adj" if dom.endswith("adj") else "solve_path"
    bnames = {1: "k_solve", 2: "k_solve_thin", 3: "k_solve_range"}
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / PEAK_GBPS, 4), "traffic": None,
                "kernel": f"{dom} call (main kernel {bnames.get(binfo.get(bkey), 'k_solve')})",
                "bytes_alg_per_call": traffic[dom][0]}
    cpu = None
    if not args.no_cpu:
        t0 = time.time()
        done = 0
        for m in w.batch:
            xr = O.sptrsv(m["L"], m["B"])
            O.sptrsv_adj(m["L"], xr, m["G"])
            done += 1
            if time.time() - t0 > args.cpu_seconds:
                break
        cpu_s = time.time() - t0
        frac_rows = sum(m["L"].n_rows for m in w.batch[:done]) / sum(m.n_rows for m in mats)
        cpu_step = cpu_s / frac_rows
        cpu = {"value": round(bytes_step / cpu_step / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {done} of {len(mats)} matrices (solve and adjoint), {cpu_s:.1f} s, "
                         f"scaled by their share of the rows to {cpu_step * 1e3:.0f} ms per step"}
    out = {
        "metric": "SpMV/SpTRSV fwd+adjoint effective HBM GB/s and % of peak vs plain, FP64",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "matrices": len(mats), "rows": sum(m.n_rows for m in mats),
                   "nnz_L": sum(m.nnz for m in mats), "nrhs_range": [min(ks), max(ks)],
                   "max_levels": ddf.ddf_plan_info(p)["max_levels"], "inspect_s": round(t_insp, 3)},
        "pct_of_peak": round(100 * value / PEAK_GBPS, 2),
        "per_op": per_op, "bytes_alg_per_step": bytes_step, "parity": {"sptrsv_rel_err": rel},
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
