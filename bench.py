"""Benchmark of the DDF hot path on one MI355X.

One step = SpMV forward, SpMV adjoint (A^T g and dA), SpTRSV forward and SpTRSV adjoint
(L^T lambda = g and dL) on one synthetic workload, FP64, inputs resident in HBM, the calls one
after the other on one stream.  Protocol: W untimed warm-up steps, then K timed steps; before
each timed step 1 GiB of scratch is overwritten (untimed) so that neither the 256 MB
Infinity Cache nor the L2s hold the step's data; each step and each call is bracketed by HIP
events on the stream the calls launch on; medians are reported.

The value is whole-step effective HBM bandwidth: the algorithmic bytes of the four calls
(values, plan tables, vectors read once and written once; see ddf_plan_traffic) over the
median step time.  The roofline covers the dominant kernel (the main kernel of the slowest
call): its algorithmic bytes per launch over its own duration, measured with HIP events that
the library records around that kernel.  The plain GPU comparators (CSR-vector SpMV,
FP64-atomic adjoint, one launch per level) are timed the same way.  The CPU baseline is the
oracle on whole steps of the same workload, single-threaded and on every host core (OpenMP
over independent rows), and its outputs check the GPU's (parity).

    python bench.py [--steps K] [--warmup W] [--workload c5|c2|c3|c1|c4] [--tsync]

The default workload is the 27-point Laplacian on 170^3 with 8 right-hand sides (the largest
single-GPU configuration).  With --workload c4 (256 triangular matrices with 1..32 right-hand
sides each) a step is the batched solve and its adjoint; the comparator is one launch per
matrix.  --tsync measures the dependent-hop latency of the solve kernels on a bidiagonal chain.
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
FLUSH_BYTES = 1 << 30
METRIC = "SpMV/SpTRSV fwd+adjoint effective HBM GB/s and % of peak vs plain, FP64"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--profile-op", default="", help="run only these ops K times each (for rocprofv3)")
    ap.add_argument("--tsync", action="store_true", help="dependent-hop latency of the solve kernels")
    ap.add_argument("--ablation", action="store_true",
                    help="BLAS-only ablation: full plans against column-slice plans on the workload")
    ap.add_argument("--cost-model", action="store_true",
                    help="Eq. (1) plan cost against measured SpMV kernel time over a family of patterns")
    return ap.parse_args()


# ddf_inspect's phases (ddf_plan_info_t.phase_seconds)
PHASES = ["alg1_forward", "adjoint_plan", "packing", "single_block_records", "schedules_uploads"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def kernels_sha():
    """Digest of the library's sources (kernels and the schedules that drive them)."""
    d = os.path.join(ROOT, "paper_2111_12243_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".cpp", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:12]


def profile_value(name, key):
    """A figure from a committed profile summary, when it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"sources_sha:\s*(\w+)", txt)
    m = re.search(re.escape(key) + r":\s*([0-9.eE+-]+)", txt)
    if not m_sha or not m or m_sha.group(1) != kernels_sha():
        return None
    return float(m.group(1))


class Timer:
    """K timed reps of a table of calls: a flush before each rep, HIP events around the rep
    and around each call, on the current stream."""

    def __init__(self, torch, dev):
        self.torch = torch
        self.flush_buf = torch.empty(FLUSH_BYTES // 8, dtype=torch.float64, device=dev)

    def flush(self):
        self.flush_buf.fill_(1.0)

    def run(self, table, reps, warm):
        torch = self.torch
        for _ in range(warm):
            for f in table.values():
                f()
        torch.cuda.synchronize()
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        steps, marks = [], {n: [] for n in table}
        for _ in range(reps):
            self.flush()
            s0, s1 = ev(), ev()
            s0.record()
            for name, f in table.items():
                a, b = ev(), ev()
                a.record()
                f()
                b.record()
                marks[name].append((a, b))
            s1.record()
            steps.append((s0, s1))
        torch.cuda.synchronize()
        step_ms = [a.elapsed_time(b) for a, b in steps]
        op_ms = {n: [a.elapsed_time(b) for a, b in m] for n, m in marks.items()}
        return step_ms, op_ms


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
    if args.tsync:
        return bench_tsync(args, np, torch, ddf, I, dev)
    if args.cost_model:
        return bench_cost_model(args, np, torch, ddf, I, dev)
    if args.ablation:
        return bench_ablation(args, np, torch, ddf, I, dev)
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
    ops = {
        "spmv": lambda: ddf.ddf_spmv_v(pA, vA, X, Y, k),
        "spmv_adj": lambda: ddf.ddf_spmv_adjoint(pA, vA, X, Gy, GX, GVA, k),
    }
    plain = {
        "spmv": lambda: ddf.ddf_plain_spmv(pA, vA, X, Y, k),
        "spmv_adj": lambda: ddf.ddf_plain_spmv_adjoint(pA, vA, X, Gy, GX, GVA, k),
    }
    plan_of = {"spmv": pA, "spmv_adj": pA}
    if pL is not None:
        vL, Bv, Gx = d(L.values), d(w.B), d(w.Gx)
        Xs = torch.empty_like(Bv)
        GB = torch.empty_like(Bv)
        GVL = torch.empty(L.nnz, dtype=torch.float64, device=dev)
        ops["sptrsv"] = lambda: ddf.ddf_sptrsv_v(pL, vL, Bv, Xs, k)
        ops["sptrsv_adj"] = lambda: ddf.ddf_sptrsv_adjoint(pL, vL, Xs, Gx, GB, GVL, k)
        plain["sptrsv"] = lambda: ddf.ddf_plain_sptrsv(pL, vL, Bv, Xs, k)
        plain["sptrsv_adj"] = lambda: ddf.ddf_plain_sptrsv_adjoint(pL, vL, Xs, Gx, GB, GVL, k)
        plan_of["sptrsv"] = plan_of["sptrsv_adj"] = pL

    if not args.no_tune:
        t0 = time.time()
        ddf.ddf_autotune(pA, ddf.DDF_OP_SPMV, k, budget_ms=1500)
        ddf.ddf_autotune(pA, ddf.DDF_OP_SPMV_ADJ, k, budget_ms=1500)
        if pL is not None:
            ddf.ddf_autotune(pL, ddf.DDF_OP_SPTRSV, k, budget_ms=3000)
            ddf.ddf_autotune(pL, ddf.DDF_OP_SPTRSV_ADJ, k, budget_ms=3000)
        torch.cuda.synchronize()
        log(f"[bench] autotune {time.time() - t0:.1f}s")

    opcode = {"spmv": ddf.DDF_OP_SPMV, "spmv_adj": ddf.DDF_OP_SPMV_ADJ, "sptrsv": ddf.DDF_OP_SPTRSV,
              "sptrsv_adj": ddf.DDF_OP_SPTRSV_ADJ}
    traffic = {n: ddf.ddf_plan_traffic(plan_of[n], opcode[n], k) for n in ops}

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

    timer = Timer(torch, dev)
    step_ms, op_ms_all = timer.run(ops, args.steps, args.warmup)
    ms = median(step_ms)
    op_ms = {n: median(v) for n, v in op_ms_all.items()}
    if pL is not None:
        ddf.ddf_plan_sync_status(pL)
    log(f"[bench] DDF step {ms:.3f} ms (median of {args.steps}; min {min(step_ms):.3f}, max {max(step_ms):.3f})")
    plain_steps, plain_ops_all = timer.run(plain, args.plain_steps, 1)
    ms_plain = median(plain_steps)
    plain_ops = {n: median(v) for n, v in plain_ops_all.items()}
    log(f"[bench] plain step {ms_plain:.3f} ms")

    # the dominant kernel: the main kernel of the slowest call, timed by itself with the events
    # the library records around it (same flush protocol, same stream)
    dom = max(op_ms, key=lambda n: op_ms[n])
    pdom = plan_of[dom]
    ker_ms = []
    for _ in range(args.steps):
        timer.flush()
        ddf.ddf_plan_time_kernels(pdom, 1)
        ops[dom]()
        kms, calls, launches = ddf.ddf_plan_kernel_time(pdom)
        ker_ms.append(kms / max(calls, 1))
    ddf.ddf_plan_time_kernels(pdom, 0)
    kernel_ms = median(ker_ms)
    per_op = {}
    for name in ops:
        t = op_ms[name]
        ba, bc, fl = traffic[name]
        per_op[name] = {"ms": round(t, 4), "gbps_alg": round(ba / t / 1e6, 1),
                        "pct_peak": round(100 * ba / t / 1e6 / PEAK_GBPS, 2),
                        "gbps_csr_equiv": round(bc / t / 1e6, 1), "gflops": round(fl / t / 1e6, 2),
                        "bytes_alg": ba, "plain_ms": round(plain_ops[name], 4),
                        "speedup_vs_plain": round(plain_ops[name] / t, 3)}
        log(f"[bench] {name}: {per_op[name]}")

    info_L = ddf.ddf_plan_info(pL) if pL is not None else {}
    info_A = ddf.ddf_plan_info(pA)
    names = {1: "k_solve_df", 2: "k_solve_thin", 3: "k_solve_range"}
    kernel_of = {"spmv": "k_spmv1" if k == 1 else "k_spmvN", "spmv_adj": "k_spmv1" if k == 1 else "k_spmvN"}
    if pL is not None:
        kernel_of["sptrsv"] = names[info_L["solve_path"]]
        kernel_of["sptrsv_adj"] = names[info_L["solve_path_adj"]]
    # algorithmic bytes of the dominant call's main kernel (the adjoints' value gradient and value
    # gather run in kernels of their own)
    kop = {"spmv": ddf.DDF_OP_SPMV, "spmv_adj": ddf.DDF_OP_SPMV_ADJ_KERNEL, "sptrsv": ddf.DDF_OP_SPTRSV,
           "sptrsv_adj": ddf.DDF_OP_SPTRSV_ADJ_KERNEL}[dom]
    ba_dom = ddf.ddf_plan_traffic(pdom, kop, k)[0]
    ach = ba_dom / (kernel_ms / 1e3) / 1e9
    wl = args.workload
    # HBM bytes per launch of the dominant kernel, from the committed counter summary of this
    # call (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), when taken on these sources
    fetch = profile_value(f"traffic_{dom}_{wl}.md", f"hbm_bytes_per_launch_{kernel_of[dom]}")
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / PEAK_GBPS, 4), "traffic": fetch,
                "kernel": kernel_of[dom], "call": dom, "kernel_ms": round(kernel_ms, 4),
                "bytes_alg_per_launch": ba_dom}
    if dom.startswith("sptrsv"):
        # two-term bound of a level-ordered solve: t >= max(bytes / peak, levels x t_sync), with
        # t_sync the measured latency of one dependent hop of this kernel (bench.py --tsync)
        tsync = profile_value("tsync.md", f"{kernel_of[dom]}_k{1 if k <= 2 else 8}_us_per_hop")
        nlev = int(info_L["n_parts"])
        roofline["levels"] = nlev
        roofline["t_sync_us"] = tsync
        if tsync:
            floor_ms = max(ba_dom / PEAK_GBPS / 1e6, nlev * tsync / 1e3)
            roofline["two_term_floor_ms"] = round(floor_ms, 4)
            roofline["frac_of_two_term_floor"] = round(floor_ms / kernel_ms, 4)

    # inspector cost and its amortisation (Sec. V-C): NER = inspector time over the time one
    # executor run saves against the plain kernel; the inspector time includes the device
    # tables' upload (ddf_inspect's wall time, both plans of a pattern for the forward and
    # adjoint calls)
    t_insp = {"spmv": tA, "spmv_adj": tA, "sptrsv": tL, "sptrsv_adj": tL}
    ner = {n: (round(t_insp[n] * 1e3 / (plain_ops[n] - op_ms[n]), 1) if plain_ops[n] > op_ms[n] else None)
           for n in ops}
    bytes_step = sum(t[0] for t in traffic.values())
    value = bytes_step / (ms / 1e3) / 1e9
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args, np, w, A, L, bytes_step, {
            "spmv": Y, "spmv_adj": (GX, GVA), "sptrsv": Xs if pL is not None else None,
            "sptrsv_adj": (GB, GVL) if pL is not None else None}, ops)

    out = {
        "metric": METRIC,
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n": A.n_rows, "nnz_A": A.nnz, "nnz_L": L.nnz if L is not None else 0,
                   "levels": info_L.get("n_parts", 0), "nrhs": k,
                   "solve_kernel": {"fwd": kernel_of.get("sptrsv"), "adj": kernel_of.get("sptrsv_adj")},
                   "codelets_A_by_type": info_A["codelets_by_type"], "ops_A_by_type": info_A["ops_by_type"],
                   "codelets_L_by_type": info_L.get("codelets_by_type"), "ops_L_by_type": info_L.get("ops_by_type"),
                   "inspect_s": {"A": round(tA, 3), "L": round(tL, 3)}, "ner": ner,
                   "inspect_phases_s": {"A": [round(v, 3) for v in info_A["phase_seconds"]],
                                        "L": [round(v, 3) for v in info_L["phase_seconds"]] if info_L else None,
                                        "phases": PHASES},
                   "timing": "median of K steps, 1 GiB written between steps, one stream"},
        "pct_of_peak": round(100 * value / PEAK_GBPS, 2),
        "plain": {"ms_per_step": round(ms_plain, 4), "value": round(bytes_step / (ms_plain / 1e3) / 1e9, 2),
                  "speedup_vs_plain": round(ms_plain / ms, 3)},
        "per_op": per_op, "bytes_alg_per_step": bytes_step,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(args, np, w, A, L, bytes_step, gpu_out, ops):
    """The oracle on whole steps of the workload: single-threaded, then on every host core
    (OpenMP over independent rows); each for about --cpu-seconds.  Its outputs on the same
    inputs check the GPU's outputs (the error measures of the parity tests)."""
    import oracle as O

    def serial_step():
        y = O.spmv(A, w.X)
        gx, gv = O.spmv_adj(A, w.X, w.Gy)
        out = {"spmv": y, "spmv_adj": (gx, gv)}
        if L is not None:
            x = O.sptrsv(L, w.B)
            out["sptrsv"] = x
            out["sptrsv_adj"] = O.sptrsv_adj(L, x, w.Gx)
        return out

    def timed(step):
        t0 = time.time()
        n, out = 0, None
        while True:
            out = step()
            n += 1
            if time.time() - t0 > args.cpu_seconds:
                break
        return (time.time() - t0) / n, n, out

    s1, n1, ref = timed(serial_step)
    log(f"[bench] cpu oracle, 1 core: {s1 * 1e3:.1f} ms/step ({n1} steps)")
    mA = O.ManyCore(A)
    mL = O.ManyCore(L, triangular=True) if L is not None else None

    def many_step():
        mA.spmv(w.X)
        mA.spmv_adj(w.X, w.Gy)
        if mL is not None:
            x = mL.sptrsv(w.B)
            mL.sptrsv_adj(x, w.Gx)

    sN, nN, _ = timed(many_step)
    cores = O.omp_threads()
    log(f"[bench] cpu oracle, {cores} threads: {sN * 1e3:.1f} ms/step ({nN} steps)")

    # parity of the GPU outputs of the last timed step (same inputs) against the oracle's
    def rel_prod(M, Xin, got, want):
        from types import SimpleNamespace
        absM = SimpleNamespace(n_rows=M.n_rows, n_cols=M.n_cols, row_ptr=M.row_ptr, col_idx=M.col_idx,
                               values=np.abs(M.values))
        scale = O.spmv(absM, np.abs(Xin))
        nz = scale > 0
        return float(np.max(np.abs(got - want)[nz] / scale[nz])) if nz.any() else 0.0

    def rel_norm(got, want):
        return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))

    for f in ops.values():  # the GPU outputs of one step on the same inputs
        f()
    import torch
    torch.cuda.synchronize()
    parity = {"spmv_elementwise": rel_prod(A, w.X, gpu_out["spmv"].cpu().numpy(), ref["spmv"])}
    AT, _ = O.transpose(A)
    parity["spmv_adj_gx_elementwise"] = rel_prod(AT, w.Gy, gpu_out["spmv_adj"][0].cpu().numpy(), ref["spmv_adj"][0])
    parity["spmv_adj_gv_normwise"] = rel_norm(gpu_out["spmv_adj"][1].cpu().numpy(), ref["spmv_adj"][1])
    if L is not None:
        parity["sptrsv_normwise"] = rel_norm(gpu_out["sptrsv"].cpu().numpy(), ref["sptrsv"])
        parity["sptrsv_adj_lambda_normwise"] = rel_norm(gpu_out["sptrsv_adj"][0].cpu().numpy(), ref["sptrsv_adj"][0])
        parity["sptrsv_adj_gv_normwise"] = rel_norm(gpu_out["sptrsv_adj"][1].cpu().numpy(), ref["sptrsv_adj"][1])
    parity = {kk: float(f"{v:.3e}") for kk, v in parity.items()}
    log(f"[bench] parity against the oracle: {parity}")
    return {"value": round(bytes_step / sN / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "ms_per_step": round(sN * 1e3, 1),
            "sample": f"{nN} whole steps of {w.name} (SpMV fwd+adj, SpTRSV fwd+adj), plain C loops, "
                      f"OpenMP over independent rows on {cores} threads",
            "single_core": {"value": round(bytes_step / s1 / 1e9, 3), "cores": 1, "ms_per_step": round(s1 * 1e3, 1),
                            "sample": f"{n1} whole steps, the serial oracle"},
            "parity": parity}


def bench_tsync(args, np, torch, ddf, I, dev):
    """Latency of one dependent hop of each solve kernel: a bidiagonal chain of n rows (n levels
    of one row each) solved by the dataflow kernel, the single-block kernel and one launch per
    level; microseconds per level (the t_sync of the two-term solve bound)."""
    out = {}
    for name, path, n, k in (("k_solve_df", 1, 50000, 1), ("k_solve_df", 1, 50000, 8), ("k_solve_thin", 2, 50000, 1),
                             ("k_solve_range", 3, 5000, 1), ("k_solve_range", 3, 5000, 8)):
        rows = np.concatenate([np.arange(1, n), np.arange(n)])
        cols = np.concatenate([np.arange(n - 1), np.arange(n)])
        L = I.csr_from_pairs(n, n, rows, cols, np.random.default_rng(1).uniform(1, 2, rows.size))
        p = ddf.ddf_inspect(1, L, ddf.ddf_opts_default(solve_path=path, build_adjoint=0))
        assert ddf.ddf_plan_info(p)["solve_path"] == path
        b = torch.from_numpy(np.random.default_rng(2).uniform(-1, 1, (n, k))).to(dev)
        x = torch.empty_like(b)
        ts = []
        for _ in range(args.warmup + 5):
            ddf.ddf_plan_time_kernels(p, 1)
            ddf.ddf_sptrsv(p, b, x, k)
            kms, _, _ = ddf.ddf_plan_kernel_time(p)
            ts.append(kms)
        ddf.ddf_plan_time_kernels(p, 0)
        ddf.ddf_plan_sync_status(p)
        us = median(ts[args.warmup:]) * 1e3 / n
        out[f"{name}_k{k}_us_per_hop"] = round(us, 4)
        log(f"[bench] {name}, {k} right-hand side(s): {us:.3f} us per dependent level ({n} levels)")
    out["sources_sha"] = kernels_sha()
    print(json.dumps(out), flush=True)


def cost_model_patterns(np, I):
    """A family of seeded sparse patterns of about 2-8M stored entries: stencils of several
    shapes, banded matrices with gaps, random rows of column runs, power-law rows, and random
    scattered columns (the plan's codelet mix goes from all-BLAS to all-PSC II)."""
    pats = []
    for nx in (160, 224):
        pats.append((f"5pt_{nx}^2", I.laplacian(nx * 4, nx, 1, I.OFFS_5PT, 4.0)))
    for nx in (60, 80):
        pats.append((f"27pt_{nx}^3", I.laplacian(nx, nx, nx, I.OFFS_27PT, 26.0)))
    offs7 = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    pats.append(("7pt_100^3", I.laplacian(100, 100, 100, offs7, 6.0)))
    for b, n in ((1, 1 << 20), (4, 1 << 19), (16, 1 << 18)):
        # band of 2b + 1 diagonals
        rows = np.repeat(np.arange(n), 2 * b + 1)
        cols = rows + np.tile(np.arange(-b, b + 1), n)
        ok = (cols >= 0) & (cols < n)
        pats.append((f"band{2 * b + 1}_{n}", I.csr_from_pairs(n, n, rows[ok], cols[ok], np.ones(int(ok.sum())))))
    for gap, n in ((3, 1 << 19), (7, 1 << 19)):
        # strided rows: columns i, i + gap, i + 2 gap, ... (PSC I with a shared table)
        rows = np.repeat(np.arange(n), 6)
        cols = (rows + np.tile(np.arange(6) * gap * np.arange(1, 7), n)) % n
        pats.append((f"gap{gap}_{n}", I.csr_from_pairs(n, n, rows, cols, np.ones(rows.size))))
    def unique_pairs(n, rows, cols):
        key = np.unique(rows.astype(np.int64) * n + cols)
        return I.csr_from_pairs(n, n, key // n, key % n, np.ones(key.size))

    for seed, n, d in ((1, 400000, 4), (2, 300000, 12)):
        # d random columns per row
        rng = np.random.default_rng(900 + seed)
        rows = np.repeat(np.arange(n), d)
        pats.append((f"random{d}_{n}", unique_pairs(n, rows, rng.integers(0, n, rows.size))))
    for seed, n, ln in ((3, 300000, 4), (4, 300000, 12)):
        # two runs of ln consecutive columns per row, at random places
        rng = np.random.default_rng(900 + seed)
        starts = rng.integers(0, n - ln, (n, 2))
        rows = np.repeat(np.arange(n), 2 * ln)
        cols = (starts[:, :, None] + np.arange(ln)[None, None, :]).reshape(-1)
        pats.append((f"runs{ln}_{n}", unique_pairs(n, rows, cols)))
    for n in (300000, 600000):
        pats.append((f"chunglu_{n}", I.c3_chung_lu(n=n).A))
    return pats


def bench_ablation(args, np, torch, ddf, I, dev):
    """The BLAS-only ablation (Sec. V-A for SpMV, V-B for SpTRSV): the workload's forward SpMV
    and forward solve with the full inspector's plan against the plan whose windows are covered
    by BLAS codelets only (column slices of rows, partial sums combined with FP64 atomics).  The
    solve's slices run one launch per level, so the full plan's one-launch-per-level solve is
    timed too: that ratio holds the executor fixed and isolates the codelet types.  Same timing
    protocol as the main bench (flush, HIP events, medians)."""
    w = I.workload(args.workload)
    k, A, L = w.k, w.A, w.L
    log(f"[ablation] workload {w.name}, k={k}")

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

    plans, tinsp = {}, {}
    cases = [("spmv_ddf", 0, A, 0, 0), ("spmv_blas_only", 0, A, 1, 0)]
    if L is not None:
        cases += [("sptrsv_ddf", 1, L, 0, 0), ("sptrsv_ddf_level", 1, L, 0, 3), ("sptrsv_blas_only", 1, L, 1, 0)]
    for name, kind, M, ob, path in cases:
        t0 = time.time()
        plans[name] = ddf.ddf_inspect(kind, M, ddf.ddf_opts_default(only_blas=ob, build_adjoint=0, solve_path=path))
        tinsp[name] = round(time.time() - t0, 3)
        log(f"[ablation] {name}: inspect {tinsp[name]}s")
    vA, X = d(A.values), d(w.X)
    vL, B = (d(L.values), d(w.B)) if L is not None else (None, None)
    out = {n: torch.empty((A.n_rows if n.startswith("spmv") else L.n_rows, k), dtype=torch.float64, device=dev)
           for n in plans}
    ops = {n: (lambda n=n: ddf.ddf_spmv_v(plans[n], vA, X, out[n], k)) if n.startswith("spmv")
           else (lambda n=n: ddf.ddf_sptrsv_v(plans[n], vL, B, out[n], k)) for n in plans}
    timer = Timer(torch, dev)
    _, op_all = timer.run(ops, args.steps, args.warmup)
    ms = {n: median(v) for n, v in op_all.items()}
    for n in ms:
        log(f"[ablation] {n}: {ms[n]:.4f} ms")

    def rel(a, b):
        a, b = out[a].cpu().numpy(), out[b].cpu().numpy()
        return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))

    def cods(n):
        i = ddf.ddf_plan_info(plans[n])
        return {"codelets": int(i["n_codelets"]), "by_type": [int(v) for v in i["codelets_by_type"]],
                "plan_bytes": int(i["dev_plan_bytes"]), "inspect_s": tinsp[n]}

    res = {
        "metric": "blas_only_ablation", "workload": w.name, "nrhs": k, "steps": args.steps,
        "spmv": {"ddf_ms": round(ms["spmv_ddf"], 4), "blas_only_ms": round(ms["spmv_blas_only"], 4),
                 "ratio": round(ms["spmv_blas_only"] / ms["spmv_ddf"], 3), "paper_ratio": 10.0,
                 "max_rel_diff": rel("spmv_blas_only", "spmv_ddf"),
                 "ddf": cods("spmv_ddf"), "blas_only": cods("spmv_blas_only")},
        "sptrsv": None if L is None else {
            "ddf_ms": round(ms["sptrsv_ddf"], 4), "ddf_level_ms": round(ms["sptrsv_ddf_level"], 4),
            "blas_only_ms": round(ms["sptrsv_blas_only"], 4),
            "ratio": round(ms["sptrsv_blas_only"] / ms["sptrsv_ddf"], 3),
            "ratio_same_executor": round(ms["sptrsv_blas_only"] / ms["sptrsv_ddf_level"], 3),
            "paper_ratio": 3.9, "max_rel_diff": rel("sptrsv_blas_only", "sptrsv_ddf"),
            "ddf": cods("sptrsv_ddf"), "blas_only": cods("sptrsv_blas_only")},
        "timing": "median of K steps, 1 GiB written between steps, one stream",
    }
    print(json.dumps(res), flush=True)


def bench_cost_model(args, np, torch, ddf, I, dev):
    """The cost model of Eq. (1) against the GPU (the analogue of the paper's Fig. 5, which
    fits measured codelet time against the model): per pattern the summed Eq. (1) cost of the
    SpMV plan and the measured time of its SpMV kernel (one right-hand side, median of K with
    a 1 GiB flush before each), then a least-squares line time = a cost + b and its r^2, beside
    the same fit against the stored-entry count."""
    timer = Timer(torch, dev)
    pts = []
    for name, A in cost_model_patterns(np, I):
        p = ddf.ddf_inspect(ddf.DDF_SPMV, A, ddf.ddf_opts_default(build_adjoint=0))
        cod = ddf.ddf_plan_export(p, 0)["codelets"]
        cost = int(cod[:, 17].sum())
        x = torch.from_numpy(np.random.default_rng(5).uniform(-1, 1, (A.n_cols, 1))).to(dev)
        y = torch.empty((A.n_rows, 1), dtype=torch.float64, device=dev)
        ker = []
        for _ in range(args.steps):
            timer.flush()
            ddf.ddf_plan_time_kernels(p, 1)
            ddf.ddf_spmv(p, x, y, 1)
            kms, calls, _ = ddf.ddf_plan_kernel_time(p)
            ker.append(kms / max(calls, 1))
        t = median(ker) * 1e3
        share = [int(v) for v in np.bincount(cod[:, 0], weights=cod[:, 7], minlength=3)]
        pts.append({"pattern": name, "nnz": A.nnz, "eq1_cost": cost, "us": round(t, 2), "ops_by_type": share})
        log(f"[bench] {name}: nnz {A.nnz} cost {cost} {t:.1f} us ops by type {share}")
        del p

    def fit(xs, ys):
        xs, ys = np.asarray(xs, float), np.asarray(ys, float)
        a, b = np.polyfit(xs, ys, 1)
        r = ys - (a * xs + b)
        return a, b, 1.0 - float(r @ r) / float(((ys - ys.mean()) ** 2).sum())

    us = [q["us"] for q in pts]
    a, b, r2 = fit([q["eq1_cost"] for q in pts], us)
    a2, b2, r2n = fit([q["nnz"] for q in pts], us)
    print(json.dumps({"points": pts, "fit_eq1": {"us_per_cost_unit": a, "us0": b, "r2": round(r2, 4)},
                      "fit_nnz": {"us_per_entry": a2, "us0": b2, "r2": round(r2n, 4)},
                      "sources_sha": kernels_sha()}), flush=True)


def bench_batch(args, np, torch, ddf, I, dev):
    """The batched solve and its adjoint on the batch workload (256 matrices, 1..32 right-hand sides)."""
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
    if not args.no_tune:
        ddf.ddf_autotune(p, ddf.DDF_OP_SPTRSV, 1, budget_ms=4000)
        ddf.ddf_autotune(p, ddf.DDF_OP_SPTRSV_ADJ, 1, budget_ms=4000)
    ops = {"sptrsv_batch": lambda: ddf.ddf_sptrsv_batch(p, vals, B, X),
           "sptrsv_batch_adj": lambda: ddf.ddf_sptrsv_batch_adjoint(p, vals, X, G, GB, GV)}
    if args.profile_op:
        # a leg per name, as in the single-matrix bench: "copy" calibrates the counters, and a
        # one-element fill ends each leg
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
    timer = Timer(torch, dev)
    step_ms, op_all = timer.run(ops, args.steps, args.warmup)
    ddf.ddf_plan_sync_status(p)
    ms = median(step_ms)
    op_ms = {n: median(v) for n, v in op_all.items()}
    log(f"[bench] batch step {ms:.3f} ms {op_ms}")
    pm_steps, _ = timer.run({"pm": lambda: ddf.ddf_sptrsv_batch_per_matrix(p, vals, B, X)}, 2, 1)
    per_matrix_ms = median(pm_steps)
    # graph replay of the forward and the adjoint launch
    graph_ms = {}
    for adj, name in ((0, "sptrsv_batch"), (1, "sptrsv_batch_adj")):
        g = (ddf.ddf_graph_create_batch(p, 1, vals, G, X, GB, GV) if adj
             else ddf.ddf_graph_create_batch(p, 0, vals, B, None, X, None))
        gs, _ = timer.run({"g": lambda: ddf.ddf_graph_launch(g)}, 3, 1)
        graph_ms[name] = median(gs)
        ddf.ddf_graph_destroy(g)
    traffic = {"sptrsv_batch": ddf.ddf_plan_traffic(p, ddf.DDF_OP_SPTRSV, 1),
               "sptrsv_batch_adj": ddf.ddf_plan_traffic(p, ddf.DDF_OP_SPTRSV_ADJ, 1)}
    bytes_step = sum(t[0] for t in traffic.values())
    value = bytes_step / (ms / 1e3) / 1e9
    per_op = {n: {"ms": round(op_ms[n], 4), "gbps_alg": round(traffic[n][0] / op_ms[n] / 1e6, 1),
                  "pct_peak": round(100 * traffic[n][0] / op_ms[n] / 1e6 / PEAK_GBPS, 2),
                  "graph_replay_ms": round(graph_ms[n], 4)} for n in ops}
    per_op["sptrsv_batch"]["plain_ms"] = round(per_matrix_ms, 4)
    per_op["sptrsv_batch"]["speedup_vs_plain"] = round(per_matrix_ms / op_ms["sptrsv_batch"], 3)
    dom = max(per_op, key=lambda n: per_op[n]["ms"])
    kop = ddf.DDF_OP_SPTRSV_ADJ_KERNEL if dom.endswith("adj") else ddf.DDF_OP_SPTRSV
    ker = []
    for _ in range(args.steps):
        timer.flush()
        ddf.ddf_plan_time_kernels(p, 1)
        ops[dom]()
        kms, calls, _ = ddf.ddf_plan_kernel_time(p)
        ker.append(kms / max(calls, 1))
    ddf.ddf_plan_time_kernels(p, 0)
    kernel_ms = median(ker)
    binfo = ddf.ddf_plan_info(p)
    bkey = "solve_path_adj" if dom.endswith("adj") else "solve_path"
    bnames = {1: "k_solve_df", 2: "k_solve_thin", 3: "k_solve_range"}
    ba_dom = ddf.ddf_plan_traffic(p, kop, 1)[0]
    ach = ba_dom / (kernel_ms / 1e3) / 1e9
    kname = bnames.get(binfo.get(bkey))
    roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                "frac": round(ach / PEAK_GBPS, 4),
                "traffic": profile_value(f"traffic_{dom}_c4.md", f"hbm_bytes_per_launch_{kname}"),
                "kernel": kname, "call": dom, "kernel_ms": round(kernel_ms, 4), "bytes_alg_per_launch": ba_dom}
    cpu = None
    if not args.no_cpu:
        import oracle as O
        t0 = time.time()
        done, rel = 0, 0.0
        xh = None
        ops["sptrsv_batch"]()
        torch.cuda.synchronize()
        xh = X.cpu().numpy()
        off = 0
        for m in w.batch:
            xr = O.sptrsv(m["L"], m["B"])
            O.sptrsv_adj(m["L"], xr, m["G"])
            n_, k_ = m["L"].n_rows, m["k"]
            got = xh[off:off + n_ * k_].reshape(n_, k_)
            rel = max(rel, float(np.max(np.abs(got - xr)) / max(np.max(np.abs(xr)), 1e-300)))
            off += n_ * k_
            done += 1
            if time.time() - t0 > args.cpu_seconds:
                break
        cpu_s = time.time() - t0
        frac_rows = sum(m["L"].n_rows for m in w.batch[:done]) / sum(m.n_rows for m in mats)
        cpu_step = cpu_s / frac_rows
        cpu = {"value": round(bytes_step / cpu_step / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {done} of {len(mats)} matrices (solve and adjoint), {cpu_s:.1f} s, "
                         f"scaled by their share of the rows to {cpu_step * 1e3:.0f} ms per step",
               "parity": {"sptrsv_normwise_max_over_sampled": float(f"{rel:.3e}")}}
    out = {
        "metric": METRIC,
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "matrices": len(mats), "rows": sum(m.n_rows for m in mats),
                   "nnz_L": sum(m.nnz for m in mats), "nrhs_range": [min(ks), max(ks)],
                   "max_levels": binfo["max_levels"], "inspect_s": round(t_insp, 3),
                   "inspect_phases_s": [round(v, 3) for v in binfo["phase_seconds"]], "phases": PHASES,
                   "ner": {"sptrsv_batch": round(t_insp * 1e3 / (per_matrix_ms - op_ms["sptrsv_batch"]), 1)
                           if per_matrix_ms > op_ms["sptrsv_batch"] else None},
                   "solve_kernel": {"fwd": bnames.get(binfo["solve_path"]), "adj": bnames.get(binfo["solve_path_adj"])}},
        "pct_of_peak": round(100 * value / PEAK_GBPS, 2),
        "per_op": per_op, "bytes_alg_per_step": bytes_step,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
