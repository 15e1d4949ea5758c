"""Benchmark of the coronal FV-MHD hot path on one MI355X.

One step = one pass of the hot path over the large workload (6 x 96 x 96 x
240 = 13,271,040 cells, FP64): ghost fill + residual, JVP (with a B_r-map
direction), VJP (state and B_r-map gradients) and the Eq. 2 residual norms.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-ensemble]

The line also carries the ensemble figure: 64 uneven instances (29.95M
cells), residual + JVP of all of them as one captured graph of persistent
launches against 64 single-instance launches in sequence.

Prints ONE JSON line.  `value` is the throughput of whole steps in Mcell/s
(cells x steps / wall time of the timed region, inputs resident in HBM).
Per-kernel durations come from HIP events recorded on the launch stream by
the library over the timed region.  The `roofline` entry is the residual's
(the metric's HBM fraction is stated for the 13M-cell residual): its
algorithmic bytes per cell times the cells, over its kernels' average time
per launch; `roofline_ops` gives the same, with counter traffic and the FP64
work against the vector peak, for the residual, the JVP and the VJP.
The CPU baseline times the oracle (test infrastructure) on bounded samples:
per operation on one thread and on all threads, with the host's nproc and
CPU model.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic HBM bytes per cell and operation (FP64 SoA, 9 variables)
ALG_BYTES = {"residual": 144, "jvp": 216, "vjp": 216}
OP_KERNELS = {
    "residual": ("fused_march",),
    "jvp": ("grad_march_jvp", "flux_march_jvp"),
    "vjp": ("grad_march_fwd", "adjoint", "adjoint_ghosts", "adjoint_gather"),
}


def profile_record(prefix: str, match: dict):
    """A record line ("<prefix>: {json}") from the rocprofv3 summaries in
    profiles/ whose keys match; returns (record, source) with record None when
    the kernel sources changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith(prefix + ": "):
                    continue
                rec = json.loads(line[len(prefix) + 2:])
                if any(rec.get(k) != v for k, v in match.items()):
                    continue
                h = hashlib.sha1()
                for src in rec["sources"]:
                    with open(os.path.join(ROOT, "paper_2209_04481_amd", "csrc", src), "rb") as g:
                        h.update(g.read())
                rel = os.path.relpath(path, ROOT)
                if h.hexdigest() != rec["sources_sha1"]:
                    return None, rel + " (stale: kernel sources changed)"
                return rec, rel
    return None, None


def host_cpu_info():
    """nproc and the CPU model of the host (lscpu), for the baseline record."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip()
        info["nproc"] = int(out)
    except Exception:
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    return info


def _oracle_sample(inst, n: int, seed: int):
    """A contiguous block of n cells in the middle of the shell, with a JVP
    direction on its distance-2 stencil and VJP weights on the block."""
    import torch

    from oracle import mhd
    from oracle.grid import Grid as OGrid
    og = OGrid(inst.N, inst.Nr, inst.r_nodes)
    U = torch.from_numpy(inst.U)
    br = torch.from_numpy(inst.br)
    n = min(n, inst.ncells)
    start = (inst.ncells - n) // 2
    cells = torch.arange(start, start + n)
    gen = torch.Generator().manual_seed(seed)
    v = torch.zeros_like(U)
    st = mhd._Stencil(og, cells)
    v[:, st.D2] = torch.randn(9, st.D2.numel(), dtype=torch.float64, generator=gen) * U[:, st.D2].abs()
    w = torch.randn(9, n, dtype=torch.float64, generator=gen)
    return og, U, br, cells, v, w


def cpu_baseline(insts: dict, ncells_sample: int = 10000, reps: int = 3):
    """The oracle (plain float64 PyTorch CPU code) timed on the host: per
    workload, the residual and the JVP on a contiguous block of cells, on one
    thread and on all the threads torch uses, the median of `reps` runs each;
    and the whole step (residual + JVP + VJP) on all threads, whose rate on
    the first workload is the record's value."""
    import statistics

    import torch

    from oracle import mhd, solve
    info = host_cpu_info()
    nthr = torch.get_num_threads()
    per = {}
    value = None
    for name, inst in insts.items():
        og, U, br, cells, v, w = _oracle_sample(inst, ncells_sample, inst.seed)
        n = cells.numel()
        op = mhd.Params()
        ops = {"residual": lambda: mhd.residual(og, U, br, op, cells=cells),
               "jvp": lambda: solve.jvp(og, U, br, op, v, cells=cells)}
        rec = {}
        for opn, fn in ops.items():
            r = {}
            for label, th in (("1_thread", 1), ("all_threads", nthr)):
                torch.set_num_threads(th)
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    fn()
                    ts.append(time.perf_counter() - t0)
                r[label + "_mcells_per_s"] = round(n / statistics.median(ts) / 1e6, 5)
            r["ideal_all_core_mcells_per_s"] = round(r["1_thread_mcells_per_s"] * info["nproc"], 4)
            rec[opn] = r
        torch.set_num_threads(nthr)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            mhd.residual(og, U, br, op, cells=cells)
            solve.jvp(og, U, br, op, v, cells=cells)
            solve.vjp(og, U, br, op, w, cells=cells)
            ts.append(time.perf_counter() - t0)
        rec["step_all_threads_mcells_per_s"] = round(n / statistics.median(ts) / 1e6, 5)
        rec["sample_cells"] = n
        per[name] = rec
        if value is None:
            value = rec["step_all_threads_mcells_per_s"]
    first = next(iter(insts))
    return {"value": value, "unit": "Mcell/s (residual+JVP+VJP step)", "cores": nthr, "kind": "oracle",
            "sample": f"{ncells_sample} contiguous cells (distance-2 stencil gathered) of each of the "
                      f"{', '.join(insts)} workloads, median of {reps} runs; value: the {first} workload's step "
                      f"on {nthr} threads",
            "nproc": info["nproc"], "host": {k: v for k, v in info.items() if k != "nproc"},
            "per_workload": per}


def bench_solver(with_sensitivity: bool):
    """The 1.66M-cell workload: residual and JVP (20 calls each, percentiles
    of the library's event times), one backward-Euler step (CFL 1e3,
    GMRES(30), no restart), the first steps of the steady march and,
    optionally, the 20-step B_r sensitivity (CFL 0.05, tight solves,
    checkpoints every 5 steps)."""
    import numpy as np
    import torch

    import coronal_inputs as ci
    from paper_2209_04481_amd import Context, Grid, Params

    inst = ci.workload("medium")
    grid = Grid(inst.N, inst.Nr, inst.r_nodes)
    ctx = Context(grid, Params())
    ctx.set_inner_br(torch.from_numpy(inst.br).cuda())
    U = torch.from_numpy(inst.U).cuda()
    out = torch.empty_like(U)
    # residual and JVP on this workload: 20 calls each after a warm-up, library event times per call
    v = torch.from_numpy(ci.scaled_direction(inst.U, inst.seed)).cuda()
    dbr = torch.from_numpy(ci.br_direction(grid.nb, inst.seed)).cuda()
    Jv = torch.empty_like(U)
    ctx.residual(U, out=out)
    ctx.jvp(U, v, dbr, out=Jv)
    ctx.timing_enable(True)
    ctx.timing_read()
    per = {"residual": [], "jvp": []}
    for _ in range(20):
        ctx.residual(U, out=out)
        t = ctx.timing_read()
        per["residual"].append(sum(t[k][0] for k in OP_KERNELS["residual"] if k in t))
        ctx.jvp(U, v, dbr, out=Jv)
        t = ctx.timing_read()
        per["jvp"].append(sum(t[k][0] for k in OP_KERNELS["jvp"] if k in t))
    ctx.timing_enable(False)
    op_pct = {op: [round(float(np.percentile(x, q)), 4) for q in (10, 50, 90)] for op, x in per.items()}
    del Jv
    ctx.be_step(U, cfl=1e3, m=30, out=out)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        _, hist = ctx.be_step(U, cfl=1e3, m=30, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    res = {"workload": f"medium: 6x{inst.N}x{inst.N}x{inst.Nr} ({inst.ncells} cells)",
           "op_ms_p10_p50_p90": op_pct,
           "be_step_ms": round(ms, 2), "gmres_iterations": int(len(hist)),
           "ms_per_gmres_iteration": round(ms / max(len(hist), 1), 3), "final_relative_residual": float(hist[-1])}
    print(f"[bench] backward-Euler step: {ms:.1f} ms", file=sys.stderr, flush=True)
    # the same step with GMRES right-preconditioned by V/dt (a library option; the step above is the
    # unpreconditioned one of the specification)
    ctx.set_preconditioner(1)
    ctx.be_step(U, cfl=1e3, m=30, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, hist_j = ctx.be_step(U, cfl=1e3, m=30, out=out)
    torch.cuda.synchronize()
    ms_j = (time.perf_counter() - t0) * 1e3 / reps
    ctx.set_preconditioner(0)
    res["jacobi"] = {"be_step_ms": round(ms_j, 2), "final_relative_residual": float(hist_j[-1]),
                     "relative_residual_after_10": float(hist_j[9]),
                     "note": "GMRES(30) right-preconditioned by the step's diagonal V/dt (cfv_set_preconditioner)"}
    # the march to a steady state: the first 8 steps under the paper's CFL law (from 2, doubling every
    # 200 steps up to 128)
    Us = U.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    from paper_2209_04481_amd.binding import CfvNonPhysical
    try:
        mh, cfls = ctx.steady(Us, 8, cfl0=2.0, cfl_max=128.0, every=200, m=30)
        stop = "completed"
    except CfvNonPhysical as e:
        mh, cfls, stop = e.hist, e.cfls, "non-finite state"
    torch.cuda.synchronize()
    ms_st = (time.perf_counter() - t0) * 1e3 / max(len(cfls), 1)
    res["steady_march"] = {"steps": int(len(cfls)), "ms_per_step": round(ms_st, 2), "end": stop,
                           "cfl": [float(c) for c in cfls],
                           "log10_monitor_V_x": [round(float(x), 3) for x in mh[:, 1]],
                           "log10_monitor_rho": [round(float(x), 3) for x in mh[:, 0]]}
    print(f"[bench] steady march: {ms_st:.1f} ms per step", file=sys.stderr, flush=True)
    del Us
    if with_sensitivity:
        from paper_2209_04481_amd.sensitivity import Sensitivity
        br = torch.from_numpy(inst.br).cuda()
        sens = Sensitivity(ctx, U, cfl=0.05, nsteps=20, every=5, max_restarts=16, layer=2)
        t0 = time.perf_counter()
        sens.gradient(br)
        torch.cuda.synchronize()
        res["sensitivity_s"] = round(time.perf_counter() - t0, 2)
        res["sensitivity"] = "dL/dB_r after 20 steps (CFL 0.05, solves to 1e-12, checkpoints every 5)"
        print(f"[bench] sensitivity: {res['sensitivity_s']} s", file=sys.stderr, flush=True)
    return res


def bench_efield(ctx, U, reps: int = 20):
    """The E-field diagnostic and the E-free state on the bench state: kernel
    times from HIP events on the launch stream, and algorithmic HBM rates
    (stats only: rho, rho v, B read, 56 B/cell; with the field also written,
    80 B/cell; E-free state: 9 rows read and written, 144 B/cell)."""
    import torch
    nc = U.shape[1]
    st = torch.empty(8, dtype=torch.float64, device="cuda")
    E = torch.empty(3, nc, dtype=torch.float64, device="cuda")
    U0 = torch.empty_like(U)
    out = {}
    for name, fn, kern, bpc in (("stats", lambda: ctx.efield(U, field=False, stats=st), "efield", 56),
                                ("field", lambda: ctx.efield(U, stats=st, E=E), "efield", 80),
                                ("efree", lambda: ctx.efree_state(U, out=U0), "efree", 144)):
        fn()
        torch.cuda.synchronize()
        ctx.timing_enable(True)
        ctx.timing_read()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ms, n = ctx.timing_read()[kern]
        ctx.timing_enable(False)
        avg = ms / n
        gbs = bpc * nc / (avg * 1e-3) / 1e9
        out[name] = {"avg_ms": round(avg, 4), "alg_bytes_per_cell": bpc, "GB/s": round(gbs, 1),
                     "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    out["max_abs_E_r_theta_phi_mag"] = [float(x) for x in st[:4].cpu()]
    out["rms_E_r_theta_phi_mag"] = [float(x) for x in st[4:].cpu()]
    return out


def bench_ensemble(reps: int, solve_reps: int = 2):
    """64 uneven instances (29.95M cells): residual + JVP of all of them as one
    captured graph of two persistent launches, against 64 single-instance
    launches in sequence on the same stream (not captured)."""
    import torch

    import coronal_inputs as ci
    from paper_2209_04481_amd import Context, Ensemble, Grid, Params
    from paper_2209_04481_amd.autotune import autotune

    t0 = time.time()
    insts = ci.ensemble_instances()
    ctxs, U, v = [], [], []
    for q, inst in enumerate(insts):
        c = Context(Grid(inst.N, inst.Nr, inst.r_nodes), Params())
        c.set_inner_br(torch.from_numpy(inst.br).cuda())
        ctxs.append(c)
        U.append(torch.from_numpy(inst.U).cuda())
        v.append(torch.from_numpy(ci.scaled_direction(inst.U, 900 + q)).cuda())
    del insts
    R = [torch.empty_like(u) for u in U]
    J = [torch.empty_like(u) for u in U]
    cells = sum(c.grid.ncells for c in ctxs)
    print(f"[bench] ensemble inputs: {len(ctxs)} instances, {cells} cells in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    ens = Ensemble(ctxs)
    ens.bind(U, v=v, R=R, Jv=J)
    best, ms = autotune(ens, reps=3, stream=s, use_cache=False)
    ens.capture(s)
    ens.replay(s)
    s.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        ens.replay(s)
    b.record(s)
    b.synchronize()
    batched = a.elapsed_time(b) / reps
    with torch.cuda.stream(s):
        for c, u, w, r, j in zip(ctxs, U, v, R, J):
            c.jvp(u, w, out=j, R=r)
        s.synchronize()
        a.record(s)
        for _ in range(reps):
            for c, u, w, r, j in zip(ctxs, U, v, R, J):
                c.jvp(u, w, out=j, R=r)
        b.record(s)
        b.synchronize()
    sequential = a.elapsed_time(b) / reps
    print(f"[bench] ensemble: batched {batched:.3f} ms, sequential {sequential:.3f} ms", file=sys.stderr, flush=True)
    solve = bench_ensemble_solve(ens, ctxs, U, s, solve_reps) if solve_reps > 0 else None
    return {"instances": len(ctxs), "cells": cells, "op": "residual + JVP per instance",
            "batched_graph_ms": round(batched, 4), "sequential_ms": round(sequential, 4),
            "speedup": round(sequential / batched, 3), "speedup_target": 3.0, "repeats": reps,
            "batched_mcells_per_s": round(cells / (batched * 1e-3) / 1e6, 1),
            "tuning": best.as_dict(), "autotune_ms": {k: round(x, 4) for k, x in ms.items()},
            "solve": solve}


def bench_ensemble_solve(ens, ctxs, U, s, reps: int, cfl: float = 1e3, m: int = 30):
    """One backward-Euler step (GMRES(30), CFL 1e3) of all instances: one
    captured graph of the lockstep device solve, against cfv_be_step of each
    instance in sequence (one host synchronisation per GMRES iteration)."""
    import torch
    U_new = [torch.empty_like(u) for u in U]
    hist = torch.zeros(len(ctxs), m, dtype=torch.float64, device="cuda")
    ens.bind_be_step(U, U_new, cfl, m, hist)
    ens.capture(s)
    ens.replay(s)
    s.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        ens.replay(s)
    b.record(s)
    b.synchronize()
    batched = a.elapsed_time(b) / reps
    with torch.cuda.stream(s):
        outs = [torch.empty_like(u) for u in U]
        for c, u, o in zip(ctxs, U, outs):
            c.be_step(u, cfl=cfl, m=m, out=o)
        s.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for c, u, o in zip(ctxs, U, outs):
                c.be_step(u, cfl=cfl, m=m, out=o)
        s.synchronize()
        sequential = (time.perf_counter() - t0) * 1e3 / reps
    diff = max(float(((x - u) - (y - u)).norm() / (y - u).norm()) for x, y, u in zip(U_new, outs, U))
    print(f"[bench] ensemble solve: batched {batched:.1f} ms, sequential {sequential:.1f} ms", file=sys.stderr,
          flush=True)
    return {"op": f"backward-Euler step, GMRES({m}), CFL {cfl:g}, per instance", "batched_graph_ms": round(batched, 2),
            "sequential_ms": round(sequential, 2), "speedup": round(sequential / batched, 3), "speedup_target": 3.0,
            "repeats": reps,
            "max_rel_step_difference": diff}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["tiny", "medium", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000)
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also copy a 1 GiB buffer twice (reference dispatches for HBM counters)")
    ap.add_argument("--ensemble-reps", type=int, default=50)
    ap.add_argument("--solve-reps", type=int, default=2)
    ap.add_argument("--no-solver", action="store_true")
    ap.add_argument("--efield-reps", type=int, default=20)
    ap.add_argument("--sweep-reps", type=int, default=100,
                    help="steps of the per-operation percentile pass (library event times per call)")
    ap.add_argument("--sensitivity", action="store_true", help="also time the 20-step B_r sensitivity (about 57 s)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import coronal_inputs as ci
    from paper_2209_04481_amd import Context, Grid, Params

    torch.cuda.set_device(0)
    t_gen = time.time()
    inst = ci.workload(args.workload)
    print(f"[bench] inputs for {args.workload}: {inst.ncells} cells in {time.time() - t_gen:.1f} s",
          file=sys.stderr, flush=True)
    grid = Grid(inst.N, inst.Nr, inst.r_nodes)
    ctx = Context(grid, Params())
    U = torch.from_numpy(inst.U).cuda()
    br = torch.from_numpy(inst.br).cuda()
    v = torch.from_numpy(ci.scaled_direction(inst.U, inst.seed)).cuda()
    dbr = torch.from_numpy(ci.br_direction(grid.nb, inst.seed)).cuda()
    w = torch.randn(9, inst.ncells, dtype=torch.float64, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(inst.seed))
    ctx.set_inner_br(br)
    R = torch.empty_like(U)
    Jv = torch.empty_like(U)
    gU = torch.empty_like(U)
    gbr = torch.empty(grid.nb, dtype=torch.float64, device="cuda")
    nrm = torch.empty(9, dtype=torch.float64, device="cuda")

    def step():
        ctx.residual(U, out=R)
        ctx.jvp(U, v, dbr, out=Jv)
        ctx.vjp(U, w, out=gU, gbr=gbr)
        ctx.norms(R, out=nrm)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    ctx.timing_enable(True)
    ctx.timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    times = ctx.timing_read()
    ctx.timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps

    # per-operation spread: the same steps again, the library's event times read after each one
    ctx.timing_enable(True)
    ctx.timing_read()
    per_step = {op: [] for op in OP_KERNELS}
    for _ in range(args.sweep_reps):
        step()
        t_step = ctx.timing_read()
        for op, ks in OP_KERNELS.items():
            per_step[op].append(sum(t_step[k][0] for k in ks if k in t_step))
    ctx.timing_enable(False)

    # the same step with R taken from the JVP's dual pass (cfv_jvp with R):
    # the outputs of the step above from one march fewer
    R_sep = R.clone()
    R.zero_()

    def step_fused():
        ctx.jvp(U, v, dbr, out=Jv, R=R)
        ctx.vjp(U, w, out=gU, gbr=gbr)
        ctx.norms(R, out=nrm)

    step_fused()
    torch.cuda.synchronize()
    tf0 = time.perf_counter()
    for _ in range(args.steps):
        step_fused()
    torch.cuda.synchronize()
    tf1 = time.perf_counter()
    r_diff = float(((R - R_sep).abs().max() / R_sep.abs().max()).item())

    nc = inst.ncells
    per_kernel = {k: {"avg_ms": ms / n, "launches": n} for k, (ms, n) in times.items()}
    op_ms = {}
    for op, ks in OP_KERNELS.items():
        op_ms[op] = sum(times[k][0] / times[k][1] for k in ks if k in times)
    vrec, vsrc = profile_record("valu-record", {"workload": args.workload})

    def op_roofline(op):
        """HBM roofline of one operation (algorithmic bytes over its kernels'
        average time per launch, from HIP events on the launch stream), the
        counter traffic of the committed rocprofv3 record (null once the
        kernel sources changed), and its FP64 work against the vector peak."""
        achieved = ALG_BYTES[op] * nc / (op_ms[op] * 1e-3) / 1e9
        trec, traffic_src = profile_record("traffic-record", {"kernel": op, "workload": args.workload})
        r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": trec["bytes_per_launch"] if trec else None,
             "traffic_note": ("bytes per launch: rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy; "
                              f"from {traffic_src}") if traffic_src else None,
             "kernel": f"{op} ({' + '.join(OP_KERNELS[op])})", "avg_ms": round(op_ms[op], 4),
             "alg_bytes_per_cell": ALG_BYTES[op]}
        if trec:
            r["traffic_bytes_per_cell"] = round(trec["bytes_per_launch"] / nc, 1)
        if vrec and op in vrec["flop_per_cell"]:
            f = vrec["flop_per_cell"][op]
            tf = f * nc / (op_ms[op] * 1e-3) / 1e12
            r["fp64"] = {"flop_per_cell": f, "tflops": round(tf, 2), "peak_tflops": FP64_PEAK_TFLOPS,
                         "frac": round(tf / FP64_PEAK_TFLOPS, 4),
                         "floor_ms": round(f * nc / (FP64_PEAK_TFLOPS * 1e12) * 1e3, 4),
                         "source": vsrc}
        return r

    # the headline is the residual's: the metric's "% of HBM roofline" is
    # stated for the 13M-cell residual
    roofline = op_roofline("residual")
    roofline_ops = {op: op_roofline(op) for op in OP_KERNELS}

    out = {
        "metric": "Mcell-residuals/s and JVP+VJP/s FP64 at 13M cells; % of HBM roofline; ensemble speedup",
        "value": round(nc * args.steps / (t1 - t0) / 1e6, 2),
        "unit": "Mcell/s (residual+JVP+VJP step)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: cubed-sphere shell 6x{inst.N}x{inst.N}x{inst.Nr} "
                               f"({nc} cells), r in [1, 21.5], Parker wind + dipole, 1% noise, "
                               f"B_r map l<=31, Barth-Jespersen limiter"},
        "residual_mcells_per_s": round(nc / (op_ms["residual"] * 1e-3) / 1e6, 1),
        "residuals_per_s": round(1e3 / op_ms["residual"], 2),
        "jvp_per_s": round(1e3 / op_ms["jvp"], 2),
        "vjp_per_s": round(1e3 / op_ms["vjp"], 2),
        "op_ms": {k: round(x, 4) for k, x in op_ms.items()},
        "op_ms_p10_p50_p90": {op: [round(float(np.percentile(v, q)), 4) for q in (10, 50, 90)]
                              for op, v in per_step.items()},
        "kernels": {k: {"avg_ms": round(d["avg_ms"], 4), "launches": d["launches"]} for k, d in per_kernel.items()},
        "roofline": roofline,
        "roofline_ops": roofline_ops,
        "step_r_from_jvp": {"mcells_per_s": round(nc * args.steps / (tf1 - tf0) / 1e6, 2),
                            "ms_per_step": round((tf1 - tf0) * 1e3 / args.steps, 4),
                            "max_rel_r_difference": r_diff,
                            "note": "the step with R written by the JVP launch (cfv_jvp with R) instead of a "
                                    "residual launch of its own; not the headline value"},
    }
    if vrec:
        out["fp64_valu"] = {
            op: {"flop_per_cell": f, "tflops": round(f * nc / (op_ms[op] * 1e-3) / 1e12, 2),
                 "frac": round(f * nc / (op_ms[op] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}
            for op, f in vrec["flop_per_cell"].items()}
        out["fp64_valu_note"] = (f"executed FP64 flops per cell from rocprofv3 counters ({vsrc}) over the measured "
                                 f"operation times; peak {FP64_PEAK_TFLOPS} TFLOP/s")
    out["efield"] = bench_efield(ctx, U, args.efield_reps)
    if not args.no_solver:
        out["solver"] = bench_solver(args.sensitivity)
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for q in range(2):
            b.copy_(a)
            ev[q + 1].record()
        torch.cuda.synchronize()
        cms = [ev[q].elapsed_time(ev[q + 1]) for q in range(2)]
        out["copy_calibration"] = {"bytes_moved": 2 * a.numel() * 8, "ms": [round(x, 4) for x in cms],
                                   "gbs": round(2 * a.numel() * 8 / (min(cms) * 1e-3) / 1e9, 1)}
        del a, b
    if not args.no_ensemble:
        del ctx, U, v, w, R, Jv, gU
        torch.cuda.empty_cache()
        out["ensemble"] = bench_ensemble(args.ensemble_reps, args.solve_reps)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        insts = {args.workload: inst}
        if args.workload == "large":
            insts["medium"] = ci.workload("medium")
        out["cpu_baseline"] = cpu_baseline(insts, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
