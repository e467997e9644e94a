"""Benchmark: batched JFNK solves of NLTE columns on one MI355X.

One step = one complete JFNK solve (residual evaluations, preconditioner,
GMRES, Newton) of every column of the workload, starting from LTE, with all
inputs resident in HBM (column setup is done before the timed region).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line: formal-solution depth-points per second over the whole
solve (depth-points = frequencies x 2 x angles x depths per residual call,
summed over every residual call of every column), plus columns converged/s,
the roofline of the formal-solution kernel and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2406_17234_amd import synth as S  # noqa: E402

# MI355X FP32 vector peak: 157.3 TFLOP/s (256 CUs, 2.4 GHz), i.e. 7.87e13 FMA
# lane-operations per second.  The issue-rate probes measure what the
# non-packed FMA that the kernels use reaches of it.
PEAK_VALU_OPS = 157.3e12 / 2
# algorithmic work per depth-point: ~10 VALU ops plus half an exp and half a
# reciprocal (shared by the two rays of an angle), each transcendental
# counted as the FMA issue slots it costs: 4 unless the issue-rate probes
# have measured it (main() then replaces this value)
TRANS_SLOTS = 4.0
OPS_PER_DP = 10.0 + 0.5 * TRANS_SLOTS + 0.5 * TRANS_SLOTS

# HBM bytes per F-mode k_formal launch (the roofline kernel) from FETCH_SIZE /
# WRITE_SIZE counter runs of this workload, each scaled by the same counter on
# a plain copy kernel; valid only for the kernel source they were taken on
# (hash of its files).
TRAFFIC = {
    "batch6": {"source": "25d629d1e1f31708", "bytes_per_launch": 5.2228e+09,
               "read": 4.8958e+11 / 192, "written": 5.1320e+11 / 192},
}
# the same for the F-mode velocity formal solution of the 512-column velocity
# batch (mean over the profiled solve's 140 launches)
TRAFFIC_VEL = {"source": "9f5debcc6ac80876", "columns": 512, "bytes_per_launch": 6.4376e+09,
               "read": 5.4273e+09, "written": 1.0103e+09}
KERNEL_SOURCES = ["paper_2406_17234_amd/csrc/nlte_residual.hip",
                  "paper_2406_17234_amd/csrc/nlte_kernels.h",
                  "paper_2406_17234_amd/csrc/nlte_internal.h"]
VEL_KERNEL_SOURCES = ["paper_2406_17234_amd/csrc/nlte_velocity.hip",
                      "paper_2406_17234_amd/csrc/nlte_kernels.h",
                      "paper_2406_17234_amd/csrc/nlte_internal.h"]


def kernel_source_hash(files=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


WORKLOADS = {
    # name: (description, maker(i), ncol default, precision, ftol)
    "batch6": ("4096 chromosphere columns, 6-level atom (5 lines + 5 edges), "
               "T perturbed +-10%, Nz U{64..160}, Nnu U{400..800}, 5 mu x 2; "
               "FP32 formal solution, FP64 rates/solve", S.batch6_column, 4096, 1, 1e-6),
    "batch6_fp64": ("4096 chromosphere columns as batch6, all FP64", S.batch6_column, 4096, 0, 1e-8),
    "chromo6": ("1 column: 6-level atom, 82-depth chromosphere, ~600 frequencies, 5 mu x 2, FP64",
                lambda i: S.chromo6(), 1, 0, 1e-8),
    "chromo6_fp32": ("1 column as chromo6, FP32 formal solution", lambda i: S.chromo6(), 1, 1, 1e-6),
    "slab3": ("1 column: 3-level atom, isothermal slab, 64 depths, 81 frequencies, 3 mu x 2, FP64",
              lambda i: S.slab3(), 1, 0, 1e-8),
    "chromo11": ("1 column: 11-level atom (20 lines + 10 edges), 256 depths, ~4000 frequencies, "
                 "8 mu x 2, FP32 formal solution", lambda i: S.chromo11(), 1, 1, 1e-6),
}


def _oracle_column(args):
    """CPU baseline worker: the FP64 oracle's JFNK solve of one column."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import nlte_oracle as O
    maker_name, i, ftol, rtol = args
    prob = WORKLOADS[maker_name][1](i)
    tb = O.setup(prob)
    t0 = time.perf_counter()
    s = O.solve(tb, ftol=ftol, rtol=rtol, maxiter=50)
    dt = time.perf_counter() - t0
    return dt, s.calls * prob.depth_points(), bool(s.converged)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_single(args):
    """The oracle on one core: a full JFNK solve of a small configuration, or
    (for the 11-level stress column, whose solve would take far longer than
    the benchmark allows) a few residual calls."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle import nlte_oracle as O
    name, ftol = args
    prob = {"C1_slab3": S.slab3, "C2_chromo6": S.chromo6, "C5_chromo11": S.chromo11,
            "V_chromo6_vel": S.chromo6_vel}[name]()
    tb = O.setup(prob)
    if name == "C5_chromo11":
        t0 = time.perf_counter()
        calls = 2
        for _ in range(calls):
            O.residual(tb, tb.nstar)
        dt = time.perf_counter() - t0
        return {"config": name, "kind": "residual calls", "calls": calls, "s_per_call": dt / calls,
                "depth_points_per_s": calls * prob.depth_points() / dt, "cores": 1}
    rtol = 1e-2 if name == "V_chromo6_vel" else 1e-3
    t0 = time.perf_counter()
    s = O.solve(tb, ftol=ftol, rtol=rtol, maxiter=80)
    dt = time.perf_counter() - t0
    return {"config": name, "kind": "JFNK solve", "ftol": ftol, "rtol": rtol, "s_per_solve": dt,
            "calls": s.calls, "s_per_call": dt / max(s.calls, 1), "converged": bool(s.converged),
            "depth_points_per_s": s.calls * prob.depth_points() / dt, "cores": 1}


def oracle_single_columns():
    """C1, C2, C5 and the velocity-step column on one core each, run side by
    side (one process per configuration)."""
    jobs = [("C1_slab3", 1e-8), ("C2_chromo6", 1e-8), ("C5_chromo11", None), ("V_chromo6_vel", 1e-8)]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        return {r["config"]: r for r in pool.map(_oracle_single, jobs)}


def gpu_single_columns(ctx, nlte):
    """Latency of one-column solves on the GPU: C1 (3-level slab, FP64, stop
    at 1e-8) and C2 (6-level chromosphere, FP64 and FP32 form); median of 5
    solves after one warm-up, setup excluded."""
    import torch
    out = {}
    for name, prob, prec, ftol in [("C1_slab3_fp64", S.slab3(), nlte.FP64, 1e-8),
                                   ("C2_chromo6_fp64", S.chromo6(), nlte.FP64, 1e-8),
                                   ("C2_chromo6_fp32", S.chromo6(), nlte.FP32_FORM, 1e-6)]:
        col = nlte.Column(ctx, prob, precision=prec)
        opts = nlte.default_opts(ftol=ftol, rtol=1e-3, maxiter=50)
        col.solve(opts=opts)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st, rc = col.solve(opts=opts)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        col.close()
        out[name] = {"ms_per_solve": float(np.median(ts)) * 1e3, "newton_iters": st["newton_iters"],
                     "residual_calls": st["f_calls"], "status": st["status"], "ftol": ftol}
    return out


def cpu_baseline(workload, ncol, ftol, rtol, budget_s=20.0):
    """Time the oracle on a bounded sample (one column per process, a pool of
    up to 16 processes, started before any GPU use)."""
    procs = max(1, min(16, os.cpu_count() or 1, ncol))
    sample = list(range(min(ncol, procs)))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_column, [(workload, i, ftol, rtol) for i in sample])
    wall = time.perf_counter() - t0
    dp = sum(r[1] for r in res)
    return {
        "value": dp / wall, "unit": "depth-points/s", "cores": procs, "kind": "oracle",
        "sample": f"{len(sample)} columns of the workload ({workload} columns 0..{len(sample) - 1}), "
                  f"one FP64 NumPy JFNK solve per process, {procs} processes, wall {wall:.1f} s",
        "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
        "columns_per_s": len(sample) / wall,
        "converged": sum(r[2] for r in res),
    }


def serve_run(ctx, nlte, rate, duration_s, warm_s, first_id, budget_gb, max_active, opts):
    """One served stream: Poisson arrivals (rate per second over duration_s)
    of mixed 3/6/11-level requests (FP32 form), each submitted at its arrival
    time as a problem description; the server creates a request's column
    when it admits it within the HBM budget (setup is part of its latency)
    and frees it at retirement.  Latency = finish - scheduled arrival (so a
    submission that runs late counts against it); statistics over the
    requests arriving after warm_s."""
    import torch
    arrivals = S.stream_arrivals(duration_s, rate, seed=4 + first_id)
    nreq = len(arrivals)
    t0 = time.perf_counter()
    probs = [S.stream_request(first_id + j) for j in range(nreq)]
    preps = [nlte.Prepared(p) for p in probs]
    outs = [torch.empty(p.atmos.nz, p.atom.nlev, dtype=torch.float64, device="cuda:0")
            for p in probs]
    gen_s = time.perf_counter() - t0
    print(f"[bench] stream at {rate:g}/s: {nreq} requests prepared in {gen_s:.1f} s",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    srv = nlte.Server(ctx, hbm_budget=int(budget_gb * (1 << 30)), max_active=max_active, opts=opts)
    t_create = time.perf_counter()  # the server's clock starts at creation
    tickets = []
    t_start = time.perf_counter()
    for i, ta in enumerate(arrivals):
        dt = t_start + ta - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.submit_problem(preps[i], outs[i], nlte.FP32_FORM))
    t_sub = time.perf_counter() - t_start
    srv.drain(1200.0)
    wall = time.perf_counter() - t_start
    res = [srv.poll(t)[1] for t in tickets]
    info = srv.info()
    srv.close()
    base_ms = (t_start - t_create) * 1e3
    arr_ms = base_ms + arrivals * 1e3
    done = np.array([r["t_done_ms"] for r in res])
    lat = done - arr_ms
    setup_ms = np.array([r["t_done_ms"] - r["t_admit_ms"] for r in res])
    conv = np.array([r["status"] == 0 for r in res])
    win = arrivals >= warm_s
    t_end_arr = base_ms + duration_s * 1e3
    finished_in_window = np.sum((done >= base_ms + warm_s * 1e3) & (done <= t_end_arr))
    dp = float(sum(r["f_calls"] * p.depth_points() for r, p in zip(res, probs)))
    return {
        "arrival_rate_per_s": rate, "arrival_window_s": duration_s, "warmup_s": warm_s,
        "requests": nreq, "requests_measured": int(win.sum()),
        "finish_rate_per_s_during_arrivals": float(finished_in_window) / max(duration_s - warm_s, 1e-9),
        "columns_per_s_overall": nreq / ((done.max() - arr_ms.min()) * 1e-3),
        "converged_fraction": float(conv[win].mean()),
        "converged_fraction_by_levels": {str(l): float(np.mean([c for c, p in zip(conv, probs)
                                                               if p.atom.nlev == l]))
                                         for l in (3, 6, 11)},
        "fp64_fallback_fraction": float(np.mean([r["precision"] == 0 for r in res])),
        "latency_ms_p50": float(np.percentile(lat[win], 50)),
        "latency_ms_p99": float(np.percentile(lat[win], 99)),
        "latency_ms_max": float(lat[win].max()),
        "admit_to_done_ms_p50": float(np.percentile(setup_ms[win], 50)),
        "queue_at_end_of_arrivals": int(np.sum(np.array([r["t_admit_ms"] for r in res]) > t_end_arr)),
        "depth_points_per_s": dp / ((done.max() - arr_ms.min()) * 1e-3),
        "hbm_budget_gb": budget_gb, "peak_active_gb": info["peak_active_bytes"] / (1 << 30),
        "max_active": max_active, "server_steps": info["steps"], "submit_s": t_sub, "wall_s": wall,
    }


def serve_stream(ctx, nlte, args, ftol):
    """Served stream (config C4): first a short overload probe at the
    configured rate (the server's capacity is what it finishes per second
    while saturated), then a sustained run at 80% of that capacity: a warm-up
    followed by the measured window, latency percentiles over the window."""
    opts = nlte.default_opts(ftol=ftol, rtol=args.rtol, maxiter=50,
                             max_krylov_total=args.max_krylov_total,
                             fp64_fallback=args.fp64_fallback)
    out = {}
    if args.serve_full:
        out["full_rate"] = serve_run(ctx, nlte, args.serve_rate, args.serve_seconds + args.serve_warmup,
                                     args.serve_warmup, 0, args.serve_budget_gb, args.serve_max_active, opts)
        return out
    probe = serve_run(ctx, nlte, args.serve_rate, args.serve_probe_seconds, 0.0, 0,
                      args.serve_budget_gb, args.serve_max_active, opts)
    out["overload_probe"] = probe
    cap = probe["columns_per_s_overall"]
    rate = max(10.0, round(0.8 * cap, -1))
    out["sustained"] = serve_run(ctx, nlte, rate, args.serve_seconds + args.serve_warmup,
                                 args.serve_warmup, 1_000_000, args.serve_budget_gb,
                                 args.serve_max_active, opts)
    return out


def single_fp64(ctx, nlte, problems, rtol, batch_outs):
    """The plain single-column FP64 GPU JFNK on the same columns, one solve at
    a time, at two stops: the scaled residual 1e-8, and 1e-6, the stop of the
    batched FP32 form.  Each column's populations are compared with a tight
    FP64 solve (1e-12), and so are those of the batched FP32 form, so the
    columns/s figures are quoted with the accuracy each reaches."""
    import torch
    cols = [nlte.Column(ctx, p, precision=nlte.FP64) for p in problems]
    tight = [c.solve(opts=nlte.default_opts(ftol=1e-12, rtol=1e-6, maxiter=80))[0].cpu().numpy()
             for c in cols]
    out = {"columns": len(cols)}
    for ftol in (1e-8, 1e-6):
        opts = nlte.default_opts(ftol=ftol, rtol=rtol, maxiter=50)
        cols[0].solve(opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [c.solve(opts=opts) for c in cols]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = max(float(np.max(np.abs(r[0].cpu().numpy() / t - 1))) for r, t in zip(res, tight))
        out[f"ftol_{ftol:g}"] = {"columns_per_s": len(cols) / dt, "ms_per_column": dt / len(cols) * 1e3,
                                 "converged_fraction": float(np.mean([r[2]["status"] == 0 for r in res])),
                                 "max_rel_error_vs_tight_fp64": err}
    out["batched_fp32_form_max_rel_error_vs_tight_fp64"] = max(
        float(np.max(np.abs(o.cpu().numpy() / t - 1))) for o, t in zip(batch_outs, tight))
    for c in cols:
        c.close()
    return out


def f_only(ctx, nlte, problems, prec, runs=100, tune=True):
    """F-only loop: a residual plan over the columns (graph-captured, launch
    shape tuned), evaluated at LTE populations `runs` times after warm-up.
    Returns formal-solution depth-points per second over whole F evaluations
    (opacity, formal solution, rates and rate equations included)."""
    import torch
    cols = [nlte.Column(ctx, p, precision=prec) for p in problems]
    ns = [c.lte() for c in cols]
    Fs = [torch.empty_like(n) for n in ns]
    plan = nlte.Plan(ctx, cols, ns, Fs, graph=True, tune=tune)
    info = plan.info()
    for _ in range(3):
        plan.run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(runs):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / runs
    dp = info["depth_points"]
    plan.close()
    for c in cols:
        c.close()
    rate = dp / (ms * 1e-3)
    return {"columns": len(problems), "runs": runs, "ms_per_F": ms, "depth_points_per_F": dp,
            "depth_points_per_s": rate, "alu_frac": rate * OPS_PER_DP / PEAK_VALU_OPS,
            "opac_depths": info["opac_depths"], "formal_wpb": info["formal_wpb"]}


def vel_bytes_per_eval(p):
    """Algorithmic HBM bytes of one column's F-mode velocity formal solution
    (k_formal_vel, which also takes the line rates): per ray-depth-point, the
    ray's V of every line window covering the frequency (8 B each); per
    (depth, frequency), the ray-independent opacity written and read back
    (32 B), the ingoing half of J written and read back (16 B) and J (8 B)."""
    g = p.grid
    cover = np.zeros(g.nnu)
    for t in range(p.atom.nline):
        cover[g.win_lo[t]:g.win_hi[t]] += 1.0
    nray = 2 * len(g.mu)
    return p.atmos.nz * (nray * 8.0 * cover.sum() + 56.0 * g.nnu)


def velocity_leg(ctx, nlte, ncol):
    """Velocity fields (Sect. 3.5).  The velocity-step column of the paper's
    test solved alone (FP64, Krylov tolerance 1e-2, stop at 1e-8; median of 3
    after a warm-up), and a batch of ncol velocity columns: FP64 batch solve
    (one warm-up, one timed), a profiled solve for the roofline of the F-mode
    velocity formal-solution launches (its algorithmic bytes over their
    time), the FP32-form batch solve (against the FP64 batch's populations),
    and F-only loops of the batch (FP64, FP32 form, and FP64 without the
    velocity field: same depths and frequencies)."""
    import torch
    out = {}
    p = S.chromo6_vel()
    col = nlte.Column(ctx, p, precision=nlte.FP64)
    o1 = nlte.default_opts(ftol=1e-8, rtol=1e-2, maxiter=80)
    col.solve(opts=o1)
    ts = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st, _ = col.solve(opts=o1)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    col.close()
    out["chromo6_vel_alone"] = {"dims": p.dims, "ms_per_solve": float(np.median(ts)) * 1e3,
                                "newton_iters": st["newton_iters"], "residual_calls": st["f_calls"],
                                "status": st["status"], "ftol": 1e-8, "rtol": 1e-2}
    probs = [S.batch6_vel_column(i) for i in range(ncol)]
    cols = [nlte.Column(ctx, q, precision=nlte.FP64) for q in probs]
    ob = nlte.default_opts(ftol=1e-8, rtol=1e-3, maxiter=50, max_krylov_total=200)
    nlte.solve_batch(ctx, cols, ob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, bst, _ = nlte.solve_batch(ctx, cols, ob)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.profile(True)
    outs64, pst, _ = nlte.solve_batch(ctx, cols, ob)
    prof = ctx.read_profile()
    ctx.profile(False)
    ref64 = [o.cpu().numpy() for o in outs64]
    for c in cols:
        c.close()
    # the FP32 form of the same batch (stop at 1e-6, FP64 fallback after 12)
    cols32 = [nlte.Column(ctx, q, precision=nlte.FP32_FORM) for q in probs]
    o32 = nlte.default_opts(ftol=1e-6, rtol=1e-3, maxiter=50, max_krylov_total=200, fp64_fallback=12)
    nlte.solve_batch(ctx, cols32, o32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs32, st32, _ = nlte.solve_batch(ctx, cols32, o32)
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t0
    for c in cols32:
        c.close()
    f32c = np.array([s["f_calls"] for s in st32], dtype=np.float64)
    err32 = max(float(np.max(np.abs(o.cpu().numpy() / r - 1.0))) for o, r in zip(outs32, ref64))
    dp = np.array([q.depth_points() for q in probs], dtype=np.float64)
    bf = np.array([s["f_calls"] for s in bst], dtype=np.float64)
    own = np.array([s["f_calls"] - s["precond_calls"] for s in pst], dtype=np.float64)
    nbytes = float((own * np.array([vel_bytes_per_eval(q) for q in probs])).sum())
    achieved = nbytes / (prof["formal_f_ms"] * 1e-3) / 1e9 if prof["formal_f_ms"] > 0 else None
    out["batch"] = {
        "workload": f"{ncol} velocity columns (batch6 recipe with a 2-8 km/s velocity step, "
                    "depth-optimised, core-resolving line grid), FP64",
        "columns": ncol,
        "mean_nz": float(np.mean([q.atmos.nz for q in probs])),
        "mean_nnu": float(np.mean([q.grid.nnu for q in probs])),
        "ms_per_solve": el * 1e3,
        "depth_points_per_s": float((bf * dp).sum()) / el,
        "converged_fraction": float(np.mean([s["status"] == 0 for s in bst])),
        "columns_converged_per_s": float(np.sum([s["status"] == 0 for s in bst])) / el,
        "residual_calls_per_column": float(bf.mean()),
        "newton_iters_mean": float(np.mean([s["newton_iters"] for s in bst])),
        "kernel_ms_per_solve_profiled": {k: prof[k] for k in ("opacity_ms", "formal_ms", "depth_ms",
                                                              "assemble_ms", "solver_ms")},
    }
    out["batch_fp32_form"] = {
        "ms_per_solve": el32 * 1e3,
        "depth_points_per_s": float((f32c * dp).sum()) / el32,
        "converged_fraction": float(np.mean([s["status"] == 0 for s in st32])),
        "columns_converged_per_s": float(np.sum([s["status"] == 0 for s in st32])) / el32,
        "residual_calls_per_column": float(f32c.mean()),
        "fp64_fallback_fraction": float(np.mean([s["precision"] == 0 for s in st32])),
        "max_rel_error_vs_fp64_batch": err32,
    }
    out["roofline"] = {
        "kernel": "k_formal_vel<double, false, 5> (F-mode velocity formal solution: opacity made per ray, "
                  "line rates taken in the kernel)",
        "launches": prof["formal_f_launches"],
        "launch_avg_ms": prof["formal_f_ms"] / max(1, prof["formal_f_launches"]),
        "bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
        "frac": achieved / 8000.0 if achieved else None,
        "algorithmic_bytes_per_launch": nbytes / max(1, prof["formal_f_launches"]),
        "traffic": (TRAFFIC_VEL["bytes_per_launch"]
                    if TRAFFIC_VEL["source"] == kernel_source_hash(VEL_KERNEL_SOURCES)
                    and ncol == TRAFFIC_VEL["columns"] else None),
        "traffic_unit": "bytes per launch (mean)",
    }
    out["f_only_fp64"] = f_only(ctx, nlte, probs, nlte.FP64)
    out["f_only_fp32_form"] = f_only(ctx, nlte, probs, nlte.FP32_FORM)
    out["f_only_fp64_static_twin"] = f_only(ctx, nlte, [S.batch6_vel_column(i, static=True)
                                                        for i in range(ncol)], nlte.FP64)
    return out


def copy_calibration(nbytes=256 << 20, reps=3):
    """A plain elementwise copy (y = 1.0 * x, fp32) of known size: it reads and
    writes nbytes each, so HBM byte counters read for it give their scale."""
    import torch
    x = torch.rand(nbytes // 4, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))


def issue_rates(ctx, nlte):
    """The denominators of the VALU roofline, measured: lane operations per
    second of the FP32 and FP64 FMA, the FP32 exponential and reciprocal on a
    full device (nlte_issue_rate), the FP32 FMA's rate against the peak used
    for `peak`, and what an exponential or a reciprocal costs in FP32 FMA
    issue slots."""
    ops = {"fma_f32": nlte.PROBE_FMA_F32, "fma_f64": nlte.PROBE_FMA_F64,
           "exp_f32": nlte.PROBE_EXP_F32, "rcp_f32": nlte.PROBE_RCP_F32}
    r = {k: ctx.issue_rate(op, 16384) for k, op in ops.items()}
    out = {k: v for k, v in r.items()}
    out["unit"] = "lane-ops/s"
    out["fma_f32_vs_peak"] = r["fma_f32"] / PEAK_VALU_OPS
    out["exp_slots"] = r["fma_f32"] / r["exp_f32"]
    out["rcp_slots"] = r["fma_f32"] / r["rcp_f32"]
    print(f"[bench] issue rates: " + ", ".join(f"{k} {v:.3e}" for k, v in r.items()),
          file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch6", choices=list(WORKLOADS))
    ap.add_argument("--ncol", type=int, default=None)
    ap.add_argument("--rtol", type=float, default=1e-3)
    ap.add_argument("--max-krylov-total", type=int, default=200,
                    help="Krylov budget per column solve (0: none); bounds the cost of columns "
                         "that do not converge, which otherwise set the length of the batch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-fallback", type=int, default=12,
                    help="FP32-form columns not converged after this many Newton iterations "
                         "continue in FP64 (0: never)")
    ap.add_argument("--oracle-single", type=int, default=1,
                    help="also time the oracle on one core for the C1, C2 and C5 configurations")
    ap.add_argument("--fp64-batch", type=int, default=1,
                    help="also time the batch solve with every column in FP64 (the paper's precision)")
    ap.add_argument("--single-fp64", type=int, default=16,
                    help="columns of the workload also solved one at a time in FP64 (0: skip)")
    ap.add_argument("--f-only", type=int, default=1,
                    help="also time F-only loops (graph-replayed residual plans) of the workload "
                         "in FP32 form and FP64 and of the 11-level stress column")
    ap.add_argument("--bicgstab", type=int, default=1,
                    help="also time the batch solve with the BiCGSTAB inner solver (one solve "
                         "after one warm-up; 0: skip)")
    ap.add_argument("--tangent", type=int, default=1,
                    help="also time the batch solve with tangent-linear Jacobian-vector products "
                         "(one solve after one warm-up; 0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="measured window of the sustained served stream, after its warm-up "
                         "(0: skip serving)")
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0,
                    help="arrival rate of the overload probe (and of --serve-full)")
    ap.add_argument("--serve-probe-seconds", type=float, default=2.0,
                    help="arrival window of the overload probe that measures capacity")
    ap.add_argument("--serve-full", action="store_true",
                    help="serve --serve-rate arrivals for warm-up + window instead of the probe "
                         "and the sustained run (long: the queue grows when the rate exceeds "
                         "capacity)")
    ap.add_argument("--serve-budget-gb", type=float, default=96.0)
    ap.add_argument("--serve-max-active", type=int, default=2048)
    ap.add_argument("--launch", default="eager", choices=["eager", "tune", "graph", "graph+tune"],
                    help="step replay of the timed batch solves (HIP graphs, launch-shape tuner); "
                         "graph replay of the full 4096-column batch is not cleared for use "
                         "(a host-side crash in its second solve is not understood yet)")
    ap.add_argument("--profile-fonly", default=None,
                    choices=["batch6_fp32", "batch6_fp64", "chromo11_fp32", "chromo11_fp64",
                             "chromo11_fp32_scan", "chromo11_fp64_scan"],
                    help="only run that F-only loop (--runs evaluations) and print its figures: "
                         "a short command for profilers")
    ap.add_argument("--runs", type=int, default=100)
    ap.add_argument("--issue-rates", type=int, default=1,
                    help="measure the VALU issue rates behind the roofline's peak (0: skip)")
    ap.add_argument("--velocity", type=int, default=512,
                    help="columns of the velocity-field batch leg (0: skip the velocity leg)")
    ap.add_argument("--velocity-only", action="store_true",
                    help="only run the velocity leg and print its figures")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy kernel (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile_fonly:
        from paper_2406_17234_amd import nlte
        ctx = nlte.Context(0)
        name = args.profile_fonly
        probs = ([S.batch6_column(i) for i in range(args.ncol or 4096)]
                 if name.startswith("batch6") else [S.chromo11()])
        prec = (nlte.FP64 if "fp64" in name else nlte.FP32_FORM) | (nlte.DEPTH_SCAN if "scan" in name else 0)
        print(json.dumps({name: f_only(ctx, nlte, probs, prec, runs=args.runs)}))
        return
    if args.velocity_only:
        from paper_2406_17234_amd import nlte
        print(json.dumps({"velocity": velocity_leg(nlte.Context(0), nlte, args.velocity or 512)}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); columns are "
              f"independent, so several GPUs would each run their own share of the batch.",
              file=sys.stderr)
        sys.exit(2)

    desc, maker, ncol_def, prec, ftol = WORKLOADS[args.workload]
    ncol = args.ncol or ncol_def
    t0 = time.perf_counter()
    problems = [maker(i) for i in range(ncol)]
    gen_s = time.perf_counter() - t0
    print(f"[bench] generated {ncol} columns in {gen_s:.1f} s", file=sys.stderr, flush=True)

    cpu = None
    oracle_single = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, ncol, ftol, args.rtol)
        print(f"[bench] cpu baseline {cpu['value']:.3e} dp/s", file=sys.stderr, flush=True)
        if args.oracle_single:
            oracle_single = oracle_single_columns()
            print(f"[bench] oracle single columns: " +
                  ", ".join(f"{k} {v.get('s_per_solve', v['s_per_call']):.2f} s"
                            for k, v in oracle_single.items()), file=sys.stderr, flush=True)

    import torch
    from paper_2406_17234_amd import nlte
    ctx = nlte.Context(0)
    rates = None
    if args.issue_rates:
        global OPS_PER_DP
        rates = issue_rates(ctx, nlte)
        OPS_PER_DP = 10.0 + 0.5 * rates["exp_slots"] + 0.5 * rates["rcp_slots"]
    t0 = time.perf_counter()
    cols = [nlte.Column(ctx, p, precision=prec) for p in problems]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"[bench] created {ncol} columns in {setup_s:.1f} s", file=sys.stderr, flush=True)
    dp_col = np.array([p.depth_points() for p in problems], dtype=np.float64)
    launch = {"eager": 0, "tune": nlte.NLTE_SOLVE_TUNE, "graph": nlte.NLTE_SOLVE_GRAPH,
              "graph+tune": nlte.NLTE_SOLVE_GRAPH | nlte.NLTE_SOLVE_TUNE}[args.launch]
    opts = nlte.default_opts(ftol=ftol, rtol=args.rtol, maxiter=50,
                             max_krylov_total=args.max_krylov_total,
                             fp64_fallback=args.fp64_fallback, launch=launch)

    for w in range(args.warmup):
        _, st, rc = nlte.solve_batch(ctx, cols, opts)
        print(f"[bench] warmup {w} rc={rc}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats_all = []
    for k in range(args.steps):
        batch_outs, st, rc = nlte.solve_batch(ctx, cols, opts)
        stats_all.append(st)
        print(f"[bench] step {k} rc={rc}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    replay = ctx.read_profile()
    # the same solve launched eagerly (no graphs, one wave per formal
    # workgroup), and once more with per-phase HIP events (eager by necessity)
    # for the phase breakdown and the roofline of the F-mode formal launches
    opts_e = nlte.default_opts(ftol=ftol, rtol=args.rtol, maxiter=50,
                               max_krylov_total=args.max_krylov_total,
                               fp64_fallback=args.fp64_fallback, launch=0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nlte.solve_batch(ctx, cols, opts_e)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t1) * 1e3
    ctx.profile(True)
    _, st_prof, _ = nlte.solve_batch(ctx, cols, opts_e)
    prof = ctx.read_profile()
    ctx.profile(False)
    print(f"[bench] eager solve {eager_ms:.0f} ms; replayed {elapsed / args.steps * 1e3:.0f} ms "
          f"(wpb {replay['last_formal_wpb']}, tune {replay['last_tune_ms']})", file=sys.stderr, flush=True)

    f_calls = np.array([[s["f_calls"] for s in st] for st in stats_all], dtype=np.float64)
    conv = np.array([[s["status"] == 0 for s in st] for st in stats_all])
    total_dp = float((f_calls * dp_col[None, :]).sum())
    # depth-points of the profiled solve's F-mode evaluations in the columns'
    # own precision (the launches on the solve stream that formal_f_ms
    # times); FP64 evaluations of fallback columns are all subtracted, a
    # slight undercount
    pf = np.array([s["f_calls"] for s in st_prof], dtype=np.float64)
    ppc = np.array([s["precond_calls"] for s in st_prof], dtype=np.float64)
    p64 = np.array([s["fp64_evals"] for s in st_prof], dtype=np.float64)
    own = pf - ppc - (p64 if prec == 1 else 0.0)
    fmode_dp = float((np.maximum(own, 0.0) * dp_col).sum())
    ms_per_step = elapsed / args.steps * 1e3
    value = total_dp / elapsed
    achieved = (fmode_dp * OPS_PER_DP / (prof["formal_f_ms"] * 1e-3) / 1e12
                if prof["formal_f_ms"] > 0 else None)
    peak = PEAK_VALU_OPS / 1e12
    tr = TRAFFIC.get(args.workload)
    traffic = tr["bytes_per_launch"] if (tr and tr["source"] == kernel_source_hash()
                                         and args.ncol is None) else None
    out = {
        "metric": "formal-solution depth-points/s",
        "value": value,
        "unit": "depth-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "columns": ncol,
                   "ftol": ftol, "rtol": args.rtol, "maxiter": 50,
                   "max_krylov_total": args.max_krylov_total, "fp64_fallback": args.fp64_fallback,
                   "mean_nz": float(np.mean([p.atmos.nz for p in problems])),
                   "mean_nnu": float(np.mean([p.grid.nnu for p in problems]))},
        "columns_converged_per_s": float(conv.sum()) / elapsed,
        "converged_fraction": float(conv.mean()),
        "residual_calls_per_column": float(f_calls.mean()),
        "newton_iters_mean": float(np.mean([[s["newton_iters"] for s in st] for st in stats_all])),
        "fp64_fallback_fraction": float(np.mean([[s["precision"] == 0 and prec == 1 for s in st]
                                                 for st in stats_all])),
        "launch": {"mode": args.launch, "formal_wpb": replay["last_formal_wpb"],
                   "tune_ms_per_step_wpb_1_2_4": replay["last_tune_ms"],
                   "graph_captures_per_solve": replay["last_captures"],
                   "eager_ms_per_solve": eager_ms},
        "kernel_ms_per_solve_eager_profiled": {k: prof[k] for k in
                                               ("opacity_ms", "formal_ms", "depth_ms",
                                                "assemble_ms", "solver_ms")},
        "roofline": {
            "kernel": ("k_formal<float, false, 5>" if prec == 1 else "k_formal<double, false, 5>") +
                      " (F-mode depth recursion; in launches over at least 4096 chunks it"
                      " also makes the opacity, not counted in achieved)",
            "launches": prof["formal_f_launches"],
            "launch_avg_ms": prof["formal_f_ms"] / max(1, prof["formal_f_launches"]),
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TOP/s",
            "frac": (achieved / peak) if achieved else None,
            "ops_per_depth_point": OPS_PER_DP,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (mean)",
        },
        "cpu_baseline": cpu,
    }
    if rates:
        out["roofline"]["issue_rates_measured"] = rates
    def other_solve(label, **kw):
        # the same batch solved with another inner solver or product: one
        # warm-up solve, one timed solve
        o2 = nlte.default_opts(ftol=ftol, rtol=args.rtol, maxiter=50,
                               max_krylov_total=args.max_krylov_total,
                               fp64_fallback=args.fp64_fallback, launch=launch, **kw)
        nlte.solve_batch(ctx, cols, o2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, bst, _ = nlte.solve_batch(ctx, cols, o2)
        torch.cuda.synchronize()
        bel = time.perf_counter() - t0
        bf = np.array([s["f_calls"] for s in bst], dtype=np.float64)
        print(f"[bench] {label} solve {bel * 1e3:.0f} ms", file=sys.stderr, flush=True)
        return {
            "ms_per_solve": bel * 1e3,
            "depth_points_per_s": float((bf * dp_col).sum()) / bel,
            "converged_fraction": float(np.mean([s["status"] == 0 for s in bst])),
            "columns_converged_per_s": float(np.sum([s["status"] == 0 for s in bst])) / bel,
            "residual_calls_per_column": float(bf.mean()),
            "newton_iters_mean": float(np.mean([s["newton_iters"] for s in bst])),
            "jacobian_products_per_column": float(np.mean([s["krylov_iters"] for s in bst])),
            "fp64_fallback_fraction": float(np.mean([s["precision"] == 0 and prec == 1
                                                     for s in bst])),
        }

    if args.bicgstab:
        out["bicgstab"] = other_solve("BiCGSTAB", krylov_method=nlte.KRYLOV_BICGSTAB)
    if args.tangent:
        # residual calls count each tangent product as one (a formal solution
        # carrying its derivative)
        out["tangent_jv"] = other_solve("tangent-product", jv_method=nlte.JV_TANGENT)
    if args.fp64_batch and prec == 1:
        # the same batch with every column in FP64 (the paper's precision),
        # same stop and options, one warm-up solve and one timed solve
        cols64 = [nlte.Column(ctx, p, precision=nlte.FP64) for p in problems]
        o64 = nlte.default_opts(ftol=ftol, rtol=args.rtol, maxiter=50,
                                max_krylov_total=args.max_krylov_total, launch=launch)
        nlte.solve_batch(ctx, cols64, o64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st64, _ = nlte.solve_batch(ctx, cols64, o64)
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t0
        f64 = np.array([s["f_calls"] for s in st64], dtype=np.float64)
        out["fp64_batch"] = {
            "ms_per_solve": el64 * 1e3,
            "depth_points_per_s": float((f64 * dp_col).sum()) / el64,
            "converged_fraction": float(np.mean([s["status"] == 0 for s in st64])),
            "columns_converged_per_s": float(np.sum([s["status"] == 0 for s in st64])) / el64,
            "residual_calls_per_column": float(f64.mean()),
            "newton_iters_mean": float(np.mean([s["newton_iters"] for s in st64])),
        }
        print(f"[bench] FP64 batch solve {el64 * 1e3:.0f} ms", file=sys.stderr, flush=True)
        for c in cols64:
            c.close()
    if args.f_only:
        for c in cols:
            c.close()
        cols = []
        fo = {}
        for name, probs, prec in [("batch6_fp32", problems, nlte.FP32_FORM),
                                  ("batch6_fp64", problems, nlte.FP64),
                                  ("chromo11_fp32", [S.chromo11()], nlte.FP32_FORM),
                                  ("chromo11_fp64", [S.chromo11()], nlte.FP64),
                                  ("chromo11_fp32_scan", [S.chromo11()], nlte.FP32_FORM | nlte.DEPTH_SCAN),
                                  ("chromo11_fp64_scan", [S.chromo11()], nlte.FP64 | nlte.DEPTH_SCAN)]:
            fo[name] = f_only(ctx, nlte, probs, prec)
            print(f"[bench] F-only {name}: {fo[name]['depth_points_per_s']:.3e} dp/s", file=sys.stderr, flush=True)
        out["f_only"] = fo
    if args.single_fp64 > 0:
        out["single_column_fp64"] = single_fp64(ctx, nlte, problems[:args.single_fp64], args.rtol,
                                                batch_outs[:args.single_fp64])
    out["single_column_latency"] = gpu_single_columns(ctx, nlte)
    if oracle_single:
        out["oracle_single_column_1core"] = oracle_single
    if args.velocity > 0:
        for c in cols or []:
            c.close()
        cols = None
        out["velocity"] = velocity_leg(ctx, nlte, args.velocity)
        print(f"[bench] velocity: alone {out['velocity']['chromo6_vel_alone']['ms_per_solve']:.0f} ms, "
              f"batch {out['velocity']['batch']['ms_per_solve']:.0f} ms", file=sys.stderr, flush=True)
    if args.serve_seconds > 0:
        for c in cols or []:
            c.close()
        cols = None
        out["served"] = serve_stream(ctx, nlte, args, 1e-6)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
