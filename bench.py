#!/usr/bin/env python3
"""Benchmark of the FRG flow-diagram quadrature on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = one evaluation of the scale-up workload (d = 3, exponential
regulator, 4096 momenta log-spaced in [1e-4, 20] x 512 masses uniform in
[-0.9, 10], 128 radial x 32 angular Gauss-Legendre nodes: 2 097 152
integrals, 8.59e9 integrand evaluations) through frg_integrate_grid, inputs
resident in HBM.  Prints ONE JSON line: throughput in integrand evaluations
per second (plus integrals/s), the roofline of the dominant kernel, the FP64
oracle timed on the host cores on a bounded sample, and secondary figures
measured outside the timed region (uneven batched vs plain launches,
compensated FP32, served-flow latency) when their parts are built.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ALU roofline of the FP64 path.  FP64 rate of MI355X: 78.6 TFLOP/s, i.e.
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 FMA/s, the same on the
# vector units and on the FP64 matrix cores, which share it (a kernel that
# mixes the two takes the sum of their times).  Floor of the per-evaluation
# work of the grid kernel: for one radial node and a group of G angular terms
# of a lane row, c/(Hq + delta)^2 sum_k mu_k/(delta + H_k) = N(delta)/P(delta)
# with per-momentum polynomial coefficients, so each (term, mass) costs one
# multiply-add of P and one of N (power sums over 16-mass tiles on the matrix
# cores, or nested on the vector units); the two extra powers of the radial
# factor, the reciprocal of P, its Newton step and the accumulation are
# shared by the G = 32 terms of a group and the coefficient build by every
# mass of the momentum, and are left out of the floor: 2 FMAs per eval.
VALU_LANE_CYCLES = 256 * 4 * 16 * 2.4e9
# HBM bytes per grid-kernel launch from rocprofv3 FETCH_SIZE / WRITE_SIZE,
# scaled by a 1 GiB device copy read the same way (fetch x2.00, write x1.00):
# 461.0 KiB x 2.00 + 16384 KiB x 1.00.
TRAFFIC = 461.0 * 1024 * 2.00 + 16384 * 1024 * 1.00
CYCLES_PER_EVAL_FLOOR = 2
PEAK_EVALS = VALU_LANE_CYCLES / CYCLES_PER_EVAL_FLOOR
TRAFFIC_SOURCE = ("rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of grid_coef_kernel on this workload "
                  "(profiles/grid_kernel_scaleup_d3_hbm_traffic.md), not measured in this run")
# Point-list (uneven sets) roofline: the algorithmic FP64 vector work of one
# evaluation with the regulator evaluated per term, taken at the middle of the
# estimated ranges -- exponential: one expm1-class transcendental, one
# division, one reciprocal and ~3 FMA/add, 35-45 instructions -> 40;
# Litim: compare/select, one reciprocal, ~3 FMA/add, 8-12 -> 10 -- weighted by
# the workload's evaluations per regulator.
OPS_PER_EVAL = {0: 40.0, 1: 10.0}
# FP64 vector instructions per evaluation of points_persistent_kernel on the
# uneven sets, from SQ_INSTS_VALU x 64 / evaluations
# (profiles/points_persistent_kernel_uneven_sets.md).
POINT_VALU_PER_EVAL_PROFILE = 21.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device-to-device copy of 1 GiB (PMC traffic calibration)")
    ap.add_argument("--only", choices=["uneven64", "uneven32", "tab4096", "tab1m", "tab1mcache", "tabsweep", "pflow",
                                       "vertex", "fvlpa", "serving"],
                    default=None,
                    help="profiling aid: run only --steps persistent launches of the uneven sets "
                         "(FP64 or FP32C), --steps momentum-flow "
                         "or finite-volume LPA solves or vertex-diagram calls, --steps calls "
                         "of the tabulated variant (rows of 4096 or 2^20 nodes, the default "
                         "form; tab1mcache: 2^20 nodes, cache-streamed; tabsweep: both long-row "
                         "forms over rows, row lengths and momenta), or --steps "
                         "served flow requests (after --warmup more), and print their timing")
    return ap.parse_args()


def only_uneven(prec_name, steps, warmup):
    import torch
    from paper_2607_24908_amd import frg, workloads
    prec = frg.FRG_PREC_FP64 if prec_name == "uneven64" else frg.FRG_PREC_FP32C
    ctx = frg.frg_create(0)
    sets = workloads.uneven_sets(seed=0)
    ds = [dict(quad=frg.make_quad(s.quad.d, s.quad.reg, s.quad.k, s.quad.q_max, s.quad.n_r,
                                  s.quad.n_a, prec),
               p=torch.as_tensor(s.p, device="cuda"), m2=torch.as_tensor(s.m2, device="cuda"),
               out=torch.empty(s.p.size, dtype=torch.float64, device="cuda")) for s in sets]
    evals = sum(s.n_evals for s in sets)
    for _ in range(warmup):
        frg.frg_integrate(ctx, ds, flags=frg.FRG_PERSISTENT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        frg.frg_integrate(ctx, ds, flags=frg.FRG_PERSISTENT)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    frg.frg_destroy(ctx)
    print(json.dumps({"only": prec_name, "steps": steps, "ms_per_launch": dt * 1e3,
                      "evals_per_s": evals / dt}), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_info():
    model, flags = "unknown", []
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                if line.startswith("flags"):
                    fl = line.split(":", 1)[1].split()
                    flags = sorted(x for x in fl if x.startswith(("avx", "sse4", "fma", "amx")))
                    break
    except OSError:
        pass
    return model, flags


def cpu_baseline(w, gpu_out, checks, workloads):
    """The oracle leg.  The FP64 oracle, as it stands: OpenMP over points on
    the host cores on 1/4 of the workload (every 4th mass for all momenta,
    about 20-30 core-seconds), and single-threaded on 1/256 of it (every 16th
    momentum of that sample).  The 524 288 results of the first run are
    compared with the GPU's results of the timed region, element by element;
    so are the GPU results of the plain d = 4 grid, the 256 uneven sets and
    (as a per-result histogram) the compensated-FP32 precision workload."""
    import oracle
    q = w.quad
    m2 = w.m2[::4]
    P = np.repeat(w.p, m2.size)
    M = np.tile(m2, w.p.size)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 64))
    t0 = time.perf_counter()
    ref = oracle.integrate(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, P, M, threads=cores)
    dt = time.perf_counter() - t0
    evals = P.size * q.n_r * q.n_a
    got = gpu_out.reshape(w.p.size, w.m2.size)[:, ::4].ravel()
    rel = np.abs(got - ref) / np.abs(ref)
    parity = {"max_rel_err": float(rel.max()), "median_rel_err": float(np.median(rel)),
              "compared": int(rel.size), "tol": 1e-12,
              "what": "every 4th mass x all 4096 momenta of the timed region's output vs the "
                      "FP64 oracle"}
    P1 = np.repeat(w.p[::16], m2.size)
    M1 = np.tile(m2, w.p[::16].size)
    t1 = time.perf_counter()
    oracle.integrate(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, P1, M1, threads=1)
    dt1 = time.perf_counter() - t1
    ev1 = P1.size * q.n_r * q.n_a
    parity["others"] = oracle_checks(oracle, checks, workloads, cores)
    model, flags = cpu_info()
    base = {"value": evals / dt, "unit": "integrand evals/s", "cores": cores, "kind": "oracle",
            "sample": f"1/4 of the workload: all {w.p.size} momenta x every 4th mass "
                      f"({P.size} integrals, {evals:.3e} evals), {dt:.2f} s wall on {cores} "
                      f"threads; single thread: 1/256 ({P1.size} integrals), {dt1:.2f} s",
            "single_thread_value": ev1 / dt1, "cpu_model": model, "simd_flags": flags,
            "compiled": "-O2 -fno-fast-math -ffp-contract=off, OpenMP over points"}
    return base, parity


def oracle_checks(oracle, checks, workloads, cores):
    """Element-by-element comparison of GPU results kept by `secondary` with
    the FP64 oracle; the compensated-FP32 results as a log-binned histogram of
    the relative error of every result."""
    out = {}
    if "plain_d4" in checks:
        w = workloads.plain_d4()
        q = w.quad
        ref = oracle.integrate_grid(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, w.p, w.m2).ravel()
        out["plain_d4"] = {"max_rel_err": float(np.max(np.abs(checks["plain_d4"] - ref) / ref)),
                           "compared": int(ref.size)}
    if "uneven_seed0" in checks:
        worst, n = 0.0, 0
        f32 = checks.get("fp32c_uneven_seed0")
        w32, n32, above, bmax = 0.0, 0, 0, 0.0
        for i, (s, got) in enumerate(zip(workloads.uneven_sets(seed=0), checks["uneven_seed0"])):
            q = s.quad
            ref = oracle.integrate(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, s.p, s.m2, threads=cores)
            worst = max(worst, float(np.max(np.abs(got - ref) / ref)))
            n += ref.size
            if f32:
                o32, err, used = f32[i]
                rel = np.abs(o32 - ref) / ref
                w32 = max(w32, float(rel.max()))
                sel = used == 0
                n32 += int(sel.sum())
                above += int(np.sum(rel[sel] > err[sel] + 1e-13))
                bmax = max(bmax, float(err[sel].max()) if sel.any() else 0.0)
        out["uneven_sets_seed0"] = {"max_rel_err": worst, "compared": n}
        if f32:
            out["fp32c_uneven_sets_seed0"] = {
                "max_rel_err": w32, "compared": n, "fp32_returned": n32,
                "fp32_results_above_their_bound": above, "max_bound_returned": bmax, "tol": 1e-7}
    if checks.get("precision_d4"):
        edges = 10.0 ** np.arange(-17, -3)
        rels, ests, fp32 = [], [], []
        for wk, o32, err, used in checks["precision_d4"]:
            q = wk.quad
            ref = oracle.integrate_grid(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a, wk.p,
                                        wk.m2).ravel()  # the point order of np.repeat/np.tile
            rels.append(np.abs(o32 - ref) / ref)
            ests.append(err)
            fp32.append(used == 0)
        rel, est, f32 = np.concatenate(rels), np.concatenate(ests), np.concatenate(fp32)
        counts, _ = np.histogram(np.clip(rel, 1e-17, 1e-4 * 0.999), bins=edges)
        out["fp32c_precision_d4_seeds012"] = {
            "results": int(rel.size), "fp32_returned": int(f32.sum()),
            "max_rel_err": float(rel.max()),
            "max_rel_err_fp32_returned": float(rel[f32].max()) if f32.any() else None,
            "fp32_results_above_their_bound": int(np.sum(rel[f32] > est[f32] + 1e-13)),
            "histogram_rel_err": {f"[1e{int(np.log10(a))},1e{int(np.log10(b))})": int(c)
                                  for a, b, c in zip(edges[:-1], edges[1:], counts)},
            "tol": 1e-7}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(integral sets and flows would shard across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)
    if args.only in ("pflow", "vertex", "fvlpa"):
        import torch
        from paper_2607_24908_amd import frg, workloads
        ctx = frg.frg_create(0)
        fn = {"pflow": momentum_flow, "vertex": vertex, "fvlpa": fv_lpa}[args.only]
        r = fn(ctx, frg, workloads, torch, reps=args.steps)
        print(json.dumps({"only": args.only, **r}), flush=True)
        return
    if args.only == "serving":
        from paper_2607_24908_amd import frg, workloads
        r = serving(frg, workloads, n_warm=args.warmup, n_timed=args.steps)
        print(json.dumps({"only": args.only, **r}), flush=True)
        return
    if args.only == "tabsweep":
        import torch
        from paper_2607_24908_amd import frg, workloads
        tab_forms_sweep(frg.frg_create(0), frg, workloads, torch)
        return
    if args.only in ("tab4096", "tab1m", "tab1mcache"):
        import torch
        from paper_2607_24908_amd import frg, workloads
        ctx = frg.frg_create(0)
        if args.only == "tab1mcache":
            frg.frg_tune_set(ctx, "tab_seg", 0)
        n_s = 4096 if args.only == "tab4096" else 1 << 20
        r = tabulated(ctx, frg, workloads, torch, which=(n_s,), reps=args.steps)
        print(json.dumps({"only": args.only, **r[f"tabulated_{n_s}"]}), flush=True)
        return
    if args.only:
        only_uneven(args.only, args.steps, args.warmup)
        return
    import torch
    from paper_2607_24908_amd import frg, workloads
    assert torch.cuda.is_available(), "no GPU"
    ctx = frg.frg_create(0)
    w = workloads.scaleup_d3()
    q = w.quad
    quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
    P = torch.as_tensor(w.p, dtype=torch.float64, device="cuda")
    M = torch.as_tensor(w.m2, dtype=torch.float64, device="cuda")
    out = torch.empty(w.n_integrals, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    log(f"workload {w.name}: {w.n_integrals} integrals, {w.n_evals:.3e} evals")
    for _ in range(args.warmup):
        frg.frg_integrate_grid(ctx, quad, P, M, out, stream=stream)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} done")
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        frg.frg_integrate_grid(ctx, quad, P, M, out, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"timed {args.steps} steps: {gpu_ms:.3f} ms/step (events), wall {wall:.3f} s")
    res = out.cpu().numpy()
    assert np.all(np.isfinite(res)) and np.all(res > 0), "non-finite results"
    ms_step = wall * 1e3 / args.steps
    evals_s = w.n_evals / (ms_step * 1e-3)
    kernel_s = gpu_ms * 1e-3
    achieved = w.n_evals / kernel_s / 1e9
    line = {
        "metric": "integrand evals/s (FP64, plain scale-up d=3 grid)",
        "value": evals_s,
        "unit": "integrand evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seedless deterministic grid: log-spaced p, uniform m^2)",
        "config": {"workload": w.name, "n_p": int(w.p.size), "n_m": int(w.m2.size), "d": q.d,
                   "regulator": "exp", "k": q.k, "q_max": q.q_max, "n_radial": q.n_r,
                   "n_angular": q.n_a, "evals_per_step": int(w.n_evals),
                   "integrals_per_step": int(w.n_integrals), "entry": "frg_integrate_grid"},
        "integrals_per_s": w.n_integrals / (ms_step * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_EVALS / 1e9,
                     "unit": "Geval/s", "frac": achieved * 1e9 / PEAK_EVALS, "traffic": TRAFFIC,
                     "kernel": "grid_coef_kernel<exp> (16-mass tiles, FP64 matrix cores)",
                     "kernel_ms": gpu_ms,
                     "evals_per_launch": int(w.n_evals), "traffic_unit": "bytes per launch",
                     "traffic_source": TRAFFIC_SOURCE,
                     "peak_basis": "FP64 3.93e13 FMA/s (vector or matrix) / 2 FMAs per eval"},
    }
    checks = {}
    if not args.no_secondary:
        line["secondary"] = secondary(ctx, frg, workloads, torch, checks)
    if args.copy_calibration:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"], line["parity"] = cpu_baseline(w, res, checks, workloads)
        log(f"parity vs oracle on {line['parity']['compared']} results: max rel err "
            f"{line['parity']['max_rel_err']:.2e}")
        others = line["parity"]["others"]
        worst64 = max([line["parity"]["max_rel_err"]] +
                      [v["max_rel_err"] for k, v in others.items() if not k.startswith("fp32c")])
        if not worst64 <= 1e-12:
            print(json.dumps(line), flush=True)
            sys.exit("FP64 parity against the oracle exceeds 1e-12")
    frg.frg_destroy(ctx)
    print(json.dumps(line), flush=True)


def timed(fn, torch, reps=5):
    """Seconds per call of fn over `reps` calls after max(2, reps // 2)
    warm-up calls (the clock ramps up under load)."""
    for _ in range(max(2, reps // 2)):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def events_time(fn, torch, reps=30, warm=3):
    """Seconds per call from HIP events recorded on the current stream around
    `reps` back-to-back calls (the calls enqueue on that stream)."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps


def uneven_sets_figures(ctx, frg, workloads, torch):
    """Batched uneven sets (256 sets, seed 0): one persistent launch replayed
    from a HIP graph against one plain launch per set, the roofline of the
    persistent kernel, and the autotuned launch shape against the default."""
    import tempfile
    sets = workloads.uneven_sets(seed=0)
    evals = sum(s.n_evals for s in sets)
    n_int = sum(s.p.size for s in sets)
    ds = []
    for s in sets:
        q = s.quad
        ds.append(dict(quad=frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a),
                       p=torch.as_tensor(s.p, device="cuda"), m2=torch.as_tensor(s.m2, device="cuda"),
                       out=torch.empty(s.p.size, dtype=torch.float64, device="cuda")))
    arr = frg.make_set_array(ds)
    st = torch.cuda.current_stream().cuda_stream

    def call(flags):
        return lambda: frg.frg_integrate_array(ctx, arr, len(ds), flags=flags, stream=st)

    t_plain = timed(call(frg.FRG_PLAIN), torch)
    t_pers = timed(call(frg.FRG_PERSISTENT), torch, reps=20)
    t_graph = events_time(call(frg.FRG_PERSISTENT | frg.FRG_GRAPH), torch, reps=30)
    default_out = torch.cat([d["out"] for d in ds])
    # the project's autotuner: time the candidate shapes of this key once,
    # keep the fastest, replay with it; the results must not change
    cache = os.path.join(tempfile.gettempdir(), f"frg_autotune_{os.getpid()}.txt")
    frg.frg_autotune(ctx, 1, cache)
    call(frg.FRG_PERSISTENT)()
    frg.frg_autotune(ctx, 0, None)
    t_tuned = events_time(call(frg.FRG_PERSISTENT | frg.FRG_GRAPH), torch, reps=30)
    tuned_same = bool(torch.equal(torch.cat([d["out"] for d in ds]), default_out))
    try:
        tuned_line = open(cache).read().strip().splitlines()[-1]
        os.remove(cache)
    except OSError:
        tuned_line = ""
    ops = sum(s.n_evals * OPS_PER_EVAL[s.quad.reg] for s in sets) / evals
    peak = VALU_LANE_CYCLES / ops
    achieved = evals / t_graph
    roof = {"bound": "alu", "achieved": achieved / 1e9, "peak": peak / 1e9, "unit": "Geval/s",
            "frac": achieved / peak, "traffic": None,
            "kernel": "points_persistent_kernel<false> (graph replay incl. its counter reset)",
            "kernel_ms": t_graph * 1e3, "evals_per_launch": int(evals),
            "ops_per_eval": ops,
            "peak_basis": "FP64 vector 3.93e13 lane-ops/s / ops per eval (exponential 40, Litim 10, "
                          "weighted by this set mix)",
            "valu_insts_per_eval_profile": POINT_VALU_PER_EVAL_PROFILE,
            "valu_busy_est": achieved * POINT_VALU_PER_EVAL_PROFILE / VALU_LANE_CYCLES}
    out = {"sets": len(sets), "integrals": n_int, "evals": evals,
           "plain_evals_per_s": evals / t_plain, "persistent_evals_per_s": evals / t_pers,
           "graph_evals_per_s": evals / t_graph, "graph_integrals_per_s": n_int / t_graph,
           "graph_ms": t_graph * 1e3, "batched_over_plain": t_plain / t_graph,
           "roofline": roof,
           "autotuned": {"graph_ms": t_tuned * 1e3, "default_graph_ms": t_graph * 1e3,
                         "tuned_choice": tuned_line, "results_bitwise_equal": tuned_same}}
    log(f"uneven sets: plain {evals / t_plain:.3e}, persistent {evals / t_pers:.3e}, graph "
        f"{evals / t_graph:.3e} evals/s (frac {achieved / peak:.2f} of {peak:.3e}); tuned graph "
        f"{t_tuned * 1e3:.3f} ms vs {t_graph * 1e3:.3f} ms, same bits {tuned_same}")
    return out, ds


def secondary(ctx, frg, workloads, torch, checks):
    """Figures for the other workloads, measured after the timed region.
    `checks` receives GPU results that the oracle leg compares."""
    sec = {}
    sec["uneven_sets_seed0"], ds = uneven_sets_figures(ctx, frg, workloads, torch)
    checks["uneven_seed0"] = [d["out"].cpu().numpy() for d in ds]
    sets = workloads.uneven_sets(seed=0)
    evals = sum(s.n_evals for s in sets)
    n_int = sum(s.p.size for s in sets)
    t_plain = evals / sec["uneven_sets_seed0"]["plain_evals_per_s"]
    t_graph = evals / sec["uneven_sets_seed0"]["graph_evals_per_s"]
    # plain d = 4 grid: latency of one small call
    w = workloads.plain_d4()
    q = w.quad
    quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
    P = torch.as_tensor(w.p, device="cuda")
    M = torch.as_tensor(w.m2, device="cuda")
    out = torch.empty(w.n_integrals, dtype=torch.float64, device="cuda")
    t1 = timed(lambda: frg.frg_integrate_grid(ctx, quad, P, M, out), torch, reps=50)
    sec["plain_d4"] = {"ms_per_call": t1 * 1e3, "evals_per_s": w.n_evals / t1,
                       "integrals_per_s": w.n_integrals / t1}
    checks["plain_d4"] = out.cpu().numpy()
    # compensated FP32 on the point kernel (uneven sets): the exponential
    # of the regulator is evaluated per term there, which is what FP32 replaces
    ds32 = []
    for s, d in zip(sets, ds):
        q = s.quad
        ds32.append(dict(quad=frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a,
                                            frg.FRG_PREC_FP32C), p=d["p"], m2=d["m2"],
                         out=torch.empty_like(d["out"]), err_est=torch.empty_like(d["out"]),
                         used_fp64=torch.empty(d["out"].numel(), dtype=torch.uint8,
                                               device="cuda")))
    t32 = timed(lambda: frg.frg_integrate(ctx, ds32, flags=frg.FRG_PLAIN), torch)
    arr32 = frg.make_set_array(ds32)
    st = torch.cuda.current_stream().cuda_stream
    t32g = events_time(lambda: frg.frg_integrate_array(ctx, arr32, len(ds32),
                                                       flags=frg.FRG_PERSISTENT | frg.FRG_GRAPH,
                                                       stream=st), torch, reps=30)
    torch.cuda.synchronize()
    checks["fp32c_uneven_seed0"] = [(a["out"].cpu().numpy(), a["err_est"].cpu().numpy(),
                                     a["used_fp64"].cpu().numpy()) for a in ds32]
    exp_work = sum(s.n_evals for s in sets if s.quad.reg == workloads.REG_EXP)
    work32 = sum(int((u == 0).sum()) * s.quad.n_r * s.quad.n_a
                 for s, (_, _, u) in zip(sets, checks["fp32c_uneven_seed0"]))
    n32 = sum(int((u == 0).sum()) for _, _, u in checks["fp32c_uneven_seed0"])
    sec["fp32c_uneven_sets_seed0"] = {
        "fp32c_plain_evals_per_s": evals / t32, "fp32c_graph_evals_per_s": evals / t32g,
        "fp32c_graph_integrals_per_s": n_int / t32g, "fp64_plain_evals_per_s": evals / t_plain,
        "fp64_graph_evals_per_s": evals / t_graph, "graph_speedup_vs_fp64": t_graph / t32g,
        "fp32_returned": n32, "fp32_share_of_exp_work": work32 / exp_work,
        "max_bound_returned": max(float(e[u == 0].max()) if (u == 0).any() else 0.0
                                  for _, e, u in checks["fp32c_uneven_seed0"]),
        "note": "Litim points and points whose bound exceeds 1e-7 are FP64; the oracle leg "
                "compares every result"}
    log(f"fp32c uneven: plain {evals / t32:.3e}, graph {evals / t32g:.3e} evals/s "
        f"(fp64 plain {evals / t_plain:.3e}, graph {evals / t_graph:.3e}), "
        f"FP32 share of the exponential work {work32 / exp_work:.3f}")
    # compensated FP32 on the precision workload (the plain d = 4 shape, half
    # of the masses near the pole; three seeds) as point lists, kept for the
    # oracle leg's per-result histogram
    checks["precision_d4"] = []
    for seed in (0, 1, 2):
        wk = workloads.precision_d4(seed)
        q = wk.quad
        P = torch.as_tensor(np.repeat(wk.p, wk.m2.size), device="cuda")
        M = torch.as_tensor(np.tile(wk.m2, wk.p.size), device="cuda")
        d32 = [dict(quad=frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a,
                                       frg.FRG_PREC_FP32C), p=P, m2=M,
                    out=torch.empty(P.numel(), dtype=torch.float64, device="cuda"),
                    err_est=torch.empty(P.numel(), dtype=torch.float64, device="cuda"),
                    used_fp64=torch.empty(P.numel(), dtype=torch.uint8, device="cuda"))]
        d64 = [dict(quad=frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a), p=P, m2=M,
                    out=torch.empty(P.numel(), dtype=torch.float64, device="cuda"))]
        tp32 = timed(lambda: frg.frg_integrate(ctx, d32, flags=frg.FRG_PERSISTENT), torch, 20)
        tp64 = timed(lambda: frg.frg_integrate(ctx, d64, flags=frg.FRG_PERSISTENT), torch, 20)
        torch.cuda.synchronize()
        used = d32[0]["used_fp64"].cpu().numpy()
        checks["precision_d4"].append((wk, d32[0]["out"].cpu().numpy(),
                                       d32[0]["err_est"].cpu().numpy(), used))
        if seed == 0:
            sec["fp32c_precision_d4_seed0_points"] = {
                "evals": wk.n_evals, "fp32c_evals_per_s": wk.n_evals / tp32,
                "fp64_evals_per_s": wk.n_evals / tp64, "fp32_returned": int((used == 0).sum()),
                "results": int(used.size)}
            log(f"precision_d4 points: fp32c {wk.n_evals / tp32:.3e} evals/s, "
                f"fp64 {wk.n_evals / tp64:.3e}, FP32 {int((used == 0).sum())}/{used.size}")
    sec.update(tabulated(ctx, frg, workloads, torch))
    sec["vertex"] = vertex(ctx, frg, workloads, torch)
    sec["momentum_flow"] = momentum_flow(ctx, frg, workloads, torch)
    sec["fv_lpa"] = fv_lpa(ctx, frg, workloads, torch)
    sec["serving"] = serving(frg, workloads)
    sec["serving_500"] = serving(frg, workloads, n_warm=30, n_timed=300, seed=1, rate=500.0)
    return sec


def vertex(ctx, frg, workloads, torch, reps=20):
    """Two-external-momentum diagram: 256 configurations x 512 masses, 48 x 8
    x 16 rule (coefficient form over the azimuthal nodes); the same 2-FMA
    floor per (term, mass) as the scale-up grid."""
    w = workloads.vertex_d3()
    q = w.quad
    quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
    args = [torch.as_tensor(a, device="cuda") for a in (w.p1, w.p2, w.c12, w.m2)]
    out = torch.empty(w.n_integrals, dtype=torch.float64, device="cuda")
    t = timed(lambda: frg.frg_integrate_vertex(ctx, quad, w.n_phi, *args, out), torch, reps)
    log(f"vertex {w.name}: {t * 1e3:.3f} ms, {w.n_evals / t:.3e} evals/s")
    return {"workload": w.name, "ms_per_call": t * 1e3, "evals_per_s": w.n_evals / t,
            "integrals_per_s": w.n_integrals / t,
            "frac_of_2op_floor": w.n_evals / t / PEAK_EVALS}


def fv_lpa(ctx, frg, workloads, torch, reps=3):
    """Finite-volume LPA: 128 O(4) flows of 256 cells, 64 radial nodes, 2000
    SSP-RK3 steps (6000 right-hand sides: 257 interfaces x 128 flows, three
    threshold masses per Goldstone interface); time per whole solve."""
    w = workloads.fvlpa_d3()
    fv = frg.make_fvlpa(w.d, w.N, w.reg, w.n_r, w.lam, w.kappa, w.n_cells, w.sigma_max)
    U0 = torch.as_tensor(w.u0, device="cuda")
    U = torch.empty_like(U0)
    tr = torch.empty(w.n_flows, dtype=torch.float64, device="cuda")

    def run():
        U.copy_(U0)
        frg.frg_fvlpa_solve(ctx, fv, w.t_end, w.n_steps, U, tr)

    t = timed(run, torch, reps)
    reached = int((tr == w.t_end).sum().item())
    rhs = 3 * w.n_steps
    log(f"finite-volume LPA {w.name}: {t * 1e3:.1f} ms per solve, {rhs / t:.3e} right-hand "
        f"sides/s, {reached}/{w.n_flows} flows to t_end")
    return {"workload": w.name, "ms_per_solve": t * 1e3, "rhs_per_s": rhs / t,
            "interface_fluxes_per_s": rhs * w.n_flows * (w.n_cells + 1) / t,
            "flows_to_t_end": reached, "flows": w.n_flows}


def momentum_flow(ctx, frg, workloads, torch, reps=3):
    """Momentum-dependent two-point flows: 64 flows x 256 momentum nodes,
    128 x 32 rule, 100 RK4 steps (400 right-hand sides, each one launch that
    redoes the previous stage's update, builds the table rows and tadpoles
    and evaluates the tabulated diagram over all flows and nodes), all on
    the device; time per whole solve."""
    w = workloads.pflow_d3()
    pf = frg.make_pflow(w.d, w.reg, w.n_r, w.n_a, w.lam, w.kappa, w.n_s, w.s_max)
    l3 = torch.as_tensor(w.lam3, device="cuda")
    l4 = torch.as_tensor(w.lam4, device="cuda")
    S0 = torch.as_tensor(w.sigma0, device="cuda")
    S = torch.empty_like(S0)
    tr = torch.empty(w.n_flows, dtype=torch.float64, device="cuda")

    def run():
        S.copy_(S0)
        frg.frg_pflow_solve(ctx, pf, l3, l4, w.t_end, w.n_steps, S, tr)

    t = timed(run, torch, reps)
    reached = int((tr == w.t_end).sum().item())
    log(f"momentum flow {w.name}: {t * 1e3:.2f} ms per solve, {w.n_evals / t:.3e} evals/s, "
        f"{reached}/{w.n_flows} flows to t_end")
    return {"workload": w.name, "ms_per_solve": t * 1e3, "evals_per_solve": w.n_evals,
            "evals_per_s": w.n_evals / t, "rhs_per_s": 4 * w.n_steps / t,
            "flows_to_t_end": reached, "flows": w.n_flows}


def tabulated(ctx, frg, workloads, torch, which=(4096, 1 << 20), reps=None, steps_only=False):
    """Tabulated-propagator variant: 1024 momenta x 64 rows, rows of 4096 nodes
    (staged in LDS) and of 2^20 nodes (8 MB rows read through the caches).
    Each evaluation gathers two neighbouring table values (16 B)."""
    res = {}
    for n_s in which:
        w = workloads.tabulated_d3(n_s=n_s)
        q = w.quad
        quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
        G = torch.as_tensor(w.g, device="cuda")
        P = torch.as_tensor(w.p, device="cuda")
        out = torch.empty(w.n_integrals, dtype=torch.float64, device="cuda")
        t = timed(lambda: frg.frg_integrate_tab(ctx, quad, G, w.s_max, P, out), torch,
                  reps or (10 if n_s <= 8192 else 5))
        tb = w.g.nbytes
        seg = frg.frg_tune_get(ctx, "tab_seg")
        form = ("rows in LDS" if n_s <= 6144 else
                "segmented" if seg == 1 or (seg == 2 and tb > 256 * 2 ** 20) else "cache-streamed")
        res[f"tabulated_{n_s}"] = {
            "form": form,
            "workload": w.name, "ms_per_call": t * 1e3, "evals_per_s": w.n_evals / t,
            "integrals_per_s": w.n_integrals / t, "table_bytes": tb,
            "rows_in_lds": n_s <= 6144, "gathered_bytes_per_eval": 16,
            "gathered_GB_per_s": 16 * w.n_evals / t / 1e9, "table_GB_per_s_if_read_once": tb / t / 1e9}
        log(f"tabulated n_s={n_s}: {t * 1e3:.3f} ms, {w.n_evals / t:.3e} evals/s, "
            f"gathered {16 * w.n_evals / t / 1e9:.0f} GB/s")
        del G
    return res


def tab_forms_sweep(ctx, frg, workloads, torch):
    """Both forms of rows longer than the LDS (knob tab_seg 0: cache-streamed,
    1: segmented) on the same inputs over rows, row lengths and momenta:
    host-timed ms per call (10 after 3) and their largest relative
    difference, one JSON line per shape."""
    for n_s in (1 << 14, 1 << 16, 1 << 20):
        for n_p in (64, 1024):
            for n_rows in (1, 4, 16, 64):
                w = workloads.tabulated_d3(n_s=n_s, n_p=n_p, n_rows=n_rows)
                q = w.quad
                quad = frg.make_quad(q.d, q.reg, q.k, q.q_max, q.n_r, q.n_a)
                G = torch.as_tensor(w.g, device="cuda")
                P = torch.as_tensor(w.p, device="cuda")
                ms, outs = {}, {}
                for seg in (0, 1):
                    frg.frg_tune_set(ctx, "tab_seg", seg)
                    out = torch.empty(w.n_integrals, dtype=torch.float64, device="cuda")
                    ms[seg] = timed(lambda: frg.frg_integrate_tab(ctx, quad, G, w.s_max, P, out),
                                    torch, 10) * 1e3
                    outs[seg] = out.cpu().numpy()
                rel = float(np.max(np.abs(outs[1] - outs[0]) / np.abs(outs[0])))
                print(json.dumps({"n_s": n_s, "n_p": n_p, "n_rows": n_rows,
                                  "table_MiB": w.g.nbytes / 2 ** 20, "cache_ms": ms[0],
                                  "segmented_ms": ms[1], "cache_over_segmented": ms[0] / ms[1],
                                  "max_rel_diff": rel}), flush=True)
                del G
    frg.frg_tune_set(ctx, "tab_seg", 2)


def serving(frg, workloads, n_warm=50, n_timed=1000, seed=0, rate=50.0):
    """Poisson stream of LPA O(N) flow requests through frg_submit /
    frg_poll: n_warm requests, then n_timed whose latencies (done - submit on
    the library's monotonic clock) are reported, separately for flows that
    reach t = -9 and flows that stop at the propagator pole."""
    n_req = n_warm + n_timed
    reqs = workloads.lpa_requests(seed=seed, n=n_req, rate=rate)
    ctx = frg.frg_create(0)
    outs, keep, tickets, res = [], [], [], {}
    t0 = time.perf_counter()
    i = 0
    while len(res) < n_req:
        now = time.perf_counter() - t0
        while i < n_req and reqs[i].arrival_s <= now:
            r = reqs[i]
            U = np.zeros(r.n_grid)
            lpa = frg.make_lpa(d=r.d, N=r.N, reg=r.reg, n_radial=r.n_r,
                               q_max_over_k=r.q_max_over_k, Lambda=r.Lambda, n_grid=r.n_grid,
                               rho_max=r.rho_max)
            q = frg.make_request(lpa, r.lam, r.rho0, r.t_end, r.rtol, r.atol, U)
            outs.append(U)
            keep.append(q)
            tickets.append(frg.frg_submit(ctx, q))
            i += 1
        for tk in tickets:
            if tk not in res:
                rc, rr = frg.frg_poll(ctx, tk)
                if rc == frg.FRG_OK:
                    res[tk] = rr
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    rs = [res[t] for t in tickets][n_warm:]
    lat = np.array([x.done_s - x.submit_s for x in rs])
    span = max(x.done_s for x in rs) - min(x.submit_s for x in rs)
    done, launches, mean_batch = frg.frg_server_stats(ctx)
    frg.frg_destroy(ctx)
    okm = np.array([x.status == frg.FRG_OK for x in rs])
    polem = np.array([x.status == frg.FRG_E_DOMAIN for x in rs])

    def pct(mask):
        if not mask.any():
            return None
        return {"flows": int(mask.sum()), "p50_ms": float(np.percentile(lat[mask], 50) * 1e3),
                "p99_ms": float(np.percentile(lat[mask], 99) * 1e3),
                "mean_steps": float(np.mean([x.steps for x, m in zip(rs, mask) if m]))}

    r0 = reqs[0]
    out = {"requests": n_timed, "warmup_requests": n_warm, "rate_per_s": rate,
           "grid": "128..1024", "N": "1,2,4", "rtol": r0.rtol, "atol": r0.atol,
           "completed_to_t_end": int(okm.sum()), "stopped_at_pole": int(polem.sum()),
           "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
           "to_t_end": pct(okm), "at_pole": pct(polem),
           "mean_latency_ms": float(lat.mean() * 1e3), "flows_per_s": n_timed / span,
           "wall_s": wall,
           "rhs_calls_total": int(sum(x.rhs_calls for x in rs)),
           "launches": launches, "mean_flows_per_launch": mean_batch}
    log(f"serving at {rate:.0f}/s: p50 {out['p50_latency_ms']:.1f} ms, p99 "
        f"{out['p99_latency_ms']:.1f} ms, {int(okm.sum())} to t_end, {int(polem.sum())} at the "
        f"pole, mean batch {mean_batch:.2f}")
    return out


if __name__ == "__main__":
    main()
