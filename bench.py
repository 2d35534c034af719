#!/usr/bin/env python3
"""Throughput of the CR operator apply A x = (S^-1 + B Y^T N^-1 Y B) x.

One step = one apply_A of a batch of R right-hand sides on the full
workload (default: N_side 2048, lmax 4096, R = 8): beam prologue, Legendre
synthesis, ring FFT + N^-1 + adjoint ring FFT, Legendre adjoint and the
prior/beam epilogue -- every step of the hot path, all in the HIP library.
Inputs (x ~ N(0, S), N^-1 with mask) are resident in HBM before timing.

The reported value is the float32 mixed path (the path the full-scale
workload names); the split-bfloat16 and float64 paths are timed beside it.
Each path's throughput comes with its accuracy: its apply against the float64
apply and a 9-cycle W-cycle solve of manufactured right-hand sides with that
path's cycles and float64 refinement, checked against 1e-3 uK max pixel error
("gate").  A sweep over RHS per launch (1, 8, 32, 64) follows, and the CPU
oracle is timed on the host's cores ("cpu_baseline").

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A·x applies/s (SHT pair) at Nside 2048, ℓmax 4096; FP64 vs mixed at 1e-3 μK"
PEAK_FP64 = 78.6e12           # MI355X FP64 FLOP/s (vector and dense MFMA)
PEAK_FP32 = 157.3e12          # MI355X FP32 dense MFMA FLOP/s
PEAK_HBM = 8.0e12             # MI355X HBM3E bytes/s
PEAK_BF16 = 2.5e15            # MI355X dense bf16 MFMA FLOP/s

# The full-scale workload names the float32 mixed path; it is the headline.
DEFAULT_PATHS = "fp32,bf16x3,fp64"

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE (x2.0) + WRITE_SIZE
# (x1.0), the factors from a plain copy of known size; recorded in
# profiles/apply_A_c5_r8_hbm_traffic.md.  Only kernels unchanged since those
# counters were taken are listed (a changed kernel reports traffic null).
# Key: (library timer name, Legendre path, workload, RHS per launch).
MEASURED_TRAFFIC = {
    ("legendre_adjoint", "fp32", "c5", 8): 4.919e9 + 4.303e9,
    ("legendre_adjoint", "bf16x3", "c5", 8): 4.932e9 + 4.301e9,
    ("legendre_adjoint", "fp64", "c5", 8): 9.106e9 + 8.596e9,
    ("legendre_synth", "fp32", "c5", 8): 10.441e9 + 9.056e9,
    ("legendre_synth", "bf16x3", "c5", 8): 6.720e9 + 4.995e9,
    ("legendre_synth", "fp64", "c5", 8): 16.365e9 + 9.934e9,
    ("ring_apply", "fp32", "c5", 8): 1.216e9 + 0.537e9 + 3 * (0.718e9 + 0.537e9),
    ("ring_apply", "bf16x3", "c5", 8): 1.219e9 + 0.537e9 + 3 * (0.718e9 + 0.537e9),
    ("ring_apply", "fp64", "c5", 8): 1.772e9 + 1.074e9 + 3 * (1.285e9 + 1.075e9),
}
# Matrix-core busy fraction (SQ_VALU_MFMA_BUSY_CYCLES over 1024 SIMDs x
# 2.4 GHz x duration) of the same kernels, from
# profiles/legendre_c5_r8_mfma_counters.md; kernels changed since are absent.
MEASURED_MFMA_BUSY = {
    ("legendre_synth", "fp32", "c5", 8): 0.404,
    ("legendre_adjoint", "fp32", "c5", 8): 0.353,
    ("legendre_synth", "bf16x3", "c5", 8): 0.119,
    ("legendre_adjoint", "bf16x3", "c5", 8): 0.089,
    ("legendre_synth", "fp64", "c5", 8): 0.551,
    ("legendre_adjoint", "fp64", "c5", 8): 0.372,
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def legendre_useful_flops(nside: int, lmax: int, R: int) -> float:
    """4 flops (cos and sin FMAs) per (l, m, ring pair, RHS) over the full
    triangle 0 <= m <= l <= lmax and all 2 N_side ring pairs.  The kernels skip
    the region where every lambda is below 2^-112 (about 27% of the triangle
    at N_side 2048 / lmax 4096); the count keeps it, so a rate is per useful
    product of the whole transform."""
    ntri = (lmax + 1) * (lmax + 2) // 2
    return 4.0 * ntri * 2 * nside * R


def recurrence_flops(nside: int, lmax: int, R: int) -> float:
    """3 flops (one multiply, one FMA) per (l, m, ring pair) of the scaled
    three-term recurrence, once per chunk of 8 RHS, full triangle."""
    ntri = (lmax + 1) * (lmax + 2) // 2
    return 3.0 * ntri * 2 * nside * ((R + 7) // 8)


def min_bytes(name: str, nside: int, lmax: int, R: int, path: str):
    """The method's minimum HBM bytes of one launch: x, y and N^-1 once, and the
    m-major <-> ring-major round trip of the two-stage SHT once each way, with
    F and G as complex numbers of the path's FFT precision (16 B float64,
    8 B on the mixed paths)."""
    nrings, npix, nalm = 4 * nside - 1, 12 * nside * nside, (lmax + 1) ** 2
    fg = (16.0 if path == "fp64" else 8.0) * nrings * (lmax + 1) * R
    vec = 8.0 * nalm * R
    if name == "legendre_synth":
        return vec + fg                     # x in, F out
    if name == "legendre_adjoint":
        return fg + 2 * vec                 # G in, x in and y out (y = D x + B v)
    if name == "ring_apply":
        return 2 * fg + 8.0 * npix          # F in, G out, N^-1
    if name in ("ring_synth", "ring_adjoint"):
        return fg + 8.0 * npix * R
    return None


def cpu_baseline(cfg, R: int, x_host, ninv_host, measured=("c1", "c2", "c3"), budget_s: float = 20.0):
    """The CPU oracle on the machine's host cores.

    value: one full apply of the benchmark workload estimated from a bounded
    sample -- the oracle's per-order Legendre step (both directions, R RHS) on
    orders spread over [0, lmax] run by its worker pool (all host cores), and
    its ring step (serial, as in the oracle) on 64 rings -- extrapolated by
    work (order m costs ~ lmax - m + 1; ring work ~ pixels).
    measured: whole oracle applies of R RHS at the smaller workloads, timed."""
    import numpy as np

    import workloads
    from oracle import geometry as ogeo
    from oracle import operator as oop
    from oracle import pool
    from oracle import sht as osht

    nw = pool.worker_count()
    lmax, nside = cfg.lmax, cfg.nside
    geom = ogeo.healpix_rings(nside)
    # start the workers outside the timed region
    tiny = ogeo.healpix_rings(2)
    pool.run(osht._synth_orders, [(4, tiny, [(0, np.zeros((1, 5)), np.zeros((1, 5)))])] * nw, nw)
    # Legendre sample: rounds of nw orders until the budget is used
    picked, t_leg_sample = [], 0.0
    order = np.random.default_rng(0).permutation(lmax + 1)
    t_all = time.perf_counter()
    while time.perf_counter() - t_all < budget_s and len(picked) < lmax + 1:
        ms = [int(m) for m in order[len(picked): len(picked) + nw]]
        groups = [(lmax, geom, [(m,) + tuple(np.ascontiguousarray(v) for v in osht.split_m(x_host, m, lmax))])
                  for m in ms]
        ggroups = [(lmax, geom, [(m, np.zeros((R, geom.nrings)), np.zeros((R, geom.nrings)))]) for m in ms]
        t0 = time.perf_counter()
        pool.run(osht._synth_orders, groups, nw)
        pool.run(osht._adjoint_orders, ggroups, nw)
        t_leg_sample += time.perf_counter() - t0
        picked += ms
    work = lambda ms: float(sum(lmax - m + 1 for m in ms))
    t_leg = t_leg_sample * work(range(lmax + 1)) / work(picked)
    # ring sample: synthesis and adjoint ring step on spread rings
    rings = np.unique(np.linspace(0, geom.nrings - 1, 64).astype(int))
    sub_pix = int(geom.nphi[rings].sum())
    F = np.random.default_rng(0).standard_normal((R, 1, lmax + 1))
    t0 = time.perf_counter()
    for k in rings:
        g1 = ogeo.RingGeometry(nside, geom.z[k:k + 1], geom.sint[k:k + 1], geom.nphi[k:k + 1],
                               geom.phi0[k:k + 1], np.array([0]))
        mp = osht.ring_synth(F, F, g1)
        osht.ring_adjoint(mp * ninv_host[geom.start[k]: geom.start[k] + geom.nphi[k]], lmax, g1)
    t_ring = (time.perf_counter() - t0) * (geom.npix / sub_pix)
    total = t_leg + t_ring
    meas = {}
    for name in measured:
        c = workloads.get_config(name)
        dd = workloads.workload_inputs(c)
        xs = np.stack([workloads.prior_sample(c, r) for r in range(R)])
        t0 = time.perf_counter()
        oop.apply_A(xs, dd["cl"], dd["bl"], dd["ninv"], c.nside)
        dt = time.perf_counter() - t0
        meas[name] = {"nside": c.nside, "lmax": c.lmax, "nrhs": R, "s_per_apply": dt,
                      "rhs_applies_per_s": R / dt}
        log(f"[bench] oracle apply {name} (N_side {c.nside}, lmax {c.lmax}, {R} RHS): {dt:.2f} s")
    return {
        "value": R / total,
        "unit": "RHS-applies/s",
        "cores": nw,
        "kind": "oracle",
        "sample": (f"oracle Legendre step (both directions, {R} RHS) on {len(picked)} of "
                   f"{lmax + 1} orders (random, spread over [0, lmax]) through its {nw}-process "
                   f"pool, and its serial ring step on {len(rings)} rings, of the N_side {nside}, "
                   f"lmax {lmax} workload, extrapolated by work to one apply of {R} RHS "
                   f"(estimated {total:.0f} s per apply)"),
        "measured_full_applies": meas,
    }


def run_path(mlcr, torch, op, x, y, prec, steps, warmup, label):
    """Warm up, then time `steps` applies; returns (ms per step, per-kernel ms per launch)."""
    for i in range(warmup):
        mlcr.apply_A(op, x, prec=prec, out=y)
        torch.cuda.synchronize()
        log(f"[bench] {label} warmup {i + 1}/{warmup} done")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with mlcr.KernelTimer() as kt:
        e0.record(stream)
        for i in range(steps):
            mlcr.apply_A(op, x, prec=prec, out=y)
        e1.record(stream)
        torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    kernels = {k: (v[0] / v[1]) for k, v in kt.result.items()}
    log(f"[bench] {label}: {steps} steps, {ms_step:.3f} ms/step")
    for k, v in sorted(kernels.items(), key=lambda t: -t[1]):
        log(f"[bench]   {k:18s} {v:9.3f} ms/launch")
    return ms_step, kernels


def roofline(kernels, cfg, R, path: str):
    """Roofline of the dominant kernel of one apply (HIP events on its stream).

    Legendre kernels on the float32 / float64 paths are matrix-core bound:
    achieved = useful flops (legendre_useful_flops) per launch time, against
    the dense peak of the kernel's own dtype.  The split-bfloat16 kernels are
    bound by the vector work around the matrix cores (the counters show ~22
    VALU instructions per MFMA): achieved = recurrence flops per launch time
    against the float64 vector peak, with the useful matrix-core rate beside
    it.  Other kernels are HBM bound against the method's minimum bytes."""
    dom = max(kernels, key=lambda k: kernels[k])
    sec = kernels[dom] / 1e3
    key = (dom, path, cfg.name, R)
    if dom.startswith("legendre"):
        useful = legendre_useful_flops(cfg.nside, cfg.lmax, R)
        if path == "bf16x3":
            work = recurrence_flops(cfg.nside, cfg.lmax, R)
            roof = {"bound": "alu", "kernel": dom, "achieved": work / sec / 1e12,
                    "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                    "work_per_launch": work, "work": "float64 recurrence flops, full triangle",
                    "useful_mfma_tflops": useful / sec / 1e12,
                    "useful_frac_of_bf16_peak": useful / sec / PEAK_BF16}
        else:
            peak = PEAK_FP64 if path == "fp64" else PEAK_FP32
            roof = {"bound": "mfma", "kernel": dom, "achieved": useful / sec / 1e12,
                    "peak": peak / 1e12, "unit": "TFLOP/s", "work_per_launch": useful,
                    "work": "useful flops, full triangle (the skipped negligible region counted)"}
    else:
        mb = min_bytes(dom, cfg.nside, cfg.lmax, R, path)
        roof = {"bound": "hbm", "kernel": dom, "achieved": mb / sec / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "work_per_launch": mb, "work": "method's minimum bytes"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = MEASURED_TRAFFIC.get(key)
    roof["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-scaled)"
    roof["min_bytes"] = min_bytes(dom, cfg.nside, cfg.lmax, R, path)
    roof["mfma_busy_counters"] = MEASURED_MFMA_BUSY.get(key)
    roof["kernel_ms"] = {k: round(v, 4) for k, v in kernels.items()}
    return roof


def level_profile(S, b, prec):
    """Per-level time of one W-cycle (mlcr_solver_profile): profiles of a
    3-cycle and a 1-cycle solve, halved difference, so that the starting
    residual drops out and the top level holds the cycle's float64 residual.
    Rows: top, pixel levels, dense bottom; columns: applications of A_h,
    level SHTs (Y_h), smoother (dense solve at the bottom), transfers."""
    runs = {}
    for n in (1, 3):
        S.set_profile(True)
        S.solve(b, rtol=0.0, max_cycles=n, prec=prec, raise_on_noconv=False)
        runs[n] = S.profile()
        S.set_profile(False)
    ms = (runs[3]["ms"] - runs[1]["ms"]) / 2
    calls = (runs[3]["calls"] - runs[1]["calls"]) // 2
    return {"kinds": ["A_h", "level SHTs", "smoother", "transfers"],
            "ms_per_cycle": [[round(float(v), 3) for v in row] for row in ms],
            "calls_per_cycle": [[int(v) for v in row] for row in calls],
            "cycle_ms": round(float(ms.sum()), 2)}


def solve_bench(mlcr, torch, cfg, geom, op, xt, R, paths, max_cycles, target=1e-3, pcg=False,
                graph=False, levels=False):
    """W-cycle solves of b = A x_true (x_true ~ N(0, S), b by the float64
    apply); cycle by cycle, the max pixel error |Y (x - x_true)| (float64
    synthesis, all pixels) until every RHS is within `target` uK.  Reports
    the time to get there per path (setup excluded), the speedup of each
    path over float64 and, if asked, the per-level time of one cycle."""
    precs = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}
    t0 = time.time()
    S = mlcr.Solver(op, max_nrhs=R)
    torch.cuda.synchronize()
    setup = time.time() - t0
    log(f"[bench] solver setup {setup:.1f}s, {S.info()}")
    b = mlcr.apply_A(op, xt)
    out = {"metric": f"W-cycle solve time to {target:g} uK max pixel error",
           "unit": "s", "higher_is_better": False, "n_gpus": 1, "nrhs": R,
           "config": {"workload": f"{cfg.name}: HEALPix Nside {cfg.nside}, lmax {cfg.lmax}, "
                                  f"{R} RHS per solve, manufactured b = A x_true",
                      "nside": cfg.nside, "lmax": cfg.lmax, "nrhs": R},
           "setup_s": setup, "paths": {}}
    # one untimed cycle per path: per-grid tables and workspaces are made on first use
    for p in paths:
        S.solve(b, rtol=0.0, max_cycles=1, prec=precs[p], raise_on_noconv=False)
    torch.cuda.synchronize()
    for p in paths:
        # error history: one cycle per call (each call also recomputes the
        # starting residual, so these times are not the solve time)
        x = torch.zeros_like(b)
        elapsed, hist = 0.0, []
        for c in range(max_cycles):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x, info = S.solve(b, x0=x, rtol=0.0, max_cycles=1, prec=precs[p],
                              raise_on_noconv=False)
            torch.cuda.synchronize()
            elapsed += time.perf_counter() - t
            err = float(mlcr.sht_synth(geom, x - xt).abs().amax())
            hist.append({"cycle": c + 1, "max_err_uK": err, "rho": max(i["rho"] for i in info)})
            log(f"[bench] {p} cycle {c + 1}: max pixel error {err:.3e} uK")
            if err <= target:
                break
        ok = hist[-1]["max_err_uK"] <= target
        nc = len(hist)
        # the solve time: those cycles in one call, timed whole (direct launches,
        # then with the cycles replayed from a HIP graph if asked)
        times = {}
        for mode in ((False, True) if graph else (False,)):
            S.set_graph(mode)
            S.solve(b, rtol=0.0, max_cycles=nc, prec=precs[p], raise_on_noconv=False)
            torch.cuda.synchronize()
            t = time.perf_counter()
            x1, _ = S.solve(b, rtol=0.0, max_cycles=nc, prec=precs[p], raise_on_noconv=False)
            torch.cuda.synchronize()
            times[mode] = time.perf_counter() - t
            err1 = float(mlcr.sht_synth(geom, x1 - xt).abs().amax())
            log(f"[bench] {p}: {nc} cycles in one call ({'graph' if mode else 'direct'}): "
                f"{times[mode]:.3f}s, max pixel error {err1:.3e} uK")
        S.set_graph(False)
        out["paths"][p] = {"time_s": times[False] if ok else None, "cycles": nc, "reached": ok,
                           "history": hist}
        if levels:
            lv = level_profile(S, b, precs[p])
            out["paths"][p]["levels"] = lv
            log(f"[bench] {p}: per-level ms per cycle (A_h, SHTs, smoother, transfers), "
                f"cycle {lv['cycle_ms']} ms:")
            for h, (row, cr) in enumerate(zip(lv["ms_per_cycle"], lv["calls_per_cycle"])):
                log(f"[bench]   level {h}: {row}  calls {cr}")
        if graph:
            out["paths"][p]["graph_time_s"] = times[True] if ok else None
            out["paths"][p]["graph_stats"] = S.graph_stats()
        if pcg:
            # CG with the cycle as preconditioner: k iterations from zero, k = 1, 2, ...
            # until the error is within target (each run timed whole)
            for k in range(1, max_cycles + 1):
                torch.cuda.synchronize()
                t = time.perf_counter()
                x, info = S.solve_pcg(b, rtol=0.0, max_iter=k, prec=precs[p], raise_on_noconv=False)
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                err = float(mlcr.sht_synth(geom, x - xt).abs().amax())
                log(f"[bench] {p} pcg {k} iterations: max pixel error {err:.3e} uK, {el:.2f}s")
                if err <= target:
                    break
            out["paths"][p]["pcg"] = {"time_s": el if err <= target else None, "iterations": k,
                                      "max_err_uK": err}
    t64 = out["paths"].get("fp64", {}).get("time_s")
    for p, v in out["paths"].items():
        v["speedup_vs_fp64"] = (t64 / v["time_s"]) if (t64 and v["time_s"]) else None
    return out


def mixed_bench(mlcr, torch, paths, rtol=1e-8, max_cycles=40):
    """Mixed batch of independent problems (one RHS each, own grid and band
    limit): the problems solved one after another vs one grouped solve."""
    import workloads
    precs = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}
    probs, grids = [], {}
    t0 = time.time()
    for k, name in enumerate(workloads.MIXED_BATCH):
        cfg = workloads.get_config(name)
        if name not in grids:
            d = workloads.workload_inputs(cfg)
            g = mlcr.Geometry(cfg.nside, cfg.lmax)
            op = mlcr.Operator(g, d["cl"], d["bl"], torch.from_numpy(d["ninv"]).cuda(), max_nrhs=1)
            grids[name] = (g, op)
        g, op = grids[name]
        S = mlcr.Solver(op, max_nrhs=1)
        xt = torch.from_numpy(workloads.prior_sample(cfg, k)[None]).cuda()
        probs.append((name, S, mlcr.apply_A(op, xt)))
    torch.cuda.synchronize()
    log(f"[bench] mixed batch {workloads.MIXED_BATCH}: setup {time.time() - t0:.1f}s")
    out = {"metric": "mixed-batch W-cycle solve time to rtol", "unit": "s", "higher_is_better": False,
           "n_gpus": 1, "rtol": rtol,
           "config": {"workload": "mixed batch: " + ", ".join(
               f"{n} (N_side {workloads.get_config(n).nside}, lmax {workloads.get_config(n).lmax})"
               for n in workloads.MIXED_BATCH) + ", 1 RHS each"},
           "paths": {}}
    for p in paths:
        for _, S, b in probs:        # untimed: tables and workspaces on first use
            S.solve(b, rtol=0.0, max_cycles=1, prec=precs[p], raise_on_noconv=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _, S, b in probs:
            S.solve(b, rtol=rtol, max_cycles=max_cycles, prec=precs[p])
        torch.cuda.synchronize()
        seq = time.perf_counter() - t
        t = time.perf_counter()
        _, infos = mlcr.solve_grouped([S for _, S, _ in probs], [b for _, _, b in probs], rtol=rtol,
                                      max_cycles=max_cycles, prec=precs[p])
        torch.cuda.synchronize()
        grp = time.perf_counter() - t
        cyc = [i[0]["cycles"] for i in infos]
        log(f"[bench] mixed {p}: one after another {seq:.2f}s, grouped {grp:.2f}s, cycles {cyc}")
        out["paths"][p] = {"sequential_s": seq, "grouped_s": grp, "speedup": seq / grp, "cycles": cyc}
    return out


def gate(mlcr, torch, cfg, geom, op, x, outs, paths, R, cycles=9, target=1e-3):
    """The accuracy each path's throughput is counted at: its apply against the
    float64 apply, and a W-cycle solve of manufactured b = A x_true (float64
    apply) with that path's cycles and float64 refinement, whose max pixel
    error (float64 synthesis over all pixels) must reach `target` uK."""
    precs = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}
    out = {"target_uK": target, "cycles": cycles, "paths": {}}
    t0 = time.time()
    S = mlcr.Solver(op, max_nrhs=R)
    torch.cuda.synchronize()
    out["solver_setup_s"] = time.time() - t0
    b = mlcr.apply_A(op, x)
    import workloads
    d = workloads.workload_inputs(cfg)
    import numpy as np
    ell = np.arange(cfg.lmax + 1)
    sigma_prior = float(np.sqrt(np.sum((2 * ell + 1) * d["cl"]) / (4 * np.pi)))
    for p in paths:
        S.solve(b, rtol=0.0, max_cycles=1, prec=precs[p], raise_on_noconv=False)   # tables, workspaces
        torch.cuda.synchronize()
        t = time.perf_counter()
        xs, info = S.solve(b, rtol=0.0, max_cycles=cycles, prec=precs[p], raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        err = float(mlcr.sht_synth(geom, xs - x).abs().amax())
        ent = {"solve_s": el, "max_pixel_error_uK": err, "reached": err <= target,
               "certificate_uK": sigma_prior * max(i["s_half_res"] for i in info),
               "rho": max(i["rho"] for i in info)}
        if p != "fp64" and "fp64" in outs and p in outs:
            dlt = outs[p] - outs["fp64"]
            ent["apply_rel_l2_vs_fp64"] = float(dlt.norm() / outs["fp64"].norm())
            ent["apply_max_elem_vs_fp64"] = float(dlt.abs().amax() / outs["fp64"].abs().amax())
        out["paths"][p] = ent
        log(f"[bench] gate {p}: {cycles} cycles {el:.2f} s, max pixel error {err:.3e} uK "
            f"(certificate {ent['certificate_uK']:.3e})")
        del xs
    t64 = out["paths"].get("fp64", {}).get("solve_s")
    for p, v in out["paths"].items():
        v["speedup_vs_fp64_at_equal_accuracy"] = (t64 / v["solve_s"]) if (t64 and v["reached"]) else None
    return out


def r_sweep(mlcr, torch, cfg, geom, d, paths, rs=(1, 8, 32, 64), steps=3):
    """Apply throughput against the RHS count of one launch (independent
    realizations batched, so one lambda feeds more columns)."""
    import numpy as np
    precs = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}
    dev = torch.device("cuda:0")
    ninv = torch.from_numpy(d["ninv"]).to(dev)
    op = mlcr.Operator(geom, d["cl"], d["bl"], ninv, max_nrhs=max(rs))
    x = torch.from_numpy(np.stack([workloads_prior(cfg, r) for r in range(max(rs))])).to(dev)
    out = {}
    for p in paths:
        out[p] = {}
        for R in rs:
            xr = x[:R].contiguous()
            y = torch.empty_like(xr)
            ms, kern = run_path(mlcr, torch, op, xr, y, precs[p], steps, 1, f"{p} R={R}")
            leg = {k: v for k, v in kern.items() if k.startswith("legendre")}
            ent = {"ms_per_apply": ms, "rhs_applies_per_s": R / (ms / 1e3),
                   "kernel_ms": {k: round(v, 4) for k, v in kern.items()}}
            for k, v in leg.items():
                ent[f"{k}_useful_tflops"] = legendre_useful_flops(cfg.nside, cfg.lmax, R) / (v / 1e3) / 1e12
            out[p][str(R)] = ent
            del y
    del op, x
    torch.cuda.synchronize()
    return out


def workloads_prior(cfg, r):
    import workloads
    return workloads.prior_sample(cfg, r)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--nrhs", type=int, default=0)
    ap.add_argument("--paths", default=DEFAULT_PATHS,
                    help="Legendre paths to time; the first is the reported value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gate", action="store_true",
                    help="skip the per-path accuracy gate (apply vs float64, 9-cycle solve)")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the sweep over RHS per launch (1, 8, 32, 64)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shapes instead of tuning each "
                         "path on the workload before timing it")
    ap.add_argument("--graph", action="store_true",
                    help="with --solve: also time whole solves with the cycle replayed from a HIP graph")
    ap.add_argument("--pcg", action="store_true",
                    help="with --solve: also time CG with the cycle as preconditioner")
    ap.add_argument("--levels", action="store_true",
                    help="with --solve: also the per-level time of one W-cycle per path")
    ap.add_argument("--mixed", action="store_true",
                    help="time the mixed batch of independent problems solved one after another "
                         "and as one grouped solve")
    ap.add_argument("--solve", action="store_true",
                    help="time W-cycle solves to 1e-3 uK max pixel error (manufactured "
                         "solutions) with the float64 and mixed paths instead of applies")
    ap.add_argument("--max-cycles", type=int, default=16)
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="only run a plain device-to-device copy of this many GiB (a "
                         "known-size reference for HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path "
              "(RHS sharding, or an m/ring all-to-all per SHT) is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * 2 ** 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n, "read": 8 * n, "written": 8 * n}), flush=True)
        return

    import paper_1308_5299_amd as mlcr
    from paper_1308_5299_amd import autotune
    import workloads

    if args.mixed:
        paths = [p.strip() for p in args.paths.split(",") if p.strip()]
        print(json.dumps(mixed_bench(mlcr, torch, paths)), flush=True)
        return
    cfg = workloads.get_config(args.config)
    R = args.nrhs or cfg.nrhs
    paths = [p.strip() for p in args.paths.split(",") if p.strip()]
    precs = {"fp64": mlcr.FP64, "fp32": mlcr.FP32, "bf16x3": mlcr.BF16X3}
    for p in paths:
        if p not in precs:
            sys.exit(f"unknown path {p}")
    log(f"[bench] config {cfg.name}: nside {cfg.nside} lmax {cfg.lmax} R {R} paths {paths}")
    t0 = time.time()
    d = workloads.workload_inputs(cfg)
    x_host = np.stack([workloads.prior_sample(cfg, r) for r in range(R)])
    log(f"[bench] inputs ready in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ninv = torch.from_numpy(d["ninv"]).to(dev)
    x = torch.from_numpy(x_host).to(dev)
    t0 = time.time()
    geom = mlcr.Geometry(cfg.nside, cfg.lmax)
    op = mlcr.Operator(geom, d["cl"], d["bl"], ninv, max_nrhs=R)
    torch.cuda.synchronize()
    log(f"[bench] geometry + operator ready in {time.time() - t0:.1f}s")

    if args.solve:
        print(json.dumps(solve_bench(mlcr, torch, cfg, geom, op, x, R, paths, args.max_cycles,
                                     pcg=args.pcg, graph=args.graph, levels=args.levels)),
              flush=True)
        return

    res, outs, tuned = {}, {}, {}
    for p in paths:
        if not args.no_autotune:
            # launch shapes picked by timing each choice on this workload (not timed)
            t0 = time.time()
            tr = autotune.tune(op, R, precs[p], reps=2)
            tuned[p] = tr["tuning"]
            log(f"[bench] {p} autotune {tr['tuning']} in {time.time() - t0:.1f}s: "
                f"{tr['timings_ms']}")
        y = torch.empty_like(x)
        res[p] = run_path(mlcr, torch, op, x, y, precs[p], args.steps, args.warmup, p)
        outs[p] = y

    head = paths[0]
    ms_step, kernels = res[head]
    value = R / (ms_step / 1e3)
    roof = roofline(kernels, cfg, R, head)
    others = {p: {"value": R / (res[p][0] / 1e3), "ms_per_step": res[p][0],
                  "roofline": roofline(res[p][1], cfg, R, p)}
              for p in paths[1:]}

    gt = None
    if not args.no_gate:
        log("[bench] accuracy gate: applies vs float64 and 9-cycle solves per path")
        gt = gate(mlcr, torch, cfg, geom, op, x, outs, paths, R)
    del outs
    sweep = None
    if not args.no_sweep and cfg.name == "c5":
        log("[bench] RHS sweep")
        del op
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        sweep = r_sweep(mlcr, torch, cfg, geom, d, [p for p in ("fp32", "bf16x3") if p in paths])

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample (all host cores)")
        cpu = cpu_baseline(cfg, R, x_host, d["ninv"])
        log(f"[bench] cpu baseline {cpu['value']:.3e} {cpu['unit']} on {cpu['cores']} cores")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "RHS-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}[head],
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: HEALPix Nside {cfg.nside}, lmax {cfg.lmax}, "
                               f"{R} RHS per apply, {head} Legendre contraction and ring FFTs "
                               f"(float64 recurrence seeds and scaling, float64 in/out)",
                   "nside": cfg.nside, "lmax": cfg.lmax, "nrhs": R, "prec": head,
                   "global_batch": R},
        "roofline": roof,
        "cpu_baseline": cpu,
        "other_paths": others,
        "gate": gt,
        "rhs_sweep": sweep,
        "tuning": tuned or None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
