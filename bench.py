"""Benchmark: BiCGStab iterations/s and HBM roofline on the paper's 600x595x1536 mesh.

One step is one BiCGStab iteration of the whole hot path (P1, P2, P3 with their
scalar steps) over the 548,352,000-cell system, with every input resident in HBM
before the timed region starts.  The timed region is one call of the solver with a
fixed iteration count.  That call includes its prologue and epilogue: coefficient
scaling, r0 = b - A x0, x update and the FP64 true residual.

Printed: one JSON line with the metric, the roofline of the dominant kernel, the
mixed BF16+refinement form, accuracy of converged runs against the manufactured
solution, the batched form (64 uneven systems), the served form (a Poisson request
stream through the queue against a serial loop of single solves, p50/p99 latency), the
solver pattern of the paper's SIMPLE loop (Algorithm 2), one GPU's z-slab share of the mesh
for an 8-GPU split, the 2D 9-point workload of section IV at 4800^2 and 22800^2, and the
FP64 CPU oracle timed on a bounded slab of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# Algorithmic bytes per cell of each pass (Jacobi-scaled: 6 coefficient arrays), by
# schedule.  Three passes (the solver's default):
#   P1 reads p, r0 and 6 coefficients and writes s;
#   P2 reads r, s, r0 and 6 coefficients (q = r - alpha s formed on the fly) and writes y;
#   P3 reads d, p, r, s, y, r0 and writes d, r, p.
# Four passes (q stored): P2a reads r, s and writes q; P2b reads q, r0 and the
# coefficients and writes y; P3 reads q instead of r.
# Slots of s7_info.pass_ms: 0 P1, 1 P2a, 2 P2 or P2b, 3 P3.
BYTES = {
    ("f32", 3): {"p1": 36, "p2": 40, "p3": 36},
    ("f32", 4): {"p1": 36, "p2a": 12, "p2b": 36, "p3": 36},
    ("16", 3): {"p1": 18, "p2": 20, "p3": 22},  # BF16/FP16 vectors and coefficients, FP32 d
    ("16", 4): {"p1": 18, "p2a": 6, "p2b": 18, "p3": 22},
}
SLOT = {"p1": 0, "p2a": 1, "p2": 2, "p2b": 2, "p3": 3}
# Bytes per cell that an FP32 solve moves once, outside its iterations (Jacobi mode): the
# scaled coefficient copies (7 read, 6 written), r0 = b - A x0 in FP64 (7 coefficients, b,
# x; r, r0, p, d written), x += d in FP64, and the FP64 true residual at exit.
SETUP_BYTES_FP32 = {"coefficient copies": 28 + 24, "r0": 28 + 8 + 8 + 16, "x update": 4 + 8 + 8,
                    "true residual": 28 + 8 + 8}
# s7_info.schedule: 1 three passes, 2 four passes, 3 three passes on cell pairs, 5 three
# passes with the stencil operand staged in LDS
PASSES = {1: 3, 2: 4, 3: 3, 5: 3}
KERNEL = {
    1: {"p1": "k_p1 (P1: s = A p, (r0,s))",
        "p2": "k_p2f (P2: y = A q with q = r - alpha s formed on the fly, five dot products)",
        "p3": "k_p3 (P3: x, r, p updates, (r0,r), (r,r))"},
    2: {"p1": "k_p1 (P1: s = A p, (r0,s))",
        "p2a": "k_p2a (P2a: q = r - alpha s, (q,q))",
        "p2b": "k_p2 (P2b: y = A q, four dot products)",
        "p3": "k_p3 (P3: x, r, p updates, (r0,r), (r,r))"},
    3: {"p1": "k_p1_pair (P1 on x-adjacent cell pairs: s = A p, (r0,s))",
        "p2": "k_p2f_pair (P2 on cell pairs: y = A q with q = r - alpha s on the fly, five dot products)",
        "p3": "k_p3 (P3: x, r, p updates, (r0,r), (r,r))"},
    5: {"p1": "k_p1_lds (P1, p of a tile and one row either side staged in LDS: s = A p, (r0,s))",
        "p2": "k_p2f_lds (P2, q = r - alpha s of a tile and one row either side staged in LDS: "
              "y = A q, five dot products)",
        "p3": "k_p3 (P3: x, r, p updates, (r0,r), (r,r))"},
}
# SURVEY's per-pass split of the same iteration for the Jacobi-scaled FP32 system (p
# formed in P1 there, in P3 here): P1 48, P2 36, P3 32, 116 B per cell and iteration
SURVEY_BYTES = {"p1": 48, "p2": 36, "p3": 32}
BATCH_BYTES = sum(BYTES[("f32", 3)].values())  # the batched engine runs the three-pass schedule
SPLIT_CELLS = 1 << 21  # the queue's default: larger requests take the single-system path
SRC_FILES = ["paper_2010_03660_amd/csrc/s7_device.hpp", "paper_2010_03660_amd/csrc/s7_passes.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in SRC_FILES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_cells: int, kernel: str, schedule: int, lds_tile: int = 0, xcd_run: int = 0):
    """HBM bytes per launch of pass `kernel` from the committed counter summary: the
    record of the form this run used (schedule, staged tile, XCD tile order), if the
    kernel sources have not changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_paper600x595x1536_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("cells") != n_cells:
        return None
    for form in t.get("forms", []):
        if (form.get("schedule") == schedule and form.get("lds_tile", 0) == lds_tile
                and form.get("xcd_run", 0) == xcd_run):
            return form.get("bytes_per_launch")
    return None


def host_cores() -> int:
    """Host threads this process may use: OMP_NUM_THREADS if set (the GPU machines set it to
    their CPU share), else the CPUs of its affinity mask."""
    try:
        t = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        t = 0
    return t if t > 0 else len(os.sched_getaffinity(0))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(nx: int, ny: int, nz_full: int, slab: int, iters: int):
    """The FP64 oracle (C, CSR, Algorithm 1) on a slab of `slab` z-planes of the same
    workload, on all host cores (the SpMV row loop threaded; inner products and vector
    updates single-threaded) and on one core; the time per iteration is scaled to the
    full mesh by cell count."""
    import oracle
    import synth
    oracle.build(force=False)
    prob = synth.make_problem(nx, ny, slab, seed=0)
    A = oracle.build_csr(nx, ny, slab, prob.coef)
    b = oracle.spmv(A, prob.xstar)
    cores = host_cores()
    times = {}
    try:
        for t in (cores, 1):
            oracle.set_threads(t)
            t0 = time.perf_counter()
            res = oracle.bicgstab(A, b, tol=1e-300, max_iter=iters)
            times[t] = time.perf_counter() - t0
            assert res.iters == iters
    finally:
        oracle.set_threads(1)
    scale = nz_full / slab
    return {"value": iters / times[cores] / scale, "unit": "iter/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "single_core_value": iters / times[1] / scale,
            "sample": f"{iters} iterations on a {nx}x{ny}x{slab} slab of the same recipe "
                      f"({times[cores]:.1f} s on {cores} threads, {times[1]:.1f} s on one), "
                      f"scaled by cell count to {nx}x{ny}x{nz_full}"}

BATCH_REPEATS = 5  # timed calls of a batched leg (after a warm-up call); the median is reported


def repeat_timed(once, k: int = BATCH_REPEATS):
    """Runs once() k times; returns the last (status, infos) and the sorted times."""
    ts, last = [], None
    for _ in range(k):
        rc, infos, dt = once()
        ts.append(dt)
        last = (rc, infos)
    return last[0], last[1], sorted(ts)


def batched_leg(s7, torch, dev):
    """64 systems of uneven size (each side uniform over {24,...,128}), seeds 1000+s,
    tolerance 1e-7: the batched solver (median of five calls) against a loop of single
    solves."""
    import synth
    shapes, seeds = synth.batch_shapes(64, seed=0)
    coefs, bs, xs, xst = [], [], [], []
    for d, sd in zip(shapes, seeds):
        n = d[0] * d[1] * d[2]
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
        xx = torch.empty(n, dtype=torch.float64, device=dev)
        bb = torch.empty(n, dtype=torch.float64, device=dev)
        s7.generate_problem(d, sd, 0, c, xx, bb)
        coefs.append(c), bs.append(bb), xst.append(xx)
        xs.append(torch.zeros(n, dtype=torch.float64, device=dev))
    cells = [d[0] * d[1] * d[2] for d in shapes]
    ws = torch.empty(s7.batched_workspace_bytes(shapes), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    # the arguments are marshalled once; the timed region is the C call
    call = s7.batched_call(shapes, coefs, bs, xs, [1e-7] * 64, [2000] * 64, ws=ws,
                           opt=s7.default_options(tune=1))

    def batched():
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = call()
        torch.cuda.synchronize()
        return rc, infos, time.perf_counter() - t0

    batched()  # warm-up: autotunes the size class and captures the launch graph
    rc, infos, ts = repeat_timed(batched)
    dt = ts[len(ts) // 2]
    iters = [i.iters for i in infos]
    err = max(float(torch.linalg.vector_norm(x - xx) / torch.linalg.vector_norm(xx))
              for x, xx in zip(xs, xst))
    cell_iters = sum(c * k for c, k in zip(cells, iters))
    # the same systems, one single-system solve after another
    sws = torch.empty(max(s7.workspace_bytes(d) for d in shapes), dtype=torch.uint8, device=dev)
    o1 = s7.default_options(tune=1)
    for d, c, bb, x in zip(shapes, coefs, bs, xs):  # warm-up: tunes each size class
        s7.bicgstab_solve(d, c, bb, x, 1e-7, 3, ws=sws, opt=o1)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, c, bb, x in zip(shapes, coefs, bs, xs):
        s7.bicgstab_solve(d, c, bb, x, 1e-7, 2000, ws=sws, opt=o1)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t0
    return {
        "workload": "64 systems, sides uniform over {24,32,48,64,96,128}, FP32, rtol 1e-7",
        "cells": sum(cells), "status": rc, "iters_min_max": [min(iters), max(iters)],
        "systems_per_s": round(64 / dt, 2), "seconds": round(dt, 4),
        "seconds_min_max": [round(ts[0], 4), round(ts[-1], 4)], "timed_calls": len(ts),
        "cell_iters_per_s": round(cell_iters / dt, 1),
        "alg_GB/s": round(cell_iters * BATCH_BYTES / dt / 1e9, 1),
        # the one-time passes of every FP32 solve counted too (start, epilogue)
        "alg_GB/s_with_setup_bytes": round((cell_iters * BATCH_BYTES + sum(cells) * sum(SETUP_BYTES_FP32.values()))
                                           / dt / 1e9, 1),
        "max_rel_err_vs_xstar": err,
        "serial_single_solves_s": round(dts, 4), "speedup_vs_serial": round(dts / dt, 2),
    }


def batched_small_leg(s7, torch, dev, nsys: int = 256, side: int = 16):
    """Many tiny systems (256 of 16^3, seeds 3000+s, FP32 to 1e-7): one work item per
    phase and system, so the per-phase latency of a workgroup sets the time rather than
    bandwidth.  The batched solver (median of five calls) against a loop of single solves."""
    dims = (side, side, side)
    n = side ** 3
    coefs, bs, xs, xst = [], [], [], []
    for k in range(nsys):
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
        xx = torch.empty(n, dtype=torch.float64, device=dev)
        bb = torch.empty(n, dtype=torch.float64, device=dev)
        s7.generate_problem(dims, 3000 + k, 0, c, xx, bb)
        coefs.append(c), bs.append(bb), xst.append(xx)
        xs.append(torch.zeros(n, dtype=torch.float64, device=dev))
    shapes = [dims] * nsys
    ws = torch.empty(s7.batched_workspace_bytes(shapes), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    call = s7.batched_call(shapes, coefs, bs, xs, [1e-7] * nsys, [2000] * nsys, ws=ws,
                           opt=s7.default_options(tune=1))

    def batched():
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = call()
        torch.cuda.synchronize()
        return rc, infos, time.perf_counter() - t0

    batched()
    rc, infos, ts = repeat_timed(batched)
    dt = ts[len(ts) // 2]
    iters = [i.iters for i in infos]
    err = max(float(torch.linalg.vector_norm(x - xx) / torch.linalg.vector_norm(xx)) for x, xx in zip(xs, xst))
    sws = torch.empty(s7.workspace_bytes(dims), dtype=torch.uint8, device=dev)
    o1 = s7.default_options(tune=1)
    s7.bicgstab_solve(dims, coefs[0], bs[0], xs[0], 1e-7, 3, ws=sws, opt=o1)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c, bb, x in zip(coefs, bs, xs):
        s7.bicgstab_solve(dims, c, bb, x, 1e-7, 2000, ws=sws, opt=o1)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t0
    return {
        "workload": f"{nsys} systems of {side}^3, FP32, rtol 1e-7", "status": rc,
        "iters_min_max": [min(iters), max(iters)], "systems_per_s": round(nsys / dt, 1),
        "seconds": round(dt, 5), "seconds_min_max": [round(ts[0], 5), round(ts[-1], 5)],
        "us_per_iteration_per_system": round(dt / max(iters) * 1e6, 1),
        "max_rel_err_vs_xstar": err, "serial_single_solves_s": round(dts, 4),
        "speedup_vs_serial": round(dts / dt, 2),
    }


# Bytes per cell and iteration of the pipelined batched iteration (FP32, Jacobi):
# A reads r, w, p, s, r0, the stencil operands t, z, v and six coefficients and writes
# p, s, z, v, q, y; B reads y, t, v, q, p, d and six coefficients and writes d, r, w, t.
# The residual replacement every 10 iterations (about 20 B per cell and iteration) is
# not counted.
PIPE_BATCH_BYTES = (20 + 12 + 24 + 24) + (12 + 12 + 24 + 16)


def pipelined_batched_leg(s7, torch, dev):
    """The pipelined BiCGStab in the persistent batched kernel (two hand-offs per
    iteration) beside the classical batched solve (three), on the two batched workloads:
    64 systems of uneven size (seeds 1000+s, as the batched leg) and 256 systems of 16^3
    (seeds 3000+s), FP32 to 1e-7, each timed as the median of five calls."""
    import synth
    out = {}
    shapes64, seeds64 = synth.batch_shapes(64, seed=0)
    for key, shapes, seeds in (("64_uneven", shapes64, seeds64),
                               ("256_of_16cubed", [(16, 16, 16)] * 256, [3000 + k for k in range(256)])):
        coefs, bs, xs, xst = [], [], [], []
        for d, sd in zip(shapes, seeds):
            n = d[0] * d[1] * d[2]
            c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
            xx = torch.empty(n, dtype=torch.float64, device=dev)
            bb = torch.empty(n, dtype=torch.float64, device=dev)
            s7.generate_problem(d, sd, 0, c, xx, bb)
            coefs.append(c), bs.append(bb), xst.append(xx)
            xs.append(torch.zeros(n, dtype=torch.float64, device=dev))
        cells = [d[0] * d[1] * d[2] for d in shapes]
        ns = len(shapes)
        wsp = torch.empty(s7.batched_workspace_bytes_pipelined(shapes), dtype=torch.uint8, device=dev)
        wsc = torch.empty(s7.batched_workspace_bytes(shapes), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        calls = {
            "pipelined": s7.batched_pipelined_call(shapes, coefs, bs, xs, [1e-7] * ns, [2000] * ns, ws=wsp),
            "classical": s7.batched_call(shapes, coefs, bs, xs, [1e-7] * ns, [2000] * ns, ws=wsc,
                                         opt=s7.default_options(tune=1)),
        }
        res = {}
        for name, call in calls.items():
            def once():
                for x in xs:
                    x.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rc, infos = call()
                torch.cuda.synchronize()
                return rc, infos, time.perf_counter() - t0

            once()  # warm-up (the classical call autotunes its size class)
            rc, infos, ts = repeat_timed(once)
            dt = ts[len(ts) // 2]
            iters = [i.iters for i in infos]
            err = max(float(torch.linalg.vector_norm(x - xx) / torch.linalg.vector_norm(xx))
                      for x, xx in zip(xs, xst))
            cell_iters = sum(c * k for c, k in zip(cells, iters))
            r = {"status": rc, "seconds": round(dt, 5), "seconds_min_max": [round(ts[0], 5), round(ts[-1], 5)],
                 "systems_per_s": round(ns / dt, 1), "iters_min_max": [min(iters), max(iters)],
                 "iters_total": sum(iters), "max_rel_err_vs_xstar": err,
                 "max_rel_res_true": max(i.rel_res_true for i in infos)}
            bpc = PIPE_BATCH_BYTES if name == "pipelined" else BATCH_BYTES
            r["alg_GB/s"] = round(cell_iters * bpc / dt / 1e9, 1)
            r["bytes_per_cell_iter"] = bpc
            res[name] = r
        res["workload"] = (f"{ns} systems, FP32, rtol 1e-7, " +
                           ("sides uniform over {24,32,48,64,96,128}" if key == "64_uneven" else "16^3 each"))
        res["pipelined_time_over_classical"] = round(res["pipelined"]["seconds"] / res["classical"]["seconds"], 3)
        out[key] = res
        del coefs, bs, xs, xst, wsp, wsc, calls
        torch.cuda.empty_cache()
    return out


def cube256_leg(s7, torch, dev, steps: int, warmup: int, tune: bool):
    """256^3 with the anisotropic z-slab field (the z coefficients scaled up to 10x in a
    centred slab): `steps` fixed iterations timed on the graph path (iterations/s, GFLOPS
    and HBM fraction), the per-pass times from a second run with HIP events, then a run
    converged to a recurrence residual of 1e-6 (as the workload asks) and one to 1e-9,
    whose error against x* is below 1e-6 (the FP32 error floor is near 3e-7)."""
    import synth
    wl = synth.WORKLOADS["cube256_zslab"]
    dims = wl["dims"]
    n = dims[0] * dims[1] * dims[2]
    c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
    xs = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    s7.generate_problem(dims, wl["seed"], wl["recipe"], c, xs, b)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    ws = torch.empty(s7.workspace_bytes(dims), dtype=torch.uint8, device=dev)

    def run(iters, rtol=1e-300, profile=0):
        x.zero_()
        o = s7.default_options(profile=profile, tune=1 if tune else 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s7.bicgstab_solve(dims, c, b, x, rtol, iters, ws=ws, opt=o)
        torch.cuda.synchronize()
        return info, time.perf_counter() - t0

    run(warmup)
    info, dt = run(steps)
    assert info.iters == steps, info.as_dict()
    pinfo, _ = run(steps, profile=1)
    by = BYTES[("f32", PASSES[info.schedule])]
    pm = {k: pinfo.pass_ms[SLOT[k]] / max(pinfo.pass_count[SLOT[k]], 1) for k in by}
    out = {"workload": f"BiCGStab FP32 on {dims[0]}x{dims[1]}x{dims[2]}, z-slab anisotropy "
                       f"(recipe {wl['recipe']}, seed {wl['seed']}), {steps} fixed iterations",
           "iter_per_s": round(steps / dt, 2), "gflops": round(44 * n * steps / dt / 1e9, 1),
           "schedule": info.schedule,
           "hbm_frac_per_iteration": round(sum(by.values()) * n * steps / dt / 1e9 / HBM_PEAK_GBS, 4),
           "hbm_frac_kernels_only": round(sum(by.values()) * n / (sum(pm.values()) * 1e-3) / 1e9
                                          / HBM_PEAK_GBS, 4),
           "passes": {k: {"avg_ms": round(ms, 4), "GB/s": round(by[k] * n / (ms * 1e-3) / 1e9, 1)}
                      for k, ms in pm.items()}}
    for rtol in (1e-6, 1e-9):
        ic, tc = run(wl["max_iter"], rtol=rtol)
        out[f"converged_rtol{rtol:g}"] = {
            "status": ic.status, "iters": ic.iters, "seconds": round(tc, 4),
            "rel_res_true": ic.rel_res_true,
            "rel_err_vs_xstar": float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))}
    del c, xs, b, x, ws
    torch.cuda.empty_cache()
    return out


def pipelined_leg(s7, torch, dev, steps: int):
    """The pipelined BiCGStab against the classical solve, FP32, Jacobi: iterations per
    second on the paper's mesh (`steps` iterations, residual replacements included), and
    converged solves to 1e-6 on 256^3 and 32^3 (the latter where kernel boundaries and
    reductions, not bandwidth, set the time)."""
    out = {}
    for dims in ((600, 595, 1536), (256, 256, 256), (32, 32, 32)):
        n = dims[0] * dims[1] * dims[2]
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
        xs = torch.empty(n, dtype=torch.float64, device=dev)
        b = torch.empty(n, dtype=torch.float64, device=dev)
        s7.generate_problem(dims, 0, 0, c, xs, b)
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        wsp = torch.empty(s7.workspace_bytes_pipelined(dims), dtype=torch.uint8, device=dev)
        wsc = torch.empty(s7.workspace_bytes(dims), dtype=torch.uint8, device=dev)

        def timed(fn, rtol, iters):
            x.zero_()
            fn(rtol, 3)  # warm-up: graphs
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = fn(rtol, iters)
            torch.cuda.synchronize()
            return info, time.perf_counter() - t0

        pipe = lambda rtol, it: s7.bicgstab_solve_pipelined(dims, c, b, x, rtol, it, ws=wsp)
        clas = lambda rtol, it: s7.bicgstab_solve(dims, c, b, x, rtol, it, ws=wsc)
        key = "x".join(str(v) for v in dims)
        if n > 100_000_000:
            ip, tp = timed(pipe, 1e-300, steps)
            ic, tc = timed(clas, 1e-300, steps)
            out[key] = {"iterations": steps, "pipelined_iter_per_s": round(ip.iters / tp, 2),
                        "classical_iter_per_s": round(ic.iters / tc, 2)}
        else:
            ip, tp = timed(pipe, 1e-6, 2000)
            ep = float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))
            ic, tc = timed(clas, 1e-6, 2000)
            ec = float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))
            out[key] = {"rtol": 1e-6,
                        "pipelined": {"ms": round(tp * 1e3, 3), "iters": ip.iters, "status": ip.status,
                                      "rel_res_true": ip.rel_res_true, "rel_err_vs_xstar": ep},
                        "classical": {"ms": round(tc * 1e3, 3), "iters": ic.iters, "status": ic.status,
                                      "rel_res_true": ic.rel_res_true, "rel_err_vs_xstar": ec}}
        del c, xs, b, x, wsp, wsc
        torch.cuda.empty_cache()
    return out


def batched_2d9_leg(s7, torch, dev):
    """64 2D 9-point systems, each side uniform over {96,...,512}, seeds 2000+s,
    tolerance 1e-7: the batched solver (median of five calls) against a loop of single
    solves."""
    import synth
    shapes, seeds = synth.batch_shapes_2d9(64, seed=0)
    coefs, bs, xs, xst = [], [], [], []
    for (nx, ny), sd in zip(shapes, seeds):
        n = nx * ny
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(9)]
        xx = torch.empty(n, dtype=torch.float64, device=dev)
        bb = torch.empty(n, dtype=torch.float64, device=dev)
        s7.generate_problem_2d9(nx, ny, sd, c, xx, bb)
        coefs.append(c), bs.append(bb), xst.append(xx)
        xs.append(torch.zeros(n, dtype=torch.float64, device=dev))
    cells = [nx * ny for nx, ny in shapes]
    ws = torch.empty(s7.batched_workspace_bytes_2d9(shapes), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    call = s7.batched_call_2d9(shapes, coefs, bs, xs, [1e-7] * 64, [2000] * 64, ws=ws,
                               opt=s7.default_options(tune=1))

    def batched():
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, infos = call()
        torch.cuda.synchronize()
        return rc, infos, time.perf_counter() - t0

    batched()  # warm-up: autotunes the size class and captures the launch graph
    rc, infos, ts = repeat_timed(batched)
    dt = ts[len(ts) // 2]
    iters = [i.iters for i in infos]
    err = max(float(torch.linalg.vector_norm(x - xx) / torch.linalg.vector_norm(xx))
              for x, xx in zip(xs, xst))
    cell_iters = sum(c * k for c, k in zip(cells, iters))
    sws = torch.empty(max(s7.workspace_bytes_2d9(nx, ny) for nx, ny in shapes), dtype=torch.uint8, device=dev)
    for (nx, ny), c, bb, x in zip(shapes, coefs, bs, xs):  # warm-up: graphs per size
        s7.bicgstab_solve_2d9(nx, ny, c, bb, x, 1e-7, 3, ws=sws)
    for x in xs:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (nx, ny), c, bb, x in zip(shapes, coefs, bs, xs):
        s7.bicgstab_solve_2d9(nx, ny, c, bb, x, 1e-7, 2000, ws=sws)
    torch.cuda.synchronize()
    dts = time.perf_counter() - t0
    return {
        "workload": "64 2D 9-point systems, sides uniform over {96,128,192,256,384,512}, FP32, rtol 1e-7",
        "cells": sum(cells), "status": rc, "iters_min_max": [min(iters), max(iters)],
        "systems_per_s": round(64 / dt, 2), "seconds": round(dt, 4),
        "seconds_min_max": [round(ts[0], 4), round(ts[-1], 4)], "timed_calls": len(ts),
        "cell_iters_per_s": round(cell_iters / dt, 1),
        "alg_GB/s": round(cell_iters * sum(BYTES_2D9.values()) / dt / 1e9, 1),
        "max_rel_err_vs_xstar": err,
        "serial_single_solves_s": round(dts, 4), "speedup_vs_serial": round(dts / dt, 2),
    }


def simple_leg(s7, torch, dev, dims, outer: int):
    """The solver pattern of Algorithm 2 (SIMPLE): per outer iteration the momentum
    systems u, v, w, capped at 5 BiCGStab iterations, then the continuity system, capped
    at 20; every solve warm-starts from its previous solution.  The three momentum solves
    go into one batched call, against three single-system calls; both autotuned.  On the paper's
    100x400x100 momentum mesh (4M cells) the batched call runs each system alone (at
    least split_cells cells); on a compact mesh they share one persistent launch."""
    dims = tuple(dims)
    n = dims[0] * dims[1] * dims[2]
    coefs, bs, xs = [], [], []
    for f in range(4):
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
        xx = torch.empty(n, dtype=torch.float64, device=dev)
        bb = torch.empty(n, dtype=torch.float64, device=dev)
        s7.generate_problem(dims, 2000 + f, 0, c, xx, bb)
        coefs.append(c), bs.append(bb)
        xs.append(torch.zeros(n, dtype=torch.float64, device=dev))
    ws = torch.empty(max(s7.batched_workspace_bytes([dims] * 3), s7.workspace_bytes(dims)),
                     dtype=torch.uint8, device=dev)

    o = s7.default_options(tune=1)

    def run(batched: bool):
        for x in xs:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(outer):
            if batched:
                s7.bicgstab_solve_batched([dims] * 3, coefs[:3], bs[:3], xs[:3], [1e-12] * 3, [5] * 3, ws=ws,
                                          opt=o)
            else:
                for f in range(3):
                    s7.bicgstab_solve(dims, coefs[f], bs[f], xs[f], 1e-12, 5, ws=ws, opt=o)
            s7.bicgstab_solve(dims, coefs[3], bs[3], xs[3], 1e-12, 20, ws=ws, opt=o)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    run(True)  # warm-up: autotunes each size class and captures the launch graphs
    run(False)
    tb, ts = run(True), run(False)
    return {"workload": f"SIMPLE pattern on {dims[0]}x{dims[1]}x{dims[2]}: u, v, w capped at 5 "
                        f"iterations, p at 20, "
                        f"warm-started, {outer} outer iterations",
            "outer_per_s_batched": round(outer / tb, 2), "outer_per_s_single": round(outer / ts, 2),
            "us_per_cell_outer_batched": round(tb / outer / n * 1e6, 5)}


# 2D 9-point, Jacobi (8 coefficient arrays), FP32: algorithmic bytes per cell
BYTES_2D9 = {"p1": (1 + 1 + 8) * 4 + 4,   # p, r0, 8 coef; s
             "p2": (2 + 1 + 8) * 4 + 4,   # r, s, r0, 8 coef; y
             "p3": 6 * 4 + 3 * 4}         # d, p, r, s, y, r0; d, r, p


BYTES_2D9_16 = {"p1": (1 + 1 + 8) * 2 + 2,
                "p2": (2 + 1 + 8) * 2 + 2,
                "p3": 4 + 5 * 2 + 4 + 2 * 2}  # d FP32; p, r, s, y, r0 16-bit; d, r, p written


def stencil9_leg(s7, torch, dev, steps: int, warmup: int):
    """The 2D 9-point workload of section IV at the two sizes the paper names: FP32
    BiCGStab, `steps` timed iterations with the passes timed by HIP events, and the
    BF16 inner iteration inside FP64 refinement."""
    out = []
    for nx, ny in ((4800, 4800), (22800, 22800)):
        n = nx * ny
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(9)]
        xs = torch.empty(n, dtype=torch.float64, device=dev)
        b = torch.empty(n, dtype=torch.float64, device=dev)
        s7.generate_problem_2d9(nx, ny, 0, c, xs, b)
        # s7_stencil9_apply alone: u = A v with the nine caller arrays, 44 B per cell
        v = xs.to(torch.float32)
        u = torch.empty_like(v)
        stream = torch.cuda.current_stream()
        for _ in range(3):
            s7.stencil9_apply(nx, ny, c, v, u, stream=stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            s7.stencil9_apply(nx, ny, c, v, u, stream=stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        apply_ms = e0.elapsed_time(e1) / 20
        del v, u
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        ws = torch.empty(max(s7.workspace_bytes_2d9(nx, ny, pr) for pr in (s7.FP32, s7.BF16_IR)),
                         dtype=torch.uint8, device=dev)
        o = s7.default_options(profile=1)
        s7.bicgstab_solve_2d9(nx, ny, c, b, x, 1e-300, warmup, ws=ws, opt=o)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s7.bicgstab_solve_2d9(nx, ny, c, b, x, 1e-300, steps, ws=ws, opt=o)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pm = {k: info.pass_ms[SLOT[k]] / max(info.pass_count[SLOT[k]], 1) for k in BYTES_2D9}
        per_iter = sum(BYTES_2D9.values()) * n
        # a converged run to rtol 1e-8: error against the manufactured solution
        x.zero_()
        conv = s7.bicgstab_solve_2d9(nx, ny, c, b, x, 1e-8, 2000, ws=ws)
        err = float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))
        # BF16 storage inside FP64 refinement: inner iterations timed, then converged to 1e-10
        x.zero_()
        s7.bicgstab_solve_2d9(nx, ny, c, b, x, 1e-300, warmup, prec=s7.BF16_IR, ws=ws, opt=o)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i16 = s7.bicgstab_solve_2d9(nx, ny, c, b, x, 1e-300, steps, prec=s7.BF16_IR, ws=ws, opt=o)
        torch.cuda.synchronize()
        dt16 = time.perf_counter() - t0
        x.zero_()
        c16 = s7.bicgstab_solve_2d9(nx, ny, c, b, x, 1e-10, 2000, prec=s7.BF16_IR, ws=ws)
        err16 = float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))
        out.append({"workload": f"2D 9-point, FP32, Jacobi, {nx}x{ny} ({n} cells)",
                    "stencil9_apply": {"avg_launch_ms": round(apply_ms, 4), "bytes_per_cell": 44,
                                       "GB/s": round(44 * n / (apply_ms * 1e-3) / 1e9, 1),
                                       "frac": round(44 * n / (apply_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                    "bf16_ir": {"inner_iter_per_s": round(i16.iters / dt16, 2),
                                "bytes_per_cell_inner_iteration": sum(BYTES_2D9_16.values()),
                                "converged_rtol1e-10": {"status": c16.status, "inner_iters": c16.iters,
                                                        "outer": c16.outer_iters, "rel_res_true": c16.rel_res_true,
                                                        "rel_err_vs_xstar": err16}},
                    "iter_per_s": round(info.iters / dt, 2),
                    "bytes_per_cell_iteration": sum(BYTES_2D9.values()),
                    "hbm_frac_per_iteration": round(per_iter * info.iters / dt / 1e9 / HBM_PEAK_GBS, 4),
                    "passes": {k: {"avg_ms": round(ms, 4), "GB/s": round(BYTES_2D9[k] * n / (ms * 1e-3) / 1e9, 1)}
                               for k, ms in pm.items()},
                    "converged_rtol1e-8": {"status": conv.status, "iters": conv.iters,
                                           "rel_res_true": conv.rel_res_true, "rel_err_vs_xstar": err}})
        del c, xs, b, x, ws
        torch.cuda.empty_cache()
    return out


def served_leg(s7, torch, dev, nreq: int, rate: float, burst: int, arena_gb: float, sample: int):
    """The request stream: Poisson arrivals at `rate` per second, sides log-uniform in
    [16,256] per axis, half FP32 at rtol 1e-6 and half BF16 + FP64 refinement at 1e-10.
    The queue (continuous batching) and a serial loop of single-system solves serve the
    same stream.  Latency runs from the scheduled arrival to the result; it includes the
    client's generation of the request's inputs on the device."""
    import queue as pyqueue
    import threading

    import numpy as np

    import synth
    prec_of = {"fp32": s7.FP32, "bf16_ir": s7.BF16_IR}
    gen_stream = torch.cuda.Stream(device=dev)

    def make(r):
        n = r.dims[0] * r.dims[1] * r.dims[2]
        with torch.cuda.stream(gen_stream):
            c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
            xx = torch.empty(n, dtype=torch.float64, device=dev)
            bb = torch.empty(n, dtype=torch.float64, device=dev)
            x = torch.zeros(n, dtype=torch.float64, device=dev)
        s7.generate_problem(r.dims, r.seed, 0, c, xx, bb, stream=gen_stream)
        gen_stream.synchronize()
        return c, bb, x, xx

    def err_of(x, xx):
        return float(torch.linalg.vector_norm(x - xx) / torch.linalg.vector_norm(xx))

    def summarize(rs, lat, t_first, t_last, errs, status):
        lat = np.array(lat) * 1e3
        out = {"solves_per_s": round(len(lat) / (t_last - t_first), 2),
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "mean_ms": round(float(lat.mean()), 3), "max_ms": round(float(lat.max()), 3),
               "not_ok": int(sum(1 for st in status if st != s7.OK))}
        for m in ("fp32", "bf16_ir"):
            e = [v for r, v in zip(rs, errs) if r.mode == m]
            if e:
                out[f"max_rel_err_vs_xstar_{m}"] = float(f"{max(e):.3e}")
        return out

    def run_queue(rs, arena, keep=()):
        q = s7.queue_create(arena)
        handoff = pyqueue.Queue()
        t0 = time.perf_counter()

        def producer():
            try:
                for r in rs:
                    wait = t0 + r.arrival_s - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                    c, bb, x, xx = make(r)
                    t_sub = time.perf_counter()
                    tk = s7.queue_submit(q, r.dims, c, bb, x, r.rtol, 4000, prec_of[r.mode])
                    handoff.put((r, tk, t_sub, c, bb, x, xx))
            finally:
                handoff.put(None)

        th = threading.Thread(target=producer)
        th.start()
        lat, errs, status, kept, done = [], [], [], {}, []
        while True:
            item = handoff.get()
            if item is None:
                break
            r, tk, t_sub, c, bb, x, xx = item
            rc, info = s7.queue_wait(q, tk)
            t_done = t_sub + info.t_ms * 1e-3
            done.append(t_done)
            lat.append(t_done - (t0 + r.arrival_s))
            status.append(rc)
            errs.append(err_of(x, xx))
            if r.rid in keep:
                kept[r.rid] = x.clone()
        th.join()
        s7.queue_destroy(q)
        if len(status) != len(rs):
            raise RuntimeError("the request producer stopped early")
        return summarize(rs, lat, t0 + rs[0].arrival_s, max(done), errs, status), kept

    def run_serial(rs):
        ws = torch.empty(max(s7.workspace_bytes(r.dims, prec_of[r.mode]) for r in rs),
                         dtype=torch.uint8, device=dev)
        t0 = time.perf_counter()
        lat, errs, status = [], [], []
        for r in rs:
            wait = t0 + r.arrival_s - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            c, bb, x, xx = make(r)
            info = s7.bicgstab_solve(r.dims, c, bb, x, r.rtol, 4000, prec=prec_of[r.mode], ws=ws)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - (t0 + r.arrival_s))
            status.append(info.status)
            errs.append(err_of(x, xx))
        return summarize(rs, lat, t0 + rs[0].arrival_s, time.perf_counter(), errs, status)

    arena = torch.empty(int(arena_gb * (1 << 30)), dtype=torch.uint8, device=dev)
    res = {"workload": f"{nreq} requests, Poisson arrivals at {rate:g}/s, sides log-uniform in "
                       f"[16,256] per axis, 50/50 FP32 rtol 1e-6 / BF16+FP64 IR rtol 1e-10",
           "arena_GiB": arena_gb, "latency": "scheduled arrival to result"}
    warm = synth.serve_stream(8, rate=1e9, seed=1)
    run_queue(warm, arena)
    run_serial(warm)

    reqs = synth.serve_stream(nreq, rate=rate, seed=0)
    print(f"[bench] served stream: {nreq} requests at {rate:g}/s through the queue",
          file=sys.stderr, flush=True)
    keep = set(r.rid for r in reqs[:: max(1, nreq // sample)]) if sample else set()
    res["queue"], kept = run_queue(reqs, arena, keep)
    print("[bench] served stream: serial single-system loop", file=sys.stderr, flush=True)
    res["serial"] = run_serial(reqs)
    if burst:
        # capacity: the first `burst` requests all arrive at once
        br = [synth.Request(r.rid, 0.0, r.dims, r.mode, r.rtol, r.seed) for r in reqs[:burst]]
        print(f"[bench] burst of {burst} requests", file=sys.stderr, flush=True)
        res["burst"] = {"requests": burst, "queue": run_queue(br, arena)[0], "serial": run_serial(br)}
    # each sampled request solved alone, through the path the queue gave it (the batch
    # engine, or the single-system path from 2^21 cells), must match its served result
    same = 0
    for rid in sorted(kept):
        r = reqs[rid]
        c, bb, x, xx = make(r)
        if r.dims[0] * r.dims[1] * r.dims[2] >= SPLIT_CELLS:
            s7.bicgstab_solve(r.dims, c, bb, x, r.rtol, 4000, prec=prec_of[r.mode])
        else:
            s7.bicgstab_solve_batched([r.dims], [c], [bb], [x], [r.rtol], [4000], prec=prec_of[r.mode])
        torch.cuda.synchronize()
        same += bool(torch.equal(x, kept[rid]))
    res["alone_vs_mix_identical"] = f"{same}/{len(kept)}"
    return res

def served_2d9_leg(s7, torch, dev, nreq: int, arena_gb: float, sample: int = 10):
    """A burst of `nreq` 2D 9-point requests arriving at once: sides log-uniform in
    [64, 1024] per axis, 50/50 FP32 rtol 1e-6 / BF16+FP64 IR rtol 1e-10.  The queue and a
    serial loop of single-system calls serve the same burst; the inputs are generated
    beforehand, and latency runs from the burst's start to each result."""
    import numpy as np

    import synth
    prec_of = {"fp32": s7.FP32, "bf16_ir": s7.BF16_IR}
    reqs = synth.serve_stream_2d9(nreq, seed=0)

    def make(r):
        nx, ny = r.dims
        n = nx * ny
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(9)]
        xx = torch.empty(n, dtype=torch.float64, device=dev)
        bb = torch.empty(n, dtype=torch.float64, device=dev)
        s7.generate_problem_2d9(nx, ny, r.seed, c, xx, bb)
        return c, bb, torch.zeros(n, dtype=torch.float64, device=dev), xx

    data = [make(r) for r in reqs]
    torch.cuda.synchronize()
    arena = torch.empty(int(arena_gb * (1 << 30)), dtype=torch.uint8, device=dev)

    def summarize(rs, lat, t_total, status):
        lat = np.array(lat) * 1e3
        out = {"solves_per_s": round(len(lat) / t_total, 2),
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "not_ok": int(sum(1 for st in status if st != s7.OK))}
        for m in ("fp32", "bf16_ir"):
            e = [float(torch.linalg.vector_norm(d[2] - d[3]) / torch.linalg.vector_norm(d[3]))
                 for r, d in zip(rs, data) if r.mode == m]
            if e:
                out[f"max_rel_err_vs_xstar_{m}"] = float(f"{max(e):.3e}")
        return out

    def run_queue(rs):
        for d in data[:len(rs)]:
            d[2].zero_()
        torch.cuda.synchronize()
        q = s7.queue_create(arena)
        t0 = time.perf_counter()
        subs = []
        for r, (c, bb, x, xx) in zip(rs, data):
            subs.append((time.perf_counter(), s7.queue_submit_2d9(q, *r.dims, c, bb, x, r.rtol, 4000,
                                                                 prec_of[r.mode])))
        lat, status = [], []
        for t_sub, tk in subs:
            rc, info = s7.queue_wait(q, tk)
            lat.append(t_sub - t0 + info.t_ms * 1e-3)
            status.append(rc)
        s7.queue_destroy(q)
        return summarize(rs, lat, max(lat), status)

    def run_serial(rs):
        ws = torch.empty(max(s7.workspace_bytes_2d9(*r.dims, prec_of[r.mode]) for r in rs),
                         dtype=torch.uint8, device=dev)
        for d in data[:len(rs)]:
            d[2].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, status = [], []
        for r, (c, bb, x, xx) in zip(rs, data):
            info = s7.bicgstab_solve_2d9(*r.dims, c, bb, x, r.rtol, 4000, prec=prec_of[r.mode], ws=ws)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            status.append(info.status)
        return summarize(rs, lat, lat[-1], status)

    run_queue(reqs[:8])  # warm-up
    run_serial(reqs[:8])
    res = {"workload": f"burst of {nreq} 2D 9-point requests, sides log-uniform in [64,1024] per axis, "
                       f"50/50 FP32 rtol 1e-6 / BF16+FP64 IR rtol 1e-10",
           "cells": sum(r.dims[0] * r.dims[1] for r in reqs), "latency": "burst start to result"}
    print(f"[bench] served 2D burst: {nreq} requests through the queue", file=sys.stderr, flush=True)
    res["queue"] = run_queue(reqs)
    keep = list(range(0, nreq, max(1, nreq // sample)))
    kept = {i: data[i][2].clone() for i in keep}
    print("[bench] served 2D burst: serial single-system loop", file=sys.stderr, flush=True)
    res["serial"] = run_serial(reqs)
    # each sampled request solved alone by the batched 2D call must match its served result
    same = 0
    for i in keep:
        r, (c, bb, x, xx) = reqs[i], data[i]
        x.zero_()
        s7.bicgstab_solve_batched_2d9([r.dims], [c], [bb], [x], [r.rtol], [4000], prec=prec_of[r.mode])
        torch.cuda.synchronize()
        same += bool(torch.equal(x, kept[i]))
    res["alone_vs_mix_identical"] = f"{same}/{len(keep)}"
    del data, arena
    torch.cuda.empty_cache()
    return res


def served_mixed_leg(s7, torch, dev, nreq: int, rate: float):
    """3D and 2D requests in one Poisson stream at `rate` per second (each operator half
    of it: the 3D stream's sides log-uniform in [16,256] per axis, the 2D stream's in
    [64,1024]; 50/50 FP32 rtol 1e-6 / BF16+FP64 IR rtol 1e-10), through the queue and
    through a serial loop of single-system calls.  Inputs are generated beforehand;
    latency runs from the scheduled arrival to the result."""
    import queue as pyqueue
    import threading

    import numpy as np

    import synth
    prec_of = {"fp32": s7.FP32, "bf16_ir": s7.BF16_IR}
    half = nreq // 2
    reqs = [("3d", r) for r in synth.serve_stream(half, rate=rate / 2, seed=5)]
    reqs += [("2d", r) for r in synth.serve_stream_2d9(nreq - half, rate=rate / 2, seed=5)]
    reqs.sort(key=lambda kr: kr[1].arrival_s)

    def make(kind, r):
        n = int(np.prod(r.dims))
        c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7 if kind == "3d" else 9)]
        xx = torch.empty(n, dtype=torch.float64, device=dev)
        bb = torch.empty(n, dtype=torch.float64, device=dev)
        if kind == "3d":
            s7.generate_problem(r.dims, r.seed, 0, c, xx, bb)
        else:
            s7.generate_problem_2d9(*r.dims, r.seed, c, xx, bb)
        return c, bb, torch.zeros(n, dtype=torch.float64, device=dev), xx

    data = [make(k, r) for k, r in reqs]
    torch.cuda.synchronize()
    arena = torch.empty(32 << 30, dtype=torch.uint8, device=dev)

    def summarize(lat, status):
        out = {}
        for kind in ("3d", "2d"):
            v = np.array([t for (k, r), t in zip(reqs, lat) if k == kind]) * 1e3
            out[kind] = {"p50_ms": round(float(np.percentile(v, 50)), 3),
                         "p99_ms": round(float(np.percentile(v, 99)), 3)}
        out["not_ok"] = int(sum(1 for st in status if st != s7.OK))
        out["max_rel_err_vs_xstar"] = float(f"{max(float(torch.linalg.vector_norm(d[2] - d[3]) / torch.linalg.vector_norm(d[3])) for d in data):.3e}")
        return out

    def run_queue():
        for d in data:
            d[2].zero_()
        torch.cuda.synchronize()
        q = s7.queue_create(arena)
        handoff = pyqueue.Queue()
        t0 = time.perf_counter()

        def producer():
            try:
                for (kind, r), (c, bb, x, xx) in zip(reqs, data):
                    wait = t0 + r.arrival_s - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                    t_sub = time.perf_counter()
                    if kind == "3d":
                        tk = s7.queue_submit(q, r.dims, c, bb, x, r.rtol, 4000, prec_of[r.mode])
                    else:
                        tk = s7.queue_submit_2d9(q, *r.dims, c, bb, x, r.rtol, 4000, prec_of[r.mode])
                    handoff.put((r, tk, t_sub))
            finally:
                handoff.put(None)

        th = threading.Thread(target=producer)
        th.start()
        lat, status = [], []
        while True:
            item = handoff.get()
            if item is None:
                break
            r, tk, t_sub = item
            rc, info = s7.queue_wait(q, tk)
            lat.append(t_sub + info.t_ms * 1e-3 - (t0 + r.arrival_s))
            status.append(rc)
        th.join()
        s7.queue_destroy(q)
        if len(status) != len(reqs):
            raise RuntimeError("the request producer stopped early")
        return summarize(lat, status)

    def run_serial():
        ws = torch.empty(max(s7.workspace_bytes(r.dims, prec_of[r.mode]) if k == "3d" else
                             s7.workspace_bytes_2d9(*r.dims, prec_of[r.mode]) for k, r in reqs),
                         dtype=torch.uint8, device=dev)
        for d in data:
            d[2].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, status = [], []
        for (kind, r), (c, bb, x, xx) in zip(reqs, data):
            wait = t0 + r.arrival_s - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            if kind == "3d":
                info = s7.bicgstab_solve(r.dims, c, bb, x, r.rtol, 4000, prec=prec_of[r.mode], ws=ws)
            else:
                info = s7.bicgstab_solve_2d9(*r.dims, c, bb, x, r.rtol, 4000, prec=prec_of[r.mode], ws=ws)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - (t0 + r.arrival_s))
            status.append(info.status)
        return summarize(lat, status)

    print(f"[bench] mixed 3D/2D stream: {nreq} requests at {rate:g}/s", file=sys.stderr, flush=True)
    res = {"workload": f"{nreq} requests, Poisson at {rate:g}/s, half 3D 7-point (sides log-uniform in [16,256]) "
                       f"and half 2D 9-point (sides in [64,1024]), 50/50 FP32 rtol 1e-6 / BF16+FP64 IR rtol 1e-10",
           "latency": "scheduled arrival to result", "queue": run_queue()}
    print("[bench] mixed 3D/2D stream: serial single-system loop", file=sys.stderr, flush=True)
    res["serial"] = run_serial()
    del data, arena
    torch.cuda.empty_cache()
    return res


# Streaming probes of s7_bandwidth_probe: kind & 3 selects the pattern, +4 non-temporal
# stores, +8 non-temporal loads.  Bytes moved per element of each of the three arrays.
PROBE_KINDS = [("read", 0, 4), ("read NT", 8, 4), ("copy", 1, 8), ("copy NT", 13, 8),
               ("triad", 2, 12), ("triad NT", 14, 12), ("6R/2W", 3, 16), ("6R/2W NT", 15, 16)]
# bytes read and written per element, for the counter calibration
PROBE_RW = {0: (4, 0), 1: (4, 4), 2: (8, 4), 3: (12, 4)}


def probe_leg(s7, torch, dev, counters_only: bool):
    """The streaming ceilings of this GPU: each probe over three 2 GiB arrays with 16-byte
    accesses, timed with HIP events for several grid sizes (best median reported).  With
    counters_only, one dispatch of each probe at 1024 workgroups: the calibration run for
    the byte counters (its kernels run in the order of PROBE_KINDS)."""
    n = 1 << 29
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.ones(n, dtype=torch.float32, device=dev)
    c = torch.ones(n, dtype=torch.float32, device=dev)
    out = {"elements_per_array": n, "kinds": {}}
    for name, kind, bpe in PROBE_KINDS:
        rd, wr = PROBE_RW[kind & 3]
        if counters_only:
            s7.bandwidth_probe(kind, 4, a, b, c, n, 1024)
            torch.cuda.synchronize()
            out["kinds"][name] = {"kind": kind, "read_bytes": rd * n, "write_bytes": wr * n}
            continue
        best = None
        for blocks in (256, 1024, 4096, 16384):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ts = []
            for _ in range(6):
                e0.record()
                s7.bandwidth_probe(kind, 4, a, b, c, n, blocks)  # torch's current stream
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
            med = sorted(ts[1:])[len(ts[1:]) // 2]
            gbs = bpe * n / (med * 1e-3) / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, blocks, med)
        out["kinds"][name] = {"kind": kind, "GB/s": round(best[0], 1), "blocks": best[1],
                              "median_ms": round(best[2], 4), "frac_of_8TBs": round(best[0] / HBM_PEAK_GBS, 4)}
    return out


# The P2 kernel designs of s7_p2_design_probe, in the order they are reported
P2_DESIGNS = [("flat cell pairs", 0, 0), ("one-plane tiles, plain order", 1, 1),
              ("one-plane tiles, band per XCD", 1, 0), ("two-plane tiles, plain order", 2, 1),
              ("two-plane tiles, band per XCD", 2, 0), ("z-march, 8 planes", 3, 8),
              ("z-march, 16 planes", 3, 16), ("z-march, 32 planes", 3, 32), ("z-march, 64 planes", 3, 64)]


def p2_designs_leg(s7, torch, dev, dims, reps: int = 10):
    """The P2 pass (q = r - alpha s on the fly, y = A q, five sums) in the kernel designs of
    s7_p2_design_probe, on the unit-diagonal operator of the seeded recipe at `dims` with
    random r, s, r0: ms per launch (HIP events, average of `reps` after a warm-up) and the
    algorithmic rate at 40 B per cell.  Every design must write the same y as the first."""
    nx, ny, nz = dims
    n = nx * ny * nz
    c = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
    s7.generate_problem(dims, 0, 0, c, None, None)
    w = []
    for a in range(1, 7):
        v = (c[a] / c[0]).view(nz, ny, nx)
        # outward links zeroed on the faces: w, e, s, n, b, t
        [lambda t: t[:, :, 0], lambda t: t[:, :, -1], lambda t: t[:, 0, :], lambda t: t[:, -1, :],
         lambda t: t[0], lambda t: t[-1]][a - 1](v).zero_()
        w.append(v.reshape(-1))
    del c
    g = torch.Generator(device=dev).manual_seed(7)
    r = torch.rand(n, dtype=torch.float32, device=dev, generator=g) - 0.5
    s = torch.rand(n, dtype=torch.float32, device=dev, generator=g) - 0.5
    rh = torch.rand(n, dtype=torch.float32, device=dev, generator=g) - 0.5
    y = torch.empty(n, dtype=torch.float32, device=dev)
    y0 = None
    rows = []
    for name, kind, param in P2_DESIGNS:
        ms, _ = s7.p2_design_probe(kind, param, dims, w, r, s, rh, 0.37, y, reps=reps)
        torch.cuda.synchronize()
        if y0 is None:
            y0 = y.clone()
        rows.append({"design": name, "kind": kind, "param": param, "ms": round(ms, 4),
                     "GB/s_at_40B": round(40.0 * n / (ms * 1e-3) / 1e9, 1),
                     "frac_of_8TBs": round(40.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "y_same_as_first": bool(torch.equal(y, y0))})
    return {"workload": f"P2 designs at {nx}x{ny}x{nz}, FP32, unit diagonal", "cells": n, "reps": reps,
            "designs": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dims", type=str, default="600,595,1536")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--cpu-slab", type=int, default=64)
    ap.add_argument("--cpu-iters", type=int, default=48)
    ap.add_argument("--schedule", type=int, default=0, choices=(0, 1, 2, 3, 5),
                    help="schedule of the single-system solver (s7_options.schedule: 1 three passes, "
                         "2 four, 3 three on cell pairs, 5 three with LDS-staged stencil operands; "
                         "0: autotuned, or the library's default with --no-tune)")
    ap.add_argument("--no-tune", action="store_true",
                    help="fixed default launch parameters instead of autotuned ones")
    ap.add_argument("--lds-tile", type=int, default=0, choices=(0, 2048, 4096, 8192),
                    help="tile of the staged passes (s7_options.lds_tile; 0: tuned, or 4096 with --no-tune)")
    ap.add_argument("--xcd-run", type=int, default=0,
                    help="XCD tile order of the stencil passes (s7_options.xcd_run; 0: tuned, or plain with --no-tune)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-simple", action="store_true")
    ap.add_argument("--no-shard", action="store_true")
    ap.add_argument("--no-apply", action="store_true", help="skip the stencil_apply leg")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed calls of the headline for its median and spread (0: none)")
    ap.add_argument("--no-2d9", action="store_true")
    ap.add_argument("--no-pipelined", action="store_true")
    ap.add_argument("--simple-dims", type=int, nargs=3, default=[100, 400, 100])
    ap.add_argument("--simple-outer", type=int, default=15)
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the served stream (the whole workload is 10000)")
    ap.add_argument("--no-cube256", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-burst", type=int, default=400,
                    help="requests of the all-at-once capacity run (0: skip)")
    ap.add_argument("--serve-sample", type=int, default=100,
                    help="served requests re-solved alone for the identity check")
    ap.add_argument("--arena-gb", type=float, default=64.0)
    ap.add_argument("--serve-mixed", type=int, default=400,
                    help="requests in the mixed 3D/2D Poisson stream leg (0: skip)")
    ap.add_argument("--serve-2d9-burst", type=int, default=200,
                    help="2D 9-point requests in the served burst leg (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run one dispatch of each streaming probe on 2 GiB arrays "
                         "(calibrates the HBM byte counters)")
    ap.add_argument("--p2-designs", action="store_true",
                    help="only time the P2 kernel designs of s7_p2_design_probe at --dims and print one JSON line")
    ap.add_argument("--probe", action="store_true",
                    help="only measure the streaming ceilings (copy, triad, 6-read/2-write, read-only; "
                         "cached and non-temporal) and print them as JSON")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this solver has no multi-GPU path (z-slab sharding is "
              "a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2010_03660_amd as s7
    s7.lib()
    dev = torch.device("cuda:0")

    if args.p2_designs:
        print(json.dumps(p2_designs_leg(s7, torch, dev, tuple(int(v) for v in args.dims.split(",")))), flush=True)
        return
    if args.copy_probe or args.probe:
        print(json.dumps(probe_leg(s7, torch, dev, counters_only=args.copy_probe)), flush=True)
        return

    nx, ny, nz = (int(v) for v in args.dims.split(","))
    n = nx * ny * nz
    dims = (nx, ny, nz)
    print(f"[bench] mesh {nx}x{ny}x{nz} ({n} cells): generating on device", file=sys.stderr,
          flush=True)
    coef = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(7)]
    xs = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.empty(n, dtype=torch.float64, device=dev)
    s7.generate_problem(dims, 0, 0, coef, xs, b)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    ws_bytes = max(s7.workspace_bytes(dims, p) for p in (s7.FP32, s7.BF16_IR))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def run(prec, iters, rtol=1e-300, profile=0):
        x.zero_()
        o = s7.default_options(profile=profile, schedule=args.schedule, lds_tile=args.lds_tile,
                               xcd_run=args.xcd_run, tune=0 if args.no_tune else 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s7.bicgstab_solve(dims, coef, b, x, rtol, iters, prec=prec, ws=ws, opt=o)
        torch.cuda.synchronize()
        return info, time.perf_counter() - t0

    # ---- plain FP32: warmup, then exactly `steps` timed iterations on the production
    # path (iterations replayed from captured hipGraphs)
    print(f"[bench] FP32 warmup {args.warmup} iterations", file=sys.stderr, flush=True)
    run(s7.FP32, args.warmup)
    print(f"[bench] FP32 timed {args.steps} iterations", file=sys.stderr, flush=True)
    info, dt = run(s7.FP32, args.steps)
    assert info.iters == args.steps, info.as_dict()
    ips = args.steps / dt
    sched = info.schedule  # the schedule the (tuned) solve ran
    # the same timed call repeated: median and spread beside the one timed region above
    rep_ips = []
    for _ in range(args.repeats):
        rinfo, rdt = run(s7.FP32, args.steps)
        assert rinfo.iters == args.steps, rinfo.as_dict()
        rep_ips.append(args.steps / rdt)
    rep_ips.sort()
    # the same steps again without graphs, every pass bracketed by HIP events on the
    # solver's stream: the per-kernel times of the roofline
    print(f"[bench] FP32 {args.steps} iterations with per-pass HIP events", file=sys.stderr, flush=True)
    pinfo, pdt = run(s7.FP32, args.steps, profile=1)
    assert pinfo.iters == args.steps and pinfo.schedule == sched, pinfo.as_dict()
    bytes32 = BYTES[("f32", PASSES[sched])]
    pass_ms = {k: pinfo.pass_ms[SLOT[k]] / max(pinfo.pass_count[SLOT[k]], 1) for k in bytes32}
    dom = max(bytes32, key=lambda k: pass_ms[k])  # the kernel with the largest share of an iteration
    dom_gbs = bytes32[dom] * n / (pass_ms[dom] * 1e-3) / 1e9
    iter_bytes = sum(bytes32.values()) * n
    kernel_ms_iter = sum(pass_ms.values())
    traffic = traffic_from_profile(n, dom, sched, pinfo.lds_tile, pinfo.xcd_run if sched == 5 else 0)
    roofline = {"bound": "hbm", "kernel": KERNEL[sched][dom],
                "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": bytes32[dom] * n,
                "bytes_per_cell": bytes32[dom], "lds_tile": pinfo.lds_tile, "xcd_run": pinfo.xcd_run,
                "avg_launch_ms": round(pass_ms[dom], 4),
                "frac_at_survey_bytes_per_cell": round(SURVEY_BYTES[dom] * n / (pass_ms[dom] * 1e-3) / 1e9
                                                       / HBM_PEAK_GBS, 4)
                if sched in (1, 3, 5) else None,
                "timing": "HIP events around each launch on the solver's stream, averaged over a second "
                          "run of the same steps without graphs"}
    passes = {k: {"avg_ms": round(ms, 4), "GB/s": round(bytes32[k] * n / (ms * 1e-3) / 1e9, 1)}
              for k, ms in pass_ms.items()}
    survey_iter_bytes = sum(SURVEY_BYTES.values()) * n
    out = {
        "metric": "BiCGStab iter/s + %HBM peak at 600x595x1536; served solves/s, p99 latency",
        "value": round(ips, 3), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded 7-point variable-coefficient recipe, b = A x*)",
        "config": {"workload": f"BiCGStab FP32, one system on the {nx}x{ny}x{nz} mesh",
                   "cells": n, "jacobi": True, "schedule": sched, "passes_per_iteration": PASSES[sched],
                   "bytes_per_cell_iteration": sum(bytes32.values()),
                   "timed": "one solve call of `steps` iterations (prologue and epilogue included), "
                            "iterations replayed from captured hipGraphs"},
        "gflops": round(44 * n * ips / 1e9, 1),
        "hbm_frac_per_iteration": round(iter_bytes * ips / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_frac_per_iteration_at_survey_bytes": round(survey_iter_bytes * ips / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_frac_kernels_only": round(iter_bytes / (kernel_ms_iter * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        # the same timed call with the bytes of its one-time passes counted too
        "hbm_frac_whole_call_with_setup_bytes": round((iter_bytes * args.steps
                                                       + sum(SETUP_BYTES_FP32.values()) * n)
                                                      / dt / 1e9 / HBM_PEAK_GBS, 4),
        "profiled_iter_per_s": round(args.steps / pdt, 3),
        "repeats": {"calls": len(rep_ips), "median_iter_per_s": round(rep_ips[len(rep_ips) // 2], 3) if rep_ips else None,
                    "min_max_iter_per_s": [round(rep_ips[0], 3), round(rep_ips[-1], 3)] if rep_ips else None},
        "passes": passes,
        "roofline": roofline,
    }

    # ---- s7_stencil_apply alone on the same mesh: u = A v with the caller's seven
    # FP32 coefficient arrays, 36 B per cell (7 coefficients and v read, u written)
    if not args.no_apply:
        print("[bench] stencil apply: 20 timed launches", file=sys.stderr, flush=True)
        v = xs.to(torch.float32)
        u = torch.empty_like(v)
        stream = torch.cuda.current_stream()
        for _ in range(3):
            s7.stencil_apply(dims, coef, v, u, stream=stream.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20):
            s7.stencil_apply(dims, coef, v, u, stream=stream.cuda_stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        out["stencil_apply"] = {"workload": f"u = A v, FP32, {nx}x{ny}x{nz}, the caller's 7 coefficient arrays",
                                "avg_launch_ms": round(ms, 4), "bytes_per_cell": 36,
                                "GB/s": round(36 * n / (ms * 1e-3) / 1e9, 1),
                                "frac": round(36 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                "form": "x-adjacent pairs, v staged in LDS (2048-cell tiles, band per XCD)"
                                if nx % 2 == 0 and n >= (1 << 18) else "single cells",
                                "timing": "HIP events around 20 launches on the caller's stream"}
        del v, u

    # ---- one GPU's share of an 8-GPU z-slab decomposition of the same mesh:
    # the first nz/8 planes, a contiguous prefix of every array
    if not args.no_shard and nz >= 8:
        dims8 = (nx, ny, nz // 8)
        n8 = nx * ny * (nz // 8)
        print(f"[bench] z-slab share {dims8}: FP32 timed {args.steps} iterations", file=sys.stderr, flush=True)
        c8, b8, x8 = [c[:n8] for c in coef], b[:n8], x[:n8]
        o8 = s7.default_options(profile=1, schedule=args.schedule,
                                tune=0 if args.no_tune else 1)
        s7.bicgstab_solve(dims8, c8, b8, x8, 1e-300, args.warmup, ws=ws, opt=o8)
        x8.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i8 = s7.bicgstab_solve(dims8, c8, b8, x8, 1e-300, args.steps, ws=ws, opt=o8)
        torch.cuda.synchronize()
        dt8 = time.perf_counter() - t0
        by8 = BYTES[("f32", PASSES[i8.schedule])]
        pm8 = {k: i8.pass_ms[SLOT[k]] / max(i8.pass_count[SLOT[k]], 1) for k in by8}
        out["z_slab_share_of_8"] = {
            "workload": f"FP32 on {dims8[0]}x{dims8[1]}x{dims8[2]}, one GPU's z-slab of the "
                        f"{nx}x{ny}x{nz} mesh split over 8 GPUs (halo exchange and all-reduce not included)",
            "iter_per_s": round(i8.iters / dt8, 2), "schedule": i8.schedule,
            "hbm_frac_per_iteration": round(sum(by8.values()) * n8 * i8.iters / dt8 / 1e9 / HBM_PEAK_GBS, 4),
            "passes_GB/s": {k: round(by8[k] * n8 / (ms * 1e-3) / 1e9, 1) for k, ms in pm8.items()}}

    # ---- mixed: BF16 storage, FP32 arithmetic, inside FP64 refinement
    if not args.no_mixed:
        print(f"[bench] BF16+IR timed {args.steps} inner iterations", file=sys.stderr, flush=True)
        run(s7.BF16_IR, args.warmup)
        info16, dt16 = run(s7.BF16_IR, args.steps, profile=1)
        it16 = info16.iters
        bytes16 = BYTES[("16", PASSES[info16.schedule])]
        p16 = {k: info16.pass_ms[SLOT[k]] / max(info16.pass_count[SLOT[k]], 1) for k in bytes16}
        out["mixed_bf16_ir"] = {
            "iter_per_s": round(it16 / dt16, 3), "inner_iters": it16, "schedule": info16.schedule,
            "outer_steps": info16.outer_iters,
            "passes_GB/s": {k: round(bytes16[k] * n / (p16[k] * 1e-3) / 1e9, 1) for k in p16},
            "kernel_bytes_per_iter": sum(bytes16.values()) * n,
        }

    # ---- accuracy: converged runs against the manufactured solution x*
    if not args.no_accuracy:
        print("[bench] converged runs", file=sys.stderr, flush=True)
        acc = {}
        for name, prec, rtol in (("fp32_rtol1e-9", s7.FP32, 1e-9),
                                 ("bf16_ir_rtol1e-10", s7.BF16_IR, 1e-10)):
            if prec != s7.FP32 and args.no_mixed:
                continue
            inf, t = run(prec, 2000, rtol=rtol)
            err = float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))
            acc[name] = {"status": inf.status, "iters": inf.iters, "outer": inf.outer_iters,
                         "rel_res_true": inf.rel_res_true, "rel_err_vs_xstar": err,
                         "seconds": round(t, 3)}
        out["accuracy"] = acc

    del ws, coef, xs, b, x
    torch.cuda.empty_cache()
    if not args.no_cube256:
        print("[bench] 256^3 z-slab: 200 timed iterations and converged runs", file=sys.stderr, flush=True)
        out["cube256_zslab"] = cube256_leg(s7, torch, dev, 200, args.warmup, not args.no_tune)
    if not args.no_batched:
        print("[bench] batched: 64 uneven systems", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(s7, torch, dev)
        print("[bench] batched: 256 systems of 16^3", file=sys.stderr, flush=True)
        out["batched_small"] = batched_small_leg(s7, torch, dev)
        torch.cuda.empty_cache()
    if not args.no_pipelined:
        print("[bench] pipelined BiCGStab", file=sys.stderr, flush=True)
        out["pipelined"] = pipelined_leg(s7, torch, dev, args.steps)
        print("[bench] pipelined BiCGStab, batched", file=sys.stderr, flush=True)
        out["pipelined_batched"] = pipelined_batched_leg(s7, torch, dev)
    if not args.no_simple:
        print("[bench] SIMPLE pattern", file=sys.stderr, flush=True)
        out["simple_pattern"] = [simple_leg(s7, torch, dev, args.simple_dims, args.simple_outer),
                                 simple_leg(s7, torch, dev, (40, 40, 40), 4 * args.simple_outer)]
        torch.cuda.empty_cache()
    if not args.no_2d9:
        print("[bench] 2D 9-point", file=sys.stderr, flush=True)
        out["stencil9_2d"] = stencil9_leg(s7, torch, dev, args.steps, args.warmup)
        if not args.no_batched:
            print("[bench] batched 2D 9-point: 64 uneven meshes", file=sys.stderr, flush=True)
            out["batched_2d9"] = batched_2d9_leg(s7, torch, dev)
            torch.cuda.empty_cache()
    if not args.no_serve:
        out["served"] = served_leg(s7, torch, dev, args.serve_requests, args.serve_rate,
                                   args.serve_burst, args.arena_gb, args.serve_sample)
        torch.cuda.empty_cache()
        if not args.no_2d9 and args.serve_2d9_burst > 0:
            out["served_2d9"] = served_2d9_leg(s7, torch, dev, args.serve_2d9_burst, 16.0)
        if not args.no_2d9 and args.serve_mixed > 0:
            out["served_mixed"] = served_mixed_leg(s7, torch, dev, args.serve_mixed, args.serve_rate)
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(nx, ny, nz, min(args.cpu_slab, nz), args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
