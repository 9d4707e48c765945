"""Benchmark: BiCGStab iterations/s and HBM roofline on the paper's 600x595x1536 mesh.

One step is one BiCGStab iteration of the whole hot path (P1, P2, P3 with their
scalar steps) over the 548,352,000-cell system, with every input resident in HBM
before the timed region starts.  The timed region is one call of the solver with a
fixed iteration count.  That call includes its prologue and epilogue: coefficient
scaling, r0 = b - A x0, x update and the FP64 true residual.

Printed: one JSON line with the metric, roofline of the dominant kernel (P1), the
mixed BF16+refinement form, accuracy of converged runs against the manufactured
solution, and the FP64 CPU oracle timed on a bounded slab of the same workload.
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
# Algorithmic bytes per cell of each pass (FP32 storage, Jacobi-scaled: 6 coefficient arrays).
# P1 reads p, r0 and 6 coefficients and writes s.
# P2a reads r, s and writes q.
# P2b reads q, r0 and 6 coefficients and writes y.
# P3 reads d, p, q, s, y, r0 and writes d, r, p.
BYTES_FP32 = {"p1": 36, "p2a": 12, "p2b": 36, "p3": 36}
BYTES_16 = {"p1": 18, "p2a": 6, "p2b": 18, "p3": 22}  # BF16/FP16 vectors and coefficients, FP32 d
SRC_FILES = ["paper_2010_03660_amd/csrc/s7_device.hpp", "paper_2010_03660_amd/csrc/s7_single.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in SRC_FILES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_cells: int, kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if still current."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_paper600x595x1536_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash() or t.get("cells") != n_cells:
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(nx: int, ny: int, nz_full: int, slab: int, iters: int):
    """The FP64 oracle (single-threaded C) on a slab of `slab` z-planes of the same
    workload; the time per iteration is scaled to the full mesh by cell count."""
    import numpy as np

    import oracle
    import synth
    oracle.build(force=False)
    prob = synth.make_problem(nx, ny, slab, seed=0)
    A = oracle.build_csr(nx, ny, slab, prob.coef)
    b = oracle.spmv(A, prob.xstar)
    t0 = time.perf_counter()
    res = oracle.bicgstab(A, b, tol=1e-300, max_iter=iters)
    t = time.perf_counter() - t0
    assert res.iters == iters
    per_iter_full = t / iters * (nz_full / slab)
    return {"value": 1.0 / per_iter_full, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} iterations on a {nx}x{ny}x{slab} slab of the same recipe "
                      f"({t:.1f} s), scaled by cell count to {nx}x{ny}x{nz_full}"}


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
    ap.add_argument("--cpu-iters", type=int, default=8)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 2 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this solver has no multi-GPU path (z-slab sharding is "
              "a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2010_03660_amd as s7
    s7.lib()
    dev = torch.device("cuda:0")

    if args.copy_probe:
        src = torch.ones(1 << 29, dtype=torch.float32, device=dev)  # 2 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 4, "launches": 3}))
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
        o = s7.default_options(profile=profile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s7.bicgstab_solve(dims, coef, b, x, rtol, iters, prec=prec, ws=ws, opt=o)
        torch.cuda.synchronize()
        return info, time.perf_counter() - t0

    # ---- plain FP32: warmup, then exactly `steps` timed iterations
    print(f"[bench] FP32 warmup {args.warmup} iterations", file=sys.stderr, flush=True)
    run(s7.FP32, args.warmup)
    print(f"[bench] FP32 timed {args.steps} iterations", file=sys.stderr, flush=True)
    info, dt = run(s7.FP32, args.steps, profile=1)
    assert info.iters == args.steps, info.as_dict()
    ips = args.steps / dt
    names = ("p1", "p2a", "p2b", "p3")
    kname = {"p1": "k_p1 (P1: s = A p, (r0,s))",
             "p2a": "k_p2a (P2a: q = r - alpha s)",
             "p2b": "k_p2 (P2b: y = A q and five dot products)",
             "p3": "k_p3 (P3: x, r, p updates, (r0,r), (r,r))"}
    pass_ms = {k: info.pass_ms[i] / max(info.pass_count[i], 1) for i, k in enumerate(names)}
    dom = max(names, key=lambda k: pass_ms[k])  # the kernel with the largest share of an iteration
    dom_gbs = BYTES_FP32[dom] * n / (pass_ms[dom] * 1e-3) / 1e9
    iter_bytes = sum(BYTES_FP32.values()) * n
    kernel_ms_iter = sum(pass_ms.values())
    traffic = traffic_from_profile(n, dom)
    roofline = {"bound": "hbm", "kernel": kname[dom],
                "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": BYTES_FP32[dom] * n,
                "avg_launch_ms": round(pass_ms[dom], 4)}
    passes = {k: {"avg_ms": round(ms, 4), "GB/s": round(BYTES_FP32[k] * n / (ms * 1e-3) / 1e9, 1)}
              for k, ms in pass_ms.items()}
    out = {
        "metric": "BiCGStab iter/s + %HBM peak at 600x595x1536; served solves/s, p99 latency",
        "value": round(ips, 3), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded 7-point variable-coefficient recipe, b = A x*)",
        "config": {"workload": f"BiCGStab FP32, one system on the {nx}x{ny}x{nz} mesh",
                   "cells": n, "jacobi": True, "timed": "one solve call of `steps` iterations"},
        "gflops": round(44 * n * ips / 1e9, 1),
        "hbm_frac_per_iteration": round(iter_bytes * ips / 1e9 / HBM_PEAK_GBS, 4),
        "hbm_frac_kernels_only": round(iter_bytes / (kernel_ms_iter * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "passes": passes,
        "roofline": roofline,
    }

    # ---- mixed: BF16 storage, FP32 arithmetic, inside FP64 refinement
    if not args.no_mixed:
        print(f"[bench] BF16+IR timed {args.steps} inner iterations", file=sys.stderr, flush=True)
        run(s7.BF16_IR, args.warmup)
        info16, dt16 = run(s7.BF16_IR, args.steps, profile=1)
        it16 = info16.iters
        p16 = {k: info16.pass_ms[i] / max(info16.pass_count[i], 1)
               for i, k in enumerate(("p1", "p2a", "p2b", "p3"))}
        out["mixed_bf16_ir"] = {
            "iter_per_s": round(it16 / dt16, 3), "inner_iters": it16,
            "outer_steps": info16.outer_iters,
            "passes_GB/s": {k: round(BYTES_16[k] * n / (p16[k] * 1e-3) / 1e9, 1) for k in p16},
            "kernel_bytes_per_iter": sum(BYTES_16.values()) * n,
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
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(nx, ny, nz, min(args.cpu_slab, nz), args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
