"""Host-side logic that needs no GPU: the workload generators' statistics, the
benchmark's contract checks and its traffic bookkeeping."""
import json
import math
import os
import subprocess
import sys

import numpy as np

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_serve_stream_statistics():
    """Poisson arrivals at 200/s, sides log-uniform in [16, 256], half FP32 at 1e-6 and
    half BF16+refinement at 1e-10, seeds 10^6 + id."""
    reqs = synth.serve_stream(10000, rate=200.0, seed=0)
    t = np.array([r.arrival_s for r in reqs])
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 1 / 200) < 0.05 / 200  # mean gap within 5 %
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05  # exponential: std = mean
    sides = np.array([r.dims for r in reqs])
    assert sides.min() >= 16 and sides.max() <= 256
    logs = np.log(sides.astype(float))
    # log-uniform: the mean of log(side) sits midway between log 16 and log 256
    assert abs(logs.mean() - 0.5 * (math.log(16) + math.log(256))) < 0.02
    modes = [r.mode for r in reqs]
    assert abs(modes.count("fp32") / len(modes) - 0.5) < 0.02
    assert all(r.rtol == (1e-6 if r.mode == "fp32" else 1e-10) for r in reqs)
    assert [r.seed for r in reqs[:3]] == [1_000_000, 1_000_001, 1_000_002]
    assert [r.rid for r in reqs] == list(range(10000))
    assert synth.serve_stream(50, seed=0)[7].dims == reqs[7].dims  # a prefix of the same stream


def test_batch_shapes():
    shapes, seeds = synth.batch_shapes(64, seed=0)
    assert len(shapes) == 64 and seeds == [1000 + s for s in range(64)]
    flat = [v for d in shapes for v in d]
    assert set(flat) <= {24, 32, 48, 64, 96, 128}
    assert len(set(flat)) == 6  # every side value occurs
    assert synth.batch_shapes(64, seed=0) == (shapes, seeds)


def test_bench_refuses_several_gpus():
    """One GPU only: --gpus 2 exits with status 2 and says why, before touching a GPU."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_traffic_is_reported_only_for_current_kernels(tmp_path, monkeypatch):
    """bench.py reads the committed counter summary only for the form the run used
    (schedule, staged tile, XCD tile order), on the same mesh and kernel sources."""
    sys.path.insert(0, ROOT)
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash covers the kernel sources under ROOT: give the temporary root the real ones
    for f in bench.SRC_FILES:
        os.makedirs(os.path.dirname(tmp_path / f), exist_ok=True)
        (tmp_path / f).write_bytes(open(os.path.join(ROOT, f), "rb").read())
    n = 548352000
    rec = {"cells": n, "source_hash": bench.kernel_source_hash(),
           "forms": [{"schedule": 3, "bytes_per_launch": 123.0},
                     {"schedule": 5, "lds_tile": 2048, "xcd_run": -1, "bytes_per_launch": 456.0}]}
    (prof / "p2_paper600x595x1536_traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile(n, "p2", 3) == 123.0
    assert bench.traffic_from_profile(n, "p2", 5, 2048, -1) == 456.0
    assert bench.traffic_from_profile(n, "p2", 5, 2048, 1) is None  # another tile order
    assert bench.traffic_from_profile(n, "p2", 5, 4096, -1) is None  # another tile
    assert bench.traffic_from_profile(n, "p2", 1) is None  # another schedule
    assert bench.traffic_from_profile(n // 2, "p2", 3) is None  # another mesh
    assert bench.traffic_from_profile(n, "p1", 3) is None  # no summary
    (tmp_path / bench.SRC_FILES[0]).write_text("// changed\n")
    assert bench.traffic_from_profile(n, "p2", 3) is None  # kernels changed since


def test_bench_byte_accounting_matches_the_design():
    """Bytes per cell and iteration of each schedule (Jacobi: 6 coefficient arrays)."""
    sys.path.insert(0, ROOT)
    import bench
    assert sum(bench.BYTES[("f32", 3)].values()) == 112
    assert sum(bench.BYTES[("f32", 4)].values()) == 120
    # the one-time passes of an FP32 solve: copies 52, r0 60, x update 20, true residual 44
    assert sum(bench.SETUP_BYTES_FP32.values()) == 176
    assert sum(bench.BYTES[("16", 3)].values()) == 60
    assert sum(bench.BYTES[("16", 4)].values()) == 64
    # P1: p, r0 and 6 coefficients read, s written, 4 bytes each
    assert bench.BYTES[("f32", 3)]["p1"] == (1 + 1 + 6) * 4 + 4
    assert set(bench.KERNEL) == set(bench.PASSES) == {1, 2, 3, 5}
    # the survey's split of the same Jacobi FP32 iteration (p formed in P1 there): 116 B
    assert sum(bench.SURVEY_BYTES.values()) == 116


def test_bench_byte_accounting_2d9():
    """2D 9-point, Jacobi (8 coefficient arrays): 128 B per cell and iteration in FP32,
    68 B with 16-bit storage (the FP32 correction d stays 4 bytes)."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.BYTES_2D9 == {"p1": 44, "p2": 48, "p3": 36}
    assert sum(bench.BYTES_2D9.values()) == 128
    assert bench.BYTES_2D9_16 == {"p1": 22, "p2": 24, "p3": 22}
    assert sum(bench.BYTES_2D9_16.values()) == 68


def test_batch_shapes_2d9():
    shapes, seeds = synth.batch_shapes_2d9(64, seed=0)
    assert len(shapes) == 64 and seeds == [2000 + s for s in range(64)]
    flat = [v for d in shapes for v in d]
    assert set(flat) == set(synth.BATCH_SIDES_2D9)  # every side value occurs
    assert all(len(d) == 2 for d in shapes)
    assert max(nx * ny for nx, ny in shapes) < 2 ** 21  # every mesh stays in the shared launch
    assert synth.batch_shapes_2d9(64, seed=0) == (shapes, seeds)


def test_serve_stream_2d9_statistics():
    """2D requests: sides log-uniform in [64, 1024] per axis, half FP32 at 1e-6 and half
    BF16+refinement at 1e-10, seeds 3 * 10^6 + id, a stream of its own."""
    reqs = synth.serve_stream_2d9(4000, seed=0)
    sides = np.array([r.dims for r in reqs])
    assert sides.shape == (4000, 2) and sides.min() >= 64 and sides.max() <= 1024
    logs = np.log(sides.astype(float))
    assert abs(logs.mean() - 0.5 * (math.log(64) + math.log(1024))) < 0.03
    modes = [r.mode for r in reqs]
    assert abs(modes.count("fp32") / len(modes) - 0.5) < 0.03
    assert all(r.rtol == (1e-6 if r.mode == "fp32" else 1e-10) for r in reqs)
    assert [r.seed for r in reqs[:2]] == [3_000_000, 3_000_001]
    assert synth.serve_stream_2d9(10, seed=0)[3].dims == reqs[3].dims
