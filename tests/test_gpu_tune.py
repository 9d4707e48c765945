"""GPU tests of the autotuner (options.tune = 1).

Tuning times short trials on synthetic contents of the caller's workspace, so the
caller's arrays must come out exactly as an untuned solve with the chosen parameters
would leave them, and the result must match the FP64 oracle.  Choices are cached per
size class and appended to the file named by S7_TUNE_CACHE."""
import os

import numpy as np
import pytest

import oracle
from tests.conftest import gpu_available
from tests.gpu_helpers import coef_dev, dev, host, problem, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s7(tmp_path_factory):
    if not gpu_available():
        pytest.skip("no GPU")
    path = tmp_path_factory.mktemp("tune") / "s7tune.txt"
    os.environ["S7_TUNE_CACHE"] = str(path)  # read at the first tuned call of the process
    import paper_2010_03660_amd as s7
    s7.lib()
    yield s7, path
    os.environ.pop("S7_TUNE_CACHE", None)


def solve(s7, dims, coef, b, x0, **opt):
    import torch
    x = dev(x0.copy())
    info = s7.bicgstab_solve(dims, coef, dev(b), x, opt.pop("rtol", 1e-8), 2000,
                             prec=opt.pop("prec", 0), opt=s7.default_options(**opt))
    torch.cuda.synchronize()
    return host(x), info


def test_trials_leave_caller_arrays_untouched(s7):
    """Trials of untuned classes run on synthetic workspace contents: with max_iter = 0
    the caller's x must come back exactly as x0 (single and batched forms)."""
    import torch
    s7, path = s7
    dims = (128, 128, 64)  # a size class no other test tunes
    prob, A, b = problem(dims, seed=51)
    x = torch.full((A.n,), 0.25, dtype=torch.float64, device="cuda")
    info = s7.bicgstab_solve(dims, coef_dev(prob), dev(b), x, 1e-8, 0, opt=s7.default_options(tune=1))
    torch.cuda.synchronize()
    assert info.status == s7.NOT_CONVERGED and info.iters == 0
    assert bool((x == 0.25).all())
    shapes = [(50, 50, 50), (20, 20, 20), (10, 10, 10)]
    probs = [problem(d, seed=52 + i) for i, d in enumerate(shapes)]
    xs = [torch.full((A.n,), 0.25, dtype=torch.float64, device="cuda") for p, A, b in probs]
    rc, infos = s7.bicgstab_solve_batched(shapes, [coef_dev(p) for p, A, b in probs],
                                          [dev(b) for p, A, b in probs], xs, [1e-8] * 3, [0] * 3,
                                          opt=s7.default_options(tune=1))
    torch.cuda.synchronize()
    assert rc == s7.NOT_CONVERGED and all(i.iters == 0 for i in infos)
    assert all(bool((x == 0.25).all()) for x in xs)
    text = path.read_text()
    assert "s7tune2 1 " in text and "s7tune2 2 " in text


@pytest.mark.parametrize("prec", [0, 1])
def test_tuned_single_solve(s7, prec):
    s7, path = s7
    dims = (70, 40, 20)
    prob, A, b = problem(dims, seed=31)
    coef = coef_dev(prob)
    x0 = np.linspace(-0.5, 0.5, A.n)
    rtol = 1e-8 if prec == 0 else 1e-10
    x1, i1 = solve(s7, dims, coef, b, x0, tune=1, prec=prec, rtol=rtol)  # trials, then the solve
    x2, i2 = solve(s7, dims, coef, b, x0, tune=1, prec=prec, rtol=rtol)  # cached choice
    assert np.array_equal(x1, x2) and i1.iters == i2.iters
    ref = oracle.bicgstab(A, b, x0=x0, tol=1e-13, max_iter=2000)
    assert i1.status == s7.OK and rel_err(x1, ref.x) <= (1e-6 if prec == 0 else 1e-7)
    # the recorded choice (schedule, streaming split, staged tile, XCD tile order), set
    # explicitly, reproduces the tuned solve bit for bit
    line = [l for l in path.read_text().split("\n") if l.startswith(f"s7tune2 1 {prec} ")][-1].split()
    sched, sb, tile, xr = (int(v) for v in line[6:10])
    xe, ie = solve(s7, dims, coef, b, x0, schedule=sched, stream_blocks=sb, lds_tile=tile, xcd_run=xr,
                   prec=prec, rtol=rtol)
    assert np.array_equal(xe, x1) and ie.iters == i1.iters
    assert i1.schedule == sched and (sched != 5 or i1.lds_tile == tile)


def test_tuned_batched_solve(s7):
    import torch
    s7, path = s7
    shapes = [(24, 32, 48), (17, 5, 9), (40, 24, 20), (64, 24, 32), (2, 1, 1)]
    probs = [problem(d, seed=40 + i) for i, d in enumerate(shapes)]
    coefs = [coef_dev(p) for p, A, b in probs]
    bs = [dev(b) for p, A, b in probs]

    def run(**opt):
        xs = [torch.zeros(A.n, dtype=torch.float64, device="cuda") for p, A, b in probs]
        rc, infos = s7.bicgstab_solve_batched(shapes, coefs, bs, xs, [1e-8] * len(shapes),
                                              [2000] * len(shapes), opt=s7.default_options(**opt))
        torch.cuda.synchronize()
        return rc, infos, [host(x) for x in xs]

    rc, infos, xs = run(tune=1)
    assert rc == s7.OK
    for (p, A, b), x in zip(probs, xs):
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(x, ref.x) <= 1e-6
    rc2, infos2, xs2 = run(tune=1)
    assert all(np.array_equal(a, c) for a, c in zip(xs, xs2))
    # the tuned chunk is one of the candidates: an explicit run reproduces the result
    chunk = int([l for l in path.read_text().split("\n") if l.startswith("s7tune2 2 ")][-1].split()[6])
    rc3, infos3, xs3 = run(chunk_cells=chunk)
    assert all(np.array_equal(a, c) for a, c in zip(xs, xs3))


def test_tuning_trials_are_logged(s7, tmp_path):
    """S7_TUNE_LOG receives one line per trial: for a mesh with an even nx the staged
    passes with tiles of 2048, 4096 and 8192 cells in both tile orders, cell pairs, and
    single cells in three and four passes, then the streaming splits of the best."""
    s7, path = s7
    log = tmp_path / "trials.txt"
    os.environ["S7_TUNE_LOG"] = str(log)
    try:
        dims = (96, 64, 48)  # a size class no other test tunes
        prob, A, b = problem(dims, seed=53)
        x, info = solve(s7, dims, coef_dev(prob), b, np.zeros(A.n), tune=1)
    finally:
        os.environ.pop("S7_TUNE_LOG", None)
    assert info.status == s7.OK
    trials = [l for l in log.read_text().split("\n") if l.startswith("single ")]
    forms = {tuple(int(f.split("=")[1]) for f in l.split() if f.split("=")[0] in ("schedule", "lds_tile", "xcd_run"))
             for l in trials}
    assert {(5, t, xr) for t in (2048, 4096, 8192) for xr in (1, -1)} <= forms
    assert {(3, 0, 0), (1, 0, 0), (2, 0, 0)} <= forms
    assert all(float(l.split("ms_per_iteration=")[1]) > 0 for l in trials)
