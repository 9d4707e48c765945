"""GPU parity of the batched persistent solver (s7_bicgstab_solve_batched).

Each system of a batch is checked against the FP64 oracle.  Each system's result
must not depend on the rest of the batch: solved alone through the same path, it
comes out bit for bit the same, because its sums run in a fixed per-system order
(per unit of 1024 cells, each unit summed by one wavefront).  Nor may it depend on
the work-item size (chunk_cells), which the serving loop sizes by load."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import gpu_available
from tests.gpu_helpers import coef_dev, dev, host, problem, rel_err

pytestmark = pytest.mark.gpu

UNEVEN = [(24, 32, 48), (64, 24, 32), (17, 5, 9), (33, 17, 9), (40, 24, 20), (2, 1, 1),
          (96, 48, 24), (31, 29, 27)]


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def make_batch(shapes, seeds):
    probs = [problem(d, seed=s) for d, s in zip(shapes, seeds)]
    return probs


def run_batch(s7, shapes, probs, rtol, max_iter=1000, prec=0, **opt):
    import torch
    coefs = [coef_dev(p) for p, A, b in probs]
    bs = [dev(b) for p, A, b in probs]
    xs = [torch.zeros(A.n, dtype=torch.float64, device="cuda") for p, A, b in probs]
    o = s7.default_options(**opt)
    rc, infos = s7.bicgstab_solve_batched(shapes, coefs, bs, xs, [rtol] * len(shapes),
                                          [max_iter] * len(shapes), prec=prec, opt=o)
    torch.cuda.synchronize()
    return rc, infos, [host(x) for x in xs]


def test_uneven_batch_matches_oracle(s7):
    seeds = [100 + i for i in range(len(UNEVEN))]
    probs = make_batch(UNEVEN, seeds)
    rc, infos, xs = run_batch(s7, UNEVEN, probs, rtol=1e-8)
    assert rc == s7.OK, [i.as_dict() for i in infos]
    for (p, A, b), info, x in zip(probs, infos, xs):
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert info.status == s7.OK
        assert rel_err(x, ref.x) <= 1e-6
        assert abs(info.rel_res_true - oracle.true_rel_residual(A, b, x)) <= 1e-3 * info.rel_res_true + 1e-15
        r8 = oracle.bicgstab(A, b, tol=1e-8, max_iter=2000)
        assert abs(info.iters - r8.iters) <= max(3, 0.2 * r8.iters)


@pytest.mark.parametrize("chunk", [1024, 4096, 16384])
def test_alone_equals_in_mix_bitwise(s7, chunk):
    seeds = [200 + i for i in range(len(UNEVEN))]
    probs = make_batch(UNEVEN, seeds)
    rc, infos, xs = run_batch(s7, UNEVEN, probs, rtol=1e-8, chunk_cells=chunk)
    for k in (0, 3, 6):
        rc1, inf1, x1 = run_batch(s7, [UNEVEN[k]], [probs[k]], rtol=1e-8, chunk_cells=chunk)
        assert np.array_equal(x1[0], xs[k]), k
        assert inf1[0].iters == infos[k].iters


def test_result_does_not_depend_on_chunk_size(s7):
    """Chunks of one unit, of part of a unit group (2048 cells: two of the four
    wavefronts idle), of one group and of several groups, and the default (chunks
    halved by load), give the same iterates bit for bit: staged pairs (even nx up to
    1024), unstaged pairs (nx above 1024), single cells (odd nx), FP32 and BF16+IR."""
    shapes = [(24, 32, 48), (17, 5, 9), (1030, 6, 4), (96, 48, 24), (2, 1, 1)]
    probs = make_batch(shapes, [300 + i for i in range(len(shapes))])
    for prec, rtol in ((0, 1e-8), (1, 1e-10)):
        runs = [run_batch(s7, shapes, probs, rtol=rtol, prec=prec, chunk_cells=c)
                for c in (1024, 2048, 4096, 12288, 0)]
        rc0, inf0, x0 = runs[0]
        assert rc0 == s7.OK, [i.as_dict() for i in inf0]
        for rc, infos, xs in runs[1:]:
            assert rc == rc0
            for k in range(len(shapes)):
                assert np.array_equal(xs[k], x0[k]), (prec, k)
                assert infos[k].iters == inf0[k].iters and infos[k].outer_iters == inf0[k].outer_iters
        for (p, A, b), x in zip(probs, x0):
            ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
            assert rel_err(x, ref.x) <= (1e-6 if prec == 0 else 1e-7)


def test_batched_iterates_track_oracle(s7):
    shapes = [(40, 24, 20), (33, 17, 9)]
    probs = make_batch(shapes, [7, 8])
    for k in (1, 2, 5):
        rc, infos, xs = run_batch(s7, shapes, probs, rtol=1e-300, max_iter=k)
        for (p, A, b), info, x in zip(probs, infos, xs):
            ref = oracle.bicgstab(A, b, tol=1e-300, max_iter=k)
            assert info.status == s7.NOT_CONVERGED and info.iters == k
            assert rel_err(x, ref.x) <= 1e-4
            assert abs(info.rel_res_rec - ref.res_rec) <= 1e-3 * ref.res_rec


def test_batched_edge_systems(s7):
    import torch
    # a zero right-hand side, an exact breakdown and a regular system in one batch
    shapes = [(9, 7, 5), (2, 1, 1), (33, 17, 9)]
    p0, A0, b0 = problem(shapes[0], seed=2)
    coef_bd = [np.zeros(2, np.float32) for _ in range(7)]
    coef_bd[0][:] = 0.0
    coef_bd[2][0] = 1.0
    coef_bd[1][1] = -1.0
    p2, A2, b2 = problem(shapes[2], seed=3)
    coefs = [coef_dev(p0), [dev(c) for c in coef_bd], coef_dev(p2)]
    bs = [dev(np.zeros(A0.n)), dev(np.array([1.0, 0.0])), dev(b2)]
    xs = [torch.ones(A0.n, dtype=torch.float64, device="cuda"),
          torch.zeros(2, dtype=torch.float64, device="cuda"),
          torch.zeros(A2.n, dtype=torch.float64, device="cuda")]
    rc, infos = s7.bicgstab_solve_batched(shapes, coefs, bs, xs, [1e-8] * 3, [100] * 3,
                                          opt=s7.default_options(jacobi=0))
    torch.cuda.synchronize()
    assert infos[0].status == s7.OK and np.all(host(xs[0]) == 0)
    assert infos[1].status == s7.BREAKDOWN and infos[1].reason == s7.REASON_RS_ZERO
    assert infos[2].status == s7.OK
    ref = oracle.bicgstab(A2, b2, tol=1e-12, max_iter=1000, jacobi_scaling=False)
    assert rel_err(host(xs[2]), ref.x) <= 1e-6
    assert rc == s7.BREAKDOWN


@pytest.mark.parametrize("prec", ["bf16_ir", "fp16_ir"])
def test_batched_mixed_precision(s7, prec):
    shapes = [(32, 32, 32), (24, 48, 17), (40, 24, 20)]
    probs = make_batch(shapes, [5, 6, 7])
    rc, infos, xs = run_batch(s7, shapes, probs, rtol=1e-10, max_iter=2000,
                              prec=s7.PREC_NAMES[prec])
    assert rc == s7.OK, [i.as_dict() for i in infos]
    for (p, A, b), info, x in zip(probs, infos, xs):
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert info.rel_res_true <= 1e-10
        assert rel_err(x, ref.x) <= 1e-7
        assert info.outer_iters > 1


def test_batch_workload_64_systems(s7):
    """64 systems, each side uniform over {24,...,128}, per-system seeds, tolerance 1e-7:
    every system checked against the oracle on a sample, all checked for status and
    true residual."""
    import torch
    shapes, seeds = synth.batch_shapes(64, seed=0)
    n_total = sum(int(np.prod(s)) for s in shapes)
    coefs, bs, xs, xstars = [], [], [], []
    for d, sd in zip(shapes, seeds):
        n = int(np.prod(d))
        c = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(7)]
        xsd = torch.empty(n, dtype=torch.float64, device="cuda")
        bd = torch.empty(n, dtype=torch.float64, device="cuda")
        s7.generate_problem(d, sd, 0, c, xsd, bd)
        coefs.append(c)
        bs.append(bd)
        xstars.append(xsd)
        xs.append(torch.zeros(n, dtype=torch.float64, device="cuda"))
    rc, infos = s7.bicgstab_solve_batched(shapes, coefs, bs, xs, [1e-7] * 64, [2000] * 64)
    torch.cuda.synchronize()
    assert rc == s7.OK
    assert n_total > 5_000_000
    for k, (d, sd, info) in enumerate(zip(shapes, seeds, infos)):
        assert info.status == s7.OK
        assert info.rel_res_true <= 1e-6
        err = float(torch.linalg.vector_norm(xs[k] - xstars[k]) / torch.linalg.vector_norm(xstars[k]))
        assert err <= 1e-5
    for k in (0, 17, 63):
        p, A, b = problem(shapes[k], seed=seeds[k])
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(host(xs[k]), ref.x) <= 1e-5


def test_batch_workload_64_systems_vs_oracle(s7):
    """The same 64 systems solved in one batched call at recurrence tolerance 1e-8 (the
    FP32 error floor is near 3e-7, so 1e-7 leaves errors up to about 5e-6), every one
    checked against the FP64 oracle's solution at 1e-6.  The oracle runs the 64 systems
    on host threads (its C calls release the interpreter lock)."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    shapes, seeds = synth.batch_shapes(64, seed=0)
    coefs, bs, xs = [], [], []
    for d, sd in zip(shapes, seeds):
        n = int(np.prod(d))
        c = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(7)]
        bd = torch.empty(n, dtype=torch.float64, device="cuda")
        s7.generate_problem(d, sd, 0, c, torch.empty(n, dtype=torch.float64, device="cuda"), bd)
        coefs.append(c)
        bs.append(bd)
        xs.append(torch.zeros(n, dtype=torch.float64, device="cuda"))
    rc, infos = s7.bicgstab_solve_batched(shapes, coefs, bs, xs, [1e-8] * 64, [2000] * 64)
    torch.cuda.synchronize()
    assert rc == s7.OK
    xh = [host(x) for x in xs]
    del coefs, bs, xs

    def check(k):
        p, A, b = problem(shapes[k], seed=seeds[k])
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        return ref.status, rel_err(xh[k], ref.x)

    with ThreadPoolExecutor(max_workers=8) as ex:
        res = list(ex.map(check, range(64)))
    for k, (status, err) in enumerate(res):
        assert status == oracle.OK and infos[k].status == s7.OK, k
        assert err <= 1e-6, (k, shapes[k], err)


def test_simple_pattern_warm_started(s7):
    """The application pattern of Algorithm 2 (SIMPLE): per outer iteration, the three
    momentum systems u, v, w in one batched call capped at 5 iterations, then the
    continuity system capped at 20, each warm-started from its previous solution.  Three
    outer iterations, each result checked against the oracle running the same capped,
    warm-started solves in FP64."""
    import torch
    dims = (32, 24, 20)
    probs = [problem(dims, seed=900 + f) for f in range(4)]  # u, v, w, p
    coefs = [coef_dev(p) for p, A, b in probs]
    bs = [dev(b) for p, A, b in probs]
    xs = [torch.zeros(A.n, dtype=torch.float64, device="cuda") for p, A, b in probs]
    xo = [np.zeros(A.n) for p, A, b in probs]
    for it in range(3):
        rc, infos = s7.bicgstab_solve_batched([dims] * 3, coefs[:3], bs[:3], xs[:3], [1e-12] * 3, [5] * 3)
        info_p = s7.bicgstab_solve(dims, coefs[3], bs[3], xs[3], 1e-12, 20)
        torch.cuda.synchronize()
        assert all(i.iters == 5 for i in infos) and info_p.iters == 20
        for f, (p, A, b) in enumerate(probs):
            ref = oracle.bicgstab(A, b, x0=xo[f], tol=1e-12, max_iter=5 if f < 3 else 20)
            xo[f] = ref.x
            assert rel_err(host(xs[f]), ref.x) <= 1e-4, (it, f)


def test_large_systems_run_alone(s7):
    """Systems of split_cells cells or more leave the shared launch for the multi-kernel
    path: each comes out bit for bit as from bicgstab_solve, and the systems left in the
    shared launch come out as in a batch that routes nothing."""
    import torch
    shapes = [(24, 32, 48), (40, 24, 20), (17, 5, 9), (48, 40, 24)]  # 36864, 19200, 765, 46080 cells
    probs = make_batch(shapes, [300 + i for i in range(4)])
    rc, infos, xs = run_batch(s7, shapes, probs, rtol=1e-8, split_cells=20000)
    rc0, infos0, xs0 = run_batch(s7, shapes, probs, rtol=1e-8, split_cells=-1)
    assert rc == s7.OK and rc0 == s7.OK
    for k in (1, 2):
        assert np.array_equal(xs[k], xs0[k]) and infos[k].iters == infos0[k].iters
    for k in (0, 3):
        p, A, b = probs[k]
        x1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        info1 = s7.bicgstab_solve(shapes[k], coef_dev(p), dev(b), x1, 1e-8, 1000,
                                  opt=s7.default_options(split_cells=20000))
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), xs[k]) and info1.iters == infos[k].iters
        assert infos[k].schedule == info1.schedule
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(xs[k], ref.x) <= 1e-6
