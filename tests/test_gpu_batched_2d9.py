"""GPU parity of the batched 2D 9-point solve (section IV's operator, section
VIII-B's many compact problems) against the FP64 oracle.

Uneven meshes in one persistent launch (one-cell and one-row meshes, ragged
chunk tails, several chunks per system), with and without Jacobi scaling, in
FP32 and in 16-bit storage inside FP64 refinement; a system's result does not
depend on the rest of the batch; edge systems (b = 0, an exact breakdown) sit
beside regular ones; large meshes leave the shared launch for the multi-kernel
path and come out as from the single-system call."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import gpu_available
from tests.gpu_helpers import dev, host, rel_err

pytestmark = pytest.mark.gpu

# 1, 3, 5, 153, 4257, 1750 and 60000 cells: a 60000-cell mesh spans four
# default chunks (16384 cells) with a ragged last one
UNEVEN9 = [(1, 1), (3, 1), (1, 5), (17, 9), (129, 33), (250, 7), (300, 200)]


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def problems9(shapes, seeds):
    out = []
    for d, s in zip(shapes, seeds):
        p = synth.make_problem_2d9(*d, seed=s)
        A = oracle.build_csr_2d9(*d, p.coef)
        out.append((p, A, oracle.spmv(A, p.xstar)))
    return out


def run9(s7, shapes, probs, rtol, max_iter=1000, prec=0, x0=None, **opt):
    import torch
    coefs = [[dev(c) for c in p.coef] for p, A, b in probs]
    bs = [dev(b) for p, A, b in probs]
    xs = [torch.zeros(A.n, dtype=torch.float64, device="cuda") for p, A, b in probs]
    rc, infos = s7.bicgstab_solve_batched_2d9(shapes, coefs, bs, xs, [rtol] * len(shapes),
                                              [max_iter] * len(shapes), prec=prec,
                                              opt=s7.default_options(**opt))
    torch.cuda.synchronize()
    return rc, infos, [host(x) for x in xs]


@pytest.mark.parametrize("jacobi", [1, 0])
def test_uneven_batch_matches_oracle(s7, jacobi):
    probs = problems9(UNEVEN9, [400 + i for i in range(len(UNEVEN9))])
    rc, infos, xs = run9(s7, UNEVEN9, probs, rtol=1e-8, jacobi=jacobi)
    assert rc == s7.OK, [i.as_dict() for i in infos]
    for (p, A, b), info, x in zip(probs, infos, xs):
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000, jacobi_scaling=bool(jacobi))
        assert info.status == s7.OK and info.schedule == 1
        assert rel_err(x, ref.x) <= 1e-6
        assert abs(info.rel_res_true - oracle.true_rel_residual(A, b, x)) <= 1e-3 * info.rel_res_true + 1e-15
        r8 = oracle.bicgstab(A, b, tol=1e-8, max_iter=2000, jacobi_scaling=bool(jacobi))
        assert abs(info.iters - r8.iters) <= max(3, 0.2 * r8.iters)


@pytest.mark.parametrize("chunk", [1024, 4096])
def test_alone_equals_in_mix_bitwise(s7, chunk):
    probs = problems9(UNEVEN9, [500 + i for i in range(len(UNEVEN9))])
    rc, infos, xs = run9(s7, UNEVEN9, probs, rtol=1e-8, chunk_cells=chunk)
    assert rc == s7.OK
    for k in (0, 4, 6):
        rc1, inf1, x1 = run9(s7, [UNEVEN9[k]], [probs[k]], rtol=1e-8, chunk_cells=chunk)
        assert np.array_equal(x1[0], xs[k]), k
        assert inf1[0].iters == infos[k].iters


def test_result_does_not_depend_on_chunk_size(s7):
    """The 9-point phases keep their sums per unit of 1024 cells too: chunk sizes
    of one unit, two, one unit group, three groups and the load-sized default give
    the same iterates bit for bit (staged rows up to 1024 cells, unstaged above)."""
    shapes = [(129, 33), (300, 200), (1100, 9), (3, 1)]
    probs = problems9(shapes, [520 + i for i in range(len(shapes))])
    for prec, rtol in ((0, 1e-8), (1, 1e-10)):
        runs = [run9(s7, shapes, probs, rtol=rtol, prec=prec, chunk_cells=c) for c in (1024, 2048, 4096, 12288, 0)]
        rc0, inf0, x0 = runs[0]
        assert rc0 == s7.OK, [i.as_dict() for i in inf0]
        for rc, infos, xs in runs[1:]:
            assert rc == rc0
            for k in range(len(shapes)):
                assert np.array_equal(xs[k], x0[k]), (prec, k)
                assert infos[k].iters == inf0[k].iters
        for (p, A, b), x in zip(probs, x0):
            ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
            assert rel_err(x, ref.x) <= (1e-6 if prec == 0 else 1e-7)


def test_batched_iterates_track_oracle(s7):
    shapes = [(129, 33), (300, 200)]
    probs = problems9(shapes, [7, 8])
    for k in (1, 2, 5):
        rc, infos, xs = run9(s7, shapes, probs, rtol=1e-300, max_iter=k)
        for (p, A, b), info, x in zip(probs, infos, xs):
            ref = oracle.bicgstab(A, b, tol=1e-300, max_iter=k)
            assert info.status == s7.NOT_CONVERGED and info.iters == k
            assert rel_err(x, ref.x) <= 1e-4
            assert abs(info.rel_res_rec - ref.res_rec) <= 1e-3 * ref.res_rec


def test_batched_edge_systems(s7):
    """b = 0 (x = 0 exactly), an exact breakdown ((r0, A p) = 0 on the 2 x 1 mesh
    [[0, 1], [-1, 0]]) and a regular system in one batch."""
    import torch
    shapes = [(9, 7), (2, 1), (129, 33)]
    (p0, A0, b0), (p2, A2, b2) = problems9([shapes[0], shapes[2]], [2, 3])
    coef_bd = [np.zeros(2, np.float32) for _ in range(9)]
    coef_bd[2][0] = 1.0   # cell 0, east link
    coef_bd[1][1] = -1.0  # cell 1, west link
    coefs = [[dev(c) for c in p0.coef], [dev(c) for c in coef_bd], [dev(c) for c in p2.coef]]
    bs = [dev(np.zeros(A0.n)), dev(np.array([1.0, 0.0])), dev(b2)]
    xs = [torch.ones(A0.n, dtype=torch.float64, device="cuda"),
          torch.zeros(2, dtype=torch.float64, device="cuda"),
          torch.zeros(A2.n, dtype=torch.float64, device="cuda")]
    rc, infos = s7.bicgstab_solve_batched_2d9(shapes, coefs, bs, xs, [1e-8] * 3, [100] * 3,
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
    shapes = [(64, 48), (129, 33), (300, 200), (1, 5)]
    probs = problems9(shapes, [5, 6, 7, 8])
    rc, infos, xs = run9(s7, shapes, probs, rtol=1e-10, max_iter=2000, prec=s7.PREC_NAMES[prec])
    assert rc == s7.OK, [i.as_dict() for i in infos]
    for (p, A, b), info, x in zip(probs, infos, xs):
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert info.rel_res_true <= 1e-10
        assert abs(info.rel_res_true - oracle.true_rel_residual(A, b, x)) <= 1e-3 * info.rel_res_true + 1e-16
        assert rel_err(x, ref.x) <= 1e-7


def test_large_meshes_run_alone(s7):
    """Meshes of split_cells cells or more leave the shared launch: each comes out bit
    for bit as from bicgstab_solve_2d9, the others as in a batch that routes nothing."""
    import torch
    shapes = [(200, 150), (129, 33), (17, 9), (250, 120)]  # 30000, 4257, 153, 30000 cells
    probs = problems9(shapes, [600 + i for i in range(4)])
    rc, infos, xs = run9(s7, shapes, probs, rtol=1e-8, split_cells=20000)
    rc0, infos0, xs0 = run9(s7, shapes, probs, rtol=1e-8, split_cells=-1)
    assert rc == s7.OK and rc0 == s7.OK
    for k in (1, 2):
        assert np.array_equal(xs[k], xs0[k]) and infos[k].iters == infos0[k].iters
    for k in (0, 3):
        p, A, b = probs[k]
        x1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        info1 = s7.bicgstab_solve_2d9(*shapes[k], [dev(c) for c in p.coef], dev(b), x1, 1e-8, 1000,
                                      opt=s7.default_options(split_cells=20000))
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), xs[k]) and info1.iters == infos[k].iters
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(xs[k], ref.x) <= 1e-6


def test_tuned_batch_matches_oracle(s7):
    """With tune = 1 the chunk size and grid come from timed trials on the workspaces;
    the solves then start from the caller's data and reach the oracle's solution."""
    shapes = [(64, 48), (129, 33), (300, 200)]
    probs = problems9(shapes, [700, 701, 702])
    rc, infos, xs = run9(s7, shapes, probs, rtol=1e-8, tune=1)
    assert rc == s7.OK
    for (p, A, b), info, x in zip(probs, infos, xs):
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(x, ref.x) <= 1e-6


def test_many_small_meshes(s7):
    """128 meshes with sides drawn from {16, 24, 32, 48, 64}, seeded per system: every
    system converges, and a sample of them matches the oracle."""
    rng = np.random.default_rng(9)
    shapes = [tuple(int(v) for v in rng.choice([16, 24, 32, 48, 64], 2)) for _ in range(128)]
    probs = problems9(shapes, [800 + i for i in range(128)])
    rc, infos, xs = run9(s7, shapes, probs, rtol=1e-7)
    assert rc == s7.OK and all(i.status == s7.OK for i in infos)
    for k in (0, 17, 64, 127):
        p, A, b = probs[k]
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(xs[k], ref.x) <= 1e-5


def test_batch_workload_64_meshes(s7):
    """The batched 2D workload the benchmark times: 64 meshes, each side uniform over
    {96,...,512}, seeds 2000 + s, tolerance 1e-7, autotuned.  Every system is checked
    for status, true residual and error against x*; a sample against the oracle."""
    import torch
    shapes, seeds = synth.batch_shapes_2d9(64, seed=0)
    coefs, bs, xs, xstars = [], [], [], []
    for (nx, ny), sd in zip(shapes, seeds):
        n = nx * ny
        c = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(9)]
        xsd = torch.empty(n, dtype=torch.float64, device="cuda")
        bd = torch.empty(n, dtype=torch.float64, device="cuda")
        s7.generate_problem_2d9(nx, ny, sd, c, xsd, bd)
        coefs.append(c)
        bs.append(bd)
        xstars.append(xsd)
        xs.append(torch.zeros(n, dtype=torch.float64, device="cuda"))
    rc, infos = s7.bicgstab_solve_batched_2d9(shapes, coefs, bs, xs, [1e-7] * 64, [2000] * 64,
                                              opt=s7.default_options(tune=1))
    torch.cuda.synchronize()
    assert rc == s7.OK
    for k, info in enumerate(infos):
        assert info.status == s7.OK and info.rel_res_true <= 1e-6, k
        err = float(torch.linalg.vector_norm(xs[k] - xstars[k]) / torch.linalg.vector_norm(xstars[k]))
        assert err <= 1e-5, (k, err)
    big = max(range(64), key=lambda k: shapes[k][0] * shapes[k][1])
    for k in (0, 31, big):
        (p, A, b), = problems9([shapes[k]], [seeds[k]])
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(host(xs[k]), ref.x) <= 1e-5, k
