"""GPU parity of the pipelined BiCGStab in the persistent batched kernel
(s7_bicgstab_solve_batched_pipelined) against the oracle's pipelined variant, which is
itself pinned to SciPy's BiCGStab and the classical oracle.

Each iteration is two phases of the persistent kernel.  z and v are formed at the
stencil's neighbour cells in one, w and t in the other.  The residual is replaced
every 10 iterations and at once after a candidate stop, and every stop is verified on
the FP64 true residual.  So the solves run to 1e-8 and meet the 1e-6 bar against the
oracle's solution, as the multi-kernel pipelined path does.  The first iterates (k =
1, 2, 5: before any replacement) track the oracle's to 1e-4, the bar of the
multi-kernel path.  A system's result depends only on the system: not on the rest of
the batch, nor on the work-item size."""
import numpy as np
import pytest

import oracle
from tests.conftest import gpu_available
from tests.gpu_helpers import coef_dev, dev, host, problem, rel_err

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (3, 1, 2), (9, 7, 5), (33, 17, 9), (64, 48, 20), (17, 5, 9), (24, 32, 48), (1030, 6, 4),
          (80, 64, 64)]


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def run(s7, shapes, probs, rtol, max_iter=2000, x0=None, bs=None, coefs=None, **opt):
    import torch
    coefs = coefs if coefs is not None else [coef_dev(p) for p, A, b in probs]
    bs = bs if bs is not None else [dev(b) for p, A, b in probs]
    xs = [dev(np.zeros(int(np.prod(d))) if x0 is None else x0[k]) for k, d in enumerate(shapes)]
    rtols = rtol if isinstance(rtol, list) else [rtol] * len(shapes)
    mis = max_iter if isinstance(max_iter, list) else [max_iter] * len(shapes)
    print("pipelined batch", shapes, opt, flush=True)
    rc, infos = s7.bicgstab_solve_batched_pipelined(shapes, coefs, bs, xs, rtols, mis,
                                                    opt=s7.default_options(**opt))
    torch.cuda.synchronize()
    return rc, infos, [host(x) for x in xs]


@pytest.mark.parametrize("jacobi", [1, 0])
def test_batch_matches_oracle(s7, jacobi):
    probs = [problem(d, seed=50 + k) for k, d in enumerate(SHAPES)]
    rc, infos, xs = run(s7, SHAPES, probs, rtol=1e-8, jacobi=jacobi)
    assert rc == s7.OK, [i.as_dict() for i in infos]
    for (p, A, b), info, x, d in zip(probs, infos, xs, SHAPES):
        ref = oracle.bicgstab_pipelined(A, b, tol=1e-12, max_iter=2000, jacobi_scaling=bool(jacobi))
        assert ref.status == oracle.OK
        assert info.status == s7.OK and info.schedule == 4, d
        # a verified stop: the true residual of the iterated system is at most 1e-8
        # (the unscaled one reported here differs by the spread of the diagonal)
        assert info.rel_res_true <= 3e-8, (d, info.as_dict())
        assert rel_err(x, ref.x) <= 1e-6, d
        assert abs(info.rel_res_true - oracle.true_rel_residual(A, b, x)) <= 1e-3 * info.rel_res_true + 1e-15
        if A.n >= 300:
            r8 = oracle.bicgstab_pipelined(A, b, tol=1e-8, max_iter=2000, jacobi_scaling=bool(jacobi))
            assert abs(info.iters - r8.iters) <= max(5, 0.3 * r8.iters), (d, info.iters, r8.iters)


@pytest.mark.parametrize("dims", [(33, 17, 9), (34, 17, 9)])
def test_iterates_track_oracle(s7, dims):
    """Three copies of one system with caps of 1, 2 and 5 iterations, in one batch: an
    odd nx (single cells) and an even one (the LDS-staged phases on cell pairs)."""
    prob, A, b = problem(dims, seed=4)
    ks = [1, 2, 5]
    rc, infos, xs = run(s7, [dims] * 3, [(prob, A, b)] * 3, rtol=1e-300, max_iter=ks)
    for k, info, x in zip(ks, infos, xs):
        ref = oracle.bicgstab_pipelined(A, b, tol=1e-300, max_iter=k)
        assert info.status == s7.NOT_CONVERGED and info.iters == k
        assert rel_err(x, ref.x) <= 1e-4, k
        assert abs(info.rel_res_rec - ref.res_rec) <= 1e-3 * ref.res_rec


@pytest.mark.parametrize("chunk", [1024, 4096, 16384])
def test_alone_equals_in_mix_bitwise(s7, chunk):
    """Every system's iterates are the same bits alone and in a batch, at any work-item
    size, and under the default load-sized chunks: staged pairs (even nx up to 1024),
    single cells (odd nx, and even nx above 1024)."""
    shapes = [(24, 32, 48), (17, 5, 9), (96, 48, 24), (2, 1, 1), (64, 48, 20), (1030, 6, 4)]
    probs = [problem(d, seed=70 + k) for k, d in enumerate(shapes)]
    rc, infos, xs = run(s7, shapes, probs, rtol=1e-8, chunk_cells=chunk)
    rc0, infos0, xs0 = run(s7, shapes, probs, rtol=1e-8)
    for k in range(len(shapes)):
        assert np.array_equal(xs[k], xs0[k]) and infos[k].iters == infos0[k].iters, k
    for k in (0, 2, 4, 5):
        rc1, inf1, x1 = run(s7, [shapes[k]], [probs[k]], rtol=1e-8, chunk_cells=chunk)
        assert np.array_equal(x1[0], xs[k]), k
        assert inf1[0].iters == infos[k].iters


def test_degenerate_cases(s7):
    """b = 0 (x = 0, no iteration), max_iter = 0 (x0 back), a diagonal A (the half-step
    exit of iteration 0), in one batch with an ordinary system; then the exact
    breakdown of Algorithm 1 without scaling."""
    dims = (9, 7, 5)
    prob, A, b = problem(dims, seed=2)
    n = 24
    d = (1.0 + np.arange(n) % 5).astype(np.float32)
    cd = [d] + [np.zeros(n, np.float32) for _ in range(6)]
    bd = np.linspace(-1.0, 1.0, n)
    shapes = [dims, dims, (4, 3, 2), dims]
    coefs = [coef_dev(prob), coef_dev(prob), [dev(c) for c in cd], coef_dev(prob)]
    bs = [dev(np.zeros(A.n)), dev(b), dev(bd), dev(b)]
    x0 = [np.ones(A.n), np.full(A.n, 0.5), np.zeros(n), np.zeros(A.n)]
    rc, infos, xs = run(s7, shapes, None, rtol=[1e-6, 1e-6, 1e-6, 1e-8], max_iter=[1000, 0, 1000, 1000], x0=x0, bs=bs,
                        coefs=coefs)
    assert infos[0].status == s7.OK and infos[0].iters == 0 and np.all(xs[0] == 0)
    assert infos[1].status == s7.NOT_CONVERGED and infos[1].iters == 0 and np.all(xs[1] == 0.5)
    assert infos[2].status == s7.OK and infos[2].iters == 1
    assert rel_err(xs[2], bd / d.astype(np.float64)) <= 1e-6
    ref = oracle.bicgstab_pipelined(A, b, tol=1e-12, max_iter=2000)
    assert infos[3].status == s7.OK and rel_err(xs[3], ref.x) <= 1e-6
    assert rc == s7.NOT_CONVERGED
    # A = [[0, 1], [-1, 0]], b = (1, 0): (r0, A r0) = 0
    cb = [np.zeros(2, np.float32) for _ in range(7)]
    cb[2][0] = 1.0
    cb[1][1] = -1.0
    rc, infos, xs = run(s7, [(2, 1, 1)], None, rtol=1e-8, coefs=[[dev(c) for c in cb]],
                        bs=[dev(np.array([1.0, 0.0]))], jacobi=0)
    assert infos[0].status == s7.BREAKDOWN and infos[0].reason == s7.REASON_RS_ZERO


def test_split_system_runs_alone_on_the_multi_kernel_path(s7):
    """A system of split_cells cells or more is solved by s7_bicgstab_solve_pipelined in
    its slice: the same bits as that call; the others still match the oracle."""
    import torch
    shapes = [(40, 24, 20), (9, 7, 5)]
    probs = [problem(d, seed=90 + k) for k, d in enumerate(shapes)]
    rc, infos, xs = run(s7, shapes, probs, rtol=1e-8, split_cells=4096)
    p, A, b = probs[0]
    x1 = dev(np.zeros(A.n))
    i1 = s7.bicgstab_solve_pipelined(shapes[0], coef_dev(p), dev(b), x1, 1e-8, 2000)
    torch.cuda.synchronize()
    assert np.array_equal(host(x1), xs[0]) and i1.iters == infos[0].iters
    p, A, b = probs[1]
    ref = oracle.bicgstab_pipelined(A, b, tol=1e-12, max_iter=2000)
    assert infos[1].status == s7.OK and rel_err(xs[1], ref.x) <= 1e-6


def test_invalid_arguments(s7):
    import torch
    dims = (9, 7, 5)
    prob, A, b = problem(dims, seed=2)
    x = dev(np.zeros(A.n))
    with pytest.raises(s7.S7Error):
        s7.bicgstab_solve_batched_pipelined([(0, 5, 5)], [coef_dev(prob)], [dev(b)], [x], [1e-8], [10])
    with pytest.raises(s7.S7Error):
        s7.bicgstab_solve_batched_pipelined([dims], [coef_dev(prob)], [dev(b)], [x], [0.0], [10])
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(s7.S7Error):
        s7.bicgstab_solve_batched_pipelined([dims], [coef_dev(prob)], [dev(b)], [x], [1e-8], [10], ws=ws)
