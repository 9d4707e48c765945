"""GPU checks of the P2 design probe (s7_p2_design_probe): every kernel design of the
three-pass P2 (q = r - alpha s on the fly, y = A q, five sums; Algorithm 1 on the stencil
of section IV) computes the same y bit for bit, that y is A q to FP32 accuracy against
an FP64 evaluation, and the five sums match FP64 dot products.  The meshes include a
partial in-plane tile (a plane of fewer than 2048 cells) and an odd number of planes
(the two-plane design's last tile holds one plane), and z-march depths that do and do
not divide nz."""
import numpy as np
import pytest

import synth
from tests.conftest import gpu_available
from tests.gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

DESIGNS = [(0, 0), (1, 1), (1, 0), (2, 1), (2, 0), (3, 1), (3, 4), (3, 8), (3, 64)]


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def unit_operator(dims, seed):
    """The six off-diagonal coefficients of D^-1 A (FP32, divided in FP32 as the
    solver's working copies are), outward links zeroed on the faces."""
    nx, ny, nz = dims
    prob = synth.make_problem(nx, ny, nz, seed=seed)
    diag = prob.coef[0].astype(np.float32)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inside = [i > 0, i < nx - 1, j > 0, j < ny - 1, k > 0, k < nz - 1]
    out = []
    for a in range(1, 7):
        c = (prob.coef[a].astype(np.float32) / diag).astype(np.float32)
        out.append(np.where(inside[a - 1].ravel(), c, np.float32(0)).astype(np.float32))
    return out


def apply_unit(dims, c6, q):
    """(D^-1 A) q in FP64."""
    nx, ny, nz = dims
    v = q.astype(np.float64).reshape(nz, ny, nx)
    y = v.copy()
    pads = [(lambda a: np.pad(a, ((0, 0), (0, 0), (1, 0)))[:, :, :-1]),   # w: v(i-1)
            (lambda a: np.pad(a, ((0, 0), (0, 0), (0, 1)))[:, :, 1:]),    # e: v(i+1)
            (lambda a: np.pad(a, ((0, 0), (1, 0), (0, 0)))[:, :-1, :]),   # s: v(j-1)
            (lambda a: np.pad(a, ((0, 0), (0, 1), (0, 0)))[:, 1:, :]),    # n: v(j+1)
            (lambda a: np.pad(a, ((1, 0), (0, 0), (0, 0)))[:-1, :, :]),   # b: v(k-1)
            (lambda a: np.pad(a, ((0, 1), (0, 0), (0, 0)))[1:, :, :])]    # t: v(k+1)
    for a in range(6):
        y += c6[a].astype(np.float64).reshape(nz, ny, nx) * pads[a](v)
    return y.ravel()


@pytest.mark.parametrize("dims", [(64, 48, 20), (40, 30, 11)])
def test_designs_agree_and_match_fp64(s7, dims):
    import torch
    n = int(np.prod(dims))
    rng = np.random.default_rng(17)
    r = rng.standard_normal(n).astype(np.float32)
    s = rng.standard_normal(n).astype(np.float32)
    rh = rng.standard_normal(n).astype(np.float32)
    alpha = np.float32(0.37)
    c6 = unit_operator(dims, seed=5)
    cd = [dev(c) for c in c6]
    rd, sd, hd = dev(r), dev(s), dev(rh)
    # q = fl32(r - alpha s) (one rounding: the product of two FP32 values is exact in FP64)
    q = (r.astype(np.float64) - np.float64(alpha) * s.astype(np.float64)).astype(np.float32)
    yref = apply_unit(dims, c6, q)
    scale = apply_unit(dims, [np.abs(c) for c in c6], np.abs(q))
    first = None
    for kind, param in DESIGNS:
        print("p2 design", dims, kind, param, flush=True)
        y = torch.empty(n, dtype=torch.float32, device="cuda")
        ms, sums = s7.p2_design_probe(kind, param, dims, cd, rd, sd, hd, float(alpha), y, reps=2)
        torch.cuda.synchronize()
        yh = host(y)
        assert ms > 0
        if first is None:
            first = yh
        else:
            assert np.array_equal(yh, first), (kind, param)
        assert np.all(np.abs(yh - yref) <= 8 * 2.0 ** -24 * scale + 1e-30), (kind, param)
        qd, yd, hdd = q.astype(np.float64), yh.astype(np.float64), rh.astype(np.float64)
        want = [qd @ yd, yd @ yd, qd @ qd, hdd @ qd, hdd @ yd]
        for got, w, base in zip(sums, want, [np.abs(qd) @ np.abs(yd), yd @ yd, qd @ qd,
                                             np.abs(hdd) @ np.abs(qd), np.abs(hdd) @ np.abs(yd)]):
            assert abs(got - w) <= 1e-10 * base, (kind, param)


def test_probe_rejects_unsupported_meshes(s7):
    import torch
    dims = (36, 8, 4)  # nx not a multiple of 8
    n = int(np.prod(dims))
    z = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(s7.S7Error):
        s7.p2_design_probe(1, 0, dims, [z] * 6, z, z, z, 0.5, z)
