"""GPU parity of the stencil apply and the device generator against the oracle.

s7_stencil_apply takes two forms: single cells, and (even nx, at least 2^18 cells, aligned
arrays) x-adjacent pairs with v staged in LDS in 2048-cell tiles.  Both are checked
against the oracle's SpMV, on ragged tails and with non-finite outward coefficients."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import gpu_available
from tests.gpu_helpers import U32, abs_row_bound, coef_dev, dev, host

pytestmark = pytest.mark.gpu

# several tiles in x (62 columns each) and y (4 or 8 rows), ragged tails, z chunks; the
# staged form for 200x33x65 (a ragged last tile), 130x70x40 and 1024x16x17 (long rows);
# 4098x4x17 has rows too long for the staging LDS and takes single cells
SHAPES = [(1, 1, 1), (2, 1, 1), (1, 1, 7), (5, 3, 2), (62, 4, 3), (63, 9, 7), (64, 17, 33),
          (130, 70, 20), (200, 33, 65), (17, 100, 40), (130, 70, 40), (1024, 16, 17), (4098, 4, 17)]


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def _apply(s7, dims, coef, v):
    import torch
    u = torch.full_like(v, float("nan"))
    s7.stencil_apply(dims, coef, v, u)
    torch.cuda.synchronize()
    return host(u)


@pytest.mark.parametrize("dims", SHAPES)
def test_stencil_apply_matches_oracle_spmv(s7, dims):
    prob = synth.make_problem(*dims, seed=21)
    A = oracle.build_csr(*dims, prob.coef)
    v = prob.xstar.astype(np.float32)
    u = _apply(s7, dims, coef_dev(prob), dev(v))
    ref = oracle.spmv(A, v.astype(np.float64))
    bound = 8 * U32 * abs_row_bound(A, v.astype(np.float64))
    assert np.all(np.isfinite(u))
    assert np.all(np.abs(u - ref) <= bound + 1e-30), np.max(np.abs(u - ref) / bound)


@pytest.mark.parametrize("dims", [(70, 11, 6), (70, 64, 64)])
def test_outward_coefficients_are_ignored(s7, dims):
    prob = synth.make_problem(*dims, seed=5)
    A = oracle.build_csr(*dims, prob.coef)
    coef = [c.copy() for c in prob.coef]
    nx, ny, nz = dims
    c3 = [c.reshape(nz, ny, nx) for c in coef]
    c3[1][:, :, 0] = np.nan
    c3[2][:, :, -1] = np.inf
    c3[3][:, 0, :] = np.nan
    c3[4][:, -1, :] = -np.inf
    c3[5][0] = np.nan
    c3[6][-1] = np.nan
    v = prob.xstar.astype(np.float32)
    u = _apply(s7, dims, [dev(c) for c in coef], dev(v))
    ref = oracle.spmv(A, v.astype(np.float64))
    bound = 8 * U32 * abs_row_bound(A, v.astype(np.float64))
    assert np.all(np.abs(u - ref) <= bound)


def test_staged_and_single_cell_forms_agree(s7):
    """The same apply through the staged pairs (aligned v) and through single cells (v
    one element into a buffer, so not 16-byte aligned) gives the same values."""
    import torch
    dims = (200, 33, 65)
    prob = synth.make_problem(*dims, seed=4)
    coef = coef_dev(prob)
    v = prob.xstar.astype(np.float32)
    a = _apply(s7, dims, coef, dev(v))
    buf = torch.empty(v.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = dev(v)
    b = _apply(s7, dims, coef, buf[1:])
    assert np.array_equal(a, b)


def test_stencil_apply_deterministic(s7):
    dims = (130, 70, 20)
    prob = synth.make_problem(*dims, seed=1)
    coef = coef_dev(prob)
    v = dev(prob.xstar.astype(np.float32))
    assert np.array_equal(_apply(s7, dims, coef, v), _apply(s7, dims, coef, v))


@pytest.mark.parametrize("dims,recipe", [((37, 29, 23), 0), ((64, 64, 64), 1), ((5, 1, 9), 1)])
def test_device_generator_bit_identical(s7, dims, recipe):
    import torch
    n = int(np.prod(dims))
    coef = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(7)]
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    s7.generate_problem(dims, 77, recipe, coef, xs, b)
    torch.cuda.synchronize()
    prob = synth.make_problem(*dims, seed=77, recipe=recipe)
    for a in range(7):
        assert np.array_equal(host(coef[a]).view(np.uint32), prob.coef[a].view(np.uint32)), a
    assert np.array_equal(host(xs), prob.xstar)
    A = oracle.build_csr(*dims, prob.coef)
    bref = oracle.spmv(A, prob.xstar)
    bound = 4 * 2.0 ** -53 * abs_row_bound(A, prob.xstar)
    assert np.all(np.abs(host(b) - bref) <= bound)


def test_paper_mesh_stencil_sampled(s7):
    """600x595x1536 (the paper's mesh), the launch shape the benchmark uses: sampled
    outputs checked one by one against the oracle on the planes around them."""
    import torch
    dims = synth.PAPER_MESH
    nx, ny, nz = dims
    n = nx * ny * nz
    coef = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(7)]
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    s7.generate_problem(dims, 0, 0, coef, xs, None)
    v = xs.to(torch.float32)
    del xs
    u = torch.empty_like(v)
    s7.stencil_apply(dims, coef, v, u)
    torch.cuda.synchronize()
    for k in (0, 1, 767, nz - 2, nz - 1):
        # the CSR of the slab of planes k-1..k+1 is exact on the rows of plane k: each
        # z-link of those rows lands inside the slab or outside the mesh
        planes = [p for p in (k - 1, k, k + 1) if 0 <= p < nz]
        prob = synth.make_problem(nx, ny, nz, seed=0, planes=planes)
        A = oracle.build_csr(nx, ny, len(planes), prob.coef)
        vs = prob.xstar.astype(np.float32).astype(np.float64)
        kk = planes.index(k)
        r0, r1 = kk * nx * ny, (kk + 1) * nx * ny
        ref = oracle.spmv_rows(A, vs, r0, r1)
        got = host(u[k * nx * ny:(k + 1) * nx * ny])
        bound = 8 * U32 * abs_row_bound(A, vs)[r0:r1]
        assert np.all(np.abs(got - ref) <= bound + 1e-30), k
