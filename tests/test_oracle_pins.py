"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against something the paper or mathematics fixes:
a dense matrix assembled from the stencil definition, LAPACK dense solves,
closed-form eigenpairs of separable constant-coefficient operators, SciPy's
independent BiCGStab implementation, a hand-worked example, invariants of the
recurrence, and degenerate cases.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def dense_from_definition(nx, ny, nz, coef):
    """Dense A assembled cell by cell: (Av)_c = diag v_c + xm v_(i-1) + xp v_(i+1) + ... ."""
    n = nx * ny * nz
    A = np.zeros((n, n))
    diag, xm, xp, ym, yp, zm, zp = [np.asarray(c, dtype=np.float64) for c in coef]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = i + nx * (j + ny * k)
                A[c, c] = diag[c]
                for (ii, jj, kk), cf in (((i - 1, j, k), xm), ((i + 1, j, k), xp),
                                         ((i, j - 1, k), ym), ((i, j + 1, k), yp),
                                         ((i, j, k - 1), zm), ((i, j, k + 1), zp)):
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        A[c, ii + nx * (jj + ny * kk)] = cf[c]
    return A


def csr_to_dense(A):
    return sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).toarray()


def to_scipy(A):
    return sp.csr_matrix((A.val.copy(), A.col.copy(), A.rowptr.copy()), shape=(A.n, A.n))


MESHES = [(1, 1, 1), (2, 1, 1), (3, 2, 2), (4, 3, 5), (5, 4, 3), (6, 6, 6)]


@pytest.mark.parametrize("dims", MESHES)
def test_csr_equals_dense_definition(oracle_mod, dims):
    prob = synth.make_problem(*dims, seed=11)
    A = oracle_mod.build_csr(*dims, prob.coef)
    D = dense_from_definition(*dims, prob.coef)
    assert np.array_equal(csr_to_dense(A), D)
    # CSR columns strictly ascending within each row
    for r in range(A.n):
        cols = A.col[A.rowptr[r]:A.rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)
    x = synth.xstar_values(5, np.arange(A.n))
    np.testing.assert_allclose(oracle_mod.spmv(A, x), D @ x, rtol=0, atol=1e-13)


def test_orientation_xp_multiplies_plus_neighbour(oracle_mod):
    # v = e_(i+1): (A v)_i must pick up xp_i, not xm_i
    nx, ny, nz = 4, 1, 1
    coef = [np.full(4, 10.0, np.float32)] + [np.zeros(4, np.float32) for _ in range(6)]
    coef[1][:] = -1.0  # xm
    coef[2][:] = -3.0  # xp
    A = oracle_mod.build_csr(nx, ny, nz, coef)
    v = np.zeros(4)
    v[2] = 1.0
    y = oracle_mod.spmv(A, v)
    assert y[1] == -3.0 and y[3] == -1.0 and y[2] == 10.0


def _toeplitz_eigpair(n, m, p, k):
    """1D tridiag(m, ., p): eigenvalue shift and eigenvector, i = 1..n."""
    i = np.arange(1, n + 1, dtype=np.float64)
    th = k * math.pi / (n + 1)
    lam = 2.0 * math.copysign(1.0, p) * math.sqrt(m * p) * math.cos(th)
    v = (m / p) ** (i / 2.0) * np.sin(i * th)
    return lam, v


@pytest.mark.parametrize("mp", [((-1.0, -1.0), (-1.0, -1.0), (-1.0, -1.0), 6.0),
                                ((-1.25, -0.75), (-0.625, -1.125), (-1.5, -0.5), 6.5)])
def test_separable_toeplitz_eigenpairs(oracle_mod, mp):
    (mx, px), (my, py), (mz, pz), d = mp
    nx, ny, nz = 7, 5, 6
    n = nx * ny * nz
    coef = [np.full(n, v, np.float32) for v in (d, mx, px, my, py, mz, pz)]
    A = oracle_mod.build_csr(nx, ny, nz, coef)
    for (kx, ky, kz) in [(1, 1, 1), (2, 3, 1), (7, 5, 6), (4, 2, 5)]:
        lx, vx = _toeplitz_eigpair(nx, mx, px, kx)
        ly, vy = _toeplitz_eigpair(ny, my, py, ky)
        lz, vz = _toeplitz_eigpair(nz, mz, pz, kz)
        lam = d + lx + ly + lz
        v = np.einsum("k,j,i->kji", vz, vy, vx).ravel()
        Av = oracle_mod.spmv(A, v)
        assert np.linalg.norm(Av - lam * v) <= 1e-13 * np.linalg.norm(lam * v) + 1e-14
        if mx == px:
            # the textbook Dirichlet Laplacian spectrum
            ref = 6.0 - 2 * sum(math.cos(kk * math.pi / (nn + 1))
                                for kk, nn in ((kx, nx), (ky, ny), (kz, nz)))
            assert abs(lam - ref) < 1e-14
    # a solve with an eigenvector as right-hand side returns v / lambda
    lx, vx = _toeplitz_eigpair(nx, mx, px, 2)
    ly, vy = _toeplitz_eigpair(ny, my, py, 1)
    lz, vz = _toeplitz_eigpair(nz, mz, pz, 3)
    lam = d + lx + ly + lz
    v = np.einsum("k,j,i->kji", vz, vy, vx).ravel()
    for jac in (False, True):
        res = oracle_mod.bicgstab(A, v, tol=1e-13, max_iter=200, jacobi_scaling=jac)
        assert res.status == oracle_mod.OK
        assert np.linalg.norm(res.x - v / lam) <= 1e-11 * np.linalg.norm(v / lam)


def test_orientation_pinned_by_nonsymmetric_eigvec(oracle_mod):
    # With xm and xp swapped, the eigenvector of the closed form is no longer one.
    nx, ny, nz = 9, 1, 1
    m, p, d = -1.5, -0.5, 4.0
    coef = [np.full(9, v, np.float32) for v in (d, m, p, 0, 0, 0, 0)]
    A = oracle_mod.build_csr(nx, ny, nz, coef)
    lam, v = _toeplitz_eigpair(nx, m, p, 1)
    assert np.linalg.norm(oracle_mod.spmv(A, v) - (d + lam) * v) < 1e-13 * np.linalg.norm(v)
    coef_sw = [coef[0], coef[2], coef[1]] + coef[3:]
    A2 = oracle_mod.build_csr(nx, ny, nz, coef_sw)
    assert np.linalg.norm(oracle_mod.spmv(A2, v) - (d + lam) * v) > 1e-3 * np.linalg.norm(v)


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 4, 2), (4, 4, 4), (5, 3, 6), (6, 6, 6)])
@pytest.mark.parametrize("jac", [True, False])
def test_dense_lu(oracle_mod, dims, jac):
    prob = synth.make_problem(*dims, seed=3)
    A = oracle_mod.build_csr(*dims, prob.coef)
    D = dense_from_definition(*dims, prob.coef)
    b = D @ prob.xstar
    ref = np.linalg.solve(D, b)
    res = oracle_mod.bicgstab(A, b, tol=1e-13, max_iter=500, jacobi_scaling=jac)
    assert res.status == oracle_mod.OK
    assert np.linalg.norm(res.x - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("jac", [False, True])
def test_iterates_match_scipy_bicgstab(oracle_mod, jac):
    """SciPy's BiCGStab (van der Vorst recurrences, r_tilde = r0) is an independent
    implementation of the same iteration: after k iterations from x0 = 0 the iterates agree."""
    dims = (5, 4, 3)
    prob = synth.make_problem(*dims, seed=7)
    A = oracle_mod.build_csr(*dims, prob.coef)
    S = to_scipy(A)
    b = S @ prob.xstar
    if jac:
        dvals = np.asarray(prob.coef[0], dtype=np.float64)
        S = sp.diags(1.0 / dvals) @ S
        bs = b / dvals
    else:
        bs = b
    for k in range(1, 8):
        res = oracle_mod.bicgstab(A, b, tol=1e-300, max_iter=k, jacobi_scaling=jac)
        assert res.iters == k and res.status == oracle_mod.NOT_CONVERGED
        xs, info = spla.bicgstab(S, bs, x0=np.zeros(A.n), rtol=0.0, atol=0.0, maxiter=k)
        assert np.linalg.norm(res.x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_golden_hand_worked_2x1x1(oracle_mod):
    with open(os.path.join(GOLDEN, "bicgstab_2x1x1.json")) as f:
        g = json.load(f)
    coef = [np.array(g["coef"][nm], np.float32) for nm in synth.COEF_NAMES]
    A = oracle_mod.build_csr(*g["dims"], coef)
    st = oracle_mod.Stepper(A, np.array(g["b"]), tol=1e-12, max_iter=10, jacobi_scaling=False)
    st.step()
    it0 = g["iter0"]
    np.testing.assert_allclose(st.s, it0["s"], rtol=0, atol=1e-15)
    assert abs(st.st.alpha - it0["alpha"]) < 1e-15
    np.testing.assert_allclose(st.q, it0["q"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(st.y, it0["y"], rtol=0, atol=1e-15)
    assert abs(st.st.omega - it0["omega"]) < 1e-15
    np.testing.assert_allclose(st.x, it0["x"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(st.r, it0["r"], rtol=0, atol=1e-15)
    assert abs(st.st.beta - it0["beta"]) < 1e-15
    np.testing.assert_allclose(st.p, it0["p"], rtol=0, atol=1e-15)
    st.step()
    np.testing.assert_allclose(st.s, g["iter1"]["s"], rtol=0, atol=1e-15)
    a1 = g["iter1"]["alpha"]
    assert abs(st.st.alpha - a1[0] / a1[1]) < 1e-15
    assert st.done and st.st.half_exit == 1 and st.st.iter == g["iterations"]
    sol = [a / b for a, b in g["solution"]]
    np.testing.assert_allclose(st.x, sol, rtol=0, atol=1e-15)


def test_recurrence_tracks_true_residual(oracle_mod):
    wl = synth.WORKLOADS["cube32"]
    dims = wl["dims"]
    prob = synth.make_problem(*dims, seed=wl["seed"], recipe=wl["recipe"])
    A = oracle_mod.build_csr(*dims, prob.coef)
    b = oracle_mod.spmv(A, prob.xstar)
    st = oracle_mod.Stepper(A, b, tol=1e-12, max_iter=500, jacobi_scaling=True)
    nb = np.linalg.norm(st.b)
    n = 0
    while not st.done:
        st.step()
        n += 1
        true_r = st.b - oracle_mod.spmv(st.A, st.x)
        assert np.linalg.norm(st.r - true_r) / nb <= 1e-12
    assert st.st.status == oracle_mod.OK and 20 < n < 200


def test_manufactured_solution(oracle_mod):
    wl = synth.WORKLOADS["cube32"]
    dims = wl["dims"]
    prob = synth.make_problem(*dims, seed=wl["seed"], recipe=wl["recipe"])
    A = oracle_mod.build_csr(*dims, prob.coef)
    b = oracle_mod.spmv(A, prob.xstar)
    res = oracle_mod.bicgstab(A, b, tol=1e-12, max_iter=500)
    assert res.status == oracle_mod.OK
    assert np.linalg.norm(res.x - prob.xstar) <= 1e-9 * np.linalg.norm(prob.xstar)
    assert res.rel_res_true <= 1e-11


def test_diagonal_matrix_half_step_exit(oracle_mod):
    dims = (4, 3, 2)
    n = 24
    d = (1.0 + np.arange(n) % 5).astype(np.float32)
    coef = [d] + [np.zeros(n, np.float32) for _ in range(6)]
    A = oracle_mod.build_csr(*dims, coef)
    b = synth.xstar_values(9, np.arange(n))
    res = oracle_mod.bicgstab(A, b, tol=1e-10, max_iter=50, jacobi_scaling=True)
    assert res.status == oracle_mod.OK and res.iters == 1 and res.half_exit
    assert np.array_equal(res.x, b / d.astype(np.float64))
    # unscaled A = c I: also exits at the half step of the first iteration
    coef2 = [np.full(n, 3.0, np.float32)] + coef[1:]
    A2 = oracle_mod.build_csr(*dims, coef2)
    res2 = oracle_mod.bicgstab(A2, b, tol=1e-10, max_iter=50, jacobi_scaling=False)
    assert res2.status == oracle_mod.OK and res2.iters == 1 and res2.half_exit
    np.testing.assert_allclose(res2.x, b / 3.0, rtol=1e-15)


def test_zero_rhs_and_zero_iterations(oracle_mod):
    dims = (3, 3, 3)
    prob = synth.make_problem(*dims, seed=2)
    A = oracle_mod.build_csr(*dims, prob.coef)
    x0 = np.ones(A.n)
    res = oracle_mod.bicgstab(A, np.zeros(A.n), x0=x0, tol=1e-8, max_iter=10)
    assert res.status == oracle_mod.OK and res.iters == 0 and np.all(res.x == 0)
    b = oracle_mod.spmv(A, prob.xstar)
    res = oracle_mod.bicgstab(A, b, x0=x0, tol=1e-8, max_iter=0)
    assert res.status == oracle_mod.NOT_CONVERGED and res.iters == 0 and np.all(res.x == x0)
    # starting at the solution: converged before the first iteration
    res = oracle_mod.bicgstab(A, b, x0=prob.xstar, tol=1e-8, max_iter=10)
    assert res.status == oracle_mod.OK and res.iters == 0


def test_exact_breakdown(oracle_mod):
    # A = [[0, 1], [-1, 0]], b = (1, 0): s = (0, -1), (r0, s) = 0 exactly
    coef = [np.zeros(2, np.float32) for _ in range(7)]
    coef[2][0] = 1.0   # xp of cell 0
    coef[1][1] = -1.0  # xm of cell 1
    A = oracle_mod.build_csr(2, 1, 1, coef)
    res = oracle_mod.bicgstab(A, np.array([1.0, 0.0]), tol=1e-8, max_iter=10, jacobi_scaling=False)
    assert res.status == oracle_mod.BREAKDOWN and res.reason == oracle_mod.REASON_RS_ZERO


@pytest.mark.parametrize("case", ["yy_zero", "rho_zero"])
def test_golden_breakdowns(oracle_mod, case):
    """The two exact breakdowns of the scalar steps, on hand-worked 2x1x1 systems
    (tests/golden/bicgstab_breakdowns.json): (y,y) = 0 after the q-step, and
    (r0, r_1) = 0 after a full step.  Every intermediate value is exact."""
    with open(os.path.join(GOLDEN, "bicgstab_breakdowns.json")) as f:
        g = json.load(f)[case]
    coef = [np.array(g["coef"][nm], np.float32) for nm in synth.COEF_NAMES]
    A = oracle_mod.build_csr(*g["dims"], coef)
    b = np.array(g["b"])
    st = oracle_mod.Stepper(A, b, tol=1e-8, max_iter=10, jacobi_scaling=False)
    st.step()
    assert np.array_equal(st.s, g["s"]) and st.st.sigma == g["sigma"] and st.st.alpha == g["alpha"]
    assert np.array_equal(st.q, g["q"]) and np.array_equal(st.y, g["y"])
    if "omega" in g:
        assert st.st.omega == g["omega"]
        assert np.array_equal(st.x, g["x"]) and np.array_equal(st.r, g["r"])
    reason = getattr(oracle_mod, "REASON_" + g["reason"])
    assert st.done and st.st.status == oracle_mod.BREAKDOWN and st.st.reason == reason
    assert st.st.iter == g["iters"]
    res = oracle_mod.bicgstab(A, b, tol=1e-8, max_iter=10, jacobi_scaling=False)
    assert res.status == oracle_mod.BREAKDOWN and res.reason == reason and res.iters == g["iters"]


@pytest.mark.parametrize("dims,rows", [((5, 4, 3), (0, 60)), ((5, 4, 3), (20, 40)),
                                       ((7, 3, 4), (17, 53)), ((6, 6, 6), (215, 216)),
                                       ((4, 1, 1), (1, 3)), ((3, 5, 2), (0, 0))])
def test_spmv_rows_equals_rows_of_spmv_and_dense(oracle_mod, dims, rows):
    """The row-range product (used on sampled planes of meshes too large for the whole
    product) equals the same rows of the full product and of the dense matrix from the
    stencil definition, on ragged row ranges that start and end inside planes."""
    prob = synth.make_problem(*dims, seed=23)
    A = oracle_mod.build_csr(*dims, prob.coef)
    v = synth.xstar_values(24, np.arange(A.n))
    r0, r1 = rows
    part = oracle_mod.spmv_rows(A, v, r0, r1)
    assert part.shape == (r1 - r0,)
    assert np.array_equal(part, oracle_mod.spmv(A, v)[r0:r1])
    D = dense_from_definition(*dims, prob.coef)
    np.testing.assert_allclose(part, (D @ v)[r0:r1], rtol=1e-14, atol=1e-14)


def test_nonfinite_input_is_breakdown(oracle_mod):
    dims = (3, 2, 2)
    prob = synth.make_problem(*dims, seed=4)
    coef = [c.copy() for c in prob.coef]
    coef[3][5] = np.nan
    A = oracle_mod.build_csr(*dims, coef)
    b = np.ones(A.n)
    res = oracle_mod.bicgstab(A, b, tol=1e-8, max_iter=10, jacobi_scaling=False)
    assert res.status == oracle_mod.BREAKDOWN and res.reason == oracle_mod.REASON_NONFINITE


def test_spmv_threads_do_not_change_results(oracle_mod):
    """The oracle's SpMV row loop may run on several threads to time it on all host
    cores; every row is still summed left to right, so the product and a whole solve
    are bit for bit those of one thread."""
    dims = (20, 16, 12)
    prob = synth.make_problem(*dims, seed=25)
    A = oracle_mod.build_csr(*dims, prob.coef)
    b = oracle_mod.spmv(A, prob.xstar)
    r1 = oracle_mod.bicgstab(A, b, tol=1e-10, max_iter=500)
    try:
        oracle_mod.set_threads(4)
        y4 = oracle_mod.spmv(A, prob.xstar)
        r4 = oracle_mod.bicgstab(A, b, tol=1e-10, max_iter=500)
    finally:
        oracle_mod.set_threads(1)
    assert np.array_equal(y4, b)
    assert r4.iters == r1.iters and np.array_equal(r4.x, r1.x)


def test_table1_flop_accounting():
    with open(os.path.join(GOLDEN, "table1_ops.json")) as f:
        g = json.load(f)
    s = g["single"]
    assert [sum(v[i] for k, v in s.items() if k != "total") for i in range(2)] == s["total"]
    m = g["mixed"]
    assert [sum(v[i] for k, v in m.items() if k != "total") for i in range(3)] == m["total"]
    assert sum(s["total"]) == sum(m["total"]) == g["flops_per_point_per_iter"]
    pts = int(np.prod(g["mesh"]))
    assert abs(g["flops_per_point_per_iter"] * pts / g["seconds_per_iter"] / 1e15 - g["pflops"]) < 0.01
    from paper_2010_03660_amd import FLOPS_PER_CELL_ITER
    assert FLOPS_PER_CELL_ITER == g["flops_per_point_per_iter"]
