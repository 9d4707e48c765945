"""Pins of the oracle's 2D 9-point operator (section IV, "SpMV (2D)").

The CSR is checked against a dense matrix assembled from the definition and
against single-coefficient probes (orientation); the operator against the
closed-form eigenpairs of a separable constant-coefficient 9-point stencil
(a Kronecker product of two tridiagonal Toeplitz matrices); the solve against
LAPACK and a manufactured solution, with the recurrence tracking the true
residual throughout.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth

# (di, dj) of each coefficient array, in the order (diag, w, e, s, n, sw, se, nw, ne)
OFFSETS = ((0, 0), (-1, 0), (1, 0), (0, -1), (0, 1), (-1, -1), (1, -1), (-1, 1), (1, 1))


def dense_from_definition(nx, ny, coef):
    """(Av)_(i,j) = sum over the nine offsets (di,dj) of c_(di,dj)(i,j) v(i+di, j+dj)."""
    n = nx * ny
    A = np.zeros((n, n))
    cs = [np.asarray(c, dtype=np.float64) for c in coef]
    for j in range(ny):
        for i in range(nx):
            c = i + nx * j
            for (di, dj), cf in zip(OFFSETS, cs):
                if 0 <= i + di < nx and 0 <= j + dj < ny:
                    A[c, (i + di) + nx * (j + dj)] = cf[c]
    return A


def csr_to_dense(A):
    return sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n)).toarray()


@pytest.mark.parametrize("dims", [(1, 1), (3, 1), (1, 3), (2, 2), (5, 4), (4, 6), (7, 3)])
def test_csr_equals_dense_definition(oracle_mod, dims):
    prob = synth.make_problem_2d9(*dims, seed=5)
    A = oracle_mod.build_csr_2d9(*dims, prob.coef)
    assert np.array_equal(csr_to_dense(A), dense_from_definition(*dims, prob.coef))
    for r in range(A.n):
        cols = A.col[A.rowptr[r]:A.rowptr[r + 1]]
        assert np.all(np.diff(cols) > 0)


@pytest.mark.parametrize("which", range(1, 9))
def test_orientation_single_coefficient(oracle_mod, which):
    """Only array `which` is 1: (A e_c) is 1 exactly at the rows whose (di,dj) neighbour is c."""
    nx, ny = 5, 4
    coef = [np.zeros(nx * ny, np.float32) for _ in range(9)]
    coef[which][:] = 1.0
    A = oracle_mod.build_csr_2d9(nx, ny, coef)
    di, dj = OFFSETS[which]
    ci, cj = 2, 1
    e = np.zeros(nx * ny)
    e[ci + nx * cj] = 1.0
    y = oracle_mod.spmv(A, e)
    want = np.zeros(nx * ny)
    want[(ci - di) + nx * (cj - dj)] = 1.0
    assert np.array_equal(y, want)


def _toeplitz_eigpair(n, m, p, k):
    """tridiag(m, 0, p) of order n: eigenvalue and eigenvector (components i = 1..n)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    th = k * math.pi / (n + 1)
    lam = 2.0 * math.copysign(1.0, p) * math.sqrt(m * p) * math.cos(th)
    return lam, (m / p) ** (i / 2.0) * np.sin(i * th)


@pytest.mark.parametrize("t", [((-1.0, 4.0, -1.0), (-1.0, 4.0, -1.0)),
                               ((-1.25, 4.5, -0.75), (-0.5, 3.0, -1.5))])
def test_separable_kronecker_eigenpairs(oracle_mod, t):
    """c_(di,dj) = tx[di] ty[dj] makes A = Ty (x) Tx: eigenvalue (dx + lx)(dy + ly), vector vy (x) vx."""
    (mx, dx, px), (my, dy, py) = t
    tx = {-1: mx, 0: dx, 1: px}
    ty = {-1: my, 0: dy, 1: py}
    nx, ny = 7, 6
    coef = [np.full(nx * ny, tx[di] * ty[dj], np.float32) for di, dj in OFFSETS]
    A = oracle_mod.build_csr_2d9(nx, ny, coef)
    for kx, ky in ((1, 1), (3, 2), (7, 6)):
        lx, vx = _toeplitz_eigpair(nx, mx, px, kx)
        ly, vy = _toeplitz_eigpair(ny, my, py, ky)
        v = np.outer(vy, vx).ravel()  # x fastest
        lam = (dx + lx) * (dy + ly)
        assert np.allclose(oracle_mod.spmv(A, v), lam * v, rtol=0, atol=1e-12 * np.abs(lam * v).max())


@pytest.mark.parametrize("jac", [True, False])
def test_dense_lu(oracle_mod, jac):
    nx, ny = 6, 5
    prob = synth.make_problem_2d9(nx, ny, seed=9)
    A = oracle_mod.build_csr_2d9(nx, ny, prob.coef)
    b = np.sin(np.arange(A.n) + 1.0)
    ref = np.linalg.solve(dense_from_definition(nx, ny, prob.coef), b)
    res = oracle_mod.bicgstab(A, b, tol=1e-13, max_iter=500, jacobi_scaling=jac)
    assert res.status == oracle_mod.OK
    assert np.linalg.norm(res.x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_manufactured_solution_and_recurrence(oracle_mod):
    nx, ny = 48, 40
    prob = synth.make_problem_2d9(nx, ny, seed=0)
    A = oracle_mod.build_csr_2d9(nx, ny, prob.coef)
    b = oracle_mod.spmv(A, prob.xstar)
    st = oracle_mod.Stepper(A, b, tol=1e-12, max_iter=500, jacobi_scaling=True)
    nb = np.linalg.norm(st.b)
    n = 0
    while not st.done:
        st.step()
        n += 1
        assert np.linalg.norm(st.r - (st.b - oracle_mod.spmv(st.A, st.x))) / nb <= 1e-12
    assert st.st.status == oracle_mod.OK and 5 < n < 300
    assert np.linalg.norm(st.x - prob.xstar) <= 1e-9 * np.linalg.norm(prob.xstar)


def test_recipe_is_diagonally_dominant_and_seeded():
    p = synth.make_problem_2d9(9, 7, seed=3)
    off = sum(np.abs(c.astype(np.float64)) for c in p.coef[1:])
    assert np.all(p.coef[0].astype(np.float64) > off)
    assert all(np.all((c >= -1.0) & (c < -0.5)) for c in p.coef[1:])
    q = synth.make_problem_2d9(9, 7, seed=3)
    assert all(np.array_equal(a, b) for a, b in zip(p.coef, q.coef))
    r = synth.make_problem_2d9(9, 7, seed=4)
    assert not np.array_equal(p.coef[1], r.coef[1])


def test_row_bands_of_the_recipe_and_their_products(oracle_mod):
    """The recipe on a band of y-rows equals those rows of the whole mesh, and the
    9-point CSR of rows j-1..j+1 gives row j of the whole mesh's product exactly (the
    check the paper-size GPU tests make on sampled rows)."""
    nx, ny = 13, 9
    full = synth.make_problem_2d9(nx, ny, seed=7)
    A = oracle_mod.build_csr_2d9(nx, ny, full.coef)
    v = np.random.default_rng(3).standard_normal(nx * ny)
    Av = oracle_mod.spmv(A, v)
    for j in (0, 1, 4, ny - 2, ny - 1):
        band = [q for q in (j - 1, j, j + 1) if 0 <= q < ny]
        sub = synth.make_problem_2d9(nx, ny, seed=7, rows=band)
        lo, hi = band[0] * nx, (band[-1] + 1) * nx
        assert all(np.array_equal(c, f[lo:hi]) for c, f in zip(sub.coef, full.coef))
        assert np.array_equal(sub.xstar, full.xstar[lo:hi])
        Ab = oracle_mod.build_csr_2d9(nx, len(band), sub.coef)
        kk = band.index(j)
        row = oracle_mod.spmv_rows(Ab, v[lo:hi], kk * nx, (kk + 1) * nx)
        assert np.array_equal(row, Av[j * nx:(j + 1) * nx]), j
