"""Pins of the oracle's pipelined BiCGStab (one reduction per iteration, the matrix
products carried by recurrences; Cools and Vanroose 2017) against things other than
itself.

In exact arithmetic its iterates are those of Algorithm 1, so SciPy's independent
BiCGStab and the classical oracle fix them; LAPACK fixes the converged solution; the
degenerate cases reduce to the classical ones; and the recurrence residual it stops
on must track the true residual.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def problem(oracle_mod, dims, seed):
    prob = synth.make_problem(*dims, seed=seed)
    A = oracle_mod.build_csr(*dims, prob.coef)
    return prob, A, oracle_mod.spmv(A, prob.xstar)


def to_scipy(A):
    return sp.csr_matrix((A.val, A.col, A.rowptr), shape=(A.n, A.n))


@pytest.mark.parametrize("jac", [False, True])
def test_iterates_match_scipy_bicgstab(oracle_mod, jac):
    """After k iterations from x0 = 0 the iterate equals SciPy's BiCGStab iterate
    (shadow vector r0) up to rounding."""
    dims = (5, 4, 3)
    prob, A, b = problem(oracle_mod, dims, 7)
    S = to_scipy(A)
    if jac:
        dvals = np.asarray(prob.coef[0], dtype=np.float64)
        S, bs = sp.diags(1.0 / dvals) @ S, b / dvals
    else:
        bs = b
    for k in range(1, 9):
        res = oracle_mod.bicgstab_pipelined(A, b, tol=1e-300, max_iter=k, jacobi_scaling=jac)
        assert res.iters == k and res.status == oracle_mod.NOT_CONVERGED
        xs, info = spla.bicgstab(S, bs, x0=np.zeros(A.n), rtol=0.0, atol=0.0, maxiter=k)
        assert np.linalg.norm(res.x - xs) <= 1e-12 * np.linalg.norm(xs), k


@pytest.mark.parametrize("dims", [(9, 7, 5), (16, 8, 4)])
def test_scalars_and_count_match_classical(oracle_mod, dims):
    """rho_i, alpha_i, omega_i and the recurrence residual after each iteration agree
    with the classical oracle's, and the solve stops after the same number of iterations."""
    prob, A, b = problem(oracle_mod, dims, 3)
    c = oracle_mod.bicgstab(A, b, tol=1e-10, max_iter=500, ntrace=12)
    p = oracle_mod.bicgstab_pipelined(A, b, tol=1e-10, max_iter=500, ntrace=12)
    assert c.status == p.status == oracle_mod.OK and c.iters == p.iters
    for a, b_ in ((c.rho, p.rho), (c.alpha, p.alpha), (c.omega, p.omega), (c.res_trace, p.res_trace)):
        np.testing.assert_allclose(b_, a, rtol=1e-9)
    assert np.linalg.norm(p.x - c.x) <= 1e-9 * np.linalg.norm(c.x)


@pytest.mark.parametrize("dims", [(2, 2, 2), (4, 4, 4), (6, 6, 6)])
@pytest.mark.parametrize("jac", [True, False])
def test_dense_lu(oracle_mod, dims, jac):
    prob, A, b = problem(oracle_mod, dims, 3)
    D = to_scipy(A).toarray()
    ref = np.linalg.solve(D, b)
    res = oracle_mod.bicgstab_pipelined(A, b, tol=1e-13, max_iter=500, jacobi_scaling=jac)
    assert res.status == oracle_mod.OK
    assert np.linalg.norm(res.x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_recurrence_tracks_true_residual(oracle_mod):
    """The residual it stops on is the recurrence r_k; after k iterations it agrees with
    ||b - A x_k|| / ||b|| to 1e-10 (the recurrences for w, t, s, z must not drift)."""
    prob, A, b = problem(oracle_mod, (12, 10, 8), 5)
    for k in (1, 5, 10, 20, 30):
        res = oracle_mod.bicgstab_pipelined(A, b, tol=1e-300, max_iter=k, jacobi_scaling=False)
        assert res.iters == k
        assert abs(res.res_rec - res.rel_res_true) <= 1e-10, (k, res.res_rec, res.rel_res_true)


def test_manufactured_solution(oracle_mod):
    prob, A, b = problem(oracle_mod, (32, 32, 32), 0)
    res = oracle_mod.bicgstab_pipelined(A, b, tol=1e-12, max_iter=500)
    assert res.status == oracle_mod.OK
    assert np.linalg.norm(res.x - prob.xstar) <= 1e-9 * np.linalg.norm(prob.xstar)


def test_degenerate_cases_as_classical(oracle_mod):
    n, dims = 24, (4, 3, 2)
    d = (1.0 + np.arange(n) % 5).astype(np.float32)
    coef = [d] + [np.zeros(n, np.float32) for _ in range(6)]
    A = oracle_mod.build_csr(*dims, coef)
    b = synth.xstar_values(9, np.arange(n))
    # diagonal A with Jacobi scaling: half-step exit in iteration 0 with x = b / diag
    res = oracle_mod.bicgstab_pipelined(A, b, tol=1e-10, max_iter=50)
    assert res.status == oracle_mod.OK and res.iters == 1 and res.half_exit
    assert np.array_equal(res.x, b / d.astype(np.float64))
    # b = 0: x = 0 at once; max_iter = 0: x0 back
    res = oracle_mod.bicgstab_pipelined(A, np.zeros(n), x0=np.ones(n), tol=1e-8)
    assert res.status == oracle_mod.OK and res.iters == 0 and np.all(res.x == 0)
    prob, A3, b3 = problem(oracle_mod, (5, 4, 3), 2)
    res = oracle_mod.bicgstab_pipelined(A3, b3, x0=np.full(A3.n, 0.5), max_iter=0)
    assert res.status == oracle_mod.NOT_CONVERGED and res.iters == 0 and np.all(res.x == 0.5)
    # exact breakdown: A = [[0, 1], [-1, 0]], b = (1, 0): (r0, A r0) = 0
    coef2 = [np.zeros(2, np.float32) for _ in range(7)]
    coef2[2][0] = 1.0
    coef2[1][1] = -1.0
    A2 = oracle_mod.build_csr(2, 1, 1, coef2)
    res = oracle_mod.bicgstab_pipelined(A2, np.array([1.0, 0.0]), tol=1e-8, max_iter=10, jacobi_scaling=False)
    assert res.status == oracle_mod.BREAKDOWN and res.reason == oracle_mod.REASON_RS_ZERO
    # a non-finite coefficient
    coefn = [c.copy() for c in prob.coef]
    coefn[3][5] = np.nan
    An = oracle_mod.build_csr(5, 4, 3, coefn)
    res = oracle_mod.bicgstab_pipelined(An, np.ones(An.n), tol=1e-8, max_iter=10, jacobi_scaling=False)
    assert res.status == oracle_mod.BREAKDOWN and res.reason == oracle_mod.REASON_NONFINITE


def test_a_planted_sign_error_is_caught(oracle_mod):
    """The first pin is sharp: the SciPy iterate after 3 iterations differs from the
    iterate of the same recurrences with the sign of omega in the w update flipped
    (emulated here in NumPy, on the CPU) by far more than the pin's 1e-12."""
    prob, A, b = problem(oracle_mod, (5, 4, 3), 7)
    S = to_scipy(A)

    def run(sign, k):
        x = np.zeros(A.n)
        r = b.copy()
        rh = r.copy()
        w = S @ r
        t = S @ w
        p = s = z = v = np.zeros(A.n)
        rho = rh @ r
        alpha, beta, omega = rho / (rh @ w), 0.0, 0.0
        for _ in range(k):
            p = r + beta * (p - omega * s)
            s = w + beta * (s - omega * z)
            z = t + beta * (z - omega * v)
            q = r - alpha * s
            y = w - alpha * z
            v = S @ z
            omega = (q @ y) / (y @ y)
            x = x + alpha * p + omega * q
            r = q - omega * y
            w = y + sign * omega * (t - alpha * v)
            rho_new = rh @ q - omega * (rh @ y)
            beta = (alpha / omega) * (rho_new / rho)
            sigma = (rh @ w) + beta * ((rh @ s) - omega * (rh @ z))
            rho, alpha = rho_new, rho_new / sigma
            t = S @ w
        return x

    xs, info = spla.bicgstab(S, b, x0=np.zeros(A.n), rtol=0.0, atol=0.0, maxiter=3)
    assert np.linalg.norm(run(-1.0, 3) - xs) <= 1e-12 * np.linalg.norm(xs)
    assert np.linalg.norm(run(+1.0, 3) - xs) > 1e-3 * np.linalg.norm(xs)
