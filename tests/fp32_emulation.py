"""CPU emulations of the GPU's FP32-storage BiCGStab iterations (test helpers).

Every vector is rounded to FP32 after each operation and the inner products are taken in
FP64, as the GPU kernels do.  The classical iteration is Algorithm 1; the pipelined one
is the single-reduction variant of the oracle (oracle_bicgstab_pipelined), with optional
residual replacement.  These are not bit-exact copies of the GPU arithmetic (the GPU
fuses multiply-adds and orders its sums differently); they show what FP32 storage does
to the recurrences and to the stopping iteration."""
import numpy as np
import scipy.sparse as sp

import oracle
import synth

F = np.float32


def system(dims, seed, jacobi=True):
    """(A, b, S, bs): the oracle's CSR and b = A x*, and the iterated system with its
    matrix entries rounded to FP32 (Jacobi-scaled unless jacobi is False).  Two dims
    give the 2D 9-point operator, three the 7-point one."""
    if len(dims) == 2:
        prob = synth.make_problem_2d9(*dims, seed=seed)
        A = oracle.build_csr_2d9(*dims, prob.coef)
    else:
        prob = synth.make_problem(*dims, seed=seed)
        A = oracle.build_csr(*dims, prob.coef)
    b = oracle.spmv(A, prob.xstar)
    As, bs = oracle.jacobi(A, b) if jacobi else (A, b)
    S = sp.csr_matrix((As.val.astype(F).astype(np.float64), As.col, As.rowptr), shape=(A.n, A.n))
    return A, b, S, bs


def mv(S, v):
    return (S @ v.astype(np.float64)).astype(F)


def dot(a, b):
    return float(a.astype(np.float64) @ b.astype(np.float64))


def classical_fp32(S, bs, tol, max_iter=2000, count=False):
    """Algorithm 1 with FP32 vectors; returns x (and the iteration count if count)."""
    r = bs.astype(F)
    rh, p, x = r.copy(), r.copy(), np.zeros_like(r)
    nb, rho = np.linalg.norm(bs), dot(r, r)
    it = 0
    while it < max_iter:
        it += 1
        s = mv(S, p)
        a = F(rho / dot(rh, s))
        q = r - a * s
        if np.sqrt(dot(q, q)) / nb <= tol:
            x = x + a * p
            break
        y = mv(S, q)
        om = F(dot(q, y) / dot(y, y))
        x = x + a * p + om * q
        r = q - om * y
        if np.sqrt(dot(r, r)) / nb <= tol:
            break
        rho_new = dot(rh, r)
        p = r + F((a / om) * (rho_new / rho)) * (p - om * s)
        rho = rho_new
    return (x, it) if count else x


def pipelined_fp32(S, bs, tol, max_iter=2000, replace_every=0):
    r = bs.astype(F)
    rh, x = r.copy(), np.zeros_like(r)
    xs = np.zeros(len(bs))  # the FP64 iterate that absorbs x at each replacement
    w = mv(S, r)
    t = mv(S, w)
    p = s = z = v = np.zeros_like(r)
    nb, rho = np.linalg.norm(bs), dot(r, r)
    alpha, beta, om = rho / dot(rh, w), 0.0, 0.0
    for it in range(max_iter):
        if replace_every and it > 0 and it % replace_every == 0:
            xs, x = xs + x.astype(np.float64), np.zeros_like(r)
            r = (bs - S @ xs).astype(F)
            w = mv(S, r)
            t = mv(S, w)
            s = mv(S, p)
            z = mv(S, s)
            v = mv(S, z)
            rho = dot(rh, r)
            alpha = rho / (dot(rh, w) + beta * (dot(rh, s) - om * dot(rh, z)))
        a, bt, o = F(alpha), F(beta), F(om)
        p = r + bt * (p - o * s)
        s = w + bt * (s - o * z)
        z = t + bt * (z - o * v)
        q = r - a * s
        y = w - a * z
        v = mv(S, z)
        if np.sqrt(dot(r, r)) / nb <= tol:
            return xs + x
        if np.sqrt(dot(q, q)) / nb <= tol:
            return xs + (x + a * p)
        om = dot(q, y) / dot(y, y)
        x = x + a * p + F(om) * q
        r = q - F(om) * y
        w = y - F(om) * (t - a * v)
        rho_new = dot(rh, q) - om * dot(rh, y)
        beta = (alpha / om) * (rho_new / rho)
        sigma = dot(rh, y) - om * (dot(rh, t) - alpha * dot(rh, v)) + beta * (dot(rh, s) - om * dot(rh, z))
        rho, alpha = rho_new, rho_new / sigma
        t = mv(S, w)
    return xs + x
