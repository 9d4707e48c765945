"""Shared helpers of the GPU tests: device copies of synthetic problems and
oracle references (the oracle runs on the host CPU)."""
import numpy as np

import oracle
import synth

U32 = 2.0 ** -24


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def coef_dev(prob):
    return [dev(c) for c in prob.coef]


def problem(dims, seed=0, recipe=synth.RECIPE_IID):
    """(prob, CSR, b) with b = A x* computed by the oracle in FP64."""
    prob = synth.make_problem(*dims, seed=seed, recipe=recipe)
    A = oracle.build_csr(*dims, prob.coef)
    b = oracle.spmv(A, prob.xstar)
    return prob, A, b


def abs_row_bound(A, v):
    """sum_j |a_ij v_j| per row (FP64), the scale of the rounding error of row i."""
    absA = oracle.CSR(A.n, A.rowptr, A.col, np.abs(A.val), A.dims)
    return oracle.spmv(absA, np.abs(v))


def rel_err(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
