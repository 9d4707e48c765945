"""Why the GPU's pipelined BiCGStab replaces its residuals: with FP32 storage, the
pipelined recurrences for the matrix products drift from the matrix they stand for.

Both iterations are emulated here on the CPU with every vector rounded to FP32 after
each operation and the inner products taken in FP64, as the GPU kernels do.  At the
same recurrence tolerance the classical iteration's true residual stays near its
recurrence residual, while the pipelined one's (y = w - alpha z in place of A q,
w = y - omega (t - alpha v) in place of A r) ends orders of magnitude above it.  The
FP64 oracle of each iteration reaches the solution (tests/test_oracle_pins_pipelined.py),
so the difference is the storage precision, not the recurrences themselves.  Recomputing
r = b - A x and the products from their definitions every 10 iterations, as the GPU
solve does, brings the true residual back to the classical iteration's level."""
import numpy as np

import oracle
from tests.fp32_emulation import classical_fp32, pipelined_fp32, system


def test_pipelined_recurrences_drift_in_fp32_storage():
    A, b, S, bs = system((9, 7, 5), 11)
    xc = classical_fp32(S, bs, 1e-6).astype(np.float64)
    xp = pipelined_fp32(S, bs, 1e-6).astype(np.float64)
    rc = oracle.true_rel_residual(A, b, xc)
    rp = oracle.true_rel_residual(A, b, xp)
    assert rc <= 1e-5, rc
    assert rp >= 1e-3, rp


def test_residual_replacement_restores_the_true_residual():
    for dims in ((9, 7, 5), (33, 17, 9), (64, 48, 20)):
        A, b, S, bs = system(dims, 11)
        x = pipelined_fp32(S, bs, 1e-6, replace_every=10).astype(np.float64)
        assert oracle.true_rel_residual(A, b, x) <= 3e-6, dims
