"""The solve that allocates nothing (s7_bicgstab_solve_noalloc): its workspace is the
library's fixed per-GPU array.  Checked through the C-ABI against s7_bicgstab_solve with
a caller workspace (bit for bit: same kernels, same options, no tuning) and against the
FP64 oracle (1e-6 relative at recurrence tolerance 1e-8), on two calls in a row, the
second with a smaller system, so that the second reuses the array the first left
behind."""
import numpy as np
import pytest

import oracle
from tests.conftest import gpu_available
from tests.gpu_helpers import coef_dev, dev, host, problem, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def test_noalloc_matches_solve_two_calls(s7):
    import torch
    for dims, seed in (((64, 48, 40), 31), ((33, 17, 9), 32)):
        prob, A, b = problem(dims, seed=seed)
        coef, bd = coef_dev(prob), dev(b)
        n = A.n
        opt = s7.default_options(tune=0)
        xa = torch.zeros(n, dtype=torch.float64, device="cuda")
        ia = s7.bicgstab_solve_noalloc(dims, coef, bd, xa, 1e-8, 2000, opt=opt)
        xb = torch.zeros(n, dtype=torch.float64, device="cuda")
        ib = s7.bicgstab_solve(dims, coef, bd, xb, 1e-8, 2000, prec=s7.FP32, opt=opt)
        torch.cuda.synchronize()
        assert ia.status == s7.OK and ib.status == s7.OK, (ia.as_dict(), ib.as_dict())
        assert ia.iters == ib.iters and ia.schedule == ib.schedule
        assert np.array_equal(host(xa), host(xb)), dims
        assert ia.rel_res_true == ib.rel_res_true
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(host(xa), ref.x) <= 1e-6


def test_noalloc_rejects_systems_beyond_the_fixed_workspace(s7):
    import torch
    dims = (128, 128, 128)  # about 109 MB of workspace
    assert s7.workspace_bytes(dims) > s7.NOALLOC_WS_BYTES
    n = 128 ** 3
    coef = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(7)]
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(s7.S7Error) as e:
        s7.bicgstab_solve_noalloc(dims, coef, b, x, 1e-8, 10)
    assert e.value.code == s7.EINVAL
    assert "fixed workspace" in s7.last_error()
