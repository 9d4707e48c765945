"""GPU tests of 2D 9-point requests in the request queue (section IV's operator in
the serving form), against the FP64 oracle.

2D requests share the arena, the admission order, the large-request thread and
the batch engine with 3D requests: one persistent launch runs both operators.
As for 3D, a request's result does not depend on what else is resident: served
in a mix it comes out bit for bit as the batched 2D call computes it alone, and a
large mesh comes out as from the single-system 2D call."""
import numpy as np
import pytest

import oracle
import synth
from tests.conftest import gpu_available
from tests.gpu_helpers import coef_dev, dev, host, problem, rel_err

pytestmark = pytest.mark.gpu

MIX9 = [((64, 48), 0), ((17, 9), 1), ((129, 33), 0), ((1, 5), 1), ((250, 7), 2), ((300, 200), 0)]
MIX3 = [((24, 32, 20), 0), ((17, 13, 9), 1)]
RTOL = {0: 1e-8, 1: 1e-10, 2: 1e-10}


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def problem9(dims, seed):
    p = synth.make_problem_2d9(*dims, seed=seed)
    A = oracle.build_csr_2d9(*dims, p.coef)
    return p, A, oracle.spmv(A, p.xstar)


def zeros(n):
    import torch
    return torch.zeros(n, dtype=torch.float64, device="cuda")


def run_queue(s7, submit_all, arena_bytes, **opt):
    import torch
    ar = torch.empty(s7.queue_table_bytes() + arena_bytes, dtype=torch.uint8, device="cuda")
    q = s7.queue_create(ar, opt=s7.default_options(**opt))
    try:
        tickets = submit_all(q)
        out = [s7.queue_wait(q, t) for t in tickets]
    finally:
        s7.queue_destroy(q)
    return out


@pytest.mark.parametrize("epoch", [0, 5])
def test_served_2d9_beside_3d_matches_oracle_and_alone(s7, epoch):
    """2D requests in three precisions, interleaved with 3D requests in the same
    persistent launches, with time slices (epoch 0) or 5-iteration epochs and a tight
    arena: each result matches the oracle and equals the batched call of its operator
    on that request alone (load-sized chunks in the queue, default ones alone)."""
    import torch
    p9 = [problem9(d, 900 + i) for i, (d, pr) in enumerate(MIX9)]
    p3 = [problem(d, seed=950 + i) for i, (d, pr) in enumerate(MIX3)]
    c9 = [[dev(c) for c in p.coef] for p, A, b in p9]
    b9 = [dev(b) for p, A, b in p9]
    x9 = [zeros(A.n) for p, A, b in p9]
    c3 = [coef_dev(p) for p, A, b in p3]
    b3 = [dev(b) for p, A, b in p3]
    x3 = [zeros(A.n) for p, A, b in p3]
    torch.cuda.synchronize()

    def submit_all(q):
        t = []
        for i, ((nx, ny), pr) in enumerate(MIX9):
            t.append(s7.queue_submit_2d9(q, nx, ny, c9[i], b9[i], x9[i], RTOL[pr], 2000, pr))
            if i < len(MIX3):
                d, pr3 = MIX3[i]
                t.append(s7.queue_submit(q, d, c3[i], b3[i], x3[i], RTOL[pr3], 2000, pr3))
        return t
    big = max(s7.workspace_bytes_2d9(nx, ny, pr) for (nx, ny), pr in MIX9)
    out = run_queue(s7, submit_all, 3 * big + (4 << 20), graph_iters=epoch)
    assert all(rc == s7.OK for rc, info in out), [info.as_dict() for rc, info in out]
    order = []
    for i in range(len(MIX9)):
        order.append(("2d", i))
        if i < len(MIX3):
            order.append(("3d", i))
    res = dict(zip(order, out))
    for i, ((nx, ny), pr) in enumerate(MIX9):
        p, A, b = p9[i]
        rc, info = res[("2d", i)]
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert rel_err(host(x9[i]), ref.x) <= (1e-6 if pr == 0 else 1e-7), i
        x1 = zeros(A.n)
        rc1, inf1 = s7.bicgstab_solve_batched_2d9([(nx, ny)], [c9[i]], [b9[i]], [x1], [RTOL[pr]], [2000],
                                                  prec=pr)
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), host(x9[i])), i
        assert inf1[0].iters == info.iters and inf1[0].outer_iters == info.outer_iters, i
    for i, (d, pr) in enumerate(MIX3):
        p, A, b = p3[i]
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert rel_err(host(x3[i]), ref.x) <= (1e-6 if pr == 0 else 1e-7), i
        x1 = zeros(A.n)
        rc1, inf1 = s7.bicgstab_solve_batched([d], [c3[i]], [b3[i]], [x1], [RTOL[pr]], [2000], prec=pr)
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), host(x3[i])), i
        assert inf1[0].iters == res[("3d", i)][1].iters, i


def test_large_2d9_requests_take_the_single_system_path(s7):
    """With split_cells = 20000, 2D meshes of at least that many cells run on the
    large-request thread: each equals bicgstab_solve_2d9 alone, bit for bit."""
    import torch
    mix = [((200, 150), 0), ((129, 33), 0), ((250, 120), 1)]
    probs = [problem9(d, 980 + i) for i, (d, pr) in enumerate(mix)]
    cs = [[dev(c) for c in p.coef] for p, A, b in probs]
    bs = [dev(b) for p, A, b in probs]
    xs = [zeros(A.n) for p, A, b in probs]
    torch.cuda.synchronize()
    out = run_queue(s7, lambda q: [s7.queue_submit_2d9(q, *d, cs[i], bs[i], xs[i], RTOL[pr], 2000, pr)
                                   for i, (d, pr) in enumerate(mix)], 64 << 20, split_cells=20000)
    for i, ((d, pr), (p, A, b), (rc, info)) in enumerate(zip(mix, probs, out)):
        assert rc == s7.OK, (i, info.as_dict())
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert rel_err(host(xs[i]), ref.x) <= (1e-6 if pr == 0 else 1e-7), i
        x1 = zeros(A.n)
        if d[0] * d[1] >= 20000:
            i1 = s7.bicgstab_solve_2d9(*d, cs[i], bs[i], x1, RTOL[pr], 2000, prec=pr,
                                       opt=s7.default_options(split_cells=20000))
        else:
            rc1, inf1 = s7.bicgstab_solve_batched_2d9([d], [cs[i]], [bs[i]], [x1], [RTOL[pr]], [2000], prec=pr)
            i1 = inf1[0]
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), host(xs[i])) and i1.iters == info.iters, i


def test_submit_2d9_refuses_what_cannot_fit(s7):
    import torch
    ar = torch.empty(s7.queue_table_bytes() + (1 << 20), dtype=torch.uint8, device="cuda")
    q = s7.queue_create(ar)
    try:
        c = [torch.empty(1, dtype=torch.float32, device="cuda") for _ in range(9)]
        with pytest.raises(s7.S7Error) as e:
            s7.queue_submit_2d9(q, 1000, 1000, c, zeros(1), zeros(1), 1e-8, 10)
        assert e.value.code == s7.ENOMEM
        with pytest.raises(s7.S7Error) as e:
            s7.queue_submit_2d9(q, 0, 10, c, zeros(1), zeros(1), 1e-8, 10)
        assert e.value.code == s7.EINVAL
    finally:
        s7.queue_destroy(q)


def test_served_burst_workload(s7):
    """The first 40 requests of the benchmark's 2D request stream (sides log-uniform in
    [64, 1024], 50/50 FP32 at 1e-6 and BF16+IR at 1e-10), submitted at once: all reach
    their manufactured solutions, a sample matches the oracle."""
    import torch
    reqs = synth.serve_stream_2d9(40, seed=0)
    data = []
    for r in reqs:
        nx, ny = r.dims
        n = nx * ny
        c = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(9)]
        xs = torch.empty(n, dtype=torch.float64, device="cuda")
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        s7.generate_problem_2d9(nx, ny, r.seed, c, xs, b)
        data.append((c, b, zeros(n), xs))
    torch.cuda.synchronize()
    prec = {"fp32": s7.FP32, "bf16_ir": s7.BF16_IR}
    out = run_queue(s7, lambda q: [s7.queue_submit_2d9(q, *r.dims, c, b, x, r.rtol, 4000, prec[r.mode])
                                   for r, (c, b, x, xs) in zip(reqs, data)], 4 << 30)
    for r, (c, b, x, xs), (rc, info) in zip(reqs, data, out):
        assert rc == s7.OK, (r, info.as_dict())
        err = float(torch.linalg.vector_norm(x - xs) / torch.linalg.vector_norm(xs))
        assert err <= (1e-3 if r.mode == "fp32" else 1e-8), (r, err)
    for k in (0, 7, 21):
        r = reqs[k]
        p, A, b = problem9(r.dims, r.seed)
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=4000)
        # FP32 at rtol 1e-6 stops near its own tolerance; BF16+IR reaches 1e-10
        assert rel_err(host(data[k][2]), ref.x) <= (5e-4 if r.mode == "fp32" else 1e-8), (k, r.mode)
