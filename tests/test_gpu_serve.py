"""GPU tests of the request queue (continuous batching over the batch engine).

Results are checked against the FP64 oracle.  A request's result must not
depend on what else is resident: its sums run in a fixed per-system order and
its Krylov state stays on the device across epochs, so served in a mix it comes
out bit for bit as the batched entry point computes it alone."""
import numpy as np
import pytest

import oracle
from tests.conftest import gpu_available
from tests.gpu_helpers import coef_dev, dev, host, problem, rel_err

pytestmark = pytest.mark.gpu

MIX = [((24, 32, 48), 0), ((17, 5, 9), 1), ((40, 24, 20), 0), ((33, 17, 9), 1), ((2, 1, 1), 0),
       ((31, 29, 27), 1), ((64, 24, 32), 0), ((9, 7, 5), 1)]  # (dims, prec)
RTOL = {0: 1e-8, 1: 1e-10}


@pytest.fixture(scope="module")
def s7():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2010_03660_amd as s7
    s7.lib()
    return s7


def arena(s7, nbytes):
    import torch
    return torch.empty(s7.queue_table_bytes() + nbytes, dtype=torch.uint8, device="cuda")


def inputs(probs):
    import torch
    coefs = [coef_dev(p) for p, A, b in probs]
    bs = [dev(b) for p, A, b in probs]
    xs = [torch.zeros(A.n, dtype=torch.float64, device="cuda") for p, A, b in probs]
    torch.cuda.synchronize()
    return coefs, bs, xs


def serve(s7, reqs, arena_bytes, epoch=0, chunk=0):
    """Submits every request, then collects them all.  reqs: (dims, coef, b, x, rtol, max_iter, prec)."""
    ar = arena(s7, arena_bytes)
    q = s7.queue_create(ar, opt=s7.default_options(graph_iters=epoch, chunk_cells=chunk))
    try:
        tickets = [s7.queue_submit(q, *r) for r in reqs]
        out = [s7.queue_wait(q, t) for t in tickets]
    finally:
        s7.queue_destroy(q)
    return out


def test_served_mix_matches_oracle(s7):
    probs = [problem(d, seed=300 + i) for i, (d, p) in enumerate(MIX)]
    coefs, bs, xs = inputs(probs)
    reqs = [(d, coefs[i], bs[i], xs[i], RTOL[p], 2000, p) for i, (d, p) in enumerate(MIX)]
    out = serve(s7, reqs, 64 << 20)
    for i, ((d, prec), (p, A, b), (rc, info)) in enumerate(zip(MIX, probs, out)):
        assert rc == s7.OK and info.status == s7.OK, (i, info.as_dict())
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        x = host(xs[i])
        assert rel_err(x, ref.x) <= (1e-6 if prec == 0 else 1e-7), i
        if prec == 0:  # the recurrence reaches rtol; the true residual sits at the FP32 floor
            assert info.rel_res_rec <= RTOL[prec] and info.rel_res_true <= 1e-6
        else:
            assert info.rel_res_true <= RTOL[prec]
        assert abs(info.rel_res_true - oracle.true_rel_residual(A, b, x)) <= 1e-3 * info.rel_res_true + 1e-15
        assert info.t_ms >= info.t_wait_ms >= 0.0
        assert info.outer_iters == 1 if prec == 0 else info.outer_iters > 1


@pytest.mark.parametrize("epoch", [0, 1, 5, 16])
def test_served_equals_alone_bitwise(s7, epoch):
    """Served in a mix, with time slices (epoch 0, the default) or epochs of 1, 5
    or 16 iterations and admission delayed by a tight arena, each request matches
    the batched entry point run on that request alone (one epoch for the whole
    solve).  The queue sizes its work items by load (its chunks shrink as the
    resident set drains) and the alone run uses the default chunks: the sums are
    kept per 1024-cell unit, so the results still agree bit for bit."""
    import torch
    probs = [problem(d, seed=400 + i) for i, (d, p) in enumerate(MIX)]
    coefs, bs, xs = inputs(probs)
    reqs = [(d, coefs[i], bs[i], xs[i], RTOL[p], 2000, p) for i, (d, p) in enumerate(MIX)]
    # room for about three of the larger requests at a time
    big = max(s7.workspace_bytes(d, p) for d, p in MIX)
    out = serve(s7, reqs, 3 * big + (1 << 20), epoch=epoch)
    waited = 0
    for i, ((d, prec), (rc, info)) in enumerate(zip(MIX, out)):
        x1 = torch.zeros_like(xs[i])
        rc1, inf1 = s7.bicgstab_solve_batched([d], [coefs[i]], [bs[i]], [x1], [RTOL[prec]], [2000],
                                              prec=prec, opt=s7.default_options(chunk_cells=16384))
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), host(xs[i])), i
        assert inf1[0].iters == info.iters and inf1[0].status == info.status, i
        assert inf1[0].outer_iters == info.outer_iters, i
        waited += info.t_wait_ms > 0.0
    assert waited >= 1


def test_poll_semantics(s7):
    """EAGAIN while running; the status once done; the ticket is released on
    collection; unknown tickets are ENOTFOUND."""
    import torch
    d = (64, 64, 64)
    p, A, b = problem(d, seed=9)
    coefs, bs, xs = inputs([(p, A, b)])
    ar = arena(s7, 2 * s7.workspace_bytes(d, 0))
    q = s7.queue_create(ar)
    try:
        t = s7.queue_submit(q, d, coefs[0], bs[0], xs[0], 1e-300, 1500, 0)
        rc, _ = s7.queue_poll(q, t)
        assert rc == s7.EAGAIN
        rc, info = s7.queue_wait(q, t)
        assert rc == s7.NOT_CONVERGED and info.iters == 1500
        with pytest.raises(s7.S7Error) as e:
            s7.queue_poll(q, t)
        assert e.value.code == s7.ENOTFOUND
        with pytest.raises(s7.S7Error) as e:
            s7.queue_wait(q, t + 100)
        assert e.value.code == s7.ENOTFOUND
        # a short request after the long one: poll until done
        t2 = s7.queue_submit(q, d, coefs[0], bs[0], xs[0], 1e-6, 1500, 0)
        for _ in range(200000):
            rc, info = s7.queue_poll(q, t2)
            if rc != s7.EAGAIN:
                break
        assert rc == s7.OK and info.status == s7.OK
        assert info.rel_res_true <= 1.5e-6
    finally:
        s7.queue_destroy(q)
    torch.cuda.synchronize()


def test_admission_by_footprint(s7):
    """An arena that holds one request at a time serves them one after
    another in submission order; a request larger than the arena is refused."""
    import torch
    shapes = [(32, 32, 32), (32, 24, 40), (40, 32, 24)]  # any two exceed the arena
    probs = [problem(d, seed=500 + i) for i, d in enumerate(shapes)]
    coefs, bs, xs = inputs(probs)
    need = max(s7.workspace_bytes(d, 0) for d in shapes)
    ar = arena(s7, need)
    q = s7.queue_create(ar)
    try:
        with pytest.raises(s7.S7Error) as e:
            s7.queue_submit(q, (64, 64, 64), coefs[0], bs[0], xs[0], 1e-8, 100, 0)
        assert e.value.code == s7.ENOMEM
        tickets = [s7.queue_submit(q, d, coefs[i], bs[i], xs[i], 1e-8, 2000, 0) for i, d in enumerate(shapes)]
        out = [s7.queue_wait(q, t) for t in tickets]
    finally:
        s7.queue_destroy(q)
    for i, ((p, A, b), (rc, info)) in enumerate(zip(probs, out)):
        assert rc == s7.OK
        ref = oracle.bicgstab(A, b, tol=1e-12, max_iter=2000)
        assert rel_err(host(xs[i]), ref.x) <= 1e-6
    # one at a time: each later request waited while the one before it ran
    run = [info.t_ms - info.t_wait_ms for rc, info in out]
    assert out[1][1].t_wait_ms >= out[0][1].t_wait_ms + run[0] - 1.0
    assert out[2][1].t_wait_ms >= out[1][1].t_wait_ms + run[1] - 1.0


def test_destroy_drains(s7):
    """Destroy finishes what was submitted, collected or not."""
    import torch
    shapes = [(20, 20, 20), (33, 17, 9), (12, 30, 7)]
    probs = [problem(d, seed=600 + i) for i, d in enumerate(shapes)]
    coefs, bs, xs = inputs(probs)
    ar = arena(s7, 16 << 20)
    q = s7.queue_create(ar)
    for i, d in enumerate(shapes):
        s7.queue_submit(q, d, coefs[i], bs[i], xs[i], 1e-10, 2000, 1)
    s7.queue_destroy(q)
    torch.cuda.synchronize()
    for i, (p, A, b) in enumerate(probs):
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert rel_err(host(xs[i]), ref.x) <= 1e-7


def test_served_degenerate_requests(s7):
    """A zero right-hand side (x = 0 exactly) and an exact breakdown, served
    among regular requests, with FP32 and BF16 refinement."""
    import torch
    d0 = (9, 7, 5)
    p0, A0, b0 = problem(d0, seed=2)
    coef_bd = [np.zeros(2, np.float32) for _ in range(7)]
    coef_bd[2][0] = 1.0
    coef_bd[1][1] = -1.0
    d2 = (33, 17, 9)
    p2, A2, b2 = problem(d2, seed=3)
    c0, cbd, c2 = coef_dev(p0), [dev(c) for c in coef_bd], coef_dev(p2)
    z = dev(np.zeros(A0.n))
    xs = [torch.ones(A0.n, dtype=torch.float64, device="cuda"),
          torch.ones(A0.n, dtype=torch.float64, device="cuda"),
          torch.zeros(2, dtype=torch.float64, device="cuda"),
          torch.zeros(A2.n, dtype=torch.float64, device="cuda")]
    bbd, bb2 = dev(np.array([1.0, 0.0])), dev(b2)
    torch.cuda.synchronize()
    ar = arena(s7, 16 << 20)
    q = s7.queue_create(ar, opt=s7.default_options(jacobi=0))
    try:
        ts = [s7.queue_submit(q, d0, c0, z, xs[0], 1e-8, 100, 0),
              s7.queue_submit(q, d0, c0, z, xs[1], 1e-8, 100, 1),
              s7.queue_submit(q, (2, 1, 1), cbd, bbd, xs[2], 1e-8, 100, 0),
              s7.queue_submit(q, d2, c2, bb2, xs[3], 1e-8, 1000, 0)]
        out = [s7.queue_wait(q, t) for t in ts]
    finally:
        s7.queue_destroy(q)
    assert out[0][0] == s7.OK and np.all(host(xs[0]) == 0)
    assert out[1][0] == s7.OK and np.all(host(xs[1]) == 0)
    assert out[2][0] == s7.BREAKDOWN and out[2][1].reason == s7.REASON_RS_ZERO
    assert out[3][0] == s7.OK
    ref = oracle.bicgstab(A2, b2, tol=1e-12, max_iter=1000, jacobi_scaling=False)
    assert rel_err(host(xs[3]), ref.x) <= 1e-6


def test_large_requests_take_the_single_system_path(s7):
    """With split_cells = 20000, requests of at least that many cells run on the
    single-system path beside the batch engine: each result equals that path's result
    alone (bit for bit), the small ones equal the batched path alone, and all match the
    oracle."""
    import torch
    probs = [problem(d, seed=700 + i) for i, (d, p) in enumerate(MIX)]
    coefs, bs, xs = inputs(probs)
    reqs = [(d, coefs[i], bs[i], xs[i], RTOL[p], 2000, p) for i, (d, p) in enumerate(MIX)]
    ar = arena(s7, 64 << 20)
    q = s7.queue_create(ar, opt=s7.default_options(split_cells=20000))
    try:
        out = [s7.queue_wait(q, s7.queue_submit(q, *r)) for r in reqs[:1]]  # one alone first
        out += [s7.queue_wait(q, t) for t in [s7.queue_submit(q, *r) for r in reqs[1:]]]
    finally:
        s7.queue_destroy(q)
    big = 0
    for i, ((d, prec), (p, A, b), (rc, info)) in enumerate(zip(MIX, probs, out)):
        assert rc == s7.OK, (i, info.as_dict())
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert rel_err(host(xs[i]), ref.x) <= (1e-6 if prec == 0 else 1e-7), i
        x1 = torch.zeros_like(xs[i])
        if int(np.prod(d)) >= 20000:
            big += 1
            i1 = s7.bicgstab_solve(d, coefs[i], bs[i], x1, RTOL[prec], 2000, prec=prec)
        else:
            rc1, inf1 = s7.bicgstab_solve_batched([d], [coefs[i]], [bs[i]], [x1], [RTOL[prec]], [2000],
                                                  prec=prec)
            i1 = inf1[0]
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), host(xs[i])), i
        assert i1.iters == info.iters, i
    assert big >= 3


def test_three_precisions_resident_together(s7):
    """FP32, BF16+IR and FP16+IR requests share the persistent launches: each result
    reaches the oracle's solution and equals the same request solved alone."""
    import torch
    mix = [((24, 32, 20), 0), ((17, 13, 9), 2), ((40, 24, 20), 1), ((33, 17, 9), 2), ((9, 7, 5), 0),
           ((31, 29, 27), 2)]
    rtol = {0: 1e-8, 1: 1e-10, 2: 1e-10}
    probs = [problem(d, seed=700 + i) for i, (d, p) in enumerate(mix)]
    coefs, bs, xs = inputs(probs)
    reqs = [(d, coefs[i], bs[i], xs[i], rtol[p], 2000, p) for i, (d, p) in enumerate(mix)]
    out = serve(s7, reqs, 64 << 20, chunk=1024)
    for i, ((d, prec), (p, A, b), (rc, info)) in enumerate(zip(mix, probs, out)):
        assert rc == s7.OK and info.status == s7.OK, (i, info.as_dict())
        ref = oracle.bicgstab(A, b, tol=1e-13, max_iter=2000)
        assert rel_err(host(xs[i]), ref.x) <= (1e-6 if prec == 0 else 1e-7), i
        x1 = torch.zeros_like(xs[i])
        rc1, inf1 = s7.bicgstab_solve_batched([d], [coefs[i]], [bs[i]], [x1], [rtol[prec]], [2000], prec=prec,
                                              opt=s7.default_options(chunk_cells=1024))
        torch.cuda.synchronize()
        assert np.array_equal(host(x1), host(xs[i])) and inf1[0].iters == info.iters, i
