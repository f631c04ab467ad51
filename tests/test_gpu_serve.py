"""Serving form: the request loop (afsai_server_*) admits SPD systems of mixed sizes by their
device footprint and overlaps their setups and solves.

Bars: every request's x is bit for bit the x of a separate afsai_setup + pcg_solve with the same
parameters, whether it was served alone or among many, and it is the FP64 oracle's PCG solution
on the oracle's G: the same iteration count and x within 1e-10 relative with G stored in FP64;
with G stored in FP32, converged to the same rtol, iteration count within 2 and x within 1e-6
relative (the bound of the single-solve FP32-G parity test).  At no time do the admitted
requests hold more than the budget or more slots than allowed; a request larger than the budget
is refused; a failing request reports its error without disturbing the others.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

KMAX, S, EPS = 5, 1, 1e-2


@pytest.fixture(scope="module")
def af():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2010_14175_amd as af

    af.lib()
    return af


def _vec(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()


def _requests():
    """Mixed kinds and sizes: 7-point (plain, log-normal, anisotropic; k_max = 5, s = 1) and
    27-point 3-dof (k_max = 10, s = 2): each request carries its own setup parameters."""
    probs = [synth.poisson7(12), synth.elasticity27(6), synth.poisson7(7)]
    probs += synth.aniso_batch(nsys=5, seed=11, side_lo=5, side_hi=14)
    A = synth.lap7_lognormal(9, 8, 10, 1.0, 4)
    probs.append(synth.Problem("lognormal7", A, *synth._rhs(A, 77), KMAX, S))
    return probs


X_RTOL = 1e-10


def _serve(af, probs, budget, slots, g_prec=0, max_heavy=0, heavy_nnz=0):
    srv = af.Server(budget, slots, KMAX, S, EPS, rtol=1e-8, setup_threads=2, g_prec=g_prec, max_heavy=max_heavy,
                    heavy_nnz=heavy_nnz)
    data = []
    for pb in probs:
        dA = af.DeviceCSR.from_host(pb.A)
        b = _vec(pb.b)
        x = _vec(np.full(pb.n, 7.0))  # overwritten by the server
        data.append((dA, b, x, srv.submit(dA, b, x, kmax=pb.kmax, s=pb.s)))
    results = {}
    while len(results) < len(probs):
        for r in srv.poll(wait_ms=1000):
            results[r.ticket] = r
    srv.close()
    return [(x.cpu().numpy(), results[t]) for (_, _, x, t) in data]


def _alone(af, pb):
    dA = af.DeviceCSR.from_host(pb.A)
    P = af.setup(dA, pb.kmax, pb.s, EPS)
    x, info = af.pcg_solve(dA, P, _vec(pb.b), rtol=1e-8)
    return x.cpu().numpy(), info


def test_served_results_equal_separate_solves(af):
    probs = _requests()
    mixed = _serve(af, probs, 1 << 34, 6)
    single = _serve(af, probs, 1 << 34, 1)
    for pb, (xm, rm), (xs, rs) in zip(probs, mixed, single):
        xa, ia = _alone(af, pb)
        assert rm.status == af.OK and rm.converged and rm.iters == ia.iters, pb.name
        assert rs.iters == ia.iters
        assert np.array_equal(xm.view(np.int64), xa.view(np.int64)), f"{pb.name}: mix differs from alone"
        assert np.array_equal(xs.view(np.int64), xa.view(np.int64)), f"{pb.name}: one slot differs from alone"
        assert rm.true_relres == ia.true_relres
        # against the oracle: its setup of the same matrix and its textbook PCG
        ro = oracle.pcg(pb.A, oracle.setup(pb.A, pb.kmax, pb.s, EPS), pb.b, 1e-8)
        assert rm.iters == ro.iters, (pb.name, rm.iters, ro.iters)
        assert np.linalg.norm(xm - ro.x) <= X_RTOL * np.linalg.norm(ro.x), pb.name


def test_served_fp32_g_against_oracle(af):
    """The serving workload's precision form (G stored in FP32, FP64 PCG): every served x in a
    mix of four slots against the oracle's FP64 solution, and bit for bit the x of the same
    request served alone."""
    probs = _requests()
    mixed = _serve(af, probs, 1 << 34, 4, g_prec=af.F32)
    single = _serve(af, probs, 1 << 34, 1, g_prec=af.F32)
    for pb, (xm, rm), (xs, rs) in zip(probs, mixed, single):
        ro = oracle.pcg(pb.A, oracle.setup(pb.A, pb.kmax, pb.s, EPS), pb.b, 1e-8)
        assert rm.status == af.OK and rm.converged and rm.true_relres <= 1.5e-8, pb.name
        assert abs(rm.iters - ro.iters) <= 2, (pb.name, rm.iters, ro.iters)
        assert np.linalg.norm(xm - ro.x) <= 1e-6 * np.linalg.norm(ro.x), pb.name
        assert rs.iters == rm.iters and np.array_equal(xm.view(np.int64), xs.view(np.int64)), pb.name


def test_admission_respects_budget_and_slots(af):
    probs = _requests()
    fps = []
    srv = af.Server(1 << 40, 1, KMAX, S, EPS)
    for pb in probs:  # footprints as the server estimates them
        dA = af.DeviceCSR.from_host(pb.A)
        b, x = _vec(pb.b), _vec(np.zeros(pb.n))
        srv.submit(dA, b, x, kmax=pb.kmax, s=pb.s)
    done = []
    while len(done) < len(probs):
        done += srv.poll(wait_ms=1000)
    srv.close()
    fps = sorted(r.footprint for r in done)
    budget = fps[-1] + fps[-2] - 1  # the two largest never fit together, smaller pairs do
    out = _serve(af, probs, budget, 3)
    res = [r for _, r in out]
    assert all(r.status == af.OK for r in res)
    events = sorted([(r.admit_ms, 1, r) for r in res] + [(r.done_ms, 0, r) for r in res], key=lambda e: (e[0], e[1]))
    held, slots = 0, 0
    for _, kind, r in events:
        held += r.footprint if kind else -r.footprint
        slots += 1 if kind else -1
        assert held <= budget and slots <= 3
    # admission in arrival order, and requests overlapped
    admits = [r.admit_ms for r in res]
    assert admits == sorted(admits)
    assert any(b.admit_ms < a.done_ms for a, b in zip(res, res[1:]))


def test_heavy_requests_one_at_a_time(af):
    """Requests from heavy_nnz entries on are heavy: at most one of them is admitted at any
    instant, they are admitted in arrival order among themselves, lighter ones pass a heavy
    one that waits, and every result is still the one the request gets alone."""
    probs = _requests()
    nnz = sorted(pb.A.nnz for pb in probs)
    heavy_nnz = nnz[len(nnz) // 2]  # the larger half is heavy
    out = _serve(af, probs, 1 << 40, 4, max_heavy=1, heavy_nnz=heavy_nnz)
    res = [r for _, r in out]
    assert all(r.status == af.OK for r in res)
    heavy = [pb.A.nnz >= heavy_nnz for pb in probs]
    events = sorted([(r.admit_ms, 1, h) for r, h in zip(res, heavy)] + [(r.done_ms, 0, h) for r, h in zip(res, heavy)],
                    key=lambda e: (e[0], e[1]))
    held = 0
    for _, kind, h in events:
        if h:
            held += 1 if kind else -1
        assert held <= 1
    hadm = [r.admit_ms for r, h in zip(res, heavy) if h]
    assert hadm == sorted(hadm)
    for (x, r), pb in zip(out, probs):
        xa, ia = _alone(af, pb)
        assert r.iters == ia.iters and np.array_equal(x.view(np.int64), xa.view(np.int64)), pb.name


def test_refuses_oversize_and_isolates_failures(af):
    pb = synth.poisson7(10)
    dA = af.DeviceCSR.from_host(pb.A)
    b, x = _vec(pb.b), _vec(np.zeros(pb.n))
    srv = af.Server(1 << 20, 2, KMAX, S, EPS)
    with pytest.raises(af.AfsaiError) as e:
        srv.submit(dA, b, x)
    assert e.value.code == af.ERR_TOO_LARGE
    srv.close()
    # an indefinite matrix fails its setup; the request beside it is unaffected
    bad = synth.CSR.from_dense(np.diag([1.0, -1.0, 2.0]))
    dB = af.DeviceCSR.from_host(bad)
    bb, xb = _vec([1.0, 1.0, 1.0]), _vec(np.zeros(3))
    srv = af.Server(1 << 34, 4, KMAX, S, EPS)
    tb = srv.submit(dB, bb, xb)
    tg = srv.submit(dA, b, x)
    res = {}
    while len(res) < 2:
        for r in srv.poll(wait_ms=1000):
            res[r.ticket] = r
    srv.close()
    assert res[tb].status == af.ERR_NOT_SPD
    xa, ia = _alone(af, pb)
    assert res[tg].status == af.OK and res[tg].iters == ia.iters
    assert np.array_equal(x.cpu().numpy().view(np.int64), xa.view(np.int64))
