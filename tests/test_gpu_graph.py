"""PCG iterations replayed from captured HIP graphs equal the iterations enqueued kernel by
kernel, bit for bit: the same kernels with the same arguments, captured once per solve (once
per buffer parity in the fused form) and launched once per iteration.

Each case solves several times in a row, with other eager work on the device between the
solves, and compares every solve (iteration count, x, residuals) with the enqueued form; it
covers the fused and separate forms, plain CG, a split SELL layout for A, the batched solver,
the null stream and a stream of its own, and the profiled form (which never uses graphs).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


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


def _bits(t):
    return t.cpu().numpy().view(np.int64)


def _solves(af, dA, P, b, reps=3, stream=None, maxit=None):
    import torch

    out = []
    r = _vec(synth.uniform(9, 1, dA.n))
    for k in range(reps):
        x = torch.zeros_like(b)
        if stream is not None:
            stream.wait_stream(torch.cuda.current_stream())
        x, info = af.pcg_solve(dA, P, b, x=x, stream=stream, maxit=maxit, raise_on_error=False)
        # eager work between the solves: a preconditioner application and a torch reduction
        if P is not None:
            P.apply(r, stream=stream)
        float((x * x).sum())
        torch.cuda.synchronize()
        out.append((x.clone(), info))
    return out


def _with(af, value, fn):
    try:
        af.set_option(af.OPT_PCG_GRAPH, value)
        return fn()
    finally:
        af.set_option(af.OPT_PCG_GRAPH, 0)


def _eager(af, fn):
    return _with(af, 1, fn)


def _graph(af, fn):
    return _with(af, 2, fn)


def _same(a, b):
    for (xa, ia), (xb, ib) in zip(a, b):
        assert ia.iters == ib.iters and ia.status == ib.status
        assert np.array_equal(_bits(xa), _bits(xb))
        assert ia.relres == ib.relres and ia.true_relres == ib.true_relres


@pytest.mark.parametrize("form", [0, 1, 2])
@pytest.mark.parametrize("make", [lambda: synth.elasticity27(8), lambda: synth.poisson7(9)])
def test_graph_equals_enqueued(af, form, make):
    """form 0: automatic (fused here), 1: separate updates, 2: fused; poisson7(9) gets a split
    SELL layout for A, which forces the separate form."""
    Pb = make()
    dA = af.DeviceCSR.from_host(Pb.A)
    P = af.setup(dA, 8, 2, 1e-2)
    b = _vec(Pb.b)
    try:
        af.set_option(af.OPT_PCG_FORM, form)
        g = _graph(af, lambda: _solves(af, dA, P, b))
        e = _eager(af, lambda: _solves(af, dA, P, b))
        a = _solves(af, dA, P, b)
    finally:
        af.set_option(af.OPT_PCG_FORM, 0)
    assert g[0][1].converged
    _same(g, e)
    _same(g, a)
    _same(g[1:], g[:-1])


def test_graph_plain_cg_and_maxit(af):
    Pb = synth.poisson7(10)
    dA = af.DeviceCSR.from_host(Pb.A)
    b = _vec(Pb.b)
    _same(_graph(af, lambda: _solves(af, dA, None, b)), _eager(af, lambda: _solves(af, dA, None, b)))
    P = af.setup(dA, 5, 1, 1e-2)
    g = _graph(af, lambda: _solves(af, dA, P, b, maxit=7))
    assert g[0][1].iters == 7 and g[0][1].status == af.ERR_NOT_CONVERGED
    _same(g, _eager(af, lambda: _solves(af, dA, P, b, maxit=7)))


def test_graph_on_own_stream(af):
    import torch

    Pb = synth.elasticity27(7)
    dA = af.DeviceCSR.from_host(Pb.A)
    P = af.setup(dA, 6, 2, 1e-2)
    b = _vec(Pb.b)
    s = torch.cuda.Stream()
    g = _graph(af, lambda: _solves(af, dA, P, b, stream=s))
    _same(g, _eager(af, lambda: _solves(af, dA, P, b)))


def test_graph_batched(af):
    probs = synth.aniso_batch(nsys=6, seed=4, side_lo=3, side_hi=12)
    A, off, b, _ = synth.block_diag(probs)
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 5, 1, 1e-2)
    bv = _vec(b)

    def run():
        res = []
        for _ in range(2):
            x, infos = af.pcg_solve_batched(dA, P, off, bv, rtol=1e-8)
            res.append((x.clone(), [i.iters for i in infos]))
        return res

    g, e = _graph(af, run), _eager(af, run)
    for (xg, ig), (xe, ie) in zip(g, e):
        assert ig == ie
        assert np.array_equal(_bits(xg), _bits(xe))


def test_profiled_solve_equals_graph(af):
    """The kernel timer switches graphs off; the iterates do not change."""
    Pb = synth.elasticity27(7)
    dA = af.DeviceCSR.from_host(Pb.A)
    P = af.setup(dA, 6, 2, 1e-2)
    b = _vec(Pb.b)
    g = _graph(af, lambda: _solves(af, dA, P, b, reps=1))
    af.profile_read(reset=True)
    af.profile_enable(True)
    try:
        p = _graph(af, lambda: _solves(af, dA, P, b, reps=1))
        times = af.profile_read(reset=True)
    finally:
        af.profile_enable(False)
    _same(g, p)
    # every iteration's products were timed one by one
    assert times["spmv_GT_dot"][0] >= p[0][1].iters
