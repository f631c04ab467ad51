"""Batching form: many independent SPD systems set up and solved together through
afsai_setup_batched / pcg_solve_batched.

Bars: each system's G is the one a separate afsai_setup of that system gives, bit for bit, and
the oracle's on the block-diagonal matrix (patterns identical, values within 1e-10 relative per
row); each system's PCG iterates equal those of a separate pcg_solve (iteration count and
x bit for bit), for preconditioned and plain CG, including systems that stop early, zero
right-hand sides and systems that hit maxit.
"""
import numpy as np
import pytest

import oracle
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


def _factor(P):
    rp, ci, va = P.export()
    return rp.cpu().numpy(), ci.cpu().numpy(), va.cpu().numpy()


def _batch(nsys, lo, hi, seed=3, kmax=5, s=1):
    probs = synth.aniso_batch(nsys=nsys, seed=seed, side_lo=lo, side_hi=hi, kmax=kmax, s=s)
    A, off, b, x = synth.block_diag(probs)
    return probs, A, off, b, x


@pytest.mark.parametrize("nsys,lo,hi", [(9, 2, 7), (6, 8, 16)])
def test_batched_setup_equals_standalone_and_oracle(af, nsys, lo, hi):
    probs, A, off, b, _ = _batch(nsys, lo, hi)
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 5, 1, 1e-2)
    rp, ci, va = _factor(P)
    # per system: a separate setup of the system alone
    for k, pb in enumerate(probs):
        Pk = af.setup(af.DeviceCSR.from_host(pb.A), 5, 1, 1e-2)
        rk, ck, vk = _factor(Pk)
        o = off[k]
        a0, a1 = rp[o], rp[off[k + 1]]
        np.testing.assert_array_equal(rp[o:off[k + 1] + 1] - a0, rk)
        np.testing.assert_array_equal(ci[a0:a1] - o, ck)
        assert np.array_equal(va[a0:a1].view(np.int64), vk.view(np.int64)), f"system {k}: values differ"
    # the oracle on the block-diagonal matrix
    G = oracle.setup(A, 5, 1, 1e-2)
    np.testing.assert_array_equal(G.row_ptr, rp)
    np.testing.assert_array_equal(G.col, ci)
    row = np.repeat(np.arange(A.n), np.diff(rp))
    scale = np.maximum.reduceat(np.abs(G.val), rp[:-1])[row]
    assert np.all(np.abs(va - G.val) <= 1e-10 * scale)


@pytest.mark.parametrize("precond", [True, False])
def test_batched_pcg_equals_standalone(af, precond):
    """Systems of 8 .. 4,096 rows (several SELL slices and vector blocks each)."""
    probs, A, off, b, _ = _batch(7, 2, 16)
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 5, 1, 1e-2) if precond else None
    x, infos = af.pcg_solve_batched(dA, P, off, _vec(b), rtol=1e-8)
    xh = x.cpu().numpy()
    for k, pb in enumerate(probs):
        dk = af.DeviceCSR.from_host(pb.A)
        Pk = af.setup(dk, 5, 1, 1e-2) if precond else None
        xk, ik = af.pcg_solve(dk, Pk, _vec(pb.b), rtol=1e-8)
        assert infos[k].iters == ik.iters, f"system {k}: {infos[k].iters} vs {ik.iters} iterations"
        assert infos[k].converged and ik.converged
        assert np.array_equal(xh[off[k]:off[k + 1]].view(np.int64), xk.cpu().numpy().view(np.int64)), k
        assert infos[k].true_relres == pytest.approx(ik.true_relres, rel=1e-12, abs=1e-30)


def test_batched_apply_equals_standalone(af):
    """z = G^T (G r) with a batched preconditioner (the whole batch as one launch, its G^T
    windows aligned at every system's first slice) equals each system's own preconditioner
    applied to its share of r, bit for bit, and the oracle's G^T (G r) within 1e-10."""
    probs, A, off, b, _ = _batch(7, 2, 16)
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 5, 1, 1e-2)
    r = synth.uniform(11, 4, A.n, -1.0, 1.0)
    z = P.apply(_vec(r)).cpu().numpy()
    for k, pb in enumerate(probs):
        Pk = af.setup(af.DeviceCSR.from_host(pb.A), 5, 1, 1e-2)
        zk = Pk.apply(_vec(r[off[k]:off[k + 1]])).cpu().numpy()
        assert np.array_equal(z[off[k]:off[k + 1]].view(np.int64), zk.view(np.int64)), k
    G = oracle.setup(A, 5, 1, 1e-2).to_scipy()
    zo = G.T @ (G @ r)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)


def test_batched_setup_wide_rows(af):
    """Batches of 27-point 3-dof systems (rows of up to 81 entries): the candidate tables are
    sized from the longest row of the batch, so every system's G equals its separate setup
    bit for bit (the batch check once overwrote that length, and such batches overflowed)."""
    probs = [synth.elasticity27(N, sigma=2.0, seed=40 + N) for N in (5, 7, 9, 11)]
    A, off, _, _ = synth.block_diag(probs)
    P = af.setup_batched(af.DeviceCSR.from_host(A), off, 10, 2, 1e-2)
    rp, ci, va = _factor(P)
    for k, pb in enumerate(probs):
        rk, ck, vk = _factor(af.setup(af.DeviceCSR.from_host(pb.A), 10, 2, 1e-2))
        lo, hi = rp[off[k]], rp[off[k + 1]]
        assert np.array_equal(rp[off[k]:off[k + 1] + 1] - lo, rk), k
        assert np.array_equal(ci[lo:hi] - off[k], ck), k
        assert np.array_equal(va[lo:hi].view(np.int64), vk.view(np.int64)), k


def test_batched_column_runs(af):
    """A batch of 3-dof systems (375 .. 3,993 rows, slices starting at every system's first row,
    ragged last slices) in the separate-update form multiplies with A's column-run layout: each
    system's iterates equal its separate solve and the per-entry layout's bit for bit."""
    import torch

    probs = [synth.elasticity27(N, sigma=2.0, seed=40 + N) for N in (5, 7, 9, 11)]
    A, off, b, _ = synth.block_diag(probs)
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 10, 2, 1e-2)
    af.set_option(af.OPT_PCG_FORM, 1)
    try:
        x, infos = af.pcg_solve_batched(dA, P, off, _vec(b), rtol=1e-8)
        af.set_option(af.OPT_SELL_RUNS, 1)
        xe, infe = af.pcg_solve_batched(dA, P, off, _vec(b), rtol=1e-8)
        af.set_option(af.OPT_SELL_RUNS, 0)
        xh = x.cpu().numpy()
        assert torch.equal(x, xe)
        for k, pb in enumerate(probs):
            assert infos[k].iters == infe[k].iters and infos[k].converged
            dk = af.DeviceCSR.from_host(pb.A)
            Pk = af.setup(dk, 10, 2, 1e-2)
            xk, ik = af.pcg_solve(dk, Pk, _vec(pb.b), rtol=1e-8)
            assert infos[k].iters == ik.iters, (k, infos[k].iters, ik.iters)
            assert np.array_equal(xh[off[k]:off[k + 1]].view(np.int64), xk.cpu().numpy().view(np.int64)), k
    finally:
        af.set_option(af.OPT_SELL_RUNS, 0)
        af.set_option(af.OPT_PCG_FORM, 0)


def test_batched_pcg_against_oracle(af):
    probs, A, off, b, _ = _batch(5, 3, 9)
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 5, 1, 1e-2)
    x, infos = af.pcg_solve_batched(dA, P, off, _vec(b), rtol=1e-8)
    xh = x.cpu().numpy()
    for k, pb in enumerate(probs):
        G = oracle.setup(pb.A, 5, 1, 1e-2)
        res = oracle.pcg(pb.A, G, pb.b, 1e-8)
        assert infos[k].iters == res.iters
        xo = res.x
        assert np.linalg.norm(xh[off[k]:off[k + 1]] - xo) <= 1e-10 * np.linalg.norm(xo)


def test_batched_mixed_stops(af):
    """One zero right-hand side (x = 0, no iteration), one system far harder than the others,
    and a maxit that stops only the hard one: every other system is still exact."""
    probs = synth.aniso_batch(nsys=4, seed=5, side_lo=4, side_hi=6)
    hard = synth.poisson7(12)
    probs.append(hard)
    A, off, b, _ = synth.block_diag(probs)
    b = b.copy()
    b[off[1]:off[2]] = 0.0  # system 1: zero right-hand side
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 5, 1, 1e-2)
    solo = []
    for k, pb in enumerate(probs):
        dk = af.DeviceCSR.from_host(pb.A)
        Pk = af.setup(dk, 5, 1, 1e-2)
        xk, ik = af.pcg_solve(dk, Pk, _vec(b[off[k]:off[k + 1]]), rtol=1e-8, raise_on_error=False)
        solo.append((xk.cpu().numpy(), ik))
    maxit = max(i.iters for _, i in solo[:-1]) + 1
    assert solo[-1][1].iters > maxit
    x, infos = af.pcg_solve_batched(dA, P, off, _vec(b), rtol=1e-8, maxit=maxit, raise_on_error=False)
    xh = x.cpu().numpy()
    assert infos[0].status == af.ERR_NOT_CONVERGED
    assert infos[1].iters == 0 and infos[1].converged and not xh[off[1]:off[2]].any()
    assert infos[-1].iters == maxit and not infos[-1].converged
    for k in (0, 2, 3):
        assert infos[k].converged and infos[k].iters == solo[k][1].iters
        assert np.array_equal(xh[off[k]:off[k + 1]].view(np.int64), solo[k][0].view(np.int64))


def test_batched_errors(af):
    probs, A, off, b, _ = _batch(3, 3, 5)
    dA = af.DeviceCSR.from_host(A)
    with pytest.raises(af.AfsaiError):
        af.setup_batched(dA, [0, 10, 5, A.n], 5, 1, 1e-2)  # offsets decrease
    with pytest.raises(af.AfsaiError):
        af.setup_batched(dA, [0, A.n - 1], 5, 1, 1e-2)  # does not end at n
    # a coupling entry between systems 0 and 1
    d = A.to_scipy().tolil()
    i, j = int(off[1]) - 1, int(off[1])
    d[i, j] = d[j, i] = -0.01
    coupled = synth.CSR.from_scipy(d.tocsr())
    with pytest.raises(af.AfsaiError) as e:
        af.setup_batched(af.DeviceCSR.from_host(coupled), off, 5, 1, 1e-2)
    assert e.value.code == af.ERR_BAD_MATRIX
    P = af.setup_batched(dA, off, 5, 1, 1e-2)
    with pytest.raises(af.AfsaiError):
        af.pcg_solve(dA, P, _vec(b))  # a batch handle needs the batched solver
    with pytest.raises(af.AfsaiError):
        af.pcg_solve_batched(dA, P, [0, int(off[2]), A.n], _vec(b))  # other offsets


def test_full_batch512_against_oracle(af):
    """The full batched workload: 512 anisotropic 7-point systems (sides U{10..40}, 7,788,665
    rows), one batched setup and one batched solve, in the launch configuration of the batched
    benchmark.  Every row of G against the oracle's setup of the block-diagonal matrix (patterns
    identical, values within 1e-10), and every system's PCG against the oracle's PCG on that
    system with the oracle's G: the same iteration count and x within 1e-10."""
    probs, A, off, b, _ = _batch(512, 10, 40, seed=3)
    assert A.n == 7788665
    dA = af.DeviceCSR.from_host(A)
    P = af.setup_batched(dA, off, 5, 1, 1e-2)
    x, infos = af.pcg_solve_batched(dA, P, off, _vec(b), rtol=1e-8)
    xh = x.cpu().numpy()
    rp, ci, va = _factor(P)
    G = oracle.setup(A, 5, 1, 1e-2)
    np.testing.assert_array_equal(G.row_ptr, rp)
    np.testing.assert_array_equal(G.col, ci)
    # per-row relative error (infinity norm); every row has at least its diagonal entry
    dmax = np.maximum.reduceat(np.abs(va - G.val), G.row_ptr[:-1])
    vmax = np.maximum.reduceat(np.abs(G.val), G.row_ptr[:-1])
    assert np.max(dmax / vmax) <= 1e-10
    for k, pb in enumerate(probs):
        o0, o1 = int(off[k]), int(off[k + 1])
        a0, a1 = int(G.row_ptr[o0]), int(G.row_ptr[o1])
        Gk = oracle.Factor((G.row_ptr[o0:o1 + 1] - a0).astype(np.int32), (G.col[a0:a1] - o0).astype(np.int32),
                           G.val[a0:a1], None)
        ro = oracle.pcg(pb.A, Gk, pb.b, 1e-8)
        assert infos[k].converged and infos[k].iters == ro.iters, (k, infos[k].iters, ro.iters)
        assert np.linalg.norm(xh[o0:o1] - ro.x) <= 1e-10 * np.linalg.norm(ro.x), k
