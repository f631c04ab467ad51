"""afsai_apply_noalloc (the entry point that allocates nothing) against afsai_apply.

Both run the same two products (t = G r, z = G^T t) with the same kernels and launch shapes;
only the home of the intermediate t differs (a fixed device array of the library instead of
the handle's workspace), so z must agree bit for bit.  Two handles are used in a row, the
second smaller than the first, so the shared array holds the first call's values when the
second one runs.  Every call goes through the C ABI (ctypes).
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


def _case(af, pb, g_prec, seed):
    import torch

    dA = af.DeviceCSR.from_host(pb.A)
    P = af.setup(dA, pb.kmax, pb.s, pb.eps, g_prec=g_prec)
    r = torch.from_numpy(synth.uniform(seed, 4, pb.n)).cuda()
    z_ref = P.apply(r)
    z = torch.full_like(r, float("nan"))
    P.apply_noalloc(r, z)
    torch.cuda.synchronize()
    return P, r, z_ref.cpu().numpy(), z.cpu().numpy()


def test_noalloc_equals_apply_two_calls(af):
    import torch

    print("[no_alloc] 27-point 24^3 (41,472 rows, FP64 G), then 7-point 9^3 (729 rows, FP32 G)", flush=True)
    big = synth.elasticity27(24, 1.0, 2, kmax=10, s=2)
    P1, r1, z1_ref, z1 = _case(af, big, af.F64, 11)
    assert np.array_equal(z1, z1_ref), "first call differs from afsai_apply"
    small = synth.poisson7(9)
    P2, r2, z2_ref, z2 = _case(af, small, af.F32, 12)
    assert np.array_equal(z2, z2_ref), "second (smaller) call differs from afsai_apply"
    # the result is the preconditioner application of the oracle's definition (eq. prec)
    rp, ci, va = (t.cpu().numpy() for t in P2.export())
    Go = oracle.Factor(rp, ci, va, None)
    zo = oracle.apply(Go, r2.cpu().numpy())
    np.testing.assert_allclose(z2, zo, rtol=1e-12, atol=1e-13 * np.abs(zo).max())
    # a third call on the first handle again gives its first result
    z3 = torch.full_like(r1, float("nan"))
    P1.apply_noalloc(r1, z3)
    torch.cuda.synchronize()
    assert np.array_equal(z3.cpu().numpy(), z1_ref)
    P1.close()
    P2.close()


def test_noalloc_rejects_bad_arguments(af):
    import ctypes

    pb = synth.poisson7(6)
    dA = af.DeviceCSR.from_host(pb.A)
    P = af.setup(dA, pb.kmax, pb.s, pb.eps)
    import torch

    r = torch.from_numpy(synth.uniform(1, 4, pb.n)).cuda()
    rc = af.lib().afsai_apply_noalloc(P.handle, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(r.data_ptr()), None)
    assert rc == af.ERR_INVALID_ARG
    rc = af.lib().afsai_apply_noalloc(None, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(r.data_ptr()), None)
    assert rc == af.ERR_INVALID_ARG
    P.close()
