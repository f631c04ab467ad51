"""The autotuner (paper_2010_14175_amd.tune): its choices are cached by shape and leave the
results unchanged -- the setup's G bit for bit, the PCG iteration count equal and x bit for
bit (within 1e-10 when the choice changes the layout of G^T, whose fused dot products are then
summed in another order)."""
import json

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


def _factor(P):
    return [t.cpu().numpy() for t in P.export()]


def _check_same(af, tune, dA, kmax, s, b, choice, offsets=None):
    def run():
        if offsets is None:
            P = af.setup(dA, kmax, s, 1e-2)
            x, info = af.pcg_solve(dA, P, b, rtol=1e-8)
            infos = [info]
        else:
            P = af.setup_batched(dA, offsets, kmax, s, 1e-2)
            x, infos = af.pcg_solve_batched(dA, P, offsets, b, rtol=1e-8)
        g = _factor(P)
        P.close()
        return g, x.cpu().numpy(), [i.iters for i in infos]

    g0, x0, it0 = run()
    with tune.apply(choice):
        g1, x1, it1 = run()
    for a, c in zip(g0, g1):
        np.testing.assert_array_equal(a, c)
    assert it0 == it1, (it0, it1)
    if choice["pcg"].get("gt_layout"):
        assert np.linalg.norm(x1 - x0) <= 1e-10 * np.linalg.norm(x0)
    else:
        assert np.array_equal(x0.view(np.int64), x1.view(np.int64))


def test_tune_single_system(af, tmp_path):
    import torch

    from paper_2010_14175_amd import tune

    pb = synth.elasticity27(10, 1.0, 2, kmax=10, s=2)
    dA = af.DeviceCSR.from_host(pb.A)
    b = torch.from_numpy(pb.b).cuda()
    cache = str(tmp_path / "tune.json")
    choice = tune.autotune(dA, pb.kmax, pb.s, pb.eps, b, reps=1, cache=cache)
    print(f"[tune] {choice}", flush=True)
    assert set(choice) >= {"key", "setup", "pcg", "setup_ms", "pcg_ms"}
    assert choice["setup_ms"] <= choice["default_setup_ms"] and choice["pcg_ms"] <= choice["default_pcg_ms"]
    with open(cache) as fh:
        assert json.load(fh)[choice["key"]] == choice
    assert tune.autotune(dA, pb.kmax, pb.s, pb.eps, b, reps=1, cache=cache) == choice  # from the cache
    _check_same(af, tune, dA, pb.kmax, pb.s, b, choice)
    # every candidate knob on its own gives the same results too
    for c in ({"setup": {"lanes": 64, "table": 1024, "claim": 1}, "pcg": {"pcg_form": 1, "pcg_graph": 2}},
              {"setup": {"claim": 32}, "pcg": {"pcg_form": 2, "gt_layout": 1}}):
        _check_same(af, tune, dA, pb.kmax, pb.s, b, c)


def test_tune_batch(af, tmp_path):
    import torch

    from paper_2010_14175_amd import tune

    probs = synth.aniso_batch(nsys=6, seed=3, side_lo=6, side_hi=14, kmax=5, s=1)
    A, off, bh, _ = synth.block_diag(probs)
    dA = af.DeviceCSR.from_host(A)
    b = torch.from_numpy(bh).cuda()
    choice = tune.autotune(dA, 5, 1, 1e-2, b, offsets=off, reps=1, cache=str(tmp_path / "tune.json"))
    print(f"[tune] {choice}", flush=True)
    _check_same(af, tune, dA, 5, 1, b, choice, offsets=off)
    for c in ({"setup": {"lanes": 16, "table": 256}, "pcg": {"pcg_form": 2}},
              {"setup": {"lanes": 64, "claim": 2}, "pcg": {"pcg_graph": 2, "gt_layout": 1}}):
        _check_same(af, tune, dA, 5, 1, b, c, offsets=off)
