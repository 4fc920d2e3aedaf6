"""GPU parity of the nonlinear normal law (penetration to the power p).

Force tolerances are those of the linear law with the force scale at the
workload's maximum penetration D taken as k_n D^p (passed to the comparison
as an effective k_n D^(p-1)); the FP32 power (log2 / exp2) adds a few 1e-7
relative.  Gradients: block-norm relative 1e-4 against the oracle's dual
numbers, with the cancellation-aware scale of the linear case.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2408_06506_amd import workloads as wl  # noqa: E402
from tests.parity import near_decision_mask, compare, gpu_outputs_np, grad_blocks_close  # noqa: E402

pytestmark = pytest.mark.gpu

D = 2e-3


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_06506_amd import api as _api
    return _api


@pytest.mark.parametrize("p", [1.5, 2.0])
def test_forward_nonlinear_law(api, p):
    for tun in (dict(), dict(block=128, tile_taxels=128, schedule=2, grid=3, order=1)):
        sc = wl.make_small(cfg_id=85, n_env=6)
        _say(f"hunt-crossley p={p} {tun}")
        plan = api.Plan(sc, tun)
        plan.set_normal_law(p)
        st = plan.state(sc.state())
        out = plan.forward(st)
        torch.cuda.synchronize()
        s64 = oracle.state64(sc)
        s64["normal_exponent"] = np.float64(p)
        ref = oracle.force_field(sc, s64)
        kn = float(sc.params[:, 0].max())
        compare(sc, gpu_outputs_np(out), ref, D=D, kn=kn * D ** (p - 1), what=f"p={p}")
        # the observation pass uses the same law
        plan.set_observation(wl.scene_observation_bins(sc), 140)
        obs, out2 = plan.observe(st, fields=True)
        torch.cuda.synchronize()
        for k in ("depth", "normal", "fn", "ft", "wrench"):
            assert torch.equal(out[k], out2[k]), k
        obs_ref = oracle.observation(sc, ref, wl.scene_observation_bins(sc), 140)
        err = np.abs(obs.cpu().numpy() - obs_ref)
        assert err.max() <= 1e-4 * kn * D ** p + 1e-5 * np.abs(obs_ref).max()
        plan.close()


def test_linear_exponent_is_the_default_law(api):
    sc = wl.make_small(cfg_id=86, n_env=4)
    plan = api.Plan(sc)
    st = plan.state(sc.state())
    a = plan.forward(st)
    plan.set_normal_law(1.0)
    b = plan.forward(st)
    plan.set_normal_law(1.5)
    c = plan.forward(st)
    torch.cuda.synchronize()
    for k in ("depth", "normal", "fn", "ft", "wrench"):
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(a["depth"], c["depth"]) and not torch.equal(a["fn"], c["fn"])
    from paper_2408_06506_amd import _abi
    for bad in (0.5, 5.0, float("nan")):
        with pytest.raises(_abi.TacslError):
            plan.set_normal_law(bad)
    plan.close()


def test_adjoint_nonlinear_law(api):
    sc = wl.make_small(cfg_id=87, n_env=8)
    wa, wb = wl.loss_weights(sc.n_taxels, 4)
    _say("hunt-crossley adjoint")
    plan = api.Plan(sc, dict(tile_taxels=64, schedule=2, grid=3, block=64))
    plan.set_normal_law(1.5)
    st = plan.state(sc.state())
    s64 = oracle.state64(sc)
    s64["normal_exponent"] = np.float64(1.5)
    keep = near_decision_mask(sc, s64, 2e-3)
    wa, wb = (wa * keep).astype(np.float32), (wb * keep).astype(np.float32)
    g = plan.backward(st, torch.as_tensor(wa, device=plan.device), torch.as_tensor(wb, device=plan.device))
    torch.cuda.synchronize()
    gg = np.concatenate([g["g_obj_pose"].cpu().numpy(), g["g_obj_twist"].cpu().numpy(),
                         g["g_params"].cpu().numpy()], axis=1).astype(np.float64)
    _, ref, gabs = oracle.grad(sc, s64, wa, wb, with_abs=True)
    grad_blocks_close(gg, ref, 1e-4, what="p=1.5", g_abs=gabs)
    plan.close()
