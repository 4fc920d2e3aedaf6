"""The spatial execution order (tuning order 5), rebuilt on the device every
call, must visit every tile exactly once: outputs pre-filled with NaN come
out bitwise equal to those of the static orders, for the forward pass, the
adjoint and a captured substep graph whose poses change between steps."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2408_06506_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

SPATIAL = [dict(block=256, tile_taxels=0, schedule=0, order=5),
           dict(block=64, tile_taxels=64, schedule=0, order=5),
           dict(block=128, tile_taxels=128, schedule=1, grid=16, order=5)]


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_06506_amd import api as _api
    return _api


def _nan_outputs(plan):
    out = plan.new_outputs()
    for k in ("depth", "normal", "fn", "ft", "wrench"):
        out[k].fill_(float("nan"))
    return out


@pytest.mark.parametrize("tun", SPATIAL, ids=[str(i) for i in range(len(SPATIAL))])
def test_spatial_order_forward_and_adjoint(api, tun):
    for sc in (wl.make_small(cfg_id=90, n_env=9), wl.make_uneven_small(cfg_id=12, n_env=12, substeps=1)):
        _say(f"spatial order {sc.name} {tun}")
        ref_plan = api.Plan(sc, dict(block=tun["block"], tile_taxels=tun["tile_taxels"]))
        plan = api.Plan(sc, tun)
        st = plan.state(sc.state())
        ref = ref_plan.forward(st)
        for rep in range(2):
            out = plan.forward(st, _nan_outputs(plan))
            torch.cuda.synchronize()
            for k in ("depth", "normal", "fn", "ft", "wrench"):
                assert torch.equal(out[k], ref[k]), (k, rep)
        wa, wb = wl.loss_weights(sc.n_taxels, 2)
        wa_t, wb_t = torch.as_tensor(wa, device=plan.device), torch.as_tensor(wb, device=plan.device)
        g0 = ref_plan.backward(st, wa_t, wb_t)
        g1 = plan.backward(st, wa_t, wb_t)
        torch.cuda.synchronize()
        for k in ("g_obj_pose", "g_obj_twist", "g_params"):
            assert torch.equal(g0[k], g1[k]), k
        plan.close()
        ref_plan.close()


def test_spatial_order_in_a_substep_graph(api):
    sc = wl.make_uneven_small(cfg_id=13, n_env=12, substeps=4)
    plan = api.Plan(sc, dict(block=128, tile_taxels=0, schedule=0, order=5))
    ref_plan = api.Plan(sc, dict(block=128))
    states = [plan.state(sc.state(s)) for s in range(4)]
    outs = [_nan_outputs(plan) for _ in range(4)]
    _say("spatial order graph")
    g = api.SubstepGraph(plan, states, outs)
    for rep in range(2):
        for o in outs:
            for k in ("depth", "fn", "wrench"):
                o[k].fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        for s in range(4):
            ref = ref_plan.forward(states[s])
            torch.cuda.synchronize()
            for k in ("depth", "normal", "fn", "ft", "wrench"):
                assert torch.equal(outs[s][k], ref[k]), (rep, s, k)
    g.close()
    plan.close()
    ref_plan.close()
