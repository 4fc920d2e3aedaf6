"""Allocation-free forward (tacsl_force_field_noalloc) against tacsl_force_field.

Both entry points run the same kernels; the new one takes the buffers a call
writes and reads back (prologue records, tile partials, queue counter, spatial
order) from the library's static device scratch instead of the plan.  Two
calls in a row through the C-ABI, the second on a smaller scene, each
compared bit for bit with the plan-buffer entry point and with the oracle, in
launch shapes that use every scratch buffer; a plan that needs more scratch
than the array holds is refused before anything is launched.
"""
import ctypes
import types

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2408_06506_amd import _abi  # noqa: E402
from paper_2408_06506_amd import workloads as wl  # noqa: E402
from tests.parity import compare, gpu_outputs_np  # noqa: E402

pytestmark = pytest.mark.gpu

FIELDS = ("depth", "normal", "fn", "ft", "wrench")


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_06506_amd import api as _api
    return _api


def _noalloc(plan, st, out):
    """One call of tacsl_force_field_noalloc through the C-ABI; returns its status."""
    s = plan._state_struct(st)
    o = plan._out_struct(out)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return int(plan._lib.tacsl_force_field_noalloc(plan._plan, ctypes.byref(s), ctypes.byref(o), stream))


@pytest.mark.parametrize("tun", [dict(block=256, tile_taxels=128, schedule=2, grid=16, order=5),
                                 dict(block=128, tile_taxels=64, schedule=1, grid=5, order=1),
                                 dict(block=512, tile_taxels=0, schedule=0, order=0)])
def test_noalloc_matches_plan_buffers(api, tun):
    for cfg, n_env in ((70, 8), (71, 3)):  # the second call on a smaller scene
        sc = wl.make_small(cfg_id=cfg, n_env=n_env)
        _say(f"noalloc {tun} scene {cfg} ({sc.n_inst} pads, {sc.n_taxels} taxels)")
        plan = api.Plan(sc, tun)
        st = plan.state(sc.state())
        ref = plan.forward(st)
        out = plan.new_outputs()
        for k in FIELDS:
            out[k].fill_(float("nan"))
        rc = _noalloc(plan, st, out)
        torch.cuda.synchronize()
        assert rc == 0, _abi.STATUS_NAMES.get(rc, rc)
        for k in FIELDS:
            assert torch.equal(out[k], ref[k]), k
        compare(sc, gpu_outputs_np(out), oracle.force_field(sc, oracle.state64(sc)), D=2e-3, kn=1e4,
                what=f"noalloc {tun}")
        plan.close()


def test_noalloc_refuses_oversized_plan(api):
    """180000 one-taxel pads need ~22 MB of call buffers: refused with
    TACSL_ERR_UNSUPPORTED before any launch; the plan-buffer call still runs."""
    n = 180000
    sc = types.SimpleNamespace(
        n_env=1, n_inst=n, inst_env=np.zeros(n, np.int32), inst_tmpl=np.zeros(n, np.int32),
        env_sdf=np.zeros(1, np.int32), tmpl_offset=np.array([0, 1], np.int64),
        tmpl_xyz=np.zeros((3, 1), np.float32), sdf_dims=np.array([[4, 4, 4]], np.int32),
        sdf_origin=np.full((1, 3), -1.0, np.float32), sdf_spacing=np.array([0.5], np.float32),
        sdf_offset=np.zeros(1, np.int64), sdf_data=np.ones(64, np.float32))
    plan = api.Plan(sc, dict(tile_taxels=0, order=0))
    q = np.tile(np.array([1, 0, 0, 0, 0, 0, 0], np.float32), (n, 1))
    st = plan.state(dict(pad_pose=q, obj_pose=q[:1], pad_twist=np.zeros((n, 6), np.float32),
                         obj_twist=np.zeros((1, 6), np.float32), params=np.array([[1e4, 10, 100, 0.8]], np.float32)))
    out = plan.new_outputs()
    _say("noalloc oversized plan")
    assert _noalloc(plan, st, out) == -6
    plan.forward(st, out)
    torch.cuda.synchronize()
    assert torch.all(out["depth"] == 0)
    plan.close()
