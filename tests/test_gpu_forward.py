"""GPU parity of the forward force field against the FP64 oracle (MI355X)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2408_06506_amd import workloads as wl  # noqa: E402
from tests.parity import compare, gpu_outputs_np, rows_of  # noqa: E402

pytestmark = pytest.mark.gpu

KN = 1e4


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_06506_amd import api as _api
    return _api


def _run(api, scene, tun=None, step=None, plan=None):
    p = plan or api.Plan(scene, tun)
    st = p.state(scene.state(step))
    out = p.forward(st)
    torch.cuda.synchronize()
    return p, out


def test_tiny_ball_100_steps(api):
    """1 pad of 20x25 against the r = 10 mm sphere, 100 seeded steps."""
    sc0 = wl.make_c1(0)
    _say("c1 plan")
    plan = api.Plan(sc0)
    assert plan.offsets().tolist() == oracle.offsets(sc0).tolist()
    for step in range(100):
        sc = wl.make_c1(step)
        st = plan.state(sc.state())
        out = plan.forward(st)
        torch.cuda.synchronize()
        ref = oracle.force_field(sc, oracle.state64(sc))
        compare(sc, gpu_outputs_np(out), ref, D=1e-3, kn=KN, what=f"c1 step {step}")
        assert int(out["status"].item()) == 0


TUNINGS = [
    dict(),
    dict(block=64),
    dict(block=64, tile_taxels=64),
    dict(block=512, tile_taxels=512, order=2),
    dict(block=128, tile_taxels=128, schedule=1, grid=7, order=1),
    dict(block=256, tile_taxels=256, schedule=2, grid=5, order=3),
    dict(block=128, schedule=2, grid=3, order=1),
    dict(block=128, tile_taxels=128, schedule=0, order=4),
    dict(block=256, tile_taxels=0, schedule=0, order=5),
]


@pytest.mark.parametrize("seed", [0, 1])
def test_small_scenes_all_tunings(api, seed):
    """Eight objects, ragged 37x23 template, rotating objects and pads."""
    sc = wl.make_small(cfg_id=60 + seed, n_env=8)
    ref = oracle.force_field(sc, oracle.state64(sc))
    base = None
    for tun in TUNINGS:
        _say(f"small seed {seed} tuning {tun}")
        plan, out = _run(api, sc, tun)
        g = gpu_outputs_np(out)
        compare(sc, g, ref, D=2e-3, kn=KN, what=f"small{seed} {tun}")
        if base is None:
            base = g
        else:  # per-taxel outputs do not depend on the launch shape
            for k in ("depth", "normal", "fn", "ft"):
                assert np.array_equal(g[k], base[k]), (k, tun)
        plan.close()


def test_uneven_batch(api):
    sc = wl.make_uneven_small(cfg_id=12, n_env=12, substeps=3)
    for tun in (dict(), dict(block=128, tile_taxels=128, schedule=2, order=2),
                dict(block=64, tile_taxels=64, schedule=1, order=1)):
        _say(f"uneven tuning {tun}")
        plan = api.Plan(sc, tun)
        for step in range(3):
            st = plan.state(sc.state(step))
            out = plan.forward(st)
            torch.cuda.synchronize()
            ref = oracle.force_field(sc, oracle.state64(sc, step=step))
            compare(sc, gpu_outputs_np(out), ref, D=2e-3, kn=KN, what=f"uneven step {step} {tun}")
        plan.close()


def test_deterministic_run_to_run(api):
    sc = wl.make_small(cfg_id=70, n_env=6)
    plan = api.Plan(sc, dict(block=128, tile_taxels=128, schedule=2, grid=4))
    st = plan.state(sc.state())
    _say("determinism")
    a = {k: v.clone() for k, v in plan.forward(st).items()}
    b = plan.forward(st)
    torch.cuda.synchronize()
    for k in ("depth", "normal", "fn", "ft", "wrench"):
        assert torch.equal(a[k], b[k]), k


def test_plain_scale_full(api):
    """1024 envs x 2 pads x 40x50 on five objects at 128^3: every taxel."""
    sc = wl.make_c2()
    _say("c2 full")
    plan, out = _run(api, sc)
    assert plan.offsets().tolist() == oracle.offsets(sc).tolist()
    ref = oracle.force_field(sc, oracle.state64(sc))
    compare(sc, gpu_outputs_np(out), ref, D=2e-3, kn=KN, what="c2")
    assert int(out["status"].item()) == 0


def test_roofline_shape_sampled(api):
    """8192 envs x 2 pads x 80x100, eight objects at 256^3: 512 sampled pads."""
    sc = wl.make_c3()
    _say("c3 full launch")
    plan, out = _run(api, sc)
    rng = np.random.default_rng(3)
    sel = np.sort(rng.choice(sc.n_inst, 512, replace=False)).astype(np.int32)
    off = plan.offsets()
    assert off.tolist() == oracle.offsets(sc).tolist()
    rows = rows_of(off, sel)
    g = gpu_outputs_np(out, rows=torch.as_tensor(rows))
    g["wrench"] = out["wrench"][torch.as_tensor(sel, dtype=torch.long)].cpu().numpy().astype(np.float64)
    ref = oracle.force_field(sc, oracle.state64(sc), sel=sel)
    compare(sc, g, ref, D=2e-3, kn=KN, sel=sel, what="c3")  # stricter than the 4 mm cap
    # properties that hold at any size, on every taxel
    d = out["depth"]
    assert torch.all(d >= 0)
    fnm = torch.linalg.vector_norm(out["fn"], dim=0)
    ftm = torch.linalg.vector_norm(out["ft"], dim=0)
    assert torch.all((d > 0) | (fnm == 0))
    assert torch.all(ftm <= 0.8 * fnm * (1 + 1e-5) + 1e-6)
    frac = (d > 0).float().mean().item()
    print(f"c3 realized contact fraction {frac:.4f}")
    assert 0.62 < frac < 0.75
    # the launches the benchmark times (autotuned on MI355X, either of two
    # within noise): per-taxel outputs bitwise those of the default launch,
    # wrenches (summed per tile) against the oracle
    for tile in (4096, 0):
        _say(f"c3 benchmark launch, tile {tile}")
        plan.set_tuning(dict(block=512, tile_taxels=tile, schedule=0, grid=2048, order=5))
        out2 = plan.forward(plan.state(sc.state()))
        torch.cuda.synchronize()
        for k in ("depth", "normal", "fn", "ft"):
            assert torch.equal(out[k], out2[k]), (k, tile)
        g2 = gpu_outputs_np(out2, rows=torch.as_tensor(rows))
        g2["wrench"] = out2["wrench"][torch.as_tensor(sel, dtype=torch.long)].cpu().numpy().astype(np.float64)
        compare(sc, g2, ref, D=2e-3, kn=KN, sel=sel, what=f"c3 benchmark launch, tile {tile}")
        del out2
    plan.close()


def test_nonfinite_pose_sets_status_and_zero_pad(api):
    sc = wl.make_small(cfg_id=71, n_env=3)
    plan = api.Plan(sc)
    st = plan.state(sc.state())
    st["pad_pose"][1, 4] = float("nan")
    st["obj_pose"][2, :4] = 0.0
    _say("status bits")
    out = plan.forward(st)
    torch.cuda.synchronize()
    assert int(out["status"].item()) == 3
    off = plan.offsets()
    bad_pads = [1] + [i for i in range(sc.n_inst) if sc.inst_env[i] == 2]
    for i in bad_pads:
        sl = slice(int(off[i]), int(off[i + 1]))
        assert torch.all(out["depth"][sl] == 0) and torch.all(out["fn"][:, sl] == 0)
        assert torch.all(out["wrench"][i] == 0)
    good = [i for i in range(sc.n_inst) if i not in bad_pads]
    ref = oracle.force_field(sc, oracle.state64(sc), sel=np.array(good, np.int32))
    rows = torch.as_tensor(rows_of(off, good))
    g = gpu_outputs_np(out, rows=rows)
    g["wrench"] = out["wrench"][torch.as_tensor(good)].cpu().numpy().astype(np.float64)
    compare(sc, g, ref, D=2e-3, kn=KN, sel=good, what="good pads")


def test_empty_scene(api):
    sc = wl.make_small(cfg_id=72, n_env=2)
    sc.n_inst = 0
    sc.inst_env = np.zeros(0, np.int32)
    sc.inst_tmpl = np.zeros(0, np.int32)
    sc.pad_pose = np.zeros((0, 7), np.float32)
    sc.pad_twist = np.zeros((0, 6), np.float32)
    _say("empty scene")
    plan = api.Plan(sc)
    assert plan.n_taxels == 0
    out = plan.forward(plan.state(sc.state()))
    torch.cuda.synchronize()
    assert out["depth"].numel() == 0 and out["wrench"].shape == (0, 6)


def test_substep_graph_matches_eager(api):
    sc = wl.make_uneven_small(cfg_id=13, n_env=9, substeps=5)
    plan = api.Plan(sc, dict(tile_taxels=256, schedule=2, order=2))
    states = [plan.state(sc.state(s)) for s in range(5)]
    eager = []
    for s in range(5):
        eager.append({k: v.clone() for k, v in plan.forward(states[s]).items()})
    torch.cuda.synchronize()
    outs = [plan.new_outputs() for _ in range(5)]
    _say("graph capture")
    g = api.SubstepGraph(plan, states, outs)
    for rep in range(3):
        for o in outs:
            for v in o.values():
                v.fill_(-7.0) if v.dtype == torch.float32 else v.zero_()
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for s in range(5):
            for k in ("depth", "normal", "fn", "ft", "wrench"):
                assert torch.equal(outs[s][k], eager[s][k]), (rep, s, k)
    g.close()
    plan.close()


def test_rejected_tuning_keeps_the_plan_usable(api):
    """A tuning rejected by the library leaves the installed work list in place."""
    from paper_2408_06506_amd import _abi
    sc = wl.make_small(cfg_id=95, n_env=3)
    plan = api.Plan(sc, dict(block=128, tile_taxels=128, order=5))
    st = plan.state(sc.state())
    ref = plan.forward(st)
    torch.cuda.synchronize()
    for bad in (dict(block=96), dict(order=6), dict(tile_taxels=10)):
        with pytest.raises(_abi.TacslError):
            plan.set_tuning(bad)
    assert plan.tuning["order"] == 5 and plan.tuning["tile_taxels"] == 128
    out = plan.forward(st)
    torch.cuda.synchronize()
    for k in ("depth", "normal", "fn", "ft", "wrench"):
        assert torch.equal(out[k], ref[k]), k
    plan.close()


def test_batched_uneven_full_size(api):
    """4096 envs, 8192 pads of three resolutions on 24 grids (64/128/256^3),
    100 substeps in one HIP graph with the kind of launch the benchmark
    times (persistent dynamic queue), each substep stepping the object poses
    in the graph before its forward: recorded poses equal to the workload's,
    per-taxel outputs of substeps 0, 1, 49 and 99 and the wrenches of all 100
    substeps on 64 sampled pads."""
    from tests.parity import compare_wrench
    sc = wl.make_c4()
    S = sc.obj_pose_steps.shape[0]
    _say("c4 batched plan")
    plan = api.Plan(sc, dict(block=512, tile_taxels=1024, schedule=2, grid=1024, order=0))
    states = [plan.state(sc.state(s)) for s in range(S)]
    out = plan.new_outputs()
    wrench = torch.empty(S, sc.n_inst, 6, device=plan.device)
    # the graph steps the object poses itself (closed form from the substep-0
    # pose and twist) before each substep's forward
    poses = torch.empty(S, sc.n_env, 7, device=plan.device)
    path = dict(pose0=states[0]["obj_pose"], twist=states[0]["obj_twist"], dt=float(sc.meta["dt"]), poses=poses)
    graph = api.SubstepGraph(plan, states, [dict(out, wrench=wrench[s]) for s in range(S)], paths=path)
    _say("c4 graph launch")
    graph.launch()
    torch.cuda.synchronize()
    # recorded poses = the workload's closed-form substep poses, bit for bit
    assert np.array_equal(poses.cpu().numpy(), sc.obj_pose_steps)
    sel = np.sort(np.random.default_rng(21).choice(sc.n_inst, 64, replace=False)).astype(np.int32)
    off = plan.offsets()
    assert off.tolist() == oracle.offsets(sc).tolist()
    rows = torch.as_tensor(rows_of(off, sel))
    ws = wrench[:, torch.as_tensor(sel, dtype=torch.long)].cpu().numpy().astype(np.float64)
    for s in range(S):
        ref = oracle.force_field(sc, oracle.state64(sc, step=s), sel=sel)
        if s == S - 1:
            g = gpu_outputs_np(out, rows=rows)
            g["wrench"] = ws[s]
            compare(sc, g, ref, D=2e-3, kn=KN, sel=sel, what=f"c4 graph substep {s}")
        else:
            compare_wrench(sc, ws[s], ref, D=2e-3, kn=KN, sel=sel, extra_contacts=8, what=f"c4 graph substep {s}")
        if s in (0, 1, 49):
            o = plan.forward(states[s])
            torch.cuda.synchronize()
            g = gpu_outputs_np(o, rows=rows)
            g["wrench"] = o["wrench"][torch.as_tensor(sel, dtype=torch.long)].cpu().numpy().astype(np.float64)
            compare(sc, g, ref, D=2e-3, kn=KN, sel=sel, what=f"c4 eager substep {s}")
            assert np.array_equal(g["wrench"], ws[s])  # graph replay = eager launch
    graph.close()
    plan.close()


def test_fused_record_matches_prologue(api):
    """Launches of at most one workgroup per CU compute each pad's record in the
    forward kernel instead of a prologue launch; the outputs, wrenches and
    status bits are bitwise those of the prologue path."""
    sc = wl.make_small(cfg_id=73, n_env=12)
    res = {}
    # tile 0: 24 tiles (fused); tile 64: 24 x 14 tiles, more than the CUs
    # (prologue); order 5 always takes the prologue
    for name, tun in (("fused", dict(tile_taxels=0, order=0)), ("prologue", dict(tile_taxels=64, order=0)),
                      ("spatial", dict(tile_taxels=0, order=5))):
        _say(f"fused vs prologue: {name} {tun}")
        plan = api.Plan(sc, tun)
        if name != "spatial":
            assert (plan.info().n_tiles <= plan.info().cu_count) == (name == "fused")
        st = plan.state(sc.state())
        st["pad_pose"][5, 1] = float("inf")
        out = plan.forward(st)
        torch.cuda.synchronize()
        res[name] = {k: v.clone() for k, v in out.items()}
        plan.close()
    for name in ("prologue", "spatial"):
        for k in ("depth", "normal", "fn", "ft", "status"):
            assert torch.equal(res["fused"][k], res[name][k]), (name, k)
    # the same tiles (one per pad) sum the wrench in the same order; 64-taxel
    # tiles sum per-tile partials, another FP32 order
    assert torch.equal(res["fused"]["wrench"], res["spatial"]["wrench"])
    torch.testing.assert_close(res["fused"]["wrench"], res["prologue"]["wrench"], rtol=1e-5, atol=1e-3)
    assert int(res["fused"]["status"].item()) == 1
