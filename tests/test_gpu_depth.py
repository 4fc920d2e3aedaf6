"""GPU parity of the tactile depth image against the FP64 oracle.

Tolerance per pixel where both find the object: the GPU evaluates the ray's
grid coordinates in FP32 (about 3e-5 of a cell at grid coordinates near 250),
so phi near the hit is off by up to ~3e-5 h and the hit height by that over
|d phi / dz|: |dz| <= 1e-4 h / max(|d phi / dz|, 0.05).  Hit/miss may differ
only where the oracle's hit is ill-conditioned (|d phi / dz| < 0.05), lies
within that tolerance of the gel surface, or where a ray without an oracle
hit came within 1e-4 h of the surface.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2408_06506_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

MM = 1e-3


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_06506_amd import api as _api
    return _api


def _cams(rows, cols, ortho, cam_dist=20 * MM, gel=4 * MM):
    f = lambda v: float(np.float32(v))
    vals = dict(rows=rows, cols=cols, x0=f(-wl.PAD_W / 2), y0=f(-wl.PAD_H / 2), dx=f(wl.PAD_W / cols),
                dy=f(wl.PAD_H / rows), cam_dist=f(cam_dist), gel=f(gel), ortho=ortho)
    oc = oracle.Camera(rows, cols, int(ortho), vals["x0"], vals["y0"], vals["dx"], vals["dy"], vals["cam_dist"],
                       vals["gel"])
    return vals, oc


def _check(scene, img_gpu, img_ref, slope, phimin, cam, sel, what, max_mismatch=1e-3):
    h = np.asarray(scene.sdf_spacing, np.float64)[scene.env_sdf[scene.inst_env[sel]]][:, None, None]
    D = cam.cam_dist
    z_gpu = img_gpu.astype(np.float64) - D
    z_ref = img_ref - D
    hit_ref = slope != 0.0
    hit_gpu = z_gpu != 0.0
    tol = 1e-4 * h / np.maximum(np.abs(slope), 0.05) + 1e-12
    both = hit_ref & hit_gpu
    err = np.abs(z_gpu - z_ref)
    bad = both & (err > tol)
    if bad.any():
        w = np.unravel_index(np.argmax(np.where(bad, err / tol, 0.0)), bad.shape)
        detail = (f"pad {int(sel[w[0]])} pixel ({w[1]}, {w[2]}): z_gpu {z_gpu[w]:.9g} z_ref {z_ref[w]:.9g} "
                  f"slope {slope[w]:.4g} phimin {phimin[w]:.3g}")
        assert False, f"{what}: {bad.sum()} of {both.sum()} hits off, worst {np.max(err[both] / tol[both]):.3g}x at {detail}"
    only_ref = hit_ref & ~hit_gpu
    only_gpu = hit_gpu & ~hit_ref
    ok_ref = (np.abs(slope) < 0.05) | (np.abs(z_ref) <= tol)
    ok_gpu = phimin <= 1e-4 * h
    assert np.all(ok_ref[only_ref]), f"{what}: {only_ref.sum()} oracle-only hits, {(~ok_ref[only_ref]).sum()} well posed"
    assert np.all(ok_gpu[only_gpu]), f"{what}: {only_gpu.sum()} gpu-only hits, {(~ok_gpu[only_gpu]).sum()} unexplained"
    n_mis = only_ref.sum() + only_gpu.sum()
    assert n_mis <= max_mismatch * z_ref.size, f"{what}: {n_mis} hit/miss disagreements"
    return hit_ref.mean()


@pytest.mark.parametrize("ortho", [0, 1])
def test_depth_matches_oracle_small(api, ortho):
    sc = wl.make_small(cfg_id=71, n_env=6)
    vals, oc = _cams(40, 32, ortho)
    _say(f"depth small ortho={ortho}")
    plan = api.Plan(sc)
    plan.set_camera(**vals)
    st = plan.state(sc.state())
    status = torch.zeros(1, device=plan.device, dtype=torch.int32)
    img = plan.depth_image(st, status=status)
    img2 = plan.depth_image(st)
    torch.cuda.synchronize()
    assert torch.equal(img, img2)                      # deterministic
    assert int(status.item()) == 0
    ref, slope, pmin = oracle.depth_image(sc, oracle.state64(sc), oc)
    frac = _check(sc, img.cpu().numpy(), ref, slope, pmin, oc, np.arange(sc.n_inst), f"small ortho={ortho}")
    assert 0.1 < frac < 0.95                            # both hits and misses are exercised
    plan.close()


def test_depth_uneven_batch_and_gel_limits(api):
    sc = wl.make_uneven_small(cfg_id=12, n_env=12, substeps=1)
    vals, oc = _cams(33, 27, 0, cam_dist=15 * MM, gel=1.0 * MM)   # thin gel: objects reach through it
    _say("depth uneven, thin gel")
    plan = api.Plan(sc)
    plan.set_camera(**vals)
    st = plan.state(sc.state())
    img = plan.depth_image(st)
    torch.cuda.synchronize()
    ref, slope, pmin = oracle.depth_image(sc, oracle.state64(sc), oc)
    _check(sc, img.cpu().numpy(), ref, slope, pmin, oc, np.arange(sc.n_inst), "uneven")
    g = img.cpu().numpy()
    assert np.all(g >= vals["cam_dist"] - vals["gel"] - 1e-9) and np.all(g <= vals["cam_dist"] + 1e-9)
    assert (np.abs(g - (vals["cam_dist"] - vals["gel"])) < 1e-9).any()   # some object passes the gel bottom
    plan.close()


def test_depth_roofline_batch_sampled(api):
    """The roofline batch with the 80 x 60 pinhole camera: 64 sampled pads
    against the oracle, and no ray hits the step limit anywhere."""
    sc = wl.make_c3()
    vals, oc = _cams(80, 60, 0)
    _say("depth c3")
    plan = api.Plan(sc)
    plan.set_camera(**vals)
    st = plan.state(sc.state())
    status = torch.zeros(1, device=plan.device, dtype=torch.int32)
    img = plan.depth_image(st, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    sel = np.sort(np.random.default_rng(9).choice(sc.n_inst, 64, replace=False)).astype(np.int32)
    ref, slope, pmin = oracle.depth_image(sc, oracle.state64(sc), oc, sel=sel)
    g = img[torch.as_tensor(sel, device=plan.device, dtype=torch.int64)].cpu().numpy()
    frac = _check(sc, g, ref, slope, pmin, oc, sel, "c3 sampled")
    assert frac > 0.3
    plan.close()


def test_depth_errors_and_graph(api):
    from paper_2408_06506_amd import _abi
    sc = wl.make_small(cfg_id=72, n_env=3)
    plan = api.Plan(sc)
    st = plan.state(sc.state())
    with pytest.raises(RuntimeError):
        plan.depth_image(st)
    vals, _ = _cams(16, 12, 0)
    for bad in (dict(rows=0), dict(cols=5000), dict(dx=0.0), dict(gel=-1e-3), dict(cam_dist=1e-3),
                dict(x0=float("nan"))):
        with pytest.raises(_abi.TacslError) as e:
            plan.set_camera(**dict(vals, **bad))
        assert e.value.code == -3
    plan.set_camera(**vals)
    img = plan.depth_image(st)
    torch.cuda.synchronize()
    _say("depth graph capture")
    out = torch.empty_like(img)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.depth_image(st, image=out)
    torch.cuda.synchronize()
    base = st["obj_pose"].clone()
    for rep in range(3):
        st["obj_pose"].copy_(base)
        st["obj_pose"][:, 6] += 2e-4 * rep
        out.zero_()
        g.replay()
        ref = plan.depth_image(st)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {rep}"
    plan.clear_camera()
    import ctypes
    with pytest.raises(_abi.TacslError) as e:
        s = plan._state_struct(st)
        _abi.check(_abi.load().tacsl_depth_image(plan._plan, ctypes.byref(s), ctypes.c_void_p(img.data_ptr()),
                                                 None, None), "depth")
    assert e.value.code == -7
    plan.close()


def test_depth_single_negative_node(api):
    """Oblique rays that enter and leave the object inside one cell: the
    exact per-cell search must see the same bump as the oracle."""
    from tests.test_oracle_depth import single_node_scene
    sc, c = single_node_scene()
    f = lambda v: float(np.float32(v))
    vals = dict(rows=c["rows"], cols=c["cols"], ortho=c["ortho"], x0=f(c["x0"]), y0=f(c["y0"]), dx=f(c["dx"]),
                dy=f(c["dy"]), cam_dist=f(c["cam_dist"]), gel=f(c["gel"]))
    oc = oracle.Camera(vals["rows"], vals["cols"], vals["ortho"], vals["x0"], vals["y0"], vals["dx"], vals["dy"],
                       vals["cam_dist"], vals["gel"])
    _say("depth single negative node")
    plan = api.Plan(sc)
    plan.set_camera(**vals)
    img = plan.depth_image(plan.state(sc.state()))
    torch.cuda.synchronize()
    ref, slope, pmin = oracle.depth_image(sc, oracle.state64(sc), oc)
    frac = _check(sc, img.cpu().numpy(), ref, slope, pmin, oc, np.arange(sc.n_inst), "single node", max_mismatch=0.02)
    assert frac > 0.03
    plan.close()


@pytest.mark.parametrize("dims,kind", [((37, 44, 29), "sphere"), ((41, 9, 2), "plane")])
def test_depth_odd_noncubic_grids(api, dims, kind):
    """Grids whose sizes are not multiples of the 8-cell slope blocks (partial
    blocks on the far faces, a single cell along z for the thin grid)."""
    from tests.test_gpu_clear_mask import H, _scene
    sc, _, _ = _scene(dims, kind, seed=5)
    ext = H * (np.array(dims) - 1)
    f = lambda v: float(np.float32(v))
    rows, cols = 24, 20
    vals = dict(rows=rows, cols=cols, ortho=0, x0=f(-0.45 * ext[0]), y0=f(-0.45 * ext[1]), dx=f(0.9 * ext[0] / cols),
                dy=f(0.9 * ext[1] / rows), cam_dist=f(3 * ext[2] + 0.02), gel=f(0.5 * ext[2] + H))
    oc = oracle.Camera(rows, cols, 0, vals["x0"], vals["y0"], vals["dx"], vals["dy"], vals["cam_dist"], vals["gel"])
    _say(f"depth {kind} {dims}")
    plan = api.Plan(sc)
    plan.set_camera(**vals)
    status = torch.zeros(1, device=plan.device, dtype=torch.int32)
    img = plan.depth_image(plan.state(sc.state()), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    ref, slope, pmin = oracle.depth_image(sc, oracle.state64(sc), oc)
    frac = _check(sc, img.cpu().numpy(), ref, slope, pmin, oc, np.arange(sc.n_inst), f"{kind} {dims}")
    assert 0.05 < frac < 0.95
    plan.close()
