"""Pins of the oracle's tactile depth image (Section III-B).

Closed forms on hand-built grids: a half-space parallel to the pad (every
pixel reads D - delta, orthographic and pinhole alike, since the image holds
z-distances); an inclined half-space seen through a pinhole (the ray through
pad point (p_x, p_y, 0) meets z + delta + s x = 0 at
z = -(delta + s p_x) / (1 + s p_x / D)); a sphere (orthographic, within the
trilinear error bound over the slope); an object deeper than the gel (the
bottom of the gel); rays outside the grid box (the gel surface).
"""
import numpy as np
import pytest

import oracle
from tests.scenes import grid_nodes, single

MM = 1e-3
H = 1.0 * MM
ORIGIN = np.asarray((-16 * MM, -16 * MM, -8 * MM), np.float32)
NODES = (33, 33, 17)


def _scene(phi_fn, h=H, nodes=NODES, origin=ORIGIN):
    xx, yy, zz = grid_nodes(nodes, origin.astype(np.float64), float(np.float32(h)))
    return single(phi_fn(xx, yy, zz), origin, h, [(0.0, 0.0, 0.0)])


def _cam(ortho, rows=8, cols=6, D=20 * MM, gel=4 * MM):
    return oracle.Camera(rows, cols, int(ortho), -10 * MM, -12.5 * MM, 20 * MM / cols, 25 * MM / rows, D, gel)


def _pix(cam):
    c = np.arange(cam.cols)
    r = np.arange(cam.rows)
    return (cam.x0 + (c[None, :] + 0.5) * cam.dx) * np.ones((cam.rows, 1)), \
           (cam.y0 + (r[:, None] + 0.5) * cam.dy) * np.ones((1, cam.cols))


@pytest.mark.parametrize("ortho", [1, 0])
def test_parallel_halfspace(ortho):
    delta = 1.3 * MM
    sc = _scene(lambda x, y, z: -(z + delta))
    cam = _cam(ortho)
    img, slope, _ = oracle.depth_image(sc, oracle.state64(sc), cam)
    np.testing.assert_allclose(img[0], cam.cam_dist - delta, rtol=0, atol=1e-10)
    np.testing.assert_allclose(slope[0], -1.0, rtol=1e-6)   # phi falls by 1 per unit height


def test_inclined_halfspace_pinhole():
    delta, s = 1.0 * MM, 0.1
    sc = _scene(lambda x, y, z: -(z + delta + s * x))
    cam = _cam(0)
    img, _, _ = oracle.depth_image(sc, oracle.state64(sc), cam)
    px, _ = _pix(cam)
    D = cam.cam_dist
    want = -(delta + s * px) / (1 + s * px / D) + D
    np.testing.assert_allclose(img[0], want, rtol=0, atol=1e-10)


def test_sphere_orthographic_within_trilinear_bound():
    R, delta = 8 * MM, 2.0 * MM
    zc = R - delta
    h = 0.5 * MM
    nodes = (65, 65, 41)
    origin = np.asarray((-16 * MM, -16 * MM, -8 * MM), np.float32)
    sc = _scene(lambda x, y, z: np.sqrt(x * x + y * y + (z - zc) ** 2) - R, h=h, nodes=nodes, origin=origin)
    cam = _cam(1, rows=40, cols=32)
    img, slope, _ = oracle.depth_image(sc, oracle.state64(sc), cam)
    px, py = _pix(cam)
    rho2 = px * px + py * py
    inside = rho2 < R * R
    zhit = np.where(inside, zc - np.sqrt(np.maximum(R * R - rho2, 0.0)), 0.0)
    hit = inside & (zhit <= 0.0)
    want = np.where(hit, zhit, 0.0) + cam.cam_dist
    # trilinear interpolation of a sphere SDF errs by at most (h^2/8)(2/R) in phi;
    # in height that is divided by |d phi / dz| at the hit
    bound = (h * h / 8) * (2 / R) / np.maximum(np.abs(slope[0]), 0.2) + 1e-9
    err = np.abs(img[0] - want)
    well = hit & (np.abs(slope[0]) > 0.2) & (zhit < -0.05 * MM)
    assert well.sum() > 100
    assert np.all(err[well] <= bound[well]), np.max(err[well] / bound[well])
    far = ~inside
    np.testing.assert_allclose(img[0][far], cam.cam_dist, atol=1e-12)


def test_object_through_the_gel_and_outside_the_box():
    sc = _scene(lambda x, y, z: -(z + 6 * MM))          # object reaches 6 mm below the pad, gel is 4 mm
    cam = _cam(1)
    img, _, _ = oracle.depth_image(sc, oracle.state64(sc), cam)
    np.testing.assert_allclose(img[0], cam.cam_dist - cam.gel, atol=1e-12)
    # a grid that covers only x > 0: pixels with x < 0 see no object
    origin = np.asarray((0.5 * MM, -16 * MM, -8 * MM), np.float32)
    sc2 = _scene(lambda x, y, z: -(z + 1 * MM), nodes=(20, 33, 17), origin=origin)
    img2, _, _ = oracle.depth_image(sc2, oracle.state64(sc2), cam)
    px, _ = _pix(cam)
    np.testing.assert_allclose(img2[0][px < 0], cam.cam_dist, atol=1e-12)
    np.testing.assert_allclose(img2[0][px > 1 * MM], cam.cam_dist - 1 * MM, atol=1e-10)


def _dense_first_root(scene, state, cam, i, pix, samples=4001):
    """Brute force: sample the ray densely in z, trilinear phi in numpy (no
    cell walk), and bisect the first sign change.  Returns z of the hit or 0."""
    from paper_2408_06506_amd.workloads import quat_to_mat
    e = scene.inst_env[i]
    g = scene.env_sdf[e]
    nx, ny, nz = (int(v) for v in scene.sdf_dims[g])
    phi = scene.sdf_data[scene.sdf_offset[g]:scene.sdf_offset[g] + nx * ny * nz].reshape(nz, ny, nx).astype(np.float64)
    h = float(scene.sdf_spacing[g])
    org = scene.sdf_origin[g].astype(np.float64)
    Rp = quat_to_mat(state["pad_pose"][i, :4] / np.linalg.norm(state["pad_pose"][i, :4]))
    Ro = quat_to_mat(state["obj_pose"][e, :4] / np.linalg.norm(state["obj_pose"][e, :4]))
    tp, to = state["pad_pose"][i, 4:], state["obj_pose"][e, 4:]
    n = np.array([nx, ny, nz])

    def f(r, c, z):
        px, py = cam.x0 + (c + 0.5) * cam.dx, cam.y0 + (r + 0.5) * cam.dy
        s = np.ones_like(z) if cam.ortho else (z + cam.cam_dist) / cam.cam_dist
        X = np.stack([px * s, py * s, z], -1)
        u = ((X @ Rp.T + tp - to) @ Ro - org) / h
        inside = np.all((u >= 0) & (u <= n - 1), axis=-1)
        cc = np.clip(np.floor(u).astype(int), 0, n - 2)
        t = u - cc
        v = np.zeros(z.shape)
        for k in range(8):
            d = np.array([k & 1, (k >> 1) & 1, k >> 2])
            w = np.prod(np.where(d == 1, t, 1 - t), axis=-1)
            v += w * phi[cc[..., 2] + d[2], cc[..., 1] + d[1], cc[..., 0] + d[0]]
        return np.where(inside, v, np.inf)

    out = []
    zs = np.linspace(-cam.gel, 0.0, samples)
    for r, c in pix:
        v = f(r, c, zs)
        k = np.flatnonzero(v <= 0)
        if k.size == 0:
            out.append(0.0)
            continue
        k = k[0]
        if k == 0:
            out.append(zs[0])
            continue
        lo, hi = zs[k - 1], zs[k]
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            if f(r, c, np.array([mid]))[0] <= 0:
                hi = mid
            else:
                lo = mid
        out.append(hi)
    return np.array(out)


@pytest.mark.parametrize("ortho", [0, 1])
def test_cell_walk_matches_dense_sampling(ortho):
    """The oracle's cell walk against brute-force sampling on real scenes
    (rays crossing many cells at steep angles, grid planes hit exactly)."""
    from paper_2408_06506_amd import workloads as wl
    sc = wl.make_small(cfg_id=71, n_env=3)
    st = oracle.state64(sc)
    f32 = lambda v: float(np.float32(v))
    cam = oracle.Camera(40, 32, ortho, f32(-wl.PAD_W / 2), f32(-wl.PAD_H / 2), f32(wl.PAD_W / 32),
                        f32(wl.PAD_H / 40), f32(20 * MM), f32(4 * MM))
    img, slope, _ = oracle.depth_image(sc, st, cam)
    rng = np.random.default_rng(3)
    checked = 0
    for i in range(sc.n_inst):
        pix = [(int(r), int(c)) for r, c in zip(rng.integers(0, 40, 60), rng.integers(0, 32, 60))]
        pix += [(31, 17), (0, 0), (39, 31)]
        z_bf = _dense_first_root(sc, st, cam, i, pix)
        for (r, c), zb in zip(pix, z_bf):
            zo = img[i, r, c] - cam.cam_dist
            if abs(slope[i, r, c]) < 0.05 and zo != 0.0:
                continue        # grazing hit: ill-conditioned, either answer is fine
            assert abs(zo - zb) <= 1e-11, (i, r, c, zo, zb)
            checked += 1
    assert checked > 150


def single_node_scene():
    """A positive field with one negative node, seen by a pad whose +z runs
    along the grid diagonal (the node 2 mm deep in the gel), and an
    orthographic camera whose rays pass close to the node."""
    h = 1e-3
    n = 9
    phi = np.full((n, n, n), 0.3e-3)
    phi[4, 4, 4] = -0.7e-3
    origin = np.asarray((-4e-3, -4e-3, -4e-3), np.float32)      # node (4,4,4) at the object origin
    d = np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0)                 # pad +z along the grid diagonal
    ax = np.cross([0.0, 0.0, 1.0], d)
    ang = np.arccos(d[2])
    ax /= np.linalg.norm(ax)
    q = np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * ax])
    obj_t = np.array([0.5, 0.5, 0.5])
    t_pad = obj_t + 2e-3 * d
    sc = single(phi, origin, h, [(0.0, 0.0, 0.0)], pad_pose=tuple(q) + tuple(t_pad),
                obj_pose=(1, 0, 0, 0) + tuple(obj_t))
    cam = dict(rows=24, cols=24, ortho=1, x0=-0.6e-3, y0=-0.6e-3, dx=0.05e-3, dy=0.05e-3, cam_dist=5e-3, gel=4e-3)
    return sc, cam


def test_single_negative_node_seen_by_oblique_rays():
    """The region where the trilinear field dips below zero is a small bump
    around the node, which oblique rays enter and leave within a single cell
    (the field along such a ray is a cubic).  The cell walk must find exactly
    the hits dense sampling finds."""
    sc, c = single_node_scene()
    st = oracle.state64(sc)
    cam = oracle.Camera(c["rows"], c["cols"], c["ortho"], c["x0"], c["y0"], c["dx"], c["dy"], c["cam_dist"], c["gel"])
    img, slope, _ = oracle.depth_image(sc, st, cam)
    pix = [(r, c_) for r in range(cam.rows) for c_ in range(cam.cols)]
    z_bf = _dense_first_root(sc, st, cam, 0, pix, samples=40001)
    hits = 0
    for (r, c_), zb in zip(pix, z_bf):
        zo = img[0, r, c_] - cam.cam_dist
        if abs(slope[0, r, c_]) < 0.05 and zo != 0.0:
            continue
        assert abs(zo - zb) <= 2e-9, (r, c_, zo, zb)   # dense sampling resolves 0.1 um steps
        hits += zb != 0.0
    assert 20 < hits < cam.rows * cam.cols              # the bump is seen by some rays, not all
