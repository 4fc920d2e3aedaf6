"""Seeded synthetic scenes for the tactile force field.

This module generates inputs only: exact analytic signed-distance functions
sampled at grid nodes (stored FP32), planar pad templates, world poses,
twists, contact parameters and loss weights.  It holds none of the force-field
arithmetic itself (no trilinear queries, no gradients of the sampled field, no
force law), so both the HIP path and the independent FP64 oracle can consume
what it returns.

Workload shapes follow the paper's setups: a rectangular pad pressed against a
sphere (ball rolling, Section V-A), pegs and primitive objects (Section V),
two fingers per environment (the force-field observation of Section V-B) and
the robot workspace ranges of the randomization table (Appendix C).  The
objects are analytic stand-ins for the paper's meshes, which are not
available.

Conventions
-----------
* Units are metres, m/s, rad/s.
* Poses are ``qw qx qy qz tx ty tz`` (unit quaternion, world frame).
* Twists are ``vx vy vz wx wy wz``: linear velocity of the body origin and
  angular velocity, both in the world frame.
* Pad templates are SoA ``[3][K]``; the pad is the plane z = 0 with +z pointing
  towards the object.  Taxels are numbered in 8 x 8 tiles of the grid
  (``taxel_grid_index`` maps a template index to its row and column).
* SDF grids are node-centred, isotropic spacing h, x fastest; node (i,j,k) sits
  at ``origin + h * (i, j, k)`` in the object frame; values are negative
  inside the object.
* Random streams: ``numpy.random.Generator(PCG64(SeedSequence([cfg, step])))``.
"""
from __future__ import annotations

import concurrent.futures as _fut
import dataclasses
import functools
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

MM = 1e-3

# --------------------------------------------------------------------------
# Exact analytic signed distance functions (FP64, object frame, metres).
# --------------------------------------------------------------------------


def _sd_box(p, half):
    q = np.abs(p) - np.asarray(half)
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
    inside = np.minimum(np.max(q, axis=-1), 0.0)
    return outside + inside


def _sd_extrude(d2, z, half_h):
    # exact extrusion of a 2-D signed distance along z
    w0 = d2
    w1 = np.abs(z) - half_h
    outside = np.sqrt(np.maximum(w0, 0.0) ** 2 + np.maximum(w1, 0.0) ** 2)
    inside = np.minimum(np.maximum(w0, w1), 0.0)
    return outside + inside


def _sd_cylinder(p, r, half_h):
    d2 = np.hypot(p[..., 0], p[..., 1]) - r
    return _sd_extrude(d2, p[..., 2], half_h)


def _sd_sphere(p, r):
    return np.linalg.norm(p, axis=-1) - r


def _sd_capsule(p, r, half_seg):
    z = np.clip(p[..., 2], -half_seg, half_seg)
    q = p.copy()
    q[..., 2] = p[..., 2] - z
    return np.linalg.norm(q, axis=-1) - r


def _sd_torus(p, big_r, small_r):
    qx = np.hypot(p[..., 0], p[..., 1]) - big_r
    return np.hypot(qx, p[..., 2]) - small_r


def _sd_hexagon2(px, py, apothem):
    """Exact 2-D distance to a regular hexagon with the given apothem.

    Flats are perpendicular to the directions k * 60 deg.  Inside a convex
    polygon the distance is the smallest distance to an edge line; outside it
    is the distance to the nearest edge segment.
    """
    circ = apothem * 2.0 / math.sqrt(3.0)
    ang = np.deg2rad(np.arange(6) * 60.0 + 30.0)
    verts = np.stack([circ * np.cos(ang), circ * np.sin(ang)], axis=-1)  # (6,2)
    p = np.stack([px, py], axis=-1)
    line_d = []
    seg_d = []
    for k in range(6):
        a = verts[k - 1]
        b = verts[k]
        mid = 0.5 * (a + b)
        nrm = mid / np.linalg.norm(mid)
        line_d.append((p - mid) @ nrm)
        ab = b - a
        t = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
        proj = a + t[..., None] * ab
        seg_d.append(np.linalg.norm(p - proj, axis=-1))
    line_d = np.stack(line_d, axis=-1)
    seg_d = np.stack(seg_d, axis=-1)
    inside = np.all(line_d <= 0.0, axis=-1)
    return np.where(inside, np.max(line_d, axis=-1), np.min(seg_d, axis=-1))


def _sd_hex_prism(p, apothem, half_h):
    d2 = _sd_hexagon2(p[..., 0], p[..., 1], apothem)
    return _sd_extrude(d2, p[..., 2], half_h)


@dataclasses.dataclass(frozen=True)
class ObjectSpec:
    name: str
    kind: str
    dims: Tuple[float, ...]
    extent: float  # largest bounding-box side, metres

    def sdf(self, p: np.ndarray) -> np.ndarray:
        d = self.dims
        if self.kind == "box":
            return _sd_box(p, d)
        if self.kind == "cylinder":
            return _sd_cylinder(p, d[0], d[1])
        if self.kind == "sphere":
            return _sd_sphere(p, d[0])
        if self.kind == "capsule":
            return _sd_capsule(p, d[0], d[1])
        if self.kind == "torus":
            return _sd_torus(p, d[0], d[1])
        if self.kind == "hex":
            return _sd_hex_prism(p, d[0], d[1])
        raise ValueError(self.kind)


OBJECTS: Dict[str, ObjectSpec] = {
    # box 40 mm cube
    "box": ObjectSpec("box", "box", (20 * MM, 20 * MM, 20 * MM), 40 * MM),
    # cylinder r = 20, height 40
    "cylinder": ObjectSpec("cylinder", "cylinder", (20 * MM, 20 * MM), 40 * MM),
    # sphere r = 20
    "sphere": ObjectSpec("sphere", "sphere", (20 * MM,), 40 * MM),
    # square peg 16 x 16 x 50
    "square_peg": ObjectSpec("square_peg", "box", (8 * MM, 8 * MM, 25 * MM), 50 * MM),
    # round peg r = 8, length 50
    "round_peg": ObjectSpec("round_peg", "cylinder", (8 * MM, 25 * MM), 50 * MM),
    # hex prism, 24 mm across flats, height 20
    "hex_prism": ObjectSpec("hex_prism", "hex", (12 * MM, 10 * MM), 24 * 2 / math.sqrt(3) * MM),
    # capsule r = 10, segment 30
    "capsule": ObjectSpec("capsule", "capsule", (10 * MM, 15 * MM), 50 * MM),
    # torus R = 15, r = 6
    "torus": ObjectSpec("torus", "torus", (15 * MM, 6 * MM), 42 * MM),
    # small sphere of the tiny ball-rolling case, r = 10
    "sphere10": ObjectSpec("sphere10", "sphere", (10 * MM,), 20 * MM),
}

FIVE_OBJECTS = ["box", "cylinder", "sphere", "square_peg", "round_peg"]
EIGHT_OBJECTS = ["box", "cylinder", "sphere", "square_peg", "round_peg",
                 "hex_prism", "capsule", "torus"]


def grid_geometry(obj: ObjectSpec, n: int, spacing: Optional[float] = None):
    """Cubic n^3 grid centred on the object origin.

    Default spacing leaves a 6 mm margin on each side of the largest extent.
    Returns (origin[3], h) in FP64.
    """
    h = spacing if spacing is not None else (obj.extent + 12 * MM) / (n - 1)
    o = -0.5 * h * (n - 1)
    return np.array([o, o, o], dtype=np.float64), float(h)


def _sample_slab(obj, origin, h, n, k0, k1):
    xs = origin[0] + h * np.arange(n, dtype=np.float64)
    ys = origin[1] + h * np.arange(n, dtype=np.float64)
    zs = origin[2] + h * np.arange(k0, k1, dtype=np.float64)
    zz, yy, xx = np.meshgrid(zs, ys, xs, indexing="ij")
    p = np.stack([xx, yy, zz], axis=-1)
    return obj.sdf(p).astype(np.float32)


@functools.lru_cache(maxsize=64)
def voxelize(name: str, n: int, spacing: Optional[float] = None):
    """Sample the exact SDF of object ``name`` at the n^3 nodes.

    Returns (values float32 [n*n*n] x-fastest, origin float32[3], h float32).
    The FP32-rounded origin and spacing are the ones the scene reports, and the
    node values are the FP64 distances at those rounded node positions.
    """
    obj = OBJECTS[name]
    origin, h = grid_geometry(obj, n, spacing)
    origin32 = origin.astype(np.float32)
    h32 = np.float32(h)
    o64 = origin32.astype(np.float64)
    h64 = float(h32)
    out = np.empty((n, n, n), dtype=np.float32)
    slab = max(1, (1 << 21) // (n * n))
    ranges = [(k, min(n, k + slab)) for k in range(0, n, slab)]

    def work(r):
        out[r[0]:r[1]] = _sample_slab(obj, o64, h64, n, r[0], r[1])

    with _fut.ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(work, ranges))
    out.setflags(write=False)
    return out.reshape(-1), origin32, h32


# --------------------------------------------------------------------------
# Pad templates
# --------------------------------------------------------------------------

PAD_W = 20 * MM
PAD_H = 25 * MM


TAXEL_BLOCK = 8


def taxel_grid_index(nx: int, ny: int, block: int = TAXEL_BLOCK) -> np.ndarray:
    """Template numbering of an nx x ny taxel grid: (j, i) of every template
    index, in block x block tiles (tiles row-major, taxels row-major within a
    tile).  64 consecutive taxels then form a compact 8 x 8 patch."""
    ij = []
    for jb in range(0, ny, block):
        for ib in range(0, nx, block):
            for j in range(jb, min(jb + block, ny)):
                for i in range(ib, min(ib + block, nx)):
                    ij.append((j, i))
    return np.asarray(ij, dtype=np.int64).reshape(-1, 2)


@functools.lru_cache(maxsize=32)
def pad_template(nx: int, ny: int, width: float = PAD_W, height: float = PAD_H, block: int = TAXEL_BLOCK):
    """Planar pad of nx x ny taxels at cell centres, SoA float32 [3][nx*ny].

    Taxels are numbered in block x block tiles (``taxel_grid_index``); use
    ``block=max(nx, ny)`` for plain row-major numbering.
    """
    px = width / nx
    py = height / ny
    ji = taxel_grid_index(nx, ny, block)
    x = -0.5 * width + (ji[:, 1] + 0.5) * px
    y = -0.5 * height + (ji[:, 0] + 0.5) * py
    z = np.zeros_like(x)
    t = np.stack([x, y, z]).astype(np.float32)
    t.setflags(write=False)
    return t


# --------------------------------------------------------------------------
# Rotation helpers (generator geometry only)
# --------------------------------------------------------------------------


def quat_to_mat(q):
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def mat_to_quat(r):
    """Rotation matrix -> unit quaternion (w >= 0), Shepperd's method."""
    r = np.asarray(r, dtype=np.float64)
    shp = r.shape[:-2]
    r = r.reshape(-1, 3, 3)
    q = np.empty((r.shape[0], 4))
    tr = r[:, 0, 0] + r[:, 1, 1] + r[:, 2, 2]
    diag = np.stack([tr, r[:, 0, 0], r[:, 1, 1], r[:, 2, 2]], axis=-1)
    k = np.argmax(diag, axis=-1)
    for idx in range(r.shape[0]):
        m = r[idx]
        if k[idx] == 0:
            s = math.sqrt(1.0 + tr[idx]) * 2
            q[idx] = [0.25 * s, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif k[idx] == 1:
            s = math.sqrt(1.0 + m[0, 0] - m[1, 1] - m[2, 2]) * 2
            q[idx] = [(m[2, 1] - m[1, 2]) / s, 0.25 * s, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif k[idx] == 2:
            s = math.sqrt(1.0 + m[1, 1] - m[0, 0] - m[2, 2]) * 2
            q[idx] = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, 0.25 * s, (m[1, 2] + m[2, 1]) / s]
        else:
            s = math.sqrt(1.0 + m[2, 2] - m[0, 0] - m[1, 1]) * 2
            q[idx] = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, 0.25 * s]
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    return q.reshape(shp + (4,))


def axis_angle_mat(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis, axis=-1, keepdims=True)
    x, y, z = axis[..., 0], axis[..., 1], axis[..., 2]
    c = np.cos(angle)
    s = np.sin(angle)
    C = 1 - c
    r = np.empty(axis.shape[:-1] + (3, 3))
    r[..., 0, 0] = c + x * x * C
    r[..., 0, 1] = x * y * C - z * s
    r[..., 0, 2] = x * z * C + y * s
    r[..., 1, 0] = y * x * C + z * s
    r[..., 1, 1] = c + y * y * C
    r[..., 1, 2] = y * z * C - x * s
    r[..., 2, 0] = z * x * C - y * s
    r[..., 2, 1] = z * y * C + x * s
    r[..., 2, 2] = c + z * z * C
    return r


def random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    return q


# --------------------------------------------------------------------------
# Pad placement against an object (analytic SDF, FP64)
# --------------------------------------------------------------------------


def _surface_points(obj: ObjectSpec, rng, n):
    """Outermost surface crossing along random rays from the object origin."""
    pts = np.zeros((n, 3))
    nrm = np.zeros((n, 3))
    todo = np.arange(n)
    smax = obj.extent
    step = 0.25 * MM
    ss = np.arange(smax, 0.0, -step)
    while todo.size:
        d = rng.standard_normal((todo.size, 3))
        d /= np.linalg.norm(d, axis=-1, keepdims=True)
        vals = obj.sdf(d[:, None, :] * ss[None, :, None])  # (m, S)
        neg = vals < 0
        hit = neg.any(axis=1)
        first = np.argmax(neg, axis=1)
        ok = hit & (first > 0)
        lo = ss[first] * 1.0  # inside
        hi = ss[np.maximum(first - 1, 0)] * 1.0  # outside
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            v = obj.sdf(d * mid[:, None])
            inside = v < 0
            lo = np.where(inside, mid, lo)
            hi = np.where(inside, hi, mid)
        p = d * (0.5 * (lo + hi))[:, None]
        e = 1e-7
        g = np.stack([
            obj.sdf(p + np.array([e, 0, 0])) - obj.sdf(p - np.array([e, 0, 0])),
            obj.sdf(p + np.array([0, e, 0])) - obj.sdf(p - np.array([0, e, 0])),
            obj.sdf(p + np.array([0, 0, e])) - obj.sdf(p - np.array([0, 0, e])),
        ], axis=-1)
        gn = np.linalg.norm(g, axis=-1)
        ok &= gn > 1e-12
        sel = todo[ok]
        pts[sel] = p[ok]
        nrm[sel] = g[ok] / gn[ok][:, None]
        todo = todo[~ok]
    return pts, nrm


def _pad_frames(rng, normals, max_tilt_deg=5.0):
    """Pad rotation in the object frame: +z along -normal, random spin and tilt."""
    n = normals.shape[0]
    z = -normals
    helper = np.where(np.abs(z[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    e1 = np.cross(z, helper)
    e1 /= np.linalg.norm(e1, axis=-1, keepdims=True)
    e2 = np.cross(z, e1)
    alpha = rng.uniform(0.0, 2 * np.pi, n)
    x = np.cos(alpha)[:, None] * e1 + np.sin(alpha)[:, None] * e2
    y = np.cross(z, x)
    r = np.stack([x, y, z], axis=-1)  # columns = pad axes in object frame
    tilt = np.deg2rad(rng.uniform(0.0, max_tilt_deg, n))
    gam = rng.uniform(0.0, 2 * np.pi, n)
    ax = np.cos(gam)[:, None] * x + np.sin(gam)[:, None] * y
    rt = axis_angle_mat(ax, tilt)
    return rt @ r


def _draw_pads(obj, rng, n):
    """Random part of pad placement: surface point, outward normal, pad frame."""
    q, nrm = _surface_points(obj, rng, n)
    r = _pad_frames(rng, nrm)
    return q, nrm, r


def _bisect_offsets(obj, tmpl_sub, q, nrm, r, pen_target, frac_target=None, pen_cap=None, iters=36):
    """Deterministic part of pad placement (no random draws).

    ``tmpl_sub`` are the taxel positions (pad frame, FP64 [K,3]) used to
    measure penetration.  The pad moves along the surface normal; the offset
    is bisected so that the deepest taxel penetration equals ``pen_target``
    (or, when ``frac_target`` is given, so that that fraction of taxels is
    inside, with the deepest penetration capped at ``pen_cap``).  Returns the
    pad origins in the object frame.
    """
    n = q.shape[0]
    xk = np.einsum("nij,kj->nki", r, tmpl_sub)  # (n, K, 3)

    def depth_stats(off):
        p = q + nrm * off[:, None]
        v = obj.sdf(p[:, None, :] + xk)
        return -v.min(axis=1), (v < 0).mean(axis=1)

    def bisect(fn, target):
        lo = np.full(n, -10 * MM)  # deep
        hi = np.full(n, 10 * MM)  # clear
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            deeper = fn(mid) > target
            lo = np.where(deeper, mid, lo)
            hi = np.where(deeper, hi, mid)
        return 0.5 * (lo + hi)

    if frac_target is None:
        off = bisect(lambda o: depth_stats(o)[0], pen_target)
    else:
        off_f = bisect(lambda o: depth_stats(o)[1] - 1e-9, frac_target)
        off_c = bisect(lambda o: depth_stats(o)[0], pen_cap)
        off = np.maximum(off_f, off_c)
    return q + nrm * off[:, None]


# --------------------------------------------------------------------------
# Scenes
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Scene:
    """Host arrays describing one synthetic workload (FP32 as consumed)."""
    name: str
    n_env: int
    n_inst: int
    inst_env: np.ndarray  # int32 [I]
    inst_tmpl: np.ndarray  # int32 [I]
    env_sdf: np.ndarray  # int32 [E]
    tmpl_offset: np.ndarray  # int64 [n_tmpl+1]
    tmpl_xyz: np.ndarray  # float32 [3][T_tmpl]
    sdf_dims: np.ndarray  # int32 [n_sdf][3]
    sdf_origin: np.ndarray  # float32 [n_sdf][3]
    sdf_spacing: np.ndarray  # float32 [n_sdf]
    sdf_offset: np.ndarray  # int64 [n_sdf]
    sdf_data: np.ndarray  # float32 [total nodes]
    pad_pose: np.ndarray  # float32 [I][7]
    obj_pose: np.ndarray  # float32 [E][7]
    pad_twist: np.ndarray  # float32 [I][6]
    obj_twist: np.ndarray  # float32 [E][6]
    params: np.ndarray  # float32 [E][4]
    sdf_names: List[str] = dataclasses.field(default_factory=list)
    tmpl_names: List[str] = dataclasses.field(default_factory=list)
    obj_pose_steps: Optional[np.ndarray] = None  # float32 [S][E][7] (substep loop)
    meta: Dict[str, object] = dataclasses.field(default_factory=dict)

    @property
    def n_tmpl(self):
        return int(self.tmpl_offset.size - 1)

    @property
    def n_sdf(self):
        return int(self.sdf_spacing.size)

    def inst_counts(self):
        c = np.diff(self.tmpl_offset)
        return c[self.inst_tmpl].astype(np.int64)

    @property
    def n_taxels(self):
        return int(self.inst_counts().sum())

    def state(self, step: Optional[int] = None):
        obj_pose = self.obj_pose if step is None else self.obj_pose_steps[step]
        return dict(pad_pose=self.pad_pose, obj_pose=obj_pose, pad_twist=self.pad_twist,
                    obj_twist=self.obj_twist, params=self.params)


def rng_for(cfg_id: int, step: int = 0):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg_id, step])))


DEFAULT_PARAMS = (1e4, 10.0, 1e2, 0.8)  # k_n, k_d, k_t, mu


def build_scene(name: str, cfg_id: int, step: int, env_obj: Sequence[str],
                env_grid: Sequence[int], env_res: Sequence[Tuple[int, int]],
                pads_per_env: int = 2, pen_range=(0.0, 2 * MM), frac_target=None,
                pen_cap=2 * MM, vmax=0.1, wmax=0.0, pad_vmax=0.0, pad_wmax=0.0,
                params=DEFAULT_PARAMS, grid_spacing: Optional[Dict[Tuple[str, int], float]] = None,
                placement_subsample: Optional[int] = None) -> Scene:
    """Assemble a scene from per-environment object, grid size and pad resolution.

    Environments are independent; every environment holds ``pads_per_env``
    pads on opposite sides of its object (two fingers).
    """
    rng = rng_for(cfg_id, step)
    E = len(env_obj)
    # SDF pool: one grid per distinct (object, N)
    keys: List[Tuple[str, int]] = []
    env_sdf = np.empty(E, dtype=np.int32)
    for e in range(E):
        k = (env_obj[e], int(env_grid[e]))
        if k not in keys:
            keys.append(k)
        env_sdf[e] = keys.index(k)
    datas, dims, origins, spacings, offsets = [], [], [], [], []
    off = 0
    for (oname, n) in keys:
        sp = None if grid_spacing is None else grid_spacing.get((oname, n))
        vals, o32, h32 = voxelize(oname, n, sp)
        datas.append(vals)
        dims.append((n, n, n))
        origins.append(o32)
        spacings.append(h32)
        offsets.append(off)
        off += vals.size
    sdf_data = np.concatenate(datas) if len(datas) > 1 else datas[0].copy()
    # templates: one per distinct resolution
    res_keys: List[Tuple[int, int]] = []
    env_tmpl = np.empty(E, dtype=np.int32)
    for e in range(E):
        r = tuple(env_res[e])
        if r not in res_keys:
            res_keys.append(r)
        env_tmpl[e] = res_keys.index(r)
    tmpls = [pad_template(*r) for r in res_keys]
    tmpl_offset = np.zeros(len(tmpls) + 1, dtype=np.int64)
    tmpl_offset[1:] = np.cumsum([t.shape[1] for t in tmpls])
    tmpl_xyz = np.concatenate(tmpls, axis=1).astype(np.float32)

    I = E * pads_per_env
    inst_env = np.repeat(np.arange(E, dtype=np.int32), pads_per_env)
    inst_tmpl = env_tmpl[inst_env].astype(np.int32)

    # object world poses: uniform SO(3), workspace translation ranges
    q_o = random_quats(rng, E)
    t_o = np.stack([rng.uniform(0.4, 0.6, E), rng.uniform(-0.1, 0.1, E),
                    rng.uniform(0.0, 0.2, E)], axis=-1)
    R_o = quat_to_mat(q_o)

    pad_R = np.zeros((I, 3, 3))
    pad_t = np.zeros((I, 3))
    # place pads group by (object, resolution) so the analytic SDF is vectorised;
    # random draws happen in a fixed sequential order, bisection runs threaded
    groups: Dict[Tuple[str, Tuple[int, int]], List[int]] = {}
    for i in range(I):
        e = inst_env[i]
        groups.setdefault((env_obj[e], tuple(env_res[e])), []).append(i)
    jobs = []
    for (oname, res), insts in sorted(groups.items()):
        obj = OBJECTS[oname]
        t = pad_template(*res).astype(np.float64).T
        if placement_subsample:
            # evenly spread taxels covering the whole pad, edges included
            nx, ny = res
            ii = np.unique(np.round(np.linspace(0, nx - 1, min(nx, placement_subsample[0]))).astype(int))
            jj = np.unique(np.round(np.linspace(0, ny - 1, min(ny, placement_subsample[1]))).astype(int))
            t = t[(jj[:, None] * nx + ii[None, :]).reshape(-1)]
        insts = np.asarray(insts)
        pen = rng.uniform(pen_range[0], pen_range[1], insts.size)
        q, nrm, r = _draw_pads(obj, rng, insts.size)
        jobs.append((obj, t, insts, q, nrm, r, pen))

    def place(job):
        obj, t, insts, q, nrm, r, pen = job
        pad_R[insts] = r
        pad_t[insts] = _bisect_offsets(obj, t, q, nrm, r, pen, frac_target=frac_target, pen_cap=pen_cap)

    with _fut.ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(place, jobs))
    # compose to world
    Rw = np.einsum("iab,ibc->iac", R_o[inst_env], pad_R)
    tw = t_o[inst_env] + np.einsum("iab,ib->ia", R_o[inst_env], pad_t)
    pad_pose = np.concatenate([mat_to_quat(Rw), tw], axis=-1).astype(np.float32)
    obj_pose = np.concatenate([q_o, t_o], axis=-1).astype(np.float32)

    obj_twist = np.zeros((E, 6))
    obj_twist[:, :3] = rng.uniform(-vmax, vmax, (E, 3))
    if wmax:
        obj_twist[:, 3:] = rng.uniform(-wmax, wmax, (E, 3))
    pad_twist = np.zeros((I, 6))
    if pad_vmax:
        pad_twist[:, :3] = rng.uniform(-pad_vmax, pad_vmax, (I, 3))
    if pad_wmax:
        pad_twist[:, 3:] = rng.uniform(-pad_wmax, pad_wmax, (I, 3))
    prm = np.tile(np.asarray(params, dtype=np.float64), (E, 1))

    return Scene(
        name=name, n_env=E, n_inst=I, inst_env=inst_env, inst_tmpl=inst_tmpl,
        env_sdf=env_sdf, tmpl_offset=tmpl_offset, tmpl_xyz=tmpl_xyz,
        sdf_dims=np.asarray(dims, dtype=np.int32).reshape(-1, 3),
        sdf_origin=np.asarray(origins, dtype=np.float32).reshape(-1, 3),
        sdf_spacing=np.asarray(spacings, dtype=np.float32),
        sdf_offset=np.asarray(offsets, dtype=np.int64), sdf_data=sdf_data,
        pad_pose=pad_pose, obj_pose=obj_pose,
        pad_twist=pad_twist.astype(np.float32), obj_twist=obj_twist.astype(np.float32),
        params=prm.astype(np.float32), sdf_names=[f"{k[0]}@{k[1]}" for k in keys],
        tmpl_names=[f"{r[0]}x{r[1]}" for r in res_keys],
    )


# --------------------------------------------------------------------------
# The five workloads (and reduced variants with the same structure)
# --------------------------------------------------------------------------

CONFIGS = {
    1: "tiny: 1 env x 1 pad 20x25, sphere r=10 mm at 64^3 / 0.5 mm, 100 seeded steps",
    2: "scale: 1024 envs x 2 pads x 40x50, 5 objects at 128^3",
    3: "roofline: 8192 envs x 2 pads x 80x100, 8 objects at 256^3, ~70% contact",
    4: "batched uneven: 4096 envs, pads {20x25,40x50,80x100}, grids {64,128,256}^3 x 8 objects, 100 substeps",
    5: "differentiation: 1024 envs x 2 pads x 40x50, 5 objects at 128^3, seeded loss weights",
}


def make_c1(step: int = 0) -> Scene:
    """One pad of 20x25 taxels at 1 mm pitch against a r = 10 mm sphere."""
    return build_scene("c1", 1, step, ["sphere10"], [64], [(20, 25)], pads_per_env=1,
                       pen_range=(0.0, 1 * MM), vmax=0.05,
                       grid_spacing={("sphere10", 64): 0.5 * MM})


def make_c2(n_env: int = 1024, res=(40, 50), grid: int = 128, cfg_id: int = 2) -> Scene:
    rng = rng_for(cfg_id, 1000)
    objs = [FIVE_OBJECTS[k] for k in rng.integers(0, 5, n_env)]
    return build_scene(f"c{cfg_id}", cfg_id, 0, objs, [grid] * n_env, [res] * n_env,
                       pen_range=(0.0, 2 * MM), vmax=0.1)


C3_PEN_CAP = 4 * MM
C3_FRAC_TARGET = 0.8


def make_c3(n_env: int = 8192, res=(80, 100), grid: int = 256) -> Scene:
    objs = [EIGHT_OBJECTS[e % 8] for e in range(n_env)]
    # ~70% of taxels in contact on average: narrow objects (16 mm pegs, the
    # torus tube) cap what a 20x25 mm pad can touch, and the curved ones need
    # 2.5-4 mm of penetration, so each pad aims at 80% with a 4 mm cap
    # (realized mean ~0.66)
    return build_scene("c3", 3, 0, objs, [grid] * n_env, [res] * n_env,
                       frac_target=C3_FRAC_TARGET, pen_cap=C3_PEN_CAP, vmax=0.1,
                       placement_subsample=(16, 20))


C4_RES = [(20, 25), (40, 50), (80, 100)]
C4_GRIDS = [64, 128, 256]
C4_DT = 1e-4
C4_SUBSTEPS = 100


def make_c4(n_env: int = 4096, substeps: int = C4_SUBSTEPS, grids=C4_GRIDS) -> Scene:
    """Uneven batch; object positions advance by v * dt per substep (pads at rest)."""
    rng = rng_for(4, 1000)
    objs = [EIGHT_OBJECTS[k] for k in rng.integers(0, 8, n_env)]
    res = [C4_RES[k] for k in rng.integers(0, 3, n_env)]
    gr = [grids[k] for k in rng.integers(0, len(grids), n_env)]
    sc = build_scene("c4", 4, 0, objs, gr, res, pen_range=(1 * MM, 1 * MM), vmax=0.1,
                     placement_subsample=(10, 12))
    v = sc.obj_twist[:, :3].astype(np.float64)
    base = sc.obj_pose.astype(np.float64)
    steps = np.repeat(base[None], substeps, axis=0)
    s = np.arange(substeps, dtype=np.float64)[:, None, None]
    steps[:, :, 4:7] = base[None, :, 4:7] + v[None] * (s * C4_DT)
    sc.obj_pose_steps = steps.astype(np.float32)
    sc.meta["dt"] = C4_DT
    sc.meta["groups"] = sorted({(r, g) for r, g in zip(res, gr)})
    return sc


def make_c5(n_env: int = 1024) -> Scene:
    return make_c2(n_env=n_env, cfg_id=5)


def loss_weights(n_taxels: int, seed: int = 5):
    """Seeded N(0,1) weights a (for f_n) and b (for f_t), float32 [3][T] each."""
    rng = rng_for(5, 2000 + seed)
    a = rng.standard_normal((3, n_taxels)).astype(np.float32)
    b = rng.standard_normal((3, n_taxels)).astype(np.float32)
    return a, b


def make_small(cfg_id: int = 11, n_env: int = 6, grid: int = 48, res=(37, 23),
               objs=None, wmax=0.5, pad_vmax=0.05, pad_wmax=0.3, step: int = 0) -> Scene:
    """A reduced scene for oracle-sized parity: ragged template, rotations on."""
    objs = objs or [EIGHT_OBJECTS[e % 8] for e in range(n_env)]
    return build_scene(f"small{cfg_id}", cfg_id, step, objs, [grid] * n_env, [res] * n_env,
                       pen_range=(0.2 * MM, 2 * MM), vmax=0.1, wmax=wmax,
                       pad_vmax=pad_vmax, pad_wmax=pad_wmax)


def make_uneven_small(cfg_id: int = 12, n_env: int = 12, substeps: int = 3) -> Scene:
    """A reduced uneven batch (3 pad resolutions x 3 grid sizes) with substeps."""
    rng = rng_for(cfg_id, 1000)
    objs = [EIGHT_OBJECTS[k] for k in rng.integers(0, 8, n_env)]
    res_choices = [(7, 9), (20, 25), (31, 17)]
    grid_choices = [24, 40, 56]
    res = [res_choices[e % 3] for e in range(n_env)]
    gr = [grid_choices[(e // 3) % 3] for e in range(n_env)]
    sc = build_scene(f"uneven{cfg_id}", cfg_id, 0, objs, gr, res, pen_range=(0.5 * MM, 1.5 * MM),
                     vmax=0.1, wmax=0.3)
    v = sc.obj_twist[:, :3].astype(np.float64)
    base = sc.obj_pose.astype(np.float64)
    steps = np.repeat(base[None], substeps, axis=0)
    s = np.arange(substeps, dtype=np.float64)[:, None, None]
    steps[:, :, 4:7] = base[None, :, 4:7] + v[None] * (s * C4_DT)
    sc.obj_pose_steps = steps.astype(np.float32)
    return sc


def subset_scene(scene: Scene, envs: Sequence[int], name: Optional[str] = None) -> Scene:
    """The environments ``envs`` of ``scene`` (with their pads, grids and
    templates) as a scene of their own; pads keep their relative order."""
    envs = np.asarray(envs, dtype=np.int64)
    emap = -np.ones(scene.n_env, np.int64)
    emap[envs] = np.arange(envs.size)
    insts = np.flatnonzero(emap[scene.inst_env] >= 0)
    sdf_used = np.unique(scene.env_sdf[envs])
    smap = -np.ones(scene.n_sdf, np.int64)
    smap[sdf_used] = np.arange(sdf_used.size)
    tmpl_used = np.unique(scene.inst_tmpl[insts])
    tmap = -np.ones(scene.n_tmpl, np.int64)
    tmap[tmpl_used] = np.arange(tmpl_used.size)
    sizes = (scene.sdf_dims[:, 0].astype(np.int64) * scene.sdf_dims[:, 1] * scene.sdf_dims[:, 2])
    datas = [scene.sdf_data[scene.sdf_offset[g]:scene.sdf_offset[g] + sizes[g]] for g in sdf_used]
    offs = np.concatenate([[0], np.cumsum([d.size for d in datas])[:-1]]).astype(np.int64)
    tparts = [scene.tmpl_xyz[:, scene.tmpl_offset[p]:scene.tmpl_offset[p + 1]] for p in tmpl_used]
    toff = np.concatenate([[0], np.cumsum([t.shape[1] for t in tparts])]).astype(np.int64)
    sub = Scene(
        name=name or f"{scene.name}-sub", n_env=int(envs.size), n_inst=int(insts.size),
        inst_env=emap[scene.inst_env[insts]].astype(np.int32), inst_tmpl=tmap[scene.inst_tmpl[insts]].astype(np.int32),
        env_sdf=smap[scene.env_sdf[envs]].astype(np.int32), tmpl_offset=toff,
        tmpl_xyz=np.concatenate(tparts, axis=1) if tparts else np.zeros((3, 0), np.float32),
        sdf_dims=scene.sdf_dims[sdf_used].copy(), sdf_origin=scene.sdf_origin[sdf_used].copy(),
        sdf_spacing=scene.sdf_spacing[sdf_used].copy(), sdf_offset=offs,
        sdf_data=np.concatenate(datas) if datas else np.zeros(0, np.float32),
        pad_pose=scene.pad_pose[insts].copy(), obj_pose=scene.obj_pose[envs].copy(),
        pad_twist=scene.pad_twist[insts].copy(), obj_twist=scene.obj_twist[envs].copy(),
        params=scene.params[envs].copy(), sdf_names=[scene.sdf_names[g] for g in sdf_used] if scene.sdf_names else [],
        tmpl_names=[scene.tmpl_names[p] for p in tmpl_used] if scene.tmpl_names else [],
        obj_pose_steps=None if scene.obj_pose_steps is None else scene.obj_pose_steps[:, envs].copy(),
        meta=dict(scene.meta, parent=scene.name, envs=envs, insts=insts))
    return sub


def c4_groups(scene: Scene):
    """Environments of the uneven batch grouped by (pad resolution, grid size)."""
    keys = {}
    for e in range(scene.n_env):
        i = int(np.flatnonzero(scene.inst_env == e)[0])
        key = (int(np.diff(scene.tmpl_offset)[scene.inst_tmpl[i]]), tuple(scene.sdf_dims[scene.env_sdf[e]]))
        keys.setdefault(key, []).append(e)
    return [np.asarray(v) for _, v in sorted(keys.items())]


# ---------------------------------------------------------------------------
# Contact batches for the implicit soft-contact impulse (Section III-A).
# Only draws: contacts grouped by environment as a contact buffer lists them,
# stiffness and damping per environment from the randomization ranges of
# Appendix C (kappa in [150, 350] N/m, c in [0, 1] N s/m).
# ---------------------------------------------------------------------------
IMPULSE_DT = 1.0 / 240.0  # one substep of a 60 Hz frame split in 4


@dataclasses.dataclass
class Contacts:
    eps: np.ndarray       # [n] contact distance (m), negative when interpenetrating
    eps_dot: np.ndarray   # [n] separation velocity (m/s)
    inv_mass: np.ndarray  # [n] inverse effective inertia (1/kg), 0 for an immovable body
    env: np.ndarray       # [n] int32 environment of each contact (non-decreasing)
    kc: np.ndarray        # [n_env, 2] (kappa, c)
    dt: float

    @property
    def n(self) -> int:
        return int(self.eps.size)


def make_contacts(n_env: int, per_env: int, seed: int = 31, dt: float = IMPULSE_DT, ragged: bool = False) -> Contacts:
    """Seeded contact batch: `per_env` contacts per environment (on average when
    ragged), 75 % interpenetrating by up to 4 mm, the rest up to 2 mm apart
    (speculative contacts); separation velocities ~ N(0, 5 cm/s); effective
    masses of 0.02 - 0.5 kg, one contact in ten against an immovable body."""
    rng = np.random.default_rng(seed)
    if ragged:
        counts = rng.integers(0, 2 * per_env + 1, n_env)
    else:
        counts = np.full(n_env, per_env)
    env = np.repeat(np.arange(n_env, dtype=np.int32), counts)
    n = env.size
    inside = rng.random(n) < 0.75
    eps = np.where(inside, -rng.uniform(0.0, 4 * MM, n), rng.uniform(0.0, 2 * MM, n)).astype(np.float32)
    eps_dot = rng.normal(0.0, 0.05, n).astype(np.float32)
    inv_mass = (1.0 / rng.uniform(0.02, 0.5, n)).astype(np.float32)
    inv_mass[rng.random(n) < 0.1] = 0.0
    kc = np.stack([rng.uniform(150.0, 350.0, n_env), rng.uniform(0.0, 1.0, n_env)], 1).astype(np.float32)
    return Contacts(eps, eps_dot, inv_mass, env, kc, float(dt))


# ---------------------------------------------------------------------------
# Observation layout: the 14 x 10 x 3 force-field observation per finger of
# Section V-B.  Bins split the pad's taxel grid into bins_y rows (along the
# 25 mm pad height) by bins_x columns (along the 20 mm width); a taxel at grid
# position (j, i) belongs to bin (j * bins_y // ny) * bins_x + (i * bins_x // nx).
# ---------------------------------------------------------------------------
OBS_BINS_X = 10
OBS_BINS_Y = 14


def pad_observation_bins(nx: int, ny: int, bins_x: int = OBS_BINS_X, bins_y: int = OBS_BINS_Y,
                         block: int = TAXEL_BLOCK) -> np.ndarray:
    """Bin of every template taxel of an nx x ny pad (template numbering)."""
    ji = taxel_grid_index(nx, ny, block)
    return ((ji[:, 0] * bins_y // ny) * bins_x + (ji[:, 1] * bins_x // nx)).astype(np.int32)


def scene_observation_bins(scene: Scene, bins_x: int = OBS_BINS_X, bins_y: int = OBS_BINS_Y) -> np.ndarray:
    """Concatenated bin maps of the scene's templates (named "<nx>x<ny>")."""
    parts = []
    for name in scene.tmpl_names:
        nx, ny = (int(v) for v in name.split("x"))
        parts.append(pad_observation_bins(nx, ny, bins_x, bins_y))
    return np.concatenate(parts) if parts else np.zeros(0, np.int32)
