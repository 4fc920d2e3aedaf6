"""FP64 CPU oracle of the tactile force field -- test infrastructure only.

A plain, step-by-step evaluation of the penalty force field of Section III-C
(SDF query at the tactile points, finite-difference normal, normal spring with
depth-scaled damping, Coulomb-capped friction) written in C++ (FP64) and
driven through ctypes.  It is used by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, and by nothing else; it shares no code with
the HIP library.  Every function is pinned in tests/test_oracle_*.py against
closed forms, invariants, special cases and hand-derived worked examples.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tacsl_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(ctypes.Structure):
    _fields_ = [("n_env", ctypes.c_int32), ("n_inst", ctypes.c_int32),
                ("n_tmpl", ctypes.c_int32), ("n_sdf", ctypes.c_int32),
                ("inst_env", ctypes.c_void_p), ("inst_tmpl", ctypes.c_void_p),
                ("env_sdf", ctypes.c_void_p), ("tmpl_offset", ctypes.c_void_p),
                ("tmpl_xyz", ctypes.c_void_p), ("sdf_dims", ctypes.c_void_p),
                ("sdf_origin", ctypes.c_void_p), ("sdf_spacing", ctypes.c_void_p),
                ("sdf_offset", ctypes.c_void_p), ("sdf_data", ctypes.c_void_p)]


class _State(ctypes.Structure):
    _fields_ = [("pad_pose", ctypes.c_void_p), ("obj_pose", ctypes.c_void_p),
                ("pad_twist", ctypes.c_void_p), ("obj_twist", ctypes.c_void_p),
                ("params", ctypes.c_void_p), ("obj_pose_delta", ctypes.c_void_p),
                ("normal_exponent", ctypes.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_offsets.argtypes = [P, P]
        lib.oracle_force_field.argtypes = [P, P, ctypes.c_int, P, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_grad.argtypes = [P, P, P, P, P, ctypes.c_int, P, P, P, P, ctypes.c_int]
        lib.oracle_loss.argtypes = [P, P, P, P, P, ctypes.c_int, P, P, ctypes.c_int]
        lib.oracle_signature.argtypes = [P, P, P, ctypes.c_int]
        lib.oracle_decision_values.argtypes = [P, P, P, ctypes.c_int]
        lib.oracle_footprint.argtypes = [P, P, ctypes.c_int, P]
        lib.oracle_footprint.restype = ctypes.c_int64
        lib.oracle_depth_image.argtypes = [P, P, P, ctypes.c_int, P, P, P, P, ctypes.c_int]
        lib.oracle_contact_impulse.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_double, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Bound:
    """Keeps the numpy buffers alive while the C structs point at them."""

    def __init__(self, scene, state):
        self.keep = []

        def c(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self.keep.append(a)
            return a

        self.sc = _Scene(
            int(scene.n_env), int(scene.n_inst), int(scene.tmpl_offset.size - 1), int(scene.sdf_spacing.size),
            _ptr(c(scene.inst_env, np.int32)), _ptr(c(scene.inst_tmpl, np.int32)),
            _ptr(c(scene.env_sdf, np.int32)), _ptr(c(scene.tmpl_offset, np.int64)),
            _ptr(c(scene.tmpl_xyz, np.float32)), _ptr(c(scene.sdf_dims, np.int32)),
            _ptr(c(scene.sdf_origin, np.float32)), _ptr(c(scene.sdf_spacing, np.float32)),
            _ptr(c(scene.sdf_offset, np.int64)), _ptr(c(scene.sdf_data, np.float32)))
        delta = state.get("obj_pose_delta")
        self.st = _State(
            _ptr(c(state["pad_pose"], np.float64)), _ptr(c(state["obj_pose"], np.float64)),
            _ptr(c(state["pad_twist"], np.float64)), _ptr(c(state["obj_twist"], np.float64)),
            _ptr(c(state["params"], np.float64)),
            None if delta is None else _ptr(c(delta, np.float64)),
            float(state.get("normal_exponent", 1.0)))


def offsets(scene):
    b = _Bound(scene, _dummy_state(scene))
    out = np.zeros(scene.n_inst + 1, dtype=np.int64)
    _load().oracle_offsets(ctypes.byref(b.sc), _ptr(out))
    return out


def _dummy_state(scene):
    return dict(pad_pose=np.zeros((scene.n_inst, 7)), obj_pose=np.zeros((scene.n_env, 7)),
                pad_twist=np.zeros((scene.n_inst, 6)), obj_twist=np.zeros((scene.n_env, 6)),
                params=np.zeros((scene.n_env, 4)))


def force_field(scene, state, sel=None, nthreads=0, signature=False):
    """Evaluate the selected instances (default: all).  Returns a dict of FP64 arrays.

    ``state`` holds pad_pose, obj_pose, pad_twist, obj_twist, params and an
    optional obj_pose_delta, each widened to FP64 (pass the FP32 inputs of the
    GPU path to compare like with like), and optionally normal_exponent (the
    power p of the penetration in the normal law, 1 by default).
    """
    if sel is None:
        sel = np.arange(scene.n_inst, dtype=np.int32)
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    counts = np.diff(scene.tmpl_offset)[scene.inst_tmpl[sel]]
    Ts = int(counts.sum())
    b = _Bound(scene, state)
    out = dict(depth=np.zeros(Ts), normal=np.zeros((3, Ts)), fn=np.zeros((3, Ts)),
               ft=np.zeros((3, Ts)), wrench=np.zeros((sel.size, 6)))
    sig = np.zeros((Ts, 4), dtype=np.int32) if signature else None
    _load().oracle_force_field(ctypes.byref(b.sc), ctypes.byref(b.st), int(sel.size), _ptr(sel),
                               _ptr(out["depth"]), _ptr(out["normal"]), _ptr(out["fn"]),
                               _ptr(out["ft"]), _ptr(out["wrench"]), _ptr(sig), int(nthreads))
    if signature:
        out["sig"] = sig
    return out


def grad(scene, state, wa, wb, sel_env=None, mask=None, nthreads=0, with_abs=False):
    """Loss per selected env and its 16-direction gradient (dual numbers).

    Columns: dt(3), dtheta(3), v_o(3), w_o(3), k_n, k_d, k_t, mu.  With
    ``with_abs`` also returns, per env and column, the sum over taxels of the
    absolute per-taxel contributions (the scale of a cancelling sum).
    """
    if sel_env is None:
        sel_env = np.arange(scene.n_env, dtype=np.int32)
    sel_env = np.ascontiguousarray(sel_env, dtype=np.int32)
    b = _Bound(scene, state)
    wa = np.ascontiguousarray(wa, dtype=np.float64)
    wb = np.ascontiguousarray(wb, dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    loss = np.zeros(sel_env.size)
    g = np.zeros((sel_env.size, 16))
    gabs = np.zeros((sel_env.size, 16)) if with_abs else None
    _load().oracle_grad(ctypes.byref(b.sc), ctypes.byref(b.st), _ptr(wa), _ptr(wb), _ptr(m),
                        int(sel_env.size), _ptr(sel_env), _ptr(loss), _ptr(g), _ptr(gabs), int(nthreads))
    if with_abs:
        return loss, g, gabs
    return loss, g


def loss(scene, state, wa, wb, sel_env=None, mask=None, nthreads=0):
    if sel_env is None:
        sel_env = np.arange(scene.n_env, dtype=np.int32)
    sel_env = np.ascontiguousarray(sel_env, dtype=np.int32)
    b = _Bound(scene, state)
    wa = np.ascontiguousarray(wa, dtype=np.float64)
    wb = np.ascontiguousarray(wb, dtype=np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    out = np.zeros(sel_env.size)
    _load().oracle_loss(ctypes.byref(b.sc), ctypes.byref(b.st), _ptr(wa), _ptr(wb), _ptr(m),
                        int(sel_env.size), _ptr(sel_env), _ptr(out), int(nthreads))
    return out


def signature(scene, state, nthreads=0):
    b = _Bound(scene, state)
    T = int(np.diff(scene.tmpl_offset)[scene.inst_tmpl].sum())
    sig = np.zeros((T, 4), dtype=np.int32)
    _load().oracle_signature(ctypes.byref(b.sc), ctypes.byref(b.st), _ptr(sig), int(nthreads))
    return sig


def decision_values(scene, state, nthreads=0):
    """Per taxel (global order) the FP64 values the force law's discrete
    decisions compare: columns (phi, |g|, k_t |v_t|, mu |s|) and the
    sensitivity of the friction cap to phi, |d(mu |s|)/d phi|; NaN where the
    step is not reached (Section III-C: contact where the SDF is negative, a
    degenerate gradient, and the friction min(k_t |v_t|, mu |f_n|))."""
    b = _Bound(scene, state)
    T = int(np.diff(scene.tmpl_offset)[scene.inst_tmpl].sum())
    m = np.zeros((T, 5), dtype=np.float64)
    _load().oracle_decision_values(ctypes.byref(b.sc), ctypes.byref(b.st), _ptr(m), int(nthreads))
    return m


def footprint(scene, state, sel=None):
    if sel is None:
        sel = np.arange(scene.n_inst, dtype=np.int32)
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    b = _Bound(scene, state)
    return int(_load().oracle_footprint(ctypes.byref(b.sc), ctypes.byref(b.st), int(sel.size), _ptr(sel)))


def state64(scene, step=None, obj_pose_delta=None):
    """The scene's FP32 state widened to FP64 (what the GPU path consumes)."""
    st = {k: np.asarray(v, dtype=np.float64) for k, v in scene.state(step).items()}
    if obj_pose_delta is not None:
        st["obj_pose_delta"] = np.asarray(obj_pose_delta, dtype=np.float64)
    return st


def contact_impulse(eps, epsdot, inv_mass, env, kc, dt):
    """Implicit soft-contact impulse per contact (Section III-A); FP64 arrays."""
    eps = np.ascontiguousarray(eps, np.float64)
    epsdot = np.ascontiguousarray(epsdot, np.float64)
    inv_mass = np.ascontiguousarray(inv_mass, np.float64)
    env = None if env is None else np.ascontiguousarray(env, np.int32)
    kc = np.ascontiguousarray(kc, np.float64).reshape(-1, 2)
    lam = np.zeros(eps.size)
    dv = np.zeros(eps.size)
    _load().oracle_contact_impulse(int(eps.size), _ptr(eps), _ptr(epsdot), _ptr(inv_mass), _ptr(env), _ptr(kc),
                                   float(dt), _ptr(lam), _ptr(dv))
    return lam, dv


def observation(scene, ff, tmpl_bin, n_bins, scale=(1.0, 1.0, 1.0), clip=0.0, sel=None):
    """Force-field observation per pad (the 14 x 10 x 3 policy input of
    Section V-B): channels (|f_n|, f_t,x, f_t,y) of the pad-frame forces,
    averaged over the taxels of each bin, divided by the channel scale and
    clipped to [-clip, clip] (clip <= 0: no clipping); an empty bin is 0.

    ``ff`` is the output of ``force_field`` for the same ``sel`` (taxel rows
    instance-major); ``tmpl_bin`` gives the bin of each template taxel (-1:
    none).  Returns FP64 [n_sel][n_bins][3]."""
    sel = np.arange(scene.n_inst) if sel is None else np.asarray(sel)
    tmpl_bin = np.asarray(tmpl_bin)
    scale = np.asarray(scale, np.float64)
    obs = np.zeros((sel.size, n_bins, 3))
    row = 0
    for s, i in enumerate(sel):
        p = scene.inst_tmpl[i]
        a, b = int(scene.tmpl_offset[p]), int(scene.tmpl_offset[p + 1])
        cnt = b - a
        bins = tmpl_bin[a:b]
        fn = ff["fn"][:, row:row + cnt]
        ft = ff["ft"][:, row:row + cnt]
        row += cnt
        ch = np.stack([np.linalg.norm(fn, axis=0), ft[0], ft[1]], axis=1)
        m = bins >= 0
        counts = np.bincount(bins[m], minlength=n_bins)
        for c in range(3):
            sums = np.bincount(bins[m], weights=ch[m, c], minlength=n_bins)
            mean = np.divide(sums, counts, out=np.zeros(n_bins), where=counts > 0)
            obs[s, :, c] = mean / scale[c]
    if clip > 0:
        obs = np.clip(obs, -clip, clip)
    return obs


class Camera(ctypes.Structure):
    """Tactile camera: pixel (r, c) looks through the pad-plane point
    (x0 + (c + 1/2) dx, y0 + (r + 1/2) dy, 0); pinhole at (0, 0, -cam_dist)
    unless ortho; the gel spans z in [-gel, 0]."""
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("ortho", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("cam_dist", ctypes.c_double), ("gel", ctypes.c_double)]


def depth_image(scene, state, cam, sel=None, nthreads=0):
    """Tactile depth image per selected pad (Section III-B): z-distance from the
    camera plane to the first point inside the gel where the object's trilinear
    SDF is <= 0, else to the gel surface.  Returns (image, slope, phimin), each
    FP64 [n_sel][rows][cols]; slope = d(phi)/dz at the hit (0 without one),
    phimin = smallest phi sampled along the searched ray segment."""
    if sel is None:
        sel = np.arange(scene.n_inst, dtype=np.int32)
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    b = _Bound(scene, state)
    shape = (sel.size, cam.rows, cam.cols)
    img, sl, pm = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    _load().oracle_depth_image(ctypes.byref(b.sc), ctypes.byref(b.st), ctypes.byref(cam), int(sel.size), _ptr(sel),
                               _ptr(img), _ptr(sl), _ptr(pm), int(nthreads))
    return img, sl, pm


def pose_path(pose0, twist, t):
    """Object poses after moving for time ``t`` at a constant twist (FP64):
    the origin moves at the constant velocity v, t_o(t) = t_o + v t, and the
    body turns at the constant world-frame angular velocity w,
    R_o(t) = Exp(w t) R_o, i.e. q(t) = q_w(t) q_0 (Hamilton product) with
    q_w(t) = (cos(|w| t / 2), sin(|w| t / 2) w / |w|).  This is the seeded
    pose update of the substep loop of the batched workload (the state a
    simulator hands to the tactile step after each dynamics step, notation
    appendix).  pose0 [E][7] = (qw qx qy qz tx ty tz), twist [E][6] = (v, w)."""
    p0 = np.asarray(pose0, dtype=np.float64).reshape(-1, 7)
    tw = np.asarray(twist, dtype=np.float64).reshape(-1, 6)
    t = float(t)
    trans = p0[:, 4:7] + tw[:, :3] * t
    rv = tw[:, 3:6] * t
    ang = np.linalg.norm(rv, axis=1)
    half = 0.5 * ang
    # sin(|a|/2)/|a| = sinc(|a| / (2 pi)) / 2, well defined at a = 0
    s = 0.5 * np.sinc(half / np.pi)
    qe = np.concatenate([np.cos(half)[:, None], s[:, None] * rv], axis=1)
    w1, x1, y1, z1 = qe.T
    w2, x2, y2, z2 = p0[:, :4].T
    q = np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                  w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                  w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                  w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], axis=1)
    return np.concatenate([q, trans], axis=1)
