"""Python binding over libtacsl: plans, forward/backward calls, autograd, graphs.

PyTorch supplies device memory and streams; every step of the force field
runs in the library's HIP kernels.  The calls are asynchronous on the current
torch stream.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _abi

STATE_KEYS = ("pad_pose", "obj_pose", "pad_twist", "obj_twist", "params")


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(x, device):
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=torch.float32)
        return t.contiguous()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device=device)


def tuning(block=0, tile_taxels=0, schedule=0, grid=0, order=0) -> _abi.Tuning:
    return _abi.Tuning(int(block), int(tile_taxels), int(schedule), int(grid), int(order))


def _tuning_obj(t):
    if t is None:
        return None
    if isinstance(t, _abi.Tuning):
        return t
    return tuning(**t)


class _HostScene:
    """Host-side arrays of a scene plus the ctypes descriptor pointing at them."""

    def __init__(self, scene, tmpl_dev_ptr=None, sdf_dev_ptr=None):
        self.inst_env = _np(scene.inst_env, np.int32)
        self.inst_tmpl = _np(scene.inst_tmpl, np.int32)
        self.env_sdf = _np(scene.env_sdf, np.int32)
        self.tmpl_offset = _np(scene.tmpl_offset, np.int64)
        self.sdf_dims = _np(scene.sdf_dims, np.int32).reshape(-1, 3)
        self.sdf_origin = _np(scene.sdf_origin, np.float32).reshape(-1, 3)
        self.sdf_spacing = _np(scene.sdf_spacing, np.float32).reshape(-1)
        self.sdf_offset = _np(scene.sdf_offset, np.int64).reshape(-1)
        self.n_env = int(scene.n_env)
        self.n_inst = int(scene.n_inst)
        self.desc = _abi.SceneDesc(
            self.n_env, self.n_inst, int(self.tmpl_offset.size - 1), int(self.sdf_spacing.size),
            self.inst_env.ctypes.data, self.inst_tmpl.ctypes.data, self.env_sdf.ctypes.data,
            self.tmpl_offset.ctypes.data, tmpl_dev_ptr, self.sdf_dims.ctypes.data,
            self.sdf_origin.ctypes.data, self.sdf_spacing.ctypes.data, self.sdf_offset.ctypes.data,
            sdf_dev_ptr)


def validate_scene(scene, tmpl_ptr=1, sdf_ptr=1) -> int:
    """Host-only validation (no GPU).  Device pointers are only checked for NULL."""
    lib = _abi.load()
    hs = _HostScene(scene, tmpl_ptr, sdf_ptr)
    return int(lib.tacsl_validate_scene(ctypes.byref(hs.desc)))


def build_worklist(scene, tun=None, xcd_count=8):
    """Host-only tile work list of ``scene`` (see tacsl_build_worklist)."""
    lib = _abi.load()
    hs = _HostScene(scene, 1, 1)
    t = _tuning_obj(tun)
    n = ctypes.c_int64(0)
    tref = ctypes.byref(t) if t is not None else None
    _abi.check(lib.tacsl_build_worklist(ctypes.byref(hs.desc), tref, xcd_count, 0, ctypes.byref(n),
                                        None, None, None, None), "tacsl_build_worklist")
    m = n.value
    inst = np.zeros(max(m, 1), np.int32)
    k0 = np.zeros(max(m, 1), np.int32)
    cnt = np.zeros(max(m, 1), np.int32)
    order = np.zeros(max(m, 1), np.int32)
    _abi.check(lib.tacsl_build_worklist(ctypes.byref(hs.desc), tref, xcd_count, m, ctypes.byref(n),
                                        inst.ctypes.data, k0.ctypes.data, cnt.ctypes.data,
                                        order.ctypes.data), "tacsl_build_worklist")
    return dict(inst=inst[:m], k0=k0[:m], count=cnt[:m], order=order[:m])


class Plan:
    """A scene prepared on the current GPU (libtacsl plan).

    ``scene`` is any object with the host arrays of a scene description
    (inst_env, inst_tmpl, env_sdf, tmpl_offset, tmpl_xyz, sdf_dims,
    sdf_origin, sdf_spacing, sdf_offset, sdf_data, n_env, n_inst), e.g.
    ``workloads.Scene``.  Template positions and SDF node values are only
    needed while the plan is created (the plan keeps its own copies).
    """

    def __init__(self, scene, tun=None, device="cuda"):
        self._lib = _abi.load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._plan = ctypes.c_void_p(None)
        tmpl = torch.as_tensor(_np(scene.tmpl_xyz, np.float32).reshape(3, -1), device=self.device)
        sdf = torch.as_tensor(_np(scene.sdf_data, np.float32).reshape(-1), device=self.device)
        self._hs = _HostScene(scene, tmpl.data_ptr() if tmpl.numel() else None,
                              sdf.data_ptr() if sdf.numel() else None)
        t = _tuning_obj(tun)
        with torch.cuda.device(self.device):
            torch.cuda.synchronize()
            _abi.check(self._lib.tacsl_plan_create(ctypes.byref(self._hs.desc),
                                                   ctypes.byref(t) if t is not None else None,
                                                   ctypes.byref(self._plan)), "tacsl_plan_create")
        del sdf, tmpl
        self.n_env = self._hs.n_env
        self.n_inst = self._hs.n_inst
        info = self.info()
        self.n_taxels = int(info.n_taxels)
        self._tmpl_T = int(self._hs.tmpl_offset[-1]) if self._hs.tmpl_offset.size else 0
        self.obs_bins = 0
        self._cam = None
        self._graphs: List["SubstepGraph"] = []

    # -- inspection --------------------------------------------------------
    def info(self) -> _abi.PlanInfo:
        info = _abi.PlanInfo()
        _abi.check(self._lib.tacsl_plan_get_info(self._plan, ctypes.byref(info)), "tacsl_plan_get_info")
        return info

    def offsets(self) -> np.ndarray:
        out = np.zeros(self.n_inst + 1, np.int64)
        _abi.check(self._lib.tacsl_plan_offsets(self._plan, out.ctypes.data), "tacsl_plan_offsets")
        return out

    def set_tuning(self, tun):
        t = _tuning_obj(tun)
        with torch.cuda.device(self.device):
            _abi.check(self._lib.tacsl_plan_set_tuning(self._plan, ctypes.byref(t)), "tacsl_plan_set_tuning")

    @property
    def tuning(self) -> Dict[str, int]:
        return self.info().tuning.as_dict()

    def timer_start(self, capacity: int):
        """Record the main kernel's duration for the next ``capacity`` calls."""
        _abi.check(self._lib.tacsl_plan_timer_start(self._plan, int(capacity)), "tacsl_plan_timer_start")

    def timer_read(self, capacity: int) -> np.ndarray:
        ms = np.zeros(max(int(capacity), 1), np.float32)
        n = ctypes.c_int32(0)
        _abi.check(self._lib.tacsl_plan_timer_read(self._plan, int(capacity), ctypes.byref(n), ms.ctypes.data),
                   "tacsl_plan_timer_read")
        return ms[:n.value].astype(np.float64)

    # -- calls -------------------------------------------------------------
    def state(self, st: Dict[str, object], obj_pose_delta=None) -> Dict[str, torch.Tensor]:
        """Move a state dict (numpy or tensors) to device FP32 tensors."""
        out = {k: _dev_f32(st[k], self.device) for k in STATE_KEYS}
        d = obj_pose_delta if obj_pose_delta is not None else st.get("obj_pose_delta")
        if d is not None:
            out["obj_pose_delta"] = _dev_f32(d, self.device)
        return out

    def _check_state(self, st):
        shapes = dict(pad_pose=(self.n_inst, 7), obj_pose=(self.n_env, 7), pad_twist=(self.n_inst, 6),
                      obj_twist=(self.n_env, 6), params=(self.n_env, 4), obj_pose_delta=(self.n_env, 6))
        for k, shp in shapes.items():
            t = st.get(k)
            if t is None:
                if k == "obj_pose_delta":
                    continue
                raise ValueError(f"state is missing {k}")
            if (not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous()
                    or tuple(t.shape) != shp or t.device != self.device):
                raise ValueError(f"state[{k}] must be a contiguous float32 {shp} tensor on {self.device}")

    def _state_struct(self, st):
        return _abi.State(*(_ptr(st.get(k)) for k in STATE_KEYS + ("obj_pose_delta",)))

    def new_outputs(self) -> Dict[str, torch.Tensor]:
        T = self.n_taxels
        f = dict(device=self.device, dtype=torch.float32)
        return dict(depth=torch.empty(T, **f), normal=torch.empty(3, T, **f), fn=torch.empty(3, T, **f),
                    ft=torch.empty(3, T, **f), wrench=torch.empty(self.n_inst, 6, **f),
                    status=torch.zeros(1, device=self.device, dtype=torch.int32))

    def _check_outputs(self, out):
        T = self.n_taxels
        shapes = dict(depth=(T,), normal=(3, T), fn=(3, T), ft=(3, T), wrench=(self.n_inst, 6))
        for k, shp in shapes.items():
            t = out[k]
            if (t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != shp
                    or t.device != self.device):
                raise ValueError(f"outputs[{k}] must be a contiguous float32 {shp} tensor on {self.device}")

    def _out_struct(self, out):
        return _abi.Outputs(*(_ptr(out.get(k)) for k in ("depth", "normal", "fn", "ft", "wrench", "status")))

    def forward(self, st: Dict[str, torch.Tensor], out: Optional[Dict[str, torch.Tensor]] = None,
                stream=None) -> Dict[str, torch.Tensor]:
        self._check_state(st)
        if out is None:
            out = self.new_outputs()
        self._check_outputs(out)
        s = self._state_struct(st)
        o = self._out_struct(out)
        _abi.check(self._lib.tacsl_force_field(self._plan, ctypes.byref(s), ctypes.byref(o),
                                               _stream_handle(stream)), "tacsl_force_field")
        return out

    def forward_noalloc(self, st: Dict[str, torch.Tensor], out: Dict[str, torch.Tensor],
                        stream=None) -> Dict[str, torch.Tensor]:
        """Forward through tacsl_force_field_noalloc: the call's work buffers
        come from the library's static device scratch (nothing is allocated;
        calls on one GPU must not overlap).  ``out`` is required."""
        self._check_state(st)
        self._check_outputs(out)
        s = self._state_struct(st)
        o = self._out_struct(out)
        _abi.check(self._lib.tacsl_force_field_noalloc(self._plan, ctypes.byref(s), ctypes.byref(o),
                                                       _stream_handle(stream)), "tacsl_force_field_noalloc")
        return out

    def set_observation(self, tmpl_bin, n_bins: int, scale=(1.0, 1.0, 1.0), clip: float = 0.0):
        """Install the observation epilogue: per pad and bin the mean of
        (|f_n|, f_t,x, f_t,y) over the bin's taxels, / scale, clipped to +-clip.
        ``tmpl_bin``: int32 bin of each template taxel (-1: none); n_bins = 0 removes it."""
        tb = np.zeros(0, np.int32) if tmpl_bin is None else _np(tmpl_bin, np.int32).reshape(-1)
        if n_bins and tb.size != self._tmpl_T:
            raise ValueError(f"tmpl_bin must hold {self._tmpl_T} entries")
        sc = _np(scale, np.float32).reshape(3)
        _abi.check(self._lib.tacsl_plan_set_observation(self._plan, int(n_bins), tb.ctypes.data if tb.size else None,
                                                        sc.ctypes.data,
                                                        float(clip)), "tacsl_plan_set_observation")
        self.obs_bins = int(n_bins)

    def new_observation(self) -> torch.Tensor:
        return torch.empty(self.n_inst, self.obs_bins, 3, device=self.device, dtype=torch.float32)

    def observe(self, st: Dict[str, torch.Tensor], obs: Optional[torch.Tensor] = None,
                out: Optional[Dict[str, torch.Tensor]] = None, fields: bool = False, stream=None):
        """Forward pass with the fused observation epilogue.  With fields=False
        (and no ``out`` fields) only the observation and the wrench are written.
        Returns (obs, out)."""
        self._check_state(st)
        if not self.obs_bins:
            raise RuntimeError("no observation set on this plan (call set_observation first)")
        if obs is None:
            obs = self.new_observation()
        if (obs.dtype != torch.float32 or not obs.is_contiguous() or tuple(obs.shape) != (self.n_inst, self.obs_bins, 3)
                or obs.device != self.device):
            raise ValueError(f"obs must be a contiguous float32 ({self.n_inst}, {self.obs_bins}, 3) tensor")
        if out is None:
            if fields:
                out = self.new_outputs()
            else:
                f = dict(device=self.device, dtype=torch.float32)
                out = dict(wrench=torch.empty(self.n_inst, 6, **f),
                           status=torch.zeros(1, device=self.device, dtype=torch.int32))
        if "depth" in out:
            self._check_outputs(out)
            o = self._out_struct(out)
        else:
            o = _abi.Outputs(None, None, None, None, _ptr(out["wrench"]), _ptr(out.get("status")))
        s = self._state_struct(st)
        _abi.check(self._lib.tacsl_force_field_observe(self._plan, ctypes.byref(s), ctypes.byref(o), _ptr(obs),
                                                       _stream_handle(stream)), "tacsl_force_field_observe")
        return obs, out

    def set_normal_law(self, exponent: float = 1.0):
        """Power p of the penetration in the normal law (1: linear)."""
        _abi.check(self._lib.tacsl_plan_set_normal_law(self._plan, float(exponent)), "tacsl_plan_set_normal_law")

    def set_camera(self, rows: int, cols: int, x0: float, y0: float, dx: float, dy: float, cam_dist: float,
                   gel: float, ortho: bool = False):
        """Install the tactile camera (pad frame; see tacsl_camera)."""
        cam = _abi.Camera(int(rows), int(cols), int(bool(ortho)), float(x0), float(y0), float(dx), float(dy),
                          float(cam_dist), float(gel))
        _abi.check(self._lib.tacsl_plan_set_camera(self._plan, ctypes.byref(cam)), "tacsl_plan_set_camera")
        self._cam = cam

    def clear_camera(self):
        _abi.check(self._lib.tacsl_plan_set_camera(self._plan, None), "tacsl_plan_set_camera")
        self._cam = None

    def depth_image(self, st: Dict[str, torch.Tensor], image: Optional[torch.Tensor] = None,
                    status: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Tactile depth image of every pad, float32 (n_inst, rows, cols)."""
        self._check_state(st)
        cam = getattr(self, "_cam", None)
        if cam is None:
            raise RuntimeError("no camera set on this plan (call set_camera first)")
        shape = (self.n_inst, cam.rows, cam.cols)
        if image is None:
            image = torch.empty(shape, device=self.device, dtype=torch.float32)
        if image.dtype != torch.float32 or not image.is_contiguous() or tuple(image.shape) != shape \
                or image.device != self.device:
            raise ValueError(f"image must be a contiguous float32 {shape} tensor on {self.device}")
        s = self._state_struct(st)
        _abi.check(self._lib.tacsl_depth_image(self._plan, ctypes.byref(s), _ptr(image), _ptr(status),
                                               _stream_handle(stream)), "tacsl_depth_image")
        return image

    def backward(self, st: Dict[str, torch.Tensor], w_fn: torch.Tensor, w_ft: torch.Tensor,
                 grads: Optional[Dict[str, torch.Tensor]] = None, stream=None) -> Dict[str, torch.Tensor]:
        self._check_state(st)
        T = self.n_taxels
        for name, w in (("w_fn", w_fn), ("w_ft", w_ft)):
            if (w.dtype != torch.float32 or not w.is_contiguous() or tuple(w.shape) != (3, T)
                    or w.device != self.device):
                raise ValueError(f"{name} must be a contiguous float32 (3, {T}) tensor on {self.device}")
        if grads is None:
            f = dict(device=self.device, dtype=torch.float32)
            grads = dict(g_obj_pose=torch.empty(self.n_env, 6, **f), g_obj_twist=torch.empty(self.n_env, 6, **f),
                         g_params=torch.empty(self.n_env, 4, **f),
                         status=torch.zeros(1, device=self.device, dtype=torch.int32))
        g = _abi.Grads(_ptr(w_fn), _ptr(w_ft), _ptr(grads["g_obj_pose"]), _ptr(grads["g_obj_twist"]),
                       _ptr(grads["g_params"]), _ptr(grads.get("status")))
        s = self._state_struct(st)
        _abi.check(self._lib.tacsl_force_field_backward(self._plan, ctypes.byref(s), ctypes.byref(g),
                                                        _stream_handle(stream)), "tacsl_force_field_backward")
        return grads

    def close(self):
        if self._plan:
            for g in list(self._graphs):
                g.close()
            torch.cuda.synchronize(self.device)
            _abi.check(self._lib.tacsl_plan_destroy(self._plan), "tacsl_plan_destroy")
            self._plan = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SubstepGraph:
    """One HIP graph replaying forward evaluations of one or more plans.

    ``SubstepGraph(plan, states, outs)`` captures ``len(states)`` substeps of
    one plan.  ``SubstepGraph([p0, p1, ...], states, outs)`` takes per-plan
    lists and captures substep-major (all plans' launches of substep 0, then
    substep 1, ...).
    """

    def __init__(self, plans, states, outs, paths=None):
        if isinstance(plans, Plan):
            plans, states, outs = [plans], [states], [outs]
            paths = None if paths is None else [paths]
        plans = list(plans)
        n_steps = len(states[0]) if states else 0
        if (not plans or len(states) != len(plans) or len(outs) != len(plans) or n_steps == 0
                or any(len(s) != n_steps or len(o) != n_steps for s, o in zip(states, outs))):
            raise ValueError("need one list of states and outputs per plan, all of the same non-zero length")
        for p, ss, oo in zip(plans, states, outs):
            for st, out in zip(ss, oo):
                p._check_state(st)
                p._check_outputs(out)
        self.plans = plans
        self._keep = (states, outs, paths)
        parr_paths = None
        if paths is not None:
            if len(paths) != len(plans):
                raise ValueError("need one pose path (or None) per plan")
            items = []
            for p, path in zip(plans, paths):
                if path is None:
                    items.append(_abi.PosePath(None, None, 0.0, None))
                    continue
                pose0, twist, dt, poses = path["pose0"], path["twist"], float(path["dt"]), path["poses"]
                for name, t, shp in (("pose0", pose0, (p.n_env, 7)), ("twist", twist, (p.n_env, 6)),
                                     ("poses", poses, (n_steps, p.n_env, 7))):
                    if (t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != shp
                            or t.device != p.device):
                        raise ValueError(f"path[{name}] must be a contiguous float32 {shp} tensor on {p.device}")
                items.append(_abi.PosePath(_ptr(pose0), _ptr(twist), dt, _ptr(poses)))
            parr_paths = (_abi.PosePath * len(plans))(*items)
        self._paths = parr_paths
        n = n_steps * len(plans)
        sarr = (_abi.State * n)(*[plans[p]._state_struct(states[p][s]) for s in range(n_steps)
                                  for p in range(len(plans))])
        oarr = (_abi.Outputs * n)(*[plans[p]._out_struct(outs[p][s]) for s in range(n_steps)
                                    for p in range(len(plans))])
        parr = (ctypes.c_void_p * len(plans))(*[p._plan.value for p in plans])
        self._g = ctypes.c_void_p(None)
        lib = plans[0]._lib
        torch.cuda.synchronize(plans[0].device)
        _abi.check(lib.tacsl_graph_create_path(len(plans), parr, n_steps, parr_paths, sarr, oarr,
                                               ctypes.byref(self._g)), "tacsl_graph_create_path")
        for p in plans:
            p._graphs.append(self)

    def launch(self, stream=None):
        _abi.check(self.plans[0]._lib.tacsl_graph_launch(self._g, _stream_handle(stream)), "tacsl_graph_launch")

    def close(self):
        if self._g:
            torch.cuda.synchronize(self.plans[0].device)
            self.plans[0]._lib.tacsl_graph_destroy(self._g)
            self._g = ctypes.c_void_p(None)
            for p in self.plans:
                if self in p._graphs:
                    p._graphs.remove(self)


class _ForceFieldFn(torch.autograd.Function):
    """f_n, f_t differentiable w.r.t. obj_pose_delta (6-DoF twist), obj_twist and params.

    The state tensors are kept with ``save_for_backward``, so changing any of
    them in place between the forward and the backward pass (an optimizer
    step, say) raises autograd's version error instead of silently
    differentiating at the new values."""

    @staticmethod
    def forward(ctx, plan: Plan, pad_pose, obj_pose, pad_twist, obj_twist, params, obj_pose_delta):
        st = dict(pad_pose=pad_pose.detach(), obj_pose=obj_pose.detach(), pad_twist=pad_twist.detach(),
                  obj_twist=obj_twist.detach(), params=params.detach())
        if obj_pose_delta is not None:
            st["obj_pose_delta"] = obj_pose_delta.detach()
        out = plan.forward(st)
        ctx.plan = plan
        ctx.has_delta = obj_pose_delta is not None
        saved = [pad_pose, obj_pose, pad_twist, obj_twist, params]
        if obj_pose_delta is not None:
            saved.append(obj_pose_delta)
        ctx.save_for_backward(*saved)
        ctx.mark_non_differentiable(out["depth"], out["normal"], out["wrench"])
        return out["depth"], out["normal"], out["fn"], out["ft"], out["wrench"]

    @staticmethod
    def backward(ctx, g_depth, g_normal, g_fn, g_ft, g_wrench):
        plan: Plan = ctx.plan
        saved = ctx.saved_tensors
        st = {k: t.detach() for k, t in zip(STATE_KEYS, saved[:5])}
        if ctx.has_delta:
            st["obj_pose_delta"] = saved[5].detach()
        T = plan.n_taxels
        f = dict(device=plan.device, dtype=torch.float32)
        w_fn = g_fn.contiguous() if g_fn is not None else torch.zeros(3, T, **f)
        w_ft = g_ft.contiguous() if g_ft is not None else torch.zeros(3, T, **f)
        g = plan.backward(st, w_fn, w_ft)
        need = ctx.needs_input_grad
        return (None, None, None, None, g["g_obj_twist"] if need[4] else None,
                g["g_params"] if need[5] else None, g["g_obj_pose"] if need[6] else None)


def pose_step(pose0: torch.Tensor, twist: torch.Tensor, t: float, out: Optional[torch.Tensor] = None,
              stream=None) -> torch.Tensor:
    """Object poses after time t at a constant twist (tacsl_pose_step):
    origin t_o + v t, orientation Exp(w t) R_o.  pose0 float32 [E, 7],
    twist float32 [E, 6] on one device; returns float32 [E, 7]."""
    lib = _abi.load()
    n = int(pose0.shape[0])
    for name, t_, shp in (("pose0", pose0, (n, 7)), ("twist", twist, (n, 6))):
        if t_.dtype != torch.float32 or not t_.is_contiguous() or tuple(t_.shape) != shp or t_.device != pose0.device:
            raise ValueError(f"{name} must be a contiguous float32 {shp} tensor")
    if out is None:
        out = torch.empty(n, 7, device=pose0.device, dtype=torch.float32)
    _abi.check(lib.tacsl_pose_step(n, _ptr(pose0), _ptr(twist), float(t), _ptr(out), _stream_handle(stream)),
               "tacsl_pose_step")
    return out


def force_field(plan: Plan, pad_pose, obj_pose, pad_twist, obj_twist, params, obj_pose_delta=None):
    """Differentiable forward.  Returns (depth, normal, fn, ft, wrench).

    Gradients of f_n and f_t flow to ``obj_pose_delta`` (the world-frame
    perturbation t_o + dt, Exp(dtheta) R_o; pass zeros with requires_grad to
    differentiate w.r.t. the object pose), ``obj_twist`` and ``params``.
    depth, normal and wrench are not differentiable.
    """
    return _ForceFieldFn.apply(plan, pad_pose, obj_pose, pad_twist, obj_twist, params, obj_pose_delta)


def contact_impulse(eps: torch.Tensor, eps_dot: torch.Tensor, inv_mass: torch.Tensor, kc: torch.Tensor, dt: float,
                    env: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None,
                    dv: Optional[torch.Tensor] = None, with_dv: bool = True, status: Optional[torch.Tensor] = None,
                    stream=None):
    """Batched implicit soft-contact impulse (Section III-A, closed form of the
    end-of-step Kelvin-Voigt law), enqueued on the current torch stream.

    eps, eps_dot, inv_mass: float32 [n]; kc: float32 [n_env, 2] = (kappa, c);
    env: int32 [n] or None.  Returns (lambda, dv) (dv None when with_dv is False).
    """
    lib = _abi.load()
    n = int(eps.numel())
    dev = eps.device
    for name, t in (("eps", eps), ("eps_dot", eps_dot), ("inv_mass", inv_mass)):
        if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n or t.device != dev:
            raise ValueError(f"{name} must be a contiguous float32 tensor of {n} elements on {dev}")
    if kc.dtype != torch.float32 or not kc.is_contiguous() or kc.dim() != 2 or kc.shape[1] != 2 or kc.device != dev:
        raise ValueError("kc must be a contiguous float32 (n_env, 2) tensor on the contacts' device")
    if env is not None and (env.dtype != torch.int32 or not env.is_contiguous() or env.numel() != n
                            or env.device != dev):
        raise ValueError(f"env must be a contiguous int32 tensor of {n} elements on {dev}")
    if lam is None:
        lam = torch.empty(n, device=dev, dtype=torch.float32)
    if dv is None and with_dv:
        dv = torch.empty(n, device=dev, dtype=torch.float32)
    for name, t in (("lam", lam), ("dv", dv)):
        if t is not None and (t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n
                              or t.device != dev):
            raise ValueError(f"{name} must be a contiguous float32 tensor of {n} elements on {dev}")
    _abi.check(lib.tacsl_contact_impulse(n, _ptr(eps), _ptr(eps_dot), _ptr(inv_mass), _ptr(env), int(kc.shape[0]),
                                         _ptr(kc), float(dt), _ptr(lam), _ptr(dv), _ptr(status),
                                         _stream_handle(stream)), "tacsl_contact_impulse")
    return lam, dv
