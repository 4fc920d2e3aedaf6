"""Comparison of the HIP path with the FP64 oracle (test helper).

Tolerances (the force field's error budget in FP32 against FP64):
* depth:  |d_gpu - d_ref| <= 1e-5 * max(|d_ref|, D), D = the workload's
  maximum penetration (1 mm for the tiny ball case, 2 mm otherwise);
  contact flags may therefore differ only within 1e-5 D of the surface;
* forces: ||f_gpu - f_ref|| <= 1e-4 * max(||f_ref||, k_n D);
* normals: ||n_gpu - n_ref|| <= 1e-4 where both are in contact and
  d_ref > 1e-5 D;
* wrench (per pad): |dF| <= 1e-4 * sum ||f|| + n_c k_n 1e-5 D and
  |dtau| <= 1e-4 * sum ||x|| ||f|| + sum_c ||x|| k_n 1e-5 D, where the second
  terms carry the depth floor of every taxel in contact on either side
  (n_c of them) into the sums, as the per-taxel bounds already allow.
"""
import numpy as np

import oracle


def gpu_outputs_np(out, rows=None):
    """GPU outputs as FP64 numpy; ``rows`` (a torch index tensor) selects taxels on the device."""
    o = {}
    for k in ("depth", "normal", "fn", "ft", "wrench"):
        t = out[k].detach()
        if rows is not None and k != "wrench":
            r = rows.to(t.device)
            t = t[r] if k == "depth" else t[:, r]
        o[k] = t.cpu().numpy().astype(np.float64)
    return o


def rows_of(offsets, sel):
    return np.concatenate([np.arange(offsets[i], offsets[i + 1]) for i in sel]) if len(sel) else np.zeros(0, np.int64)


def compare(scene, gpu, ref, D, kn, sel=None, what=""):
    """Assert the GPU outputs (restricted to `sel` pads) match the oracle."""
    sel = np.arange(scene.n_inst) if sel is None else np.asarray(sel)
    dg, dr = gpu["depth"], ref["depth"]
    err_d = np.abs(dg - dr)
    lim_d = 1e-5 * np.maximum(np.abs(dr), D)
    bad = err_d > lim_d
    assert not bad.any(), f"{what} depth: {bad.sum()} bad, worst {np.max(err_d / lim_d):.3g}x the bound"
    for k in ("fn", "ft"):
        e = np.linalg.norm(gpu[k] - ref[k], axis=0)
        lim = 1e-4 * np.maximum(np.linalg.norm(ref[k], axis=0), kn * D)
        bad = e > lim
        assert not bad.any(), f"{what} {k}: {bad.sum()} bad, worst {np.max(e / lim):.3g}x the bound"
    both = (dg > 0) & (dr > 1e-5 * D)
    en = np.linalg.norm(gpu["normal"][:, both] - ref["normal"][:, both], axis=0)
    assert np.all(en <= 1e-4), f"{what} normal: worst {en.max() if en.size else 0:.3g}"
    compare_wrench(scene, gpu["wrench"], ref, D, kn, sel=sel, gpu_depth=dg, what=what)


def compare_wrench(scene, wrench, ref, D, kn, sel=None, gpu_depth=None, extra_contacts=0, what=""):
    """Per-pad wrench bounds (module docstring); the taxels in contact on the
    GPU side count into the floor when ``gpu_depth`` is given.  Without it,
    ``extra_contacts`` taxels per pad (at the largest |x| of the pad) may be in
    contact on the GPU side alone, within the depth floor of the surface."""
    sel = np.arange(scene.n_inst) if sel is None else np.asarray(sel)
    dr = ref["depth"]
    dg = dr if gpu_depth is None else gpu_depth
    counts = np.diff(scene.tmpl_offset)[scene.inst_tmpl[sel]]
    starts = np.concatenate([[0], np.cumsum(counts)])
    f = ref["fn"] + ref["ft"]
    fmag = np.linalg.norm(f, axis=0)
    floor = kn * 1e-5 * D
    either = (dg > 0) | (dr > 0)
    for j, i in enumerate(sel):
        p = scene.inst_tmpl[i]
        x = scene.tmpl_xyz[:, scene.tmpl_offset[p]:scene.tmpl_offset[p + 1]].astype(np.float64)
        xn = np.linalg.norm(x, axis=0)
        sl = slice(starts[j], starts[j + 1])
        c = either[sl]
        sF = fmag[sl].sum() + 1e4 * floor * (c.sum() + extra_contacts)
        sT = (xn * fmag[sl]).sum() + 1e4 * floor * (xn[c].sum() + extra_contacts * xn.max(initial=0.0))
        dF = np.abs(wrench[j, :3] - ref["wrench"][j, :3]).max()
        dT = np.abs(wrench[j, 3:] - ref["wrench"][j, 3:]).max()
        assert dF <= 1e-4 * sF + 1e-30, f"{what} wrench F pad {i}: {dF} > 1e-4 * {sF}"
        assert dT <= 1e-4 * sT + 1e-30, f"{what} wrench torque pad {i}: {dT} > 1e-4 * {sT}"


def grad_blocks_close(g_gpu, g_ref, tol=1e-4, what="", g_abs=None):
    """Per environment and block (pose, twist, params):
    ||dg|| <= tol * max(||g_ref||, ||A||), where A (optional) is, per
    component, the sum over taxels of |per-taxel contribution| -- the scale
    of a sum that cancels, which per-taxel FP32 errors (e.g. 1e-5 relative on
    a 0.1 mm depth) are relative to."""
    for name, blk in (("pose", slice(0, 6)), ("twist", slice(6, 12)), ("params", slice(12, 16))):
        num = np.linalg.norm(g_gpu[:, blk] - g_ref[:, blk], axis=1)
        den = np.linalg.norm(g_ref[:, blk], axis=1)
        if g_abs is not None:
            den = np.maximum(den, np.linalg.norm(g_abs[:, blk], axis=1))
        ok = num <= tol * den + 1e-12
        assert ok.all(), f"{what} {name}: worst {np.max(num / np.maximum(den, 1e-30)):.3g} (env {np.argmax(num / np.maximum(den, 1e-30))})"


def oracle_forward(scene, state64, sel=None, nthreads=0):
    return oracle.force_field(scene, state64, sel=sel, nthreads=nthreads)
