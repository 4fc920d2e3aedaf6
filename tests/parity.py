"""Comparison of the HIP path with the FP64 oracle (test helper).

Tolerances (the force field's error budget in FP32 against FP64):
* depth:  |d_gpu - d_ref| <= 1e-5 * max(|d_ref|, D), D = the workload's
  maximum penetration (1 mm for the tiny ball case, 2 mm otherwise);
  contact flags may therefore differ only within 1e-5 D of the surface;
* normal force: ||df_n|| <= max(1e-4 ||f_n||, k_n 1e-5 D): the depth floor
  carried through f_n = s n, |ds/dphi| ~ k_n (measured worst 0.32 of it);
* friction: ||df_t|| <= 1e-4 max(||f_t||, k_n D): a sticking taxel's
  f_t = -k_t v_t moves by k_t |x_dot| |dn|, and the normal's own FP32 error
  reaches ~3e-5 next to SDF features (k_t |x_dot| 3e-5 ~ 5e-4 N here), so
  the floor stays at 1e-4 k_n D = 2e-3 N (measured worst 0.18 of it);
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
    """Assert the GPU outputs (restricted to `sel` pads) match the oracle.
    Prints the worst error-to-bound ratio of each field and returns them."""
    sel = np.arange(scene.n_inst) if sel is None else np.asarray(sel)
    dg, dr = gpu["depth"], ref["depth"]
    err_d = np.abs(dg - dr)
    lim_d = 1e-5 * np.maximum(np.abs(dr), D)
    bad = err_d > lim_d
    ratios = dict(depth=float(np.max(err_d / lim_d, initial=0.0)))
    assert not bad.any(), f"{what} depth: {bad.sum()} bad, worst {np.max(err_d / lim_d):.3g}x the bound"
    for k in ("fn", "ft"):
        e = np.linalg.norm(gpu[k] - ref[k], axis=0)
        fr = np.linalg.norm(ref[k], axis=0)
        lim = np.maximum(1e-4 * fr, kn * 1e-5 * D) if k == "fn" else 1e-4 * np.maximum(fr, kn * D)
        ratios[k] = float(np.max(e / lim, initial=0.0))
        bad = e > lim
        assert not bad.any(), f"{what} {k}: {bad.sum()} bad, worst {np.max(e / lim):.3g}x the bound"
    both = (dg > 0) & (dr > 1e-5 * D)
    en = np.linalg.norm(gpu["normal"][:, both] - ref["normal"][:, both], axis=0)
    ratios["normal"] = float(en.max(initial=0.0) / 1e-4)
    print(f"[parity] {what}: worst error / bound " + ", ".join(f"{k} {v:.3g}" for k, v in ratios.items()),
          flush=True)
    assert np.all(en <= 1e-4), f"{what} normal: worst {en.max() if en.size else 0:.3g}"
    compare_wrench(scene, gpu["wrench"], ref, D, kn, sel=sel, gpu_depth=dg, what=what)
    return ratios


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


def near_decision_mask(scene, state64, D, rel=1e-4):
    """Taxels whose discrete force-law decisions lie within the FP32 error of
    their thresholds, where the FP32 path and the FP64 oracle may legitimately
    decide differently and the gradient jumps (a kink of the loss): contact
    (|phi| <= 1e-5 D, the depth floor), stick/slip
    (|k_t |v_t| - mu |s|| <= rel (k_t |v_t| + mu |s|) + |d(mu |s|)/d phi| 1e-5 D:
    the cap moves with the depth error the forward tolerance allows) and the degenerate
    normal (| |g| - 1e-6 | <= rel 1e-6).  Returns a bool keep-mask [T]."""
    m = oracle.decision_values(scene, state64)
    phi, gn, ktv, cap, dcap = m[:, 0], m[:, 1], m[:, 2], m[:, 3], m[:, 4]
    with np.errstate(invalid="ignore"):
        near = np.abs(phi) <= 1e-5 * D
        near |= np.abs(ktv - cap) <= rel * (ktv + cap) + dcap * 1e-5 * D
        near |= np.abs(gn - 1e-6) <= rel * 1e-6
    return ~near


# Per-taxel relative error of the FP32 adjoint's gradient terms: measured at
# most ~1e-6 of the sum of their magnitudes on every gradient test (random
# weights, several scenes and launch shapes); the bound uses 10x that.
ABS_TERM = 1e-5


def grad_blocks_close(g_gpu, g_ref, tol=1e-4, what="", g_abs=None, abs_coef=ABS_TERM):
    """Per environment and block (pose, twist, params):
    ||dg|| <= tol ||g_ref|| + abs_coef ||A||, where A (optional) is, per
    component, the sum over taxels of |per-taxel contribution| dL_k/dtheta.
    Without A the bound is the plain relative one.  A loss with weights of
    random sign cancels between taxels, and its gradient carries the rounding
    of terms much larger than the sum: that part is bounded through A with
    the per-taxel relative error.  Prints, per block, the worst error
    relative to ||g_ref|| and to the bound; returns them as
    {block: (rel, rel_to_bound)}."""
    worst = {}
    for name, blk in (("pose", slice(0, 6)), ("twist", slice(6, 12)), ("params", slice(12, 16))):
        num = np.linalg.norm(g_gpu[:, blk] - g_ref[:, blk], axis=1)
        nref = np.linalg.norm(g_ref[:, blk], axis=1)
        bound = tol * nref + (0.0 if g_abs is None else abs_coef * np.linalg.norm(g_abs[:, blk], axis=1)) + 1e-12
        rel = num / np.maximum(nref, 1e-30)
        rel_b = num / bound
        worst[name] = (float(rel.max(initial=0.0)), float(rel_b.max(initial=0.0)))
        print(f"[grad] {what} {name}: worst |dg|/|g_ref| = {worst[name][0]:.3g}, "
              f"worst error / bound = {worst[name][1]:.3g}", flush=True)
        assert np.all(num <= bound), f"{what} {name}: worst {rel_b.max():.3g}x the bound (env {np.argmax(rel_b)})"
    return worst


def oracle_forward(scene, state64, sel=None, nthreads=0):
    return oracle.force_field(scene, state64, sel=sel, nthreads=nthreads)
