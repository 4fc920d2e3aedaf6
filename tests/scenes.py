"""Hand-built scenes for pins and edge cases (test helpers, no force-field arithmetic)."""
import numpy as np

from paper_2408_06506_amd.workloads import Scene


def single(phi, origin, h, taxels, pad_pose=(1, 0, 0, 0, 0.5, 0.0, 0.1),
           obj_pose=(1, 0, 0, 0, 0.5, 0.0, 0.1), pad_twist=(0,) * 6, obj_twist=(0,) * 6,
           params=(1e4, 10.0, 1e2, 0.8), name="custom"):
    """One environment, one pad.  ``phi`` is indexed [k][j][i] (x fastest)."""
    phi = np.ascontiguousarray(phi, dtype=np.float32)
    nz, ny, nx = phi.shape
    t = np.ascontiguousarray(np.asarray(taxels, dtype=np.float32).reshape(-1, 3).T)
    return Scene(
        name=name, n_env=1, n_inst=1,
        inst_env=np.zeros(1, np.int32), inst_tmpl=np.zeros(1, np.int32), env_sdf=np.zeros(1, np.int32),
        tmpl_offset=np.array([0, t.shape[1]], np.int64), tmpl_xyz=t,
        sdf_dims=np.array([[nx, ny, nz]], np.int32),
        sdf_origin=np.asarray(origin, np.float32).reshape(1, 3),
        sdf_spacing=np.array([h], np.float32), sdf_offset=np.zeros(1, np.int64),
        sdf_data=phi.reshape(-1),
        pad_pose=np.asarray(pad_pose, np.float32).reshape(1, 7),
        obj_pose=np.asarray(obj_pose, np.float32).reshape(1, 7),
        pad_twist=np.asarray(pad_twist, np.float32).reshape(1, 6),
        obj_twist=np.asarray(obj_twist, np.float32).reshape(1, 6),
        params=np.asarray(params, np.float32).reshape(1, 4))


def grid_nodes(n, origin, h):
    """Node coordinates (FP64) of an (nx, ny, nz) grid, arrays indexed [k][j][i]."""
    nx, ny, nz = n
    x = origin[0] + h * np.arange(nx)
    y = origin[1] + h * np.arange(ny)
    z = origin[2] + h * np.arange(nz)
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    return xx, yy, zz


def rel_velocity_pad(scene, state, inst=0):
    """Relative velocity of each tactile point w.r.t. the coincident object point, pad frame."""
    from paper_2408_06506_amd.workloads import quat_to_mat
    e = scene.inst_env[inst]
    Rp = quat_to_mat(state["pad_pose"][inst, :4])
    tp = state["pad_pose"][inst, 4:]
    to = state["obj_pose"][e, 4:]
    p = scene.inst_tmpl[inst]
    xp = scene.tmpl_xyz[:, scene.tmpl_offset[p]:scene.tmpl_offset[p + 1]].astype(np.float64).T
    xw = xp @ Rp.T + tp
    vp, wp = state["pad_twist"][inst, :3], state["pad_twist"][inst, 3:]
    vo, wo = state["obj_twist"][e, :3], state["obj_twist"][e, 3:]
    v = (vp + np.cross(wp, xw - tp)) - (vo + np.cross(wo, xw - to))
    return v @ Rp, xp, xw
