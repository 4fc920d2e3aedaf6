"""Parity where the forward pass skips the corner gathers of taxels whose cell
lies in a block of 2 x 2 x 2 cells with every node value > 0.

Odd and non-cubic grids put single-cell blocks on the last rows and partial
words at the ends of the mask; taxels fill the whole node box (max faces and
corners included) and a thin band just outside the surface, where blocks are
only partly clear.  The host computes which taxels fall in clear blocks only to
check that both kinds are present; expected values come from the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from tests import scenes  # noqa: E402
from tests.parity import compare, gpu_outputs_np, grad_blocks_close, near_decision_mask  # noqa: E402

pytestmark = pytest.mark.gpu

H = 1e-3


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_06506_amd import api as _api
    return _api


def _clear_block(phi, u):
    """Whether the cell holding grid point u lies in a block whose nodes are all > 0."""
    nz, ny, nx = phi.shape
    c = [min(int(np.floor(u[a])), n - 2) for a, n in enumerate((nx, ny, nz))]
    lo = [2 * (v // 2) for v in c]
    blk = phi[lo[2]:min(lo[2] + 3, nz), lo[1]:min(lo[1] + 3, ny), lo[0]:min(lo[0] + 3, nx)]
    return bool(np.all(blk > 0))


def _scene(dims, kind, seed):
    nx, ny, nz = dims
    origin = np.array([-(nx - 1) * H / 2, -(ny - 1) * H / 2, -(nz - 1) * H / 2])
    xx, yy, zz = scenes.grid_nodes(dims, origin, H)
    if kind == "sphere":
        ctr = origin + H * np.array([0.55 * (nx - 1), 0.4 * (ny - 1), 0.5 * (nz - 1)])
        r = 0.3 * H * min(dims)
        phi = np.sqrt((xx - ctr[0]) ** 2 + (yy - ctr[1]) ** 2 + (zz - ctr[2]) ** 2) - r
    else:  # a tilted plane through the box, the object on its low side
        lin = 0.3 * (xx - origin[0]) + 0.2 * (yy - origin[1]) + 0.93 * (zz - origin[2])
        phi = lin - 0.3 * lin.max()
    phi = phi.astype(np.float32)
    rng = np.random.default_rng(seed)
    ext = H * (np.array(dims) - 1)
    pts = [origin + rng.random((6000, 3)) * ext]
    # the max faces and the far corner (cells clamped to n - 2)
    for a in range(3):
        p = origin + rng.random((300, 3)) * ext
        p[:, a] = origin[a] + ext[a]
        pts.append(p)
    pts.append((origin + ext)[None])
    # a band just outside the surface: nodes with 0 < phi < 1.5 h, jittered
    band = np.stack([xx[(phi > 0) & (phi < 1.5 * H)], yy[(phi > 0) & (phi < 1.5 * H)],
                     zz[(phi > 0) & (phi < 1.5 * H)]], axis=1)
    if band.size:
        band = band[rng.choice(band.shape[0], min(2000, band.shape[0]), replace=False)]
        pts.append(np.clip(band + rng.uniform(-0.5, 0.5, band.shape) * H, origin, origin + ext))
    pts = np.concatenate(pts)
    # pad frame = object frame (equal poses); the object moves so f_t is non-zero
    sc = scenes.single(phi, origin, H, pts, obj_twist=(0.02, -0.01, 0.03, 0.4, -0.2, 0.3),
                       params=(1e4, 10.0, 1e2, 0.5), name=f"mask-{kind}-{nx}x{ny}x{nz}")
    u = (pts - origin) / H
    clear = np.array([_clear_block(phi, ui) for ui in u])
    return sc, phi, clear


@pytest.mark.parametrize("dims,kind", [((37, 44, 29), "sphere"), ((3, 2, 5), "plane"), ((41, 9, 2), "plane")])
def test_clear_blocks_match_oracle(api, dims, kind):
    sc, phi, clear = _scene(dims, kind, seed=sum(dims))
    ref = oracle.force_field(sc, oracle.state64(sc))
    inside = ref["depth"] > 0
    assert clear.any() and (~clear & ~inside).any() and inside.any(), "all three kinds of taxel present"
    assert not (clear & inside).any()   # the mask's premise, on the oracle's side
    D = max(float(ref["depth"].max()), H)
    for tun in (dict(), dict(block=64, tile_taxels=512, schedule=2, grid=5, order=5)):
        _say(f"clear-block mask {kind} {dims} {tun}")
        plan = api.Plan(sc, tun)
        out = plan.forward(plan.state(sc.state()))
        torch.cuda.synchronize()
        g = gpu_outputs_np(out)
        compare(sc, g, ref, D=D, kn=1e4, what=f"{kind} {dims}")
        # skipped taxels write exact zeros
        assert np.all(g["depth"][clear] == 0) and np.all(g["fn"][:, clear] == 0) and np.all(g["ft"][:, clear] == 0)
        plan.close()


def test_clear_blocks_adjoint(api):
    sc, _, clear = _scene((37, 44, 29), "sphere", seed=3)
    rng = np.random.default_rng(4)
    wa = rng.standard_normal((3, sc.n_taxels)).astype(np.float32)
    wb = rng.standard_normal((3, sc.n_taxels)).astype(np.float32)
    keep = near_decision_mask(sc, oracle.state64(sc), 2e-3)
    wa, wb = (wa * keep).astype(np.float32), (wb * keep).astype(np.float32)
    _say("clear-block mask adjoint")
    plan = api.Plan(sc)
    st = plan.state(sc.state())
    g = plan.backward(st, torch.as_tensor(wa, device=plan.device), torch.as_tensor(wb, device=plan.device))
    torch.cuda.synchronize()
    gg = np.concatenate([g["g_obj_pose"].cpu().numpy(), g["g_obj_twist"].cpu().numpy(),
                         g["g_params"].cpu().numpy()], axis=1).astype(np.float64)
    _, ref, gabs = oracle.grad(sc, oracle.state64(sc), wa, wb, with_abs=True)
    grad_blocks_close(gg, ref, 1e-4, what="mask adjoint", g_abs=gabs)
    plan.close()
