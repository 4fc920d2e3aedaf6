"""Host-side tests of the C-ABI (no GPU): exports, validation, work lists.

The library loads on a machine without a GPU; only host-only entry points are
called here (no kernel launch).
"""
import copy
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2408_06506_amd import _abi, api
from paper_2408_06506_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "tacsl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tacsl_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = _header_functions()
    assert len(names) == 25
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_abi.EXPORTS) == names
    assert lib.tacsl_abi_version() == 1


def test_status_strings():
    lib = _abi.load()
    for code, name in _abi.STATUS_NAMES.items():
        assert lib.tacsl_status_string(code).decode().startswith(name)
    assert lib.tacsl_status_string(-99).decode() == "TACSL_ERR_UNKNOWN"


def _uneven():
    return wl.make_uneven_small(cfg_id=12, n_env=12, substeps=1)


def test_valid_scenes_pass():
    for sc in (_uneven(), wl.make_c1(0), wl.make_small(n_env=3)):
        assert api.validate_scene(sc) == 0


def test_null_pointers_rejected():
    lib = _abi.load()
    assert lib.tacsl_validate_scene(None) == -1
    sc = _uneven()
    assert api.validate_scene(sc, tmpl_ptr=None) == -1
    assert api.validate_scene(sc, sdf_ptr=None) == -1


def _mut(sc, **kw):
    s = copy.copy(sc)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def test_invalid_descriptions_return_codes():
    sc = _uneven()
    # non-monotone template offsets
    off = sc.tmpl_offset.copy()
    off[1], off[2] = off[2], off[1]
    assert api.validate_scene(_mut(sc, tmpl_offset=off)) == -2
    off = sc.tmpl_offset.copy()
    off[0] = 1
    assert api.validate_scene(_mut(sc, tmpl_offset=off)) == -2
    # out-of-range ids
    ie = sc.inst_env.copy()
    ie[3] = sc.n_env
    assert api.validate_scene(_mut(sc, inst_env=ie)) == -3
    ie[3] = -1
    assert api.validate_scene(_mut(sc, inst_env=ie)) == -3
    it = sc.inst_tmpl.copy()
    it[0] = 99
    assert api.validate_scene(_mut(sc, inst_tmpl=it)) == -3
    es = sc.env_sdf.copy()
    es[0] = sc.n_sdf
    assert api.validate_scene(_mut(sc, env_sdf=es)) == -3
    # grid dimension < 2
    dims = sc.sdf_dims.copy()
    dims[1, 2] = 1
    assert api.validate_scene(_mut(sc, sdf_dims=dims)) == -2
    # non-positive or non-finite spacing, non-finite origin, negative offset
    for bad in (0.0, -1e-3, np.nan, np.inf):
        sp = sc.sdf_spacing.copy()
        sp[0] = bad
        assert api.validate_scene(_mut(sc, sdf_spacing=sp)) == -3
    org = sc.sdf_origin.copy()
    org[0, 1] = np.nan
    assert api.validate_scene(_mut(sc, sdf_origin=org)) == -3
    so = sc.sdf_offset.copy()
    so[0] = -5
    assert api.validate_scene(_mut(sc, sdf_offset=so)) == -3
    # the plan's grid copy (16 B per node, x and y rounded up to even, plus
    # one bit per 2x2x2-cell block in 32-bit words of 4x4x2 blocks) must stay
    # below 4 GiB
    def copy_bytes(n):
        nx, ny, nz = (int(v) for v in n)
        mask = ((nx // 2 + 3) // 4) * ((ny // 2 + 3) // 4) * ((nz // 2 + 1) // 2) * 4
        return ((nx + 1) // 2) * ((ny + 1) // 2) * nz * 64 + (mask + 15) // 16 * 16
    dims = sc.sdf_dims.copy()
    dims[0] = (646, 646, 646)
    assert copy_bytes(dims[0]) >= 2 ** 32
    assert api.validate_scene(_mut(sc, sdf_dims=dims)) == -6
    dims[0] = (644, 644, 644)
    assert copy_bytes(dims[0]) < 2 ** 32
    assert api.validate_scene(_mut(sc, sdf_dims=dims)) == 0
    # one x-pair slab (64 ceil(ny/2) nz bytes) must stay below 2^24 bytes
    dims[0] = (2, 800, 800)
    assert copy_bytes(dims[0]) < 2 ** 32 and 64 * 400 * 800 >= 2 ** 24
    assert api.validate_scene(_mut(sc, sdf_dims=dims)) == -6
    dims[0] = (4, 724, 723)
    assert 64 * 362 * 723 < 2 ** 24
    assert api.validate_scene(_mut(sc, sdf_dims=dims)) == 0
    # counts
    assert api.validate_scene(_mut(sc, n_env=-1)) == -2


def test_empty_scene_is_valid():
    sc = _mut(_uneven(), n_inst=0, inst_env=np.zeros(0, np.int32), inst_tmpl=np.zeros(0, np.int32))
    assert api.validate_scene(sc) == 0
    wlst = api.build_worklist(sc)
    assert wlst["inst"].size == 0


def _independent_tiles(sc, tile):
    counts = np.diff(sc.tmpl_offset)[sc.inst_tmpl]
    out = []
    for i, c in enumerate(counts):
        if c == 0:
            out.append((i, 0, 0))
            continue
        step = tile if tile > 0 else c
        k = 0
        while k < c:
            out.append((i, k, min(step, c - k)))
            k += step
    return out


@pytest.mark.parametrize("tile", [0, 64, 192, 1024])
@pytest.mark.parametrize("order", [0, 1, 2, 3, 4, 5])
def test_worklist_covers_every_taxel_once(tile, order):
    sc = _uneven()
    w = api.build_worklist(sc, dict(block=64, tile_taxels=tile, order=order))
    ref = _independent_tiles(sc, tile)
    got = list(zip(w["inst"].tolist(), w["k0"].tolist(), w["count"].tolist()))
    assert got == ref  # bit-exact, instance-major numbering
    assert sorted(w["order"].tolist()) == list(range(len(ref)))  # a permutation
    counts = np.diff(sc.tmpl_offset)[sc.inst_tmpl]
    cover = [np.zeros(c, np.int32) for c in counts]
    for s in w["order"]:
        i, k0, c = ref[s]
        cover[i][k0:k0 + c] += 1
    assert all(np.all(v == 1) for v in cover)


def test_xcd_order_groups_objects():
    sc = wl.make_c2(n_env=64, res=(8, 10), grid=24)
    w = api.build_worklist(sc, dict(order=1), xcd_count=8)
    sdf_of_tile = sc.env_sdf[sc.inst_env[w["inst"]]]
    slots = w["order"]
    # slots s with the same s % 8 run on the same XCD: few distinct objects each
    per_xcd = [len(set(sdf_of_tile[slots[x::8]].tolist())) for x in range(8)]
    assert max(per_xcd) <= 2, per_xcd
    # object-major with per-XCD runs: objects appear one after the other, and
    # within an object each XCD (slot % 8) gets a contiguous run of its tiles
    w4 = api.build_worklist(sc, dict(order=4), xcd_count=8)
    obj = sc.env_sdf[sc.inst_env[w4["inst"]]][w4["order"]]
    assert np.all(np.diff(obj) >= 0)
    for g in np.unique(obj):
        tiles_g = w4["order"][obj == g]            # the object's tiles in slot order
        rank = np.argsort(np.argsort(tiles_g))     # position in the object's own (instance-major) list
        for x in range(8):
            run = rank[x::8][:-1]                  # equal-cost segments: all rounds but the last are full
            assert np.all(np.diff(run) == 1), (g, x, run)
    # longest-first order is non-increasing in tile size
    w2 = api.build_worklist(wl.make_uneven_small(), dict(order=2, tile_taxels=256))  # block 256
    sizes = w2["count"][w2["order"]]
    assert np.all(np.diff(sizes) <= 0)


def test_bad_tunings_rejected():
    sc = _uneven()
    for bad in (dict(block=96), dict(block=1024), dict(tile_taxels=10), dict(schedule=3), dict(order=6),
                dict(grid=-1)):
        with pytest.raises(_abi.TacslError) as ei:
            api.build_worklist(sc, bad)
        assert ei.value.code == -3
    with pytest.raises(_abi.TacslError):
        api.build_worklist(sc, None, xcd_count=0)


def test_contact_impulse_host_validation():
    """Argument checks of tacsl_contact_impulse return before any launch."""
    lib = _abi.load()
    f = lib.tacsl_contact_impulse
    fake = ctypes.c_void_p(4096)  # never dereferenced: every call below is rejected on the host
    args = lambda n, n_env=1, dt=1e-3, kc=fake, eps=fake, lam=fake: (n, eps, fake, fake, None, n_env, kc, dt, lam,
                                                                      None, None, None)
    assert f(*args(-1)) == -2
    assert f(*args(10, n_env=0)) == -2
    assert f(*args(10, dt=0.0)) == -3
    assert f(*args(10, dt=-1e-3)) == -3
    assert f(*args(10, dt=float("nan"))) == -3
    assert f(*args(10, dt=float("inf"))) == -3
    assert f(*args(0)) == 0                       # nothing to do, nothing launched
    assert f(*args(0, eps=None, lam=None)) == 0
    assert f(*args(10, eps=None)) == -1
    assert f(*args(10, lam=None)) == -1
    assert f(*args(10, kc=None)) == -1
    assert f(*args(10, kc=ctypes.c_void_p(4100))) == -3   # (kappa, c) rows must be 8-byte aligned


def test_pose_step_host_validation():
    """tacsl_pose_step rejects bad arguments before any launch (no GPU needed)."""
    lib = _abi.load()
    assert lib.tacsl_pose_step(-1, 1, 1, 0.0, 1, None) == -2
    assert lib.tacsl_pose_step(3, None, 1, 0.0, 1, None) == -1
    assert lib.tacsl_pose_step(3, 1, 1, float("inf"), 1, None) == -3
    assert lib.tacsl_pose_step(0, None, None, 0.0, None, None) == 0
