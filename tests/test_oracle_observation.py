"""Pins of the oracle's force-field observation (pooled 3-channel bins per pad).

* a pad pressed flat into a half-space: every taxel carries the force of the
  hand-derived worked example (tests/golden/force_law_halfspace.json), so
  every bin must read it, scaled and clipped;
* a half-space inclined along x: |f_n| = k_n * depth is linear in x at rest,
  so each bin reads k_n times the depth at the mean x of its taxels;
* one taxel per bin reproduces the per-taxel channels; pooling preserves
  channel totals; bins without taxels read zero.
"""
import json
import os

import numpy as np

import oracle
from paper_2408_06506_amd import workloads as wl
from tests.scenes import grid_nodes, single

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _pad_scene(nx, ny, phi_fn, xdot=(0.0, 0.0, 0.0), params=(1e4, 10.0, 1e2, 0.8)):
    h = 1e-3
    n = (33, 33, 11)
    origin = np.asarray((-16e-3, -16e-3, -5e-3), np.float32)
    xx, yy, zz = grid_nodes(n, origin.astype(np.float64), float(np.float32(h)))
    tmpl = wl.pad_template(nx, ny)
    sc = single(phi_fn(xx, yy, zz), origin, h, tmpl.T, pad_twist=tuple(xdot) + (0, 0, 0), params=params)
    sc.tmpl_names = [f"{nx}x{ny}"]
    return sc


def test_flat_halfspace_reads_worked_example():
    gold = json.load(open(os.path.join(GOLD, "force_law_halfspace.json")))
    p = gold["params"]
    params = (p["k_n"], p["k_d"], p["k_t"], p["mu"])
    case = [c for c in gold["cases"] if c["name"] == "stick"][0]
    delta = case["delta"]
    sc = _pad_scene(20, 25, lambda x, y, z: -(z + delta), case["xdot"], params)
    st = oracle.state64(sc)
    st["params"] = np.asarray([params], np.float64)
    st["pad_twist"] = np.asarray([list(case["xdot"]) + [0, 0, 0]], np.float64)
    ff = oracle.force_field(sc, st)
    bins = wl.scene_observation_bins(sc)
    want = np.array([np.linalg.norm(case["fn"]), case["ft"][0], case["ft"][1]])
    obs = oracle.observation(sc, ff, bins, 140)
    np.testing.assert_allclose(obs[0], np.broadcast_to(want, (140, 3)), rtol=1e-6, atol=1e-9)
    scale = np.array([2.0, 0.5, 4.0])
    obs = oracle.observation(sc, ff, bins, 140, scale=scale, clip=3.5)
    np.testing.assert_allclose(obs[0], np.broadcast_to(np.clip(want / scale, -3.5, 3.5), (140, 3)), rtol=1e-6)
    assert np.all(obs[0][:, 1] == -3.5)   # -3 / 0.5 = -6 is clipped


def test_inclined_halfspace_bins_read_mean_depth():
    d0, slope = 1.0e-3, 0.02
    kn = 1e4
    sc = _pad_scene(40, 50, lambda x, y, z: -(z + d0 + slope * x), params=(kn, 10.0, 1e2, 0.8))
    ff = oracle.force_field(sc, oracle.state64(sc))
    bins = wl.scene_observation_bins(sc)
    obs = oracle.observation(sc, ff, bins, 140)
    x = sc.tmpl_xyz[0].astype(np.float64)
    for b in range(140):
        xm = x[bins == b].mean()
        # phi = -(d0 + slope x) at z = 0; |grad phi| normalisation does not change |f_n| = k_n * depth.
        # Node values are stored in FP32 (relative rounding 6e-8 of phi), hence 1e-6.
        np.testing.assert_allclose(obs[0, b, 0], kn * (d0 + slope * xm), rtol=1e-6)
    np.testing.assert_allclose(obs[0, :, 1:], 0.0, atol=1e-9)   # at rest: no friction


def test_one_taxel_per_bin_and_totals():
    sc = wl.make_uneven_small(cfg_id=12, n_env=6, substeps=1)
    st = oracle.state64(sc)
    ff = oracle.force_field(sc, st)
    bins = wl.scene_observation_bins(sc)
    obs = oracle.observation(sc, ff, bins, 140)
    offs = np.concatenate([[0], np.cumsum(np.diff(sc.tmpl_offset)[sc.inst_tmpl])])
    for i in range(sc.n_inst):
        p = sc.inst_tmpl[i]
        b = bins[sc.tmpl_offset[p]:sc.tmpl_offset[p + 1]]
        fn = ff["fn"][:, offs[i]:offs[i + 1]]
        ft = ff["ft"][:, offs[i]:offs[i + 1]]
        ch = np.stack([np.linalg.norm(fn, axis=0), ft[0], ft[1]], 1)
        counts = np.bincount(b, minlength=140)
        # pooled means times counts give back the channel totals
        np.testing.assert_allclose((obs[i] * counts[:, None]).sum(0), ch.sum(0), rtol=1e-12, atol=1e-12)
        assert np.all(obs[i][counts == 0] == 0)
        if sc.tmpl_names[p] == "7x9":
            assert (counts == 0).sum() == 140 - 63   # a 7 x 9 pad leaves 77 of the 14 x 10 bins empty
    # a 10 x 14 pad has exactly one taxel per bin: the observation is the per-taxel channels
    b1 = wl.pad_observation_bins(10, 14)
    assert sorted(b1.tolist()) == list(range(140))
