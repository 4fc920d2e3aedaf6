"""Pins of the oracle's constant-twist pose path (no GPU).

The path is the closed-form pose update of the batched workload's substep
loop: origin at t_o + v t, orientation Exp(w t) R_o with w the world-frame
angular velocity.  Pinned by: pure translation when w = 0 (exact), a quarter
turn about z by hand, the group property Exp(w t2) Exp(w t1) = Exp(w (t1 +
t2)), the derivative dR/dt = [w]x R at t = 0, and the unit norm.
"""
import numpy as np

import oracle


def _rot(q):
    """Rotation matrix of a unit quaternion (w, x, y, z), textbook form."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _poses(n, seed):
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    p = np.concatenate([q, rng.uniform(-0.5, 0.5, (n, 3))], 1)
    tw = np.concatenate([rng.uniform(-0.1, 0.1, (n, 3)), rng.uniform(-3, 3, (n, 3))], 1)
    return p, tw


def test_translation_only_when_not_turning():
    p, tw = _poses(16, 1)
    tw[:, 3:] = 0.0
    for t in (0.0, 1e-4, 0.0099, 0.37):
        out = oracle.pose_path(p, tw, t)
        assert np.array_equal(out[:, :4], p[:, :4])
        assert np.array_equal(out[:, 4:], p[:, 4:] + tw[:, :3] * t)


def test_quarter_turn_about_z():
    p = np.array([[1.0, 0, 0, 0, 0.1, 0.2, 0.3]])
    tw = np.array([[0.0, 0, 0, 0, 0, np.pi / 2]])
    out = oracle.pose_path(p, tw, 1.0)
    h = np.sqrt(0.5)
    assert np.allclose(out[0, :4], [h, 0, 0, h], atol=1e-15, rtol=0)
    R = _rot(out[0, :4])
    assert np.allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    assert np.array_equal(out[0, 4:], p[0, 4:])


def test_group_property_and_norm():
    p, tw = _poses(32, 2)
    a = oracle.pose_path(oracle.pose_path(p, tw, 0.013), tw, 0.021)
    b = oracle.pose_path(p, tw, 0.034)
    assert np.allclose(a, b, atol=1e-14, rtol=0)
    assert np.allclose(np.linalg.norm(b[:, :4], axis=1), 1.0, atol=1e-14, rtol=0)


def test_world_angular_velocity():
    """dR/dt at t = 0 equals [w]x R_0 (the turn is about world axes)."""
    p, tw = _poses(8, 3)
    h = 1e-6
    for e in range(p.shape[0]):
        R0 = _rot(p[e, :4])
        Rp = _rot(oracle.pose_path(p[e:e + 1], tw[e:e + 1], h)[0, :4])
        Rm = _rot(oracle.pose_path(p[e:e + 1], tw[e:e + 1], -h)[0, :4])
        w = tw[e, 3:]
        W = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        assert np.allclose((Rp - Rm) / (2 * h), W @ R0, atol=1e-8, rtol=0)
