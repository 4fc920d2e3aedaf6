"""Pins of the oracle's implicit soft-contact impulse (Section III-A).

The closed form is checked against the equations that define it in the
paper -- the force law evaluated at the end of the step together with the
semi-implicit Euler update -- not against a retyped copy of the closed form.
"""
import numpy as np

import oracle


def _draw(n, seed):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-2e-3, 5e-4, n)          # contact distance (negative: interpenetration)
    epsdot = rng.uniform(-0.2, 0.2, n)         # separation velocity
    inv_mass = rng.uniform(0.0, 20.0, n)       # 1 / effective inertia
    inv_mass[::7] = 0.0                        # immovable bodies
    env = rng.integers(0, 4, n).astype(np.int32)
    kc = np.stack([rng.uniform(150, 350, 4), rng.uniform(0.0, 1.0, 4)], 1)  # Appendix C ranges
    return eps, epsdot, inv_mass, env, kc


def test_impulse_satisfies_end_of_step_force_law():
    dt = 1e-3
    eps, epsdot, im, env, kc = _draw(4000, 0)
    lam, dv = oracle.contact_impulse(eps, epsdot, im, env, kc, dt)
    kappa, c = kc[env, 0], kc[env, 1]
    epsdot_p = epsdot + lam * im            # velocity after the impulse
    eps_p = eps + dt * epsdot_p             # position at the end of the step
    force_end = -kappa * eps_p - c * epsdot_p
    active = lam > 0
    assert active.sum() > 500 and (~active).sum() > 500
    # active contacts: lambda = dt * (force law at the end of the step)
    np.testing.assert_allclose(lam[active], dt * force_end[active], rtol=1e-12, atol=1e-18)
    # inactive: the unilateral law gives no push at the end of the step
    assert np.all(force_end[~active] <= 1e-12)
    np.testing.assert_allclose(dv, lam * im, rtol=1e-15)


def test_impulse_limits():
    dt = 2e-3
    kc = np.array([[300.0, 0.5]])
    # immovable body: the impulse reduces to dt times the end-of-step spring-damper force
    lam, _ = oracle.contact_impulse([-1e-3], [0.0], [0.0], None, kc, dt)
    alpha = dt * (dt * 300.0 + 0.5)
    np.testing.assert_allclose(lam, [dt * 300.0 * 1e-3], rtol=1e-14)
    assert alpha > 0
    # separating fast enough: no impulse
    lam, _ = oracle.contact_impulse([-1e-4], [1.0], [1.0], None, kc, dt)
    assert lam[0] == 0.0
    # no penetration and no approach: no impulse
    lam, _ = oracle.contact_impulse([1e-3], [0.0], [5.0], None, kc, dt)
    assert lam[0] == 0.0
    # linear in penetration at zero velocity, decreasing with mobility
    l1, _ = oracle.contact_impulse([-1e-3, -2e-3], [0.0, 0.0], [2.0, 2.0], None, kc, dt)
    np.testing.assert_allclose(l1[1], 2 * l1[0], rtol=1e-14)
    l2, _ = oracle.contact_impulse([-1e-3, -1e-3], [0.0, 0.0], [1.0, 10.0], None, kc, dt)
    assert l2[0] > l2[1] > 0
