"""GPU parity of the batched implicit soft-contact impulse against the FP64 oracle.

Tolerance: the kernel evaluates lambda in FP32 with a handful of roundings
(alpha, two products, a sum, the denominator, a correctly rounded division),
each within 2^-24 of its own magnitude.  The error is therefore bounded by a
small multiple of 2^-24 times the magnitude scale of the numerator terms over
the denominator; 1e-5 of that scale (about 170 units of 2^-24) is used.  Near
the gate (numerator close to zero) the bound also covers a contact whose sign
differs between FP32 and FP64, whose lambda is then below the bound.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2408_06506_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu

REL = 1e-5
BAD = 0x4


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_06506_amd import api as _api
    return _api


def _scale(c, env):
    kc = c.kc.astype(np.float64)
    e = np.zeros(c.n, np.int64) if env is None else env.astype(np.int64)
    kappa, damp = kc[e, 0], kc[e, 1]
    dt = np.float64(np.float32(c.dt))
    alpha = dt * (dt * kappa + damp)
    return (dt * kappa * np.abs(c.eps) + alpha * np.abs(c.eps_dot)) / (1.0 + alpha * c.inv_mass.astype(np.float64))


def _check(c, lam, dv, env, what):
    dt = float(np.float32(c.dt))
    l_ref, dv_ref = oracle.contact_impulse(c.eps, c.eps_dot, c.inv_mass, env, c.kc, dt)
    tol = REL * _scale(c, env) + 1e-30
    err = np.abs(lam.astype(np.float64) - l_ref)
    bad = np.flatnonzero(err > tol)
    assert bad.size == 0, f"{what}: {bad.size} lambdas off, first {bad[:5]}: {lam[bad[:5]]} vs {l_ref[bad[:5]]}"
    assert np.all(lam >= 0)
    if dv is not None:
        tol_dv = tol * c.inv_mass.astype(np.float64) + 1e-30
        bad = np.flatnonzero(np.abs(dv.astype(np.float64) - dv_ref) > tol_dv)
        assert bad.size == 0, f"{what}: {bad.size} dv off"
    return l_ref


def _dev(c, device="cuda"):
    f = lambda a: torch.as_tensor(a, device=device)
    return f(c.eps), f(c.eps_dot), f(c.inv_mass), f(c.env), f(c.kc)


def _slice(c, n):
    return wl.Contacts(c.eps[:n].copy(), c.eps_dot[:n].copy(), c.inv_mass[:n].copy(), c.env[:n].copy(), c.kc, c.dt)


@pytest.mark.parametrize("n", [1, 3, 4, 5, 257, 4099, 65543])
def test_impulse_matches_oracle(api, n):
    full = wl.make_contacts(n_env=n // 8 + 2, per_env=16, seed=40 + n % 97, ragged=True)
    assert full.n >= n
    c = _slice(full, n)
    _say(f"impulse n={n}")
    eps, ed, im, env, kc = _dev(c)
    status = torch.zeros(1, device="cuda", dtype=torch.int32)
    lam, dv = api.contact_impulse(eps, ed, im, kc, c.dt, env=env, status=status)
    lam2, dv2 = api.contact_impulse(eps, ed, im, kc[:1].contiguous(), c.dt, with_dv=False)
    torch.cuda.synchronize()
    l_ref = _check(c, lam.cpu().numpy(), dv.cpu().numpy(), c.env, f"n={n}")
    c1 = wl.Contacts(c.eps, c.eps_dot, c.inv_mass, c.env, c.kc[:1], c.dt)
    _check(c1, lam2.cpu().numpy(), None, None, f"n={n} one env row")
    assert dv2 is None
    assert int(status.item()) == 0
    if n > 1000:
        assert 0.5 < (l_ref > 0).mean() < 0.95   # both sides of the gate are exercised


def test_impulse_unaligned_and_offsets(api):
    """Arrays at 4-byte offsets take the one-contact-per-lane kernel; same results."""
    c = wl.make_contacts(n_env=300, per_env=11, seed=7)
    eps, ed, im, env, kc = _dev(c)
    _say("impulse unaligned")
    lam_a, dv_a = api.contact_impulse(eps[1:], ed[1:], im[1:], kc, c.dt, env=env[1:])
    lam_b, dv_b = api.contact_impulse(eps, ed, im, kc, c.dt, env=env)
    torch.cuda.synchronize()
    assert torch.equal(lam_a, lam_b[1:]) and torch.equal(dv_a, dv_b[1:])
    sub = wl.Contacts(c.eps[1:], c.eps_dot[1:], c.inv_mass[1:], c.env[1:], c.kc, c.dt)
    _check(sub, lam_a.cpu().numpy(), dv_a.cpu().numpy(), sub.env, "unaligned")


def test_impulse_invalid_contacts_flagged(api):
    c = wl.make_contacts(n_env=40, per_env=9, seed=3)
    bad_idx = {5: ("env", -1), 6: ("env", 40), 7: ("eps", np.nan), 8: ("inv_mass", -1e6),
               9: ("inv_mass", np.inf), 10: ("eps_dot", np.inf), 301: ("env", 1 << 30)}
    for k, (field, v) in bad_idx.items():
        getattr(c, field)[k] = v
    eps, ed, im, env, kc = _dev(c)
    status = torch.zeros(1, device="cuda", dtype=torch.int32)
    _say("impulse invalid contacts")
    lam, dv = api.contact_impulse(eps, ed, im, kc, c.dt, env=env, status=status)
    torch.cuda.synchronize()
    lam, dv = lam.cpu().numpy(), dv.cpu().numpy()
    assert int(status.item()) == BAD
    idx = np.array(sorted(bad_idx))
    assert np.all(lam[idx] == 0) and np.all(dv[idx] == 0)
    good = np.setdiff1d(np.arange(c.n), idx)
    sub = wl.Contacts(c.eps[good], c.eps_dot[good], c.inv_mass[good], c.env[good], c.kc, c.dt)
    _check(sub, lam[good], dv[good], sub.env, "valid neighbours of invalid contacts")


@pytest.mark.parametrize("n_env,per_env", [(16384, 64), (262144, 128)])
def test_impulse_full_size(api, n_env, per_env):
    """Every contact at the measured sizes: pads of the 8192-environment batch
    with 64 contacts each, and a 33.5 M-contact stream."""
    c = wl.make_contacts(n_env=n_env, per_env=per_env, seed=11)
    _say(f"impulse full n={c.n}")
    eps, ed, im, env, kc = _dev(c)
    status = torch.zeros(1, device="cuda", dtype=torch.int32)
    lam, dv = api.contact_impulse(eps, ed, im, kc, c.dt, env=env, status=status)
    torch.cuda.synchronize()
    _check(c, lam.cpu().numpy(), dv.cpu().numpy(), c.env, f"full n={c.n}")
    assert int(status.item()) == 0


def test_impulse_deterministic_and_graph_replay(api):
    c = wl.make_contacts(n_env=1000, per_env=33, seed=21, ragged=True)
    eps, ed, im, env, kc = _dev(c)
    lam_e, dv_e = api.contact_impulse(eps, ed, im, kc, c.dt, env=env)
    lam_r, _ = api.contact_impulse(eps, ed, im, kc, c.dt, env=env)
    torch.cuda.synchronize()
    assert torch.equal(lam_e, lam_r)
    lam_g = torch.empty_like(lam_e)
    dv_g = torch.empty_like(dv_e)
    _say("impulse graph capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.contact_impulse(eps, ed, im, kc, c.dt, env=env, lam=lam_g, dv=dv_g)
    torch.cuda.synchronize()
    for rep in range(3):
        eps.mul_(1.0 + 0.1 * rep)          # eager work between replays: new inputs in place
        lam_g.zero_()
        g.replay()
        lam_x, dv_x = api.contact_impulse(eps, ed, im, kc, c.dt, env=env)
        torch.cuda.synchronize()
        assert torch.equal(lam_g, lam_x), f"replay {rep}"
        assert torch.equal(dv_g, dv_x), f"replay {rep}"
