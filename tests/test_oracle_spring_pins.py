"""Pins of the oracle's incremental tangential spring (the Cundall-Strack
reading of the tangential contact force, Sec. 2.1; no GPU needed).

The spring replaces f_t = c G v_t by f_t = c G xi with xi the pair's
tangential displacement accumulated since the contact began, and lets the
contact slip at the Coulomb limit.  Each pin compares the spring against the
viscous law or a conservation property, so that a mistake in the history
(a missing increment, a wrong sign, a stale entry) fails one of them:
  * without tangential motion both laws give no tangential force: the same
    trajectory bit for bit;
  * at the first step of a contact xi = v_t dt, so the tangential impulse is
    dt times the viscous one (same v_t, same chord);
  * a contact that always slips gets the Coulomb force under both laws;
  * the pair forces stay antisymmetric: an isolated cell keeps its momentum;
  * a slipping contact remembers exactly the displacement of the Coulomb force;
  * a contact that ends is forgotten.
"""
import numpy as np

import fixtures
import oracle

L = 25e3


def _pair(dy=0.0, u=(0.0, 0.0), v=(0.0, 0.0), gap=-20.0, r=(500.0, 400.0), mu=0.3, G=80.0):
    """Two floes in one cell, centres along x (floe 1 offset by dy in y),
    overlapping by -gap metres."""
    x0 = 0.4 * L
    d = r[0] + r[1] + gap
    x1 = x0 + np.sqrt(max(d * d - dy * dy, 0.0))
    xi = np.array([x0 / L, x1 / L]) * 2.0 ** 32
    yi = np.array([0.5, 0.5 + dy / L]) * 2.0 ** 32
    w = fixtures.from_arrays(1, 1, L, [2], xi, yi, r, [1.0, 1.0], u=u, v=v, G=G)
    w.mu = mu
    return w


def _run(w, flags, nsteps, st=None):
    m = oracle.Model(w, flags | oracle.OCEAN_OFF)
    st = st if st is not None else oracle.State.from_workload(w)
    oracle.dem_steps(m, st, w.dt, nsteps)
    return st


def test_no_tangential_motion_gives_the_viscous_trajectory():
    w = _pair(u=(0.2, -0.1))
    a = _run(w, 0, 40)
    b = _run(w, oracle.SPRING, 40)
    for q in ("xs", "ys", "u", "v", "w", "th"):
        assert np.array_equal(getattr(a, q), getattr(b, q)), q
    assert not np.array_equal(a.u, w.u)    # the floes did collide


def test_first_step_impulse_is_dt_times_the_viscous_one():
    """One step from a touching pair sliding past each other, no slip: the
    tangential velocity change of each floe under the spring is dt times the
    viscous one, the normal one the same."""
    w = _pair(dy=0.0, v=(0.05, -0.03), mu=1e6, G=80.0)
    a = _run(w, 0, 1)
    b = _run(w, oracle.SPRING, 1)
    dv_a, dv_b = a.v - w.v, b.v - w.v        # along t = (0, 1) (centres along x)
    du_a, du_b = a.u - w.u, b.u - w.u        # along n
    assert np.all(np.abs(dv_a) > 0)
    np.testing.assert_allclose(dv_b, w.dt * dv_a, rtol=1e-12)
    np.testing.assert_allclose(du_b, du_a, rtol=1e-12)
    np.testing.assert_allclose(b.w - w.omega, w.dt * (a.w - w.omega), rtol=1e-12)
    # the history holds xi = v_t dt for the pair, the same on both sides
    vt = (w.v[1] - w.v[0])
    assert b.hj[0, 0] == 1 and b.hj[1, 0] == 0 and np.all(b.hj[:, 1:] == -1)
    np.testing.assert_allclose(b.hx[:, 0], [vt * w.dt, vt * w.dt], rtol=1e-6)


def test_always_slipping_contact_gets_the_coulomb_force():
    w = _pair(v=(0.2, -0.2), mu=1e-7, G=80.0)
    a = _run(w, 0, 30)
    b = _run(w, oracle.SPRING, 30)
    for q in ("xs", "ys", "u", "v", "w", "th"):
        assert np.array_equal(getattr(a, q), getattr(b, q)), q


def test_slip_keeps_the_coulomb_displacement():
    """After a step in which the contact slips, |c G xi| equals mu |f_n|."""
    w = _pair(v=(0.3, -0.3), mu=0.05, G=80.0)
    b = _run(w, oracle.SPRING, 1)
    x0 = w.xi.astype(np.float64) * 2.0 ** -32 * L
    y0 = w.yi.astype(np.float64) * 2.0 ** -32 * L
    d = np.hypot(x0[1] - x0[0], y0[1] - y0[0])
    r0, r1 = float(w.r[0]), float(w.r[1])
    c = oracle.chord(r0, r1, d)
    fn = c * w.E * (d - r0 - r1)
    np.testing.assert_allclose(abs(c * w.G * b.hx[0, 0]), w.mu * abs(fn), rtol=1e-12)
    assert abs(w.dt * (w.v[1] - w.v[0])) * c * w.G > w.mu * abs(fn)   # it did slip


def test_isolated_cell_keeps_its_momentum():
    w = fixtures.custom(1, 1, L, 60, seed=7, r_scale=fixtures.radius_scale(60, L * L, phi=0.5), G=80.0)
    rng = np.random.default_rng(7)
    w.u[:] = rng.normal(0, 0.2, w.nfloes)
    w.v[:] = rng.normal(0, 0.2, w.nfloes)
    st = _run(w, oracle.SPRING, 60)
    m = oracle.Model(w, oracle.SPRING | oracle.OCEAN_OFF)
    mass = w.rho_ice * w.h.astype(np.float64) * np.pi * w.r.astype(np.float64) ** 2
    p0 = np.array([np.sum(mass * w.u), np.sum(mass * w.v)])
    p1 = np.array([np.sum(mass * st.u), np.sum(mass * st.v)])
    scale = np.sum(mass * np.hypot(w.u, w.v))
    assert np.all(np.abs(p1 - p0) <= 1e-12 * scale)
    assert np.any(st.hj >= 0)            # contacts with history happened
    assert m.flags & oracle.SPRING


def test_a_contact_that_ends_is_forgotten():
    w = _pair(v=(0.05, -0.05), mu=1e6)
    st = _run(w, oracle.SPRING, 2)
    assert st.hj[0, 0] == 1 and st.hx[0, 0] != 0.0
    st.xs[1] = (st.xs[1] + 0.25) % 1.0        # pull floe 1 far away: no contact
    _run(w, oracle.SPRING, 1, st)
    assert np.all(st.hj == -1) and np.all(st.hx == 0.0)
