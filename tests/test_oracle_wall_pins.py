"""Pins of the oracle's walls (scenario of Sec. 4.4: floes driven into a fixed
wall): floe-wall contact in the DEM (WALLS_X) and the zero Dirichlet boundary
in x of the continuum step (DIRICHLET_X), against closed forms, conservation
and Fourier sine modes.  CPU only."""
import math

import numpy as np
import pytest

import fixtures
import oracle
from helpers import frac

L = 25e3
E, G, MU = 200.0, 5.0e3, 0.3


def _floes(xs, ys, r, u=None, v=None, omega=None, h=None, Lx=L, ocean=None):
    n = len(xs)
    h = [1.0] * n if h is None else h
    w = fixtures.from_arrays(1, 1, Lx, [n], frac(xs, Lx), frac(ys, Lx), r, h, u=u, v=v, omega=omega,
                             ocean=ocean, G=G)
    w.E, w.mu = E, MU
    return w


def _step(w, flags, dt, n=1):
    m = oracle.Model(w, flags)
    st = oracle.State.from_workload(w)
    _, stats = oracle.dem_steps(m, st, dt, n)
    return st, stats


def test_wall_normal_force_is_the_chord_law():
    """A floe at rest overlapping the wall at x = L by r - d: one step changes
    its velocity by dt c E (d - r) / m towards -x, c = 2 sqrt(r^2 - d^2) (the
    chord the wall line cuts); nothing along y, no spin."""
    r, d, h = 900.0, 700.0, 1.3
    for side, x, sgn in (("right", L - d, 1.0), ("left", d, -1.0)):
        w = _floes([x], [0.5 * L], [r], h=[h])
        dt = 30.0
        st, stats = _step(w, oracle.WALLS_X | oracle.OCEAN_OFF, dt)
        x32 = float(w.xi[0]) * 2.0 ** -32 * L
        dd = (L - x32) if sgn > 0 else x32
        hh = float(np.float32(h))
        m = w.rho_ice * hh * math.pi * r * r
        c = 2.0 * math.sqrt(r * r - dd * dd)
        du = dt * c * E * (dd - r) * sgn / m
        assert st.u[0] == pytest.approx(du, rel=1e-13), side
        assert st.v[0] == 0.0 and st.w[0] == 0.0
        assert stats[0] == 1                         # one wall contact
    # a floe exactly touching (d = r) is not in contact
    w = _floes([L - 1000.0], [0.5 * L], [1000.0])
    st, stats = _step(w, oracle.WALLS_X | oracle.OCEAN_OFF, 30.0)
    assert stats[0] == 0 and st.u[0] == 0.0


def test_head_on_bounce_reverses_the_floe_and_conserves_energy_as_dt_shrinks():
    """Ocean off, frictionless head-on approach: the floe leaves the wall with
    its speed reversed, the error (the spring is conservative; semi-implicit
    Euler keeps its energy error bounded) falling with dt towards zero; y
    momentum and spin stay exactly zero."""
    r, u0 = 800.0, 0.2
    errs = {}
    for dt in (32.0, 16.0, 8.0, 4.0, 2.0, 1.0):
        w = _floes([L - 2.0 * r], [0.5 * L], [r], u=[u0])
        T = 2.0 * (2.0 * r) / u0 + 600.0             # there and back, clear of the wall
        st, stats = _step(w, oracle.WALLS_X | oracle.OCEAN_OFF, dt, int(round(T / dt)))
        assert stats[0] > 0
        assert st.v[0] == 0.0 and st.w[0] == 0.0
        assert st.u[0] < 0.0
        errs[dt] = abs(st.u[0] / u0 + 1.0)
    assert errs[32.0] < 2e-3 and errs[16.0] < 5e-4 and errs[8.0] < 1e-5
    assert max(errs[4.0], errs[2.0], errs[1.0]) < 1e-6, errs


def test_sliding_along_a_wall_friction_opposes_the_slip_and_spins_the_floe():
    """A floe pressed into a wall (overlap) and sliding along it at v: the
    tangential force opposes v, is capped at mu |f_n|, and the spin torque
    r f_t has the sign of rolling along the wall: clockwise for a wall on the
    floe's +x side and v > 0, counter-clockwise on the -x side."""
    r, d, v = 900.0, 850.0, 0.05
    for x, spin_sign in ((L - d, -1.0), (d, 1.0)):
        w = _floes([x], [0.5 * L], [r], v=[v])
        st, _ = _step(w, oracle.WALLS_X | oracle.OCEAN_OFF, 1.0)
        m = w.rho_ice * math.pi * r * r
        fy = (st.v[0] - float(np.float32(v))) * m / 1.0
        x32 = float(w.xi[0]) * 2.0 ** -32 * L
        dd = (L - x32) if spin_sign < 0 else x32
        c = 2.0 * math.sqrt(r * r - dd * dd)
        fn = c * E * (dd - r)
        assert fy < 0.0
        assert abs(fy) <= MU * abs(fn) * (1 + 1e-12)
        assert np.sign(st.w[0]) == spin_sign
        # viscous below the cap: f_t = c G v_t with v_t = -v (t along +y on the +x wall)
        assert abs(fy) == pytest.approx(min(c * G * float(np.float32(v)), MU * abs(fn)), rel=1e-12)


def test_no_contact_or_image_across_the_walls():
    """Two floes touching across the x seam: periodic, they are a contact
    pair; between walls they are not, and each is in contact with its wall."""
    r = 500.0
    w = _floes([300.0, L - 300.0], [0.5 * L, 0.5 * L], [r, r])
    st_p, s_p = _step(w, oracle.OCEAN_OFF, 1.0)
    st_w, s_w = _step(w, oracle.WALLS_X | oracle.OCEAN_OFF, 1.0)
    m = oracle.Model(w, oracle.WALLS_X)
    assert oracle.pairs_cell(m, oracle.State.from_workload(w), 0).shape[0] == 0
    assert oracle.pairs_cell(oracle.Model(w), oracle.State.from_workload(w), 0).shape[0] == 1
    assert s_p[0] == 1 and s_w[0] == 2                # the pair, or the two wall contacts
    assert st_w.u[0] > 0.0 and st_w.u[1] < 0.0        # pushed away from their walls
    assert st_p.u[0] > 0.0 and st_p.u[1] < 0.0        # pushed apart across the seam
    # a wall acts as the floe's mirror image through it at half the force:
    # the same chord, the pair overlapping by twice the wall overlap
    assert st_w.u[0] == pytest.approx(0.5 * st_p.u[0], rel=1e-12)


def test_floe_crossing_a_wall_is_an_error():
    w = _floes([L - 10.0], [0.5 * L], [5.0], u=[1.0])
    with pytest.raises(FloatingPointError):
        _step(w, oracle.WALLS_X | oracle.OCEAN_OFF, 30.0)


def _still_moments(nx, ny, ubar=0.0):
    """Statistics rows for lf_step: one floe per cell moving at (ubar, 0), no sources."""
    mom = np.zeros((nx * ny, oracle.NMOM))
    mom[:, 0] = 1.0
    mom[:, 5] = ubar
    return mom


def _grid(nx, ny, Lc=25e3):
    return oracle.Model(fixtures.from_arrays(nx, ny, Lc, np.zeros(nx * ny, np.int32), [], [], [], []),
                        oracle.DIRICHLET_X)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_dirichlet_sine_modes_decay_by_the_stencil_multiplier(k):
    """Zero coefficients: the Dirichlet problem on nx cells is the periodic one
    on the odd extension through the ghost cells, whose sine modes
    q_i = sin(pi k (i + 1) / (nx + 1)) (uniform in y) are eigenvectors of the
    averaging stencil: one step multiplies them by (1 + cos(theta)) / 2,
    theta = pi k / (nx + 1), in all four fields."""
    nx, ny = 9, 4
    m = _grid(nx, ny)
    th = math.pi * k / (nx + 1)
    ix = np.tile(np.arange(nx), ny)
    mode = np.sin(th * (ix + 1))
    Q = np.stack([mode, 2 * mode, -mode, 0.5 * mode], axis=1)
    Qn, _ = oracle.lf_step(m, Q, _still_moments(nx, ny), 600.0)
    np.testing.assert_allclose(Qn, 0.5 * (1.0 + math.cos(th)) * Q, rtol=1e-13, atol=1e-15)


def test_dirichlet_uniform_state_loses_ice_only_at_the_walls():
    """A uniform state drifting at u > 0: interior cells keep their value;
    the west column loses a quarter (zero ghost) and the flux it no longer
    receives, q' = 3q/4 - cx u q; the east column loses a quarter but keeps
    the flux it receives with nothing leaving through the wall,
    q' = 3q/4 + cx u q (cx = dT / (2 dX)); periodic grids stay uniform."""
    nx, ny, u, dT = 6, 3, 0.2, 3000.0
    Lc = 25e3
    m = _grid(nx, ny, Lc)
    Q = np.tile([[0.7, 0.0, 0.0, 0.0]], (nx * ny, 1))
    mom = _still_moments(nx, ny, ubar=u)
    Qn, _ = oracle.lf_step(m, Q, mom, dT)
    cx = dT / (2.0 * Lc)
    ix = np.tile(np.arange(nx), ny)
    inner = (ix > 0) & (ix < nx - 1)
    np.testing.assert_allclose(Qn[inner, 0], 0.7, rtol=1e-14)
    np.testing.assert_allclose(Qn[ix == 0, 0], 0.75 * 0.7 - cx * u * 0.7, rtol=1e-14)
    np.testing.assert_allclose(Qn[ix == nx - 1, 0], 0.75 * 0.7 + cx * u * 0.7, rtol=1e-14)
    mp = oracle.Model(fixtures.from_arrays(nx, ny, Lc, np.zeros(nx * ny, np.int32), [], [], [], []))
    Qp, _ = oracle.lf_step(mp, Q, mom, dT)
    np.testing.assert_allclose(Qp[:, 0], 0.7, rtol=1e-14)


def test_walls_and_dirichlet_are_separate():
    """The coupled model's cell DEMs stay periodic under DIRICHLET_X (a floe
    crossing its cell's x edge wraps), and WALLS_X leaves the continuum step
    periodic."""
    w = _floes([L - 10.0], [0.5 * L], [5.0], u=[1.0])
    st, _ = _step(w, oracle.DIRICHLET_X | oracle.OCEAN_OFF, 30.0)
    assert 0.0 <= st.xs[0] < 0.01
    nx, ny = 5, 2
    mw = oracle.Model(fixtures.from_arrays(nx, ny, L, np.zeros(nx * ny, np.int32), [], [], [], []), oracle.WALLS_X)
    Q = np.tile([[1.0, 0.0, 0.0, 0.0]], (nx * ny, 1))
    Qn, _ = oracle.lf_step(mw, Q, _still_moments(nx, ny), 60.0)
    np.testing.assert_allclose(Qn[:, 0], 1.0, rtol=1e-15)
