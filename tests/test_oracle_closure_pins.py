"""Pins of the closure's reduced DEM, base update and inputs (oracle/closure.py)
against things other than itself: the single-floe closed form of the drag
laws of Sec. 2.1, the oracle's cell DEM (C code) for floes that never touch,
the Lax-Friedrichs step of a uniform state, and a 3 x 3 lattice whose
feature rows are written out by hand.  CPU only."""
import math

import numpy as np
import pytest

import fixtures
import oracle
from oracle import closure as ocl
from helpers import frac

L = 25e3
RHO_I, RHO_O, CD = 920.0, 1025.0, 5.5e-3


def _cell_of_floes(xs, ys, r, h, u, v, omega, U0=(0.15, -0.08), nx=1, ny=1, counts=None):
    oc = fixtures.Ocean(U0[0], U0[1])
    counts = [len(xs)] if counts is None else counts
    w = fixtures.from_arrays(nx, ny, L, counts, frac(xs, L), frac(ys, L), r, h, u=u, v=v, omega=omega, ocean=oc)
    assert (w.rho_ice, w.rho_ocean, w.cd) == (RHO_I, RHO_O, CD)
    return w


def test_single_floe_reduced_dem_is_the_closed_form():
    """One floe of radius r, thickness h in a steady uniform current: the
    reduced DEM must be the exact solution of m dv/dt = alpha du |du| and
    I dw/dt = beta dW |dW| (Sec. 2.1 with alpha = C_d rho_o pi r^2,
    beta = C_d rho_o pi r^5, m = rho_ice h pi r^2, I = m r^2):
    du(t) = du0 / (1 + k |du0| t), k = C_d rho_o / (rho_ice h), and
    dW(t) = dW0 / (1 + k_w |dW0| t), k_w = C_d rho_o r / (rho_ice h)."""
    r, h = 900.0, 1.3
    u0, v0, w0 = 0.02, 0.11, 3e-4
    w = _cell_of_floes([7000.0], [9000.0], [r], [h], [u0], [v0], [w0])
    m = oracle.Model(w)
    static = ocl.cell_static(w)
    oce = ocl.ocean_centres(w, m)
    assert np.allclose(oce[0], [0.15, -0.08, 0.0])
    red = ocl.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 100.0)
    du0 = np.array([0.15 - float(np.float32(u0)), -0.08 - float(np.float32(v0))])
    dW0 = -float(np.float32(w0))
    h = float(np.float32(h))                  # the thickness as stored
    k = CD * RHO_O / (RHO_I * h)
    kw = CD * RHO_O * r / (RHO_I * h)
    for t in (100.0, 700.0, 5000.0, 86400.0):
        dux, duy, dw = ocl.reduced_rel(red, static, t)
        tau = t - 100.0
        ref = du0 / (1.0 + k * np.linalg.norm(du0) * tau)
        np.testing.assert_allclose([dux[0], duy[0]], ref, rtol=1e-12)
        assert dw[0] == pytest.approx(dW0 / (1.0 + kw * abs(dW0) * tau), rel=1e-12)
        # sources per unit area: the floe's drag force and torque over the cell area
        mom = ocl.reduced_moments(red, static, oce, t, L * L)
        alpha = CD * RHO_O * math.pi * r * r
        beta = CD * RHO_O * math.pi * r ** 5
        np.testing.assert_allclose(mom[0, 7:9], alpha * np.linalg.norm(ref) * ref, rtol=1e-12)
        assert mom[0, 9] == pytest.approx(beta * abs(dw[0]) * dw[0], rel=1e-12)
        np.testing.assert_allclose(mom[0, 5:7], np.array([0.15, -0.08]) - ref, rtol=1e-12)
    # before its start time a reduced DEM does not move
    np.testing.assert_allclose(np.array(ocl.reduced_rel(red, static, 50.0))[:, 0], [du0[0], du0[1], dW0])


def test_sources_equal_the_oracle_drag_at_the_closed_form_state():
    """The reduced DEM's sources at time t equal the drag sums the oracle's
    statistics (C code) compute for a floe whose velocity and spin are the
    closed-form ones at t."""
    r, h = 1400.0, 0.7
    w = _cell_of_floes([12000.0], [3000.0], [r], [h], [-0.05], [0.04], [-2e-4])
    m = oracle.Model(w)
    static = ocl.cell_static(w)
    oce = ocl.ocean_centres(w, m)
    red = ocl.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 0.0)
    t = 3600.0
    dux, duy, dw = ocl.reduced_rel(red, static, t)
    st = oracle.State.from_workload(w)
    st.u[0], st.v[0], st.w[0] = 0.15 - dux[0], -0.08 - duy[0], 0.0 - dw[0]
    dem = oracle.moments(m, st)
    red_m = ocl.reduced_moments(red, static, oce, t, L * L)
    np.testing.assert_allclose(red_m[0, 7:10], dem[0, 7:10], rtol=1e-12)
    np.testing.assert_allclose(red_m[0, 5:7], dem[0, 5:7] / dem[0, 0], rtol=1e-12)


def _lattice(n_side, r, h, u, v, omega, U0=(0.15, -0.08)):
    """n_side^2 identical floes on a square lattice of the cell, far apart."""
    g = (np.arange(n_side) + 0.5) / n_side * L
    X, Y = np.meshgrid(g, g)
    n = n_side * n_side
    return _cell_of_floes(X.ravel(), Y.ravel(), [r] * n, [h] * n, [u] * n, [v] * n, [omega] * n, U0=U0)


def test_reduced_dem_tracks_the_cell_dem_of_identical_floes_first_order():
    """Identical floes that never touch, uniform current: every floe follows
    the single-floe law, so the cell DEM's statistics (U / n, L / (M r2m),
    the drag sums) converge to the reduced DEM's at first order in dt (the
    semi-implicit Euler step): the error ratio between dt and dt / 2 lies in
    [1.8, 2.2].  A wrong drag rate, spin exponent or spin mean breaks it."""
    T = 2400.0
    w = _lattice(3, 700.0, 1.1, -0.04, 0.06, 4e-4)
    m = oracle.Model(w)
    static = ocl.cell_static(w)
    oce = ocl.ocean_centres(w, m)
    red = ocl.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 0.0)
    rm = ocl.reduced_moments(red, static, oce, T, L * L)
    _, _, dwT = ocl.reduced_rel(red, static, T)
    errs = []
    for dt in (60.0, 30.0, 15.0):
        st = oracle.State.from_workload(w)
        oracle.dem_steps(m, st, dt, int(round(T / dt)))
        mom = oracle.moments(m, st)
        n, M, Lsp = mom[0, 0], mom[0, 1], mom[0, 4]
        ubar = mom[0, 5:7] / n
        W = Lsp / (M * static[0, 2])
        errs.append([abs(ubar[0] - rm[0, 5]), abs(ubar[1] - rm[0, 6]), abs(W - (0.0 - dwT[0])),
                     abs(mom[0, 7] - rm[0, 7]), abs(mom[0, 9] - rm[0, 9])])
    errs = np.array(errs)
    for q in range(errs.shape[1]):
        r1, r2 = errs[0, q] / errs[1, q], errs[1, q] / errs[2, q]
        assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, (q, r1, r2, errs[:, q])
    assert errs[2, 0] < 2e-3 * 0.2          # already close at dt = 15 s (initial |du| about 0.19 m/s)


def test_empty_cell_has_a_still_reduced_dem():
    w = _cell_of_floes([5000.0], [5000.0], [500.0], [1.0], [0.1], [0.0], [0.0], nx=2, ny=1, counts=[1, 0])
    m = oracle.Model(w)
    static = ocl.cell_static(w)
    oce = ocl.ocean_centres(w, m)
    red = ocl.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 0.0)
    assert np.all(np.isfinite(red)) and np.all(static[1] == 0.0)
    mom = ocl.reduced_moments(red, static, oce, 600.0, L * L)
    assert np.all(mom[1, 7:10] == 0.0)
    # an empty cell's coefficient <v> is 0, as the cell DEM's U / n with n = 0
    assert mom[1, 5] == 0.0 and mom[1, 6] == 0.0


def test_base_update_of_a_uniform_state():
    """Identical cells (one floe each, same place, same velocity) in a uniform
    current: the state stays uniform, so Lax-Friedrichs leaves the fluxes out
    and the base update adds dt times the sources: rho unchanged,
    P += dt alpha du |du| / A, P_w += dt beta dW |dW| / A."""
    nx = ny = 3
    r, h = 800.0, 1.5
    n = nx * ny
    w = fixtures.from_arrays(nx, ny, L, [1] * n, frac([4000.0] * n, L), frac([6000.0] * n, L), [r] * n, [h] * n,
                             u=[0.03] * n, v=[-0.02] * n, omega=[1e-4] * n, ocean=fixtures.Ocean(0.15, -0.08))
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    mom = oracle.moments(m, st)
    Q = oracle.q_from_moments(m, mom)
    static = ocl.cell_static(w)
    oce = ocl.ocean_centres(w, m)
    red = ocl.reduced_init(mom, static, oce, 0.0)
    dt, t = 30.0, 900.0
    Qb = ocl.base_update(w, m, Q, dt, red, t, static, oce)
    k = CD * RHO_O / (RHO_I * h)
    du0 = np.array([0.15 - float(np.float32(0.03)), -0.08 - float(np.float32(-0.02))])
    du = du0 / (1.0 + k * np.linalg.norm(du0) * t)
    kw = CD * RHO_O * r / (RHO_I * h)
    dW0 = -float(np.float32(1e-4))
    dW = dW0 / (1.0 + kw * abs(dW0) * t)
    alpha, beta = CD * RHO_O * math.pi * r * r, CD * RHO_O * math.pi * r ** 5
    for c in range(n):
        assert Qb[c, 0] == pytest.approx(Q[c, 0], rel=1e-14)
        np.testing.assert_allclose(Qb[c, 1:3], Q[c, 1:3] + dt * alpha * np.linalg.norm(du) * du / (L * L),
                                   rtol=1e-12)
        assert Qb[c, 3] == pytest.approx(Q[c, 3] + dt * beta * abs(dW) * dW / (L * L), rel=1e-12)


def test_feature_rows_on_a_hand_built_lattice():
    """3 x 3 periodic grid, one floe per cell (radius and thickness per cell),
    Q[c, f] = 10 c + f + 0.5: the 45 inputs of cells 0, 4 and 5 written out."""
    nx = ny = 3
    n = 9
    r = 300.0 + 50.0 * np.arange(n)
    h = 0.6 + 0.1 * np.arange(n)
    u = 0.01 * np.arange(n)
    w = fixtures.from_arrays(nx, ny, L, [1] * n, frac([5000.0] * n, L), frac([5000.0] * n, L), r, h,
                             u=u, v=-u, omega=1e-5 * np.arange(n), ocean=fixtures.Ocean(0.2, 0.1))
    m = oracle.Model(w)
    static = ocl.cell_static(w)
    oce = ocl.ocean_centres(w, m)
    red = ocl.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 60.0)
    Q = np.array([[10.0 * c + f + 0.5 for f in range(4)] for c in range(n)])
    x = ocl.features(w, Q, [0, 4, 5], red, 60.0, static, oce)     # at the start time: no relaxation
    neighbours = {0: [8, 6, 7, 2, 0, 1, 5, 3, 4],    # row iy - 1 (south) first, west to east
                  4: [0, 1, 2, 3, 4, 5, 6, 7, 8],
                  5: [1, 2, 0, 4, 5, 3, 7, 8, 6]}
    for row, c in enumerate([0, 4, 5]):
        expect = []
        for nb in neighbours[c]:
            expect += [10.0 * nb + 0.5, 10.0 * nb + 1.5, 10.0 * nb + 2.5, 10.0 * nb + 3.5]
        rc, hc = float(np.float32(r[c])), float(np.float32(h[c]))
        uc = float(np.float32(u[c]))
        expect += [0.2, 0.1, 0.0]
        expect += [math.pi * rc * rc / (L * L), hc, rc * rc]
        expect += [0.2 - uc, 0.1 - float(np.float32(-u[c])), 0.0 - float(np.float32(1e-5 * c))]
        np.testing.assert_allclose(x[row], expect, rtol=1e-12, atol=1e-15)


def test_spin_relaxes_toward_half_the_curl_at_the_cell_centre():
    """A floe at rest at the cell centre, where a shear current v_o = a k cos(k X + p)
    vanishes and its curl -a k^2 sin(k X + p) peaks: the floe stays put and its spin
    relaxes to half the curl (eq. dem_omega); the reduced DEM's spin
    curl / 2 - dW(t) matches the oracle's at first order in dt."""
    kx = 2.0 * math.pi / (4.0 * L)
    ph = 0.5 * math.pi - kx * 0.5 * L
    a = 1e-5 / kx ** 2
    oc = fixtures.Ocean.from_streamfunction([a], [kx], [0.0], [ph])
    w = fixtures.from_arrays(1, 1, L, [1], frac([0.5 * L], L), frac([0.5 * L], L), [1500.0], [0.9],
                             omega=[2e-5], ocean=oc)
    m = oracle.Model(w)
    static = ocl.cell_static(w)
    oce = ocl.ocean_centres(w, m)
    assert abs(oce[0, 1]) < 1e-12 and oce[0, 2] == pytest.approx(-1e-5, rel=1e-9)
    red = ocl.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 0.0)
    T = 3000.0
    _, _, dw = ocl.reduced_rel(red, static, T)
    errs = []
    for dt in (60.0, 30.0, 15.0):
        st = oracle.State.from_workload(w)
        oracle.dem_steps(m, st, dt, int(round(T / dt)))
        errs.append(abs(st.w[0] - (0.5 * oce[0, 2] - dw[0])))
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2, errs
    assert errs[2] < 1e-2 * abs(2e-5 + 0.5e-5)
