"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Every test here runs on the CPU and exercises only ``oracle/`` (and the input
generators).  Each test names what it pins and would fail on a plausible
mistake: a wrong sign or index in the contact law, a dropped drag term, a
transposed stencil, a wrong power of the radius, a wrong summation order.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import fixtures
import oracle
from helpers import TWO32, frac, kinetic, momentum, random_cell, two_floes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
L2 = 32768.0   # dyadic cell side: x = L xi / 2^32 is exact in FP64


# ------------------------------------------------------------ contact search
def exact_pairs(w):
    """Brute force with exact rational arithmetic: d^2 < (r_l + r_j)^2."""
    out = []
    n = w.nfloes
    for l in range(n):
        for j in range(l + 1, n):
            dxi = (int(w.xi[j]) - int(w.xi[l]) + 2 ** 31) % 2 ** 32 - 2 ** 31
            dyi = (int(w.yi[j]) - int(w.yi[l]) + 2 ** 31) % 2 ** 32 - 2 ** 31
            dx = Fraction(dxi) * Fraction(w.Lx) / (1 << 32)
            dy = Fraction(dyi) * Fraction(w.Ly) / (1 << 32)
            R = Fraction(float(w.r[l])) + Fraction(float(w.r[j]))
            if dx * dx + dy * dy < R * R:
                out.append((l, j))
    return np.array(out, np.int64).reshape(-1, 2)


@pytest.mark.parametrize("seed", range(6))
def test_pairs_brute_matches_exact_rational(seed):
    rng = np.random.default_rng(seed)
    w = random_cell(rng, 24, L2, 1500.0, 4000.0)
    got = oracle.pairs_cell(oracle.Model(w), oracle.State.from_workload(w), 0)
    ref = exact_pairs(w)
    assert len(ref) > 0
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("seed", range(12))
def test_pairs_binned_equals_brute(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 64))
    L = float(rng.choice([L2, 25000.0, 50000.0]))
    rmax = L / float(rng.choice([6.5, 9.0, 20.0]))
    w = random_cell(rng, n, L, 0.3 * rmax, rmax)
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    np.testing.assert_array_equal(oracle.pairs_cell(m, st, 0, binned=True),
                                  oracle.pairs_cell(m, st, 0, binned=False))


def test_exact_touch_is_not_contact_and_one_unit_closer_is():
    # r = 1500 + 1500 = 3000 m = 3000 * 2^17 units of L2 / 2^32
    unit = L2 / TWO32
    d_units = int(3000.0 / unit)
    assert d_units * unit == 3000.0
    for x0 in (0, 2 ** 32 - d_units // 2):          # in the interior and across the seam
        for delta, expect in ((0, 0), (-1, 1), (1, 0)):
            xi = np.array([x0, (x0 + d_units + delta) % 2 ** 32], np.uint32)
            w = fixtures.from_arrays(1, 1, L2, [2], xi, [7, 7], [1500.0, 1500.0], [1.0, 1.0])
            got = oracle.pairs_cell(oracle.Model(w), oracle.State.from_workload(w), 0)
            assert len(got) == expect, (x0, delta)


def test_chord_closed_forms():
    # equal radii: c = 2 sqrt(r^2 - d^2/4); containment: 2 min(r); tangency: 0
    for r, d in ((1.0, 1.5), (1500.0, 2900.0), (3.0, 0.5)):
        assert oracle.chord(r, r, d) == pytest.approx(2 * math.sqrt(r * r - d * d / 4), rel=1e-13)
    assert oracle.chord(2.0, 0.5, 1.0) == 1.0
    assert oracle.chord(1.0, 2.0, 3.0) == 0.0
    # 3-4-5: circles of radius 3 and 4 at distance 5 meet at right angles; chord = 2*12/5
    assert oracle.chord(3.0, 4.0, 5.0) == pytest.approx(4.8, rel=1e-14)


# ------------------------------------------------------------------- ocean
def test_scenario_4_3_divergence_matches_paper():
    g = json.load(open(os.path.join(GOLDEN, "paper_scenarios.json")))["scenario_4_3"]
    assert "0.04 pi" in g["divergence"]
    p = math.pi
    # u = 0.3 - 0.05[sin(0.1 pi x + pi y) + sin(0.1 pi x - pi y)]
    # v = 0.025[sin(0.1 pi x + pi y) - sin(0.1 pi x - pi y)]
    oc = fixtures.Ocean(0.3, 0.0, np.array([0.1 * p, 0.1 * p]), np.array([p, -p]),
                        np.array([-0.05, -0.05]), np.array([0.025, -0.025]), np.zeros(2))
    w = fixtures.from_arrays(1, 1, 1.0, [0], [], [], [], [], ocean=oc)
    m = oracle.Model(w)
    rng = np.random.default_rng(0)
    eps = 1e-5
    for X, Y in rng.uniform(0, 2, (20, 2)):
        a = oracle.ocean_at(m, X, Y)
        u_ref = 0.3 - 0.1 * math.sin(0.1 * p * X) * math.cos(p * Y)
        v_ref = 0.05 * math.cos(0.1 * p * X) * math.sin(p * Y)
        assert a[0] == pytest.approx(u_ref, abs=1e-14) and a[1] == pytest.approx(v_ref, abs=1e-14)
        dudx = (oracle.ocean_at(m, X + eps, Y)[0] - oracle.ocean_at(m, X - eps, Y)[0]) / (2 * eps)
        dvdy = (oracle.ocean_at(m, X, Y + eps)[1] - oracle.ocean_at(m, X, Y - eps)[1]) / (2 * eps)
        div = 0.04 * p * math.cos(0.1 * p * X) * math.cos(p * Y)
        assert dudx + dvdy == pytest.approx(div, abs=1e-8)
        # curl returned by the oracle = dv/dX - du/dY by central differences
        dvdx = (oracle.ocean_at(m, X + eps, Y)[1] - oracle.ocean_at(m, X - eps, Y)[1]) / (2 * eps)
        dudy = (oracle.ocean_at(m, X, Y + eps)[0] - oracle.ocean_at(m, X, Y - eps)[0]) / (2 * eps)
        assert a[2] == pytest.approx(dvdx - dudy, abs=1e-8)


def test_streamfunction_fields_are_divergence_free():
    w = fixtures.make_config(1)
    m = oracle.Model(w)
    D = w.nx * w.Lx
    eps = 1.0
    for X, Y in np.random.default_rng(1).uniform(0, D, (10, 2)):
        dudx = (oracle.ocean_at(m, X + eps, Y)[0] - oracle.ocean_at(m, X - eps, Y)[0]) / (2 * eps)
        dvdy = (oracle.ocean_at(m, X, Y + eps)[1] - oracle.ocean_at(m, X, Y - eps)[1]) / (2 * eps)
        dvdx = (oracle.ocean_at(m, X + eps, Y)[1] - oracle.ocean_at(m, X - eps, Y)[1]) / (2 * eps)
        assert abs(dudx + dvdy) < 1e-12 + 1e-6 * abs(dvdx)


# ---------------------------------------------------------- single floe drag
def _drag_run(dt, T, U0=(0.2, 0.1), w0=2e-4, r=1200.0, h=0.8):
    oc = fixtures.Ocean(U0[0], U0[1])
    w = fixtures.from_arrays(1, 1, L2 * 64, [1], frac([1000.0], L2 * 64), frac([1000.0], L2 * 64),
                             [r], [h], omega=[w0], ocean=oc)
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    oracle.dem_steps(m, st, dt, int(round(T / dt)))
    return w, st


def test_single_floe_drag_closed_form_first_order():
    """Uniform current, no contact: dv/dt = k (u_o - v)|u_o - v| with
    k = Cd rho_o / (rho_ice h) (eq. dem_v with alpha = Cd rho_o pi r^2, m = rho_ice h pi r^2):
    du(t) = du0 / (1 + k |du0| t) and x(t) = x0 + u_o t - du0/|du0| ln(1 + k|du0|t) / k.
    Spin (zero curl): w(t) = w0 / (1 + k_w |w0| t), k_w = Cd rho_o r / (rho_ice h)."""
    T = 1800.0
    errs = []
    for dt in (60.0, 30.0, 15.0):
        w, st = _drag_run(dt, T)
        U0 = np.array([0.2, 0.1])
        k = w.cd * w.rho_ocean / (w.rho_ice * 0.8)
        du0 = U0.copy()
        s0 = np.linalg.norm(du0)
        du = du0 / (1 + k * s0 * T)
        v_ref = U0 - du
        x_ref = 1000.0 + U0[0] * T - du0[0] / s0 * math.log(1 + k * s0 * T) / k
        kw = w.cd * w.rho_ocean * 1200.0 / (w.rho_ice * 0.8)
        w_ref = 2e-4 / (1 + kw * 2e-4 * T)
        x = st.xs[0] * w.Lx
        errs.append((abs(st.u[0] - v_ref[0]), abs(x - x_ref), abs(st.w[0] - w_ref)))
        assert abs(st.v[0] - v_ref[1]) < 0.05 * abs(v_ref[1])
    errs = np.array(errs)
    for q in range(3):
        assert errs[2, q] < errs[1, q] < errs[0, q]
        r1, r2 = errs[0, q] / errs[1, q], errs[1, q] / errs[2, q]
        assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, (q, r1, r2)
    assert errs[2, 0] < 5e-3 * 0.2


def test_spin_relaxes_to_half_ocean_vorticity():
    """eq. dem_omega: the drag torque vanishes at w = (curl u_o)/2.  A floe in a
    meridional current v_o = 0.3 cos(kX) drifts along y at fixed X, so the
    curl it samples is constant and its spin converges to half of it."""
    k = 2 * math.pi / 50e3
    oc = fixtures.Ocean(0.0, 0.0, np.array([k]), np.array([0.0]), np.array([0.0]), np.array([0.3]),
                        np.array([0.5 * math.pi]))
    L = 25e3
    w = fixtures.from_arrays(16, 1, L, [0, 0, 0, 1] + [0] * 12, frac([5000.0], L), frac([5000.0], L),
                             [4000.0], [2.0], ocean=oc)
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    oracle.dem_steps(m, st, 600.0, 10000)
    X = (3 + st.xs[0]) * L
    zeta = oracle.ocean_at(m, X, 0.0)[2]
    assert zeta == pytest.approx(-0.3 * k * math.sin(k * X), rel=1e-12)
    assert abs(zeta) > 1e-5
    assert st.w[0] == pytest.approx(0.5 * zeta, rel=2e-3)
    assert st.u[0] == 0.0                                   # no x forcing
    assert st.v[0] == pytest.approx(0.3 * math.cos(k * X), rel=1e-3)


# ------------------------------------------------------- two-floe collisions
def _head_on(dt, T, ocean_off=True, mu=0.3, G=5e3):
    w = two_floes(L2, 10000.0, 16000.0, 13100.0, 16000.0, 1500.0, 1500.0, 1.25, 1.25,
                  u1=(0.1, 0.0), u2=(-0.1, 0.0), mu=mu, G=G)
    m = oracle.Model(w, oracle.OCEAN_OFF if ocean_off else 0)
    st = oracle.State.from_workload(w)
    ke0, p0 = kinetic(st, w), momentum(st, w)
    oracle.dem_steps(m, st, dt, int(round(T / dt)))
    return w, m, st, ke0, p0


def test_head_on_elastic_exchange_and_conservation():
    """Ocean off, head-on, equal masses: the normal spring is conservative, so
    the collision exchanges the velocities (1-D elastic collision) in the limit
    dt -> 0; momentum is conserved at every dt; no tangential force, no spin."""
    errs = []
    for dt in (60.0, 30.0, 15.0):
        w, m, st, ke0, p0 = _head_on(dt, 6000.0)
        assert oracle.pairs_cell(m, st, 0).size == 0          # separated again
        p1 = momentum(st, w)
        scale = w.rho_ice * 1.25 * math.pi * 1500.0 ** 2 * 0.1     # one floe's momentum
        assert np.all(np.abs(p1 - p0) <= 1e-14 * scale)
        assert np.all(st.w == 0.0) and np.all(st.v == 0.0)
        assert abs(kinetic(st, w) / ke0 - 1) < 5e-3
        errs.append(max(abs(st.u[0] + 0.1), abs(st.u[1] - 0.1)))
    assert errs[2] < errs[1] < errs[0] and errs[2] < 2e-4


def test_forward_euler_flag_gains_energy():
    """The literal forward Euler reading is unstable for the contact spring at
    dt = 60 s: kinetic energy grows across a collision (hence the semi-implicit default)."""
    w = two_floes(L2, 10000.0, 16000.0, 13100.0, 16000.0, 1500.0, 1500.0, 1.25, 1.25,
                  u1=(0.1, 0.0), u2=(-0.1, 0.0))
    m = oracle.Model(w, oracle.OCEAN_OFF | oracle.FORWARD_EULER)
    st = oracle.State.from_workload(w)
    ke0 = kinetic(st, w)
    oracle.dem_steps(m, st, 60.0, 100)
    assert kinetic(st, w) / ke0 > 1.1


def test_momentum_changes_only_by_drag():
    """With the ocean on, contact forces cancel pairwise, so the cell momentum
    changes by exactly dt * sum of drag forces (momentum equation of eq:pde)."""
    oc = fixtures.random_modes(np.random.default_rng(3), 3, 4 * L2, 4 * L2)
    oc.u0, oc.v0 = 0.05, -0.02
    w = two_floes(L2, 10000.0, 16000.0, 13050.0, 16300.0, 1500.0, 1400.0, 1.0, 1.6,
                  u1=(0.15, 0.0), u2=(-0.1, 0.02), ocean=oc)
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    p0 = momentum(st, w)
    mom, stats = oracle.dem_steps(m, st, 30.0, 200, record=True)
    assert stats[0] > 0
    dp = 30.0 * mom[:, 0, [oracle.MOMENT_NAMES.index("Svx"), oracle.MOMENT_NAMES.index("Svy")]].sum(0)
    scale = np.abs(momentum(st, w)).max() + np.abs(p0).max()
    np.testing.assert_allclose(momentum(st, w) - p0, dp, atol=1e-12 * scale)
    np.testing.assert_allclose(mom[-1, 0, 2:4], momentum(_prestep(w, m, 199), w), rtol=1e-12)


def _prestep(w, m, k):
    st = oracle.State.from_workload(w)
    oracle.dem_steps(m, st, 30.0, k)
    return st


def test_oblique_sliding_contact_obeys_coulomb():
    """Ocean off, oblique impact with fast tangential slip and a large viscous
    coefficient.  Step by step, the force on floe 1 (from its velocity change)
    split along n (l -> j) and t = (-n_y, n_x) must satisfy: the tangential part
    equals the torque over the radius (torque = r F_t), it is saturated at
    mu |F_n| and has the sign of the slip v_t; F_n is repulsive.  Both spins end
    with the same sign and the kinetic energy decreases."""
    r1, r2 = 1500.0, 1300.0
    w = two_floes(L2, 10000.0, 16000.0, 12800.0, 16000.0, r1, r2, 1.0, 1.4,
                  u1=(0.1, 0.2), u2=(-0.1, -0.2), G=1e7)
    m = oracle.Model(w, oracle.OCEAN_OFF)
    st = oracle.State.from_workload(w)
    ke0 = kinetic(st, w)
    mass = w.rho_ice * 1.0 * math.pi * r1 * r1
    I = mass * r1 * r1
    dt = 5.0
    seen = 0
    for _ in range(1200):
        pre = st.copy()
        oracle.dem_steps(m, st, dt, 1)
        if oracle.pairs_cell(m, pre, 0).size == 0:
            continue
        seen += 1
        dx = ((pre.xs[1] - pre.xs[0] + 0.5) % 1.0 - 0.5) * w.Lx
        dy = ((pre.ys[1] - pre.ys[0] + 0.5) % 1.0 - 0.5) * w.Ly
        d = math.hypot(dx, dy)
        n = np.array([dx, dy]) / d
        t = np.array([-n[1], n[0]])
        F = mass * np.array([st.u[0] - pre.u[0], st.v[0] - pre.v[0]]) / dt
        Fn, Ft = F @ n, F @ t
        assert Fn < 0
        assert Ft == pytest.approx(I * (st.w[0] - pre.w[0]) / (r1 * dt), rel=1e-9, abs=1e-9 * abs(Fn))
        vt = (pre.u[1] - pre.u[0]) * t[0] + (pre.v[1] - pre.v[0]) * t[1] - pre.w[1] * r2 - pre.w[0] * r1
        assert np.sign(Ft) == np.sign(vt)
        assert abs(Ft) == pytest.approx(w.mu * abs(Fn), rel=1e-9)
    assert seen > 10
    assert oracle.pairs_cell(m, st, 0).size == 0
    assert st.w[0] != 0 and np.sign(st.w[0]) == np.sign(st.w[1])
    assert kinetic(st, w) < ke0


# ------------------------------------------------------ paper's scenarios
def _scenario_41(ncx=4, ncy=2):
    g = json.load(open(os.path.join(GOLDEN, "paper_scenarios.json")))["scenario_4_1"]
    rc = g["r_c"]
    Lc = g["domain"][0] / g["coarse_grid"][0]               # 1/12
    per = int(round(math.sqrt(g["floes_per_coarse_cell"])))  # 10 x 10 fine cells per coarse cell
    xs, ys, rs, counts = [], [], [], []
    for cy in range(ncy):
        for cx in range(ncx):
            cnt = 0
            for j in range(per):
                for i in range(per):
                    fx, fy = (i + 0.5) / per, (j + 0.5) / per
                    X = (cx + fx) * Lc
                    xs.append(fx)
                    ys.append(fy)
                    rs.append(rc * (0.2 + 0.8 * math.sin(0.25 * math.pi * X)))
                    cnt += 1
            counts.append(cnt)
    n = len(xs)
    xi = (np.round(np.array(xs) * TWO32)).astype(np.uint32)
    yi = (np.round(np.array(ys) * TWO32)).astype(np.uint32)
    # the current equals the floes' stored (FP32) velocity exactly
    oc = fixtures.Ocean(*[float(np.float32(c)) for c in g["ocean_velocity"]])
    w = fixtures.from_arrays(ncx, ncy, Lc, counts, xi, yi, rs, np.ones(n), u=np.full(n, 0.3), ocean=oc)
    w.rho_ice = w.rho_ocean = 1.0
    return g, w


def test_scenario_4_1_pure_drift():
    """Sec. 4.1: floes at the fine-cell centres drifting with the current never
    touch and feel no drag; the concentration per coarse cell is the floe area
    over the cell area and stays constant."""
    g, w = _scenario_41()
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    mom0 = oracle.moments(m, st)
    dt = 1e-4
    mom, stats = oracle.dem_steps(m, st, dt, 50, record=True)
    assert stats[0] == g["contacts"]
    assert np.all(st.w == 0.0) and np.all(st.u == np.float32(0.3))
    shift = (st.xs - np.round(oracle.State.from_workload(w).xs * TWO32) / TWO32) % 1.0
    np.testing.assert_allclose(shift * w.Lx, float(np.float32(0.3)) * 50 * dt, rtol=1e-9)
    np.testing.assert_allclose(mom[-1], mom0, rtol=1e-12, atol=1e-300)
    assert np.all(mom[:, :, 7:10] == 0.0)                   # no drag, no torque
    conc = mom0[:, 10] / (w.Lx * w.Ly)
    assert w.Lx * w.Ly == pytest.approx(g["coarse_cell_area"], rel=1e-12)
    rc = g["r_c"]
    for c in range(w.ncells):
        cx = c % w.nx
        X = (cx + (np.arange(10) + 0.5) / 10) * w.Lx
        ref = 10 * np.sum(np.pi * (rc * (0.2 + 0.8 * np.sin(0.25 * np.pi * X)).astype(np.float32).astype(np.float64)) ** 2)
        assert conc[c] == pytest.approx(ref / g["coarse_cell_area"], rel=1e-6)


def test_scenario_4_2_spin_stays_zero():
    """Sec. 4.2: a one-dimensional compressible current (0.3 - 0.1 cos(pi x), 0)
    has zero curl, and floes in aligned rows collide head-on, so the spin stays
    exactly zero although collisions happen."""
    p = math.pi
    oc = fixtures.Ocean(0.3, 0.0, np.array([p]), np.array([0.0]), np.array([-0.1]), np.array([0.0]),
                        np.array([0.5 * p]))
    Lc = 1.0 / 12
    per = 6
    xs, ys, rs, counts = [], [], [], []
    ncx = 8
    for cx in range(ncx):
        for j in range(per):
            for i in range(per):
                xs.append((i + 0.5) / per)
                ys.append((j + 0.5) / per)
                rs.append(0.49 * Lc / per)
        counts.append(per * per)
    n = len(xs)
    xi = (np.round(np.array(xs) * TWO32)).astype(np.uint32)
    yi = (np.round(np.array(ys) * TWO32)).astype(np.uint32)
    X = (np.repeat(np.arange(ncx), per * per) + np.array(xs)) * Lc
    u = 0.3 - 0.1 * np.cos(p * X)
    w = fixtures.from_arrays(ncx, 1, Lc, counts, xi, yi, rs, np.ones(n), u=u, ocean=oc, G=1.0)
    w.rho_ice = w.rho_ocean = 1.0
    w.cd = 50.0
    w.E = 1e3
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    tot = 0
    for _ in range(20):
        _, stats = oracle.dem_steps(m, st, 2e-4, 50)
        tot += stats[0]
        assert np.all(st.w == 0.0) and np.all(st.v == 0.0)
    assert tot > 0


# ---------------------------------------------------------- continuum (LF)
def _grid_model(nx, ny, L=1000.0):
    w = fixtures.from_arrays(nx, ny, L, np.zeros(nx * ny, np.int32), [], [], [], [])
    return oracle.Model(w)


def _uniform_mom(nc, ubar, vbar, n=10.0):
    mom = np.zeros((nc, oracle.NMOM))
    mom[:, 0] = n
    mom[:, 5] = ubar * n
    mom[:, 6] = vbar * n
    return mom


def test_lf_fourier_mode_amplification():
    """Uniform coefficients: LF multiplies a Fourier mode exp(i(a x + b y)) by
    g = (cos a + cos b)/2 - i (Cx sin a + Cy sin b), C = u dT / dX, for the
    conservative and the Oseen (advective) forms alike."""
    nx, ny, L, dT = 16, 8, 1000.0, 40.0
    m = _grid_model(nx, ny, L)
    ub, vb = 3.0, -5.0
    mom = _uniform_mom(nx * ny, ub, vb)
    kx, ky = 3, 2
    a, b = 2 * math.pi * kx / nx, 2 * math.pi * ky / ny
    iy, ix = np.divmod(np.arange(nx * ny), nx)
    ph = a * ix + b * iy
    Q = np.zeros((nx * ny, 4))
    for f in range(4):
        Q[:, f] = np.cos(ph + f)
    Qn, cfl = oracle.lf_step(m, Q, mom, dT)
    Cx, Cy = ub * dT / L, vb * dT / L
    g = 0.5 * (math.cos(a) + math.cos(b)) - 1j * (Cx * math.sin(a) + Cy * math.sin(b))
    for f in range(4):
        ref = np.real(g * np.exp(1j * (ph + f)))
        np.testing.assert_allclose(Qn[:, f], ref, atol=1e-14)
    assert cfl == pytest.approx(abs(Cx) + abs(Cy), rel=1e-15)


def test_lf_conserves_mass_and_spin_with_variable_coefficients():
    """Periodic telescoping: the conservative form keeps sum(rho) exactly (to
    rounding) for any coefficient field; sum(P_w) changes by dT * sum(S_w)/A."""
    nx, ny, L, dT = 12, 10, 25e3, 30.0
    m = _grid_model(nx, ny, L)
    rng = np.random.default_rng(0)
    mom = _uniform_mom(nx * ny, 0.0, 0.0)
    mom[:, 5] = rng.normal(0, 0.2, nx * ny) * mom[:, 0]
    mom[:, 6] = rng.normal(0, 0.2, nx * ny) * mom[:, 0]
    mom[:, 9] = rng.normal(0, 1e6, nx * ny)
    mom[:, 7] = rng.normal(0, 1e5, nx * ny)
    Q = np.abs(rng.normal(300, 50, (nx * ny, 4)))
    Qn, _ = oracle.lf_step(m, Q, mom, dT)
    assert Qn[:, 0].sum() == pytest.approx(Q[:, 0].sum(), rel=1e-14)
    assert Qn[:, 3].sum() == pytest.approx(Q[:, 3].sum() + dT * mom[:, 9].sum() / (L * L), rel=1e-14)
    # the Oseen momentum form does not conserve with variable coefficients, but
    # a uniform momentum field only feels the source
    Q[:, 1] = 7.0
    Qn, _ = oracle.lf_step(m, Q, mom, dT)
    np.testing.assert_allclose(Qn[:, 1], 7.0 + dT * mom[:, 7] / (L * L), rtol=1e-14)


def test_lf_uniform_state_and_empty_cells():
    nx, ny = 5, 4
    m = _grid_model(nx, ny)
    mom = _uniform_mom(nx * ny, 0.4, 0.1)
    mom[3] = 0.0                        # an empty cell: zero coefficients and sources
    Q = np.tile(np.array([[2.0, -1.0, 0.5, 3.0]]), (nx * ny, 1))
    mom[:, 0] = np.where(np.arange(nx * ny) == 3, 0.0, 10.0)
    Qn, _ = oracle.lf_step(m, Q, _uniform_mom(nx * ny, 0.4, 0.1), 10.0)
    np.testing.assert_allclose(Qn, Q, rtol=1e-15)


def test_lf_stencil_orientation():
    """A single bump advected by a positive x velocity moves mass east: the
    east neighbour gains (1/4 + C/2)... exactly the LF weights."""
    nx, ny, L, dT = 8, 8, 1000.0, 100.0
    m = _grid_model(nx, ny, L)
    mom = _uniform_mom(nx * ny, 2.0, 0.0)
    Q = np.zeros((nx * ny, 4))
    c0 = 3 * nx + 3
    Q[c0, 0] = 1.0
    Qn, _ = oracle.lf_step(m, Q, mom, dT)
    C = 2.0 * dT / L
    assert Qn[c0 + 1, 0] == pytest.approx(0.25 + 0.5 * C)   # east: receives from its west neighbour
    assert Qn[c0 - 1, 0] == pytest.approx(0.25 - 0.5 * C)
    assert Qn[c0 + nx, 0] == pytest.approx(0.25) and Qn[c0 - nx, 0] == pytest.approx(0.25)
    assert Qn[c0, 0] == 0.0


# ------------------------------------------------- coarse-to-fine resync
def test_resync_hits_targets():
    w = fixtures.custom(2, 2, 25e3, 40, seed=5, r_scale=0.3)
    rng = np.random.default_rng(2)
    w.u[:] = rng.normal(0, 0.1, w.nfloes)
    w.omega[:] = rng.normal(0, 1e-5, w.nfloes)
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    mom = oracle.moments(m, st)
    Q = oracle.q_from_moments(m, mom)
    target = Q[1] * np.array([1.03, 0.5, -2.0, 1.7])
    oracle.resync_cell(m, st, 1, target)
    Q2 = oracle.q_from_moments(m, oracle.moments(m, st))
    np.testing.assert_allclose(Q2[1], target, rtol=1e-12)
    np.testing.assert_array_equal(Q2[0], Q[0])
    # radii scaled by a common factor
    s, e = w.start[1], w.start[2]
    ratio = st.r[s:e] / w.r[s:e]
    np.testing.assert_allclose(ratio, math.sqrt(1.03), rtol=1e-14)


# --------------------------------------------------------- cell statistics
def test_moments_closed_form_identical_floes():
    """Identical floes: M = n m, P = n m v, L = n I w, U = n v, A = n pi r^2."""
    n = 9
    L = 50e3
    xi = frac(np.arange(n) * 5000.0 + 100.0, L)
    w = fixtures.from_arrays(1, 1, L, [n], xi, frac(np.full(n, 2500.0), L), np.full(n, 1000.0),
                             np.full(n, 1.5), u=np.full(n, 0.25), v=np.full(n, -0.125),
                             omega=np.full(n, 1e-4), ocean=fixtures.Ocean(0.25, -0.125))
    m = oracle.Model(w)
    mom = oracle.moments(m, oracle.State.from_workload(w))[0]
    mass = 920.0 * 1.5 * math.pi * 1e6
    I = mass * 1e6
    np.testing.assert_allclose(mom[:7], [n, n * mass, n * mass * 0.25, -n * mass * 0.125,
                                         n * I * float(np.float32(1e-4)), n * 0.25, -n * 0.125], rtol=1e-14)
    # zero translational drag (v = u_o); torque drives w back to zero:
    beta = w.cd * w.rho_ocean * math.pi * 1000.0 ** 5
    w32 = float(np.float32(1e-4))
    assert mom[7] == 0.0 and mom[8] == 0.0
    assert mom[9] == pytest.approx(-n * beta * w32 * w32, rel=1e-14)
    assert mom[10] == pytest.approx(n * math.pi * 1e6, rel=1e-15)


def test_full_path_q0_is_initial_statistics_and_steps_are_deterministic():
    w = fixtures.make_config(0)
    st, Q, mom, cfl = oracle.run_plain(w, 5)
    st2, Q2, mom2, _ = oracle.run_plain(w, 5)
    np.testing.assert_array_equal(Q, Q2)
    np.testing.assert_array_equal(st.xs, st2.xs)
    _, Q0, _, _ = oracle.run_plain(w, 0)
    m = oracle.Model(w)
    mom0 = oracle.moments(m, oracle.State.from_workload(w))
    A = w.Lx * w.Ly
    np.testing.assert_allclose(Q0[:, 0], mom0[:, 1] / A, rtol=1e-15)
    assert 0 < cfl < 1e-2
