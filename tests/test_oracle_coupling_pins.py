"""Pins of the oracle's two-way coupling (Algorithm 1 with a coarse step of N0
fine steps, N1 sub-steps and coarse-to-fine updates every n_t steps).

Each expectation comes from something other than the coupling driver itself:
the plain path it must reduce to, Fourier multipliers of the Lax-Friedrichs
stencil (diagonalised with numpy's FFT), or the DEM's own per-step statistics
recorded on a separate copy.  A wrong window (N0 - 1 samples, post-step
statistics), a wrong sub-step size, a nudge in the first coarse step, a nudge
fraction off by one sub-step or nudges off the n_t grid each fail one of them.
"""
import math

import numpy as np
import pytest

import fixtures
import oracle
from workloads import lattice_workload

RHO, PX, PY, PW = 0, 1, 2, 3


def lf_multiplier_apply(q, nx, ny, ubar, vbar, dT, L, times):
    """Apply the Lax-Friedrichs step with uniform coefficients `times` times to
    one periodic field, as the Fourier multiplier
    g = (cos a + cos b) / 2 - i (Cx sin a + Cy sin b), C = u dT / L."""
    a = 2 * np.pi * np.fft.fftfreq(nx)[None, :]
    b = 2 * np.pi * np.fft.fftfreq(ny)[:, None]
    Cx, Cy = ubar * dT / L, vbar * dT / L
    g = 0.5 * (np.cos(a) + np.cos(b)) - 1j * (Cx * np.sin(a) + Cy * np.sin(b))
    F = np.fft.fft2(np.asarray(q, np.float64).reshape(ny, nx))
    return np.real(np.fft.ifft2(F * g ** times)).reshape(-1)


def cell_rho(w, st):
    m = oracle.Model(w)
    return oracle.q_from_moments(m, oracle.moments(m, st))[:, RHO]


def test_unit_cadence_is_the_plain_path():
    """N0 = N1 = n_t = 1: every step is a coarse step, no nudge ever runs."""
    w = fixtures.make_config(0)
    a = oracle.run_plain(w, 6)
    b = oracle.run_coupled(w, 6, 1, 1, 1)
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    for x, y in zip(a[0].arrays(), b[0].arrays()):
        np.testing.assert_array_equal(x, y)


STATIC = dict(nx=6, ny=4)


def _static():
    counts = np.random.default_rng(4).integers(1, 9, STATIC["nx"] * STATIC["ny"])
    return lattice_workload(counts, seed=4, **STATIC)


@pytest.mark.parametrize("nsteps", [3, 4, 5, 6, 7, 8, 9, 10])
def test_static_floes_follow_the_schedule_n0_4_n1_2_nt_2(nsteps):
    """Floes at rest, no ocean, no contacts: the DEM only changes at nudges and
    the coarse mass only diffuses (LF with zero coefficients multiplies a mode
    by (cos a + cos b) / 2 per sub-step).  N0 = 4, N1 = 2, n_t = 2:
    j = 4: Q1 = D^2 rho0;  j = 6: rho = rho0 + (2/4)(Q1 - rho0) = D6;
    j = 8: Q2 = D^2 Q1, X0 = D6;  j = 10: rho = D6 + (2/4)(Q2 - D6)."""
    w = _static()
    nx, ny, L = STATIC["nx"], STATIC["ny"], w.Lx
    rho0 = cell_rho(w, oracle.State.from_workload(w))
    D = lambda q, k: lf_multiplier_apply(q, nx, ny, 0.0, 0.0, 1.0, L, k)
    Q1 = D(rho0, 2)
    Q2 = D(Q1, 2)
    D6 = rho0 + 0.5 * (Q1 - rho0)
    D10 = D6 + 0.5 * (Q2 - D6)
    dem = {3: rho0, 4: rho0, 5: rho0, 6: D6, 7: D6, 8: D6, 9: D6, 10: D10}[nsteps]
    coarse = rho0 if nsteps < 4 else (Q1 if nsteps < 8 else Q2)
    st, Q, mom, cfl = oracle.run_coupled(w, nsteps, 4, 2, 2, flags=oracle.OCEAN_OFF)
    np.testing.assert_allclose(Q[:, RHO], coarse, rtol=1e-13)
    np.testing.assert_allclose(Q[:, 1:], 0.0, atol=0.0)
    np.testing.assert_allclose(cell_rho(w, st), dem, rtol=1e-13)
    # positions and velocities untouched; radii of a cell scaled by one factor
    w0 = oracle.State.from_workload(w)
    np.testing.assert_array_equal(st.xs, w0.xs)
    np.testing.assert_array_equal(st.u, 0.0)
    scale = np.repeat(np.sqrt(dem / rho0), np.diff(w.start))
    np.testing.assert_allclose(st.r / w0.r, scale, rtol=1e-13)
    assert cfl == 0.0


def test_static_floes_nudge_only_on_the_n_t_grid():
    """N0 = 6, n_t = 4, N1 = 1: the only nudge of a coarse step is at r = 4
    (fraction 4/6); r = 2 is no multiple of 4 and r = 8 lies past the step."""
    w = _static()
    nx, ny, L = STATIC["nx"], STATIC["ny"], w.Lx
    rho0 = cell_rho(w, oracle.State.from_workload(w))
    Q1 = lf_multiplier_apply(rho0, nx, ny, 0.0, 0.0, 1.0, L, 1)
    D10 = rho0 + (4.0 / 6.0) * (Q1 - rho0)
    for nsteps, expect in ((9, rho0), (10, D10), (12, D10)):
        st, Q, _, _ = oracle.run_coupled(w, nsteps, 6, 1, 4, flags=oracle.OCEAN_OFF)
        np.testing.assert_allclose(cell_rho(w, st), expect, rtol=1e-13)
    np.testing.assert_allclose(Q[:, RHO], lf_multiplier_apply(Q1, nx, ny, 0.0, 0.0, 1.0, L, 1), rtol=1e-13)


@pytest.mark.parametrize("N1", [1, 3])
def test_drifting_floes_first_coarse_step_is_n1_lf_substeps(N1):
    """Every floe drifts with (u, v), no forces: the window's coefficients are
    uniform and constant, so the first coarse step multiplies each mode by
    g(dT / N1)^N1 for all four fields (the sub-step count matters through g)."""
    nx, ny = 8, 4
    counts = np.random.default_rng(7).integers(1, 9, nx * ny)
    u, v = 0.35, -0.2
    w = lattice_workload(counts, nx, ny, u=u, v=v, seed=7)
    N0 = 5
    dT = N0 * w.dt
    m = oracle.Model(w, oracle.OCEAN_OFF)
    Q0 = oracle.q_from_moments(m, oracle.moments(m, oracle.State.from_workload(w)))
    st, Q, _, cfl = oracle.run_coupled(w, N0, N0, N1, 1, flags=oracle.OCEAN_OFF)
    ub, vb = float(np.float32(u)), float(np.float32(v))
    for f in range(4):
        ref = lf_multiplier_apply(Q0[:, f], nx, ny, ub, vb, dT / N1, w.Lx, N1)
        np.testing.assert_allclose(Q[:, f], ref, rtol=1e-12, atol=1e-12 * np.abs(Q0[:, f]).max())
    assert cfl == pytest.approx((abs(ub) + abs(vb)) * dT / N1 / w.Lx, rel=1e-12)
    if N1 == 1:
        Q3 = oracle.run_coupled(w, N0, N0, 3, 1, flags=oracle.OCEAN_OFF)[1]
        assert np.abs(Q3[:, RHO] - Q[:, RHO]).max() > 1e-6 * np.abs(Q[:, RHO]).max()


def test_uniform_cells_first_coarse_step_uses_the_mean_of_the_window():
    """Identical cells under a uniform current: the coarse fields stay uniform,
    the stencil acts as the identity and the momentum gains dT times the mean
    drag source of the window's N0 pre-step states (floes accelerate, so the
    first sample, the last one and the mean of the post-step samples all differ
    from that mean).  No curl and no spin: the spin source stays zero."""
    nx, ny = 3, 2
    ocean = fixtures.Ocean(0.3, -0.1)
    w = lattice_workload(np.full(nx * ny, 7), nx, ny, seed=9, big_radius=0.0, ocean=ocean, identical=True)
    N0 = 6
    m = oracle.Model(w)
    st0 = oracle.State.from_workload(w)
    Q0 = oracle.q_from_moments(m, oracle.moments(m, st0))
    rec, _ = oracle.dem_steps(m, st0.copy(), w.dt, N0 + 1, record=True)
    A = w.Lx * w.Ly
    S = rec[:, 0, [7, 8, 9]] / A              # (Svx, Svy, Sw) per step, identical cells
    mean = S[:N0].mean(axis=0)
    assert np.abs(S[0, :2] - mean[:2]).min() > 1e-2 * np.abs(mean).max()
    assert np.abs(S[N0 - 1, :2] - mean[:2]).min() > 1e-2 * np.abs(mean).max()
    assert np.abs(S[1:N0 + 1, :2].mean(axis=0) - mean[:2]).min() > 1e-2 * np.abs(mean).max()
    for N1 in (1, 4):
        _, Q, _, _ = oracle.run_coupled(w, N0, N0, N1, 2)
        ref = Q0[0] + N0 * w.dt * np.array([0.0, mean[0], mean[1], mean[2]])
        for c in range(nx * ny):
            np.testing.assert_allclose(Q[c], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
