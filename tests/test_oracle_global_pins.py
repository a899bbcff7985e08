"""Pins of the oracle's global DEM read-out (coarse-grid statistics of one DEM
over the whole domain, the reference of the paper's error study, Sec. 4).

The global DEM itself is the oracle's cell DEM with one cell spanning the
domain (pinned in test_oracle_pins.py); what is new is the assignment of floes
to coarse cells and the per-cell sums, checked here against counts and areas
known in closed form, against additivity over cells, and against a floe
crossing a cell edge at the step its drift predicts.
"""
import math

import numpy as np
import pytest

import fixtures
import oracle

TWO32 = 2.0 ** 32


def test_scenario_4_1_coarse_counts_and_concentration():
    """480 x 240 floes at the fine-cell centres on a 48 x 24 coarse grid: 100
    floes per coarse cell (as printed in Sec. 4.1) and concentration = the sum
    of the floes' disk areas over the cell area."""
    w = fixtures.scenario_global(1)
    st = oracle.State.from_workload(w)
    mom = oracle.coarse_moments(w, st, 48, 24)
    assert np.all(mom[:, 0] == 100)
    A = (4.0 / 48) * (2.0 / 24)
    cx = np.arange(48 * 24) % 48
    for c in (0, 5, 23, 47, 48 * 24 - 1):
        X = (cx[c] * 10 + np.arange(10) + 0.5) / 120.0
        r = (1 / 240) * (0.2 + 0.8 * np.sin(0.25 * np.pi * X))
        ref = 10 * np.sum(np.pi * r.astype(np.float32).astype(np.float64) ** 2) / A
        assert mom[c, 10] / A == pytest.approx(ref, rel=1e-6)
    np.testing.assert_array_equal(mom[:, 7:10], 0.0)        # floes move with the current


def test_coarse_sums_add_up_to_the_single_cell():
    """Every additive statistic summed over the coarse cells equals the one of
    the whole domain taken as a single cell."""
    w = fixtures.custom(1, 1, 100e3, 400, seed=12, r_scale=0.3)
    rng = np.random.default_rng(3)
    w.u[:] = rng.normal(0, 0.2, w.nfloes)
    w.v[:] = rng.normal(0, 0.2, w.nfloes)
    w.omega[:] = rng.normal(0, 1e-4, w.nfloes)
    st = oracle.State.from_workload(w)
    whole = oracle.moments(oracle.Model(w), st)[0]
    for nxc, nyc in ((1, 1), (4, 4), (7, 3)):
        mom = oracle.coarse_moments(w, st, nxc, nyc)
        np.testing.assert_allclose(mom.sum(axis=0), whole, rtol=1e-10, atol=1e-9 * np.abs(whole).max())
        assert mom[:, 0].sum() == w.nfloes


def test_a_drifting_floe_changes_cell_when_its_centre_crosses_the_edge():
    """One floe at x = 0.24 L drifting with the current (0.1 L per 100 steps):
    on a 4 x 1 coarse grid it leaves cell 0 for cell 1 in the step that takes
    its centre past 0.25 L, and wraps from the last cell to the first."""
    L = 40e3
    dt = 100.0
    u = 4.0        # m/s: 400 m per step, edge at 10 km
    xi = np.array([int(0.24 * TWO32)], np.uint32)
    oc = fixtures.Ocean(u, 0.0)
    w = fixtures.from_arrays(1, 1, L, [1], xi, np.array([TWO32 // 2], np.uint64).astype(np.uint32), [500.0],
                             [1.0], u=[u], ocean=oc, dt=dt)
    st = oracle.State.from_workload(w)
    x0 = st.xs[0] * L
    cell_of = lambda s: int(np.argmax(oracle.coarse_moments(w, s, 4, 1)[:, 0]))
    for k in range(1, 80):
        oracle.run_global(w, 1, state=st)
        expect = int(((x0 + k * dt * float(np.float32(u))) % L) // (L / 4))
        assert cell_of(st) == expect, k
