"""Global DEM of the error study (Sec. 4) on the HIP path against the oracle's
run_global and coarse_moments on identical seeded inputs (needs an MI355X).

Bars: contact counts equal; floe velocities and spins, and coarse statistics,
each within 1e-5 relative (field-rms floor) or five times its storage floor
(the oracle rerun with its state rounded to the stored formats) where contacts
make that larger; positions within 1e-4 of the smallest radius; the paper's
drift scenario exact at full size.
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import rel_err
from storage import round_state

pytestmark = pytest.mark.gpu

TOL = 1e-5
TWO32 = 2.0 ** 32

sp = pytest.importorskip("paper_2303_07819_amd")


def _say(*a):
    print(*a, flush=True)


def dense_global(seed=21, L=120e3, n=1500, vel=0.3):
    """A 120 km periodic domain of 1500 floes moving at random: many contacts,
    floes crossing every coarse cell edge."""
    w = fixtures.custom(1, 1, L, n, seed=seed, r_scale=fixtures.radius_scale(n, L * L, phi=0.45))
    rng = np.random.default_rng(seed)
    w.u[:] = rng.normal(0, vel, n)
    w.v[:] = rng.normal(0, vel, n)
    w.omega[:] = rng.normal(0, 1e-4, n)
    w.dt = 30.0
    return w


def _vel(st):
    return np.stack([st.u, st.v, st.w], 1)


def _storage_floor(w, nsteps, nxc, nyc, flags=0):
    """Deviation of the oracle with its state rounded to the stored formats
    after every step: (coarse statistics, floe velocities and spins)."""
    m = oracle.Model(w, flags)
    a, b = oracle.State.from_workload(w), oracle.State.from_workload(w)
    for _ in range(nsteps):
        oracle.dem_steps(m, a, w.dt, 1)
        oracle.dem_steps(m, b, w.dt, 1)
        round_state(b)
    return (rel_err(oracle.coarse_moments(w, b, nxc, nyc, flags), oracle.coarse_moments(w, a, nxc, nyc, flags)).max(),
            rel_err(_vel(b), _vel(a)).max())


def compare(w, nsteps, nxc, nyc, flags=0, oflags=0):
    _say(f"global {w.name} n={w.nfloes} steps={nsteps} coarse {nxc}x{nyc}")
    st, stats = oracle.run_global(w, nsteps, flags=oflags)
    ref = oracle.coarse_moments(w, st, nxc, nyc, oflags)
    floor_mom, floor_vel = _storage_floor(w, nsteps, nxc, nyc, oflags)
    tol, tol_vel = max(TOL, 5.0 * floor_mom), max(TOL, 5.0 * floor_vel)
    with sp.GlobalDEM.from_workload(w, flags=flags) as g:
        g.step(w.dt, nsteps)
        f = g.read_floes()
        got = g.coarse_moments(nxc, nyc)
        gs = g.stats()
    gx = f["xi"] / TWO32
    dx = (gx - st.xs + 0.5) % 1.0 - 0.5
    dy = (f["yi"] / TWO32 - st.ys + 0.5) % 1.0 - 0.5
    e_pos = max(np.abs(dx).max() * w.Lx, np.abs(dy).max() * w.Ly) / w.r.min()
    e_vel = rel_err(np.stack([f["u"], f["v"], f["omega"]], 1), _vel(st)).max()
    e_mom = rel_err(got, ref).max()
    _say(f"  contacts {gs['contacts']} (oracle {stats[0]}), bins {gs['bins']}, position err {e_pos:.2e} r_min, "
         f"velocity {e_vel:.2e} (bar {tol_vel:.1e}), coarse statistics {e_mom:.2e} (bar {tol:.1e})")
    assert gs["contacts"] == stats[0]
    assert np.array_equal(got[:, 0], ref[:, 0])
    assert e_pos <= 1e-4
    assert e_vel <= tol_vel
    assert e_mom <= tol
    return gs


@pytest.mark.parametrize("nsteps", [1, 10])
def test_dense_domain_parity(nsteps):
    gs = compare(dense_global(), nsteps, 6, 6)
    assert gs["bins"][0] >= 3
    assert gs["contacts"] > 0 or nsteps == 1     # the floes are placed apart


def test_dense_domain_forward_euler_and_no_ocean():
    compare(dense_global(seed=5, n=800), 10, 4, 3, flags=sp.SP_OCEAN_OFF | sp.SP_FORWARD_EULER,
            oflags=oracle.OCEAN_OFF | oracle.FORWARD_EULER)


@pytest.mark.parametrize("k", [2, 3])
def test_scenarios_reduced_grid_parity(k):
    """Scenarios 4.2 and 4.3 on a 96 x 48 fine grid (4608 floes, same domain,
    radii and currents), 40 steps of the paper's dt = 1e-4."""
    w = fixtures.scenario_global(k, nfx=96, nfy=48)
    compare(w, 40, 12, 6)


def test_small_domain_single_bin():
    """Fewer than three sub-bins per side (r_max > L / 6): one sub-bin spans the
    domain.  Two of the four 3.5 km floes of a 20 km domain close a 3 km gap
    head-on (no ocean) and collide across the periodic seam."""
    L = 20e3
    fx = np.array([0.25, 0.75, 0.25, 0.75])
    fy = np.array([0.25, 0.25, 0.75, 0.75])
    xi = (np.round(fx * TWO32) % TWO32).astype(np.uint64).astype(np.uint32)
    yi = (np.round(fy * TWO32) % TWO32).astype(np.uint64).astype(np.uint32)
    w = fixtures.from_arrays(1, 1, L, [4], xi, yi, [3500.0] * 4, [1.0, 1.5, 0.8, 1.2], u=[-4.9, 4.9, 0.3, 0.0],
                             v=[0.0, 0.0, 0.0, -0.2], dt=60.0)
    gs = compare(w, 12, 2, 2, flags=sp.SP_OCEAN_OFF, oflags=oracle.OCEAN_OFF)
    assert gs["bins"] == (1, 1) and gs["contacts"] > 0


def test_scenario_4_1_full_size_exact_drift():
    """Sec. 4.1 at full size (480 x 240 floes): every floe drifts with the
    current, no contact ever forms, every displacement is the same whole
    number of position units per step and the concentration of every coarse
    cell of the 48 x 24 grid keeps its initial value."""
    w = fixtures.scenario_global(1)
    nsteps = 100
    with sp.GlobalDEM.from_workload(w) as g:
        c0 = g.coarse_moments(48, 24)
        g.step(w.dt, nsteps)
        f = g.read_floes()
        gs = g.stats()
        c1 = g.coarse_moments(48, 24)
    step = int(round(w.dt * float(np.float32(0.3)) / (w.Lx / TWO32)))
    shift = (f["xi"].astype(np.int64) - w.xi.astype(np.int64)) % (1 << 32)
    _say(f"  contacts {gs['contacts']}, bins {gs['bins']}, shift {np.unique(shift)} vs {nsteps} x {step}")
    assert gs["contacts"] == 0
    assert np.all(shift == nsteps * step)
    assert np.array_equal(f["yi"], w.yi)
    assert np.all(f["u"] == np.float32(0.3)) and np.all(f["v"] == 0.0) and np.all(f["omega"] == 0.0)
    # 100 steps move every floe by 0.003 < half a fine cell: no floe changes coarse cell
    np.testing.assert_array_equal(c1[:, 0], c0[:, 0])
    np.testing.assert_allclose(c1[:, 10], c0[:, 10], rtol=1e-15)


def test_error_paths():
    w = dense_global(n=50)
    with sp.GlobalDEM.from_workload(w) as g:
        with pytest.raises(sp.SpdemError):
            g.step(-1.0, 1)
        with pytest.raises(sp.SpdemError):
            g.coarse_moments(0, 3)
    big = fixtures.from_arrays(1, 1, 10e3, [1], [0], [0], [3000.0], [1.0])
    with pytest.raises(sp.SpdemError):
        sp.GlobalDEM.from_workload(big)


def _stable_order(prev, xi, yi, bins):
    """The previous order stably sorted by the sub-bin of every floe's
    position (xi, yi indexed by floe), and the sub-bin starts."""
    bx, by = bins
    kx = (xi.astype(np.uint64) * np.uint64(bx)) >> np.uint64(32)
    ky = (yi.astype(np.uint64) * np.uint64(by)) >> np.uint64(32)
    key = (ky * np.uint64(bx) + kx).astype(np.int64)
    order = prev[np.argsort(key[prev], kind="stable")]
    starts = np.concatenate([[0], np.cumsum(np.bincount(key, minlength=bx * by))]).astype(np.int32)
    return order, starts


def test_rebinning_is_a_stable_sort_by_sub_bin():
    """The first grouping (input order sorted by sub-bin) and every re-binning
    over 25 steps of the dense domain: the order a stable sort of the previous
    order by the sub-bins of the positions before the step gives, and its
    sub-bin starts; no floe moves more than one sub-bin per step, so no
    sub-bin falls back to a full scan."""
    w = dense_global(seed=25)
    with sp.GlobalDEM.from_workload(w) as g:
        bins = g.stats()["bins"]
        ids, starts, fb = g.read_order()
        exp, est = _stable_order(np.arange(w.nfloes), w.xi, w.yi, bins)
        assert np.array_equal(ids, exp) and np.array_equal(starts, est)
        for _ in range(25):
            f = g.read_floes()
            exp, est = _stable_order(ids, f["xi"], f["yi"], bins)
            g.step(w.dt, 1)
            ids, starts, fb = g.read_order()
            assert np.array_equal(ids, exp)
            assert np.array_equal(starts, est)
        moved = np.any(ids != np.arange(w.nfloes))
        _say(f"  bins {bins}, 25 re-binnings equal to the stable sort, full scans {fb}")
        assert fb == 0 and moved


def test_rebinning_of_a_floe_that_jumps_sub_bins():
    """One floe of a sparse domain crosses 3.5 sub-bins per step (no ocean):
    the re-binning after each of its steps finds it outside the 3 x 3 sub-bins
    of its target, gathers that sub-bin by a full scan, and still gives the
    stable sort; the coarse read-out falls back the same way; the run matches
    the oracle."""
    L, n = 100e3, 400
    w = fixtures.custom(1, 1, L, n, seed=26, r_scale=fixtures.radius_scale(n, L * L, phi=0.05))
    w.dt = 30.0
    w.u[:] = 0.0
    w.v[:] = 0.0
    with sp.GlobalDEM.from_workload(w) as g:
        bins = g.stats()["bins"]
    side = L / bins[0]
    w.u[0] = np.float32(3.5 * side / w.dt)
    _say(f"  bins {bins}, sub-bin side {side:.0f} m, fast floe {w.u[0]:.1f} m/s")
    with sp.GlobalDEM.from_workload(w, flags=sp.SP_OCEAN_OFF) as g:
        ids = g.read_order()[0]
        for _ in range(3):
            f = g.read_floes()
            exp, est = _stable_order(ids, f["xi"], f["yi"], bins)
            g.step(w.dt, 1)
            ids, starts, fb = g.read_order()
            assert np.array_equal(ids, exp) and np.array_equal(starts, est)
        fb_steps = g.read_order()[2]
        assert fb_steps >= 2                  # two target sub-bins after the first step
        got = g.coarse_moments(10, 10)
        fb_all = g.read_order()[2]
        f = g.read_floes()
    st, stats = oracle.run_global(w, 3, flags=oracle.OCEAN_OFF)
    ref = oracle.coarse_moments(w, st, 10, 10, oracle.OCEAN_OFF)
    dx = (f["xi"] / TWO32 - st.xs + 0.5) % 1.0 - 0.5
    _say(f"  full scans: re-binning {fb_steps}, coarse read-out {fb_all - fb_steps}; "
         f"position err {np.abs(dx).max() * L / w.r.min():.2e} r_min")
    assert fb_all > fb_steps
    assert np.array_equal(got[:, 0], ref[:, 0])
    assert np.abs(dx).max() * L / w.r.min() <= 1e-4
    assert rel_err(got, ref).max() <= TOL
