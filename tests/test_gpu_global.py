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
