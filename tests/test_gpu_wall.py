"""Floes driven into a wall (Sec. 4.4) on the HIP path against the oracle
(needs an MI355X): the global DEM with floe-wall contact (SP_WALL_X against
the oracle's WALLS_X), and the superparameterised model's continuum with the
zero Dirichlet boundary in x (SP_WALL_X against DIRICHLET_X) on the plain,
blocked and coupled paths.

Bars: those of test_gpu_global for the global DEM (contact counts equal,
positions within 1e-4 of the smallest radius, velocities and coarse
statistics within 1e-5 or five times their storage floor); those of
test_gpu_parity and test_gpu_coupling for the continuum paths.
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import TOL, rel_err, storage_floors
from storage import round_state, run_coupled_stored, run_plain_stored
from workloads import dense_workload

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2303_07819_amd")

TWO32 = 2.0 ** 32


def _say(*a):
    print(*a, flush=True)


def _vel(st):
    return np.stack([st.u, st.v, st.w], 1)


def wall_domain(seed=31, L=60e3, n=500, push=0.25):
    """A 60 km domain of 500 floes driven towards both walls (x velocity
    +push right of the middle, -push left of it, plus noise)."""
    w = fixtures.custom(1, 1, L, n, seed=seed, r_scale=fixtures.radius_scale(n, L * L, phi=0.45))
    rng = np.random.default_rng(seed)
    x = w.xi / TWO32
    w.u[:] = np.where(x > 0.5, push, -push) + rng.normal(0, 0.05, n)
    w.v[:] = rng.normal(0, 0.1, n)
    w.omega[:] = rng.normal(0, 1e-4, n)
    w.dt = 30.0
    return w


def compare_global(w, nsteps, nxc, nyc, oflags=oracle.WALLS_X, flags=sp.SP_WALL_X):
    _say(f"global with walls {w.name} n={w.nfloes} steps={nsteps} coarse {nxc}x{nyc}")
    m = oracle.Model(w, oflags | oracle.BINNED)
    st = oracle.State.from_workload(w)
    _, stats = oracle.dem_steps(m, st, w.dt, nsteps)
    ref = oracle.coarse_moments(w, st, nxc, nyc, oflags)
    a, b = oracle.State.from_workload(w), oracle.State.from_workload(w)
    for _ in range(nsteps):
        oracle.dem_steps(m, a, w.dt, 1)
        oracle.dem_steps(m, b, w.dt, 1)
        round_state(b)
    tol = max(TOL, 5.0 * rel_err(oracle.coarse_moments(w, b, nxc, nyc, oflags),
                                 oracle.coarse_moments(w, a, nxc, nyc, oflags)).max())
    tol_vel = max(TOL, 5.0 * rel_err(_vel(b), _vel(a)).max())
    with sp.GlobalDEM.from_workload(w, flags=flags) as g:
        g.step(w.dt, nsteps)
        f = g.read_floes()
        got = g.coarse_moments(nxc, nyc)
        gs = g.stats()
    dx = f["xi"] / TWO32 - st.xs                        # no periodic image in x
    dy = (f["yi"] / TWO32 - st.ys + 0.5) % 1.0 - 0.5
    e_pos = max(np.abs(dx).max() * w.Lx, np.abs(dy).max() * w.Ly) / w.r.min()
    e_vel = rel_err(np.stack([f["u"], f["v"], f["omega"]], 1), _vel(st)).max()
    e_mom = rel_err(got, ref).max()
    _say(f"  contacts {gs['contacts']} (oracle {stats[0]}), bins {gs['bins']}, position {e_pos:.2e} r_min, "
         f"velocity {e_vel:.2e} (bar {tol_vel:.1e}), coarse statistics {e_mom:.2e} (bar {tol:.1e})")
    assert gs["contacts"] == stats[0]
    assert np.array_equal(got[:, 0], ref[:, 0])
    assert e_pos <= 1e-4
    assert e_vel <= tol_vel
    assert e_mom <= tol
    return st, gs


@pytest.mark.parametrize("nsteps", [1, 10, 40])
def test_wall_domain_parity(nsteps):
    w = wall_domain()
    st, gs = compare_global(w, nsteps, 6, 3)
    if nsteps >= 10:
        # the walls were hit: the periodic run of the same floes differs
        m = oracle.Model(w, oracle.BINNED)
        sp_ = oracle.State.from_workload(w)
        oracle.dem_steps(m, sp_, w.dt, nsteps)
        assert not np.array_equal(sp_.u, st.u)
        assert np.all((st.xs >= 0.0) & (st.xs < 1.0))


def test_scenario_4_4_reduced_grid_parity():
    """Scenario 4.4 on a 96 x 48 fine grid (4608 floes, the paper's domain,
    radii, current and dt): 650 steps, in which the rightmost column reaches
    the wall, bounces and meets the next."""
    w = fixtures.scenario_global(4, nfx=96, nfy=48)
    st, gs = compare_global(w, 650, 12, 6)
    assert gs["contacts"] > 0


def _plain_compare(w, nsteps, k):
    st, Q, mom, _ = oracle.run_plain(w, nsteps, flags=oracle.DIRICHLET_X)
    Qs, moms = run_plain_stored(w, nsteps, flags=oracle.DIRICHLET_X)
    _, Qp, _, _ = oracle.run_plain(w, nsteps)
    with sp.Sim.from_workload(w, flags=sp.SP_WALL_X) as s:
        s.set_step_block(k)
        s.step(w.dt, nsteps)
        gm = s.read_moments(sp.MOMENTS_DEM)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
    e_m = rel_err(gm, mom, storage_floors(mom, moms)).max()
    e_q = rel_err(gq, Q, storage_floors(Q, Qs)).max()
    d_p = rel_err(Qp, Q).max()
    _say(f"dirichlet {w.name} k={k} steps={nsteps}: moments {e_m:.2e} continuum {e_q:.2e} "
         f"(periodic differs by {d_p:.1e})")
    assert d_p > 1e-3                  # the boundary matters
    assert e_m <= TOL and e_q <= TOL


@pytest.mark.parametrize("k", [1, 4, 32])
def test_plain_and_blocked_dirichlet_parity(k):
    _plain_compare(fixtures.make_config(0), 10, k)
    _plain_compare(dense_workload(seed=9, nx=4, ny=2), 10, k)


@pytest.mark.parametrize("nsteps,N0,N1,n_t", [(13, 4, 2, 2), (9, 3, 3, 1)])
def test_coupled_dirichlet_parity(nsteps, N0, N1, n_t):
    w = fixtures.make_config(0)
    st, Q, mom, cfl = oracle.run_coupled(w, nsteps, N0, N1, n_t, flags=oracle.DIRICHLET_X)
    Qs, moms = run_coupled_stored(w, nsteps, N0, N1, n_t, flags=oracle.DIRICHLET_X)
    with sp.Sim.from_workload(w, flags=sp.SP_WALL_X) as s:
        s.set_coupling(N0, N1, n_t)
        s.step(w.dt, nsteps)
        gm = s.read_moments(sp.MOMENTS_DEM)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
    e_m = rel_err(gm, mom, storage_floors(mom, moms)).max()
    e_q = rel_err(gq, Q, storage_floors(Q, Qs)).max()
    _say(f"coupled dirichlet steps={nsteps} N0={N0} N1={N1} n_t={n_t}: moments {e_m:.2e} continuum {e_q:.2e}")
    assert e_m <= TOL and e_q <= TOL


def test_wall_flag_limits_and_crossing():
    w = fixtures.make_config(0)
    with sp.Sim.from_workload(w, flags=sp.SP_WALL_X) as s:
        net = sp.MLP()
        with pytest.raises(sp.SpdemError) as ei:
            s.hybrid_set(net, np.ones(w.ncells, bool))
        assert ei.value.status == -7
        net.close()
        s.step(w.dt, 2)
    # a small fast floe jumps through the far wall in one step: SP_EWALL
    L = 25e3
    x = np.array([L - 10.0, 0.5 * L]) / L * TWO32
    wf = fixtures.from_arrays(1, 1, L, [2], x, [0.5 * TWO32, 0.25 * TWO32], [5.0, 50.0], [1.0, 1.0], u=[1.0, 0.0])
    with sp.GlobalDEM.from_workload(wf, flags=sp.SP_WALL_X | sp.SP_OCEAN_OFF) as g:
        g.step(30.0, 1)
        with pytest.raises(sp.SpdemError) as ei:
            g.read_floes()
        assert ei.value.status == -9
