"""The tangential spring (SP_TANGENTIAL_SPRING: the incremental Cundall-Strack
reading of the tangential contact force with per-contact history) on the GPU
against the oracle's spring (needs an MI355X).

Bars: those of test_gpu_parity (1e-5 after 1 and 10 steps, with the storage
floors of metrics.storage_floors); per-floe velocities of a two-floe contact
within 5e-5 of the oracle over a whole 60-step encounter (no slip, then slip:
the FP32 storage of the state, rounded every step, accumulates over it).  G is read as
the shear modulus: 80 N/m^2 against E = 200 (E / (2 (1 + 0.25))).
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import TOL, rel_err, storage_floors
from storage import run_plain_stored
from workloads import dense_workload

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2303_07819_amd")

TOL_ENCOUNTER = 5e-5    # per-floe state over a 60-step encounter
G_SHEAR = 80.0


def _say(*a):
    print(*a, flush=True)


def _compare(w, nsteps, schedule, tol):
    st, Q, mom, _ = oracle.run_plain(w, nsteps, flags=oracle.SPRING)
    Qs, moms = run_plain_stored(w, nsteps, flags=oracle.SPRING)
    with sp.Sim.from_workload(w, flags=sp.SP_TANGENTIAL_SPRING, schedule=schedule) as s:
        assert not s.step_block()[1]
        s.step(w.dt, nsteps)
        gm = s.read_moments(sp.MOMENTS_DEM)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
        f = s.read_floes()
        stats = s.stats()
    e_m, e_q = rel_err(gm, mom, storage_floors(mom, moms)), rel_err(gq, Q, storage_floors(Q, Qs))
    _say(f"spring {w.name} steps={nsteps} sched={schedule}: moments {e_m.max():.2e} continuum {e_q.max():.2e} "
         f"contacts {stats['contacts']}")
    assert e_m.max() <= tol, np.unravel_index(e_m.argmax(), e_m.shape)
    assert e_q.max() <= tol, np.unravel_index(e_q.argmax(), e_q.shape)
    return st, f, stats


@pytest.mark.parametrize("nsteps", [1, 10])
@pytest.mark.parametrize("schedule", [sp.SCHED_ALLPAIRS, sp.SCHED_BINNED])
def test_dense_contacts_spring_parity(nsteps, schedule):
    w = dense_workload(seed=21)
    w.G = G_SHEAR
    _, _, stats = _compare(w, nsteps, schedule, TOL)
    assert nsteps == 1 or stats["contacts"] > 0   # floes are placed apart


def test_spring_differs_from_the_viscous_law():
    w = dense_workload(seed=22)
    w.G = G_SHEAR
    with sp.Sim.from_workload(w) as a, sp.Sim.from_workload(w, flags=sp.SP_TANGENTIAL_SPRING) as b:
        a.step(w.dt, 10)
        b.step(w.dt, 10)
        fa, fb = a.read_floes(), b.read_floes()
    assert not np.array_equal(fa["u"], fb["u"])


@pytest.mark.parametrize("mu", [1e6, 0.05])
def test_two_floe_encounter_per_floe(mu):
    """Two floes sliding past each other through a whole contact (history
    built, then forgotten when they part): per-floe state against the oracle.
    mu = 1e6 never slips, mu = 0.05 slips."""
    L = 25e3
    r = np.array([500.0, 400.0])
    x0, dy = 0.4 * L, 300.0
    xi = np.array([x0 / L, (x0 + 880.0) / L]) * 2.0 ** 32
    yi = np.array([0.5, 0.5 + dy / L]) * 2.0 ** 32
    w = fixtures.from_arrays(1, 1, L, [2], xi, yi, r, [1.0, 1.0], u=[0.02, -0.02], v=[0.1, -0.1], G=G_SHEAR)
    w.mu = mu
    m = oracle.Model(w, oracle.SPRING | oracle.OCEAN_OFF)
    st = oracle.State.from_workload(w)
    with sp.Sim.from_workload(w, flags=sp.SP_TANGENTIAL_SPRING | sp.SP_OCEAN_OFF) as s:
        touched = False
        for k in range(60):
            oracle.dem_steps(m, st, w.dt, 1)
            s.step(w.dt, 1)
            f = s.read_floes()
            touched = touched or bool(np.any(st.hj >= 0))
            for q, o in (("u", st.u), ("v", st.v), ("omega", st.w)):
                scale = np.max(np.abs(o)) + 1e-30
                e = np.max(np.abs(f[q].astype(np.float64) - o)) / scale
                assert e <= TOL_ENCOUNTER, (k, q, e)
        assert touched and np.all(st.hj == -1)     # they met and parted
        assert s.stats()["contacts"] > 0


def test_spring_entry_point_limits():
    w = fixtures.make_config(0)
    with sp.Sim.from_workload(w, flags=sp.SP_TANGENTIAL_SPRING) as s:
        assert not s.step_block()[1]
        with pytest.raises(sp.SpdemError):
            s.set_coupling(100, 1, 10)
        with pytest.raises(sp.SpdemError):
            s.autotune(w.dt)
        s.step(w.dt, 3)
