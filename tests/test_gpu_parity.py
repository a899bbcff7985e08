"""HIP path vs the FP64 oracle on identical seeded inputs (needs an MI355X).

Bars: contact pair lists bit-exact; per-cell DEM statistics and continuum
state within 1e-5 relative after 1 and 10 steps, measured against at least
1e-3 of the component's rms over cells, a floor raised per component only
where the 32-bit storage of the state alone would use a fifth of that
allowance (metrics.storage_floors, tests/storage.py); the all-pairs and
binned schedules give the same floe state bit for bit.
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import FLOOR, TOL, rel_err, report, storage_floors
from storage import dem_cells_stored, run_plain_stored
from workloads import dense_workload, ragged_workload

pytestmark = pytest.mark.gpu

sp = pytest.importorskip("paper_2303_07819_amd")


def _sim(w, schedule=sp.SCHED_AUTO, flags=0):
    return sp.Sim.from_workload(w, flags=flags, schedule=schedule)


def _say(*a):
    print(*a, flush=True)


def compare(w, nsteps, schedule=sp.SCHED_AUTO, flags=0, oflags=0, tol=TOL):
    _say(f"compare {w.name} ncells={w.ncells} n={w.nfloes} steps={nsteps} sched={schedule}")
    st, Q, mom, _ = oracle.run_plain(w, nsteps, flags=oflags)
    Qs, moms = run_plain_stored(w, nsteps, flags=oflags)
    fm, fq = storage_floors(mom, moms), storage_floors(Q, Qs)
    with _sim(w, schedule, flags) as s:
        s.step(w.dt, nsteps)
        gm = s.read_moments(sp.MOMENTS_DEM)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
        stats = s.stats()
    e_m = rel_err(gm, mom, fm)
    e_q = rel_err(gq, Q, fq)
    _say(f"  max rel err moments {e_m.max():.2e} continuum {e_q.max():.2e} contacts {stats['contacts']}; "
         f"floors moments {fm.max():.1e} continuum {fq.max():.1e}")
    _say("  moments   " + report(gm, mom, fm, oracle.MOMENT_NAMES))
    _say("  continuum " + report(gq, Q, fq, oracle.Q_NAMES))
    assert np.array_equal(gm[:, 0], mom[:, 0])
    assert e_m.max() <= tol, np.unravel_index(e_m.argmax(), e_m.shape)
    assert e_q.max() <= tol, np.unravel_index(e_q.argmax(), e_q.shape)
    return stats


@pytest.mark.parametrize("nsteps", [1, 10])
@pytest.mark.parametrize("schedule", [sp.SCHED_ALLPAIRS, sp.SCHED_BINNED])
def test_small_config_parity(nsteps, schedule):
    compare(fixtures.make_config(0), nsteps, schedule)


@pytest.mark.parametrize("nsteps", [1, 10])
@pytest.mark.parametrize("schedule", [sp.SCHED_ALLPAIRS, sp.SCHED_BINNED])
def test_dense_contacts_parity(nsteps, schedule):
    stats = compare(dense_workload(), nsteps, schedule)
    if nsteps > 1:
        assert stats["contacts"] > 100


@pytest.mark.parametrize("schedule", [sp.SCHED_ALLPAIRS, sp.SCHED_BINNED])
def test_ragged_and_empty_cells_parity(schedule):
    compare(ragged_workload(), 1, schedule)
    compare(ragged_workload(), 10, schedule)


def test_ocean_off_and_forward_euler_flags():
    w = dense_workload(seed=3, nx=2, ny=1)
    compare(w, 10, sp.SCHED_BINNED, flags=sp.SP_OCEAN_OFF, oflags=oracle.OCEAN_OFF)
    compare(w, 3, sp.SCHED_BINNED, flags=sp.SP_FORWARD_EULER, oflags=oracle.FORWARD_EULER)


def test_schedules_bitwise_identical():
    w = dense_workload(seed=7)
    out = []
    for sched in (sp.SCHED_ALLPAIRS, sp.SCHED_BINNED):
        with _sim(w, sched) as s:
            s.step(w.dt, 10)
            out.append((s.read_floes(), s.read_moments(sp.MOMENTS_DEM), s.read_moments(sp.MOMENTS_CONTINUUM)))
    for k in out[0][0]:
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])


def _oracle_pairs_global(w, state):
    m = oracle.Model(w)
    st = w.start
    res = []
    for c in range(w.ncells):
        p = oracle.pairs_cell(m, state, c)
        if p.size:
            res.append(p + st[c])
    return np.concatenate(res) if res else np.zeros((0, 2), np.int64)


def test_pairs_bit_exact_random_overlapping_cells():
    from helpers import random_cell
    rng = np.random.default_rng(0)
    w = random_cell(rng, 300, 25e3, 300.0, 2500.0, nx=3, ny=2)
    w.counts[:] = [300, 0, 1, 300, 299, 0]
    w.counts[-1] = w.nfloes - w.counts[:-1].sum()
    with _sim(w) as s:
        got = s.read_pairs()
    ref = _oracle_pairs_global(w, oracle.State.from_workload(w))
    _say(f"pairs: {len(ref)}")
    assert len(ref) > 1000
    np.testing.assert_array_equal(got, ref)


def test_pairs_bit_exact_after_steps():
    w = dense_workload(seed=19)
    with _sim(w, sp.SCHED_BINNED) as s:
        s.step(w.dt, 10)
        f = s.read_floes()
        got = s.read_pairs()
    state = oracle.State.from_fixed(f["xi"], f["yi"], f["u"], f["v"], f["omega"], f["theta"], w.r, w.h)
    ref = _oracle_pairs_global(w, state)
    assert len(ref) > 50
    np.testing.assert_array_equal(got, ref)


def test_exact_touch_pairs():
    """d = r_l + r_j exactly is not a contact; one 2^-32 step closer is."""
    L = 32768.0
    d_units = int(3000.0 / (L / 2 ** 32))
    xi = np.array([0, d_units, 2 ** 31, 2 ** 31 + d_units - 1], np.uint32)
    w = fixtures.from_arrays(2, 1, L, [2, 2], xi, [5, 5, 9, 9], [1500.0] * 4, [1.0] * 4)
    with _sim(w) as s:
        got = s.read_pairs()
    np.testing.assert_array_equal(got, np.array([[2, 3]]))


def test_full_size_plain64_sampled_cells():
    """The benchmark workload (64x64 cells, 1,048,576 floes) in the benchmark's
    launch configuration: sampled cells' DEM statistics against the oracle run
    on those cells only (cells are independent DEMs), and the continuum of a
    few cells against the oracle's LF on their domain of dependence."""
    w = fixtures.make_config(1)
    nsteps = 10
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(w.ncells, 8, replace=False))
    _say(f"full-size plain64, sample {sample.tolist()}")
    with _sim(w) as s:
        s.step(w.dt, nsteps)
        gm = s.read_moments(sp.MOMENTS_DEM)
        sched = s.schedule()
    assert sched[0] == sp.SCHED_BINNED
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    oracle.dem_steps(m, st, w.dt, nsteps, cells=sample)
    ref = oracle.moments(m, st)[sample]
    e = rel_err(gm[sample], ref, storage_floors(ref, dem_cells_stored(w, nsteps, sample)[sample]))
    _say(f"  max rel err {e.max():.2e}")
    assert e.max() <= TOL


def test_full_size_plain64_continuum_window():
    w = fixtures.make_config(1)
    k = 2
    with _sim(w) as s:
        s.step(w.dt, k)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
    m = oracle.Model(w)
    for (cx, cy) in ((0, 0), (37, 21), (63, 63)):
        ix = (cx + np.arange(-k - 1, k + 2)) % w.nx
        iy = (cy + np.arange(-k - 1, k + 2)) % w.ny
        cells = (iy[:, None] * w.nx + ix[None, :]).reshape(-1)
        st = oracle.State.from_workload(w)
        mom0 = oracle.moments(m, st)[cells]
        mom, _ = oracle.dem_steps(m, st, w.dt, k, cells=cells, record=True)
        win = fixtures.from_arrays(ix.size, iy.size, w.Lx, np.zeros(cells.size, np.int32), [], [], [], [])
        wm = oracle.Model(win)
        Q = oracle.q_from_moments(wm, mom0)
        for j in range(k):
            Q, _ = oracle.lf_step(wm, Q, mom[j], w.dt)
        centre = (k + 1) * ix.size + (k + 1)
        ref = Q[centre]
        got = gq[cy * w.nx + cx]
        e = np.abs(got - ref) / np.maximum(np.abs(ref), FLOOR * np.sqrt(np.mean(gq ** 2, axis=0)))
        _say(f"  cell ({cx},{cy}) continuum rel err {e.max():.2e}")
        assert e.max() <= TOL


def test_error_paths():
    w = dense_workload(seed=2, nx=1, ny=1, n=64)
    s = sp.Sim(w.nx, w.ny, w.Lx, w.Ly, w.rho_ice, w.rho_ocean, w.cd, w.E, w.G, w.mu)
    with pytest.raises(sp.SpdemError) as ei:
        s.step(30.0, 1)
    assert ei.value.status == -7                          # SP_ESTATE
    bad_r = w.r.copy()
    bad_r[3] = 0.26 * w.Lx
    with pytest.raises(sp.SpdemError) as ei:
        s.set_floes(w.counts, w.xi, w.yi, w.u, w.v, w.omega, w.theta, bad_r, w.h)
    assert ei.value.status == -1                          # SP_EINVAL
    with pytest.raises(sp.SpdemError) as ei:
        s.set_floes([w.nfloes + 1], w.xi, w.yi, w.u, w.v, w.omega, w.theta, w.r, w.h)
    assert ei.value.status == -1
    u = w.u.copy()
    u[5] = np.nan
    s.set_floes(w.counts, w.xi, w.yi, u, w.v, w.omega, w.theta, w.r, w.h)
    s.step(30.0, 1)
    with pytest.raises(sp.SpdemError) as ei:
        s.synchronize()
    assert ei.value.status == -6                          # SP_ENAN
    s.close()
    big = fixtures.from_arrays(1, 1, 25e3, [1025], np.arange(1025, dtype=np.uint32) * 4000000,
                               np.zeros(1025, np.uint32), np.full(1025, 1.0), np.ones(1025))
    with pytest.raises(sp.SpdemError) as ei:
        _sim(big)
    assert ei.value.status == -8                          # SP_ECAPACITY


def test_max_cell_capacity():
    """1024 floes in one cell (the per-cell maximum) next to an empty cell."""
    w = fixtures.custom(2, 1, 25e3, [1024, 0], seed=9, r_scale=fixtures.radius_scale(1024, 25e3 ** 2, phi=0.3))
    rng = np.random.default_rng(9)
    w.u[:] = rng.normal(0, 0.2, w.nfloes)
    w.v[:] = rng.normal(0, 0.2, w.nfloes)
    compare(w, 5, sp.SCHED_BINNED)
    compare(w, 2, sp.SCHED_ALLPAIRS)
