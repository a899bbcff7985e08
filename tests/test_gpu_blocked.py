"""Blocked plain steps (K steps per DEM launch, cells resident in LDS) against
the per-step kernel and the oracle (needs an MI355X).

Bars: the floe state, contact counts and DEM statistics equal to the per-step
kernel's bit for bit (the same per-floe arithmetic); the continuum within
1e-12 relative of it (statistics summed in another fixed order); against the
oracle the bars of test_gpu_parity.
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import FLOOR, TOL, rel_err, report, storage_floors
from storage import dem_cells_stored, run_plain_stored
from workloads import dense_workload, ragged_workload, uneven_workload

pytestmark = pytest.mark.gpu


sp = pytest.importorskip("paper_2303_07819_amd")


def _say(*a):
    print(*a, flush=True)


def _run(w, k, nsteps, flags=0):
    with sp.Sim.from_workload(w, flags=flags) as s:
        s.set_step_block(k)
        active = s.step_block()[1]
        s.step(w.dt, nsteps)
        return dict(floes=s.read_floes(), mom=s.read_moments(sp.MOMENTS_DEM),
                    q=s.read_moments(sp.MOMENTS_CONTINUUM), stats=s.stats(), work=s.work(), active=active)


# the last two cases end their call in a short block of two steps (a last block
# of 12 or more steps on a small grid splits)
@pytest.mark.parametrize("name,k,nsteps", [("small", 4, 12), ("small", 5, 13), ("dense", 4, 12), ("dense", 8, 16),
                                           ("small", 32, 20), ("dense", 16, 32)])
def test_blocked_equals_per_step(name, k, nsteps):
    w = fixtures.make_config(0) if name == "small" else dense_workload()
    a = _run(w, 1, nsteps)
    b = _run(w, k, nsteps)
    _say(f"{name} k={k} steps={nsteps}: active {b['active']}, contacts {a['stats']['contacts']} / "
         f"{b['stats']['contacts']}, work {b['work']}")
    assert b["active"] and not a["active"]
    for key in a["floes"]:
        assert np.array_equal(a["floes"][key], b["floes"][key]), key
    assert a["stats"]["contacts"] == b["stats"]["contacts"]
    assert np.array_equal(a["mom"], b["mom"])
    e = rel_err(b["q"], a["q"], floor=1e-6)
    assert e.max() <= 1e-12, e.max()
    assert b["work"]["blocked_steps"] == nsteps    # the remainder runs as one shorter block
    assert b["work"]["candidate_tests"] > 0 and a["work"]["candidate_tests"] == 0


@pytest.mark.parametrize("name", ["small", "dense"])
def test_blocked_parity_with_oracle(name):
    w = fixtures.make_config(0) if name == "small" else dense_workload()
    st, Q, mom, _ = oracle.run_plain(w, 10)
    Qs, moms = run_plain_stored(w, 10)
    b = _run(w, 5, 10)
    e_m, e_q = rel_err(b["mom"], mom, storage_floors(mom, moms)).max(), rel_err(b["q"], Q, storage_floors(Q, Qs)).max()
    _say(f"{name}: moments {e_m:.2e} continuum {e_q:.2e}")
    assert b["active"]
    assert e_m <= TOL and e_q <= TOL


@pytest.mark.parametrize("calls", [(5,), (5, 20), (1, 2, 3), (31,), (33, 7)])
def test_runs_shorter_than_a_block_are_blocked(calls):
    """With the default block length (32) every sp_step call, however short,
    runs as blocked launches (a remainder is one launch of its own length):
    the work counter sees every step, and the state equals the per-step
    kernel's bit for bit."""
    w = dense_workload(seed=2)
    n = sum(calls)
    a = _run(w, 1, n)
    with sp.Sim.from_workload(w) as s:
        k, active = s.step_block()
        assert k == 32 and active
        for m in calls:
            s.step(w.dt, m)
        fl, mom, q, wk = s.read_floes(), s.read_moments(sp.MOMENTS_DEM), s.read_moments(sp.MOMENTS_CONTINUUM), s.work()
    _say(f"calls {calls}: blocked steps {wk['blocked_steps']} of {n}")
    assert wk["blocked_steps"] == n
    for key in fl:
        assert np.array_equal(fl[key], a["floes"][key]), key
    assert np.array_equal(mom, a["mom"])
    assert rel_err(q, a["q"], floor=1e-6).max() <= 1e-12


def test_blocked_flags():
    w = dense_workload(seed=4)
    for flags in (sp.SP_OCEAN_OFF, sp.SP_FORWARD_EULER, sp.SP_NO_CONTINUUM):
        a = _run(w, 1, 8, flags)
        b = _run(w, 4, 8, flags)
        for key in a["floes"]:
            assert np.array_equal(a["floes"][key], b["floes"][key]), (flags, key)


def test_large_cells_block_with_sixteen_wavefronts():
    """Cells above 64 W floes (the 1024-floe bucket at W = 8, two floes per
    lane in the per-step kernel) run blocked with 16 wavefronts, one floe per
    lane; the floe state stays that of the per-step path bit for bit."""
    w = ragged_workload()
    a = _run(w, 1, 8)
    b = _run(w, 4, 8)
    assert b["active"]
    for key in a["floes"]:
        assert np.array_equal(a["floes"][key], b["floes"][key]), key
    assert a["stats"]["contacts"] == b["stats"]["contacts"]
    e = rel_err(b["q"], a["q"], floor=1e-6)
    assert e.max() <= 1e-12, e.max()


def test_uneven_workload_blocked_parity():
    w = uneven_workload()
    st, Q, mom, _ = oracle.run_plain(w, 8)
    Qs, moms = run_plain_stored(w, 8)
    b = _run(w, 4, 8)
    e_m, e_q = rel_err(b["mom"], mom, storage_floors(mom, moms)).max(), rel_err(b["q"], Q, storage_floors(Q, Qs)).max()
    _say(f"uneven: active {b['active']} moments {e_m:.2e} continuum {e_q:.2e}")
    _say("  moments   " + report(b["mom"], mom, storage_floors(mom, moms), oracle.MOMENT_NAMES))
    _say("  continuum " + report(b["q"], Q, storage_floors(Q, Qs), oracle.Q_NAMES))
    assert b["active"]
    assert e_m <= TOL and e_q <= TOL


def test_plain64_call_ending_in_a_short_block():
    """The benchmark's call shape (20 steps after 5, blocks of 32, 1,048,576
    floes): the call ends in a short block so that the continuum updates of
    its first steps run beside it; the state equals that of per-step launches
    (floes, contacts and DEM statistics bit for bit, the continuum within
    1e-12)."""
    w = fixtures.make_config(1)
    out = []
    for k in (1, 32):
        with sp.Sim.from_workload(w) as s:
            s.set_step_block(k)
            s.step(w.dt, 5)
            s.step(w.dt, 20)
            out.append(dict(floes=s.read_floes(), mom=s.read_moments(sp.MOMENTS_DEM),
                            q=s.read_moments(sp.MOMENTS_CONTINUUM), stats=s.stats(), work=s.work()))
    a, b = out
    for key in a["floes"]:
        assert np.array_equal(a["floes"][key], b["floes"][key]), key
    assert a["stats"]["contacts"] == b["stats"]["contacts"]
    assert np.array_equal(a["mom"], b["mom"])
    e = rel_err(b["q"], a["q"], floor=1e-6)
    _say(f"plain64 5 + 20 steps, blocked against per-step: continuum max rel err {e.max():.2e}")
    assert e.max() <= 1e-12, e.max()
    assert b["work"]["blocked_steps"] == 25


def test_full_size_plain64_blocks():
    """The benchmark workload in its default configuration (blocks of 32):
    sampled cells' statistics after 64 steps against the oracle on those cells
    (cells are independent DEMs), and after one block of 4 the continuum of a
    few cells against the oracle's LF on their domain of dependence."""
    w = fixtures.make_config(1)
    rng = np.random.default_rng(2)
    sample = np.sort(rng.choice(w.ncells, 6, replace=False))
    with sp.Sim.from_workload(w) as s:
        assert s.step_block() == (32, True)
        s.step(w.dt, 64)
        gm = s.read_moments(sp.MOMENTS_DEM)
        work = s.work()
    assert work["blocked_steps"] == 64
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    oracle.dem_steps(m, st, w.dt, 64, cells=sample)
    ref = oracle.moments(m, st)[sample]
    e = rel_err(gm[sample], ref, storage_floors(ref, dem_cells_stored(w, 64, sample)[sample]))
    _say(f"  sampled cells after 64 blocked steps: max rel err {e.max():.2e}")
    assert e.max() <= TOL
    k = 4
    with sp.Sim.from_workload(w) as s:
        s.set_step_block(k)
        s.step(w.dt, k)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
    for (cx, cy) in ((0, 0), (29, 50), (63, 63)):
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
        ref = Q[(k + 1) * ix.size + (k + 1)]
        got = gq[cy * w.nx + cx]
        e = np.abs(got - ref) / np.maximum(np.abs(ref), FLOOR * np.sqrt(np.mean(gq ** 2, axis=0)))
        _say(f"  cell ({cx},{cy}) continuum after one block of {k}: {e.max():.2e}")
        assert e.max() <= TOL


def test_step_block_errors():
    w = fixtures.make_config(0)
    with sp.Sim.from_workload(w) as s:
        for bad in (0, -3, sp.SP_MAX_STEP_BLOCK + 1):
            with pytest.raises(sp.SpdemError):
                s.set_step_block(bad)
        assert s.step_block()[0] == 32
