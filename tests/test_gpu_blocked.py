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
from metrics import FLOOR, rel_err
from workloads import dense_workload, ragged_workload, uneven_workload

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOL_CONTACT = 5e-5

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


@pytest.mark.parametrize("name,k,nsteps", [("small", 4, 12), ("small", 5, 13), ("dense", 4, 12), ("dense", 8, 16)])
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
    assert b["work"]["blocked_steps"] == (nsteps // k) * k
    assert b["work"]["candidate_tests"] > 0 and a["work"]["candidate_tests"] == 0


@pytest.mark.parametrize("name", ["small", "dense"])
def test_blocked_parity_with_oracle(name):
    w = fixtures.make_config(0) if name == "small" else dense_workload()
    tol = TOL if name == "small" else TOL_CONTACT
    st, Q, mom, _ = oracle.run_plain(w, 10)
    b = _run(w, 5, 10)
    e_m, e_q = rel_err(b["mom"], mom).max(), rel_err(b["q"], Q).max()
    _say(f"{name}: moments {e_m:.2e} continuum {e_q:.2e}")
    assert b["active"]
    assert e_m <= tol and e_q <= tol


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
    b = _run(w, 4, 8)
    e_m, e_q = rel_err(b["mom"], mom).max(), rel_err(b["q"], Q).max()
    _say(f"uneven: active {b['active']} moments {e_m:.2e} continuum {e_q:.2e}")
    assert b["active"]
    assert e_m <= TOL_CONTACT and e_q <= TOL_CONTACT


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
    e = rel_err(gm[sample], oracle.moments(m, st)[sample])
    _say(f"  sampled cells after 64 blocked steps: max rel err {e.max():.2e}")
    assert e.max() <= TOL_CONTACT
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
