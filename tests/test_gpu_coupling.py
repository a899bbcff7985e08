"""Coupled cadence (Algorithm 1 with N0 > 1) of the HIP path against the
oracle's run_coupled on identical seeded inputs (needs an MI355X).

Bars as in test_gpu_parity: per-cell DEM statistics and continuum state
within 1e-5 relative, against floors of 1e-3 of each component's rms raised
only where the storage of the state in the GPU's formats alone (the oracle's
schedule rerun with its state rounded after every step and update,
tests/storage.py) would use a fifth of the allowance: coarse-to-fine updates
set a cell's momentum to a target close to its current value, so the FP32
rounding of the shifted velocities is amplified in the next window; radii after
re-synchronisation within FP32 rounding of the oracle's; no clamped or
invalid cell updates where the oracle has none (it never clamps; the HIP
path clamps only radii past a quarter of the cell).
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import FLOOR, TOL, rel_err, storage_floors
from storage import fp32_storage_bound, run_coupled_stored
from workloads import lattice_workload, ragged_workload

pytestmark = pytest.mark.gpu


sp = pytest.importorskip("paper_2303_07819_amd")


def _say(*a):
    print(*a, flush=True)


def compare(w, nsteps, N0, N1, n_t, flags=0, oflags=0, tol=TOL):
    _say(f"coupled {w.name} ncells={w.ncells} n={w.nfloes} steps={nsteps} N0={N0} N1={N1} n_t={n_t}")
    st, Q, mom, cfl = oracle.run_coupled(w, nsteps, N0, N1, n_t, flags=oflags)
    Qs, moms = run_coupled_stored(w, nsteps, N0, N1, n_t, flags=oflags)
    fm, fq = storage_floors(mom, moms), storage_floors(Q, Qs)
    with sp.Sim.from_workload(w, flags=flags) as s:
        s.set_coupling(N0, N1, n_t)
        s.step(w.dt, nsteps)
        gm = s.read_moments(sp.MOMENTS_DEM)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
        gf = s.read_floes()
        cp = s.coupling()
        stats = s.stats()
    e_m = rel_err(gm, mom, fm)
    e_q = rel_err(gq, Q, fq)
    e_r = np.abs(gf["r"] - st.r) / st.r
    _say(f"  max rel err moments {e_m.max():.2e} continuum {e_q.max():.2e} radii {e_r.max():.2e} "
         f"(floors {fm.max():.1e} {fq.max():.1e}) {cp}")
    assert cp["clamped"] == 0 and cp["invalid"] == 0
    assert np.array_equal(gm[:, 0], mom[:, 0])
    assert e_r.max() <= 4e-7 * max(1, cp["nudges"])
    assert e_m.max() <= tol, np.unravel_index(e_m.argmax(), e_m.shape)
    assert e_q.max() <= tol, np.unravel_index(e_q.argmax(), e_q.shape)
    if cfl > 0:
        assert stats["max_cfl"] == pytest.approx(cfl, rel=tol)
    return cp


def _static():
    counts = np.random.default_rng(4).integers(1, 9, 24)
    return lattice_workload(counts, 6, 4, seed=4)


@pytest.mark.parametrize("nsteps", [4, 6, 10])
def test_static_lattice_schedule(nsteps):
    """Floes at rest without ocean: only the schedule acts (closed forms pinned
    on the oracle); nudges at j = 6 and 10."""
    cp = compare(_static(), nsteps, 4, 2, 2, flags=sp.SP_OCEAN_OFF, oflags=oracle.OCEAN_OFF)
    assert cp["nudges"] == {4: 0, 6: 1, 10: 2}[nsteps]


@pytest.mark.parametrize("nsteps,N0,N1,n_t", [(13, 4, 2, 2), (12, 6, 1, 4), (9, 3, 3, 1)])
def test_small_config(nsteps, N0, N1, n_t):
    compare(fixtures.make_config(0), nsteps, N0, N1, n_t)


def test_drifting_lattice_with_subcycles():
    nx, ny = 8, 4
    counts = np.random.default_rng(7).integers(1, 9, nx * ny)
    w = lattice_workload(counts, nx, ny, u=0.35, v=-0.2, seed=7)
    compare(w, 17, 5, 3, 2, flags=sp.SP_OCEAN_OFF, oflags=oracle.OCEAN_OFF)


def test_ragged_and_empty_cells_first_coarse_step():
    """Empty, single-floe and 700-floe cells: window statistics and two coarse
    steps; n_t = N0 takes no coarse-to-fine update (they would clamp here, see
    the next test)."""
    cp = compare(ragged_workload(), 7, 3, 2, 3)
    assert cp["nudges"] == 0


def _first_update(w, N0):
    """Coarse step, then the first coarse-to-fine update (n_t = 1): the DEM
    cell values before it (X0), the coarse state, the values after it, the
    radii and the counters."""
    m = oracle.Model(w)
    with sp.Sim.from_workload(w) as s:
        s.set_coupling(N0, 1, 1)
        s.step(w.dt, N0)
        x0 = oracle.q_from_moments(m, s.read_moments(sp.MOMENTS_DEM))
        q = s.read_moments(sp.MOMENTS_CONTINUUM)
        s.step(w.dt, 1)
        after = oracle.q_from_moments(m, s.read_moments(sp.MOMENTS_DEM))
        f = s.read_floes()
        cp = s.coupling()
    return x0 + (1.0 / N0) * (q - x0), after, f, cp


def _on_target(w, after, target, floes, cells):
    """|after - target| <= 1e-5 max(|target|, 1e-3 rms) plus what storing the
    updated floes in FP32 alone can move the cell values (the update computes
    its shifts in FP64 and rounds the new velocities and spins once)."""
    rms = np.sqrt(np.mean(target[cells] ** 2, axis=0))
    allow = TOL * np.maximum(np.abs(target[cells]), FLOOR * rms) + fp32_storage_bound(w, floes)[cells]
    err = np.abs(after[cells] - target[cells])
    ratio = np.where(allow > 0, err / np.where(allow > 0, allow, 1.0), np.where(err > 0, np.inf, 0.0))
    _say(f"  largest error / allowance {ratio.max():.2f}; relative at the 1e-3 floor "
         f"{rel_err(after[cells], target[cells]).max():.2e}")
    return ratio.max()


def test_ragged_updates_land_on_targets_after_a_replan():
    """Single-floe cells beside dense ones get targets far above their mass;
    the coarse step re-plans the contact search for the radii they need, and
    every cell with floes lands on its target."""
    w = ragged_workload()
    target, after, f, cp = _first_update(w, 3)
    r = f["r"]
    has = np.diff(w.start) > 0
    _say(f"  counters {cp}, largest radius {r.max():.1f} (initially {w.r.max():.1f})")
    assert cp["nudges"] == 1 and cp["replans"] == 1 and cp["clamped"] == 0 and cp["invalid"] == 0
    assert r.max() > 1.5 * w.r.max()
    assert _on_target(w, after, target, f, has) <= 1.0


def test_clamp_only_past_a_quarter_cell():
    """A thin floe (h = 2 cm) alone in a cell between cells of nine 2 km floes:
    its target would need a radius past a quarter of the cell (the periodic
    cell DEM's limit); it stops there, is counted as clamped and stays below
    its target mass; every other cell lands on its target."""
    nx, ny = 4, 3
    counts = np.full(nx * ny, 9)
    counts[5] = 1
    w = lattice_workload(counts, nx, ny, r=2000.0, seed=3, big_radius=0.0)
    w.h[w.start[5]] = 0.02
    r_lim = np.float32(0.25 * w.Lx * (1.0 - 1e-6))
    target, after, f, cp = _first_update(w, 3)
    r = f["r"]
    rmax_cell = np.array([r[w.start[c]:w.start[c + 1]].max() for c in range(w.ncells)])
    clamped = rmax_cell == r_lim
    _say(f"  clamped cells {np.flatnonzero(clamped).tolist()} counters {cp}")
    assert np.flatnonzero(clamped).tolist() == [5] and cp["clamped"] == 1 and cp["invalid"] == 0
    assert after[5, 0] < target[5, 0]
    assert _on_target(w, after, target, f, ~clamped) <= 1.0


def test_unit_cadence_is_the_plain_step_and_cadence_changes_mid_run():
    w = fixtures.make_config(0)
    with sp.Sim.from_workload(w) as a, sp.Sim.from_workload(w) as b:
        a.step(w.dt, 7)
        b.set_coupling(1, 1, 1)
        b.step(w.dt, 7)
        for x, y in ((a.read_moments(sp.MOMENTS_CONTINUUM), b.read_moments(sp.MOMENTS_CONTINUUM)),
                     (a.read_moments(sp.MOMENTS_DEM), b.read_moments(sp.MOMENTS_DEM))):
            assert np.array_equal(x, y)
    # 6 coupled steps, then 3 plain ones from the state and coarse field reached
    st, Q, _, _ = oracle.run_coupled(w, 6, 4, 2, 2)
    st, Q, mom, _ = oracle.run_plain(w, 3, state=st, Q0=Q)
    with sp.Sim.from_workload(w) as s:
        s.set_coupling(4, 2, 2)
        s.step(w.dt, 6)
        s.set_coupling(1)
        s.step(w.dt, 3)
        gm = s.read_moments(sp.MOMENTS_DEM)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
    _say(f"  mid-run change: moments {rel_err(gm, mom).max():.2e} continuum {rel_err(gq, Q).max():.2e}")
    assert rel_err(gm, mom).max() <= TOL
    assert rel_err(gq, Q).max() <= TOL


def test_error_paths():
    w = fixtures.make_config(0)
    with sp.Sim.from_workload(w) as s:
        for bad in ((0, 1, 1), (2, 0, 1), (2, 1, 0), (sp.SP_MAX_COUPLING + 1, 1, 1), (2, sp.SP_MAX_COUPLING + 1, 1)):
            with pytest.raises(sp.SpdemError):
                s.set_coupling(*bad)
        s.set_coupling(4, 1, 2)
        with pytest.raises(sp.SpdemError):
            s.profile_steps(w.dt, 2)
        assert s.coupling()["N0"] == 4
    with sp.Sim.from_workload(w, flags=sp.SP_NO_CONTINUUM) as s:
        with pytest.raises(sp.SpdemError):
            s.set_coupling(4, 1, 2)


def test_full_size_plain64_first_coarse_step_and_nudge():
    """plain64 (64 x 64 cells, 1,048,576 floes) at the paper's default cadence
    N0 = 100 is too long for the oracle; at N0 = 6, N1 = 2, n_t = 3: the coarse
    state of sampled cells after the first coarse step against the oracle on
    their domain of dependence; the coarse mass is conserved; after the first
    nudge of the second coarse step every cell sits at X0 + (3/6)(Q - X0)."""
    w = fixtures.make_config(1)
    N0, N1, n_t = 6, 2, 3
    with sp.Sim.from_workload(w) as s:
        q0 = s.read_moments(sp.MOMENTS_CONTINUUM)
        s.set_coupling(N0, N1, n_t)
        s.step(w.dt, N0)
        gq = s.read_moments(sp.MOMENTS_CONTINUUM)
        x0 = oracle.q_from_moments(oracle.Model(w), s.read_moments(sp.MOMENTS_DEM))
        s.step(w.dt, n_t)
        after = oracle.q_from_moments(oracle.Model(w), s.read_moments(sp.MOMENTS_DEM))
        gq2 = s.read_moments(sp.MOMENTS_CONTINUUM)
        floes = s.read_floes()
        cp = s.coupling()
    assert cp["nudges"] == 1 and cp["clamped"] == 0 and cp["invalid"] == 0
    np.testing.assert_array_equal(gq2, gq)
    assert abs(gq[:, 0].sum() - q0[:, 0].sum()) <= 1e-12 * abs(q0[:, 0].sum())
    target = x0 + 0.5 * (gq - x0)
    assert _on_target(w, after, target, floes, np.ones(w.ncells, bool)) <= 1.0
    m = oracle.Model(w)
    k = N1
    for (cx, cy) in ((0, 0), (41, 17), (63, 63)):
        ix = (cx + np.arange(-k - 1, k + 2)) % w.nx
        iy = (cy + np.arange(-k - 1, k + 2)) % w.ny
        cells = (iy[:, None] * w.nx + ix[None, :]).reshape(-1)
        st = oracle.State.from_workload(w)
        mom0 = oracle.moments(m, st)[cells]
        rec, _ = oracle.dem_steps(m, st, w.dt, N0, cells=cells, record=True)
        win = fixtures.from_arrays(ix.size, iy.size, w.Lx, np.zeros(cells.size, np.int32), [], [], [], [])
        wm = oracle.Model(win)
        Q = oracle.q_from_moments(wm, mom0)
        mean = rec.mean(axis=0)
        for _ in range(N1):
            Q, _ = oracle.lf_step(wm, Q, mean, N0 * w.dt / N1)
        centre = (k + 1) * ix.size + (k + 1)
        got = gq[cy * w.nx + cx]
        ref = Q[centre]
        e = np.abs(got - ref) / np.maximum(np.abs(ref), FLOOR * np.sqrt(np.mean(gq ** 2, axis=0)))
        _say(f"  cell ({cx},{cy}) coarse state rel err {e.max():.2e}")
        assert e.max() <= TOL


@pytest.mark.parametrize("block", [32, 1])
def test_one_call_equals_many_calls_across_a_replan(block):
    """The ragged workload re-plans its contact search (larger sub-bins and
    skin, new list buffers) at the first coarse step (N0 = 3): 5 steps in one
    sp_step call and in 5 calls of one step give the same floes bit for bit,
    so the steps after a re-plan inside a call use the new plan."""
    w = ragged_workload()
    out = []
    for calls in ((5,), (1,) * 5):
        with sp.Sim.from_workload(w) as s:
            s.set_step_block(block)
            s.set_coupling(3, 1, 1)
            for n in calls:
                s.step(w.dt, n)
            out.append((s.read_floes(), s.coupling()))
    (fa, ca), (fb, cb) = out
    _say(f"  block={block}: {ca}")
    assert ca["replans"] >= 1 and ca == cb
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
