"""Batched uneven cells: count buckets, wavefront / tile groups, persistent
workgroups, the autotuner and graph replay (needs an MI355X).

Every batching choice must give the same floe state bit for bit (each floe's
arithmetic does not depend on how cells are grouped) and statistics equal to
FP64 rounding; the uneven workload must match the oracle like the plain one.
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import TOL, rel_err, report, storage_floors
from storage import dem_cells_stored, run_plain_stored
from workloads import uneven_workload

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2303_07819_amd")



def _say(*a):
    print(*a, flush=True)


def run(w, nsteps, waves=None, persistent=None, chunk=None, autotune=False, block=None):
    s = sp.Sim.from_workload(w)
    if block is not None:
        s.set_step_block(block)
    if chunk is not None:
        s.set_graph_chunk(chunk)
    if waves is not None:
        s.set_batching(waves, persistent)
    if autotune:
        s.autotune(w.dt, 2)
    s.step(w.dt, nsteps)
    out = (s.read_floes(), s.read_moments(sp.MOMENTS_DEM), s.read_moments(sp.MOMENTS_CONTINUUM),
           s.batching())
    s.close()
    return out


def test_uneven_buckets_cover_all_cells():
    """Every cell with floes sits in the bucket of its count; cells without
    floes are in none (they take only the continuum update)."""
    w = uneven_workload()
    assert (w.counts == 0).any()
    with sp.Sim.from_workload(w) as s:
        cells, waves, q = s.batching()
    edges = [0, 64, 128, 256, 512, 1024]
    for b in range(5):
        expect = np.sum((w.counts > edges[b]) & (w.counts <= edges[b + 1]))
        assert cells[b] == expect, (b, cells[b], expect)
    assert cells.sum() == np.sum(w.counts > 0)
    assert list(waves) == [1, 2, 4, 4, 8] and not q.any()


@pytest.mark.parametrize("nsteps", [1, 10])
def test_uneven_parity(nsteps):
    w = uneven_workload()
    _say(f"uneven {w.ncells} cells, {w.nfloes} floes, counts {w.counts.min()}..{w.counts.max()}")
    st, Q, mom, _ = oracle.run_plain(w, nsteps)
    Qs, moms = run_plain_stored(w, nsteps)
    f, gm, gq, _ = run(w, nsteps)
    em, eq = rel_err(gm, mom, storage_floors(mom, moms)).max(), rel_err(gq, Q, storage_floors(Q, Qs)).max()
    _say(f"  max rel err moments {em:.2e} continuum {eq:.2e}")
    _say("  moments   " + report(gm, mom, storage_floors(mom, moms), oracle.MOMENT_NAMES))
    _say("  continuum " + report(gq, Q, storage_floors(Q, Qs), oracle.Q_NAMES))
    assert np.array_equal(gm[:, 0], mom[:, 0])
    assert em <= TOL and eq <= TOL


def test_every_batching_gives_the_same_floes():
    w = uneven_workload(seed=8)
    rng = np.random.default_rng(0)
    w.u[:] = rng.normal(0, 0.2, w.nfloes)        # contacts within the run
    w.v[:] = rng.normal(0, 0.2, w.nfloes)
    ref = run(w, 6, chunk=0)
    for waves in (1, 2, 4, 8):
        for persistent in (0, 1):
            got = run(w, 6, waves=[waves] * 5, persistent=[persistent] * 5, chunk=0)
            _say(f"waves {waves} persistent {persistent}")
            for k in ref[0]:
                assert np.array_equal(ref[0][k], got[0][k]), (waves, persistent, k)
            np.testing.assert_allclose(got[1], ref[1], rtol=1e-12, atol=1e-300)
            np.testing.assert_allclose(got[2], ref[2], rtol=1e-12, atol=1e-300)


def test_graph_replay_equals_eager():
    w = uneven_workload(seed=4)
    eager = run(w, 37, chunk=0)
    graph = run(w, 37, chunk=8)
    for k in eager[0]:
        assert np.array_equal(eager[0][k], graph[0][k]), k
    assert np.array_equal(eager[1], graph[1])
    assert np.array_equal(eager[2], graph[2])


def test_autotune_does_not_advance_the_state():
    """Per-step launches (block length 1): the tuner picks (waves, persistent)
    per bucket; the state it leaves is the untuned one's bit for bit."""
    w = uneven_workload(seed=5)
    plain = run(w, 4, chunk=0, block=1)
    tuned = run(w, 4, chunk=0, autotune=True, block=1)
    _say(f"autotuned waves {tuned[3][1].tolist()} persistent {tuned[3][2].tolist()}")
    for k in plain[0]:
        assert np.array_equal(plain[0][k], tuned[0][k]), k
    np.testing.assert_allclose(tuned[2], plain[2], rtol=1e-12, atol=1e-300)


def test_autotune_of_blocked_steps_keeps_the_state():
    """Blocked steps (the default): the tuner times the blocked kernel per
    bucket over its wavefronts per cell and the block length; steps after
    tuning give the untuned floe state bit for bit (the per-floe arithmetic
    does not depend on W or the block length) and its continuum to FP64
    rounding."""
    w = uneven_workload(seed=6)
    rng = np.random.default_rng(1)
    w.u[:] = rng.normal(0, 0.2, w.nfloes)
    w.v[:] = rng.normal(0, 0.2, w.nfloes)
    with sp.Sim.from_workload(w) as s:
        s.step(w.dt, 37)
        f0, q0 = s.read_floes(), s.read_moments(sp.MOMENTS_CONTINUUM)
        bw0 = s.block_waves()
    with sp.Sim.from_workload(w) as s:
        best = s.autotune(w.dt, 2)
        k, active = s.step_block()
        bw = s.block_waves()
        cells = s.batching()[0]
        s.step(w.dt, 37)
        f1, q1 = s.read_floes(), s.read_moments(sp.MOMENTS_CONTINUUM)
        work = s.work()
    _say(f"blocked autotune: block {k}, waves {bw.tolist()} (default {bw0.tolist()}), best {best:.4f} ms/step")
    assert active and k in (16, 32, 64) and best > 0
    assert work["blocked_steps"] == 37
    for q in range(5):
        if cells[q]:
            assert bw[q] in (1, 2, 4, 8, 16)
    for key in f0:
        assert np.array_equal(f0[key], f1[key]), key
    np.testing.assert_allclose(q1, q0, rtol=1e-12, atol=1e-300)


def test_full_size_uneven128_sampled_cells():
    """The 128x128 uneven workload (~4 M floes) in the benchmark launch
    configuration; sampled cells, including the fullest, against the oracle."""
    w = fixtures.make_config(2)
    nsteps = 10
    rng = np.random.default_rng(2)
    sample = np.unique(np.concatenate([rng.choice(w.ncells, 6, replace=False),
                                       [int(np.argmax(w.counts)), int(np.argmin(w.counts))]]))
    _say(f"uneven128: {w.nfloes} floes, max/cell {w.counts.max()}, sample {sample.tolist()}")
    with sp.Sim.from_workload(w) as s:
        s.step(w.dt, nsteps)
        gm = s.read_moments(sp.MOMENTS_DEM)
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    oracle.dem_steps(m, st, w.dt, nsteps, cells=sample)
    ref = oracle.moments(m, st)[sample]
    e = rel_err(gm[sample], ref, storage_floors(ref, dem_cells_stored(w, nsteps, sample)[sample]))
    _say(f"  max rel err {e.max():.2e}")
    assert e.max() <= TOL
