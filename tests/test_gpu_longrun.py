"""A long run on the HIP path judged against the oracle (needs an MI355X): the
plain 64 x 64 workload (cells of 25 km, 1,048,576 floes, 256 per cell, dt =
30 s) over 10^4 steps, well into its dense phase.

1. The run stays sound: every floe finite, radii unchanged, floe
   counts, mass and ice area per cell unchanged.
2. Late-state parity: the GPU state at step 9000 is saved; ten steps from it
   on the GPU against ten oracle steps of 64 sampled cells restarted from that
   state, at the bar of the dense parity tests (1e-5 relative at a floor of
   1e-3 of each statistic's rms, raised to five times what the 32-bit state
   storage alone moves it).
3. Statistics after 1000 more steps from the reloaded state: the oracle
   restarted from the same GPU state on 256 sampled cells (the cells' DEMs
   never interact on this path, so a sample of them is a run of the same
   system) against the GPU at step 10^4 on those cells: the sample's total
   momentum and spin, the distributions over cells of |P| and of L (their
   deciles), and the mean contacts per floe and step over the 1000 steps
   (the GPU's over all cells, the oracle's over its sample).  Over 1000 steps
   the two runs' floe trajectories need not stay equal, so these are compared
   as statistics, each bar stated with its test.
"""
import os
import tempfile

import numpy as np
import pytest

import fixtures
import oracle
from metrics import TOL, rel_err, storage_floors

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2303_07819_amd")

N_LATE, N_WIN, N_PAR = 9000, 1000, 10
M_MASS, M_PX, M_PY, M_L, M_AICE = 1, 2, 3, 4, 10


def _say(*a):
    print(*a, flush=True)


def _sample(w, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(np.flatnonzero(w.counts > 0), n, replace=False)).astype(np.int32)


def _state(w, fl):
    return oracle.State.from_fixed(fl["xi"], fl["yi"], fl["u"], fl["v"], fl["omega"], fl["theta"], fl["r"], w.h)


def _stored_run(w, m, st, cells, nsteps):
    """The oracle with the listed cells' state rounded after every step to the
    formats the GPU stores: what the 32-bit storage alone changes."""
    st = st.copy()
    idx = np.concatenate([np.arange(w.start[c], w.start[c + 1]) for c in cells])
    for _ in range(nsteps):
        oracle.dem_steps(m, st, w.dt, 1, cells=cells)
        for a in (st.u, st.v, st.w):
            a[idx] = a[idx].astype(np.float32)
        for a in (st.xs, st.ys):
            a[idx] = np.round(a[idx] * 2.0 ** 32) / 2.0 ** 32 % 1.0
    return oracle.moments(m, st)[cells]


@pytest.fixture(scope="module")
def longrun():
    w = fixtures.make_config("plain64")
    oracle.set_threads(min(16, os.cpu_count() or 1))
    out = {"w": w}
    with tempfile.TemporaryDirectory() as tmp, sp.Sim.from_workload(w) as s:
        m0 = s.read_moments(sp.MOMENTS_DEM)
        s.step(w.dt, N_LATE)
        c_late = s.stats()["contacts"]
        fl = s.read_floes()
        path = os.path.join(tmp, "late.spck")
        s.save(path)
        s.step(w.dt, N_PAR)
        out["par"] = s.read_moments(sp.MOMENTS_DEM)
        s.load(path)
        assert s.stats()["contacts"] == c_late
        s.step(w.dt, N_WIN)
        out["end"] = s.read_moments(sp.MOMENTS_DEM)
        out["end_floes"] = s.read_floes()
        out["gpu_rate"] = 2.0 * (s.stats()["contacts"] - c_late) / (w.nfloes * N_WIN)
        assert s.stats()["steps"] == N_LATE + N_WIN
    out["m0"], out["late"] = m0, fl
    _say(f"GPU: {N_LATE + N_WIN} steps of {w.nfloes} floes; contacts per floe and step over the last "
         f"{N_WIN}: {out['gpu_rate']:.4f}")
    return out


def test_long_run_stays_sound(longrun):
    w, fl, m0, end = longrun["w"], longrun["end_floes"], longrun["m0"], longrun["end"]
    for k in ("u", "v", "omega", "theta", "r"):
        assert np.all(np.isfinite(fl[k])), k
    assert np.array_equal(fl["r"], w.r.astype(np.float32))
    assert np.array_equal(end[:, 0], m0[:, 0])                       # floes per cell
    np.testing.assert_allclose(end[:, M_MASS], m0[:, M_MASS], rtol=1e-13)
    np.testing.assert_allclose(end[:, M_AICE], m0[:, M_AICE], rtol=1e-13)
    # the dense phase: contacts are no longer rare
    assert longrun["gpu_rate"] > 0.1


def test_late_state_parity_over_ten_steps(longrun):
    w = longrun["w"]
    cells = _sample(w, 64, seed=90)
    m = oracle.Model(w, oracle.BINNED)
    st = _state(w, longrun["late"])
    ref_st = st.copy()
    oracle.dem_steps(m, ref_st, w.dt, N_PAR, cells=cells)
    ref = oracle.moments(m, ref_st)[cells]
    stored = _stored_run(w, m, st, cells, N_PAR)
    got = longrun["par"][cells]
    e = rel_err(got, ref, storage_floors(ref, stored)).max()
    _say(f"late-state parity, {cells.size} cells x {N_PAR} steps from step {N_LATE}: {e:.2e}")
    assert np.array_equal(got[:, 0], ref[:, 0])
    assert e <= TOL


def _deciles(x):
    return np.quantile(x, np.linspace(0.1, 0.9, 9))


def test_statistics_after_a_thousand_steps_match_the_oracle(longrun):
    w = longrun["w"]
    cells = _sample(w, 256, seed=91)
    m = oracle.Model(w, oracle.BINNED)
    st = _state(w, longrun["late"])
    _, stats = oracle.dem_steps(m, st, w.dt, N_WIN, cells=cells)
    ref = oracle.moments(m, st)[cells]
    got = longrun["end"][cells]
    nfl = int(sum(int(w.counts[c]) for c in cells))
    orc_rate = 2.0 * stats[0] / (nfl * N_WIN)
    # total momentum and spin of the sample, relative to the summed magnitudes
    d_px = abs(got[:, M_PX].sum() - ref[:, M_PX].sum()) / np.abs(ref[:, M_PX]).sum()
    d_py = abs(got[:, M_PY].sum() - ref[:, M_PY].sum()) / np.abs(ref[:, M_PY]).sum()
    d_l = abs(got[:, M_L].sum() - ref[:, M_L].sum()) / np.abs(ref[:, M_L]).sum()
    # deciles over cells of |P| and of L, relative to the median magnitude
    pg, pr = np.hypot(got[:, M_PX], got[:, M_PY]), np.hypot(ref[:, M_PX], ref[:, M_PY])
    q_p = np.abs(_deciles(pg) - _deciles(pr)).max() / np.median(pr)
    q_l = np.abs(_deciles(got[:, M_L]) - _deciles(ref[:, M_L])).max() / np.median(np.abs(ref[:, M_L]))
    # per-cell distance (how far the trajectories drifted apart), for the record
    cell_p = np.sqrt(np.mean((pg - pr) ** 2) / np.mean(pr ** 2))
    cell_l = np.sqrt(np.mean((got[:, M_L] - ref[:, M_L]) ** 2) / np.mean(ref[:, M_L] ** 2))
    d_rate = abs(longrun["gpu_rate"] - orc_rate) / orc_rate
    _say(f"after {N_WIN} steps from step {N_LATE}, {cells.size} cells: sample momentum {d_px:.2e} {d_py:.2e}, "
         f"spin {d_l:.2e}; deciles |P| {q_p:.2e}, L {q_l:.2e}; per-cell rms |P| {cell_p:.2e}, L {cell_l:.2e}; "
         f"contacts per floe-step GPU {longrun['gpu_rate']:.4f} oracle {orc_rate:.4f} ({d_rate:.2e})")
    assert np.array_equal(got[:, 0], ref[:, 0])
    # Measured when this test was written: momentum totals 2.5e-6 and 2.8e-6,
    # spin 1.5e-4, deciles 6.8e-4 (|P|) and 5.0e-3 (L), per-cell rms 3.9e-5 and
    # 1.8e-3, contact rates 1.5e-2 apart (all cells against the sample).
    # Momentum follows the common ocean forcing: the sample totals within 1e-3.
    assert d_px <= 1e-3 and d_py <= 1e-3
    # Spin is set by contacts and the drag torque: the sample total within 1 %
    # of the summed magnitudes, the deciles of |P| within 0.5 % and of L within
    # 3 % of the median.
    assert d_l <= 1e-2
    assert q_p <= 5e-3
    assert q_l <= 3e-2
    # The contact rate of the whole GPU run against the oracle's sample: 5 %.
    assert d_rate <= 5e-2
