"""Save and restore (sp_save / sp_load, Algorithm 1's final save of the run's
data): a run saved after 5 steps and restored into a fresh context continues
exactly as the straight run (needs an MI355X).

Bar: floe state, DEM statistics, continuum, contact and step counters equal
to the straight 10-step run bit for bit, on the blocked path (the default),
the per-step path (a pending continuum update saved as pending) and with the
tangential spring (contact history saved).
"""
import numpy as np
import pytest

import fixtures
from workloads import dense_workload

pytestmark = pytest.mark.gpu

sp = pytest.importorskip("paper_2303_07819_amd")


def _say(*a):
    print(*a, flush=True)


def _snapshot(s):
    return dict(floes=s.read_floes(), mom=s.read_moments(sp.MOMENTS_DEM), q=s.read_moments(sp.MOMENTS_CONTINUUM),
                stats=s.stats(), work=s.work())


def _equal(a, b):
    for key in a["floes"]:
        assert np.array_equal(a["floes"][key], b["floes"][key]), key
    assert np.array_equal(a["mom"], b["mom"])
    assert np.array_equal(a["q"], b["q"])
    assert a["stats"] == b["stats"], (a["stats"], b["stats"])
    assert a["work"] == b["work"], (a["work"], b["work"])


@pytest.mark.parametrize("name,k,flags", [("small", 32, 0), ("dense", 32, 0), ("dense", 1, 0), ("dense", 4, 0),
                                          ("small", 1, 0), ("dense", 1, sp.SP_TANGENTIAL_SPRING),
                                          ("dense", 32, sp.SP_TANGENTIAL_SPRING)])
def test_resumed_run_equals_straight_run(tmp_path, name, k, flags):
    w = fixtures.make_config(0) if name == "small" else dense_workload(seed=3)
    if flags & sp.SP_TANGENTIAL_SPRING:
        w.G = 80.0
    with sp.Sim.from_workload(w, flags=flags) as s:
        s.set_step_block(k)
        s.step(w.dt, 10)
        straight = _snapshot(s)
    path = str(tmp_path / "run.spdem")
    with sp.Sim.from_workload(w, flags=flags) as s:
        s.set_step_block(k)
        s.step(w.dt, 5)
        s.save(path)
        s.step(w.dt, 5)               # saving does not change the saved run
        after = _snapshot(s)
    # a fresh context with another initial state: everything comes from the file
    w2 = fixtures.make_config(0) if name == "small" else dense_workload(seed=3)
    w2.u = w2.u + np.float32(0.01)
    w2.G = w.G
    with sp.Sim.from_workload(w2, flags=flags) as s:
        s.set_step_block(k)
        s.load(path)
        assert s.n == w.nfloes
        s.step(w.dt, 5)
        resumed = _snapshot(s)
    _say(f"{name} k={k} flags={flags}: contacts {straight['stats']['contacts']}, steps {straight['stats']['steps']}")
    _equal(straight, after)
    _equal(straight, resumed)


def test_load_refuses_other_parameters_and_foreign_files(tmp_path):
    w = fixtures.make_config(0)
    path = str(tmp_path / "run.spdem")
    with sp.Sim.from_workload(w) as s:
        s.step(w.dt, 3)
        s.save(path)
    w.E = 2.0 * w.E
    with sp.Sim.from_workload(w) as s:
        with pytest.raises(sp.SpdemError) as e:
            s.load(path)
        assert e.value.status == -1
    bad = tmp_path / "bad.spdem"
    bad.write_bytes(b"not a simulation" * 8)
    w.E = 0.5 * w.E
    with sp.Sim.from_workload(w) as s:
        with pytest.raises(sp.SpdemError):
            s.load(str(bad))
        with pytest.raises(sp.SpdemError):
            s.load(str(tmp_path / "missing.spdem"))
        # truncated: the header alone
        (tmp_path / "cut.spdem").write_bytes(open(path, "rb").read()[:600])
        with pytest.raises(sp.SpdemError):
            s.load(str(tmp_path / "cut.spdem"))
        s.step(w.dt, 1)               # the context still works after the refusals


def test_save_refuses_hybrid_and_coupled_cadence(tmp_path):
    w = fixtures.make_config(0)
    with sp.Sim.from_workload(w) as s:
        s.set_coupling(4, 1, 2)
        s.step(w.dt, 2)
        with pytest.raises(sp.SpdemError) as e:
            s.save(str(tmp_path / "x.spdem"))
        assert e.value.status == -7
