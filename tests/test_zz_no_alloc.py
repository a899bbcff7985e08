"""The entry point that allocates nothing (sp_read_moments_noalloc) against
sp_read_moments through the C ABI (needs an MI355X): the same values bit for
bit on two calls in a row, the second on a smaller workload, for the DEM
statistics and the continuum; a context above the static scratch's 65,536
cells is refused."""
import numpy as np
import pytest

import fixtures
from workloads import dense_workload

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2303_07819_amd")


def _say(*a):
    print(*a, flush=True)


def _both(s):
    out = []
    for which in (sp.MOMENTS_DEM, sp.MOMENTS_CONTINUUM):
        a = s.read_moments(which)
        b = s.read_moments_noalloc(which)
        out.append((a, b))
    return out


def test_noalloc_read_equals_read_on_two_calls_in_a_row():
    big = fixtures.make_config(1)                 # 64 x 64 cells, 1,048,576 floes
    small = dense_workload(seed=5)                # 3 x 2 cells
    with sp.Sim.from_workload(big) as s:
        s.step(big.dt, 7)
        first = _both(s)
    with sp.Sim.from_workload(small) as s:
        s.step(small.dt, 3)
        second = _both(s)
        # a second call on the same context after more steps
        s.step(small.dt, 2)
        third = _both(s)
    for name, res in (("plain64", first), ("dense 3x2", second), ("dense 3x2 again", third)):
        for (a, b), which in zip(res, ("DEM", "continuum")):
            _say(f"{name} {which}: shape {b.shape}, equal {np.array_equal(a, b)}")
            assert a.shape == b.shape and np.array_equal(a, b)
    assert first[0][1].shape == (big.ncells, sp.NMOM) and second[0][1].shape == (small.ncells, sp.NMOM)


def test_noalloc_read_refuses_more_cells_than_its_scratch():
    nx, ny = 257, 256                             # 65,792 cells, no floes
    w = fixtures.from_arrays(nx, ny, 25e3, np.zeros(nx * ny, np.int32), [], [], [], [])
    with sp.Sim.from_workload(w) as s:
        with pytest.raises(sp.SpdemError) as ei:
            s.read_moments_noalloc(sp.MOMENTS_DEM)
        assert ei.value.status == -8              # SP_ECAPACITY
        assert s.read_moments(sp.MOMENTS_DEM).shape == (nx * ny, sp.NMOM)
