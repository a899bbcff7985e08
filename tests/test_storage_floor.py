"""How far the 32-bit storage of the floe state alone moves the cell moments,
and the parity floors derived from it.

The oracle is rerun with its state rounded after every step to the formats the
HIP path stores (positions to 2^-32 of the cell, velocities and spin to FP32);
its deviation from the pure FP64 oracle is the floor no FP32-state
implementation can beat.  The parity bar is |a - b| <= 1e-5 max(|b|, f rms)
with f = 1e-3 (the relative-error floor of the stated tolerance), raised per
component only where this deviation would use more than a fifth of the
allowance (metrics.storage_floors): a fifth of it.
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import FLOOR, STORAGE_MARGIN, TOL, rel_err, storage_floors
from storage import coupled_floor, run_plain_stored
from workloads import dense_workload, ragged_workload, uneven_workload


def test_floor_is_the_stated_one():
    assert FLOOR == 1e-3 and TOL == 1e-5 and STORAGE_MARGIN == 5.0


def test_storage_floors_definition():
    b = np.array([[1.0, 0.0], [-1.0, 2e-3], [3.0, 0.0]])
    stored = b + np.array([[0.0, 0.0], [0.0, 1e-9], [0.0, 0.0]])
    rms = np.sqrt(np.mean(b * b, axis=0))
    f = storage_floors(b, stored)
    assert f[0] == FLOOR                                   # untouched column keeps the stated floor
    assert f[1] == pytest.approx(max(FLOOR, STORAGE_MARGIN * 1e-9 / (TOL * rms[1])))
    # with the derived floor the stored result itself passes at a fifth of the bar
    assert rel_err(stored, b, f).max() <= TOL / STORAGE_MARGIN * (1 + 1e-12)


@pytest.mark.parametrize("name", ["small", "dense", "ragged", "uneven"])
def test_storage_floor(name):
    w = {"small": lambda: fixtures.make_config(0), "dense": dense_workload, "ragged": ragged_workload,
         "uneven": uneven_workload}[name]()
    _, Q, mom, _ = oracle.run_plain(w, 10)
    Qs, moms = run_plain_stored(w, 10)
    dev = max(rel_err(moms, mom).max(), rel_err(Qs, Q).max())
    fm, fq = storage_floors(mom, moms), storage_floors(Q, Qs)
    print(f"{name}: storage-only deviation after 10 steps {dev:.2e} at the 1e-3 floor; derived floors "
          f"moments {np.array2string(fm, precision=1)} continuum {np.array2string(fq, precision=1)}")
    # the storage alone passes the bar with its derived floors, at a fifth of it
    assert rel_err(moms, mom, fm).max() <= TOL / STORAGE_MARGIN * (1 + 1e-9)
    assert rel_err(Qs, Q, fq).max() <= TOL / STORAGE_MARGIN * (1 + 1e-9)
    # the storage alone stays below 1e-6 of every component's scale (rms), so
    # no derived floor passes 0.5 (allowance 5e-6 rms)
    assert max(fm.max(), fq.max()) <= 0.5
    if name == "small":
        assert dev < 5e-5            # no contacts: storage rounding is not amplified
    else:
        assert 1e-7 < dev < 1e-3     # contacts amplify it


@pytest.mark.parametrize("case", [(13, 4, 2, 2), (12, 6, 1, 4), (9, 3, 3, 1)])
def test_coupled_storage_floor(case):
    """Coupled cadence on the small configuration: a coarse-to-fine update sets
    each cell's momentum to a target close to its current value, so the FP32
    rounding of the shifted velocities is amplified in the drag sums that feed
    the next coarse step; updates every fine step (n_t = 1) lift the floor above
    1e-5 at the 1e-3 floor, which is why the coupled parity derives its floors
    from the stored rerun too."""
    floor = coupled_floor(fixtures.make_config(0), *case)
    print(f"coupled {case}: storage-only deviation {floor:.2e}")
    assert 1e-8 < floor < 1e-2
