"""How far the 32-bit storage of the floe state alone moves the cell moments.

The oracle is rerun with its state rounded after every step to the formats the
HIP path stores (positions to 2^-32 of the cell, velocities and spin to FP32);
its deviation from the pure FP64 oracle is the floor no FP32-state
implementation can beat.  The GPU bars of the parity tests are set from it:
1e-5 (the stated tolerance) on the benchmark-style workloads, and five times
this floor on contact-dominated stress workloads after 10 steps.
"""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import rel_err
from workloads import dense_workload, ragged_workload, uneven_workload


def run_stored(w, nsteps):
    m = oracle.Model(w)
    st = oracle.State.from_workload(w)
    Q = oracle.q_from_moments(m, oracle.moments(m, st))
    for _ in range(nsteps):
        mom, _ = oracle.dem_steps(m, st, w.dt, 1, record=True)
        Q, _ = oracle.lf_step(m, Q, mom[0], w.dt)
        for a in (st.u, st.v, st.w):
            a[:] = a.astype(np.float32)
        for a in (st.xs, st.ys):
            a[:] = np.round(a * 2.0 ** 32) / 2.0 ** 32 % 1.0
    return Q, oracle.moments(m, st)


@pytest.mark.parametrize("name", ["small", "dense", "ragged", "uneven"])
def test_storage_floor(name):
    w = {"small": lambda: fixtures.make_config(0), "dense": dense_workload, "ragged": ragged_workload,
         "uneven": uneven_workload}[name]()
    _, Q, mom, _ = oracle.run_plain(w, 10)
    Qs, moms = run_stored(w, 10)
    floor = max(rel_err(moms, mom).max(), rel_err(Qs, Q).max())
    print(f"{name}: storage-only deviation after 10 steps {floor:.2e}")
    if name == "small":
        assert floor < 2e-6          # no contacts: storage rounding is not amplified
    else:
        assert 1e-7 < floor < 1e-5   # contacts amplify it, but it stays below the bar
