"""The oracle rerun with its floe state rounded to the formats the HIP path
stores (positions to 2^-32 of the cell, velocities, spin and radii to FP32)
after every fine step and every coarse-to-fine update.  Its deviation from the
pure FP64 oracle is the floor no FP32-state implementation can beat; the parity
bars' per-component floors (metrics.storage_floors) are set from it."""
import numpy as np

import oracle
from metrics import rel_err


def round_state(st):
    for a in (st.u, st.v, st.w, st.r):
        a[:] = a.astype(np.float32)
    for a in (st.xs, st.ys):
        a[:] = np.round(a * 2.0 ** 32) / 2.0 ** 32 % 1.0


def run_plain_stored(w, nsteps, flags=0):
    """oracle.run_plain with the state rounded after every step: (Q, moments)."""
    m = oracle.Model(w, flags)
    st = oracle.State.from_workload(w)
    Q = oracle.q_from_moments(m, oracle.moments(m, st))
    for _ in range(nsteps):
        mom, _ = oracle.dem_steps(m, st, w.dt, 1, record=True)
        Q, _ = oracle.lf_step(m, Q, mom[0], w.dt)
        round_state(st)
    return Q, oracle.moments(m, st)


def dem_cells_stored(w, nsteps, cells, flags=0):
    """The listed cells' DEMs stepped with the state rounded after every step:
    the moments of every cell (the others at their initial state)."""
    m = oracle.Model(w, flags)
    st = oracle.State.from_workload(w)
    for _ in range(nsteps):
        oracle.dem_steps(m, st, w.dt, 1, cells=cells)
        round_state(st)
    return oracle.moments(m, st)


def run_coupled_stored(w, nsteps, N0, N1, n_t, flags=0):
    """oracle.run_coupled's schedule with the state rounded after each change."""
    model = oracle.Model(w, flags)
    st = oracle.State.from_workload(w)
    Q = oracle.q_from_moments(model, oracle.moments(model, st))
    counts = np.diff(model.start)
    window = np.zeros((model.ncells, oracle.NMOM))
    x0 = None
    for j in range(1, nsteps + 1):
        mom, _ = oracle.dem_steps(model, st, w.dt, 1, record=True)
        round_state(st)
        window += mom[0]
        r = j % N0
        if r == 0:
            for _ in range(N1):
                Q, _ = oracle.lf_step(model, Q, window / N0, N0 * w.dt / N1)
            window[:] = 0.0
            x0 = oracle.q_from_moments(model, oracle.moments(model, st))
        elif j > N0 and r % n_t == 0:
            for cell in np.flatnonzero(counts):
                oracle.resync_cell(model, st, int(cell), x0[cell] + (r / N0) * (Q[cell] - x0[cell]))
            round_state(st)
    return Q, oracle.moments(model, st)


def coupled_floor(w, nsteps, N0, N1, n_t, flags=0):
    """Largest relative deviation (moments, continuum) the storage alone causes."""
    _, Q, mom, _ = oracle.run_coupled(w, nsteps, N0, N1, n_t, flags=flags)
    Qs, ms = run_coupled_stored(w, nsteps, N0, N1, n_t, flags=flags)
    return max(rel_err(ms, mom).max(), rel_err(Qs, Q).max())


def fp32_storage_bound(w, floes):
    """Per cell [ncells, 4]: how far storing the floes' radii, velocities and
    spins in FP32 (unit roundoff u = 2^-24) can move the cell values
    (rho, P_x, P_y, P_w) = (sum m, sum m u, sum m v, sum m r^2 w) / A from
    what they were before rounding: m = rho_ice h pi r^2 carries 2u,
    m u 3u, m r^2 w 5u, summed over the cell's floes."""
    u32 = 2.0 ** -24
    r = np.asarray(floes["r"], np.float64)
    m = w.rho_ice * np.asarray(w.h, np.float64) * np.pi * r * r
    I = m * r * r
    per = np.stack([2 * u32 * m, 3 * u32 * m * np.abs(floes["u"]), 3 * u32 * m * np.abs(floes["v"]),
                    5 * u32 * I * np.abs(floes["omega"])], axis=1)
    cell = np.repeat(np.arange(w.ncells), np.diff(w.start))
    out = np.zeros((w.ncells, 4))
    np.add.at(out, cell, per)
    return out / (w.Lx * w.Ly)
