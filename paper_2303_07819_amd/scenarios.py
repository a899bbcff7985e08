"""The paper's error study (Sec. 4.1-4.4) on the GPU: the superparameterised
model (cell DEMs coupled to the coarse model at the cadence of Algorithm 1)
against the global DEM of the same floes, on several coarse grids.  In
scenario 4.4 the floes are driven into a fixed wall: the global DEM has walls
at x = 0 and x = 4 (periodic in y) and the coarse model a zero Dirichlet
boundary in x (SP_WALL_X); the cell DEMs stay doubly periodic.

Both models run in the library; this module only drives them and measures
the distance of their coarse fields: the L^2 norm over the domain, the
integral taken as a sum over the coarse cells (Sec. 4.1),
||f||_{L^2} = sqrt(sum_cells f^2 dX dY).  The superparameterised model's
fields are its coarse state: concentration rho / (rho_ice h) (unit thickness
in the scenarios) and velocity P_x / rho; the global DEM's are its coarse-grid
statistics: concentration A_ice / (dX dY) and velocity P_x / M.
"""
from __future__ import annotations

import time

import numpy as np

import fixtures
from . import GlobalDEM, Sim, MOMENTS_CONTINUUM, SP_WALL_X

# statistics slots (order of SP_MOMENTS_DEM)
M_MASS, M_PX, M_AICE = 1, 2, 10


def coarse_fields_global(mom: np.ndarray, area: float):
    """(concentration, x velocity) of the global DEM's coarse statistics."""
    conc = mom[:, M_AICE] / area
    with np.errstate(invalid="ignore", divide="ignore"):
        vx = np.where(mom[:, M_MASS] > 0, mom[:, M_PX] / np.where(mom[:, M_MASS] > 0, mom[:, M_MASS], 1.0), 0.0)
    return conc, vx


def coarse_fields_ms(Q: np.ndarray, rho_ice: float):
    """(concentration, x velocity) of the coarse state Q = (rho, P_x, P_y, P_w)."""
    conc = Q[:, 0] / rho_ice
    with np.errstate(invalid="ignore", divide="ignore"):
        vx = np.where(Q[:, 0] > 0, Q[:, 1] / np.where(Q[:, 0] > 0, Q[:, 0], 1.0), 0.0)
    return conc, vx


def l2(f: np.ndarray, dX: float, dY: float) -> float:
    return float(np.sqrt(np.sum(f * f) * dX * dY))


def study(k: int, grids=((24, 12), (48, 24), (96, 48)), times=(0.2, 1.0), N0: int = 100, N1: int = 1,
          n_t: int = 10, nfx: int = 480, nfy: int = 240, stream=None) -> dict:
    """Scenario 4.k (k = 1 .. 4): L^2 errors of concentration and x velocity of the
    superparameterised model against the global DEM at each time on each grid,
    and the convergence orders between successive grids."""
    wg = fixtures.scenario_global(k, nfx=nfx, nfy=nfy)
    flags = SP_WALL_X if k == 4 else 0
    steps = [int(round(T / wg.dt)) for T in times]
    if any(s % N0 for s in steps):
        raise ValueError("every time must be a whole number of coarse steps")
    out = {"scenario": f"4.{k}", "floes": wg.nfloes, "domain": [wg.Lx, wg.Ly], "dt": wg.dt, "N0": N0, "N1": N1,
           "n_t": n_t, "times": list(times), "grids": [list(g) for g in grids]}
    # the global DEM once, read on every grid at every time
    truth = {}
    t0 = time.perf_counter()
    with GlobalDEM.from_workload(wg, flags=flags, stream=stream) as g:
        done = 0
        for T, s in zip(times, steps):
            g.step(wg.dt, s - done)
            done = s
            for nxc, nyc in grids:
                truth[(T, nxc)] = g.coarse_moments(nxc, nyc)
        gs = g.stats()
    out["global_dem"] = {"steps": steps[-1], "seconds": time.perf_counter() - t0, "contacts": gs["contacts"],
                         "bins": list(gs["bins"])}
    errs = {"conc": {}, "vx": {}}
    for nxc, nyc in grids:
        w = fixtures.split_cells(wg, nxc, nyc)
        dX, dY = w.Lx, w.Ly
        with Sim.from_workload(w, flags=flags, stream=stream) as sim:
            sim.set_coupling(N0, N1, n_t)
            done = 0
            for T, s in zip(times, steps):
                sim.step(w.dt, s - done)
                done = s
                Q = sim.read_moments(MOMENTS_CONTINUUM)
                c_ms, v_ms = coarse_fields_ms(Q, w.rho_ice)
                c_dem, v_dem = coarse_fields_global(truth[(T, nxc)], dX * dY)
                errs["conc"].setdefault(str(T), []).append(l2(c_ms - c_dem, dX, dY))
                errs["vx"].setdefault(str(T), []).append(l2(v_ms - v_dem, dX, dY))
            cp = sim.coupling()
            out.setdefault("coupling", []).append({"grid": [nxc, nyc], "nudges": cp["nudges"],
                                                   "replans": cp["replans"], "clamped": cp["clamped"]})
    out["l2"] = errs
    dx = np.array([wg.Lx / g[0] for g in grids])
    out["dX"] = dx.tolist()
    orders = {}
    for q, per_t in errs.items():
        orders[q] = {}
        for T, e in per_t.items():
            e = np.asarray(e)
            orders[q][T] = (np.log(e[:-1] / e[1:]) / np.log(dx[:-1] / dx[1:])).tolist()
    out["order"] = orders
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="error study of Sec. 4.1-4.4 against the global DEM")
    ap.add_argument("scenarios", type=int, nargs="*", default=[1, 2, 3, 4])
    ap.add_argument("--times", type=float, nargs="+", default=[0.2, 1.0])
    args = ap.parse_args()
    for k in args.scenarios:
        print(json.dumps(study(k, times=tuple(args.times))), flush=True)
