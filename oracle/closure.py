"""Reference of the learned closure's reduced DEM, base update and network
inputs: TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``).

The closure is this build's, not the paper's: the paper closes the coarse
equations only through the cell DEMs (Sec. 2.3, Sec. 3.1).  A closure cell
replaces its DEM by a "reduced DEM": the cell's floes taken as one body under
the ocean drag laws of Sec. 2.1 (drag force alpha du |du| with
alpha = C_d rho_o pi r^2, drag torque beta dW |dW| with beta = C_d rho_o pi r^5,
dW the spin relative to half the ocean curl).  For one floe in a steady
current these laws integrate in closed form: with k = alpha / m,
du(t) = du0 / (1 + k |du0| (t - t0)), and with k_W = beta / I,
dW(t) = dW0 / (1 + k_W |dW0| (t - t0)).  The reduced DEM applies the same
closed forms to the cell as a whole, with the cell's aggregate coefficients
k_v = C_d rho_o sum pi r^2 / sum m and k_w / r2m, k_w = C_d rho_o sum pi r^5 /
sum m, r2m = sum m r^2 / sum m (so that k_w / r2m = sum beta / sum I), starting
from the cell's mean velocity U / n (eq. meang) and mean spin L / (M r2m), both
relative to the ocean current and half-curl at the cell centre.  Its
statistics: the coefficient <v> = u_o - du and the sources per unit area
rho_f k_v |du| du and rho_f k_w |dW| dW, rho_f = sum m / A (the summed drag of
the one-body cell, Sec. 2.3 sources).  The base update is the oracle's
continuum step (Sec. 3.2) driven by those statistics in every cell.

Everything is numpy FP64 from the floes as stored (FP32 radii and
thicknesses upcast exactly).  Pinned in tests/test_oracle_closure_pins.py
against the oracle's cell DEM (single floe, identical non-touching floes:
first-order agreement in dt), the single-floe closed form, a uniform state's
base update and a hand-built 3 x 3 feature lattice.
"""
from __future__ import annotations

import numpy as np

from . import NMOM, lf_step, ocean_at

# statistics columns (order of the cell DEM's statistics)
_N, _M, _PX, _PY, _L, _UX, _UY, _SVX, _SVY, _SW = range(10)


def cell_static(w) -> np.ndarray:
    """Per cell [ncells, 6]: k_v, k_w, r2m, rho_f, A_ice / A, mean h."""
    out = np.zeros((w.ncells, 6))
    area = w.Lx * w.Ly
    cdr = w.cd * w.rho_ocean
    for c in range(w.ncells):
        s, e = int(w.start[c]), int(w.start[c + 1])
        if e == s:
            continue
        r = np.asarray(w.r[s:e], np.float64)
        h = np.asarray(w.h[s:e], np.float64)
        m = w.rho_ice * h * np.pi * r ** 2                  # Sec. 2.1 mass with thickness
        msum = m.sum()
        out[c, 0] = cdr * np.sum(np.pi * r ** 2) / msum     # sum alpha / sum m
        out[c, 1] = cdr * np.sum(np.pi * r ** 5) / msum     # sum beta / sum m
        out[c, 2] = np.sum(m * r ** 2) / msum               # sum I / sum m (I = m r^2)
        out[c, 3] = msum / area
        out[c, 4] = np.sum(np.pi * r ** 2) / area
        out[c, 5] = h.mean()
    return out


def ocean_centres(w, model) -> np.ndarray:
    """Ocean (u_o, v_o, curl) at every cell centre [ncells, 3]."""
    return np.array([ocean_at(model, (c % w.nx + 0.5) * w.Lx, (c // w.nx + 0.5) * w.Ly)
                     for c in range(w.ncells)])


def reduced_init(mom, static, oce, t0) -> np.ndarray:
    """Reduced DEMs [ncells, 4] = (du0_x, du0_y, dW0, t0) from cell statistics
    [ncells, 11]: velocity relative to the ocean u_o - U / n, spin relative to
    half the curl curl / 2 - L / (M r2m); zero in a cell without floes."""
    mom = np.asarray(mom, np.float64)
    n, M, L = mom[:, _N], mom[:, _M], mom[:, _L]
    has = n > 0
    nn = np.where(has, n, 1.0)
    U = np.where(has, mom[:, _UX] / nn, 0.0)
    V = np.where(has, mom[:, _UY] / nn, 0.0)
    I = M * static[:, 2]
    ok = (M > 0) & (static[:, 2] > 0)
    W = np.where(ok, L / np.where(ok, I, 1.0), 0.0)
    out = np.zeros((mom.shape[0], 4))
    out[:, 0] = oce[:, 0] - U
    out[:, 1] = oce[:, 1] - V
    out[:, 2] = 0.5 * oce[:, 2] - W
    out[:, 3] = float(t0)
    return out


def reduced_rel(red, static, t):
    """(du_x, du_y, dW) of every reduced DEM at time t (closed-form quadratic
    drag relaxation from its start time; no change before it)."""
    tau = np.maximum(t - red[:, 3], 0.0)
    du0 = np.sqrt(red[:, 0] ** 2 + red[:, 1] ** 2)
    shrink_v = 1.0 / (1.0 + static[:, 0] * du0 * tau)
    has = static[:, 2] > 0
    k_spin = np.where(has, static[:, 1] / np.where(has, static[:, 2], 1.0), 0.0)   # sum beta / sum I
    shrink_w = 1.0 / (1.0 + k_spin * np.abs(red[:, 2]) * tau)
    return red[:, 0] * shrink_v, red[:, 1] * shrink_v, red[:, 2] * shrink_w


def reduced_moments(red, static, oce, t, area) -> np.ndarray:
    """Statistics rows [ncells, 11] of the reduced DEMs at time t, laid out as
    the cell DEM's, for the continuum step: n = 1 (so that U / n is the
    coefficient <v> = u_o - du) and the drag sums S = A x (sources per unit
    area).  Other columns zero (the continuum step does not read them)."""
    dux, duy, dw = reduced_rel(red, static, t)
    speed = np.sqrt(dux ** 2 + duy ** 2)
    out = np.zeros((red.shape[0], NMOM))
    out[:, _N] = 1.0
    out[:, _UX] = oce[:, 0] - dux
    out[:, _UY] = oce[:, 1] - duy
    out[:, _SVX] = area * static[:, 3] * static[:, 0] * speed * dux
    out[:, _SVY] = area * static[:, 3] * static[:, 0] * speed * duy
    out[:, _SW] = area * static[:, 3] * static[:, 1] * np.abs(dw) * dw
    return out


def base_update(w, model, Q, dt, red, t, static, oce) -> np.ndarray:
    """The continuum after one step of size dt (Sec. 3.2) driven in every cell
    by its reduced DEM at time t ([ncells, 4])."""
    return lf_step(model, Q, reduced_moments(red, static, oce, t, w.Lx * w.Ly), dt)[0]


def features(w, Qsrc, cells, red, t, static, oce) -> np.ndarray:
    """The 45 closure inputs of the listed cells: the continuum state
    (rho, P_x, P_y, P_w) of the 3 x 3 neighbourhood row by row from the
    south-west (periodic grid), the ocean current and curl at the cell centre,
    A_ice / A, mean h and r2m, and the reduced DEM's (du_x, du_y, dW) at t."""
    dux, duy, dw = reduced_rel(red, static, t)
    rows = []
    for c in cells:
        ix, iy = c % w.nx, c // w.nx
        x = []
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb = ((iy + dy) % w.ny) * w.nx + (ix + dx) % w.nx
                x.extend(Qsrc[nb])
        x.extend(oce[c])
        x.extend([static[c, 4], static[c, 5], static[c, 2]])
        x.extend([dux[c], duy[c], dw[c]])
        rows.append(x)
    return np.array(rows, np.float64).reshape(len(rows), 45)
