"""Reference of the closure's reduced DEM and base update, composed from the
oracle's Lax-Friedrichs step (test code).

Reduced DEM of a cell: the cell's floes as one body under the quadratic drag
laws, taken from the floes at t0 (mean velocity sum v / n, mean spin
L / (M r2m)); its velocity and spin relative to the ocean current and half-curl
at the cell centre relax in closed form, du(t) = du0 / (1 + k_v |du0| (t - t0))
and dW(t) = dW0 / (1 + (k_w / r2m) |dW0| (t - t0)).  Its statistics: the
coefficient u_o - du and the sources per unit area rho_f k_v |du| du and
rho_f k_w |dW| dW.  The base update is the oracle's continuum step with every
cell's statistics taken from its reduced DEM."""
import numpy as np

import oracle


def cell_static(w):
    """Per cell: k_v, k_w, r2m, rho_f, A_ice / A, mean h (FP64 from the stored floes)."""
    out = np.zeros((w.ncells, 6))
    A = w.Lx * w.Ly
    k = w.cd * w.rho_ocean
    for c in range(w.ncells):
        r = w.r[w.start[c]:w.start[c + 1]].astype(np.float64)
        h = w.h[w.start[c]:w.start[c + 1]].astype(np.float64)
        if r.size:
            m = w.rho_ice * h * np.pi * r * r
            out[c] = [k * np.sum(np.pi * r * r) / m.sum(), k * np.sum(np.pi * r ** 5) / m.sum(),
                      np.sum(m * r * r) / m.sum(), m.sum() / A, np.sum(np.pi * r * r) / A, h.mean()]
    return out


def ocean_centres(w, m):
    return np.array([oracle.ocean_at(m, (c % w.nx + 0.5) * w.Lx, (c // w.nx + 0.5) * w.Ly)
                     for c in range(w.ncells)])


def reduced_init(mom, static, oce, t0):
    """Reduced DEMs [ncells, 4] = (du0_x, du0_y, dW0, t0) from oracle statistics [ncells, 11]."""
    n, M, L = mom[:, 0], mom[:, 1], mom[:, 4]
    U = np.where(n > 0, mom[:, 5] / np.where(n > 0, n, 1), 0.0)
    V = np.where(n > 0, mom[:, 6] / np.where(n > 0, n, 1), 0.0)
    ok = (M > 0) & (static[:, 2] > 0)
    W = np.where(ok, L / np.where(ok, M * static[:, 2], 1), 0.0)
    return np.stack([oce[:, 0] - U, oce[:, 1] - V, 0.5 * oce[:, 2] - W, np.full(n.shape, float(t0))], axis=1)


def reduced_rel(red, static, t):
    tr = np.maximum(t - red[:, 3], 0.0)
    fu = 1.0 / (1.0 + static[:, 0] * np.hypot(red[:, 0], red[:, 1]) * tr)
    kw = np.where(static[:, 2] > 0, static[:, 1] / np.where(static[:, 2] > 0, static[:, 2], 1), 0.0)
    return red[:, 0] * fu, red[:, 1] * fu, red[:, 2] / (1.0 + kw * np.abs(red[:, 2]) * tr)


def reduced_moments(red, static, oce, t, A):
    """Statistics rows for the oracle's continuum step: n = 1, U = <v>, S = A s."""
    dux, duy, dw = reduced_rel(red, static, t)
    sp = np.hypot(dux, duy)
    mom = np.zeros((red.shape[0], oracle.NMOM))
    mom[:, 0] = 1.0
    mom[:, 5] = oce[:, 0] - dux
    mom[:, 6] = oce[:, 1] - duy
    mom[:, 7] = A * static[:, 3] * static[:, 0] * sp * dux
    mom[:, 8] = A * static[:, 3] * static[:, 0] * sp * duy
    mom[:, 9] = A * static[:, 3] * static[:, 1] * np.abs(dw) * dw
    return mom


def base_update(w, m, Q, dt, red, t, static, oce):
    """Q after the base update of every cell ([ncells, 4])."""
    return oracle.lf_step(m, Q, reduced_moments(red, static, oce, t, w.Lx * w.Ly), dt)[0]


def features(w, Qsrc, cells, red, t, static, oce):
    """The 45 closure inputs of the listed cells."""
    dux, duy, dw = reduced_rel(red, static, t)
    x = np.zeros((len(cells), 45))
    for i, c in enumerate(cells):
        ix, iy = c % w.nx, c // w.nx
        k = 0
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nb = ((iy + dy) % w.ny) * w.nx + (ix + dx) % w.nx
                x[i, k:k + 4] = Qsrc[nb]
                k += 4
        x[i, 36:39] = oce[c]
        x[i, 39:42] = [static[c, 4], static[c, 5], static[c, 2]]
        x[i, 42:45] = [dux[c], duy[c], dw[c]]
    return x
