"""Reference of the closure's coarse-only update, composed from the oracle's
Lax-Friedrichs step: transport with every coefficient <v> = P / rho (0 at or
below 1 kg/m^2) and no sources, then mean-field drag of the transported state:
the cell's ice moving with P / rho and spinning at P_w / (rho r2m) relaxes over
the step towards the ocean current and half-curl at the cell centre by the
closed form w0 / (1 + k |w0| dt) of one floe's quadratic drag (k = kappa_v,
resp. kappa_w / r2m)."""
import numpy as np

import oracle

RHO_COEF_MIN = 1.0


def mean_field_coefficients(w):
    """Per cell: kappa_v = Cd rho_o sum pi r^2 / sum m, kappa_w = Cd rho_o sum pi r^5 / sum m,
    r2m = sum m r^2 / sum m (FP64 from the stored radii and thicknesses)."""
    out = np.zeros((w.ncells, 3))
    for c in range(w.ncells):
        r = w.r[w.start[c]:w.start[c + 1]].astype(np.float64)
        h = w.h[w.start[c]:w.start[c + 1]].astype(np.float64)
        if r.size:
            m = w.rho_ice * h * np.pi * r * r
            k = w.cd * w.rho_ocean
            out[c] = [k * np.sum(np.pi * r * r) / m.sum(), k * np.sum(np.pi * r ** 5) / m.sum(),
                      np.sum(m * r * r) / m.sum()]
    return out


def transport(m, Q, dt):
    """The oracle's continuum step without sources, every coefficient <v> = P / rho."""
    mom = np.zeros((Q.shape[0], oracle.NMOM))
    mom[:, 0] = 1.0
    pos = Q[:, 0] > RHO_COEF_MIN
    mom[pos, 5] = Q[pos, 1] / Q[pos, 0]
    mom[pos, 6] = Q[pos, 2] / Q[pos, 0]
    return oracle.lf_step(m, Q, mom, dt)[0]


def relax(w, m, Qs, dt, mf=None):
    """Mean-field drag of a transported state, cell by cell."""
    mf = mean_field_coefficients(w) if mf is None else mf
    out = Qs.copy()
    for c in range(Qs.shape[0]):
        ix, iy = c % w.nx, c // w.nx
        uo, vo, zeta = oracle.ocean_at(m, (ix + 0.5) * w.Lx, (iy + 0.5) * w.Ly)
        moving = Qs[c, 0] > RHO_COEF_MIN
        rho = max(Qs[c, 0], 0.0)
        u = Qs[c, 1] / Qs[c, 0] if moving else 0.0
        v = Qs[c, 2] / Qs[c, 0] if moving else 0.0
        om = Qs[c, 3] / (Qs[c, 0] * mf[c, 2]) if moving and mf[c, 2] > 0 else 0.0
        du, dv = uo - u, vo - v
        fv = dt * mf[c, 0] * np.hypot(du, dv)
        dW = 0.5 * zeta - om
        fw = dt * mf[c, 1] / mf[c, 2] * abs(dW) if mf[c, 2] > 0 else 0.0
        out[c, 1] += rho * du * fv / (1.0 + fv)
        out[c, 2] += rho * dv * fv / (1.0 + fv)
        out[c, 3] += rho * mf[c, 2] * dW * fw / (1.0 + fw)
    return out


def base_update(w, m, Q, dt, mf=None):
    """Q after the coarse-only update of every cell ([ncells, 4])."""
    return relax(w, m, transport(m, Q, dt), dt, mf)
