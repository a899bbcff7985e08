"""FP64 oracle of the superparameterised floe DEM: TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP implementation; the two
meet only in the seeded inputs of ``fixtures``.

The DEM step, the cell statistics, the Lax-Friedrichs continuum update and the
coarse-to-fine re-synchronisation are plain C in ``dem_oracle.c`` (FP64,
compiled with gcc, no fused multiply-add); ``run_plain`` and ``run_coupled``
compose them into the plain path and the two-way coupling of Algorithm 1; the
closure network's reference (forward, backward, Adam) is numpy FP64 in
``mlp.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OCEAN_OFF = 1
FORWARD_EULER = 2
BINNED = 4
SPRING = 8          # tangential force as an incremental spring with contact history
WALLS_X = 16        # DEM: fixed walls at x = 0 and x = Lx, periodic in y only (Sec. 4.4)
DIRICHLET_X = 32    # continuum: zero state and coefficients beyond the x edges (Sec. 4.4)
HCAP = 16           # contacts remembered per floe (SPRING)
NMOM = 11
MOMENT_NAMES = ["n", "M", "Px", "Py", "L", "Ux", "Uy", "Svx", "Svy", "Sw", "Aice"]
Q_NAMES = ["rho", "Px", "Py", "Pw"]


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "dem_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Model(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("Lx", ctypes.c_double), ("Ly", ctypes.c_double),
                ("rho_ice", ctypes.c_double), ("rho_ocean", ctypes.c_double),
                ("cd", ctypes.c_double), ("E", ctypes.c_double), ("G", ctypes.c_double),
                ("mu", ctypes.c_double), ("flags", ctypes.c_int32),
                ("u0", ctypes.c_double), ("v0", ctypes.c_double), ("nmodes", ctypes.c_int32),
                ("kx", ctypes.c_void_p), ("ky", ctypes.c_void_p), ("au", ctypes.c_void_p),
                ("av", ctypes.c_void_p), ("phase", ctypes.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P, D, I32, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        MP = ctypes.POINTER(_Model)
        lib.orc_ocean_at.argtypes = [MP, D, D, P]
        lib.orc_pairs_brute.argtypes = [MP, I64, P, P, P, I64, P, P]
        lib.orc_pairs_brute.restype = I64
        lib.orc_pairs_binned.argtypes = [MP, I64, P, P, P, I64, P, P]
        lib.orc_pairs_binned.restype = I64
        lib.orc_chord.argtypes = [D, D, D]
        lib.orc_chord.restype = D
        lib.orc_moments.argtypes = [MP, P, P, P, P, P, P, P, P, P]
        lib.orc_dem_steps.argtypes = [MP, P, P, I32, P, P, P, P, P, P, P, P, D, I64, P, P, P, P]
        lib.orc_dem_steps.restype = ctypes.c_int
        lib.orc_q_from_moments.argtypes = [MP, P, P]
        lib.orc_lf_step.argtypes = [MP, P, P, D, P]
        lib.orc_lf_step.restype = D
        lib.orc_resync_cell.argtypes = [MP, I64, P, P, P, P, P, P]
        lib.orc_resync_cell.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


class Model:
    """Grid, physical constants and ocean of one workload, as the oracle sees them."""

    def __init__(self, w, flags: int = 0):
        oc = w.ocean
        self._keep = [_f64(oc.kx), _f64(oc.ky), _f64(oc.au), _f64(oc.av), _f64(oc.phase)]
        self.c = _Model(w.nx, w.ny, w.Lx, w.Ly, w.rho_ice, w.rho_ocean, w.cd, w.E, w.G, w.mu,
                        flags, oc.u0, oc.v0, oc.nmodes, *[_p(a) for a in self._keep])
        self.flags = flags
        self.nx, self.ny, self.Lx, self.Ly = w.nx, w.ny, w.Lx, w.Ly
        self.ncells = w.nx * w.ny
        self.start = np.ascontiguousarray(w.start, np.int64)

    @property
    def ref(self):
        return ctypes.byref(self.c)


class State:
    """FP64 floe state; positions are cell fractions in [0, 1)."""

    def __init__(self, xs, ys, u, v, w, th, r, h):
        self.xs, self.ys, self.u, self.v, self.w, self.th, self.r, self.h = (
            _f64(a).copy() for a in (xs, ys, u, v, w, th, r, h))
        # contact history of the tangential spring (SPRING), made by the first
        # such step: per floe HCAP partners (cell-local index, -1 none) and
        # tangential displacements
        self.hj = None
        self.hx = None

    @staticmethod
    def from_fixed(xi, yi, u, v, omega, theta, r, h) -> "State":
        """Upcast the 32-bit stored state exactly (xi / 2^32 is exact in FP64)."""
        return State(np.asarray(xi, np.float64) * 2.0 ** -32, np.asarray(yi, np.float64) * 2.0 ** -32,
                     u, v, omega, theta, r, h)

    @staticmethod
    def from_workload(w) -> "State":
        return State.from_fixed(w.xi, w.yi, w.u, w.v, w.omega, w.theta, w.r, w.h)

    def copy(self) -> "State":
        st = State(self.xs, self.ys, self.u, self.v, self.w, self.th, self.r, self.h)
        if self.hj is not None:
            st.hj, st.hx = self.hj.copy(), self.hx.copy()
        return st

    def arrays(self):
        return [self.xs, self.ys, self.u, self.v, self.w, self.th, self.r, self.h]


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's loops over cells (0: leave as is); returns the
    count in effect.  Timing only: results do not depend on it."""
    return int(_load().orc_set_threads(int(n)))


def ocean_at(model: Model, X: float, Y: float):
    out = np.zeros(3)
    _load().orc_ocean_at(model.ref, X, Y, _p(out))
    return out


def chord(rl, rj, d) -> float:
    return _load().orc_chord(rl, rj, d)


def pairs_cell(model: Model, state: State, cell: int, binned: bool = False) -> np.ndarray:
    """Contact pairs (l < j, cell-local indices) of one cell, sorted; shape [k, 2]."""
    lib = _load()
    s, e = int(model.start[cell]), int(model.start[cell + 1])
    n = e - s
    xs, ys, r = state.xs[s:e].copy(), state.ys[s:e].copy(), state.r[s:e].copy()
    fn = lib.orc_pairs_binned if binned else lib.orc_pairs_brute
    cap = max(16, 8 * n)
    while True:
        pl = np.zeros(cap, np.int32)
        pj = np.zeros(cap, np.int32)
        cnt = fn(model.ref, n, _p(xs), _p(ys), _p(r), cap, _p(pl), _p(pj))
        if cnt <= cap:
            return np.stack([pl[:cnt], pj[:cnt]], axis=1)
        cap = int(cnt)


def moments(model: Model, state: State) -> np.ndarray:
    """Cell statistics [ncells, 11] of a state (drag sums at that state)."""
    out = np.zeros((model.ncells, NMOM))
    _load().orc_moments(model.ref, _p(model.start), *[_p(a) for a in
                        (state.xs, state.ys, state.u, state.v, state.w, state.r, state.h)], _p(out))
    return out


def dem_steps(model: Model, state: State, dt: float, nsteps: int, cells=None,
              record: bool = False):
    """Advance the listed cells (default all) by nsteps fine steps in place.

    Returns (moments [nsteps, ncl, 11] of each pre-step state or None, stats)."""
    lib = _load()
    cl = None if cells is None else np.ascontiguousarray(cells, np.int32)
    ncl = model.ncells if cl is None else int(cl.size)
    mom = np.zeros((nsteps, ncl, NMOM)) if record else None
    stats = np.zeros(2, np.int64)
    spring = (model.flags & SPRING) != 0
    if spring and state.hj is None:
        state.hj = np.full((state.xs.size, HCAP), -1, np.int32)
        state.hx = np.zeros((state.xs.size, HCAP))
    rc = lib.orc_dem_steps(model.ref, _p(model.start), _p(cl), ncl, *[_p(a) for a in state.arrays()],
                           dt, nsteps, _p(mom), _p(stats), _p(state.hj) if spring else None,
                           _p(state.hx) if spring else None)
    if rc == -1:
        raise FloatingPointError("coincident floe centres")
    if rc == -2:
        raise FloatingPointError("non-finite floe state")
    if rc == -3:
        raise OverflowError(f"a floe in more than {HCAP} contacts")
    if rc == -5:
        raise FloatingPointError("a floe crossed a wall")
    if rc == -6:
        raise ValueError("the tangential spring does not run between walls")
    return mom, stats


def q_from_moments(model: Model, mom: np.ndarray) -> np.ndarray:
    Q = np.zeros((model.ncells, 4))
    _load().orc_q_from_moments(model.ref, _p(np.ascontiguousarray(mom)), _p(Q))
    return Q


def lf_step(model: Model, Q: np.ndarray, mom: np.ndarray, dT: float):
    Qn = np.zeros_like(Q)
    cfl = _load().orc_lf_step(model.ref, _p(np.ascontiguousarray(Q)), _p(np.ascontiguousarray(mom)),
                              dT, _p(Qn))
    return Qn, cfl


def resync_cell(model: Model, state: State, cell: int, target) -> None:
    s, e = int(model.start[cell]), int(model.start[cell + 1])
    sub = [a[s:e].copy() for a in (state.u, state.v, state.w, state.r)]
    t = _f64(target)
    rc = _load().orc_resync_cell(model.ref, e - s, *[_p(a) for a in sub], _p(state.h[s:e].copy()), _p(t))
    if rc:
        raise ValueError("empty cell with a nonzero target")
    state.u[s:e], state.v[s:e], state.w[s:e], state.r[s:e] = sub


def run_plain(w, nsteps: int, flags: int = 0, state: State | None = None, Q0=None):
    """The plain hot path: Q^0 from the initial statistics, then nsteps of
    (DEM step of every cell, LF step of the continuum driven by the pre-step
    statistics).  Returns (state, Q, moments of the final state, last CFL)."""
    model = Model(w, flags)
    st = State.from_workload(w) if state is None else state
    Q = q_from_moments(model, moments(model, st)) if Q0 is None else np.array(Q0, np.float64)
    mom, _ = dem_steps(model, st, w.dt, nsteps, record=True)
    cfl = 0.0
    for k in range(nsteps):
        Q, cfl = lf_step(model, Q, mom[k], w.dt)
    return st, Q, moments(model, st), cfl


def run_coupled(w, nsteps: int, N0: int, N1: int, n_t: int, flags: int = 0, state: State | None = None):
    """Two-way coupling of the coarse model and the cell DEMs (Algorithm 1;
    coarse step Sec. 3.2, coarse-to-fine update Sec. 3.3).

    The coarse state starts from the statistics of the initial floes.  Fine
    step j (j = 1 .. nsteps) advances every cell DEM by dt and adds the
    statistics of its pre-step state to the window's data.  When j is a
    multiple of N0 the coarse model advances by dT = N0 dt in N1 Lax-Friedrichs
    sub-steps of dT / N1, driven by the window's mean statistics, and the DEM
    cell values (rho, P, P_w) of the state reached are kept as the start values
    X0 of the next coarse step.  Otherwise, from the second coarse step on,
    when r = j mod N0 is a multiple of n_t, every cell with floes is
    re-synchronised to X0 + (r / N0) (Q - X0): the increments toward the latest
    coarse solution Q grow in proportion to the elapsed part of the coarse step.
    With N0 = N1 = 1 this is run_plain.  Returns (state, Q, moments of the final
    state, largest CFL number)."""
    if min(N0, N1, n_t) < 1:
        raise ValueError("N0, N1 and n_t must be positive")
    model = Model(w, flags)
    st = State.from_workload(w) if state is None else state
    Q = q_from_moments(model, moments(model, st))
    counts = np.diff(model.start)
    window = np.zeros((model.ncells, NMOM))
    x0 = None
    dT = N0 * w.dt
    cfl = 0.0
    for j in range(1, nsteps + 1):
        mom, _ = dem_steps(model, st, w.dt, 1, record=True)
        window += mom[0]
        r = j % N0
        if r == 0:
            mean = window / N0
            for _ in range(N1):
                Q, c = lf_step(model, Q, mean, dT / N1)
                cfl = max(cfl, c)
            window[:] = 0.0
            x0 = q_from_moments(model, moments(model, st))
        elif j > N0 and r % n_t == 0:
            f = r / N0
            for cell in np.flatnonzero(counts):
                resync_cell(model, st, int(cell), x0[cell] + f * (Q[cell] - x0[cell]))
    return st, Q, moments(model, st), cfl


def run_global(w, nsteps: int, flags: int = 0, state: State | None = None):
    """The global DEM of the paper's error study (Sec. 4: one DEM over the whole
    periodic domain, floes free to cross coarse cells, every pair a potential
    contact): the cell DEM of a workload with a single cell spanning the domain.
    Returns (state, stats)."""
    if w.nx != 1 or w.ny != 1:
        raise ValueError("a global workload has one cell spanning the domain")
    model = Model(w, flags)
    st = State.from_workload(w) if state is None else state
    _, stats = dem_steps(model, st, w.dt, nsteps)
    return st, stats


def coarse_moments(w, state: State, nxc: int, nyc: int, flags: int = 0) -> np.ndarray:
    """Statistics [nyc * nxc, 11] of a global state (positions as fractions of
    the domain) on a coarse grid of nxc x nyc cells: each floe counts in the
    cell that holds its centre (eq. meang over the cell's floes)."""
    cx = np.minimum((state.xs * nxc).astype(np.int64), nxc - 1)
    cy = np.minimum((state.ys * nyc).astype(np.int64), nyc - 1)
    cell = cy * nxc + cx
    order = np.argsort(cell, kind="stable")
    counts = np.bincount(cell, minlength=nxc * nyc)
    sub = Model.__new__(Model)
    oc = w.ocean
    sub._keep = [_f64(oc.kx), _f64(oc.ky), _f64(oc.au), _f64(oc.av), _f64(oc.phase)]
    sub.c = _Model(nxc, nyc, w.Lx / nxc, w.Ly / nyc, w.rho_ice, w.rho_ocean, w.cd, w.E, w.G, w.mu,
                   flags, oc.u0, oc.v0, oc.nmodes, *[_p(a) for a in sub._keep])
    sub.nx, sub.ny, sub.Lx, sub.Ly = nxc, nyc, w.Lx / nxc, w.Ly / nyc
    sub.ncells = nxc * nyc
    sub.start = np.zeros(sub.ncells + 1, np.int64)
    np.cumsum(counts, out=sub.start[1:])
    xs = state.xs[order] * nxc - cx[order]
    ys = state.ys[order] * nyc - cy[order]
    part = State(xs, ys, state.u[order], state.v[order], state.w[order], state.th[order], state.r[order],
                 state.h[order])
    return moments(sub, part)
