"""spdem: superparameterised sea-ice floe DEM on MI355X.

Thin Python binding over the C ABI of ``libspdem.so`` (declared in
``include/spdem.h``): argument marshalling only, every step of the path runs in
the HIP kernels.  There is no CPU fallback: importing the binding without the
built library raises.

Method: Deng, Stechmann & Chen, "Particle-continuum multiscale modeling of sea
ice floes" (one doubly periodic disk-floe DEM per coarse cell, Sec. 3.1; DEM of
Sec. 2.1; moment equations of Sec. 2.3 advanced by Lax-Friedrichs, Sec. 3.2).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspdem.so")

SP_OCEAN_OFF = 1
SP_FORWARD_EULER = 2
SP_NO_CONTINUUM = 4
SP_TANGENTIAL_SPRING = 8     # tangential force as an incremental spring with contact history
SP_WALL_X = 16               # walls in x: Dirichlet coarse boundary (Sim), floe-wall contact (GlobalDEM)
SP_SPRING_CAP = 8            # contacts remembered per floe (SP_TANGENTIAL_SPRING)
SP_MAX_COUPLING = 65536
SP_MAX_STEP_BLOCK = 1024
SCHED_AUTO, SCHED_ALLPAIRS, SCHED_BINNED = 0, 1, 2
MOMENTS_DEM, MOMENTS_CONTINUUM = 0, 1
NMOM = 11
TEND_FULL, TEND_RESIDUAL = 0, 1
STATUS = {0: "SP_OK", -1: "SP_EINVAL", -2: "SP_ENOMEM", -3: "SP_EDEVICE", -4: "SP_ECFL",
          -5: "SP_EOVERLAP", -6: "SP_ENAN", -7: "SP_ESTATE", -8: "SP_ECAPACITY",
          -9: "SP_EWALL"}

EXPORTED = ["sp_create", "sp_destroy", "sp_last_error", "sp_set_ocean", "sp_set_floes",
            "sp_set_floes_device", "sp_step", "sp_synchronize", "sp_read_moments", "sp_read_floes",
            "sp_read_pairs", "sp_get_stats", "sp_get_schedule", "sp_profile_steps",
            "sp_get_batching", "sp_set_batching", "sp_autotune", "sp_set_graph_chunk",
            "sp_mlp_create", "sp_mlp_destroy", "sp_mlp_last_error", "sp_mlp_set_params", "sp_mlp_get_params",
            "sp_mlp_set_norm", "sp_mlp_get_norm", "sp_mlp_fit_norm", "sp_mlp_forward", "sp_mlp_gradient",
            "sp_mlp_train_step", "sp_mlp_train_epoch", "sp_mlp_set_input_noise", "sp_closure_features", "sp_closure_sample",
            "sp_resync_cells", "sp_hybrid_set", "sp_step_hybrid", "sp_hybrid_stats", "sp_set_coupling",
            "sp_get_coupling", "sp_gdem_create", "sp_gdem_destroy", "sp_gdem_last_error", "sp_gdem_set_ocean",
            "sp_gdem_set_floes", "sp_gdem_step", "sp_gdem_read_floes", "sp_gdem_coarse_moments",
            "sp_gdem_get_stats", "sp_set_step_block", "sp_get_step_block", "sp_get_work", "sp_save", "sp_load", "sp_get_size", "sp_read_moments_noalloc", "sp_get_block_waves",
            "sp_gdem_read_order"]
NUM_BUCKETS = 5
MLP_NPARAMS, MLP_IN, MLP_OUT = 39428, 45, 4


class SpdemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("cell_lx", ctypes.c_double), ("cell_ly", ctypes.c_double),
                ("rho_ice", ctypes.c_double), ("rho_ocean", ctypes.c_double),
                ("cd", ctypes.c_double), ("E", ctypes.c_double), ("G", ctypes.c_double),
                ("mu", ctypes.c_double), ("flags", ctypes.c_uint32), ("schedule", ctypes.c_int32)]


class _GParams(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_double), ("ly", ctypes.c_double), ("rho_ice", ctypes.c_double),
                ("rho_ocean", ctypes.c_double), ("cd", ctypes.c_double), ("E", ctypes.c_double),
                ("G", ctypes.c_double), ("mu", ctypes.c_double), ("flags", ctypes.c_uint32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libspdem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2303_07819_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.sp_create.argtypes = [ctypes.POINTER(_Params), P, ctypes.POINTER(P)]
    lib.sp_destroy.argtypes = [P]
    lib.sp_destroy.restype = None
    lib.sp_last_error.argtypes = [P]
    lib.sp_last_error.restype = ctypes.c_char_p
    lib.sp_set_ocean.argtypes = [P, D, D, I32, P, P, P, P, P]
    lib.sp_set_floes.argtypes = [P, I64, P, P, P, P, P, P, P, P, P]
    lib.sp_set_floes_device.argtypes = [P, I64, P, P, P, P, P, P, P, P, P]
    lib.sp_step.argtypes = [P, D, I64]
    lib.sp_synchronize.argtypes = [P]
    lib.sp_read_moments.argtypes = [P, I32, P]
    lib.sp_read_moments_noalloc.argtypes = [P, I32, P]
    lib.sp_read_floes.argtypes = [P, P, P, P, P, P, P, P]
    lib.sp_read_pairs.argtypes = [P, I64, P, P, ctypes.POINTER(I64)]
    lib.sp_get_stats.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(D)]
    lib.sp_profile_steps.argtypes = [P, D, I64, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.sp_get_batching.argtypes = [P, P, P, P]
    lib.sp_set_batching.argtypes = [P, P, P]
    lib.sp_autotune.argtypes = [P, D, I32, ctypes.POINTER(D)]
    lib.sp_get_block_waves.argtypes = [P, P]
    lib.sp_set_graph_chunk.argtypes = [P, I32]
    lib.sp_set_step_block.argtypes = [P, I32]
    lib.sp_get_step_block.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.sp_get_work.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.sp_set_coupling.argtypes = [P, I32, I32, I32]
    lib.sp_save.argtypes = [P, ctypes.c_char_p]
    lib.sp_load.argtypes = [P, ctypes.c_char_p]
    lib.sp_get_size.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I32)]
    PI32, PI64 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    lib.sp_get_coupling.argtypes = [P, PI32, PI32, PI32, PI64, PI64, PI64, PI64]
    F = ctypes.POINTER(ctypes.c_float)
    lib.sp_mlp_create.argtypes = [P, ctypes.POINTER(P)]
    lib.sp_mlp_destroy.argtypes = [P]
    lib.sp_mlp_last_error.argtypes = [P]
    lib.sp_mlp_set_params.argtypes = [P, P]
    lib.sp_mlp_get_params.argtypes = [P, P]
    lib.sp_mlp_set_norm.argtypes = [P, P, P, P, P]
    lib.sp_mlp_get_norm.argtypes = [P, P, P, P, P]
    lib.sp_mlp_fit_norm.argtypes = [P, P, P, I64]
    lib.sp_mlp_forward.argtypes = [P, P, I64, P]
    lib.sp_mlp_gradient.argtypes = [P, P, P, I32, P, F]
    lib.sp_mlp_train_step.argtypes = [P, P, P, P, I32, ctypes.c_float, F]
    lib.sp_mlp_train_epoch.argtypes = [P, P, P, P, I64, I32, ctypes.c_float, F]
    lib.sp_mlp_set_input_noise.argtypes = [P, I32, F, ctypes.c_uint64]
    lib.sp_closure_features.argtypes = [P, P]
    lib.sp_closure_sample.argtypes = [P, D, I32, P, P]
    lib.sp_get_schedule.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.sp_resync_cells.argtypes = [P, I32, P, P, ctypes.POINTER(I32)]
    lib.sp_hybrid_set.argtypes = [P, P, P, I32, I32, D, I32, D]
    lib.sp_step_hybrid.argtypes = [P, D, I64]
    lib.sp_hybrid_stats.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I64),
                                    ctypes.POINTER(I64)]
    lib.sp_gdem_create.argtypes = [ctypes.POINTER(_GParams), P, ctypes.POINTER(P)]
    lib.sp_gdem_destroy.argtypes = [P]
    lib.sp_gdem_last_error.argtypes = [P]
    lib.sp_gdem_set_ocean.argtypes = [P, D, D, I32, P, P, P, P, P]
    lib.sp_gdem_set_floes.argtypes = [P, I64, P, P, P, P, P, P, P, P]
    lib.sp_gdem_step.argtypes = [P, D, I64]
    lib.sp_gdem_read_floes.argtypes = [P, P, P, P, P, P, P, P]
    lib.sp_gdem_coarse_moments.argtypes = [P, I32, I32, P]
    lib.sp_gdem_get_stats.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I32),
                                      ctypes.POINTER(I32)]
    lib.sp_gdem_read_order.argtypes = [P, P, P, ctypes.POINTER(I64)]
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name not in ("sp_destroy", "sp_last_error", "sp_mlp_destroy", "sp_mlp_last_error", "sp_gdem_destroy",
                        "sp_gdem_last_error"):
            fn.restype = ctypes.c_int
    lib.sp_mlp_destroy.restype = None
    lib.sp_mlp_last_error.restype = ctypes.c_char_p
    lib.sp_gdem_destroy.restype = None
    lib.sp_gdem_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _p(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(int(a.data_ptr()))    # torch tensor on the device


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dt)


class Sim:
    """One superparameterised DEM (one context of the C library)."""

    def __init__(self, nx, ny, cell_lx, cell_ly, rho_ice, rho_ocean, cd, E, G, mu,
                 flags: int = 0, schedule: int = SCHED_AUTO, stream=None):
        self._lib = load_library()
        self.nx, self.ny = int(nx), int(ny)
        self.ncells = self.nx * self.ny
        self.n = 0
        prm = _Params(self.nx, self.ny, cell_lx, cell_ly, rho_ice, rho_ocean, cd, E, G, mu,
                      flags, schedule)
        h = ctypes.c_void_p()
        st = self._lib.sp_create(ctypes.byref(prm), None if stream is None else ctypes.c_void_p(stream),
                                 ctypes.byref(h))
        if st != 0:
            raise SpdemError(st, "sp_create failed")
        self._h = h

    @classmethod
    def from_workload(cls, w, flags: int = 0, schedule: int = SCHED_AUTO, stream=None) -> "Sim":
        """Context for a workload object (grid, constants, ocean and floes)."""
        s = cls(w.nx, w.ny, w.Lx, w.Ly, w.rho_ice, w.rho_ocean, w.cd, w.E, w.G, w.mu,
                flags, schedule, stream)
        oc = w.ocean
        s.set_ocean(oc.u0, oc.v0, oc.kx, oc.ky, oc.au, oc.av, oc.phase)
        s.set_floes(w.counts, w.xi, w.yi, w.u, w.v, w.omega, w.theta, w.r, w.h)
        return s

    def _check(self, st):
        if st != 0:
            raise SpdemError(st, self._lib.sp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ ABI
    def set_ocean(self, u0, v0, kx, ky, au, av, phase):
        arrs = [_c(a, np.float64) for a in (kx, ky, au, av, phase)]
        self._check(self._lib.sp_set_ocean(self._h, float(u0), float(v0), int(arrs[0].size),
                                           *[_p(a) for a in arrs]))

    def set_floes(self, counts, xi, yi, u, v, omega, theta, r, h):
        counts = _c(counts, np.int32)
        arrs = [_c(xi, np.uint32), _c(yi, np.uint32)] + [_c(a, np.float32) for a in (u, v, omega, theta, r, h)]
        self.n = int(arrs[0].size)
        self._check(self._lib.sp_set_floes(self._h, self.n, _p(counts), *[_p(a) for a in arrs]))

    def set_floes_device(self, counts, xi, yi, u, v, omega, theta, r, h):
        """Device tensors (torch, contiguous, 4-byte elements) are copied on the stream."""
        counts = _c(counts, np.int32)
        self.n = int(xi.numel())
        self._check(self._lib.sp_set_floes_device(self._h, self.n, _p(counts),
                                                  *[_p(a) for a in (xi, yi, u, v, omega, theta, r, h)]))

    def step(self, dt: float, nsteps: int = 1):
        self._check(self._lib.sp_step(self._h, float(dt), int(nsteps)))

    def save(self, path: str):
        """Write the simulation to a file (sp_save)."""
        self._check(self._lib.sp_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """Restore a simulation saved by save() with the same parameters (sp_load)."""
        self._check(self._lib.sp_load(self._h, os.fsencode(path)))
        n = ctypes.c_int64()
        self._check(self._lib.sp_get_size(self._h, ctypes.byref(n), None))
        self.n = int(n.value)

    def synchronize(self):
        self._check(self._lib.sp_synchronize(self._h))

    def read_moments(self, which: int = MOMENTS_DEM) -> np.ndarray:
        k = NMOM if which == MOMENTS_DEM else 4
        out = np.zeros((self.ncells, k), np.float64)
        self._check(self._lib.sp_read_moments(self._h, int(which), _p(out)))
        return out

    def read_moments_noalloc(self, which: int = MOMENTS_DEM) -> np.ndarray:
        """read_moments through the entry point that allocates no device memory."""
        k = NMOM if which == MOMENTS_DEM else 4
        out = np.zeros((self.ncells, k), np.float64)
        self._check(self._lib.sp_read_moments_noalloc(self._h, int(which), _p(out)))
        return out

    def read_floes(self) -> dict:
        n = self.n
        out = dict(xi=np.zeros(n, np.uint32), yi=np.zeros(n, np.uint32), u=np.zeros(n, np.float32),
                   v=np.zeros(n, np.float32), omega=np.zeros(n, np.float32),
                   theta=np.zeros(n, np.float32), r=np.zeros(n, np.float32))
        self._check(self._lib.sp_read_floes(self._h, *[_p(out[k]) for k in
                                                       ("xi", "yi", "u", "v", "omega", "theta", "r")]))
        return out

    def read_pairs(self) -> np.ndarray:
        cnt = ctypes.c_int64(0)
        self._check(self._lib.sp_read_pairs(self._h, 0, None, None, ctypes.byref(cnt)))
        cap = int(cnt.value)
        l = np.zeros(max(cap, 1), np.int32)
        j = np.zeros(max(cap, 1), np.int32)
        self._check(self._lib.sp_read_pairs(self._h, cap, _p(l), _p(j), ctypes.byref(cnt)))
        return np.stack([l[:cap], j[:cap]], axis=1)

    def stats(self) -> dict:
        c, s, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        self._check(self._lib.sp_get_stats(self._h, ctypes.byref(c), ctypes.byref(s), ctypes.byref(m)))
        return dict(contacts=int(c.value), steps=int(s.value), max_cfl=float(m.value))

    def profile_steps(self, dt: float, nsteps: int):
        """Advance like step() and return the mean (dem_ms, lf_ms) kernel durations."""
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.sp_profile_steps(self._h, float(dt), int(nsteps), ctypes.byref(a),
                                               ctypes.byref(b)))
        return float(a.value), float(b.value)

    def batching(self):
        """(cells, waves, persistent) per count bucket."""
        c = np.zeros(NUM_BUCKETS, np.int32)
        w = np.zeros(NUM_BUCKETS, np.int32)
        q = np.zeros(NUM_BUCKETS, np.int32)
        self._check(self._lib.sp_get_batching(self._h, _p(c), _p(w), _p(q)))
        return c, w, q

    def set_batching(self, waves, persistent):
        w = _c(waves, np.int32)
        q = _c(persistent, np.int32)
        self._check(self._lib.sp_set_batching(self._h, _p(w), _p(q)))

    def autotune(self, dt: float, reps: int = 3) -> float:
        best = ctypes.c_double()
        self._check(self._lib.sp_autotune(self._h, float(dt), int(reps), ctypes.byref(best)))
        return float(best.value)

    def block_waves(self):
        """Wavefronts per cell of each bucket's blocked launches (0: empty bucket)."""
        w = np.zeros(NUM_BUCKETS, np.int32)
        self._check(self._lib.sp_get_block_waves(self._h, _p(w)))
        return w

    def set_graph_chunk(self, chunk: int):
        self._check(self._lib.sp_set_graph_chunk(self._h, int(chunk)))

    def set_step_block(self, k: int):
        """Blocked plain steps: k steps per DEM launch (1: one launch per step)."""
        self._check(self._lib.sp_set_step_block(self._h, int(k)))

    def step_block(self) -> tuple:
        k, act = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.sp_get_step_block(self._h, ctypes.byref(k), ctypes.byref(act)))
        return int(k.value), bool(act.value)

    def work(self) -> dict:
        """Candidate tests and steps counted by blocked steps since the floes were set."""
        t, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.sp_get_work(self._h, ctypes.byref(t), ctypes.byref(b)))
        return dict(candidate_tests=int(t.value), blocked_steps=int(b.value))

    def set_coupling(self, N0: int, N1: int = 1, n_t: int = 1):
        """Coupling cadence of step(): coarse step of N0 fine steps in N1
        sub-steps, coarse-to-fine updates every n_t fine steps."""
        self._check(self._lib.sp_set_coupling(self._h, int(N0), int(N1), int(n_t)))

    def coupling(self) -> dict:
        v = [ctypes.c_int32() for _ in range(3)] + [ctypes.c_int64() for _ in range(4)]
        self._check(self._lib.sp_get_coupling(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["N0", "N1", "n_t", "nudges", "replans", "clamped", "invalid"], [int(x.value) for x in v]))

    def closure_features(self, x):
        """Closure inputs of every cell into the device tensor x [ncells, 45] (float32)."""
        self._check(self._lib.sp_closure_features(self._h, _p(x)))

    def closure_sample(self, dt: float, x, t, mode: int = None):
        """Inputs at the current level into x [ncells, 45], one step, tendencies
        (TEND_FULL or TEND_RESIDUAL, default full) into t [ncells, 4]."""
        mode = TEND_FULL if mode is None else mode
        self._check(self._lib.sp_closure_sample(self._h, float(dt), int(mode), _p(x), _p(t)))

    def resync_cells(self, cells, targets) -> int:
        """Move the floes of the listed cells to targets [ncl, 4] = (rho, P_x, P_y, P_w);
        returns the number of cells whose radius scale was clamped."""
        cl = _c(cells, np.int32)
        tg = _c(targets, np.float64).reshape(-1, 4)
        assert tg.shape[0] == cl.size
        n = ctypes.c_int32()
        self._check(self._lib.sp_resync_cells(self._h, int(cl.size), _p(cl), _p(tg), ctypes.byref(n)))
        return int(n.value)

    def hybrid_set(self, net, closure_cells, check_every: int = 250, check_cells: int = 256, tol: float = 0.02,
                   fallback_steps: int = 100, net_window: float = 0.0):
        """Flag closure cells (bool array [ncells]) for the network `net` (an MLP); None removes the hybrid."""
        if closure_cells is None:
            self._check(self._lib.sp_hybrid_set(self._h, None, None, 1, 0, 1.0, 1, 0.0))
            self._net = None
            return
        m = _c(np.asarray(closure_cells).astype(np.uint8), np.uint8)
        self._check(self._lib.sp_hybrid_set(self._h, net._h, _p(m), int(check_every), int(check_cells), float(tol),
                                            int(fallback_steps), float(net_window)))
        self._net = net   # the network must outlive the hybrid

    def step_hybrid(self, dt: float, nsteps: int = 1):
        self._check(self._lib.sp_step_hybrid(self._h, float(dt), int(nsteps)))

    def hybrid_stats(self) -> dict:
        a, b = ctypes.c_int32(), ctypes.c_int32()
        c, d = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.sp_hybrid_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                              ctypes.byref(d)))
        return {"dem_cells": int(a.value), "closure_cells": int(b.value), "checks": int(c.value),
                "fallbacks": int(d.value)}

    def schedule(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.sp_get_schedule(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return int(a.value), int(b.value), int(c.value)


class MLP:
    """The closure network (one sp_mlp object).  Data arguments are device
    tensors (torch, float32 / int32, contiguous); parameters cross as host arrays."""

    def __init__(self, stream=None):
        self._lib = load_library()
        h = ctypes.c_void_p()
        st = self._lib.sp_mlp_create(None if stream is None else ctypes.c_void_p(stream), ctypes.byref(h))
        if st != 0:
            raise SpdemError(st, "sp_mlp_create failed")
        self._h = h
        self.stream = stream   # raw handle the calls run on (None: the library's own stream)

    def _check(self, st):
        if st != 0:
            raise SpdemError(st, self._lib.sp_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sp_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_params(self, theta):
        th = _c(theta, np.float32)
        assert th.size == MLP_NPARAMS
        self._check(self._lib.sp_mlp_set_params(self._h, _p(th)))

    def get_params(self) -> np.ndarray:
        th = np.zeros(MLP_NPARAMS, np.float32)
        self._check(self._lib.sp_mlp_get_params(self._h, _p(th)))
        return th

    def set_norm(self, x_mean, x_std, y_mean, y_std):
        a = [_c(v, np.float32) for v in (x_mean, x_std, y_mean, y_std)]
        self._check(self._lib.sp_mlp_set_norm(self._h, *[_p(v) for v in a]))

    def get_norm(self):
        out = [np.zeros(MLP_IN, np.float32), np.zeros(MLP_IN, np.float32), np.zeros(MLP_OUT, np.float32),
               np.zeros(MLP_OUT, np.float32)]
        self._check(self._lib.sp_mlp_get_norm(self._h, *[_p(v) for v in out]))
        return out   # x_mean, x_inv_std, y_mean, y_std

    def fit_norm(self, X, T):
        self._check(self._lib.sp_mlp_fit_norm(self._h, _p(X), _p(T), int(X.shape[0])))

    def forward(self, x, y):
        self._check(self._lib.sp_mlp_forward(self._h, _p(x), int(x.shape[0]), _p(y)))

    def gradient(self, X, T):
        g = np.zeros(MLP_NPARAMS, np.float32)
        loss = ctypes.c_float()
        self._check(self._lib.sp_mlp_gradient(self._h, _p(X), _p(T), int(X.shape[0]), _p(g), ctypes.byref(loss)))
        return g, float(loss.value)

    def train_step(self, X, T, rows, batch: int, lr: float = 1e-3) -> float:
        loss = ctypes.c_float()
        self._check(self._lib.sp_mlp_train_step(self._h, _p(X), _p(T), _p(rows), int(batch), float(lr),
                                                ctypes.byref(loss)))
        return float(loss.value)

    def train_epoch(self, X, T, perm, batch: int, lr: float = 1e-3) -> float:
        loss = ctypes.c_float()
        self._check(self._lib.sp_mlp_train_epoch(self._h, _p(X), _p(T), _p(perm), int(perm.shape[0]), int(batch),
                                                 float(lr), ctypes.byref(loss)))
        return float(loss.value)

    def set_input_noise(self, sd=None, seed: int = 0):
        """Gaussian noise of scale sd[f] (raw input units) on inputs f < len(sd)
        of every training row (None or empty: off)."""
        a = np.zeros(0, np.float32) if sd is None else np.ascontiguousarray(sd, np.float32)
        self._check(self._lib.sp_mlp_set_input_noise(self._h, int(a.size),
                                                     a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if a.size else None,
                                                     ctypes.c_uint64(int(seed) & (2**64 - 1))))


class GlobalDEM:
    """The global DEM of the paper's error study (one context of the C
    library): one periodic DEM over the whole domain, floes crossing cells."""

    def __init__(self, lx, ly, rho_ice, rho_ocean, cd, E, G, mu, flags: int = 0, stream=None):
        self._lib = load_library()
        self.n = 0
        prm = _GParams(lx, ly, rho_ice, rho_ocean, cd, E, G, mu, flags)
        h = ctypes.c_void_p()
        st = self._lib.sp_gdem_create(ctypes.byref(prm), None if stream is None else ctypes.c_void_p(stream),
                                      ctypes.byref(h))
        if st != 0:
            raise SpdemError(st, "sp_gdem_create failed")
        self._h = h

    @classmethod
    def from_workload(cls, w, flags: int = 0, stream=None) -> "GlobalDEM":
        """A global workload: one cell spanning the domain, positions as domain fractions."""
        if w.nx != 1 or w.ny != 1:
            raise ValueError("a global workload has one cell spanning the domain")
        g = cls(w.Lx, w.Ly, w.rho_ice, w.rho_ocean, w.cd, w.E, w.G, w.mu, flags, stream)
        oc = w.ocean
        arrs = [_c(a, np.float64) for a in (oc.kx, oc.ky, oc.au, oc.av, oc.phase)]
        g._check(g._lib.sp_gdem_set_ocean(g._h, float(oc.u0), float(oc.v0), int(arrs[0].size),
                                          *[_p(a) for a in arrs]))
        fl = [_c(w.xi, np.uint32), _c(w.yi, np.uint32)] + [_c(a, np.float32) for a in
                                                         (w.u, w.v, w.omega, w.theta, w.r, w.h)]
        g.n = int(fl[0].size)
        g._check(g._lib.sp_gdem_set_floes(g._h, g.n, *[_p(a) for a in fl]))
        return g

    def _check(self, st):
        if st != 0:
            raise SpdemError(st, self._lib.sp_gdem_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sp_gdem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, dt: float, nsteps: int = 1):
        self._check(self._lib.sp_gdem_step(self._h, float(dt), int(nsteps)))

    def read_floes(self) -> dict:
        n = self.n
        out = dict(xi=np.zeros(n, np.uint32), yi=np.zeros(n, np.uint32), u=np.zeros(n, np.float32),
                   v=np.zeros(n, np.float32), omega=np.zeros(n, np.float32), theta=np.zeros(n, np.float32),
                   r=np.zeros(n, np.float32))
        self._check(self._lib.sp_gdem_read_floes(self._h, *[_p(out[k]) for k in
                                                          ("xi", "yi", "u", "v", "omega", "theta", "r")]))
        return out

    def coarse_moments(self, nxc: int, nyc: int) -> np.ndarray:
        out = np.zeros((int(nxc) * int(nyc), NMOM), np.float64)
        self._check(self._lib.sp_gdem_coarse_moments(self._h, int(nxc), int(nyc), _p(out)))
        return out

    def stats(self) -> dict:
        c, s, bx, by = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.sp_gdem_get_stats(self._h, ctypes.byref(c), ctypes.byref(s), ctypes.byref(bx),
                                                ctypes.byref(by)))
        return dict(contacts=int(c.value), steps=int(s.value), bins=(int(bx.value), int(by.value)))

    def read_order(self):
        """(floe indices in the current order, sub-bin starts of that order,
        sub-bins and coarse cells gathered by a full scan so far)."""
        bx, by = self.stats()["bins"]
        ids = np.zeros(self.n, np.int32)
        starts = np.zeros(bx * by + 1, np.int32)
        fb = ctypes.c_int64()
        self._check(self._lib.sp_gdem_read_order(self._h, _p(ids), _p(starts), ctypes.byref(fb)))
        return ids, starts, int(fb.value)
