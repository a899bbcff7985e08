"""Seeded synthetic workloads shared by the HIP path and the FP64 oracle.

This module generates inputs only and holds none of the method's arithmetic:
floe radii, thicknesses, non-overlapping positions, per-cell floe counts and
the prescribed ocean current.  Every array is produced from a fixed seed, so a
workload is identical wherever it is built.

Position convention: cell-local, unsigned 32-bit fractions of the cell side,
``x = Lx * xi / 2**32`` (the cell is doubly periodic, Sec. 3.1).

Ocean convention (the current is prescribed, Sec. 2.1):
``u_o(X) = U0 + sum_m (au_m, av_m) * sin(kx_m X + ky_m Y + phase_m)`` in global
coordinates ``X = (ix + xi/2**32) Lx``.  Divergence-free fields are built from
a stream function, compressible ones (Sec. 4.2, 4.3) directly.

Workloads (sizes from the benchmark configurations; constants proposed because
the paper is nondimensional and gives no SI values):

=============  =====================================================================
``small``      4x4 cells of 50 km, 32 floes/cell, lognormal radii (median 1.5 km,
               sigma 0.5, clip [0.5, 4] km), h ~ U[0.5, 2] m, psi = A sin sin with a
               0.2 m/s peak, dt 60 s
``plain64``    64x64 cells of 25 km, 256 floes/cell, radii scaled to area fraction
               0.40, 8 seeded Fourier modes of 100-800 km at 0.15 m/s rms, dt 30 s
``uneven128``  128x128 cells of 25 km, Poisson(512 c) floes/cell with a marginal-ice-
               zone concentration field c, radii scaled to 0.40 at 512, dt 30 s
``closure256`` 256x256 cells, plain64-style fields (closure inference grid)
``hybrid512``  512x512 cells, Poisson(256 c) floes/cell, dt 30 s
=============  =====================================================================

Every 25 km-cell workload draws its 8 ocean modes as integer wave-vectors
2 <= |(p, q)| <= 16 on its own periodic domain (100-800 km wavelengths on the
64 x 64 grid, proportionally longer on the larger grids).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfxgen.so")
_lib = None

SEED_BASE = 230307819
TWO_PI = 2.0 * math.pi

# Physical constants shared by every workload.  rho_ice, Cd and mu are the
# benchmark's; rho_o is sea water; E and G are chosen for explicit stability at
# the stated time steps (the paper's runs are nondimensional).
RHO_ICE = 920.0
RHO_OCEAN = 1025.0
CD = 5.5e-3
MU = 0.3
E_NORMAL = 200.0


def build(force: bool = False) -> str:
    """Compile the generator with gcc (OpenMP); returns the library path."""
    src = os.path.join(_HERE, "fxgen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.fx_floes.argtypes = [ctypes.c_int32, P, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                 ctypes.c_int32, P, P, P, P]
        lib.fx_floes.restype = ctypes.c_int
        lib.fx_rand_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.fx_rand_u64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Ocean:
    """Prescribed current: U0 + sum_m (au_m, av_m) sin(k_m . X + phase_m)."""
    u0: float = 0.0
    v0: float = 0.0
    kx: np.ndarray = field(default_factory=lambda: np.zeros(0))
    ky: np.ndarray = field(default_factory=lambda: np.zeros(0))
    au: np.ndarray = field(default_factory=lambda: np.zeros(0))
    av: np.ndarray = field(default_factory=lambda: np.zeros(0))
    phase: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def nmodes(self) -> int:
        return int(self.kx.size)

    @staticmethod
    def from_streamfunction(a, kx, ky, phase, u0=0.0, v0=0.0) -> "Ocean":
        """psi = sum a sin(k.X + phase); u = -psi_Y, v = psi_X (divergence free)."""
        a = np.asarray(a, np.float64)
        kx = np.asarray(kx, np.float64)
        ky = np.asarray(ky, np.float64)
        ph = np.asarray(phase, np.float64)
        # d/dY [a sin(th)] = a ky cos(th) = a ky sin(th + pi/2)
        return Ocean(u0, v0, kx.copy(), ky.copy(), -a * ky, a * kx, ph + 0.5 * math.pi)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    Lx: float
    Ly: float
    dt: float
    steps: int
    counts: np.ndarray          # int32 [ncells], cell id = iy * nx + ix
    xi: np.ndarray              # uint32 [N]
    yi: np.ndarray              # uint32 [N]
    u: np.ndarray               # float32 [N]  m/s
    v: np.ndarray               # float32 [N]  m/s
    omega: np.ndarray           # float32 [N]  1/s
    theta: np.ndarray           # float32 [N]  rad
    r: np.ndarray               # float32 [N]  m
    h: np.ndarray               # float32 [N]  m
    ocean: Ocean
    rho_ice: float = RHO_ICE
    rho_ocean: float = RHO_OCEAN
    cd: float = CD
    E: float = E_NORMAL
    G: float = 5.0e3
    mu: float = MU
    conc: np.ndarray | None = None   # concentration field used for counts, if any

    @property
    def ncells(self) -> int:
        return self.nx * self.ny

    @property
    def nfloes(self) -> int:
        return int(self.xi.size)

    @property
    def start(self) -> np.ndarray:
        s = np.zeros(self.ncells + 1, np.int64)
        np.cumsum(self.counts, out=s[1:])
        return s

    @property
    def cell(self) -> np.ndarray:
        return np.repeat(np.arange(self.ncells, dtype=np.int32), self.counts)

    def params(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, Lx=self.Lx, Ly=self.Ly, rho_ice=self.rho_ice,
                    rho_ocean=self.rho_ocean, cd=self.cd, E=self.E, G=self.G, mu=self.mu)

    def state(self) -> dict:
        return dict(xi=self.xi, yi=self.yi, u=self.u, v=self.v, omega=self.omega,
                    theta=self.theta, r=self.r, h=self.h)



def lognormal_clip_m2(r_med: float, sigma: float, lo: float, hi: float) -> float:
    """E[r^2] of a lognormal(median r_med, sigma) clipped to [lo, hi] (quadrature)."""
    z = np.linspace(-10, 10, 200001)
    w = np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    r = np.clip(r_med * np.exp(sigma * z), lo, hi)
    return float(np.trapezoid(w * r * r, z))


def radius_scale(n_per_cell: float, cell_area: float, phi: float = 0.40,
                 r_med=1500.0, sigma=0.5, lo=500.0, hi=4000.0) -> float:
    """Scale s so that n floes of the clipped lognormal law cover area fraction phi."""
    return math.sqrt(phi * cell_area / (n_per_cell * math.pi * lognormal_clip_m2(r_med, sigma, lo, hi)))


def place_floes(counts: np.ndarray, Lx: float, Ly: float, seed: int, r_scale: float,
                r_med=1500.0, sigma=0.5, lo=500.0, hi=4000.0, h_lo=0.5, h_hi=2.0,
                max_tries=10000):
    lib = _load()
    counts = np.ascontiguousarray(counts, np.int32)
    ncells = counts.size
    start = np.zeros(ncells + 1, np.int64)
    np.cumsum(counts, out=start[1:])
    n = int(start[-1])
    xi = np.zeros(n, np.uint32)
    yi = np.zeros(n, np.uint32)
    r = np.zeros(n, np.float32)
    h = np.zeros(n, np.float32)
    rc = lib.fx_floes(ncells, _ptr(start), Lx, Ly, r_med, sigma, lo, hi, r_scale, h_lo, h_hi,
                      seed, max_tries, _ptr(xi), _ptr(yi), _ptr(r), _ptr(h))
    if rc != 0:
        raise RuntimeError(f"floe placement failed in cell {-rc - 1} (seed {seed})")
    return xi, yi, r, h


def random_modes(rng: np.random.Generator, nmodes: int, Dx: float, Dy: float,
                 kmin: float = 2.0, kmax: float = 16.0, rms_speed: float = 0.15) -> Ocean:
    """Divergence-free current from nmodes distinct integer wave-vectors (p, q),
    kmin <= |(p, q)| <= kmax on the periodic domain, scaled to a domain-rms speed."""
    cand = [(p, q) for p in range(-int(kmax), int(kmax) + 1) for q in range(0, int(kmax) + 1)
            if (q > 0 or p > 0) and kmin <= math.hypot(p, q) <= kmax]
    pick = rng.choice(len(cand), size=nmodes, replace=False)
    pq = np.array([cand[i] for i in pick], np.float64)
    kx = TWO_PI * pq[:, 0] / Dx
    ky = TWO_PI * pq[:, 1] / Dy
    a = rng.standard_normal(nmodes)
    ph = rng.uniform(0.0, TWO_PI, nmodes)
    # distinct, non-opposite wave-vectors are orthogonal over the domain:
    # <|u|^2> = sum a^2 |k|^2 / 2
    ms = float(np.sum(a * a * (kx * kx + ky * ky)) / 2.0)
    a *= rms_speed / math.sqrt(ms)
    return Ocean.from_streamfunction(a, kx, ky, ph)


def miz_concentration(rng: np.random.Generator, nx: int, ny: int, smooth_cells=4.0, noise=0.15):
    """c = clip(1/2 + 1/2 tanh((x - D/2) / (0.1 D)) + noise * xi, 0, 1), xi a
    periodic Gaussian field smoothed over smooth_cells with unit std: a
    marginal-ice-zone band across x (open water on the left, pack ice on the right)."""
    w = rng.standard_normal((ny, nx))
    fy = np.fft.fftfreq(ny)[:, None]
    fx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (math.pi * smooth_cells) ** 2 * (fx * fx + fy * fy))
    xi = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    xi /= xi.std()
    xc = (np.arange(nx) + 0.5) / nx
    base = 0.5 + 0.5 * np.tanh((xc - 0.5) / 0.1)
    return np.clip(base[None, :] + noise * xi, 0.0, 1.0)


def _assemble(name, nx, ny, L, dt, steps, counts, seed, r_scale, ocean, G, conc=None,
              r_med=1500.0, sigma=0.5, lo=500.0, hi=4000.0):
    xi, yi, r, h = place_floes(counts, L, L, seed, r_scale, r_med, sigma, lo, hi)
    n = xi.size
    z = np.zeros(n, np.float32)
    return Workload(name, nx, ny, L, L, dt, steps, np.asarray(counts, np.int32), xi, yi,
                    z.copy(), z.copy(), z.copy(), z.copy(), r, h, ocean, G=G, conc=conc)


CONFIG_NAMES = ["small", "plain64", "uneven128", "closure256", "hybrid512"]


def make_config(i, seed: int | None = None) -> Workload:
    """Workload i (0..4, or its name) of the benchmark configurations."""
    if isinstance(i, str):
        i = CONFIG_NAMES.index(i)
    seed = SEED_BASE + i if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    if i == 0:
        nx = ny = 4
        L = 50e3
        D = nx * L
        A = 0.2 * D / TWO_PI           # peak speed 0.2 m/s
        k = TWO_PI / D
        # A sin(kX) sin(kY) = A/2 cos(k(X-Y)) - A/2 cos(k(X+Y))
        oc = Ocean.from_streamfunction([0.5 * A, -0.5 * A], [k, k], [-k, k], [0.5 * math.pi] * 2)
        counts = np.full(nx * ny, 32, np.int32)
        return _assemble("small", nx, ny, L, 60.0, 1000, counts, seed, 1.0, oc, G=8.0e3)
    if i in (1, 3):
        nx = ny = 64 if i == 1 else 256
        L = 25e3
        oc = random_modes(rng, 8, nx * L, ny * L)
        s = radius_scale(256, L * L)
        counts = np.full(nx * ny, 256, np.int32)
        return _assemble(CONFIG_NAMES[i], nx, ny, L, 30.0, 10000 if i == 1 else 1, counts, seed, s,
                         oc, G=5.0e3)
    if i in (2, 4):
        nx = ny = 128 if i == 2 else 512
        nmax = 512 if i == 2 else 256
        L = 25e3
        oc = random_modes(rng, 8, nx * L, ny * L)
        c = miz_concentration(rng, nx, ny)
        counts = rng.poisson(nmax * c).astype(np.int32).reshape(-1)
        s = radius_scale(nmax, L * L)
        return _assemble(CONFIG_NAMES[i], nx, ny, L, 30.0, 5000 if i == 2 else 2000, counts, seed, s,
                         oc, G=3.5e3 if i == 2 else 5.0e3, conc=c)
    raise ValueError(i)


def custom(nx, ny, L, counts, seed, r_scale=1.0, ocean=None, G=5.0e3, dt=30.0,
           r_med=1500.0, sigma=0.5, lo=500.0, hi=4000.0) -> Workload:
    """A small seeded workload of any shape (tests)."""
    counts = np.broadcast_to(np.asarray(counts, np.int32), (nx * ny,)).copy()
    # wavelengths of at least two cells, as in the benchmark fields (4-32 cells)
    kmax = max(1.5, min(nx, ny) / 2.0)
    ocean = ocean if ocean is not None else random_modes(np.random.Generator(np.random.PCG64(seed)),
                                                         4, nx * L, ny * L, kmin=1.0, kmax=kmax)
    return _assemble("custom", nx, ny, L, dt, 10, counts, seed, r_scale, ocean, G,
                     r_med=r_med, sigma=sigma, lo=lo, hi=hi)


def from_arrays(nx, ny, L, counts, xi, yi, r, h, u=None, v=None, omega=None, theta=None,
                ocean=None, G=5.0e3, dt=30.0, name="explicit") -> Workload:
    """A workload from explicit per-floe arrays (cell-sorted)."""
    n = len(xi)
    f = lambda a: np.zeros(n, np.float32) if a is None else np.asarray(a, np.float32).copy()
    return Workload(name, nx, ny, float(L), float(L), dt, 1, np.asarray(counts, np.int32),
                    np.asarray(xi, np.uint32).copy(), np.asarray(yi, np.uint32).copy(),
                    f(u), f(v), f(omega), f(theta), f(r), f(h), ocean if ocean is not None else Ocean(),
                    G=G)


# ------------------------------------------------------------- closure network
MLP_SIZES = [45, 128, 128, 128, 4]


def mlp_init(seed: int) -> np.ndarray:
    """Initial closure-network parameters (flat FP32 vector, layout
    W1 [128x45], b1, W2 [128x128], b2, W3 [128x128], b3, W4 [4x128], b4):
    Kaiming-uniform weights with bound sqrt(6 / fan_in), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l in range(1, 5):
        fan_in = MLP_SIZES[l - 1]
        bound = math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-bound, bound, (MLP_SIZES[l], fan_in)).reshape(-1))
        parts.append(np.zeros(MLP_SIZES[l]))
    return np.concatenate(parts).astype(np.float32)


# ------------------------------------------------ the paper's error scenarios
# Sec. 4.1-4.3 are nondimensional: domain [0, 4] x [0, 2], floes of radius
# r = r_c (0.2 + 0.8 sin(0.25 pi x)) at the centres of a 480 x 240 fine grid
# (r_c = 1/240, half the fine-cell side), all moving with (0.3, 0) at first.
# The paper gives no densities, drag coefficient or contact constants; these
# are proposed: unit densities and thickness, a drag rate Cd rho_o / (rho_ice h)
# = 50 (relaxation time 0.2 at a 0.1 velocity difference), E = 1e4 and G = 1
# (contact frequency times dt = 0.1 or less at dt = 1e-4, light damping).
SCENARIO_CONSTANTS = dict(rho_ice=1.0, rho_ocean=1.0, cd=50.0, E=1.0e4, G=1.0, mu=0.3)


def scenario_ocean(k: int) -> Ocean:
    """Prescribed currents of Sec. 4.1 and 4.4 (uniform), 4.2
    (0.3 - 0.1 cos(pi x), 0) and 4.3 (0.3 - 0.1 sin(0.1 pi x) cos(pi y),
    0.05 cos(0.1 pi x) sin(pi y)), the last written as two plane modes."""
    p = math.pi
    u0 = float(np.float32(0.3))           # equal to the floes' stored velocity
    if k in (1, 4):
        return Ocean(u0, 0.0)
    if k == 2:
        return Ocean(u0, 0.0, np.array([p]), np.array([0.0]), np.array([-0.1]), np.array([0.0]),
                     np.array([0.5 * p]))
    if k == 3:
        return Ocean(u0, 0.0, np.array([0.1 * p, 0.1 * p]), np.array([p, -p]), np.array([-0.05, -0.05]),
                     np.array([0.025, -0.025]), np.zeros(2))
    raise ValueError(f"no scenario 4.{k}")


def scenario_global(k: int, nfx: int = 480, nfy: int = 240, Lx: float = 4.0, Ly: float = 2.0,
                    dt: float = 1e-4) -> Workload:
    """The initial state of scenario 4.k as one global DEM (a single cell
    spanning the domain; positions are fractions of the domain).  Scenario
    4.4 starts as 4.1; its walls in x are a flag of the models that run it."""
    fx = (np.arange(nfx) + 0.5) / nfx
    fy = (np.arange(nfy) + 0.5) / nfy
    X, Y = np.meshgrid(fx, fy)
    xs, ys = X.reshape(-1), Y.reshape(-1)
    rc = 0.5 * Ly / nfy
    r = rc * (0.2 + 0.8 * np.sin(0.25 * math.pi * xs * Lx))
    n = xs.size
    xi = (np.round(xs * 2.0 ** 32) % 2.0 ** 32).astype(np.uint64).astype(np.uint32)
    yi = (np.round(ys * 2.0 ** 32) % 2.0 ** 32).astype(np.uint64).astype(np.uint32)
    z = np.zeros(n, np.float32)
    w = Workload(f"scenario4.{k}", 1, 1, Lx, Ly, dt, 0, np.array([n], np.int32), xi, yi,
                 np.full(n, 0.3, np.float32), z.copy(), z.copy(), z.copy(), r.astype(np.float32),
                 np.ones(n, np.float32), scenario_ocean(k))
    for key, val in SCENARIO_CONSTANTS.items():
        setattr(w, key, val)
    return w


def split_cells(w: Workload, nxc: int, nyc: int) -> Workload:
    """The floes of a global workload distributed over nxc x nyc cells: each
    floe goes to the cell holding its centre, with cell-local fractions (the
    superparameterised model's initial state on that coarse grid)."""
    sx = w.xi.astype(np.uint64) * np.uint64(nxc)
    sy = w.yi.astype(np.uint64) * np.uint64(nyc)
    cx, cy = (sx >> np.uint64(32)).astype(np.int64), (sy >> np.uint64(32)).astype(np.int64)
    lx = (sx & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    ly = (sy & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    cell = cy * nxc + cx
    order = np.argsort(cell, kind="stable")
    counts = np.bincount(cell, minlength=nxc * nyc).astype(np.int32)
    out = Workload(f"{w.name}@{nxc}x{nyc}", nxc, nyc, w.Lx / nxc, w.Ly / nyc, w.dt, w.steps, counts,
                   lx[order], ly[order], w.u[order], w.v[order], w.omega[order], w.theta[order], w.r[order],
                   w.h[order], w.ocean)
    for key in ("rho_ice", "rho_ocean", "cd", "E", "G", "mu"):
        setattr(out, key, getattr(w, key))
    return out
