"""Small builders shared by the tests (no method arithmetic)."""
import numpy as np

import fixtures

TWO32 = 2.0 ** 32


def frac(x_m, L):
    """Metres in [0, L) -> unsigned 32-bit cell fraction (rounded)."""
    return np.asarray(np.round(np.asarray(x_m, np.float64) / L * TWO32) % TWO32, np.uint64).astype(np.uint32)


def two_floes(L, x1, y1, x2, y2, r1, r2, h1=1.0, h2=1.0, u1=(0, 0), u2=(0, 0), w1=0.0, w2=0.0,
              ocean=None, G=5.0e3, mu=0.3, E=200.0):
    w = fixtures.from_arrays(1, 1, L, [2], frac([x1, x2], L), frac([y1, y2], L), [r1, r2], [h1, h2],
                             u=[u1[0], u2[0]], v=[u1[1], u2[1]], omega=[w1, w2], ocean=ocean, G=G)
    w.mu = mu
    w.E = E
    return w


def kinetic(state, w):
    m = w.rho_ice * state.h * np.pi * state.r ** 2
    I = m * state.r ** 2
    return 0.5 * np.sum(m * (state.u ** 2 + state.v ** 2)) + 0.5 * np.sum(I * state.w ** 2)


def momentum(state, w):
    m = w.rho_ice * state.h * np.pi * state.r ** 2
    return np.array([np.sum(m * state.u), np.sum(m * state.v)])


def random_cell(rng, n, L, rmin, rmax, nx=1, ny=1):
    """n floes per cell at uniform random positions (overlaps allowed)."""
    counts = np.full(nx * ny, n, np.int32)
    N = int(counts.sum())
    xi = rng.integers(0, 2 ** 32, N, dtype=np.uint64).astype(np.uint32)
    yi = rng.integers(0, 2 ** 32, N, dtype=np.uint64).astype(np.uint32)
    r = rng.uniform(rmin, rmax, N).astype(np.float32)
    h = rng.uniform(0.5, 2.0, N).astype(np.float32)
    return fixtures.from_arrays(nx, ny, L, counts, xi, yi, r, h)
