"""Contact-heavy test workloads (seeded) shared by the CPU and GPU tests."""
import numpy as np

import fixtures
from helpers import frac


def dense_workload(seed=11, nx=3, ny=2, n=256, vel=0.2):
    """Benchmark-style cells with random initial velocities and spins, so that
    many contacts form within a few steps."""
    w = fixtures.custom(nx, ny, 25e3, n, seed=seed, r_scale=fixtures.radius_scale(n, 25e3 ** 2))
    rng = np.random.default_rng(seed)
    w.u[:] = rng.normal(0, vel, w.nfloes)
    w.v[:] = rng.normal(0, vel, w.nfloes)
    w.omega[:] = rng.normal(0, 1e-4, w.nfloes)
    w.theta[:] = rng.uniform(0, 6.28, w.nfloes)
    return w


def ragged_workload(seed=5):
    """Empty, single-floe, partial-wave and multi-floe-per-lane cells."""
    rng = np.random.default_rng(seed)
    nx, ny = 5, 3
    counts = rng.integers(0, 700, nx * ny)
    counts[0], counts[1], counts[2], counts[3] = 0, 1, 64, 257
    w = fixtures.custom(nx, ny, 25e3, counts, seed=seed, r_scale=fixtures.radius_scale(700, 25e3 ** 2))
    w.u[:] = rng.normal(0, 0.2, w.nfloes)
    w.v[:] = rng.normal(0, 0.2, w.nfloes)
    return w


def uneven_workload(seed=3, nx=12, ny=8):
    """Poisson counts from a marginal-ice-zone concentration field (0-~700 per
    cell), at rest, radii scaled to area fraction 0.40 at 512 floes."""
    rng = np.random.default_rng(seed)
    c = fixtures.miz_concentration(rng, nx, ny, smooth_cells=2.0)
    counts = rng.poisson(512 * c).reshape(-1).astype(np.int32)
    counts[0] = 0
    counts[1] = 1
    counts[2] = 700
    return fixtures.custom(nx, ny, 25e3, counts, seed=seed, r_scale=fixtures.radius_scale(512, 25e3 ** 2),
                           G=3.5e3)


def lattice_workload(counts, nx, ny, L=25e3, r=300.0, u=0.0, v=0.0, seed=0, big_radius=1000.0, ocean=None,
                     identical=False):
    """Floes on a 3 x 3 lattice of each cell (spacing L / 3, no contacts while
    radii stay below L / 6), first counts[c] lattice sites of cell c used,
    thicknesses drawn per floe (the same in every cell when identical), all
    with velocity (u, v) and no spin.  The first floe of the first cell has
    big_radius, which sizes the contact-search bins of the HIP path."""
    rng = np.random.default_rng(seed)
    counts = np.broadcast_to(np.asarray(counts, np.int32), (nx * ny,)).copy()
    assert counts.max() <= 9
    sites = (np.arange(3) + 0.5) * L / 3.0
    xs, ys, rr, hh = [], [], [], []
    h_cell = rng.uniform(0.5, 2.0, 9)
    for c in range(nx * ny):
        k = np.arange(counts[c])
        xs.append(sites[k % 3])
        ys.append(sites[k // 3])
        rr.append(np.full(counts[c], r))
        hh.append(h_cell[:counts[c]] if identical else rng.uniform(0.5, 2.0, counts[c]))
    r_all = np.concatenate(rr)
    if big_radius and r_all.size:
        r_all[0] = big_radius
    n = int(counts.sum())
    return fixtures.from_arrays(nx, ny, L, counts, frac(np.concatenate(xs), L), frac(np.concatenate(ys), L),
                                r_all, np.concatenate(hh), u=np.full(n, u), v=np.full(n, v), ocean=ocean)
