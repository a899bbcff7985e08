"""Learned closure: training data from the method's own DEM runs, training on
the GPU, and the DEM + closure hybrid measured against full DEM.

Everything here drives the C library (``Sim`` and ``MLP``); the arithmetic runs
in its kernels.  The network maps a cell's features (the continuum state of
its 3 x 3 neighbourhood, the ocean current and curl at its centre and six
static floe descriptors) to the residual tendency of its continuum state: the
part of (Q_new - Q_old) / dt that the coarse state does not determine by itself
(the drag sources and the difference between the number-averaged velocity of
the floes and P / rho).  The hybrid advances closure cells by the
Lax-Friedrichs step with <v> = P / rho plus dt times that residual.

Training runs are synthetic: grids of 25 km cells with a marginal-ice-zone
concentration field, Poisson floe counts and seeded Fourier-mode currents, so
that the network sees open water, the ice edge and pack ice.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import MLP, Sim, TEND_RESIDUAL, MOMENTS_CONTINUUM

MIZ_LO, MIZ_HI = 0.15, 0.8   # marginal ice zone: the DEM runs where lo <= c <= hi


def training_workload(seed: int, n: int = 64, nmax: int = 256):
    """A 64 x 64 grid of 25 km cells, Poisson(nmax c) floes per cell with a
    marginal-ice-zone concentration c, radii scaled to area fraction 0.40 at
    nmax, 8 Fourier modes of 100-800 km at 0.15 m/s rms, dt 30 s."""
    import fixtures
    rng = np.random.Generator(np.random.PCG64(seed))
    L = 25e3
    oc = fixtures.random_modes(rng, 8, n * L, n * L)
    c = fixtures.miz_concentration(rng, n, n)
    counts = rng.poisson(nmax * c).astype(np.int32).reshape(-1)
    s = fixtures.radius_scale(nmax, L * L)
    xi, yi, r, h = fixtures.place_floes(counts, L, L, seed, s)
    z = np.zeros(xi.size, np.float32)
    return fixtures.Workload(f"train{seed}", n, n, L, L, 30.0, 2048, counts, xi, yi, z.copy(), z.copy(),
                             z.copy(), z.copy(), r, h, oc, G=5.0e3, conc=c)


def sample_schedule(first: int = 32, every: int = 20, count: int = 128):
    """Steps at which samples are taken: the first `first` steps one by one
    (the floes spin up from rest within a few tens of steps), then every
    `every`-th step, `count` in all."""
    steps = list(range(min(first, count)))
    while len(steps) < count:
        steps.append(steps[-1] + every)
    return steps


def generate_samples(workloads, schedule=None, stream=None, log=None):
    """(features, residual tendency) of every cell at the steps of `schedule`
    of a run of each workload from its initial state; device tensors [n, 45]
    and [n, 4]."""
    import torch
    schedule = sample_schedule() if schedule is None else sorted(schedule)
    n = sum(w.ncells for w in workloads) * len(schedule)
    X = torch.empty((n, 45), device="cuda", dtype=torch.float32)
    T = torch.empty((n, 4), device="cuda", dtype=torch.float32)
    row = 0
    for w in workloads:
        t0 = time.perf_counter()
        with Sim.from_workload(w, stream=stream) as s:
            at = 0
            for k in schedule:
                if k > at:
                    s.step(w.dt, k - at)
                s.closure_sample(w.dt, X[row:row + w.ncells], T[row:row + w.ncells], mode=TEND_RESIDUAL)
                row += w.ncells
                at = k + 1
            s.synchronize()
        if log:
            log(f"samples: {w.name} {w.nfloes} floes, {at} steps in {time.perf_counter() - t0:.1f} s")
    return X, T


def train(X, T, epochs: int = 20, batch: int = 4096, lr: float = 1e-3, seed: int = 0, holdout: float = 0.05,
          stream=None, log=None):
    """Adam on the bfloat16 network from Kaiming-uniform initial weights;
    normalisation from the training rows.  Returns (net, history) with the
    mean training loss per epoch and the held-out loss (normalised MSE)."""
    import torch
    import fixtures
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    order = torch.randperm(n, generator=g)
    nval = int(n * holdout)
    val = order[:nval].to("cuda", torch.int32)
    tr = order[nval:]
    net = MLP(stream)
    net.set_params(fixtures.mlp_init(seed))
    Xtr = X[tr.to("cuda")].contiguous()
    Ttr = T[tr.to("cuda")].contiguous()
    net.fit_norm(Xtr, Ttr)
    hist = {"train": [], "val": [], "seconds": 0.0}
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(Xtr.shape[0], generator=g).to("cuda", torch.int32)
        hist["train"].append(net.train_epoch(Xtr, Ttr, perm, batch, lr))
        hist["val"].append(validation_loss(net, X, T, val))
        if log:
            log(f"epoch {ep + 1}: train {hist['train'][-1]:.4f} held-out {hist['val'][-1]:.4f}")
    torch.cuda.synchronize()
    hist["seconds"] = time.perf_counter() - t0
    hist["samples"] = int(Xtr.shape[0])
    hist["steps"] = epochs * (int(Xtr.shape[0]) // batch)
    return net, hist


def validation_loss(net, X, T, rows, chunk: int = 1 << 17) -> float:
    """Mean squared error on normalised targets over the listed rows."""
    import torch
    x_mean, x_inv, y_mean, y_std = net.get_norm()
    ym = torch.as_tensor(y_mean, device="cuda")
    ys = torch.as_tensor(y_std, device="cuda")
    tot, cnt = 0.0, 0
    for a in range(0, rows.numel(), chunk):
        idx = rows[a:a + chunk].long()
        x = X[idx].contiguous()
        y = torch.empty((idx.numel(), 4), device="cuda")
        net.forward(x, y)
        e = (y - T[idx]) / ys
        tot += float((e * e).sum())
        cnt += e.numel()
    return tot / max(cnt, 1)


def miz_mask(w):
    """True where the DEM runs in the hybrid: concentration within the marginal ice zone."""
    c = np.asarray(w.conc).reshape(-1)
    return (c >= MIZ_LO) & (c <= MIZ_HI)


def rel_l2(a, b):
    """Relative L2 error over cells, per component."""
    return np.linalg.norm(a - b, axis=0) / np.maximum(np.linalg.norm(b, axis=0), 1e-300)


def timed_run(sim, dt, nsteps, hybrid: bool, stream):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    if hybrid:
        sim.step_hybrid(dt, nsteps)
    else:
        sim.step(dt, nsteps)
    e1.record(stream)
    sim.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def hybrid_experiment(w, net, nsteps: int, stream, check_every=50, check_cells=256, tol=1.0,
                      fallback_steps=100, log=None, baseline_net=None):
    """Full DEM and the hybrid from the same initial state, nsteps each.
    Returns a dict of throughputs and errors (relative L2 per component and the
    95th percentile per-cell relative error, both against full DEM)."""
    dem = miz_mask(w)
    out = {"cells": w.ncells, "floes": w.nfloes, "steps": nsteps, "dem_cells": int(dem.sum()),
           "floes_in_dem_cells": int(w.counts[dem].sum())}
    with Sim.from_workload(w, stream=stream.cuda_stream) as s:
        s.step(w.dt, 4)                        # warm-up (graph capture), then a fresh start
        s.set_floes(w.counts, w.xi, w.yi, w.u, w.v, w.omega, w.theta, w.r, w.h)
        sec = timed_run(s, w.dt, nsteps, False, stream)
        Qf = s.read_moments(MOMENTS_CONTINUUM)
    out["full_dem_floe_steps_per_s"] = w.nfloes * nsteps / sec
    out["full_dem_ms_per_step"] = 1e3 * sec / nsteps
    if log:
        log(f"full DEM: {1e3 * sec / nsteps:.3f} ms/step")

    def run_h(model):
        with Sim.from_workload(w, stream=stream.cuda_stream) as s:
            s.hybrid_set(model, ~dem, check_every, check_cells, tol, fallback_steps)
            s.step_hybrid(w.dt, 2)             # warm-up of the network's workspace
            s.set_floes(w.counts, w.xi, w.yi, w.u, w.v, w.omega, w.theta, w.r, w.h)
            s.hybrid_set(model, ~dem, check_every, check_cells, tol, fallback_steps)
            sec = timed_run(s, w.dt, nsteps, True, stream)
            Q = s.read_moments(MOMENTS_CONTINUUM)
            return sec, Q, s.hybrid_stats()

    sec, Qh, hs = run_h(net)
    e = rel_l2(Qh, Qf)
    scale = np.sqrt(np.mean(Qf * Qf, axis=0))
    cell = np.abs(Qh - Qf) / np.maximum(np.abs(Qf), 1e-3 * scale)
    out.update({"hybrid_floe_steps_per_s": w.nfloes * nsteps / sec, "hybrid_ms_per_step": 1e3 * sec / nsteps,
                "speedup": out["full_dem_ms_per_step"] / (1e3 * sec / nsteps),
                "rel_l2": dict(zip(["rho", "Px", "Py", "Pw"], map(float, e))),
                "p95_cell_rel_err": dict(zip(["rho", "Px", "Py", "Pw"], map(float, np.percentile(cell, 95, axis=0)))),
                "checks": hs["checks"], "fallbacks": hs["fallbacks"], "clamped": hs["clamped"]})
    if log:
        log(f"hybrid: {1e3 * sec / nsteps:.3f} ms/step, rel L2 {e}, fallbacks {hs['fallbacks']}/{hs['checks']}")
    if baseline_net is not None:
        _, Qb, _ = run_h(baseline_net)
        eb = rel_l2(Qb, Qf)
        out["no_network_rel_l2"] = dict(zip(["rho", "Px", "Py", "Pw"], map(float, eb)))
        if log:
            log(f"without the network (coarse-only update in closure cells): rel L2 {eb}")
    return out


def zero_network(stream=None):
    """A network whose output is zero: closure cells then take the coarse-only update."""
    net = MLP(stream)
    net.set_params(np.zeros(39428, np.float32))
    net.set_norm(np.zeros(45, np.float32), np.ones(45, np.float32), np.zeros(4, np.float32),
                 np.ones(4, np.float32))
    return net
