"""Learned closure: training data from the method's own DEM runs, training on
the GPU, and the DEM + closure hybrid measured against full DEM.

Everything here drives the C library (``Sim`` and ``MLP``); the arithmetic runs
in its kernels.  A closure cell replaces its DEM by a reduced DEM (the cell's
floes as one body relaxing towards the ocean under the drag laws, in closed
form) whose statistics drive the continuum update as the DEM's would, and the
network adds the residual: the part of the plain method's update the reduced
DEMs miss (the spread of floe thicknesses and velocities, contacts), as a
function of the base-updated continuum state around the cell, the ocean, three
static floe descriptors and the reduced DEM's relative velocity and spin.

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


def _torch_stream(stream):
    """A torch stream object for a raw stream handle (a new stream for None).

    The library's calls run on the stream they are given; torch's own work on
    the same tensors (allocation, indexing, noise, reductions) must run on that
    stream too, inside ``torch.cuda.stream(...)``, or the two race."""
    import torch
    return torch.cuda.Stream() if stream is None else torch.cuda.ExternalStream(stream)


def training_workload(seed: int, n: int = 64, nmax: int = 256, domain_cells: int = 512):
    """A 64 x 64 window of 25 km cells drawn from the recipe of a
    domain_cells x domain_cells grid: Poisson(nmax c) floes per cell with a
    marginal-ice-zone concentration c, radii scaled to area fraction 0.40 at
    nmax, 8 Fourier modes 2 <= |(p, q)| <= 16 on the whole domain, evaluated at
    the window's place in it; dt 30 s.  The window's continuum grid is
    periodic; its cells' DEMs are independent as in any grid."""
    import fixtures
    rng = np.random.Generator(np.random.PCG64(seed))
    L = 25e3
    D = domain_cells * L
    oc = fixtures.random_modes(rng, 8, D, D)
    c_all = fixtures.miz_concentration(rng, domain_cells, domain_cells)
    ox, oy = (int(v) for v in rng.integers(0, domain_cells - n + 1, 2))
    c = c_all[oy:oy + n, ox:ox + n].copy()
    # the window's origin moves to (0, 0): shift every mode's phase
    oc.phase = oc.phase + oc.kx * ox * L + oc.ky * oy * L
    counts = rng.poisson(nmax * c).astype(np.int32).reshape(-1)
    s = fixtures.radius_scale(nmax, L * L)
    xi, yi, r, h = fixtures.place_floes(counts, L, L, seed, s)
    z = np.zeros(xi.size, np.float32)
    return fixtures.Workload(f"window{seed}", n, n, L, L, 30.0, 2048, counts, xi, yi, z.copy(), z.copy(),
                             z.copy(), z.copy(), r, h, oc, G=5.0e3, conc=c)


NET_WINDOW_STEPS = 400   # the network acts during the first 400 steps of a reduced DEM


def sample_schedule(window: int = NET_WINDOW_STEPS, first: int = 24, count: int = 64):
    """Steps at which samples are taken, all inside the network's window: the
    first `first` steps one by one (the floes spin up from rest within a few
    tens of steps), the rest spread evenly up to the window's end."""
    rest = np.linspace(first, window - 1, count - first)
    return sorted(set(range(first)) | set(int(round(v)) for v in rest))


def generate_samples(workloads, schedule=None, stream=None, log=None):
    """(features, residual tendency) of every cell at the steps of `schedule`
    of a run of each workload from its initial state; device tensors [n, 45]
    and [n, 4]."""
    import torch
    ts = _torch_stream(stream)
    schedule = sample_schedule() if schedule is None else sorted(schedule)
    n = sum(w.ncells for w in workloads) * len(schedule)
    with torch.cuda.stream(ts):
        X = torch.empty((n, 45), device="cuda", dtype=torch.float32)
        T = torch.empty((n, 4), device="cuda", dtype=torch.float32)
    row = 0
    for w in workloads:
        t0 = time.perf_counter()
        with Sim.from_workload(w, stream=ts.cuda_stream) as s:
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
          stencil_noise: float = 1.0, use_stencil: bool = True, stream=None, log=None):
    """Adam on the bfloat16 network from Kaiming-uniform initial weights;
    normalisation from the training rows.  Every epoch sees the continuum
    stencil inputs (the first 36 features) with Gaussian noise of
    stencil_noise times each column's spread added: in the plain method a
    cell's residual comes from its own floes, and a network that leans on the
    continuum state it also drives feeds its own errors back (rollouts then
    diverge although one-step errors are small).  Returns (net, history) with
    the mean training loss per epoch and the held-out loss (normalised MSE,
    clean inputs).  With use_stencil False the stencil inputs are dropped
    (zero input scale)."""
    import torch
    ts = _torch_stream(stream)
    with torch.cuda.stream(ts):
        return _train(X, T, epochs, batch, lr, seed, holdout, stencil_noise, use_stencil, ts, log)


def _train(X, T, epochs, batch, lr, seed, holdout, stencil_noise, use_stencil, ts, log):
    import torch
    import fixtures
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    order = torch.as_tensor(rng.permutation(n))
    nval = int(n * holdout)
    val = order[:nval].to("cuda", torch.int32)
    tr = order[nval:]
    net = MLP(ts.cuda_stream)
    net.set_params(fixtures.mlp_init(seed))
    Xtr = X[tr.to("cuda")].contiguous()
    Ttr = T[tr.to("cuda")].contiguous()
    net.fit_norm(Xtr, Ttr)
    if not use_stencil:
        xm, xinv, ym, ys = net.get_norm()
        xs = np.where(xinv > 0, 1.0 / np.where(xinv > 0, xinv, 1.0), 0.0).astype(np.float32)
        xs[:36] = 0.0
        net.set_norm(xm, xs, ym, ys)
    hist = {"train": [], "val": [], "seconds": 0.0, "step_seconds": 0.0, "batch": batch}
    if stencil_noise > 0:
        # the training kernel adds the noise (stencil_noise times each stencil
        # column's spread over the training rows, from the fitted normalisation)
        _, xinv, _, _ = net.get_norm()
        spread = np.where(xinv[:36] > 0, 1.0 / np.where(xinv[:36] > 0, xinv[:36], 1.0), 0.0)
        net.set_input_noise((stencil_noise * spread).astype(np.float32), seed + 1)
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(Xtr.shape[0]).astype(np.int32), device="cuda")
        ts.synchronize()
        t_ep = time.perf_counter()
        hist["train"].append(net.train_epoch(Xtr, Ttr, perm, batch, lr))   # returns synchronised
        hist["step_seconds"] += time.perf_counter() - t_ep
        hist["val"].append(validation_loss(net, X, T, val))
        if log:
            log(f"epoch {ep + 1}: train {hist['train'][-1]:.4f} held-out {hist['val'][-1]:.4f}")
    torch.cuda.synchronize()
    hist["seconds"] = time.perf_counter() - t0
    net.set_input_noise(None)
    hist["samples"] = int(Xtr.shape[0])
    hist["steps"] = epochs * (int(Xtr.shape[0]) // batch)
    return net, hist


def validation_loss(net, X, T, rows, chunk: int = 1 << 17) -> float:
    """Mean squared error on normalised targets over the listed rows: the
    network's outputs (its forward kernel) compared with the targets on the
    host (rows gathered on the network's stream)."""
    import torch
    with torch.cuda.stream(_torch_stream(net.stream)):
        return _validation_loss(net, X, T, rows, chunk)


def _validation_loss(net, X, T, rows, chunk):
    import torch
    _, _, _, y_std = net.get_norm()
    ys = np.asarray(y_std, np.float64)
    tot, cnt = 0.0, 0
    for a in range(0, rows.numel(), chunk):
        idx = rows[a:a + chunk].long()
        x = X[idx].contiguous()
        y = torch.empty((idx.numel(), 4), device="cuda")
        net.forward(x, y)
        t = T[idx]
        torch.cuda.current_stream().synchronize()
        e = (y.cpu().numpy().astype(np.float64) - t.cpu().numpy().astype(np.float64)) / ys
        tot += float((e * e).sum())
        cnt += e.size
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


def training_set(seeds=range(8), stream=None, log=None):
    """Samples of eight 64 x 64 windows (about 2.1M cell-steps)."""
    ws = [training_workload(230307900 + k) for k in seeds]
    return generate_samples(ws, stream=stream, log=log)


def _evolve(w, stream, nsteps, marks, net=None, dem=None, window=0.0, check=(250, 0, 0.02, 100), timed=False):
    """Run full DEM (net None) or the hybrid for nsteps; continuum states at
    the marks (and the seconds of the whole run when timed, without reads)."""
    out = {}
    with Sim.from_workload(w, stream=stream.cuda_stream) as s:
        if net is not None:
            s.hybrid_set(net, ~dem, check[0], check[1], check[2], check[3], window)
        if timed:
            out["seconds"] = timed_run(s, w.dt, nsteps, net is not None, stream)
            out[nsteps] = s.read_moments(MOMENTS_CONTINUUM)
            if net is not None:
                out["stats"] = s.hybrid_stats()
            return out
        at = 0
        for mk in marks:
            if net is not None:
                s.step_hybrid(w.dt, mk - at)
            else:
                s.step(w.dt, mk - at)
            at = mk
            out[mk] = s.read_moments(MOMENTS_CONTINUUM)
    return out


def hybrid_experiment(w, net, nsteps: int, stream, marks=(10, 100, 400), window_steps: int = NET_WINDOW_STEPS,
                      check=(250, 256, 0.02, 100), curve_hi=(0.9, 1.01), log=None):
    """Full DEM, the hybrid with the network and the hybrid without it (the
    reduced DEMs alone), all from the same initial state.  Throughputs of
    nsteps-step runs, relative L2 errors against full DEM per component at
    nsteps and at the marks (short horizons), 95th-percentile per-cell errors.
    Also the speed / error curve of wider DEM bands (DEM iff MIZ_LO <= c <= hi
    for each hi of curve_hi, with and without the network) and of a fallback
    policy that keeps every cell whose check fails in DEM mode, and the distance
    between two full-DEM runs whose floes differ by one position unit (2^-32
    of the cell): how far the DEM's own continuum is determined by its
    initial state over the run."""
    import torch
    dem = miz_mask(w)
    names = ["rho", "Px", "Py", "Pw"]
    res = {"cells": w.ncells, "floes": w.nfloes, "steps": nsteps, "dem_cells": int(dem.sum()),
           "floes_in_dem_cells": int(w.counts[dem].sum()), "net_window_steps": window_steps}
    window = window_steps * w.dt
    zero = zero_network(stream.cuda_stream)
    # warm-up: kernels loaded, graph captured, network workspace sized
    _evolve(w, stream, 20, (20,))
    _evolve(w, stream, 20, (20,), net, dem, window)
    full = _evolve(w, stream, nsteps, (), timed=True)
    hyb = _evolve(w, stream, nsteps, (), net, dem, window, check, timed=True)
    base = _evolve(w, stream, nsteps, (), zero, dem, window, check, timed=True)
    Qf = full[nsteps]

    def errs(Q, ref):
        cell = np.abs(Q - ref) / np.maximum(np.abs(ref), 1e-3 * np.sqrt(np.mean(ref * ref, axis=0)))
        return (dict(zip(names, map(float, rel_l2(Q, ref)))),
                dict(zip(names, map(float, np.percentile(cell, 95, axis=0)))))

    res["full_dem_ms_per_step"] = 1e3 * full["seconds"] / nsteps
    res["full_dem_floe_steps_per_s"] = w.nfloes * nsteps / full["seconds"]
    res["hybrid_ms_per_step"] = 1e3 * hyb["seconds"] / nsteps
    res["hybrid_floe_steps_per_s"] = w.nfloes * nsteps / hyb["seconds"]
    res["speedup"] = full["seconds"] / hyb["seconds"]
    res["no_network_ms_per_step"] = 1e3 * base["seconds"] / nsteps
    res["rel_l2"], res["p95_cell_rel_err"] = errs(hyb[nsteps], Qf)
    res["no_network_rel_l2"], res["no_network_p95_cell_rel_err"] = errs(base[nsteps], Qf)
    res["checks"], res["fallbacks"] = hyb["stats"]["checks"], hyb["stats"]["fallbacks"]
    # short horizons (no checks, so that only the network differs)
    fm = _evolve(w, stream, max(marks), marks)
    hm = _evolve(w, stream, max(marks), marks, net, dem, window)
    bm = _evolve(w, stream, max(marks), marks, zero, dem, window)
    res["short_horizon_rel_l2"] = {str(mk): {"network": errs(hm[mk], fm[mk])[0],
                                             "no_network": errs(bm[mk], fm[mk])[0]} for mk in marks}
    c = np.asarray(w.conc).reshape(-1)
    curve = []
    for hi in curve_hi:
        band = (c >= MIZ_LO) & (c <= hi)
        for name, nt in (("network", net), ("no_network", zero)):
            h = _evolve(w, stream, nsteps, (), nt, band, window, check, timed=True)
            curve.append({"dem_band": [MIZ_LO, hi], "closure": name, "check_cells": check[1],
                          "fallback_steps": check[3],
                          "floes_in_dem_cells": float(w.counts[band].sum()) / w.nfloes,
                          "ms_per_step": 1e3 * h["seconds"] / nsteps, "speedup": full["seconds"] / h["seconds"],
                          "rel_l2": errs(h[nsteps], Qf)[0]})
    # fallback policy: a cell whose check fails stays in DEM mode for the rest
    # of the run, with the default number of checked cells and with sixteen
    # times as many (a check pool of four times that many cells)
    for ccells in (check[1], 16 * check[1]):
        pol = (check[0], ccells, check[2], nsteps)
        h = _evolve(w, stream, nsteps, (), net, dem, window, pol, timed=True)
        curve.append({"dem_band": [MIZ_LO, MIZ_HI], "closure": "network", "check_cells": ccells,
                      "fallback_steps": nsteps, "fallbacks": h["stats"]["fallbacks"],
                      "dem_cells_at_end": h["stats"]["dem_cells"],
                      "floes_in_dem_cells": float(w.counts[dem].sum()) / w.nfloes,
                      "ms_per_step": 1e3 * h["seconds"] / nsteps, "speedup": full["seconds"] / h["seconds"],
                      "rel_l2": errs(h[nsteps], Qf)[0]})
    res["curve"] = curve
    import copy
    w2 = copy.copy(w)
    w2.xi = (w.xi ^ np.uint32(1)).astype(np.uint32)
    twin = _evolve(w2, stream, nsteps, (nsteps,))[nsteps]
    res["full_dem_twin_rel_l2"] = errs(twin, Qf)[0]
    zero.close()
    if log:
        log(f"full DEM {res['full_dem_ms_per_step']:.3f} ms/step, hybrid {res['hybrid_ms_per_step']:.3f} ms/step "
            f"(x{res['speedup']:.2f}); rel L2 at {nsteps}: {res['rel_l2']}, without network "
            f"{res['no_network_rel_l2']}; short horizons {res['short_horizon_rel_l2']}")
    torch.cuda.synchronize()
    return res


def zero_network(stream=None):
    """A network whose output is zero: closure cells then take the coarse-only update."""
    net = MLP(stream)
    net.set_params(np.zeros(39428, np.float32))
    net.set_norm(np.zeros(45, np.float32), np.ones(45, np.float32), np.zeros(4, np.float32),
                 np.ones(4, np.float32))
    return net
