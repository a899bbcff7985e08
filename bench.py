"""Throughput of the superparameterised floe DEM on one MI355X.

One step = one DEM step of every cell (contact detection, contact forces and
torques, ocean drag and torque, time update) fused with the FP64 cell
statistics, then one Lax-Friedrichs step of the continuum moments.  Default
workload: 64 x 64 cells of 25 km, 256 floes per cell (1,048,576 floes),
dt = 30 s, synthetic seeded fields.

Prints one JSON line.  `value` is floe-steps/s with the floe state resident in
HBM when timing starts; the roofline object covers the dominant kernel (the
DEM cell kernel), timed live with HIP events on the library's stream; the
CPU baseline is the FP64 oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_FLOE_STEP = 56      # read xi, yi, u, v, w, th, r, h; write xi, yi, u, v, w, th
BYTES_PER_CELL_STEP = 88      # the 11 FP64 cell statistics written
MFMA_BF16_PEAK_TFLOPS = 2500.0
# closure network 45 -> 128 -> 128 -> 128 -> 4: multiply-adds per sample of the
# forward pass, and of the backward pass (weight gradients of every layer,
# input gradients of the three upper layers)
MLP_FWD_MACS = 45 * 128 + 2 * 128 * 128 + 128 * 4
MLP_BWD_MACS = MLP_FWD_MACS + 2 * 128 * 128 + 128 * 4
TRAIN_FLOPS_PER_SAMPLE = 2 * (MLP_FWD_MACS + MLP_BWD_MACS)


def _cores():
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        cores = min(cores, int(omp))
    return cores


def _sample_cells(w, n, seed=7):
    import numpy as np
    rng = np.random.default_rng(seed)
    has = np.flatnonzero(w.counts > 0)
    return np.sort(rng.choice(has, min(n, has.size), replace=False)).astype(np.int32)


def _oracle_cells(w, cells, nsteps, threads, state=None, binned=True):
    """The oracle on the listed cells for nsteps from `state` (default the
    workload's): (seconds, floe-steps, moments of the listed cells, contacts,
    candidate pairs)."""
    import oracle
    oracle.set_threads(threads)
    m = oracle.Model(w, oracle.BINNED if binned else 0)
    st = (oracle.State.from_workload(w) if state is None else state.copy())
    t0 = time.perf_counter()
    _, stats = oracle.dem_steps(m, st, w.dt, nsteps, cells=cells)
    sec = time.perf_counter() - t0
    nfl = int(sum(int(w.counts[c]) for c in cells))
    return sec, nfl * nsteps, oracle.moments(m, st)[cells], int(stats[0]), int(stats[1])


STAT_NAMES = ["n", "M", "Px", "Py", "L", "Ux", "Uy", "Svx", "Svy", "Sw", "Aice"]


def _oracle_cells_stored(w, cells, nsteps, state=None):
    """The oracle on the listed cells with their floe state rounded after every
    step to the formats the GPU stores (positions to 2^-32 of the cell,
    velocities and spin to FP32): what the 32-bit storage alone changes.
    Returns the moments of the listed cells."""
    import numpy as np
    import oracle
    m = oracle.Model(w, oracle.BINNED)
    st = (oracle.State.from_workload(w) if state is None else state.copy())
    idx = np.concatenate([np.arange(w.start[c], w.start[c + 1]) for c in cells])
    for _ in range(nsteps):
        oracle.dem_steps(m, st, w.dt, 1, cells=cells)
        for a in (st.u, st.v, st.w):
            a[idx] = a[idx].astype(np.float32)
        for a in (st.xs, st.ys):
            a[idx] = np.round(a[idx] * 2.0 ** 32) / 2.0 ** 32 % 1.0
    return oracle.moments(m, st)[cells]


def _storage_floors(ref, stored, tol=1e-5, floor=1e-3, margin=5.0):
    """Per-statistic floor of the relative error: 1e-3 of the statistic's rms,
    raised where the storage-only deviation D would use more than 1 / margin of
    the allowance (floor margin D / (tol rms))."""
    import numpy as np
    rms = np.sqrt(np.mean(ref * ref, axis=0))
    dev = np.max(np.abs(stored - ref), axis=0)
    need = np.where(rms > 0, margin * dev / (tol * np.where(rms > 0, rms, 1.0)), 0.0)
    return np.maximum(floor, need)


def _moment_error(gm, ref, stored):
    """The GPU's per-cell statistics against the oracle's: the largest relative
    error at a floor of 1e-3 of each statistic's rms over the compared cells,
    the same per statistic, at the storage-derived floors (as the parity
    tests), and the storage-only deviation in units of the rms."""
    import numpy as np
    e_rel, e_abs = _rel_err(gm, ref)
    fl = _storage_floors(ref, stored)
    rms = np.sqrt(np.mean(ref * ref, axis=0))
    rmsd = np.where(rms > 0, rms, 1.0)
    per = {}
    for k, nm in enumerate(STAT_NAMES):
        a, _ = _rel_err(gm[:, k:k + 1], ref[:, k:k + 1])
        b, _ = _rel_err(gm[:, k:k + 1], ref[:, k:k + 1], fl[k])
        per[nm] = {"rel_err_floor_1e-3": a, "rel_err_storage_floor": b, "storage_floor": float(fl[k]),
                   "gpu_abs_err_per_rms": float(np.max(np.abs(gm[:, k] - ref[:, k])) / rmsd[k]),
                   "storage_abs_dev_per_rms": float(np.max(np.abs(stored[:, k] - ref[:, k])) / rmsd[k])}
    return {"max_rel_err": e_rel, "floor": 1e-3, "max_abs_err_per_rms": e_abs,
            "max_rel_err_storage_floors": max(v["rel_err_storage_floor"] for v in per.values()),
            "per_statistic": per}


def _rel_err(a, b, floor=1e-3):
    """Largest per-cell relative error with a floor of `floor` times the
    component's rms over the compared cells, and the largest absolute error in
    units of that rms."""
    import numpy as np
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    rms = np.sqrt(np.mean(b * b, axis=0, keepdims=True))
    den = np.maximum(np.abs(b), floor * rms)
    den = np.where(den > 0, den, 1.0)
    rmsd = np.where(rms > 0, rms, 1.0)
    return float(np.max(np.abs(a - b) / den)), float(np.max(np.abs(a - b) / rmsd))


def cpu_baseline(w, gm_after, nsteps, budget_s=10.0, dense=None, extra=None):
    """The FP64 oracle as it stands, timed on this host's cores on bounded
    samples of the workloads (cells are independent DEMs, so a sample of cells
    is a smaller instance of the same work), binned contact search (its
    sub-bin mode), OpenMP over cells.

    value: plain64 from t = 0 over the same steps the GPU took before the
    moments were read, on a sample of cells sized to about `budget_s` seconds
    on all cores; the same oracle run gives the GPU's moment error on those
    cells.  Also: one core, the brute-force search, the dense phase (from the
    GPU state after 5000 steps), the 4 x 4 small workload in full, samples of
    uneven128 and hybrid512."""
    import numpy as np
    import oracle
    cores = _cores()
    allc = oracle.set_threads(cores)
    # calibrate: one step of 64 sampled cells
    probe = _sample_cells(w, 64, seed=11)
    sec, fs, _, _, _ = _oracle_cells(w, probe, 1, cores)
    rate = fs / max(sec, 1e-4)
    ncell = int(max(16, min(w.ncells, budget_s * rate / (nsteps * float(w.counts.mean())))))
    cells = _sample_cells(w, ncell)
    sec, fs, ref, contacts, cands = _oracle_cells(w, cells, nsteps, cores)
    mcells = cells[: min(cells.size, 512)]
    me = _moment_error(gm_after[mcells], ref[: mcells.size], _oracle_cells_stored(w, mcells, nsteps))
    out = {"value": fs / sec, "unit": "floe-steps/s", "cores": allc, "kind": "oracle",
           "sample": f"{w.name}: {cells.size} of {w.ncells} cells ({fs // nsteps} floes), {nsteps} steps from t=0, "
                     f"binned contact search, FP64, OpenMP over cells on {allc} threads",
           "seconds": sec}
    moment_error = {"workload": w.name, "cells": int(mcells.size), "steps": nsteps,
                    "reference": "FP64 oracle on the sampled cells from the same initial state",
                    "statistics": "n, M, P, L, U, S_v, S_w, A_ice per cell (DEM moments)", **me}
    # one core, fewer cells
    c1 = cells[: max(8, cells.size // max(1, allc))]
    s1, f1, _, _, _ = _oracle_cells(w, c1, nsteps, 1)
    out["one_core"] = {"value": f1 / s1, "cores": 1, "sample": f"{c1.size} cells, {nsteps} steps"}
    # the oracle's brute-force search (every pair of a cell), all cores
    cb = cells[: max(8, cells.size // 8)]
    kb = max(1, min(nsteps, 5))
    sb, fb, _, _, _ = _oracle_cells(w, cb, kb, cores, binned=False)
    out["brute_force"] = {"value": fb / sb, "cores": allc, "sample": f"{cb.size} cells, {kb} steps"}
    legs = {}
    if dense is not None:
        dw, dfl, dsteps, dgm = dense
        dstate = oracle.State.from_fixed(dfl["xi"], dfl["yi"], dfl["u"], dfl["v"], dfl["omega"], dfl["theta"],
                                         dfl["r"], dw.h)
        dc = _sample_cells(dw, max(16, min(dw.ncells, cells.size)), seed=13)
        ds, dfs, dref, dcont, dcand = _oracle_cells(dw, dc, dsteps, cores, state=dstate)
        mc = dc[: min(dc.size, 512)]
        dme = _moment_error(dgm[mc], dref[: mc.size], _oracle_cells_stored(dw, mc, dsteps, state=dstate))
        legs["plain64_dense"] = {"value": dfs / ds, "cores": allc, "steps": dsteps,
                                 "sample": f"{dc.size} cells from the GPU state after 5000 steps",
                                 "contacts_per_floe_step": 2.0 * dcont / max(1, dfs),
                                 "moment_error": {"cells": int(mc.size), "steps": dsteps, **dme}}
    for name, ew, k, ncl in (extra or []):
        ec = _sample_cells(ew, ncl, seed=17)
        es, efs, _, _, _ = _oracle_cells(ew, ec, k, cores)
        legs[name] = {"value": efs / es, "cores": allc, "sample": f"{ec.size} of {ew.ncells} cells, {k} steps"}
    out["legs"] = legs
    oracle.set_threads(cores)
    return out, moment_error


PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "dem_block_kernel_plain64.md")
# the blocked kernel and the helpers it shares with the per-step kernel
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2303_07819_amd", "csrc", "dem_kernels.h"),
                  os.path.join(ROOT, "paper_2303_07819_amd", "csrc", "block_kernels.h")]
# VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one wave64 instruction occupies a SIMD for 4 cycles; non-packed FP32)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def valu_ops_per_floe_step(candidates_per_floe: float, contacts_per_floe: float) -> float:
    """Algorithmic VALU operations of one floe-step: 12 per candidate test, 70
    per contact, 160 for an 8-mode ocean, 50 for drag, update and statistics."""
    return 12.0 * candidates_per_floe + 70.0 * contacts_per_floe + 160.0 + 50.0


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        h.update(open(path, "rb").read())
    return h.hexdigest()


def copy_calibration(nbytes=1 << 30, reps=4):
    """A plain device copy of nbytes, reps times: FETCH_SIZE and WRITE_SIZE of
    its dispatches against nbytes give the scale of those counters."""
    import torch
    a = torch.ones(nbytes // 4, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def measured_traffic():
    """HBM bytes per DEM launch from the committed rocprofv3 counter summary,
    or None when the kernel source has changed since the counters were taken."""
    try:
        text = open(PROFILE_SUMMARY).read()
        src = kernel_source_hash()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "kernel_source_sha256")):
            k, v = line.strip().split(":", 1)
            parts = v.split("`")
            if len(parts) >= 3:
                vals[k.strip()] = parts[1]   # the first `quoted` value
    if vals.get("kernel_source_sha256") != src or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=512)      # 16 blocks of 32 steps
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--config", default="plain64")
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--step-block", type=int, default=0,
                    help="steps per DEM launch of the headline run (0: the library's default of 32; "
                         "1: one launch per step, replayed as captured graphs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=64)
    ap.add_argument("--no-hybrid", action="store_true",
                    help="skip training the closure and the DEM + closure run on the 512 x 512 grid")
    ap.add_argument("--hybrid-steps", type=int, default=2000)
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the autotuned run of the uneven 128 x 128 workload")
    ap.add_argument("--no-scenarios", action="store_true",
                    help="skip the error study of Sec. 4.1-4.4 against the global DEM")
    ap.add_argument("--no-coupled", action="store_true",
                    help="skip the plain64 run under the two-way coupling (N0 = 100, n_t = 10)")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the plain64 dense-phase run restored from a state saved after 5000 steps")
    ap.add_argument("--no-inference", action="store_true",
                    help="skip the closure inference timing on the 256 x 256 grid")
    ap.add_argument("--no-spring", action="store_true",
                    help="skip the plain64 run with the tangential spring (per-contact history)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of known size (for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--closure-probe", action="store_true",
                    help="only sample one 64 x 64 window and train the closure for two epochs (for counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.closure_probe:
        closure_probe()
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "cells would shard as 2-D blocks with a one-cell halo of coarse moments", file=sys.stderr)
        sys.exit(2)

    import torch
    import fixtures
    import paper_2303_07819_amd as sp

    print(f"bench: building workload {args.config}", file=sys.stderr, flush=True)
    w = fixtures.make_config(args.config)
    torch.cuda.init()
    stream = torch.cuda.Stream()          # default priority; handed to the library
    torch.cuda.set_stream(stream)
    sim = sp.Sim.from_workload(w, schedule=args.schedule, stream=stream.cuda_stream)
    if args.step_block > 0:
        sim.set_step_block(args.step_block)
    sched = sim.schedule()
    print(f"bench: {w.nfloes} floes in {w.ncells} cells, schedule {sched}", file=sys.stderr, flush=True)

    sim.step(w.dt, args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    work_before = sim.work()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(w.dt, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = w.nfloes * args.steps / (ms / 1e3)
    gm_after = sim.read_moments(sp.MOMENTS_DEM)       # judged against the oracle by the CPU leg
    work_timed = sim.work()
    roofline, contacts_per_floe_step = dem_roofline(sim, w, args.profile_steps)
    sim.close()

    out = {
        "metric": "floe-steps/sec at 1 GPU (plain DEM vs DEM+closure) at stated moment error",
        "value": value,
        "unit": "floe-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state (u32 fixed-point positions), f64 contact geometry and moment sums",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": [w.nx, w.ny], "cell_km": w.Lx / 1e3,
                   "floes": w.nfloes, "floes_per_cell": float(w.nfloes) / w.ncells, "dt_s": w.dt,
                   "schedule": ["auto", "allpairs", "binned"][sched[0]], "sub_bins": [sched[1], sched[2]],
                   "continuum": "lax-friedrichs every step", "step_block": roofline.get("steps_per_launch", 1),
                   "blocked_steps_timed": work_timed["blocked_steps"] - work_before["blocked_steps"]},
        "roofline": roofline,
        "moment_error": None,
        "contacts_per_floe_step": contacts_per_floe_step,
        "wall_s_timed": wall,
    }
    built = {}
    dense = None
    if not args.no_dense:
        out["dense"], dense = dense_leg(stream, w, args.profile_steps)
    if not args.no_uneven:
        out["uneven"], built["uneven128"] = uneven_leg(stream)
    if not args.no_inference:
        out["inference"] = inference_leg(stream)
    if not args.no_coupled:
        out["coupled"] = coupled_leg(stream)
    if not args.no_spring:
        out["spring"] = spring_leg(stream)
    if not args.no_scenarios:
        out["scenarios"] = scenario_leg(stream)
    if not args.no_hybrid:
        out["hybrid"], built["hybrid512"] = hybrid_leg(args, stream)
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        extra = [("small", fixtures.make_config(0), 1000, 16)]
        if "uneven128" in built:
            extra.append(("uneven128", built["uneven128"], 10, 256))
        if "hybrid512" in built:
            extra.append(("hybrid512", built["hybrid512"], 10, 1024))
        out["cpu_baseline"], out["moment_error"] = cpu_baseline(w, gm_after, args.warmup + args.steps, dense=dense,
                                                                extra=extra)
    print(json.dumps(out), flush=True)


def dem_roofline(sim, w, profile_steps):
    """The dominant kernel timed live with HIP events on its stream (blocked
    steps: events around every block's DEM launch) over `profile_steps` more
    steps, its work counted over the same steps: (roofline object, contacts
    per floe-step)."""
    k_block, blocked = sim.step_block()
    st0, wk0 = sim.stats(), sim.work()
    dem_ms, lf_ms = sim.profile_steps(w.dt, profile_steps)   # whole blocks when blocked
    st1, wk1 = sim.stats(), sim.work()
    dsteps = st1["steps"] - st0["steps"]
    contacts_per_floe_step = (st1["contacts"] - st0["contacts"]) * 2.0 / max(1, w.nfloes * dsteps)
    candidates_per_floe_step = (wk1["candidate_tests"] - wk0["candidate_tests"]) / max(
        1, w.nfloes * (wk1["blocked_steps"] - wk0["blocked_steps"]))
    if blocked:
        # floes resident in LDS for k_block steps: VALU binds (state read and
        # written once per launch, statistics every step)
        ops = valu_ops_per_floe_step(candidates_per_floe_step, contacts_per_floe_step)
        tops = ops * w.nfloes / (dem_ms * 1e-3) / 1e12
        bytes_step = BYTES_PER_FLOE_STEP * w.nfloes / k_block + BYTES_PER_CELL_STEP * w.ncells
        roofline = {"bound": "alu", "kernel": "dem_block_kernel", "achieved": tops, "peak": VALU_PEAK_TOPS,
                    "unit": "TFLOP/s", "frac": tops / VALU_PEAK_TOPS, "traffic": measured_traffic(),
                    "kernel_ms": dem_ms * k_block, "steps_per_launch": k_block, "lf_ms_per_step": lf_ms,
                    "ops_per_floe_step": ops, "candidates_per_floe_step": candidates_per_floe_step,
                    "contacts_per_floe_step": contacts_per_floe_step,
                    "algorithmic_ops_per_launch": ops * w.nfloes * k_block,
                    "hbm": {"algorithmic_bytes_per_launch": bytes_step * k_block,
                            "achieved_GBs": bytes_step / (dem_ms * 1e-3) / 1e9,
                            "frac": bytes_step / (dem_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    else:
        bytes_launch = BYTES_PER_FLOE_STEP * w.nfloes + BYTES_PER_CELL_STEP * w.ncells
        achieved = bytes_launch / (dem_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": "dem_step_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel_ms": dem_ms,
                    "lf_kernel_ms": lf_ms, "algorithmic_bytes_per_launch": bytes_launch}
    return roofline, contacts_per_floe_step


def dense_leg(stream, w, profile_steps, pre=5000, steps=512, check_steps=10):
    """plain64 in its dense-contact phase: `pre` steps from t = 0, saved with
    sp_save; a fresh context restored from the file (sp_load) is timed over
    `steps` steps with HIP events and profiled like the headline; another
    restored context steps `check_steps` for the CPU leg's moment check
    (returned with the floes at the restored state)."""
    import tempfile
    import torch
    import paper_2303_07819_amd as sp
    path = os.path.join(tempfile.mkdtemp(prefix="spdem_"), "plain64_dense.spdem")
    with sp.Sim.from_workload(w, stream=stream.cuda_stream) as sim:
        sim.step(w.dt, pre)
        sim.save(path)
        cont0 = sim.stats()["contacts"]
    with sp.Sim.from_workload(w, stream=stream.cuda_stream) as sim:
        sim.load(path)
        floes = sim.read_floes()
        sim.step(w.dt, check_steps)
        gm = sim.read_moments(sp.MOMENTS_DEM)
    with sp.Sim.from_workload(w, stream=stream.cuda_stream) as sim:
        sim.load(path)
        sim.step(w.dt, 32)
        sim.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(w.dt, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        roofline, cpf = dem_roofline(sim, w, profile_steps)
    os.remove(path)
    res = {"workload": w.name, "restored_from_step": pre, "steps": steps, "ms_per_step": ms,
           "floe_steps_per_s": w.nfloes / (ms * 1e-3), "contacts_per_floe_step": cpf,
           "candidates_per_floe_step": roofline.get("candidates_per_floe_step"),
           "contacts_first_5000_steps": cont0, "roofline": roofline}
    return res, (w, floes, check_steps, gm)


def inference_leg(stream, reps=20):
    """Closure inference on the 256 x 256 grid (65,536 cells, 256 floes per
    cell): the 45 inputs of every cell (sp_closure_features) and the fused
    bfloat16 MFMA forward (sp_mlp_forward), timed with HIP events over `reps`
    repetitions; the network has its initial (Kaiming-uniform) weights, which
    do not change the work."""
    import numpy as np
    import torch
    import fixtures
    import paper_2303_07819_amd as sp
    w = fixtures.make_config("closure256")
    with sp.Sim.from_workload(w, stream=stream.cuda_stream) as sim, sp.MLP(stream=stream.cuda_stream) as net:
        net.set_params(fixtures.mlp_init(230307904))
        net.set_norm(np.zeros(45, np.float32), np.ones(45, np.float32), np.zeros(4, np.float32),
                     np.ones(4, np.float32))
        with torch.cuda.stream(stream):
            X = torch.empty((w.ncells, 45), device="cuda", dtype=torch.float32)
            y = torch.empty((w.ncells, 4), device="cuda", dtype=torch.float32)
        sim.closure_features(X)
        net.forward(X, y)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        for _ in range(reps):
            sim.closure_features(X)
        ev[1].record(stream)
        for _ in range(reps):
            net.forward(X, y)
        ev[2].record(stream)
        torch.cuda.synchronize()
        feat_us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
        fwd_us = ev[1].elapsed_time(ev[2]) * 1e3 / reps
    flops = 2 * MLP_FWD_MACS * w.ncells
    return {"workload": "closure256", "cells": w.ncells, "features_us": feat_us, "forward_us": fwd_us,
            "cells_per_s": w.ncells / ((feat_us + fwd_us) * 1e-6),
            "mfma_roofline": {"bound": "mfma", "kernel": "mlp_forward_kernel", "achieved": flops / fwd_us / 1e6,
                              "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": flops / fwd_us / 1e6 / MFMA_BF16_PEAK_TFLOPS}}


def uneven_leg(stream, steps=500, warmup=20):
    """The uneven 128 x 128 workload (Poisson counts, 0 to about 700 floes per
    cell): default batching, then the autotuner's choice, each timed with HIP
    events over the same `steps` steps from the same state (saved after
    `warmup` steps and restored for the tuned run)."""
    import tempfile
    import torch
    import fixtures
    import paper_2303_07819_amd as sp
    w = fixtures.make_config("uneven128")
    path = os.path.join(tempfile.mkdtemp(prefix="spdem_"), "uneven128.spdem")

    def timed(sim):
        sim.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(w.dt, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    with sp.Sim.from_workload(w, stream=stream.cuda_stream) as sim:
        sim.step(w.dt, warmup)
        sim.save(path)
        ms_default = timed(sim)
        cells, _, _ = sim.batching()
        bw0, k0 = sim.block_waves(), sim.step_block()[0]
        sim.load(path)
        best = sim.autotune(w.dt, 5)
        ms_tuned = timed(sim)
        bw, k = sim.block_waves(), sim.step_block()[0]
    os.remove(path)
    return {"workload": "uneven128", "cells": [w.nx, w.ny], "floes": w.nfloes, "steps": steps,
            "bucket_cells": cells.tolist(), "tuned": "blocked kernel: wavefronts per cell per bucket, block length",
            "default_block_waves": bw0.tolist(), "default_step_block": k0, "default_ms_per_step": ms_default,
            "tuned_block_waves": bw.tolist(), "tuned_step_block": k, "tuner_best_ms_per_step": best,
            "tuned_ms_per_step": ms_tuned, "floe_steps_per_s": w.nfloes / (ms_tuned * 1e-3)}, w


def coupled_leg(stream, N0=100, N1=1, n_t=10, windows=5):
    """plain64 under the two-way coupling at the paper's default cadence
    (N0 = 100 fine steps per coarse step, gradual updates every n_t = 10):
    the first coarse step untimed, then `windows` coarse steps timed with HIP
    events (their fine steps, coarse steps and coarse-to-fine updates)."""
    import torch
    import fixtures
    import paper_2303_07819_amd as sp
    w = fixtures.make_config("plain64")
    steps = windows * N0
    with sp.Sim.from_workload(w, stream=stream.cuda_stream) as sim:
        sim.set_coupling(N0, N1, n_t)
        sim.step(w.dt, N0)
        sim.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(w.dt, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        cp = sim.coupling()
        cfl = sim.stats()["max_cfl"]
    return {"workload": "plain64", "N0": N0, "N1": N1, "n_t": n_t, "steps": steps, "ms_per_step": ms,
            "floe_steps_per_s": w.nfloes / (ms * 1e-3), "nudge_passes": cp["nudges"],
            "clamped_cell_updates": cp["clamped"], "invalid_cell_updates": cp["invalid"], "max_cfl": cfl}


def spring_leg(stream, steps=200, warmup=20, G_shear=80.0):
    """plain64 with the tangential force as the incremental spring
    (SP_TANGENTIAL_SPRING, G read as a shear modulus of 80 N/m^2): every floe's
    contact history read and rewritten with its contacts, in blocked launches
    of 32 steps (history staged in LDS) and in one launch per step, each timed
    with HIP events over `steps` steps after `warmup`; dem_ms from the
    library's own events around the DEM launches."""
    import torch
    import fixtures
    import paper_2303_07819_amd as sp
    w = fixtures.make_config("plain64")
    w.G = G_shear
    out = {"workload": "plain64", "G_shear": G_shear, "steps": steps}
    for name, k in (("blocked", 32), ("per_step", 1)):
        with sp.Sim.from_workload(w, flags=sp.SP_TANGENTIAL_SPRING, stream=stream.cuda_stream) as sim:
            sim.set_step_block(k)
            sim.step(w.dt, warmup)
            sim.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sim.step(w.dt, steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            dem_ms, _ = sim.profile_steps(w.dt, 32)
            out[name] = {"step_block": k, "ms_per_step": ms, "dem_kernel_ms_per_step": dem_ms,
                         "floe_steps_per_s": w.nfloes / (ms * 1e-3), "contacts_total": sim.stats()["contacts"]}
    return out


def scenario_leg(stream, ks=(1, 2, 3, 4)):
    """The paper's error study (Sec. 4.1-4.4): the superparameterised model at
    N0 = 100, n_t = 10 on 24 x 12, 48 x 24 and 96 x 48 coarse grids against the
    global DEM of the same 115,200 floes, L^2 errors at T = 0.2 and 1 (and 0.6
    for the wall scenario 4.4, whose walls are SP_WALL_X in both models)."""
    from paper_2303_07819_amd import scenarios
    out = {}
    for k in ks:
        times = (0.2, 0.6, 1.0) if k == 4 else (0.2, 1.0)
        r = scenarios.study(k, times=times, stream=stream.cuda_stream)
        g = r["global_dem"]
        out[r["scenario"]] = {"grids": r["grids"], "dX": r["dX"], "l2_conc": r["l2"]["conc"],
                              "l2_vx": r["l2"]["vx"], "order_conc": r["order"]["conc"],
                              "order_vx": r["order"]["vx"],
                              "global_dem": {"floes": r["floes"], "steps": g["steps"], "seconds": g["seconds"],
                                             "contacts": g["contacts"],
                                             "floe_steps_per_s": r["floes"] * g["steps"] / g["seconds"]}}
    return out


def training_rate(hist):
    """Closure training throughput against the bfloat16 MFMA peak."""
    flops = hist["steps"] * hist["batch"] * TRAIN_FLOPS_PER_SAMPLE
    tf = flops / max(hist["step_seconds"], 1e-12) / 1e12
    return {"bound": "mfma", "kernel": "closure training (Adam steps)", "flops": flops,
            "seconds": hist["step_seconds"], "achieved": tf, "peak": MFMA_BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": tf / MFMA_BF16_PEAK_TFLOPS}


def closure_probe():
    """One 64 x 64 window sampled, two epochs of training, then the fused
    inference forward over every sample (for rocprofv3 counters)."""
    import torch
    from paper_2303_07819_amd import closure as cl
    stream = torch.cuda.Stream()
    X, T = cl.generate_samples([cl.training_workload(230307900)], stream=stream.cuda_stream)
    net, hist = cl.train(X, T, epochs=2, stream=stream.cuda_stream)
    inf = {}
    for rows in (X.shape[0], 65536):          # the whole window, and the 256 x 256 grid's row count
        with torch.cuda.stream(stream):
            Xr = X[:rows]
            y = torch.empty((rows, 4), device="cuda")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            net.forward(Xr, y)                # weight tiles staged once
            e0.record(stream)
            net.forward(Xr, y)
            e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3
        flops = 2 * MLP_FWD_MACS * rows
        inf[str(rows)] = {"rows": int(rows), "us": us, "achieved": flops / us / 1e6, "unit": "TFLOP/s",
                          "peak": MFMA_BF16_PEAK_TFLOPS, "frac": flops / us / 1e6 / MFMA_BF16_PEAK_TFLOPS}
    net.close()
    print(json.dumps({"closure_probe": {
        "samples": hist["samples"], "adam_steps": hist["steps"], "seconds": hist["seconds"],
        "training": training_rate(hist), "inference": inf}}), flush=True)


def hybrid_leg(args, stream):
    """Plain DEM vs DEM + closure on the 512 x 512 grid (33.6M floes): the
    closure is trained here, on the GPU, from the method's own runs."""
    import time as _t
    import torch
    import fixtures
    from paper_2303_07819_amd import closure as cl

    def log(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    t0 = _t.perf_counter()
    X, T = cl.training_set(stream=stream.cuda_stream, log=log)
    t1 = _t.perf_counter()
    net, hist = cl.train(X, T, stream=stream.cuda_stream, log=log)
    del X, T
    torch.cuda.empty_cache()
    w = fixtures.make_config("hybrid512")
    log(f"hybrid512: {w.nfloes} floes in {w.ncells} cells")
    res = cl.hybrid_experiment(w, net, args.hybrid_steps, stream, log=log)
    net.close()
    res["training"] = {"samples": hist["samples"], "epochs": len(hist["train"]), "adam_steps": hist["steps"],
                       "seconds": hist["seconds"], "sampling_seconds": t1 - t0,
                       "final_train_loss": hist["train"][-1], "held_out_loss": hist["val"][-1],
                       "mfma_roofline": training_rate(hist)}
    res["workload"] = "hybrid512"
    res["metric"] = "floe-steps/s, plain DEM vs DEM + closure, relative L2 moment error vs full DEM"
    return res, w


if __name__ == "__main__":
    main()
