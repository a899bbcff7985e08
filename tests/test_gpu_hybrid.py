"""Coarse-to-fine re-synchronisation and the DEM + closure hybrid step on the
GPU against compositions of the FP64 oracle (needs an MI355X).

Bars: re-synchronised floes within 1e-5 of the oracle's re-synchronisation;
after it, the cell's P and P_w on their targets up to the FP32 storage of the
velocities; a hybrid with no closure cell identical to the plain step; a
hybrid with closure cells within 1e-5 of the oracle composition (DEM cells:
oracle DEM + LF with the closure cells' <v> from their reduced DEMs; closure
cells: the base update of oracle/closure.py plus dt T, T from the bfloat16
reference network for the features of the base-updated state)."""
import numpy as np
import pytest

import fixtures
import oracle
from metrics import TOL, rel_err
from oracle import mlp as omlp
from oracle import closure as cref
from workloads import dense_workload

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2303_07819_amd")
torch = pytest.importorskip("torch")

# per-floe velocities of the DEM cells after 6 steps: a per-floe comparison
# (the stated 1e-5 covers per-cell moments), each floe's FP32 state rounded
# every step
TOL_FLOE = 5e-5
NET_TOL = 5e-4      # network kernel vs its bfloat16 reference, relative L2 (test_gpu_closure)


def _say(*a):
    print(*a, flush=True)


# ----------------------------------------------------------- re-synchronisation
def _targets(w, m, cells, factors):
    mom = oracle.moments(m, oracle.State.from_workload(w))
    Q = oracle.q_from_moments(m, mom)
    t = np.zeros((len(cells), 4))
    for i, c in enumerate(cells):
        rho = Q[c, 0]
        t[i] = [rho * factors[0], Q[c, 1] + factors[1] * rho, Q[c, 2] + factors[2] * rho,
                Q[c, 3] + factors[3] * rho]
    return t


# (rho factor, added <v> in m/s, added <v_y>, added P_w / rho in m^2/s); none asks a
# radius above the largest one, so nothing is clamped
@pytest.mark.parametrize("factors", [(0.97, 0.01, -0.005, 20.0), (0.999, 0.0, 0.0, 0.0),
                                     (0.5, -0.05, 0.03, -50.0)])
def test_resync_matches_oracle(factors):
    w = dense_workload(seed=31)
    m = oracle.Model(w)
    cells = [0, 2, 5]
    tg = _targets(w, m, cells, factors)
    _say(f"resync factors={factors} cells={cells}")
    with sp.Sim.from_workload(w) as s:
        clamped = s.resync_cells(cells, tg)
        f = s.read_floes()
        gm = s.read_moments(sp.MOMENTS_DEM)
    assert clamped == 0
    ost = oracle.State.from_workload(w)
    for i, c in enumerate(cells):
        oracle.resync_cell(m, ost, c, tg[i])
    touched = np.zeros(w.nfloes, bool)
    for c in cells:
        touched[w.start[c]:w.start[c + 1]] = True
    # cells not listed are untouched, bit for bit
    for k, a in (("u", w.u), ("v", w.v), ("omega", w.omega), ("r", w.r)):
        assert np.array_equal(f[k][~touched], a[~touched])
    assert np.array_equal(f["xi"], w.xi) and np.array_equal(f["yi"], w.yi)
    er = np.abs(f["r"][touched] - ost.r[touched]) / ost.r[touched]
    _say(f"  radius max rel err {er.max():.2e}")
    assert er.max() <= 2.0 ** -23
    for k, ref in (("u", ost.u), ("v", ost.v), ("omega", ost.w)):
        e = rel_err(f[k][touched][:, None], ref[touched][:, None])
        _say(f"  {k} max rel err {e.max():.2e}")
        assert e.max() <= TOL
    # the cell moments land on the targets (up to the FP32 storage of u, v, w, r)
    A = w.Lx * w.Ly
    st = w.start
    for i, c in enumerate(cells):
        sl = slice(st[c], st[c + 1])
        mass = 920.0 * w.h[sl].astype(np.float64) * np.pi * ost.r[sl] ** 2
        fl_p = 2.0 ** -22 * np.sum(mass * np.abs(ost.u[sl])) / A + 1e-12 * abs(tg[i, 1])
        fl_l = 2.0 ** -22 * np.sum(mass * ost.r[sl] ** 2 * np.abs(ost.w[sl])) / A + 1e-12 * abs(tg[i, 3])
        assert abs(gm[c, 1] / A - tg[i, 0]) <= 2.0 ** -21 * tg[i, 0]
        assert abs(gm[c, 2] / A - tg[i, 1]) <= 2 * fl_p + 1e-9 * tg[i, 0]
        assert abs(gm[c, 4] / A - tg[i, 3]) <= 2 * fl_l + 1e-12 * tg[i, 0]


def test_resync_clamps_at_the_search_radius():
    w = dense_workload(seed=32)
    m = oracle.Model(w)
    rmax = float(w.r.max())
    tg = _targets(w, m, [1, 3], (4.0, 0.02, 0.0, 0.0))
    with sp.Sim.from_workload(w) as s:
        clamped = s.resync_cells([1, 3], tg)
        f = s.read_floes()
        gm = s.read_moments(sp.MOMENTS_DEM)
    assert clamped == 2
    assert f["r"].max() <= rmax
    A = w.Lx * w.Ly
    for i, c in enumerate([1, 3]):
        sl = slice(w.start[c], w.start[c + 1])
        assert np.isclose(f["r"][sl].max(), rmax, rtol=2.0 ** -23)
        assert gm[c, 1] / A < tg[i, 0]
        mass = 920.0 * w.h[sl].astype(np.float64) * np.pi * f["r"][sl].astype(np.float64) ** 2
        fl_p = 2.0 ** -22 * np.sum(mass * np.abs(f["u"][sl])) / A
        assert abs(gm[c, 2] / A - tg[i, 1]) <= 2 * fl_p + 1e-9 * tg[i, 0]


def test_resync_rejects_bad_targets():
    w = fixtures.custom(3, 2, 25e3, [10, 0, 10, 10, 10, 10], seed=33, r_scale=0.3)
    with sp.Sim.from_workload(w) as s:
        before = s.read_floes()
        good = np.array([[0.3, 0.0, 0.0, 0.0]])
        for cells, tg in (([6], good), ([-1], good), ([0, 0], np.repeat(good, 2, 0)),
                          ([0], np.array([[0.0, 0, 0, 0]])), ([0], np.array([[np.nan, 0, 0, 0]])),
                          ([1], good)):
            with pytest.raises(sp.SpdemError) as ei:
                s.resync_cells(cells, tg)
            assert ei.value.status == -1
        assert s.resync_cells([1], np.zeros((1, 4))) == 0   # an empty cell with a zero target
        after = s.read_floes()
    for k in before:
        assert np.array_equal(before[k], after[k])


# ------------------------------------------------------------------ hybrid
def _net(seed, x_mean, x_std, y_mean, y_std, zero=False):
    th = np.zeros(omlp.NPARAMS, np.float32) if zero else fixtures.mlp_init(seed)
    if not zero:
        th = th + np.random.default_rng(seed).normal(0, 0.02, th.size).astype(np.float32)
    net = sp.MLP()
    net.set_params(th)
    net.set_norm(x_mean, x_std, y_mean, y_std)
    return net, th.astype(np.float64)


class _Ref:
    """Per-workload reference data of the closure (static cell data, ocean at
    the cell centres, reduced DEMs from the initial floes)."""

    def __init__(self, w):
        self.m = oracle.Model(w)
        st = oracle.State.from_workload(w)
        self.static = cref.cell_static(w)
        self.oce = cref.ocean_centres(w, self.m)
        self.red = cref.reduced_init(oracle.moments(self.m, st), self.static, self.oce, 0.0)
        self.Q0 = oracle.q_from_moments(self.m, oracle.moments(self.m, st))

    def base(self, w, Q, t):
        return cref.base_update(w, self.m, Q, w.dt, self.red, t, self.static, self.oce)

    def features(self, w, Q, cells, t):
        return cref.features(w, Q, cells, self.red, t, self.static, self.oce)


def _net_reference(th, x, x_mean, x_std, y_mean, y_std):
    """The network's output as the configuration stores it: inputs normalised
    in FP32 and rounded to bfloat16, products on bfloat16 operands."""
    x32 = x.astype(np.float32)
    inv = np.where(x_std > 0, np.float32(1.0) / np.maximum(x_std, np.float32(1e-30)), np.float32(0.0))
    xn = omlp.bf16((x32 - x_mean) * inv.astype(np.float32))
    y = omlp.forward(th, xn, bf16_mode=True)
    return y * y_std.astype(np.float64) + y_mean.astype(np.float64)


def _oracle_hybrid(w, closure, th, norm, nsteps):
    ref = _Ref(w)
    m = ref.m
    st = oracle.State.from_workload(w)
    Q = ref.Q0.copy()
    dem_cells = np.flatnonzero(~closure).astype(np.int32)
    clos_cells = np.flatnonzero(closure)
    Ts = []
    for k in range(nsteps):
        t = k * w.dt
        Qb = ref.base(w, Q, t)
        T = _net_reference(th, ref.features(w, Qb, clos_cells, t), *norm)
        Ts.append(T)
        mom_dem, _ = oracle.dem_steps(m, st, w.dt, 1, cells=dem_cells, record=True)
        mom = cref.reduced_moments(ref.red, ref.static, ref.oce, t, w.Lx * w.Ly)   # closure cells' <v>
        mom[dem_cells] = mom_dem[0]
        Qn, _ = oracle.lf_step(m, Q, mom, w.dt)
        for i, c in enumerate(clos_cells):
            Qn[c] = Qb[c] + w.dt * T[i]
        Q = Qn
    return st, Q, np.concatenate(Ts) if Ts else np.zeros((0, 4))


def _norm_for(w):
    """Input scaling from the initial features; an output scale giving
    dt |T| ~ 1e-4 of the continuum state."""
    ref = _Ref(w)
    Qb = ref.base(w, ref.Q0, 0.0)
    x = ref.features(w, Qb, range(w.ncells), 0.0)
    x_mean = x.mean(0).astype(np.float32)
    x_std = x.std(0).astype(np.float32)
    x_std[x_std < 1e-6 * (np.abs(x_mean) + 1e-30)] = 0.0
    q_rms = np.sqrt(np.mean(ref.Q0 ** 2, axis=0)) + 1e-30
    y_std = (1e-4 * q_rms / w.dt).astype(np.float32)
    y_mean = np.zeros(4, np.float32)
    return x_mean, x_std, y_mean, y_std


def test_hybrid_without_closure_cells_is_the_plain_step():
    w = dense_workload(seed=41)
    norm = _norm_for(w)
    net, _ = _net(3, *norm)
    with sp.Sim.from_workload(w) as a, sp.Sim.from_workload(w) as b:
        a.step(w.dt, 6)
        b.hybrid_set(net, np.zeros(w.ncells, bool), check_every=2, check_cells=4)
        b.step_hybrid(w.dt, 6)
        fa, fb = a.read_floes(), b.read_floes()
        qa, qb = a.read_moments(sp.MOMENTS_CONTINUUM), b.read_moments(sp.MOMENTS_CONTINUUM)
        hs = b.hybrid_stats()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    # the same continuum arithmetic, in a kernel of its own instead of fused
    _say(f"continuum bitwise equal: {np.array_equal(qa, qb)}")
    assert rel_err(qb, qa).max() <= 1e-13
    assert hs["dem_cells"] == w.ncells and hs["closure_cells"] == 0 and hs["checks"] == 0
    net.close()


def test_hybrid_constant_tendency_closure():
    """All cells on a network whose output is its output offset: Q advances by
    the base update plus dt y_mean, the floes do not move."""
    w = fixtures.custom(4, 3, 25e3, 30, seed=42, r_scale=0.3)
    c = np.array([1e-3, -2e-4, 3e-4, 5e-2], np.float32)
    net, _ = _net(0, np.zeros(45, np.float32), np.ones(45, np.float32), c, np.ones(4, np.float32), zero=True)
    ref = _Ref(w)
    Q = ref.Q0.copy()
    with sp.Sim.from_workload(w) as s:
        s.hybrid_set(net, np.ones(w.ncells, bool), check_every=1000, check_cells=0)   # no check pool
        s.step_hybrid(w.dt, 5)
        q = s.read_moments(sp.MOMENTS_CONTINUUM)
        f = s.read_floes()
        hs = s.hybrid_stats()
    for k in range(5):
        Q = ref.base(w, Q, k * w.dt) + w.dt * c.astype(np.float64)
    e = rel_err(q, Q)
    _say(f"constant tendency max rel err {e.max():.2e}")
    assert e.max() <= TOL
    assert np.array_equal(f["u"], w.u) and np.array_equal(f["xi"], w.xi)
    assert hs == {"dem_cells": 0, "closure_cells": w.ncells, "checks": 0, "fallbacks": 0}
    net.close()


@pytest.mark.parametrize("nsteps", [1, 6])
def test_hybrid_mixed_matches_oracle(nsteps):
    w = fixtures.custom(6, 5, 25e3, 40, seed=43, r_scale=fixtures.radius_scale(40, 25e3 ** 2, phi=0.3))
    rng = np.random.default_rng(43)
    w.u[:] = rng.normal(0, 0.1, w.nfloes)
    w.v[:] = rng.normal(0, 0.1, w.nfloes)
    closure = np.array([(c % w.nx + c // w.nx) % 3 == 0 for c in range(w.ncells)])
    norm = _norm_for(w)
    net, th = _net(5, *norm)
    _say(f"hybrid mixed: {closure.sum()} closure cells of {w.ncells}, {nsteps} steps")
    st, Q, Tref = _oracle_hybrid(w, closure, th, norm, nsteps)
    with sp.Sim.from_workload(w) as s:
        s.hybrid_set(net, closure, check_every=1000, check_cells=0)   # no check pool
        s.step_hybrid(w.dt, nsteps)
        q = s.read_moments(sp.MOMENTS_CONTINUUM)
        f = s.read_floes()
    e = rel_err(q, Q)
    # closure cells take dt T from the bfloat16 network each step, whose kernel
    # matches its bfloat16 reference to NET_TOL relative L2 (the accumulation
    # order differs): the allowance adds nsteps dt NET_TOL rms(T)
    rms = np.sqrt(np.mean(Q ** 2, axis=0))
    net_allow = nsteps * w.dt * NET_TOL * np.sqrt(np.mean(Tref ** 2, axis=0))
    ratio = np.abs(q - Q)[closure] / (TOL * np.maximum(np.abs(Q[closure]), 1e-3 * rms) + net_allow)
    _say(f"  continuum max rel err {e.max():.2e} (closure cells {e[closure].max():.2e}, error / allowance "
         f"{ratio.max():.2f}; DEM cells {e[~closure].max():.2e})")
    assert e[~closure].max() <= TOL, np.unravel_index(e.argmax(), e.shape)
    assert ratio.max() <= 1.0
    dem = np.zeros(w.nfloes, bool)
    for c in np.flatnonzero(~closure):
        dem[w.start[c]:w.start[c + 1]] = True
    # closure cells' floes are not stepped
    for k, a in (("u", w.u), ("xi", w.xi), ("omega", w.omega)):
        assert np.array_equal(f[k][~dem], a[~dem])
    ou = rel_err(f["u"][dem][:, None], st.u[dem][:, None])
    _say(f"  DEM-cell floe velocity max rel err {ou.max():.2e}")
    assert ou.max() <= TOL_FLOE
    net.close()


def test_hybrid_checks_and_fallback():
    """The check pool (up to 4 check_cells closure cells, spread evenly over the
    closure cells) keeps running the DEM: its floes equal the plain method's
    bit for bit at every step, while the other closure cells' floes stay
    frozen.  A tolerance nothing meets sends every checked cell to the DEM for
    fallback_steps steps."""
    w = fixtures.custom(6, 4, 25e3, 40, seed=44, r_scale=fixtures.radius_scale(40, 25e3 ** 2, phi=0.3))
    closure = np.zeros(w.ncells, bool)
    closure[::2] = True
    norm = list(_norm_for(w))
    nclos = int(closure.sum())
    order = np.flatnonzero(closure)
    net, _ = _net(6, *norm)
    with sp.Sim.from_workload(w) as s, sp.Sim.from_workload(w) as plain:
        s.hybrid_set(net, closure, check_every=3, check_cells=2, tol=1e30, fallback_steps=4)
        s.step_hybrid(w.dt, 9)
        hs = s.hybrid_stats()
        assert hs["checks"] == 6 and hs["fallbacks"] == 0 and hs["closure_cells"] == nclos
        f = s.read_floes()
        plain.step(w.dt, 9)
        g = plain.read_floes()
    # pool of 8 of the 12 closure cells: positions 12 i // 8
    pool = {int(order[12 * i // 8]) for i in range(8)}
    for c in range(w.ncells):
        sl = slice(w.start[c], w.start[c + 1])
        if not closure[c] or c in pool:   # DEM cells and the pool step as in the plain method
            for q in ("xi", "yi", "u", "v", "omega", "theta"):
                assert np.array_equal(f[q][sl], g[q][sl]), (c, q)
        else:                             # the other closure cells keep their initial floes
            assert np.array_equal(f["xi"][sl], w.xi[sl]) and np.array_equal(f["u"][sl], w.u[sl]), c
    net.close()
    net, _ = _net(6, *norm)
    base = w.ncells - nclos
    with sp.Sim.from_workload(w) as s:
        s.hybrid_set(net, closure, check_every=3, check_cells=5, tol=1e-30, fallback_steps=4)
        s.step_hybrid(w.dt, 3)   # check at step 3: five cells fall back for steps 4-7
        hs = s.hybrid_stats()
        assert hs["fallbacks"] == 5 and hs["dem_cells"] == base + 5, hs
        s.step_hybrid(w.dt, 3)   # check at step 6: five more
        hs = s.hybrid_stats()
        assert hs["fallbacks"] == 10 and hs["dem_cells"] == base + 10, hs
        s.step_hybrid(w.dt, 1)   # step 7: the first windows end
        hs = s.hybrid_stats()
        assert hs["fallbacks"] == 10 and hs["dem_cells"] == base + 5, hs
        s.hybrid_set(None, None)
    net.close()


@pytest.mark.parametrize("tol", [1e-30, 1e30])
def test_hybrid_blocked_equals_per_step(tol):
    """The hybrid's DEM cells run as blocked launches between checks and the
    ends of fallback windows: the same floes bit for bit as one launch per
    step, the same checks and fallbacks, the continuum within 1e-12 (the DEM
    statistics are summed in another fixed order)."""
    w = fixtures.custom(6, 4, 25e3, 40, seed=45, r_scale=fixtures.radius_scale(40, 25e3 ** 2, phi=0.3))
    rng = np.random.default_rng(45)
    w.u[:] = rng.normal(0, 0.1, w.nfloes)
    w.v[:] = rng.normal(0, 0.1, w.nfloes)
    closure = np.zeros(w.ncells, bool)
    closure[1::2] = True
    norm = list(_norm_for(w))
    out = []
    for k in (1, 8):
        net, _ = _net(7, *norm)
        with sp.Sim.from_workload(w) as s:
            s.set_step_block(k)
            s.hybrid_set(net, closure, check_every=5, check_cells=3, tol=tol, fallback_steps=4)
            s.step_hybrid(w.dt, 13)
            s.step_hybrid(w.dt, 9)
            out.append(dict(f=s.read_floes(), q=s.read_moments(sp.MOMENTS_CONTINUUM), hs=s.hybrid_stats(),
                            work=s.work()))
        net.close()
    a, b = out
    _say(f"tol {tol:g}: {b['hs']}, blocked steps {b['work']['blocked_steps']}")
    assert a["hs"] == b["hs"]
    assert b["work"]["blocked_steps"] > 0 and a["work"]["blocked_steps"] == 0
    for q in a["f"]:
        assert np.array_equal(a["f"][q], b["f"][q]), q
    e = rel_err(b["q"], a["q"], floor=1e-6)
    assert e.max() <= 1e-12, e.max()


def test_trained_closure_gains_over_the_reduced_dem_alone():
    """The network trained here as the benchmark trains it (samples of eight
    64 x 64 windows of the method's own DEM runs, 20 epochs) lowers the error
    of the hybrid against full DEM on a held-out window, compared with the same
    hybrid without it (the reduced DEMs alone): the momentum error over the
    relaxation transient (60 steps, by a factor 0.7 at least) and at the end
    of the network's window (400 steps).  The spin error is reported and held
    within 1.25 times the reduced DEMs' own at 400 steps: on this window the
    network does not lower it (measured 3.5 % against 3.1 %; on the 512 x 512
    grid it does, 8.9 % against 13.9 %)."""
    from paper_2303_07819_amd import closure as cl
    stream = torch.cuda.Stream()
    X, T = cl.training_set(stream=stream.cuda_stream)
    net, hist = cl.train(X, T, stream=stream.cuda_stream)
    _say(f"training: {hist['samples']} samples, held-out loss {hist['val'][-1]:.3f}")
    assert hist["val"][-1] < 0.8
    del X, T
    w = cl.training_workload(230307993)      # held out; 3456 of 4096 cells in the ice edge band
    dem = cl.miz_mask(w)
    zero = cl.zero_network(stream.cuda_stream)
    marks = (60, 400)
    full = cl._evolve(w, stream, max(marks), marks)
    with_net = cl._evolve(w, stream, max(marks), marks, net, dem, cl.NET_WINDOW_STEPS * w.dt)
    without = cl._evolve(w, stream, max(marks), marks, zero, dem, cl.NET_WINDOW_STEPS * w.dt)
    e = {mk: (cl.rel_l2(with_net[mk], full[mk]), cl.rel_l2(without[mk], full[mk])) for mk in marks}
    for mk in marks:
        _say(f"rel L2 after {mk} steps: with network {e[mk][0]}, without {e[mk][1]}")
    e_net, e_base = e[60]
    # mass moves by transport alone; the closure cells' <v> differs from the
    # DEM's number average only slightly
    assert e_net[0] <= 1e-4 and e_base[0] <= 1e-4
    assert max(e_net[1], e_net[2]) < 0.7 * max(e_base[1], e_base[2])
    e_net, e_base = e[400]
    assert max(e_net[1], e_net[2]) < 0.7 * max(e_base[1], e_base[2])
    assert e_net[3] <= 1.25 * e_base[3]
    net.close()
    zero.close()
