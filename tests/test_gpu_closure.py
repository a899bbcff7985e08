"""Closure network on the GPU (bfloat16 MFMA, FP32 accumulation) against the
FP64 reference of oracle/mlp.py, and the per-cell feature / tendency gather
against the oracle (needs an MI355X)."""
import math

import numpy as np
import pytest

import fixtures
import oracle
from metrics import rel_err
from oracle import closure as cref
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_2303_07819_amd")
torch = pytest.importorskip("torch")


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def _say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cosine(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def make_net(seed=1):
    rng = np.random.default_rng(seed)
    th = fixtures.mlp_init(seed)
    th = th + rng.normal(0, 0.02, th.size).astype(np.float32)   # nonzero biases
    net = sp.MLP()
    net.set_params(th)
    net.set_norm(np.zeros(45), np.ones(45), np.zeros(4), np.ones(4))
    return net, th.astype(np.float64)


@pytest.mark.parametrize("M", [1, 63, 300, 4096])
def test_forward_matches_reference(M):
    net, th = make_net(1)
    x = np.random.default_rng(M).normal(0, 1, (M, 45)).astype(np.float32)
    y = torch.zeros((M, 4), device="cuda")
    net.forward(dev(x), y)
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    ref16 = omlp.forward(th, x.astype(np.float64), bf16_mode=True)
    ref64 = omlp.forward(th, x.astype(np.float64))
    e16, e64 = rel_l2(got, ref16), rel_l2(got, ref64)
    _say(f"M={M}: rel L2 vs bf16 reference {e16:.2e}, vs FP64 {e64:.2e}")
    # bfloat16 reference: only FP32-vs-FP64 accumulation differs (an activation
    # occasionally rounds to the neighbouring bfloat16); FP64: the bfloat16 storage itself
    assert e16 <= 5e-4
    assert e64 <= 2e-2
    net.close()


def test_normalisation_is_applied():
    net, th = make_net(2)
    rng = np.random.default_rng(0)
    xm, xs = rng.normal(0, 3, 45), rng.uniform(0.5, 4, 45)
    ym, ys = rng.normal(0, 2, 4), rng.uniform(0.1, 3, 4)
    xs[7] = 0.0                                  # a dropped input
    net.set_norm(xm, xs, ym, ys)
    x = rng.normal(0, 1, (100, 45)) * xs + xm
    y = torch.zeros((100, 4), device="cuda")
    net.forward(dev(x), y)
    xn = np.where(xs > 0, (x - xm) / np.where(xs > 0, xs, 1), 0.0)
    ref = omlp.forward(th, xn, bf16_mode=True) * ys + ym
    e = rel_l2(y.cpu().numpy(), ref)
    _say(f"normalised forward rel L2 {e:.2e}")
    assert e <= 2e-3
    net.close()


@pytest.mark.parametrize("B", [512, 300, 7])
def test_gradient_matches_reference(B):
    # whole 256-row blocks, a ragged tail of 16-row tiles, and a batch below one tile
    net, th = make_net(3)
    rng = np.random.default_rng(1)
    x = rng.normal(0, 1, (B, 45)).astype(np.float32)
    t = rng.normal(0, 1, (B, 4)).astype(np.float32)
    g, loss = net.gradient(dev(x), dev(t))
    ref16 = omlp.grad(th, x.astype(np.float64), t.astype(np.float64), bf16_mode=True)
    ref64 = omlp.grad(th, x.astype(np.float64), t.astype(np.float64))
    assert loss == pytest.approx(omlp.loss(th, x.astype(np.float64), t.astype(np.float64), True), rel=1e-3)
    o = 0
    for name, shp in omlp.SHAPES:
        k = int(np.prod(shp))
        a, b16, b64 = g[o:o + k].astype(np.float64), ref16[o:o + k], ref64[o:o + k]
        _say(f"{name}: rel L2 vs bf16 ref {rel_l2(a, b16):.2e}, cos vs FP64 {cosine(a, b64):.5f}, "
             f"rel L2 vs FP64 {rel_l2(a, b64):.2e}")
        assert rel_l2(a, b16) <= 2e-3 and cosine(a, b16) >= 0.99999
        assert cosine(a, b64) >= 0.99 and rel_l2(a, b64) <= 5e-2
        o += k
    net.close()


def test_adam_step_matches_closed_form():
    net, th = make_net(4)
    rng = np.random.default_rng(2)
    B = 256
    x = dev(rng.normal(0, 1, (B, 45)))
    t = dev(rng.normal(0, 1, (B, 4)))
    g, _ = net.gradient(x, t)
    rows = dev(np.arange(B), torch.int32)
    net.train_step(x, t, rows, B, lr=1e-3)
    new = net.get_params().astype(np.float64)
    th32 = th.astype(np.float32).astype(np.float64)
    ref, _, _ = omlp.adam(th32, np.zeros_like(th32), np.zeros_like(th32), g.astype(np.float64), 1, lr=1e-3)
    np.testing.assert_allclose(new, ref, rtol=0, atol=2e-7)
    net.close()


def test_training_reduces_loss_on_a_smooth_target():
    net, _ = make_net(5)
    rng = np.random.default_rng(3)
    n = 8192
    x = rng.normal(0, 1, (n, 45)).astype(np.float32)
    t = np.stack([np.sin(x[:, 0]) + 0.5 * x[:, 1], x[:, 2] * x[:, 3], np.tanh(x[:, 4]), x[:, 5] ** 2],
                 axis=1).astype(np.float32)
    X, T = dev(x), dev(t)
    net.fit_norm(X, T)
    losses = []
    for ep in range(6):
        perm = dev(np.random.default_rng(ep).permutation(n), torch.int32)
        losses.append(net.train_epoch(X, T, perm, 512, lr=2e-3))
    _say("epoch losses", [f"{l:.4f}" for l in losses])
    assert losses[-1] < 0.3 * losses[0]
    net.close()


def test_features_and_tendencies_match_oracle():
    w = fixtures.custom(6, 5, 25e3, 40, seed=21, r_scale=fixtures.radius_scale(40, 25e3 ** 2, phi=0.3))
    w.counts[3] = 0
    w = fixtures.custom(6, 5, 25e3, w.counts, seed=21, r_scale=fixtures.radius_scale(40, 25e3 ** 2, phi=0.3))
    nsteps = 3
    _, Q0, _, _ = oracle.run_plain(w, nsteps)
    _, Q1, _, _ = oracle.run_plain(w, nsteps + 1)
    m = oracle.Model(w)
    with sp.Sim.from_workload(w) as s:
        s.step(w.dt, nsteps)
        x = torch.zeros((w.ncells, 45), device="cuda")
        t = torch.zeros((w.ncells, 4), device="cuda")
        s.closure_sample(w.dt, x, t)
        torch.cuda.synchronize()
        xs, ts = x.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
    static = cref.cell_static(w)
    oce = cref.ocean_centres(w, m)
    red = cref.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 0.0)
    ref = cref.features(w, Q0, range(w.ncells), red, nsteps * w.dt, static, oce)
    e = rel_err(xs, ref)
    _say(f"features max rel err {e.max():.2e}")
    assert e.max() <= 1e-5, np.unravel_index(e.argmax(), e.shape)
    tend = (Q1 - Q0) / w.dt
    et = np.abs(ts - tend) / np.maximum(np.abs(tend), 1e-2 * np.sqrt(np.mean(tend ** 2, axis=0)))
    _say(f"tendency max rel err {et.max():.2e}")
    assert et.max() <= 1e-3


def test_residual_tendencies_match_oracle():
    """Residual samples: the features of the base-updated state Q_b (every
    cell's statistics from its reduced DEM) and the targets (Q_new - Q_b) / dt."""
    w = fixtures.custom(5, 4, 25e3, 40, seed=22, r_scale=fixtures.radius_scale(40, 25e3 ** 2, phi=0.3))
    rng = np.random.default_rng(22)
    w.u[:] = rng.normal(0, 0.1, w.nfloes)
    w.v[:] = rng.normal(0, 0.1, w.nfloes)
    w.omega[:] = rng.normal(0, 1e-4, w.nfloes)
    nsteps = 2
    _, Q0, _, _ = oracle.run_plain(w, nsteps)
    _, Q1, _, _ = oracle.run_plain(w, nsteps + 1)
    m = oracle.Model(w)
    static = cref.cell_static(w)
    oce = cref.ocean_centres(w, m)
    red = cref.reduced_init(oracle.moments(m, oracle.State.from_workload(w)), static, oce, 0.0)
    Qb = cref.base_update(w, m, Q0, w.dt, red, nsteps * w.dt, static, oce)
    ref = (Q1 - Qb) / w.dt
    xref = cref.features(w, Qb, range(w.ncells), red, nsteps * w.dt, static, oce)
    with sp.Sim.from_workload(w) as s:
        s.step(w.dt, nsteps)
        x = torch.zeros((w.ncells, 45), device="cuda")
        t = torch.zeros((w.ncells, 4), device="cuda")
        s.closure_sample(w.dt, x, t, mode=sp.TEND_RESIDUAL)
        torch.cuda.synchronize()
        xs, ts = x.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
    ex = rel_err(xs, xref)
    _say(f"base-state features max rel err {ex.max():.2e}")
    assert ex.max() <= 1e-5, np.unravel_index(ex.argmax(), ex.shape)
    # the residual is the small part of the update: measure against its own scale
    e = np.abs(ts - ref) / np.maximum(np.abs(ref), 1e-2 * np.sqrt(np.mean(ref ** 2, axis=0)))
    _say(f"residual tendency max rel err {e.max():.2e}")
    assert e.max() <= 1e-3


# ------------------------------------------------------- training input noise
def _probe_net(f):
    """A network whose first output reproduces input f (weights 2^-10 into the
    first hidden unit, which GELU halves at such small arguments in each of
    the three layers, then 2^13 out) and whose other outputs are zero."""
    p = {n: np.zeros(s) for n, s in omlp.SHAPES}
    p["W1"][0, f] = 2.0 ** -10
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0
    p["W4"][0, 0] = 2.0 ** 13
    net = sp.MLP()
    net.set_params(omlp.pack(p).astype(np.float32))
    net.set_norm(np.zeros(45), np.ones(45), np.zeros(4), np.ones(4))
    return net


def test_training_input_noise_scale_and_repeatability():
    """sp_mlp_set_input_noise: with noise of scale s on input f only, the
    probe network's first output is the input plus that noise, so the loss a
    training step reports (before its update; lr far too small to move the
    weights) is s^2 / 4 of the four outputs, within the sampling spread of
    4096 rows (2.2 % for a mean of squared normals; bar 10 %).  Every step
    draws new noise, a second network with the same seed draws the same, and
    the plain gradient never sees noise."""
    f, B = 5, 4096
    rng = np.random.default_rng(7)
    x = rng.normal(0, 1, (B, 45)).astype(np.float32)
    t = np.zeros((B, 4), np.float32)
    t[:, 0] = x[:, f]
    X, T = dev(x), dev(t)
    losses = {}
    for s in (0.0, 1.0, 2.0):
        net = _probe_net(f)
        sd = np.zeros(36, np.float32)
        sd[f] = s
        net.set_input_noise(sd if s > 0 else None, seed=11)
        losses[s] = [net.train_step(X, T, None, B, 1e-30) for _ in range(4)]
        if s > 0:
            _, g_loss = net.gradient(X, T)
            assert g_loss < 1e-4                     # the gradient's inputs are clean
        net.close()
    _say(f"reported losses: {losses}")
    assert max(losses[0.0]) < 1e-4                   # the probe reproduces its input up to rounding
    for s in (1.0, 2.0):
        for ls in losses[s]:
            assert abs(ls / (s * s / 4.0) - 1.0) < 0.1
    assert len(set(losses[1.0])) == 4                # new noise in every Adam step
    net = _probe_net(f)
    sd = np.zeros(36, np.float32)
    sd[f] = 1.0
    net.set_input_noise(sd, seed=11)
    again = [net.train_step(X, T, None, B, 1e-30) for _ in range(4)]
    net.set_input_noise(sd, seed=12)
    other = net.train_step(X, T, None, B, 1e-30)
    net.close()
    assert again == losses[1.0]                      # the same seed repeats the same draws
    assert other != losses[1.0][0]


def test_training_input_noise_limits():
    net = sp.MLP()
    with pytest.raises(sp.SpdemError):
        net.set_input_noise(np.ones(46, np.float32))
    with pytest.raises(sp.SpdemError):
        net.set_input_noise(np.array([1.0, -1.0], np.float32))
    with pytest.raises(sp.SpdemError):
        net.set_input_noise(np.array([np.nan], np.float32))
    net.set_input_noise(None)
    net.close()
