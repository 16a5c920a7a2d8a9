"""Pins of the oracle's driving (Sec. 3.1 of arXiv 1602.09079) and of the
closure support routines (restriction, MLP, Adam), which are not in the paper."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_1602_09079_amd import synth

G = 5.0 / 3.0


def test_forcing_mode_set():
    m = synth.forcing_modes(1.0, 3.0)
    assert len(m) == 43  # 86 modes with their conjugates
    kk = (m.astype(float) ** 2).sum(1)
    assert set(kk.tolist()) == {2.0, 3.0, 4.0, 5.0, 6.0, 8.0}


def test_ou_projection_is_solenoidal_and_shaped():
    nvec = synth.forcing_modes()
    th = synth.ou_stationary_start(1602, len(nvec))
    z = synth.ou_normals(1602, len(nvec), 1)[0]
    th1, ahat = O.ou_update(nvec, th, z, f=0.9, sigma=1.0, a0=2.0, kmin=1.0, kmax=3.0)
    for part in (0, 1):
        dot = (ahat[:, :, part] * nvec).sum(1)
        assert np.abs(dot).max() < 1e-14
    # paraboloid profile: |n| = 2 has the full amplitude, the ratio |ahat|/|P theta| follows 1 - (|n| - 2)^2
    kn = np.sqrt((nvec.astype(float) ** 2).sum(1))
    for j in range(len(nvec)):
        n = nvec[j] / kn[j]
        P = np.eye(3) - np.outer(n, n)
        want = 2.0 * max(0.0, 1 - (kn[j] - 2) ** 2) * (P @ th1[j])
        np.testing.assert_allclose(ahat[j], want, atol=1e-14)


def test_ou_statistics():
    """<theta> = 0 and <theta_t theta_{t+dt}> = sigma^2 f (Sec. 3.1), sampled."""
    nvec = np.array([[1, 1, 0]], dtype=np.int32)
    f, sigma = 0.8, 1.5
    nup = 20000
    z = synth.ou_normals(3, 1, nup)
    th = synth.ou_stationary_start(3, 1) * sigma
    seq = np.empty((nup, 6))
    for t in range(nup):
        th, _ = O.ou_update(nvec, th, z[t], f=f, sigma=sigma, a0=1.0, kmin=1.0, kmax=3.0)
        seq[t] = th.ravel()
    x = seq.ravel()
    assert abs(x.mean()) < 5 * sigma / math.sqrt(len(x)) * math.sqrt((1 + f) / (1 - f))
    assert x.var() == pytest.approx(sigma ** 2, rel=0.05)
    lag = (seq[1:] * seq[:-1]).mean()
    assert lag == pytest.approx(sigma ** 2 * f, rel=0.05)


def test_accel_is_real_and_divergence_free():
    nvec = synth.forcing_modes()
    th = synth.ou_stationary_start(1602, len(nvec))
    z = synth.ou_normals(1602, len(nvec), 1)[0]
    _, ahat = O.ou_update(nvec, th, z, f=0.9, sigma=1.0, a0=1.0, kmin=1.0, kmax=3.0)
    frc = O.ForcingTable(nvec, ahat)
    box = np.array([1.0, 1.0, 1.0])
    rng = np.random.default_rng(2)
    h = 1e-5
    for _ in range(5):
        x = rng.uniform(0, 1, 3)
        div = 0.0
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            div += (O.accel(frc, box, x + e)[a] - O.accel(frc, box, x - e)[a]) / (2 * h)
        assert abs(div) < 1e-6
    # a single mode against its closed form
    one = O.ForcingTable(np.array([[1, 2, 0]], dtype=np.int32), np.array([[[0.3, -0.1], [0.0, 0.2], [0.5, 0.0]]]))
    x = np.array([0.1, 0.3, 0.7])
    th = 2 * math.pi * (0.1 + 0.6)
    want = [0.3 * math.cos(th) + 0.1 * math.sin(th), -0.2 * math.sin(th), 0.5 * math.cos(th)]
    np.testing.assert_allclose(O.accel(one, box, x), want, atol=1e-15)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_constant_acceleration_source(k):
    """A constant acceleration (the n = 0 mode) on a uniform gas: R_m = -rho a,
    R_E = -m.a in the mean rows only (Sec. 3.1, source projected with the volume rule)."""
    nc = 3
    cfg = O.make_cfg(k, nc)
    x = O.gauss_legendre(k + 1)[0]
    vel = (0.2, -0.1, 0.3)
    y = O.project(cfg, synth.uniform_state(nc, x, rho=1.5, vel=vel, p=1.0))
    a = np.array([0.4, -0.7, 0.25])
    frc = O.ForcingTable(np.zeros((1, 3), dtype=np.int32), np.stack([a, np.zeros(3)], axis=1)[None])
    r = O.rhs(cfg, y, frc)
    for c in range(3):
        np.testing.assert_allclose(r[1 + c, 0], -1.5 * a[c], atol=1e-13)
    np.testing.assert_allclose(r[4, 0], -1.5 * np.dot(vel, a), atol=1e-13)
    if k > 0:
        assert np.abs(r[:, 1:]).max() < 1e-12
    assert np.abs(r[0]).max() < 1e-12


# ------------------------------------------------------------------ restriction

def test_restriction_exact_for_linears_and_conservative():
    kf, kc, nc = 2, 1, 3
    xf = O.gauss_legendre(kf + 1)[0]
    cf = O.make_cfg(kf, 2 * nc)
    yf = O.project(cf, synth.turbulence(2 * nc, xf, seed=5, kmax=2).numpy())
    yc = O.restrict(kf, kc, nc, yf)
    ccfg = O.make_cfg(kc, nc)
    np.testing.assert_allclose(O.totals(ccfg, yc), O.totals(cf, yf), rtol=1e-13, atol=1e-15)
    # restriction of a globally linear-in-cell field equals its direct coarse projection
    rng = np.random.default_rng(3)
    A = rng.standard_normal((5, 4))
    def lin(ncell, x):
        n = len(x)
        out = np.zeros((5, n, n, n, ncell, ncell, ncell))
        h = 1.0 / ncell
        for c, b, a in itertools.product(range(n), repeat=3):
            X = (np.arange(ncell)[None, None, :] + 0.5 * (1 + x[a])) * h
            Y = (np.arange(ncell)[None, :, None] + 0.5 * (1 + x[b])) * h
            Z = (np.arange(ncell)[:, None, None] + 0.5 * (1 + x[c])) * h
            for i in range(5):
                out[i, c, b, a] = A[i, 0] + A[i, 1] * X + A[i, 2] * Y + A[i, 3] * Z
        return out
    yf = O.project(cf, lin(2 * nc, xf))
    yc = O.restrict(kf, kc, nc, yf)
    yd = O.project(ccfg, lin(nc, O.gauss_legendre(kc + 1)[0]))
    np.testing.assert_allclose(yc, yd, atol=1e-13)
    # cell means of the coarse state are the averages of the children's means
    yf = O.project(cf, synth.turbulence(2 * nc, xf, seed=6, kmax=2).numpy())
    yc = O.restrict(kf, kc, nc, yf)
    m = yf[:, 0].reshape(5, nc, 2, nc, 2, nc, 2).mean(axis=(2, 4, 6))
    np.testing.assert_allclose(yc[:, 0], m, atol=1e-14)


# ------------------------------------------------------------------ MLP

def test_mlp_gradient_by_finite_differences():
    shape = (14, 9, 7, 4)
    p = synth.xavier_params(shape, seed=4)
    rng = np.random.default_rng(8)
    p = p + 0.1 * rng.standard_normal(p.shape)
    x, t = synth.random_batch(9, 6, shape[0], shape[-1])
    loss, g = O.mlp_loss_grad(p, x, t, shape)
    idx = rng.choice(len(p), 40, replace=False)
    h = 1e-6
    for j in idx:
        e = np.zeros_like(p)
        e[j] = h
        lp, _ = O.mlp_loss_grad(p + e, x, t, shape)
        lm, _ = O.mlp_loss_grad(p - e, x, t, shape)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_mlp_forward_closed_form():
    shape = (3, 2, 2, 1)
    p = np.arange(1, 1 + O.mlp_nparams(*shape), dtype=float) * 0.05
    x = np.array([[0.3, -0.2, 0.5]])
    W1 = p[:6].reshape(2, 3); b1 = p[6:8]; W2 = p[8:12].reshape(2, 2); b2 = p[12:14]
    W3 = p[14:16].reshape(1, 2); b3 = p[16:17]
    h1 = np.tanh(W1 @ x[0] + b1); h2 = np.tanh(W2 @ h1 + b2); y = W3 @ h2 + b3
    _, _, yo = O.mlp_forward(p, x, shape)
    np.testing.assert_allclose(yo[0], y, rtol=1e-15)


def test_adam_first_steps():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 0.0])
    m = np.zeros(3); v = np.zeros(3)
    O.adam(p, g, m, v, 1, lr=0.01)
    # first step: m_hat = g, v_hat = g^2, so the move is lr * g / (|g| + eps)
    np.testing.assert_allclose(p, [1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8), 0.5], rtol=1e-14)


# ---------------------------------------------------------------- closure features and correction

def _clo_cfg():
    return O.make_cfg(1, (5, 4, 3))


def test_closure_features_neighbour_order():
    """Feature j of a cell is the weight block of the neighbour at offset j
    (self, -x, +x, -y, +y, -z, +z) with periodic wrap: checked against numpy
    rolls of the state, an independent indexing."""
    cfg = _clo_cfg()
    y = np.random.default_rng(1).standard_normal(O.state_shape(cfg))
    f = O.closure_features(cfg, y)
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for j, (dx, dy, dz) in enumerate(offs):
        # value at cell (x, y, z) is y at (x+dx, y+dy, z+dz): roll by the negative offset
        nb = np.roll(y, shift=(-dz, -dy, -dx), axis=(2, 3, 4))
        want = nb.reshape(5, 4, -1).transpose(2, 0, 1)
        np.testing.assert_array_equal(f[:, j], want)


def _affine_closure(b3, bound, scale, shape=(140, 16, 16, 20)):
    """A network whose last layer is zero: its output is b3 for every input."""
    nin, nh1, nh2, nout = shape
    rng = np.random.default_rng(2)
    p = rng.standard_normal(O.mlp_nparams(*shape)) * 0.1
    off = nh1 * nin + nh1 + nh2 * nh1 + nh2
    p[off:off + nout * nh2] = 0.0
    p[off + nout * nh2:] = b3
    return O.ClosureParams(p, np.zeros(nin), np.ones(nin), scale, bound, shape=shape)


def test_closure_constant_output_closed_form():
    """Zero last layer: o = b3 everywhere, so c = scale * b3 for l > 0 and the
    zero-sum shift removes the (constant) l = 0 rows entirely."""
    cfg = _clo_cfg()
    y = np.random.default_rng(3).standard_normal(O.state_shape(cfg))
    b3 = np.linspace(-0.9, 0.9, 20)
    scale = np.linspace(0.5, 2.5, 20)
    clo = _affine_closure(b3, np.ones(20), scale, shape=(140, 16, 16, 20))
    corr, nfb = O.closure_correction(cfg, y, clo)
    assert nfb == 0
    want = (scale * b3).reshape(5, 4)
    for i in range(5):
        np.testing.assert_allclose(corr[i, 0], 0.0, atol=1e-15)
        for l in range(1, 4):
            np.testing.assert_allclose(corr[i, l], want[i, l], rtol=1e-14)


def test_closure_fallback_on_bound_and_nan():
    cfg = _clo_cfg()
    y = np.random.default_rng(4).standard_normal(O.state_shape(cfg))
    b3 = np.full(20, 0.5)
    b3[7] = 1.5  # one output beyond its bound of 1: every cell falls back
    corr, nfb = O.closure_correction(cfg, y, _affine_closure(b3, np.ones(20), np.ones(20)))
    assert nfb == 60 and np.all(corr == 0.0)
    b3[7] = np.nan
    corr, nfb = O.closure_correction(cfg, y, _affine_closure(b3, np.ones(20), np.ones(20)))
    assert nfb == 60 and np.all(corr == 0.0)


def test_closure_network_and_zero_sum_means():
    """A random network: the correction equals scale * MLP(standardised
    features) on cells within bounds (composition of the pinned pieces), the
    l = 0 rows sum to zero per field, and cells beyond a bound fall back."""
    cfg = _clo_cfg()
    rng = np.random.default_rng(5)
    y = rng.standard_normal(O.state_shape(cfg))
    shape = (140, 32, 24, 20)
    p = rng.standard_normal(O.mlp_nparams(*shape)) * 0.2
    mean = rng.standard_normal(140) * 0.1
    std = rng.uniform(0.5, 2.0, 140)
    scale = rng.uniform(0.5, 2.0, 20)
    feats = (O.closure_features(cfg, y).reshape(60, 140) - mean) / std
    _, _, o = O.mlp_forward(p, feats, shape=shape)
    bound = np.quantile(np.abs(o), 0.97, axis=0)  # some cells exceed a bound
    clo = O.ClosureParams(p, mean, std, scale, bound, shape=shape)
    corr, nfb = O.closure_correction(cfg, y, clo)
    bad = np.any(np.abs(o) > bound, axis=1)
    assert nfb == int(bad.sum()) and 0 < nfb < 60
    c = np.where(bad[:, None], 0.0, scale * o)  # [cell][i*4+l]
    c = c.reshape(60, 5, 4).transpose(1, 2, 0)
    got = corr.reshape(5, 4, 60)
    np.testing.assert_allclose(got[:, 1:], c[:, 1:], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(got[:, 0], c[:, 0] - c[:, 0].mean(axis=1, keepdims=True), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(got[:, 0].sum(axis=1), 0.0, atol=1e-12)


def test_effective_dof_gain_reads_the_ladder_unclipped():
    """Host logic of the closure report: the plain errors at 1x and 8x the cells fix a power law in
    the DOF; the closure's error maps to a DOF factor, below 1 when it loses to the plain scheme."""
    from paper_1602_09079_amd.closure import effective_dof_gain
    g = effective_dof_gain([1.0, 1.0, 1.0, 1.0, 1.0], [0.5, 0.5, 0.5, 0.25, 1.0], [0.5, 1.0, 2.0, 0.5, 0.9])
    assert np.allclose(g[:4], [8.0, 1.0, 0.125, 8.0 ** 0.5])
    assert np.isnan(g[4])  # no ladder when the finer plain run is not better
