"""Pins of the oracle's turbulence diagnostics (arXiv 1602.09079, Sec. 3.3, 4.1, 4.4):
sub-cell sampling, the velocity power spectrum, the density PDF and the rms Mach number."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import diagnostics as D

G = 5.0 / 3.0


def test_sub_points():
    np.testing.assert_array_equal(D.sub_points(4), [-0.75, -0.25, 0.25, 0.75])
    np.testing.assert_array_equal(D.sub_points(1), [0.0])


def _project_fields(cfg, fields):
    """L2 projection of point functions f(x, y, z) (global coordinates, unit box) per field."""
    k = cfg.k
    n = cfg.n[0]
    xg = O.gauss_legendre(k + 1)[0]
    q = k + 1
    qp = np.zeros((5, q, q, q, n, n, n))
    for i, f in enumerate(fields):
        for c in range(q):
            for b in range(q):
                for a in range(q):
                    xx = ((np.arange(n) + 0.5 * (1 + xg[a])) / n)[None, None, :]
                    yy = ((np.arange(n) + 0.5 * (1 + xg[b])) / n)[None, :, None]
                    zz = ((np.arange(n) + 0.5 * (1 + xg[c])) / n)[:, None, None]
                    qp[i, c, b, a] = f(xx, yy, zz) + 0 * (xx + yy + zz)
    return O.project(cfg, qp)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_sampling_reproduces_polynomials(k):
    """A state that is a polynomial of degree <= k is projected exactly, so its samples are the
    polynomial's values at the grid points x = (X + 1/2)/M; v = m/rho is exact for m = rho v0."""
    n, S = 3, 4
    cfg = O.make_cfg(k, n, gamma=G)
    rho = {1: lambda x, y, z: 1 + 0.3 * x - 0.2 * y + 0.1 * z,
           2: lambda x, y, z: 1 + 0.3 * x - 0.2 * y * y + 0.1 * x * z,
           3: lambda x, y, z: 1 + 0.3 * x * x * x - 0.2 * y * z + 0.1 * z * z}[k]
    v0 = (0.4, -0.1, 0.25)
    y = _project_fields(cfg, [rho] + [lambda x, yy, z, c=c: v0[c] * rho(x, yy, z) for c in range(3)]
                        + [lambda x, y, z: 3.0 + 0 * x])
    r, v = D.velocity_grid(cfg, y, S)
    M = n * S
    g = (np.arange(M) + 0.5) / M
    want = rho(g[None, None, :], g[None, :, None], g[:, None, None])
    np.testing.assert_allclose(r, want, rtol=0, atol=1e-13)
    for c in range(3):
        np.testing.assert_allclose(v[c], v0[c], rtol=0, atol=1e-13)


@pytest.mark.parametrize("nvec,shell", [((3, 0, 0), 3), ((1, 1, 1), 2), ((2, 1, 0), 2), ((0, 4, 4), 6),
                                        ((1, 1, 0), 1)])
def test_single_mode_lands_in_its_shell(nvec, shell):
    """cos(2 pi n.X / M) has mean square 1/2, all of it in the shell nearest to |n|."""
    M = 16
    X = np.arange(M)
    ph = 2 * np.pi * (nvec[0] * X[None, None, :] + nvec[1] * X[None, :, None] + nvec[2] * X[:, None, None]) / M
    P = D.shell_power(np.cos(ph), 16)
    want = np.zeros(16)
    want[shell] = 0.5
    np.testing.assert_allclose(P, want, rtol=0, atol=1e-15)


def test_constant_and_parseval():
    M = 12
    P = D.shell_power(np.full((M, M, M), 1.5), 4)
    np.testing.assert_allclose(P, [2.25, 0, 0, 0], atol=1e-14)
    w = np.random.default_rng(1).standard_normal((M, M, M))
    P = D.shell_power(w, M)  # shells up to sqrt(3) M/2 < M
    assert P.sum() == pytest.approx(np.mean(w ** 2), rel=1e-12)


def test_velocity_spectrum_sums_to_mean_square_velocity():
    from paper_1602_09079_amd import synth
    k, n = 2, 4
    cfg = O.make_cfg(k, n, gamma=G)
    y = O.project(cfg, synth.turbulence(n, O.gauss_legendre(3)[0], seed=8, mach=0.5).numpy())
    P = D.velocity_spectrum(cfg, y, 4)
    _, v = D.velocity_grid(cfg, y, 4)
    assert P.sum() == pytest.approx(np.mean(np.sum(v ** 2, axis=0)), rel=1e-12)
    assert P[0] < 1e-3 * P.sum()  # no bulk motion


def test_density_pdf_bins():
    k, n, S = 1, 2, 4
    cfg = O.make_cfg(k, n, gamma=G)
    y = np.zeros(O.state_shape(cfg))
    y[0, 0] = 10 ** 0.35
    y[4, 0] = 2.0
    c = D.density_pdf(cfg, y, S, 0.0, 1.0, 10)
    assert c.sum() == (n * S) ** 3 and c[1 + 3] == (n * S) ** 3
    y[0, 0, 0, 0, 0] = -1.0   # one cell of negative density: its 64 samples go below the range
    y[0, 0, 1, 1, 1] = 100.0  # one cell above the range
    c = D.density_pdf(cfg, y, S, 0.0, 1.0, 10)
    assert c[0] == S ** 3 and c[11] == S ** 3 and c[4] == (n * S) ** 3 - 2 * S ** 3


def test_rms_mach_uniform():
    cfg = O.make_cfg(1, 2, gamma=G)
    y = np.zeros(O.state_shape(cfg))
    rho, v, p = 1.3, (0.2, -0.3, 0.1), 0.9
    y[0, 0] = rho
    for i in range(3):
        y[1 + i, 0] = rho * v[i]
    y[4, 0] = p / (G - 1) + 0.5 * rho * sum(a * a for a in v)
    want = math.sqrt(sum(a * a for a in v) / (G * p / rho))
    assert D.rms_mach(cfg, y) == pytest.approx(want, rel=1e-14)
