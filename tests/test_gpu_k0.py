"""GPU parity of degree k = 0 (one weight per field: first-order Godunov finite
volume, the lowest order of arXiv 1602.09079's runs) against the FP64 oracle:
R with HLLC and with the exact Riemann solver, with the driving; device-CFL
steps in every tier; the isothermal reset and sub-cell sampling at k = 0."""
import numpy as np
import pytest

import oracle as O
from oracle import diagnostics as D
from tests.layout import from_abi, to_abi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

G = 5.0 / 3.0


@pytest.fixture(scope="module")
def dgm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_09079_amd import dg
    dg.lib()
    return dg


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(to_abi(a))).to(device="cuda", dtype=dtype)


def host(y):
    return from_abi(y.cpu().double().numpy())


def turb(n, seed=4, mach=0.6, gamma=G, riemann="hllc"):
    from paper_1602_09079_amd import synth
    cfg = O.make_cfg(0, n, gamma=gamma, riemann=riemann)
    y = O.project(cfg, synth.turbulence(n, O.gauss_legendre(1)[0], seed=seed, mach=mach).numpy())
    return cfg, y


def driving(dgm):
    from paper_1602_09079_amd import synth
    nvec = synth.forcing_modes(1.0, 3.0)
    th = synth.ou_stationary_start(3, len(nvec))
    z = synth.ou_normals(3, len(nvec), 1)[0]
    _, al = dgm.ou_update(nvec, th, z, 0.9, 1.0, 1.0, 1.0, 3.0)
    _, ao = O.ou_update(nvec, th, z, 0.9, 1.0, 1.0, 1.0, 3.0)
    return nvec, al, O.ForcingTable(nvec, ao)


def stored(y, prec):
    return y if prec == "fp64" else y.astype(np.float32).astype(np.float64)


def err_max_norm(g, w):
    g = g.reshape(5, -1)
    w = w.reshape(5, -1)
    return np.linalg.norm(g - w, axis=1) / np.linalg.norm(w, axis=1).max()


@pytest.mark.parametrize("n", [(37, 6, 5), (70, 7, 5)])
@pytest.mark.parametrize("riemann", ["hllc", "exact"])
@pytest.mark.parametrize("forcing", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rhs_parity_k0(dgm, prec, forcing, riemann, n):
    # workgroup tiles are 64 x 4 cells (x, y): (37, 6, 5) is one ragged tile in x and a ragged
    # second row of tiles in y; (70, 7, 5) has two tiles in x (the -x face of the second tile's
    # first column comes from the first tile) and ny not a multiple of 4
    cfg, y = turb(n, riemann=riemann)
    s = dgm.Solver(0, n, gamma=G, precision=prec, forcing=forcing, riemann=riemann)
    frc = None
    if forcing:
        nvec, al, frc = driving(dgm)
        s.set_forcing(nvec, al)
    r = host(s.rhs(dev(y, s.dtype)))
    err = err_max_norm(r, O.rhs(cfg, stored(y, prec), frc))
    assert np.all(err <= (1e-13 if prec == "fp64" else 2e-5)), err  # the R bars of the k >= 1 tests


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16x3"])
@pytest.mark.parametrize("n", [(20, 7, 6), (70, 7, 5)])
def test_steps_parity_k0(dgm, prec, n):
    cfg, y = turb(n, seed=5)
    s = dgm.Solver(0, n, gamma=G, precision=prec)
    yd = dev(y, s.dtype)
    t = s.step(yd, 5)
    want, tw = O.step(cfg, stored(y, prec), 0.0, 5)
    assert t == pytest.approx(tw, rel=1e-13 if prec == "fp64" else 1e-6)
    err = O.rel_l2(host(yd), want)
    assert np.all(err <= (1e-13 if prec == "fp64" else 1e-6)), err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reset_and_sampling_k0(dgm, prec):
    n = (9, 5, 4)
    cfg, y = turb(n, seed=6, gamma=1.01)
    ys = stored(y, prec)
    s = dgm.Solver(0, n, gamma=1.01, precision=prec)
    s.set_isothermal(1.0, 1.0)
    yd = dev(y, s.dtype)
    smp = s.sample(yd, 2).cpu().double().numpy()
    np.testing.assert_allclose(smp, D.sample(cfg, ys, 2), rtol=1e-13 if prec == "fp64" else 1e-6)
    s.isothermal_reset(yd)
    want, dw = O.isothermal_reset(cfg, ys, 1.0, 1.0)
    err = np.abs(host(yd) - want).max() / np.abs(want).max()
    assert err <= (1e-14 if prec == "fp64" else 1e-6), err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_limited_isothermal_steps_k0(dgm, prec):
    """k = 0 with the limiter (no higher modes to scale, but the limited time step C/2) and the
    isothermal reset after every step, device CFL steps, against the oracle."""
    n = (12, 5, 4)
    cfg, y = turb(n, seed=7, gamma=1.01)
    y, _ = O.isothermal_reset(cfg, y, 1.0, 1.0)
    s = dgm.Solver(0, n, gamma=1.01, precision=prec, limit=True, isothermal=True)
    s.set_isothermal(1.0, 1.0)
    yd = dev(y, s.dtype)
    t = s.step(yd, 3)
    want, tw, _ = O.step_isothermal(cfg, stored(y, prec), 0.0, 3, cs=1.0, rho0=1.0, limit=True)
    assert t == pytest.approx(tw, rel=1e-13 if prec == "fp64" else 1e-6)
    assert tw == pytest.approx(3 * 0.5 * O.dt(cfg, y), rel=0.05)  # the limited step is half the plain one
    err = O.rel_l2(host(yd), want)
    assert np.all(err <= (1e-12 if prec == "fp64" else 1e-6)), err
