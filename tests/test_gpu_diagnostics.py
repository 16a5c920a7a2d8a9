"""GPU parity of the turbulence diagnostics (arXiv 1602.09079, Sec. 3.3, 4.1, 4.4)
against the FP64 oracle (oracle/diagnostics.py).

* sub-cell sampling: every field at every grid point, FP64 within 1e-13 and FP32
  storage within 2e-6 of the field's largest value;
* velocity shell spectrum (hipFFT real-to-complex, even and odd M): per shell
  within 1e-12 (FP64) / 1e-5 (FP32) of the total power;
* log-density PDF: the same total; bin counts equal except for points whose
  oracle value lies within rounding of a bin edge (each such point may move to
  the neighbouring bin);
* rms Mach number within 1e-12 (FP64) / 1e-6 (FP32) relative;
* argument errors.
"""
import numpy as np
import pytest

import oracle as O
from oracle import diagnostics as D
from tests.layout import to_abi

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


def state(k, n, seed, mach=0.5, density=0.5):
    """Turbulence surrogate whose density takes on the x momentum's pattern (rho = 1 + density m_x)."""
    from paper_1602_09079_amd import synth
    cfg = O.make_cfg(k, n, gamma=G)
    y = O.project(cfg, synth.turbulence(n, O.gauss_legendre(k + 1)[0], seed=seed, mach=mach).numpy())
    y[0] = y[0] + density * y[1]
    return cfg, y


def stored(y, prec):
    return y if prec == "fp64" else y.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("k,S", [(1, 4), (2, 3), (3, 4), (3, 1), (2, 2), (4, 4), (4, 3)])
def test_sample_parity(dgm, k, S, prec):
    n = (7, 5, 3)
    cfg, y = state(k, n, 20 + k)
    want = D.sample(cfg, stored(y, prec), S)
    s = dgm.Solver(k, n, gamma=G, precision=prec)
    got = s.sample(dev(y, s.dtype), S).cpu().double().numpy()
    assert got.shape == want.shape
    for i in range(5):
        err = np.abs(got[i] - want[i]).max() / np.abs(want[i]).max()
        assert err <= (1e-13 if prec == "fp64" else 2e-6), (i, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("k,n,S", [(2, 8, 4), (3, 5, 3), (1, 6, 4), (4, 5, 4), (3, 25, 4)])
def test_velocity_spectrum_parity(dgm, k, n, S, prec):
    cfg, y = state(k, n, 30 + k, density=0.2)
    M = S * n
    want = D.velocity_spectrum(cfg, stored(y, prec), S, M)
    s = dgm.Solver(k, n, gamma=G, precision=prec)
    yd = dev(y, s.dtype)
    got = s.velocity_spectrum(yd, S, M)
    tot = want.sum()
    err = np.abs(got - want).max() / tot
    assert err <= (1e-12 if prec == "fp64" else 1e-5), err
    # shells summed in a fixed order: the same bits on a second call, and with fewer shells the
    # same leading values
    np.testing.assert_array_equal(s.velocity_spectrum(yd, S, M), got)
    np.testing.assert_array_equal(s.velocity_spectrum(yd, S, 5), got[:5])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_density_pdf_parity(dgm, prec):
    k, n, S = 2, (9, 6, 5), 4
    lo, hi, nb = -0.5, 0.3, 40
    cfg, y = state(k, n, 41)
    ys = stored(y, prec)
    want = D.density_pdf(cfg, ys, S, lo, hi, nb)
    s = dgm.Solver(k, n, gamma=G, precision=prec)
    got = s.density_pdf(dev(y, s.dtype), S, lo, hi, nb)
    assert got.sum() == want.sum() == np.prod(n) * S ** 3
    # points within rounding of a bin edge may land on either side
    r = D.sample(cfg, ys, S)[0].ravel()
    x = np.log10(r[r > 0])
    t = (x - lo) / (hi - lo) * nb
    tol = 1e-10 if prec == "fp64" else 2e-4
    near = int(np.sum(np.abs(t - np.round(t)) < tol * nb))
    assert np.abs(got - want).sum() <= 2 * near, (np.abs(got - want).sum(), near)
    assert want[1:-1].sum() > 0.9 * want.sum()  # the range covers the bulk of the points


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rms_mach_parity(dgm, prec):
    k, n = 3, (6, 5, 4)
    cfg, y = state(k, n, 50, density=0.0)
    want = D.rms_mach(cfg, stored(y, prec), 4)
    s = dgm.Solver(k, n, gamma=G, precision=prec)
    got = s.rms_mach(dev(y, s.dtype), 4)
    assert got == pytest.approx(want, rel=1e-12 if prec == "fp64" else 1e-6)
    assert 0.3 < want < 0.8


def test_diagnostics_errors(dgm):
    s = dgm.Solver(1, (4, 4, 3), gamma=G, precision="fp64")
    y = torch.ones(s.state_shape(), dtype=torch.float64, device="cuda")
    for S in (0, 5):
        with pytest.raises(dgm.DGError) as e:
            s.rms_mach(y, S)
        assert e.value.status == dgm.DG_ERR_ARG
    with pytest.raises(dgm.DGError) as e:
        s.density_pdf(y, 4, 1.0, 1.0, 10)
    assert e.value.status == dgm.DG_ERR_ARG
    with pytest.raises(dgm.DGError) as e:
        s.density_pdf(y, 4, 0.0, 1.0, 0)
    assert e.value.status == dgm.DG_ERR_ARG
    with pytest.raises(dgm.DGError) as e:
        s.velocity_spectrum(y, 2, 8)  # not a cube
    assert e.value.status == dgm.DG_ERR_UNSUPPORTED
