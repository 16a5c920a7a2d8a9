"""GPU parity of degree k = 4 (N = 35 modes, 5^3 volume and 5^2 face Gauss points per
cell: the matrix-core stage kernel) against the FP64 oracle: R with HLLC and
with the exact Riemann solver, with and without the driving; device-CFL steps in
FP64 and FP32; the isothermal reset and sub-cell sampling at k = 4; the
configurations k = 4 does not take (the limiter at k = 4 is in the limiter tests)."""
import numpy as np
import pytest

import oracle as O
from oracle import diagnostics as D
from tests.layout import from_abi, to_abi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

G = 5.0 / 3.0
K = 4


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


def turb(n, seed=4, mach=0.6, gamma=G, riemann="hllc", box=(1.0, 1.0, 1.0)):
    from paper_1602_09079_amd import synth
    cfg = O.make_cfg(K, n, box=box, gamma=gamma, riemann=riemann)
    y = O.project(cfg, synth.turbulence(n, O.gauss_legendre(K + 1)[0], seed=seed, mach=mach).numpy())
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


@pytest.mark.parametrize("riemann", ["hllc", "exact"])
@pytest.mark.parametrize("forcing", [False, True])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rhs_parity_k4(dgm, prec, forcing, riemann):
    n = (9, 6, 5)
    box = (1.0, 0.8, 0.6)  # unequal widths: each axis's scale reaches its own terms
    cfg, y = turb(n, riemann=riemann, box=box)
    s = dgm.Solver(K, n, box=box, gamma=G, precision=prec, forcing=forcing, riemann=riemann)
    frc = None
    if forcing:
        nvec, al, frc = driving(dgm)
        s.set_forcing(nvec, al)
    r = host(s.rhs(dev(y, s.dtype)))
    err = err_max_norm(r, O.rhs(cfg, stored(y, prec), frc))
    assert np.all(err <= (1e-13 if prec == "fp64" else 2e-5)), err  # the R bars of the k <= 3 tests


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_steps_parity_k4(dgm, prec):
    n = (8, 6, 5)
    cfg, y = turb(n, seed=5, mach=0.4)
    s = dgm.Solver(K, n, gamma=G, precision=prec)
    yd = dev(y, s.dtype)
    t = s.step(yd, 3)
    want, tw = O.step(cfg, stored(y, prec), 0.0, 3)
    assert t == pytest.approx(tw, rel=1e-13 if prec == "fp64" else 1e-6)
    err = O.rel_l2(host(yd), want)
    assert np.all(err <= (1e-13 if prec == "fp64" else 1e-6)), err


@pytest.mark.parametrize("n", [(31, 5, 4), (16, 4, 4)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_several_x_blocks_k4(dgm, prec, n):
    """The stage kernel updates x-blocks of 16 cells, their edge faces from a ghost product of
    the cell before and the cell after: (31, 5, 4) has a full block and a ragged one of 15 cells
    (x faces 15/16 inside the mesh and 30/0 at the periodic wrap, each formed by two blocks);
    (16, 4, 4) is one full block whose cell after is its own first cell.  R with the driving,
    then two device-CFL steps (stages 2 and 3 read y0)."""
    cfg, y = turb(n, seed=11, mach=0.5)
    s = dgm.Solver(K, n, gamma=G, precision=prec, forcing=True)
    nvec, al, frc = driving(dgm)
    s.set_forcing(nvec, al)
    r = host(s.rhs(dev(y, s.dtype)))
    err = err_max_norm(r, O.rhs(cfg, stored(y, prec), frc))
    assert np.all(err <= (1e-13 if prec == "fp64" else 2e-5)), err
    yd = dev(y, s.dtype)
    t = s.step(yd, 2)
    want, tw = O.step(cfg, stored(y, prec), 0.0, 2, frc=frc)
    assert t == pytest.approx(tw, rel=1e-13 if prec == "fp64" else 1e-6)
    err = O.rel_l2(host(yd), want)
    assert np.all(err <= (1e-13 if prec == "fp64" else 1e-6)), err


def test_mass_conserved_k4(dgm):
    """The face fluxes of the two cells of a face agree, so the total mass changes only by
    rounding (FP64, driven, exact Riemann solver)."""
    n = (8, 6, 5)
    _, y = turb(n, seed=8, riemann="exact")
    s = dgm.Solver(K, n, gamma=G, precision="fp64", forcing=True, riemann="exact")
    nvec, al, _ = driving(dgm)
    s.set_forcing(nvec, al)
    yd = dev(y, s.dtype)
    m0 = s.totals(yd)[0]
    s.step(yd, 4)
    assert abs(s.totals(yd)[0] - m0) <= 1e-13 * abs(m0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reset_and_sampling_k4(dgm, prec):
    n = (5, 4, 3)
    cfg, y = turb(n, seed=6, gamma=1.01)
    ys = stored(y, prec)
    s = dgm.Solver(K, n, gamma=1.01, precision=prec)
    s.set_isothermal(1.0, 1.0)
    yd = dev(y, s.dtype)
    smp = s.sample(yd, 4).cpu().double().numpy()
    np.testing.assert_allclose(smp, D.sample(cfg, ys, 4), rtol=1e-12 if prec == "fp64" else 2e-5,
                               atol=1e-12 if prec == "fp64" else 2e-5)
    s.isothermal_reset(yd)
    want, _ = O.isothermal_reset(cfg, ys, 1.0, 1.0)
    err = np.abs(host(yd) - want).max() / np.abs(want).max()
    assert err <= (1e-13 if prec == "fp64" else 2e-6), err


@pytest.mark.parametrize("kw", [dict(precision="bf16"), dict(precision="bf16x3")])
def test_k4_unsupported_configurations(dgm, kw):
    with pytest.raises(dgm.DGError) as e:
        dgm.Solver(K, (6, 5, 4), gamma=G, **{"precision": "fp64", **kw})
    assert e.value.status == dgm.DG_ERR_UNSUPPORTED
