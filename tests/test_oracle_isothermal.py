"""Pins of the oracle's isothermal reset (arXiv 1602.09079, Sec. 3.2)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1602_09079_amd import synth


def _eps(rho, cs, gamma, rho0):
    return cs * cs / (gamma - 1.0) * (rho / rho0) ** (gamma - 1.0)


@pytest.mark.parametrize("k,gamma,cs,rho0", [(1, 1.01, 1.0, 1.0), (2, 5.0 / 3.0, 0.7, 1.3), (3, 1.01, 1.2, 0.8)])
def test_uniform_state_closed_form(k, gamma, cs, rho0):
    """rho, m constant: E becomes |m|^2/(2 rho) + rho eps(rho) exactly, higher modes 0,
    and the dissipated energy is the box volume times the change of E."""
    box = (1.0, 2.0, 0.5)
    cfg = O.make_cfg(k, (3, 2, 2), box=box, gamma=gamma)
    y = np.zeros(O.state_shape(cfg))
    rho, m, E = 1.7, (0.3, -0.2, 0.5), 4.0
    y[0, 0] = rho
    for i in range(3):
        y[1 + i, 0] = m[i]
    y[4, 0] = E
    y[4, 1:] = 0.05  # higher energy modes are replaced as well
    yr, dis = O.isothermal_reset(cfg, y, cs, rho0)
    want = 0.5 * sum(v * v for v in m) / rho + rho * _eps(rho, cs, gamma, rho0)
    np.testing.assert_allclose(yr[4, 0], want, rtol=1e-14)
    np.testing.assert_allclose(yr[4, 1:], 0.0, atol=1e-13)
    np.testing.assert_array_equal(yr[:4], y[:4])
    vol = box[0] * box[1] * box[2]
    assert dis == pytest.approx(vol * (E - want), rel=1e-12)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_linear_density_against_gauss_rule(k):
    """rho = rhobar + a sqrt(3) xi_x at rest: rho at the Gauss nodes is rhobar + a sqrt(3) x_j,
    so the energy weight of mode (u,0,0) is 1/2 sum_j w_j P_u(x_j) e(rho_j), e = rho eps(rho),
    P_u the scaled Legendre polynomial (the y and z sums give 2 each), and every mode with
    a y or z degree is zero."""
    gamma, cs, rho0 = 1.4, 1.1, 1.0
    cfg = O.make_cfg(k, 2, gamma=gamma)
    y = np.zeros(O.state_shape(cfg))
    rb, a = 1.0, 0.3
    modes = [tuple(m) for m in O.mode_list(k)]
    y[0, 0] = rb
    y[0, modes.index((1, 0, 0))] = a
    y[4, 0] = 9.0
    yr, _ = O.isothermal_reset(cfg, y, cs, rho0)
    # textbook Gauss-Legendre rules and scaled Legendre polynomials, written out
    r6 = math.sqrt(6 / 5)
    rules = {2: ([-1 / math.sqrt(3), 1 / math.sqrt(3)], [1.0, 1.0]),
             3: ([-math.sqrt(0.6), 0.0, math.sqrt(0.6)], [5 / 9, 8 / 9, 5 / 9]),
             4: ([-math.sqrt(3 / 7 + 2 / 7 * r6), -math.sqrt(3 / 7 - 2 / 7 * r6),
                  math.sqrt(3 / 7 - 2 / 7 * r6), math.sqrt(3 / 7 + 2 / 7 * r6)],
                 [(18 - math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36, (18 + math.sqrt(30)) / 36,
                  (18 - math.sqrt(30)) / 36])}
    P = [lambda x: 1.0, lambda x: math.sqrt(3) * x, lambda x: math.sqrt(5) * (3 * x * x - 1) / 2,
         lambda x: math.sqrt(7) * (5 * x ** 3 - 3 * x) / 2]
    x, w = rules[k + 1]
    e = [(rb + a * math.sqrt(3) * xj) * _eps(rb + a * math.sqrt(3) * xj, cs, gamma, rho0) for xj in x]
    for l, (u, v, ww) in enumerate(modes):
        if v == 0 and ww == 0:
            want = 0.5 * sum(wj * P[u](xj) * ej for wj, xj, ej in zip(w, x, e))
            np.testing.assert_allclose(yr[4, l], want, rtol=1e-13, atol=1e-15)
        else:
            np.testing.assert_allclose(yr[4, l], 0.0, atol=1e-14)


def _turbulent(k, n, gamma, seed=5, mach=0.3):
    cfg = O.make_cfg(k, n, gamma=gamma)
    x = O.gauss_legendre(k + 1)[0]
    y = O.project(cfg, synth.turbulence(n, x, seed=seed, mach=mach).numpy())
    return cfg, y


@pytest.mark.parametrize("k", [1, 3])
def test_dissipated_energy_is_the_change_of_total_energy(k):
    """rho and m are untouched, so the cell-mean kinetic energy is unchanged and the
    dissipated energy equals the drop of the total energy; a second reset changes nothing."""
    cfg, y = _turbulent(k, 4, 1.01)
    rng = np.random.default_rng(3)
    y[4] *= 1.0 + 0.02 * rng.random(y[4].shape)
    yr, dis = O.isothermal_reset(cfg, y, 1.0, 1.0)
    np.testing.assert_array_equal(yr[:4], y[:4])
    t0, t1 = O.totals(cfg, y), O.totals(cfg, yr)
    assert dis == pytest.approx(t0[4] - t1[4], rel=1e-11, abs=1e-14)
    assert abs(dis) > 1e-3
    y2, dis2 = O.isothermal_reset(cfg, yr, 1.0, 1.0)
    assert abs(dis2) < 1e-13
    np.testing.assert_allclose(y2[4], yr[4], rtol=0, atol=1e-13)


def test_steps_with_reset_account_for_all_energy():
    """Without driving the scheme conserves the total energy; with the reset after every
    step the energy taken out equals the summed dissipated energy, which is positive
    (the numerical dissipation heats the gas, the reset removes the heat)."""
    cfg, y = _turbulent(1, 6, 1.01, seed=11, mach=0.5)
    y, _ = O.isothermal_reset(cfg, y, 1.0, 1.0)  # start isothermal
    e0 = O.totals(cfg, y)[4]
    y1, _, dis = O.step_isothermal(cfg, y, 0.0, 6, cs=1.0, rho0=1.0)
    e1 = O.totals(cfg, y1)[4]
    assert dis > 0
    assert e0 - e1 == pytest.approx(dis, rel=1e-9)
    # the same steps without the reset keep the energy
    y2, _ = O.step(cfg, y, O.dt(cfg, y), 1)
    assert O.totals(cfg, y2)[4] == pytest.approx(e0, rel=1e-13)
