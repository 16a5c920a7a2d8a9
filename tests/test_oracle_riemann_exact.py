"""Pins of the oracle's exact Riemann solver (the alternative numerical flux of Sec. 2.3;
Toro's exact solver), against closed forms of the wave curves written out here:
consistency, a contact, a Rankine-Hugoniot shock in three frames, a transonic
rarefaction (Riemann invariant and sonic point), symmetric collision and expansion
(closed-form star pressures), vacuum, axis rotation."""
import math

import numpy as np
import pytest

import oracle as O

G = 1.4


def cons(rho, u, v, w, p, gamma=G):
    return np.array([rho, rho * u, rho * v, rho * w, p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def rot(q, axis):
    """State with its x components moved to axis (cyclic: x -> axis)."""
    m = q[1:4]
    r = np.roll(m, axis)
    return np.concatenate([[q[0]], r, [q[4]]])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_consistency(axis):
    for q in (cons(1.0, 0.3, -0.2, 0.1, 1.0), cons(0.5, 3.0, 0.0, 0.0, 0.2), cons(2.0, -4.0, 1.0, 0.0, 0.5)):
        np.testing.assert_allclose(O.exact_riemann(q, q, axis, G), O.euler_flux(q, axis, G), rtol=1e-12,
                                   atol=1e-14)


def test_contact():
    """Same normal velocity and pressure: the flux carries the upwind side's density and
    tangential velocities; at rest it is the pressure alone."""
    qL, qR = cons(1.0, 0.4, 0.3, -0.1, 1.0), cons(0.2, 0.4, -0.5, 0.2, 1.0)
    np.testing.assert_allclose(O.exact_riemann(qL, qR, 0, G), O.euler_flux(qL, 0, G), rtol=1e-9)
    qL, qR = cons(1.0, -0.4, 0.3, -0.1, 1.0), cons(0.2, -0.4, -0.5, 0.2, 1.0)
    np.testing.assert_allclose(O.exact_riemann(qL, qR, 0, G), O.euler_flux(qR, 0, G), rtol=1e-9)
    qL, qR = cons(1.0, 0.0, 0.0, 0.0, 1.0), cons(0.2, 0.0, 0.0, 0.0, 1.0)
    np.testing.assert_allclose(O.exact_riemann(qL, qR, 0, G), [0, 1.0, 0, 0, 0], atol=1e-9)


def shock(Ms, frame):
    """Gas at rest (rho 1, p 1) entered by a right-moving shock of Mach Ms (normal-shock
    relations); velocities seen from a frame moving at shock speed + frame * c1."""
    c1 = math.sqrt(G)
    S = Ms * c1
    p2 = 1.0 + 2 * G / (G + 1) * (Ms * Ms - 1)
    r2 = (G + 1) * Ms * Ms / ((G - 1) * Ms * Ms + 2)
    u2 = S * (1 - 1.0 / r2)
    V = S + frame * c1
    return cons(r2, u2 - V, 0.2, 0.0, p2), cons(1.0, -V, 0.2, 0.0, 1.0)


@pytest.mark.parametrize("Ms", [1.5, 3.0])
def test_shock_in_three_frames(Ms):
    qL, qR = shock(Ms, 0.0)  # stationary shock: Rankine-Hugoniot makes both fluxes equal
    F = O.exact_riemann(qL, qR, 0, G)
    np.testing.assert_allclose(O.euler_flux(qL, 0, G), O.euler_flux(qR, 0, G), rtol=1e-12)
    np.testing.assert_allclose(F, O.euler_flux(qL, 0, G), rtol=1e-9, atol=1e-12)
    qL, qR = shock(Ms, 0.3)  # the shock moves left in this frame: the face sees the pre-shock gas
    np.testing.assert_allclose(O.exact_riemann(qL, qR, 0, G), O.euler_flux(qR, 0, G), rtol=1e-12)
    qL, qR = shock(Ms, -0.3)  # moves right: the face sees the post-shock gas
    np.testing.assert_allclose(O.exact_riemann(qL, qR, 0, G), O.euler_flux(qL, 0, G), rtol=1e-9)


def test_transonic_rarefaction():
    """L joined to R by a left rarefaction whose fan spans x/t = 0: the face state is the
    sonic point, u = c, fixed by the Riemann invariant u + 2c/(gamma-1) and isentropy."""
    g1 = G - 1
    rL, uL, pL = 1.0, 0.2, 1.0
    cL = math.sqrt(G * pL / rL)
    ps = 0.3 * pL
    us = uL - 2 * cL / g1 * ((ps / pL) ** (g1 / (2 * G)) - 1)
    rs = rL * (ps / pL) ** (1 / G)
    assert uL - cL < 0 < us - math.sqrt(G * ps / rs)  # transonic
    qL, qR = cons(rL, uL, 0.1, 0.0, pL), cons(rs, us, 0.1, 0.0, ps)
    c = (g1 * uL + 2 * cL) / (G + 1)
    rho = rL * (c / cL) ** (2 / g1)
    p = pL * (rho / rL) ** G
    np.testing.assert_allclose(O.exact_riemann(qL, qR, 0, G), O.euler_flux(cons(rho, c, 0.1, 0.0, p), 0, G),
                               rtol=1e-9)


@pytest.mark.parametrize("U", [0.5, 2.0])
def test_symmetric_collision(U):
    """Two equal shocks: u* = 0 and A x^2 - U^2 x - U^2 (p + B) = 0 for x = p* - p."""
    rho, p = 1.0, 1.0
    A, B = 2 / ((G + 1) * rho), (G - 1) / (G + 1) * p
    x = (U * U + math.sqrt(U ** 4 + 4 * A * U * U * (p + B))) / (2 * A)
    F = O.exact_riemann(cons(rho, U, 0, 0, p), cons(rho, -U, 0, 0, p), 0, G)
    np.testing.assert_allclose(F, [0, p + x, 0, 0, 0], atol=1e-9)


def test_symmetric_expansion_and_vacuum():
    """Two equal rarefactions: p* = p (1 - (gamma-1) U / (2c))^(2 gamma/(gamma-1)); beyond
    U = 2c/(gamma-1) vacuum forms at the face and the flux vanishes."""
    rho, p = 1.0, 1.0
    c = math.sqrt(G * p / rho)
    U = 0.5
    ps = p * (1 - (G - 1) * U / (2 * c)) ** (2 * G / (G - 1))
    F = O.exact_riemann(cons(rho, -U, 0, 0, p), cons(rho, U, 0, 0, p), 0, G)
    np.testing.assert_allclose(F, [0, ps, 0, 0, 0], atol=1e-9)
    U = 1.2 * 2 * c / (G - 1)
    F = O.exact_riemann(cons(rho, -U, 0, 0, p), cons(rho, U, 0, 0, p), 0, G)
    np.testing.assert_allclose(F, 0.0, atol=1e-14)


@pytest.mark.parametrize("axis", [1, 2])
def test_axis_rotation(axis):
    qL, qR = cons(1.0, 0.8, 0.3, -0.2, 1.5), cons(0.4, -0.3, 0.1, 0.5, 0.3)
    Fx = O.exact_riemann(qL, qR, 0, G)
    Fa = O.exact_riemann(rot(qL, axis), rot(qR, axis), axis, G)
    np.testing.assert_allclose(Fa, rot(Fx, axis), rtol=1e-12, atol=1e-14)


def test_rhs_with_exact_solver_preserves_free_stream_and_differs_from_hllc():
    from paper_1602_09079_amd import synth
    k, n = 2, 4
    cx = O.make_cfg(k, n, gamma=G, riemann="exact")
    ch = O.make_cfg(k, n, gamma=G)
    y = np.zeros(O.state_shape(cx))
    y[:, 0] = cons(1.3, 0.2, -0.4, 0.1, 0.7)[:, None, None, None]
    np.testing.assert_allclose(O.rhs(cx, y), 0.0, atol=1e-13)
    y = O.project(cx, synth.turbulence(n, O.gauss_legendre(k + 1)[0], seed=3, mach=0.5).numpy())
    rx, rh = O.rhs(cx, y), O.rhs(ch, y)
    d = np.linalg.norm(rx - rh) / np.linalg.norm(rh)
    assert 1e-6 < d < 0.1  # different fluxes, same scheme
