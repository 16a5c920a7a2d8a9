"""Pins of the oracle's operator (Sec. 2.2-2.4 of arXiv 1602.09079): projection
exactness, HLLC properties, free-stream preservation, conservation, the linear
advection special case, convergence order k+1, the SSP-RK3 amplification factor
and the CFL time step."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_1602_09079_amd import synth

G = 5.0 / 3.0


def nodes(k):
    return O.gauss_legendre(k + 1)[0]


# ------------------------------------------------------------------ projection

@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_projection_exact_for_degree_k_polynomials(k):
    """Sec. 2.2: the (k+1)-point projection is exact for polynomial data of degree <= k."""
    rng = np.random.default_rng(10 + k)
    nc = 3
    cfg = O.make_cfg(k, nc)
    n = k + 1
    x = nodes(k)
    exps = [(u, v, w) for u in range(k + 1) for v in range(k + 1) for w in range(k + 1) if u + v + w <= k]
    coef = rng.standard_normal((5, nc, nc, nc, len(exps)))  # per field per cell, monomials in xi
    qp = np.zeros((5, n, n, n, nc, nc, nc))
    for c, b, a in itertools.product(range(n), repeat=3):
        mono = np.array([x[a] ** u * x[b] ** v * x[c] ** w for (u, v, w) in exps])
        qp[:, c, b, a] = coef @ mono
    y = O.project(cfg, qp)
    # evaluate the modal expansion at random interior points and compare
    for _ in range(6):
        xi = rng.uniform(-1, 1, 3)
        ph = O.basis(k, xi)
        mono = np.array([xi[0] ** u * xi[1] ** v * xi[2] ** w for (u, v, w) in exps])
        got = np.einsum("il...,l->i...", y, ph)
        want = coef @ mono
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_mode_zero_is_cell_mean_for_linear_data():
    k = 2
    cfg = O.make_cfg(k, 4)
    x = nodes(k)
    n = k + 1
    qp = np.zeros((5, n, n, n, 4, 4, 4))
    # field = 2 + 0.5 X + 0.25 Y - Z in physical coordinates
    h = 0.25
    for c, b, a in itertools.product(range(n), repeat=3):
        X = (np.arange(4)[None, None, :] + 0.5 * (1 + x[a])) * h
        Y = (np.arange(4)[None, :, None] + 0.5 * (1 + x[b])) * h
        Z = (np.arange(4)[:, None, None] + 0.5 * (1 + x[c])) * h
        qp[:, c, b, a] = 2 + 0.5 * X + 0.25 * Y - Z
    y = O.project(cfg, qp)
    ctr = (np.arange(4) + 0.5) * h
    mean = 2 + 0.5 * ctr[None, None, :] + 0.25 * ctr[None, :, None] - ctr[:, None, None]
    np.testing.assert_allclose(y[0, 0], mean, atol=1e-14)


# ------------------------------------------------------------------ HLLC

def cons(rho, v, p, g=G):
    v = np.asarray(v, dtype=float)
    return np.array([rho, *(rho * v), p / (g - 1) + 0.5 * rho * v.dot(v)])


def rand_state(rng, vmax=0.8):
    return cons(rng.uniform(0.3, 2.0), rng.uniform(-vmax, vmax, 3), rng.uniform(0.3, 2.0))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_consistency(axis):
    rng = np.random.default_rng(axis)
    for _ in range(50):
        q = rand_state(rng, vmax=3.0)
        np.testing.assert_allclose(O.hllc(q, q, axis, G), O.euler_flux(q, axis, G), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_exact_contact(axis):
    """Equal pressure and velocity, jump in density: HLLC returns the upwind flux."""
    rng = np.random.default_rng(5 + axis)
    for sgn in (+1, -1):
        v = rng.uniform(-0.5, 0.5, 3)
        v[axis] = sgn * abs(v[axis]) + sgn * 0.05
        qL = cons(1.3, v, 0.9)
        qR = cons(0.6, v, 0.9)
        up = qL if sgn > 0 else qR
        np.testing.assert_allclose(O.hllc(qL, qR, axis, G), O.euler_flux(up, axis, G), rtol=1e-13, atol=1e-14)


def test_hllc_supersonic_upwinding():
    rng = np.random.default_rng(7)
    for axis in range(3):
        for _ in range(10):
            qL = rand_state(rng)
            qR = rand_state(rng)
            for q in (qL, qR):
                c = math.sqrt(G * (G - 1) * (q[4] - 0.5 * (q[1:4] ** 2).sum() / q[0]) / q[0])
                # make the normal velocity strongly supersonic to the right
                v = q[1:4] / q[0]
                v[axis] = 3.0 * c + 1.0 + 2.0 * abs(v).max()
                q[:] = cons(q[0], v, (G - 1) * (q[4] - 0.5 * q[0] * (q[1:4] / q[0]).dot(q[1:4] / q[0])))
            cL = math.sqrt(G * 1.0)
            F = O.hllc(qL, qR, axis, G)
            np.testing.assert_allclose(F, O.euler_flux(qL, axis, G), rtol=1e-13)
            # mirrored: everything moving left
            mL, mR = qL.copy(), qR.copy()
            mL[1 + axis] *= -1
            mR[1 + axis] *= -1
            np.testing.assert_allclose(O.hllc(mR, mL, axis, G), O.euler_flux(mL, axis, G), rtol=1e-13)


def test_hllc_rotation_and_mirror_symmetry():
    rng = np.random.default_rng(11)
    for _ in range(40):
        qL, qR = rand_state(rng), rand_state(rng)
        F0 = O.hllc(qL, qR, 0, G)
        # rotation: relabel axes (x,y,z) -> (y,z,x)
        for axis in (1, 2):
            perm = [(j - axis) % 3 for j in range(3)]  # component j of the rotated state = component perm[j]
            rL = np.array([qL[0], *[qL[1 + perm[j]] for j in range(3)], qL[4]])
            rR = np.array([qR[0], *[qR[1 + perm[j]] for j in range(3)], qR[4]])
            Fa = O.hllc(rL, rR, axis, G)
            np.testing.assert_allclose(Fa[[0, 4]], F0[[0, 4]], rtol=1e-13, atol=1e-14)
            np.testing.assert_allclose([Fa[1 + j] for j in range(3)], [F0[1 + perm[j]] for j in range(3)],
                                       rtol=1e-13, atol=1e-14)
        # mirror x -> -x: swap sides, flip normal components; flux flips sign except normal momentum
        mL, mR = qR.copy(), qL.copy()
        mL[1] *= -1
        mR[1] *= -1
        Fm = O.hllc(mL, mR, 0, G)
        want = -F0.copy()
        want[1] = F0[1]
        np.testing.assert_allclose(Fm, want, rtol=1e-12, atol=1e-13)


def _prim(q, axis, g=G):
    rho = q[0]
    v = q[1:4] / rho
    p = (g - 1) * (q[4] - 0.5 * rho * v.dot(v))
    return rho, v, p, v[axis], math.sqrt(g * p / rho)


def _subsonic_pairs(rng, count):
    """Random subsonic left/right states: |u| well below c on both sides, so S_L < 0 < S_R."""
    out = []
    while len(out) < count:
        qL = cons(rng.uniform(0.3, 2.5), rng.uniform(-0.6, 0.6, 3), rng.uniform(0.3, 2.5))
        qR = cons(rng.uniform(0.3, 2.5), rng.uniform(-0.6, 0.6, 3), rng.uniform(0.3, 2.5))
        out.append((qL, qR))
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_star_region_defining_conditions(axis):
    """The star-region flux of HLLC (Sec. 2.3 names HLLC as the numerical flux; Toro, Riemann
    Solvers and Numerical Methods for Fluid Dynamics, ch. 10) checked against the conditions
    that define it, not against its formula.  From the oracle's flux F, the star state of the
    upwind side K follows from the Rankine-Hugoniot condition across the S_K wave:
    U*_K = U_K + (F - F_K) / S_K.  HLLC's star region then has
      - one normal velocity S* = m*_n / rho* that also carries the mass flux, F_rho = rho* S*;
      - the tangential velocities of side K;
      - one pressure p* = F_n - rho* S*^2 on both sides of the contact, equal to
        p_K + rho_K (S_K - u_K)(S* - u_K) for K = L and for K = R;
      - the flux of a state moving with S* under pressure p*:
        F = (rho* S*, rho* S* v* + p* n, S* (E* + p*));
    and with the other side's star state built from the same conditions, the integral form
    (S* - S_L) U*_L + (S_R - S*) U*_R = S_R U_R - S_L U_L - (F_R - F_L) holds.
    Subsonic pairs (S_L < 0 < S_R) with S* != u_K on both branches (S* >= 0: left star,
    S* < 0: right star); Davis wave speeds as in the reading of Sec. 2.3."""
    rng = np.random.default_rng(300 + axis)
    tang = [j for j in range(3) if j != axis]
    branches = set()
    for qL, qR in _subsonic_pairs(rng, 60):
        rl, vl, pl, ul, cl = _prim(qL, axis)
        rr, vr, pr, ur, cr = _prim(qR, axis)
        SL, SR = min(ul - cl, ur - cr), max(ul + cl, ur + cr)
        assert SL < 0 < SR
        F = O.hllc(qL, qR, axis, G)
        FL, FR = O.euler_flux(qL, axis, G), O.euler_flux(qR, axis, G)
        # which star state the flux belongs to: try the left one, else the right one
        UsL = qL + (F - FL) / SL
        UsR = qR + (F - FR) / SR
        left = abs(F[0] / UsL[0] - UsL[1 + axis] / UsL[0]) < 1e-9
        K = "L" if left else "R"
        q, Us, SK, uK, pK, rK, vK = (qL, UsL, SL, ul, pl, rl, vl) if left else (qR, UsR, SR, ur, pr, rr, vr)
        rs = Us[0]
        assert rs > 0
        Ss = Us[1 + axis] / rs
        branches.add((K, Ss >= 0))
        assert (Ss >= 0) == left, "the upwind star state is the one on the side of the contact at the face"
        assert SL < Ss < SR
        assert abs(Ss - uK) > 1e-3, "the case must exercise S* != u_K"
        # mass flux carried by the contact velocity
        assert F[0] == pytest.approx(rs * Ss, rel=1e-12, abs=1e-13)
        # tangential velocities of side K, and their momentum fluxes
        for j in tang:
            assert Us[1 + j] / rs == pytest.approx(vK[j], rel=1e-12, abs=1e-13)
            assert F[1 + j] == pytest.approx(rs * Ss * vK[j], rel=1e-12, abs=1e-13)
        # one pressure across the contact: p* from the flux, and the HLLC pressure of both sides
        ps = F[1 + axis] - rs * Ss * Ss
        assert ps == pytest.approx(pl + rl * (SL - ul) * (Ss - ul), rel=1e-11)
        assert ps == pytest.approx(pr + rr * (SR - ur) * (Ss - ur), rel=1e-11)
        # energy flux of the star state
        assert F[4] == pytest.approx(Ss * (Us[4] + ps), rel=1e-11, abs=1e-12)
        # the other side's star state from the same conditions (mass and energy Rankine-Hugoniot
        # across its outer wave, velocity S*, its own tangential velocities, pressure p*)
        qo, So, Fo, vo = (qR, SR, FR, vr) if left else (qL, SL, FL, vl)
        ro = qo[0] * (So - Fo[0] / qo[0]) / (So - Ss)
        Uo = np.zeros(5)
        Uo[0] = ro
        Uo[1 + axis] = ro * Ss
        for j in tang:
            Uo[1 + j] = ro * vo[j]
        Uo[4] = (So * qo[4] - Fo[4] + Ss * ps) / (So - Ss)
        UL, UR = (Us, Uo) if left else (Uo, Us)
        lhs = (Ss - SL) * UL + (SR - Ss) * UR
        rhs = SR * qR - SL * qL - (FR - FL)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-12)
    assert branches == {("L", True), ("R", False)}, branches


def test_k0_is_first_order_godunov_fv():
    """k = 0 (one weight per field, Table 1): the volume term vanishes (the basis gradient is
    zero) and the surface term of eq. dg:eqn:surface_int reduces to the first-order Godunov
    finite-volume update R_K = sum_a (F(q_K, q_{K+a}) - F(q_{K-a}, q_K)) / h_a with the
    numerical flux of Sec. 2.3 at the face.  Built here cell by cell from the oracle's
    pointwise HLLC on a random positive state of an anisotropic mesh."""
    nc = (5, 4, 3)
    box = (1.0, 0.8, 1.5)
    cfg = O.make_cfg(0, nc, box=box)
    rng = np.random.default_rng(77)
    y = np.zeros((5, 1, nc[2], nc[1], nc[0]))
    for iz, iy, ix in itertools.product(range(nc[2]), range(nc[1]), range(nc[0])):
        y[:, 0, iz, iy, ix] = rand_state(rng)
    r = O.rhs(cfg, y)
    h = [box[a] / nc[a] for a in range(3)]
    want = np.zeros_like(y)
    for iz, iy, ix in itertools.product(range(nc[2]), range(nc[1]), range(nc[0])):
        q = y[:, 0, iz, iy, ix]
        acc = np.zeros(5)
        for a in range(3):
            d = [0, 0, 0]
            d[a] = 1
            up = y[:, 0, (iz + d[2]) % nc[2], (iy + d[1]) % nc[1], (ix + d[0]) % nc[0]]
            dn = y[:, 0, (iz - d[2]) % nc[2], (iy - d[1]) % nc[1], (ix - d[0]) % nc[0]]
            acc += (O.hllc(q, up, a, G) - O.hllc(dn, q, a, G)) / h[a]
        want[:, 0, iz, iy, ix] = acc
    np.testing.assert_allclose(r, want, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ operator

def turb_state(k, nc, seed=9079, mach=0.3):
    cfg = O.make_cfg(k, nc)
    qp = synth.turbulence(nc, nodes(k), seed=seed, mach=mach).numpy()
    return cfg, O.project(cfg, qp)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_free_stream_preservation(k):
    nc = (4, 3, 5)
    cfg = O.make_cfg(k, nc, box=(1.0, 0.75, 1.25))
    qp = synth.uniform_state(nc, nodes(k), rho=1.3, vel=(0.7, -0.4, 0.25), p=0.8)
    y = O.project(cfg, qp)
    r = O.rhs(cfg, y)
    assert np.abs(r).max() < 1e-12


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_conservation(k):
    """Only the surface term couples cells (Sec. 2.3): the cell-mean rows of R sum to zero."""
    cfg, y = turb_state(k, 6)
    r = O.rhs(cfg, y)
    s = r[:, 0].reshape(5, -1).sum(axis=1)
    scale = np.abs(r[:, 0]).reshape(5, -1).sum(axis=1)
    assert np.all(np.abs(s) <= 1e-13 * scale + 1e-14)
    t0 = O.totals(cfg, y)
    y1, _ = O.step(cfg, y, 0.0, 3)
    np.testing.assert_allclose(O.totals(cfg, y1), t0, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_linear_advection_special_case(k):
    """Uniform p and v: the Euler system reduces to linear advection of rho; the
    scheme keeps m = rho v and E = p/(g-1) + rho |v|^2/2 exactly, mode by mode."""
    nc = 5
    cfg = O.make_cfg(k, nc)
    y = O.project(cfg, synth.advected_wave(nc, nodes(k), gamma=G))
    y1, _ = O.step(cfg, y, 0.0, 4)
    for a in range(3):
        np.testing.assert_allclose(y1[1 + a], y1[0], atol=1e-14)
    want_E = 1.5 * y1[0]
    want_E[0] += 1.0 / (G - 1)
    np.testing.assert_allclose(y1[4], want_E, atol=1e-13)


def l2_error_vs_exact(cfg, y, t):
    """Continuous L2 error of rho against the exact advected wave, with a (k+3)^3 rule."""
    k = cfg.k
    m = k + 3
    x, w = O.gauss_legendre(m)
    nc = cfg.n[0]
    ex = synth.advected_wave(nc, x, gamma=G, t=t)[0]  # [c][b][a][z][y][x]
    err = 0.0
    for c, b, a in itertools.product(range(m), repeat=3):
        ph = O.basis(k, [x[a], x[b], x[c]])
        num = np.einsum("l...,l->...", y[0], ph)
        err += (w[a] * w[b] * w[c] / 8.0) * ((num - ex[c, b, a]) ** 2).sum()
    return math.sqrt(err / nc ** 3)


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_convergence_order_k_plus_1(k):
    """Sec. 2: spatial order p = k+1 on the smooth advected wave."""
    T = 0.02 if k < 4 else 0.004  # k = 4: fewer of its small steps
    errs = []
    sizes = [4, 8, 16]
    for nc in sizes:
        cfg = O.make_cfg(k, nc)
        y = O.project(cfg, synth.advected_wave(nc, nodes(k), gamma=G))
        dx = 1.0 / nc
        # SSP-RK3 is third order: for k >= 3 shrink dt like dx^((k+1)/3)
        h = 0.3 / (2 * k + 1) * dx / (3 * (1.0 + math.sqrt(G))) * (dx / 0.25) ** (max(k - 2, 0) / 3.0)
        ns = int(math.ceil(T / h))
        y1, t = O.step(cfg, y, T / ns, ns)
        errs.append(l2_error_vs_exact(cfg, y1, t))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > k + 1 - 0.3, (errs, rates)


def test_rk3_amplification_factor():
    """k = 0 with uniform v: one Fourier mode of rho is an eigenvector of the
    upwind operator; one SSP-RK3 step multiplies it by 1 + z + z^2/2 + z^3/6."""
    nc = 8
    cfg = O.make_cfg(0, nc)
    v = np.array([1.0, 0.5, 0.25])
    x = nodes(0)
    qp = synth.advected_wave(nc, x, gamma=G, vel=tuple(v))
    y = O.project(cfg, qp)
    h = 0.01
    y1, _ = O.step(cfg, y, h, 1)
    # complex Fourier coefficient of the rho perturbation for mode (1,1,1)
    idx = np.arange(nc)
    e = np.exp(-2j * np.pi * (idx[None, None, :] + idx[None, :, None] + idx[:, None, None]) / nc)
    c0 = (y[0, 0] * e).sum()
    c1 = (y1[0, 0] * e).sum()
    th = 2 * np.pi / nc
    lam = -sum(vi * nc * (1 - np.exp(-1j * th)) for vi in v)
    z = lam * h
    np.testing.assert_allclose(c1 / c0, 1 + z + z * z / 2 + z ** 3 / 6, rtol=1e-12)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_dt_closed_form_uniform(k):
    nc = (4, 5, 6)
    box = (1.0, 2.0, 0.5)
    cfg = O.make_cfg(k, nc, box=box, cfl=0.4)
    vel = (0.3, -0.5, 0.2)
    y = O.project(cfg, synth.uniform_state(nc, nodes(k), rho=1.2, vel=vel, p=0.7))
    c = math.sqrt(G * 0.7 / 1.2)
    rate = sum((abs(vel[a]) + c) / (box[a] / nc[a]) for a in range(3))
    assert O.dt(cfg, y) == pytest.approx(0.4 / (2 * k + 1) / rate, rel=1e-14)


def test_dt_advected_wave_first_step():
    """Config-1 start: dt from the 2-point-Gauss cell means; p-bar = 1 and
    v-bar = (1,1,1) in every cell, so dt = C/3 * dx / (3 (1 + c_max))."""
    cfg = O.make_cfg(1, 16)
    x = nodes(1)
    y = O.project(cfg, synth.advected_wave(16, x, gamma=G))
    rho_bar = y[0, 0]
    # independent: 2-point Gauss mean of the density in each cell
    X = (np.arange(16)[:, None] + 0.5 * (1 + x[None, :])) / 16  # [cell, gauss]
    ph = X[:, None, None, :, None, None] + X[None, :, None, None, :, None] + X[None, None, :, None, None, :]
    mean = (1 + 0.1 * np.sin(2 * np.pi * ph)).mean(axis=(3, 4, 5))
    np.testing.assert_allclose(np.transpose(rho_bar, (2, 1, 0)), mean, atol=1e-15)
    cmax = math.sqrt(G / mean.min())
    dt = 0.3 / 3 * (1 / 16) / (3 * (1 + cmax))
    assert O.dt(cfg, y) == pytest.approx(dt, rel=1e-13)
    assert dt == pytest.approx(8.8353e-4, rel=1e-4)
