"""Pins of the oracle's tables: mode count, mode list, Gauss rule, scaled Legendre
basis (Sec. 2.1, 2.2 of arXiv 1602.09079)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_mode_count_matches_table1():
    g = json.load(open(os.path.join(GOLD, "table1_dof.json")))
    for k, N, r in zip(g["k"], g["N"], g["dof_per_cell_cuberoot"]):
        assert O.nmodes(k) == N
        assert round(N ** (1.0 / 3.0), 2) == pytest.approx(r)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_mode_list_is_the_total_degree_set(k):
    ml = [tuple(r) for r in O.mode_list(k)]
    want = {(u, v, w) for u in range(k + 1) for v in range(k + 1) for w in range(k + 1) if u + v + w <= k}
    assert len(ml) == len(set(ml)) == len(want)
    assert set(ml) == want
    assert ml[0] == (0, 0, 0)
    # graded: total degree never decreases; lower-degree list is a prefix
    degs = [sum(m) for m in ml]
    assert degs == sorted(degs)
    if k > 0:
        assert ml[: O.nmodes(k - 1)] == [tuple(r) for r in O.mode_list(k - 1)]


def test_mode_list_k1_order():
    assert O.mode_list(1).tolist() == [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]


def _closed(expr):
    return eval(expr, {"sqrt": math.sqrt})


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_gauss_rule_closed_forms(n):
    g = json.load(open(os.path.join(GOLD, "gauss_legendre.json")))["rules"][str(n)]
    x, w = O.gauss_legendre(n)
    np.testing.assert_allclose(x, [_closed(e) for e in g["x"]], rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, [_closed(e) for e in g["w"]], rtol=0, atol=4e-16)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_rule_matches_library_and_is_exact(n):
    x, w = O.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)
    # exact for every monomial of degree <= 2n - 1 (Sec. 2.2)
    for j in range(2 * n):
        exact = 0.0 if j % 2 else 2.0 / (j + 1)
        assert abs(np.dot(w, x ** j) - exact) < 1e-14
    # and not for degree 2n
    assert abs(np.dot(w, x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6


def test_scaled_legendre_closed_forms():
    s3, s5, s7 = math.sqrt(3), math.sqrt(5), math.sqrt(7)
    for x in np.linspace(-1, 1, 13):
        assert O.pleg(0, x) == pytest.approx(1.0, abs=1e-15)
        assert O.pleg(1, x) == pytest.approx(s3 * x, abs=1e-15)
        assert O.pleg(2, x) == pytest.approx(s5 * (3 * x * x - 1) / 2, abs=1e-14)
        assert O.pleg(3, x) == pytest.approx(s7 * (5 * x ** 3 - 3 * x) / 2, abs=1e-14)
        assert O.dpleg(0, x) == 0.0
        assert O.dpleg(1, x) == pytest.approx(s3, abs=1e-15)
        assert O.dpleg(2, x) == pytest.approx(s5 * 3 * x, abs=1e-14)
        assert O.dpleg(3, x) == pytest.approx(s7 * (15 * x * x - 3) / 2, abs=1e-14)
    for u in range(6):
        assert O.pleg(u, 1.0) == pytest.approx(math.sqrt(2 * u + 1), abs=1e-14)
        assert O.pleg(u, -1.0) == pytest.approx((-1) ** u * math.sqrt(2 * u + 1), abs=1e-14)
        # against numpy's Legendre series
        c = np.zeros(u + 1)
        c[u] = math.sqrt(2 * u + 1)
        for x in (-0.93, -0.2, 0.41, 0.77):
            assert O.pleg(u, x) == pytest.approx(np.polynomial.legendre.legval(x, c), abs=1e-14)
            assert O.dpleg(u, x) == pytest.approx(np.polynomial.legendre.legval(x, np.polynomial.legendre.legder(c)),
                                                  abs=1e-13)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_basis_orthonormal_under_gauss_rule(k):
    """(1/8) sum_q phi_l phi_m w_q = delta_lm with (k+1)^3 points (degree 2k <= 2k+1)."""
    n = k + 1
    x, w = O.gauss_legendre(n)
    N = O.nmodes(k)
    G = np.zeros((N, N))
    for a, b, c in itertools.product(range(n), repeat=3):
        ph = O.basis(k, [x[a], x[b], x[c]])
        G += np.outer(ph, ph) * w[a] * w[b] * w[c] / 8.0
    np.testing.assert_allclose(G, np.eye(N), atol=2e-15)


def test_basis_gradient_by_finite_differences():
    k = 3
    rng = np.random.default_rng(1)
    for _ in range(5):
        xi = rng.uniform(-0.9, 0.9, 3)
        d = O.basis_grad(k, xi)
        h = 1e-6
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            fd = (O.basis(k, xi + e) - O.basis(k, xi - e)) / (2 * h)
            np.testing.assert_allclose(d[a], fd, atol=1e-8)
