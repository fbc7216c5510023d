"""Pins of the oracle's 1D rules and basis against textbook closed forms and exactness.

The Gauss-Legendre and Gauss-Lobatto closed forms are the classical tabulated
rules (e.g. Abramowitz & Stegun, Table 25.4 and eq. 25.4.32); the polynomial
exactness degrees (2q-1 for Gauss, 2p-1 for Lobatto with p+1 points) are the
defining properties of the rules used in Section 3.1.
"""
import numpy as np
import pytest

from oracle import gauss_legendre, gll, lagrange_values, lagrange_derivs

S = np.sqrt

GAUSS_CLOSED = {
    1: ([0.0], [2.0]),
    2: ([-1 / S(3), 1 / S(3)], [1.0, 1.0]),
    3: ([-S(3 / 5), 0.0, S(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    4: ([-S(3 / 7 + 2 / 7 * S(6 / 5)), -S(3 / 7 - 2 / 7 * S(6 / 5)),
         S(3 / 7 - 2 / 7 * S(6 / 5)), S(3 / 7 + 2 / 7 * S(6 / 5))],
        [(18 - S(30)) / 36, (18 + S(30)) / 36, (18 + S(30)) / 36, (18 - S(30)) / 36]),
    5: ([-S(5 + 2 * S(10 / 7)) / 3, -S(5 - 2 * S(10 / 7)) / 3, 0.0,
         S(5 - 2 * S(10 / 7)) / 3, S(5 + 2 * S(10 / 7)) / 3],
        [(322 - 13 * S(70)) / 900, (322 + 13 * S(70)) / 900, 128 / 225,
         (322 + 13 * S(70)) / 900, (322 - 13 * S(70)) / 900]),
}

GLL_CLOSED = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / S(5), 1 / S(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -S(3 / 7), 0.0, S(3 / 7), 1.0], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
    5: ([-1.0, -S(1 / 3 + 2 * S(7) / 21), -S(1 / 3 - 2 * S(7) / 21),
         S(1 / 3 - 2 * S(7) / 21), S(1 / 3 + 2 * S(7) / 21), 1.0],
        [1 / 15, (14 - S(7)) / 30, (14 + S(7)) / 30, (14 + S(7)) / 30, (14 - S(7)) / 30, 1 / 15]),
}


def exact_monomial(k):
    return 0.0 if k % 2 else 2.0 / (k + 1)


@pytest.mark.parametrize("q", sorted(GAUSS_CLOSED))
def test_gauss_closed_forms(q):
    x, w = gauss_legendre(q)
    xr, wr = GAUSS_CLOSED[q]
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=1e-15, rtol=0)


@pytest.mark.parametrize("q", range(1, 13))
def test_gauss_exactness(q):
    x, w = gauss_legendre(q)
    for k in range(2 * q):
        assert abs(np.dot(w, x ** k) - exact_monomial(k)) < 2e-15
    # and not beyond: degree 2q is integrated with an error
    assert abs(np.dot(w, x ** (2 * q)) - exact_monomial(2 * q)) > 1e-12


@pytest.mark.parametrize("q", range(1, 13))
def test_gauss_matches_numpy(q):
    x, w = gauss_legendre(q)
    xr, wr = np.polynomial.legendre.leggauss(q)
    assert np.allclose(x, xr, atol=2e-15, rtol=0)
    assert np.allclose(w, wr, atol=2e-15, rtol=0)


@pytest.mark.parametrize("p", sorted(GLL_CLOSED))
def test_gll_closed_forms(p):
    x, w = gll(p)
    xr, wr = GLL_CLOSED[p]
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=1e-15, rtol=0)


@pytest.mark.parametrize("p", range(1, 11))
def test_gll_exactness_and_roots(p):
    x, w = gll(p)
    assert x[0] == -1.0 and x[-1] == 1.0
    for k in range(2 * p):
        assert abs(np.dot(w, x ** k) - exact_monomial(k)) < 3e-15
    assert abs(np.dot(w, x ** (2 * p)) - exact_monomial(2 * p)) > 1e-12
    # interior nodes are the roots of P_p'
    if p > 1:
        dP = np.polynomial.legendre.Legendre.basis(p).deriv()
        assert np.abs(dP(x[1:-1])).max() < 1e-12 * max(1.0, np.abs(dP.coef).max())


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_tables(p):
    nodes, _ = gll(p)
    # cardinality at the nodes
    assert np.allclose(lagrange_values(nodes, nodes), np.eye(p + 1), atol=1e-14)
    xi, _ = gauss_legendre(p + 2)
    B = lagrange_values(nodes, xi)
    D = lagrange_derivs(nodes, xi)
    assert np.allclose(B.sum(1), 1.0, atol=1e-14)
    assert np.allclose(D.sum(1), 0.0, atol=1e-13)
    for k in range(p + 1):
        # B reproduces xi^k and D differentiates it exactly (degree <= p)
        assert np.allclose(B @ nodes ** k, xi ** k, atol=1e-13)
        want = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.allclose(D @ nodes ** k, want, atol=2e-12)


def test_lagrange_derivative_against_finite_difference():
    nodes, _ = gll(5)
    pts = np.linspace(-0.9, 0.9, 7)
    h = 1e-6
    fd = (lagrange_values(nodes, pts + h) - lagrange_values(nodes, pts - h)) / (2 * h)
    assert np.allclose(lagrange_derivs(nodes, pts), fd, atol=1e-7)
