"""Oracle 1D rules and nodal basis (test infrastructure; FP64, numpy).

* Gauss-Legendre rule with q points (the tensor quadrature of Section 3.1; the
  paper leaves the number of points open, the reading used here is q = p + 2).
  Nodes are the eigenvalues of the symmetric Jacobi matrix of the Legendre
  three-term recurrence, weights are 2 * (first eigenvector component)^2
  (Golub-Welsch).
* Gauss-Lobatto-Legendre (GLL) nodes for the nodal basis of Section 3 (p+1
  points): the end points +-1 and the roots of P_p', which are the Gauss points of
  the Jacobi weight (1-x)(1+x) (Jacobi alpha = beta = 1 recurrence, Golub-Welsch
  again).  Weights 2 / (p (p+1) P_p(x_j)^2).
* 1D Lagrange basis phi_j on the GLL nodes and its derivative, evaluated by the
  product formula (Section 3.1, the tables B and D of eq. B1D / eq. D1D).
"""
from __future__ import annotations

import numpy as np


def gauss_legendre(q: int):
    """q-point Gauss-Legendre rule on [-1, 1]: (nodes ascending, weights)."""
    if q < 1:
        raise ValueError("q >= 1")
    if q == 1:
        return np.array([0.0]), np.array([2.0])
    k = np.arange(1, q, dtype=np.float64)
    off = k / np.sqrt(4.0 * k * k - 1.0)
    T = np.diag(off, 1) + np.diag(off, -1)
    lam, V = np.linalg.eigh(T)
    w = 2.0 * V[0, :] ** 2
    order = np.argsort(lam)
    x, w = lam[order], w[order]
    # the rule is symmetric: symmetrise away the eigen-solver's last-bit noise
    x = 0.5 * (x - x[::-1])
    w = 0.5 * (w + w[::-1])
    return x, w


def legendre_p(n: int, x):
    """Legendre polynomial P_n(x) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p1


def gll(p: int):
    """(p+1)-point Gauss-Lobatto-Legendre rule on [-1, 1]: (nodes ascending, weights)."""
    if p < 1:
        raise ValueError("p >= 1")
    m = p - 1  # interior nodes = roots of P_p'
    if m == 0:
        inner = np.zeros(0)
    elif m == 1:
        inner = np.array([0.0])
    else:
        k = np.arange(1, m, dtype=np.float64)
        # monic Jacobi(1,1) recurrence: b_k = k (k+2) / ((2k+1)(2k+3))
        off = np.sqrt(k * (k + 2.0) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)))
        T = np.diag(off, 1) + np.diag(off, -1)
        inner = np.sort(np.linalg.eigvalsh(T))
    x = np.concatenate([[-1.0], inner, [1.0]])
    x = 0.5 * (x - x[::-1])
    w = 2.0 / (p * (p + 1) * legendre_p(p, x) ** 2)
    w = 0.5 * (w + w[::-1])
    return x, w


def lagrange_values(nodes, pts):
    """V[a, j] = phi_j(pts[a]) for the Lagrange basis on ``nodes``."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    n = nodes.size
    V = np.ones((pts.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                V[:, j] *= (pts - nodes[m]) / (nodes[j] - nodes[m])
    return V


def lagrange_derivs(nodes, pts):
    """D[a, j] = phi_j'(pts[a]) (sum over the dropped factor of the product rule)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(pts, dtype=np.float64)
    n = nodes.size
    D = np.zeros((pts.size, n))
    for j in range(n):
        for r in range(n):
            if r == j:
                continue
            term = np.full(pts.size, 1.0 / (nodes[j] - nodes[r]))
            for m in range(n):
                if m != j and m != r:
                    term *= (pts - nodes[m]) / (nodes[j] - nodes[m])
            D[:, j] += term
    return D
