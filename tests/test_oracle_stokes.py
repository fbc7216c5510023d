"""Pins of the Stokes-block oracle (gradient and divergence of the Taylor-Hood pair,
Section 3, eq. gradient and eq. divergence) against what the mathematics fixes:

* the gradient of a linear pressure a.x + c is the constant a, so (G p)_c = a_c M 1
  with M the velocity mass matrix (computed by the scalar oracle, without gradients);
* the divergence of a linear velocity A x + b is trace(A), so D u = trace(A) int psi;
* integration by parts: u . G p + p . D u = 0 for every p and every u that vanishes on
  the boundary;
* the constrained block operator keeps y_u = u on the Dirichlet DoFs and ignores their
  values in the divergence;
* planted mistakes (the Jacobian transposed, reference derivative directions swapped)
  fail the pins.
"""
import numpy as np
import pytest

from oracle import StokesDiscretization
from workloads import TaylorHoodMesh, uniform


def build(ne, p, q=None, seed=0):
    m = TaylorHoodMesh(ne, p, seed=seed)
    v = m.vel
    S = StokesDiscretization(v.elem_xyz, v.elem_dofs, v.ess, v.ndof, m.pres_dofs, m.npres, p,
                             p + 2 if q is None else q)
    return m, S


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_gradient_of_linear_pressure_is_constant(p):
    m, S = build(3, p)
    a, c0 = np.array([0.7, -1.3, 2.1]), 0.4
    xp = S.pressure_node_coords()
    pres = xp @ a + c0
    mass1 = S.vel.apply_unconstrained(np.ones(m.vel.ndof), 1.0, 0.0)
    g = S.gradient(pres)
    for c in range(3):
        assert rel(g[c], a[c] * mass1) <= 1e-13


@pytest.mark.parametrize("p", [2, 3, 4])
def test_divergence_of_linear_velocity_is_its_trace(p):
    m, S = build(3, p)
    A = np.array([[0.3, -0.2, 0.5], [1.1, -0.4, 0.25], [-0.6, 0.8, 0.9]])
    b = np.array([0.1, -0.2, 0.3])
    xv = S.velocity_node_coords()
    u = (xv @ A.T + b).T  # [3, nv]
    du = S.divergence(u)
    assert rel(du, np.trace(A) * S.pressure_mass_rowsums()) <= 1e-13
    # the volume of the unit cube
    assert abs(S.pressure_mass_rowsums().sum() - 1.0) <= 1e-13


@pytest.mark.parametrize("p", [2, 4])
def test_integration_by_parts(p):
    m, S = build(3, p)
    u = uniform(3 * m.vel.ndof, seed=7).reshape(3, -1)
    u[:, m.vel.ess.astype(bool)] = 0.0
    pres = uniform(m.npres, seed=8)
    lhs = np.sum(u * S.gradient(pres))
    rhs = pres @ S.divergence(u)
    assert abs(lhs + rhs) <= 1e-13 * (abs(lhs) + abs(rhs))
    assert abs(lhs) > 1e-3


def test_constrained_block_operator():
    m, S = build(2, 3)
    ess = m.vel.ess.astype(bool)
    u = uniform(3 * m.vel.ndof, seed=9).reshape(3, -1)
    pres = uniform(m.npres, seed=10)
    yu, yp = S.apply(u, pres, 5.0, 0.5)
    assert np.array_equal(yu[:, ess], u[:, ess])
    ub = np.zeros_like(u)
    ub[:, ess] = u[:, ess]
    _, yp_b = S.apply(ub, np.zeros(m.npres), 5.0, 0.5)
    assert np.all(yp_b == 0.0)
    # linear in (u, p), and the free rows are the unconstrained blocks on P u
    uf = u.copy()
    uf[:, ess] = 0.0
    g = S.gradient(pres)
    for c in range(3):
        h = S.vel.apply_unconstrained(uf[c], 5.0, 0.5)
        assert rel(yu[c, ~ess], h[~ess] + g[c, ~ess]) <= 1e-14
    assert rel(yp, -S.divergence(uf)) <= 1e-15


def test_quadrature_is_exact_for_the_blocks():
    """On trilinear maps the integrands are polynomials of degree <= 2p + 1 per variable,
    so q = p + 2 Gauss points integrate them exactly: more points give the same blocks."""
    m, S = build(2, 3)
    _, S2 = build(2, 3, q=7)
    pres = uniform(m.npres, seed=11)
    u = uniform(3 * m.vel.ndof, seed=12).reshape(3, -1)
    assert rel(S.gradient(pres), S2.gradient(pres)) <= 1e-13
    assert rel(S.divergence(u), S2.divergence(u)) <= 1e-13


class _TransposedJ(StokesDiscretization):
    def element_blocks(self, e0, e1):
        det, inv, _ = self.vel.geometry(e0, e1)
        wd = self.vel.Wq[None, :] * det
        gpsi = np.einsum("cQrd,Qmd->cQmr", inv, self.dPsi)  # J^{-1} instead of J^{-T}
        gphi = np.einsum("cQrd,Qld->cQlr", inv, self.vel.dPhi)
        G = np.einsum("eQ,Ql,eQmc->eclm", wd, self.vel.Phi, gpsi)
        D = np.einsum("eQ,Qm,eQlc->emcl", wd, self.Psi, gphi)
        return G, D


def test_planted_mistakes_fail_the_pins():
    m = TaylorHoodMesh(3, 2)
    v = m.vel
    T = _TransposedJ(v.elem_xyz, v.elem_dofs, v.ess, v.ndof, m.pres_dofs, m.npres, 2, 4)
    a = np.array([0.7, -1.3, 2.1])
    mass1 = T.vel.apply_unconstrained(np.ones(v.ndof), 1.0, 0.0)
    g = T.gradient(T.pressure_node_coords() @ a)
    assert max(rel(g[c], a[c] * mass1) for c in range(3)) > 1e-6
    # reference derivative directions swapped (d/dxi_1 <-> d/dxi_3) in the divergence
    _, S = build(3, 2)
    S.vel.dPhi = S.vel.dPhi[..., ::-1].copy()
    A = np.array([[0.3, -0.2, 0.5], [1.1, -0.4, 0.25], [-0.6, 0.8, 0.9]])
    u = (S.velocity_node_coords() @ A.T).T
    assert rel(S.divergence(u), np.trace(A) * S.pressure_mass_rowsums()) > 1e-3
