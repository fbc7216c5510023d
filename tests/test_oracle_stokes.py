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


# ---------------------------------------------------------------- convection N(u)
def _vel_nodes(ne, p, seed=0):
    from oracle import Discretization
    from workloads import BoxMesh
    m = BoxMesh(ne, p, seed=seed)
    d = Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2)
    # velocity node coordinates through the Stokes helper (any pressure map will do)
    pm = BoxMesh(ne, max(p - 1, 1), seed=seed)
    S = StokesDiscretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, pm.elem_dofs, pm.ndof,
                             max(p, 2), p + 2) if p >= 2 else None
    return m, d, S


@pytest.mark.parametrize("p", [2, 3, 4])
def test_convection_of_linear_velocity(p):
    """u = A x + b is linear, so (u . grad) u = A (A x + b) is linear too and lies in the
    velocity space: N(u)_c = M (A (A x + b))_c on the free rows, with the unconstrained
    mass matrix of the scalar oracle (no gradients involved)."""
    from oracle import convection
    m, d, S = _vel_nodes(3, p)
    A = np.array([[0.3, -0.2, 0.5], [1.1, -0.4, 0.25], [-0.6, 0.8, 0.9]])
    b = np.array([0.1, -0.2, 0.3])
    x = S.velocity_node_coords()
    u = (x @ A.T + b).T
    adv = ((x @ A.T + b) @ A.T).T  # A (A x + b), [3, N]
    y = convection(d, u)
    free = ~m.ess.astype(bool)
    for c in range(3):
        ref = d.apply_unconstrained(adv[c], 1.0, 0.0)
        assert rel(y[c, free], ref[free]) <= 1e-13
    assert np.all(y[:, ~free] == 0.0)


def test_convection_is_quadratic_and_vanishes_for_constants():
    from oracle import convection
    m, d, S = _vel_nodes(2, 3)
    u = uniform(3 * m.ndof, seed=13).reshape(3, -1)
    assert rel(convection(d, 2.0 * u), 4.0 * convection(d, u)) <= 1e-14
    c0 = np.stack([np.full(m.ndof, v) for v in (0.3, -1.0, 2.0)])
    assert np.abs(convection(d, c0)).max() <= 1e-13


def test_convection_planted_transpose_fails():
    """J^{-1} in place of J^{-T} in the physical gradient breaks the linear-field pin."""
    import oracle.stokes as st
    m, d, S = _vel_nodes(3, 2)
    A = np.array([[0.3, -0.2, 0.5], [1.1, -0.4, 0.25], [-0.6, 0.8, 0.9]])
    x = S.velocity_node_coords()
    u = (x @ A.T).T
    adv = ((x @ A.T) @ A.T).T
    orig = np.einsum
    def wrong(spec, *ops, **kw):
        if spec == "eQkr,eQck->eQcr":
            spec = "eQrk,eQck->eQcr"
        return orig(spec, *ops, **kw)
    st.np.einsum = wrong
    try:
        y = st.convection(d, u)
    finally:
        st.np.einsum = orig
    free = ~m.ess.astype(bool)
    ref = d.apply_unconstrained(adv[0], 1.0, 0.0)
    assert rel(y[0, free], ref[free]) > 1e-6


def test_fan_mesh_blocks_pins():
    """On the unstructured fan mesh (axis nodes shared by 3 or 6 elements, pressure map
    from the same mesh at order p - 1) the linear-field pins of the gradient, the
    divergence and the convection term hold as on the box."""
    from oracle import Discretization, convection
    from workloads import FanMesh
    p = 3
    m, pm = FanMesh(p), FanMesh(p - 1)
    S = StokesDiscretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, pm.elem_dofs, pm.ndof, p,
                             p + 2)
    a = np.array([0.7, -1.3, 2.1])
    mass1 = S.vel.apply_unconstrained(np.ones(m.ndof), 1.0, 0.0)
    g = S.gradient(S.pressure_node_coords() @ a + 0.4)
    for c in range(3):
        assert rel(g[c], a[c] * mass1) <= 1e-13
    A = np.array([[0.3, -0.2, 0.5], [1.1, -0.4, 0.25], [-0.6, 0.8, 0.9]])
    b = np.array([0.1, -0.2, 0.3])
    x = S.velocity_node_coords()
    u = (x @ A.T + b).T
    assert rel(S.divergence(u), np.trace(A) * S.pressure_mass_rowsums()) <= 1e-13
    assert abs(S.pressure_mass_rowsums().sum() - 3 * np.sin(np.pi / 3)) <= 1e-13
    d = Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2)
    y = convection(d, u)
    adv = ((x @ A.T + b) @ A.T).T
    free = ~m.ess.astype(bool)
    for c in range(3):
        ref = d.apply_unconstrained(adv[c], 1.0, 0.0)
        assert rel(y[c, free], ref[free]) <= 1e-13
