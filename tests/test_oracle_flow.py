"""Pins of the projection-step oracle (Section 4.2; oracle/flow.py) against what the
mathematics fixes:

* BDF-k and EXT-k are exact for polynomials in t of degree k and k - 1;
* the weak gradient of a linear s = a.x + c is a_c M1, the weak curl of a linear
  u = A x + b is curl(u)_c M1 with curl(u) read off A, the weak divergence satisfies
  sum_i q_i r_i = a . int V for q = a.x + c and vanishes against constants;
* the weak gradient and the weak divergence are transposes: s . div_w(V) = V . grad_w(s);
* a hydrostatic step: u = 0 and a gradient forcing f = grad phi (phi quadratic, affine
  mesh) is balanced by the pressure alone: p = phi - mean, u^{n+1} = 0;
* the time integration converges at its order: self-convergence in the step size
  (differences between runs at dt, dt/2, dt/4 to the same time) at rate ~1 for BDF1/EXT1
  and ~2 for BDF2/EXT2 on a 4^3, p = 4 mesh (on coarser meshes the differences stall at
  the mesh's equal-order consistency error);
* a manufactured Navier-Stokes solution (no-slip walls, nonzero convection and
  nonzero normal curl curl u on the walls): the errors of the steps against the exact
  velocity and pressure fall at rate ~1 (BDF1/EXT1) and ~2 (BDF2/EXT2) in the step size;
* planted mistakes (a sign in the curl, a dropped pressure gradient, a wrong BDF
  weight, a flipped or unscaled rotational term, a flipped convection term) fail the
  pins.
"""
import numpy as np
import pytest

import oracle.flow as fl
from oracle import Discretization
from workloads import BoxMesh, uniform

A = np.array([[0.3, -0.2, 0.5], [1.1, -0.4, 0.25], [-0.6, 0.8, 0.9]])
B0 = np.array([0.1, -0.2, 0.3])


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def disc(ne, p, amp=0.1, ess=True):
    m = BoxMesh(ne, p, amp=amp)
    e = m.ess if ess else np.zeros(m.ndof, dtype=np.uint8)
    return m, Discretization(m.elem_xyz, m.elem_dofs, e, m.ndof, p, p + 2)


def nodes(m, p):
    from oracle.fem import trilinear_shape
    from oracle.quadrature import gll
    pn, _ = gll(p)
    n = p + 1
    l = np.arange(n ** 3)
    XI = np.stack([pn[l % n], pn[(l // n) % n], pn[l // (n * n)]], axis=-1)
    N, _ = trilinear_shape(XI)
    x = np.zeros((m.ndof, 3))
    x[m.elem_dofs.reshape(-1)] = np.einsum("evr,mv->emr", m.elem_xyz, N).reshape(-1, 3)
    return x


@pytest.mark.parametrize("k", [1, 2, 3])
def test_bdf_ext_orders(k):
    b, a = fl.bdf_ext(k)
    t = 1.0 - np.arange(k + 1)  # t_{n+1-j} with dt = 1, t_{n+1} = 1
    for m in range(k + 1):  # d/dt t^m at t = 1
        assert abs(b @ t ** m - m) <= 1e-14
    for m in range(k):  # t^m at t = 1 from t_n, ..., t_{n+1-k}
        assert abs(a @ t[1:] ** m - 1.0) <= 1e-14
    assert abs(a @ t[1:] ** k - 1.0) > 1e-3  # not one degree more


@pytest.mark.parametrize("p", [2, 3])
def test_linear_fields(p):
    m, d = disc(3, p, ess=False)
    x = nodes(m, p)
    m1 = d.apply_unconstrained(np.ones(m.ndof), 1.0, 0.0)
    a = np.array([0.7, -1.3, 2.1])
    g = fl.weak_gradient(d, x @ a + 0.4)
    for c in range(3):
        assert rel(g[c], a[c] * m1) <= 1e-13
    u = (x @ A.T + B0).T
    curl = np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    w = fl.weak_curl(d, u)
    for c in range(3):
        assert rel(w[c], curl[c] * m1) <= 1e-13
    r = fl.weak_divergence(d, u)
    assert abs(r.sum()) <= 1e-13 * np.abs(r).sum()
    q = x @ a + 0.4
    assert abs(q @ r - sum(a[c] * (m1 @ u[c]) for c in range(3))) <= 1e-13 * np.abs(q * r).sum()
    # constants: no curl, no gradient
    assert np.abs(fl.weak_curl(d, np.ones((3, m.ndof)))).max() <= 1e-14
    assert np.abs(fl.weak_gradient(d, np.full(m.ndof, 2.5))).max() <= 1e-14


def test_gradient_and_divergence_are_transposes():
    m, d = disc(2, 3, ess=False)
    s = uniform(m.ndof, seed=3)
    v = uniform(3 * m.ndof, seed=4).reshape(3, -1)
    lhs = s @ fl.weak_divergence(d, v)
    rhs = np.sum(v * fl.weak_gradient(d, s))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("p", [2, 3])
def test_hydrostatic_step(p):
    """u = 0 and f = grad phi, phi = x^2 - y z + 0.5 z on an affine mesh (phi in V_h):
    the pressure takes all of the forcing (p = phi - int phi), the velocity stays 0."""
    m, d = disc(2, p, amp=0.0)
    x = nodes(m, p)
    phi = x[:, 0] ** 2 - x[:, 1] * x[:, 2] + 0.5 * x[:, 2]
    f = np.stack([2 * x[:, 0], -x[:, 2], -x[:, 1] + 0.5])
    st = fl.ProjectionStepper(d, dt=0.01, nu=0.1, order=2)
    un, pn = st.step(np.zeros((3, m.ndof)), f)
    m1 = st.m1
    assert rel(pn, phi - (m1 @ phi) / m1.sum()) <= 1e-12
    assert np.abs(un).max() <= 1e-12 * np.abs(f).max()


def test_planted_mistakes_fail():
    m, d = disc(3, 2, ess=False)
    x = nodes(m, 2)
    m1 = d.apply_unconstrained(np.ones(m.ndof), 1.0, 0.0)
    u = (x @ A.T + B0).T
    curl = np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    orig = fl.curl_of
    # first component with the wrong sign
    fl.curl_of = lambda g: np.stack([g[..., 1, 2] - g[..., 2, 1], g[..., 0, 2] - g[..., 2, 0],
                                     g[..., 1, 0] - g[..., 0, 1]], axis=-1)
    try:
        w = fl.weak_curl(d, u)
    finally:
        fl.curl_of = orig
    assert rel(w[0], curl[0] * m1) > 1e-3
    # the pressure gradient dropped from the Helmholtz right-hand side: the hydrostatic
    # balance fails
    m2, d2 = disc(2, 2, amp=0.0)
    x2 = nodes(m2, 2)
    f = np.stack([2 * x2[:, 0], -x2[:, 2], -x2[:, 1] + 0.5])
    og = fl.weak_gradient
    fl.weak_gradient = lambda dd, s: np.zeros((3, dd.ndof))
    try:
        un, _ = fl.ProjectionStepper(d2, dt=0.01, nu=0.1).step(np.zeros((3, m2.ndof)), f)
    finally:
        fl.weak_gradient = og
    assert np.abs(un).max() > 1e-4


def _self_convergence(order, bdf=None):
    m, d = disc(4, 4, amp=0.0)
    x = nodes(m, 4)
    f = np.stack([10 * np.sin(np.pi * x[:, 2]), 10 * x[:, 0] * x[:, 1], 10 * np.cos(np.pi * x[:, 0])])
    T, res = 0.05, []
    orig = fl.bdf_ext
    if bdf is not None:
        fl.bdf_ext = bdf
    try:
        for nsteps in (5, 10, 20):
            st = fl.ProjectionStepper(d, dt=T / nsteps, nu=0.1, order=order)
            u = np.zeros((3, m.ndof))
            for _ in range(nsteps):
                u, _p = st.step(u, f)
            res.append(u)
    finally:
        fl.bdf_ext = orig
    e = [np.linalg.norm(res[i] - res[i + 1]) for i in range(2)]
    return np.log2(e[0] / e[1])


@pytest.mark.parametrize("order,lo,hi", [(1, 0.8, 1.2), (2, 1.7, 2.3)])
def test_time_integration_order(order, lo, hi):
    rate = _self_convergence(order)
    assert lo <= rate <= hi, rate


def test_wrong_bdf_weight_loses_the_order():
    good = fl.bdf_ext

    def bad(k):
        b, a = good(k)
        b = b.copy()
        if k == 2:
            b[2] = 0.45  # instead of 1/2
        return b, a
    rate = _self_convergence(2, bad)
    assert not (1.7 <= rate <= 2.3), rate


# ---------------------------------------------------------------------------------
# Manufactured Navier-Stokes solution (tests/ns_manufactured.py): the errors of the
# oracle's steps against the exact velocity and pressure fall at the scheme's order in
# the step size, and each term of the step is pinned by a planted mistake that breaks
# the convergence: the sign of the rotational term L* (eq. projLinear), its factor nu,
# and the sign of the extrapolated convection term N* (eq. projKnown).  3^3 affine
# mesh, p = 4, nu = 0.1, T = 0.3; the time errors stay above the spatial floor for
# 8 and 16 steps.
from ns_manufactured import run as ns_run  # noqa: E402  (tests/ is on the path)

NS_NU, NS_T = 0.1, 0.3


def _ns(order, nsteps, cls=fl.ProjectionStepper):
    m, d = disc(3, 4, amp=0.0)
    x = nodes(m, 4)
    m1 = d.apply_unconstrained(np.ones(m.ndof), 1.0, 0.0)
    eu, ep, _, _ = ns_run(lambda dt: cls(d, dt=dt, nu=NS_NU, order=order), x, m1, NS_NU, NS_T, nsteps)
    return eu, ep


@pytest.mark.parametrize("order,lo,hi,plo", [(1, 0.8, 1.2, 0.8), (2, 1.6, 2.4, 1.6)])
def test_manufactured_navier_stokes_converges_in_time(order, lo, hi, plo):
    eu8, ep8 = _ns(order, 8)
    eu16, ep16 = _ns(order, 16)
    ru, rp = np.log2(eu8 / eu16), np.log2(ep8 / ep16)
    assert lo <= ru <= hi, (eu8, eu16, ru)
    assert rp >= plo, (ep8, ep16, rp)
    if order == 2:
        assert eu16 < 5e-3 and ep16 < 0.3, (eu16, ep16)


class _FlippedRotational(fl.ProjectionStepper):
    def rotational_term(self, ustar):
        return -super().rotational_term(ustar)


class _RotationalWithoutNu(fl.ProjectionStepper):
    def rotational_term(self, ustar):
        return super().rotational_term(ustar) / self.nu


class _FlippedConvection(fl.ProjectionStepper):
    def convection_term(self, u):
        return -super().convection_term(u)


@pytest.mark.parametrize("cls", [_FlippedRotational, _RotationalWithoutNu, _FlippedConvection])
def test_manufactured_navier_stokes_rejects_planted_terms(cls):
    good, _ = _ns(2, 16)
    with np.errstate(all="ignore"):
        bad, _ = _ns(2, 16, cls)
    assert not np.isfinite(bad) or bad > 5 * good, (good, bad)
