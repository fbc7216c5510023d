"""Pins of the oracle solvers (Section 5, Section 5.3) and of the discretization as a whole.

* Jacobi-PCG reaches the sparse direct solution of the constrained system.
* Manufactured Poisson problem -Lap u = 3 pi^2 u, u = sin(pi x) sin(pi y) sin(pi z),
  homogeneous Dirichlet: the L2 error decays at rate p + 1 (the high-order accuracy
  the paper observes for smooth solutions).
* FP32-inner iterative refinement reaches the FP64 true-residual bound.
* Adjoint gradient: central finite differences of J with exact (direct) solves, the
  homogeneity identity sum_Q nu_Q dJ/dnu_Q = -beta lambda^T K(nu) u (K linear in nu),
  and planted mistakes that these reject.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import Discretization, pcg, ir_pcg, adjoint_gradient, objective
from workloads import BoxMesh, f_manufactured, u_manufactured, rhs_uniform, nu_uniform


def make(ne, p, seed=0):
    m = BoxMesh(ne, p, seed=seed)
    return m, Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2)


def poisson_rhs(m, d):
    xq = d.qpoint_coords()
    return d.load(f_manufactured(xq[..., 0], xq[..., 1], xq[..., 2]))


def test_pcg_matches_direct_solve_poisson_p2_4e():
    m, d = make(4, 2)
    b = poisson_rhs(m, d)
    A = d.assemble(0.0, 1.0)
    x_direct = spla.spsolve(A.tocsc(), b)
    dinv = 1.0 / d.diagonal(0.0, 1.0)
    x, it, rr = pcg(lambda v: d.apply(v, 0.0, 1.0), b, dinv, rtol=1e-12)
    assert rr <= 1e-12
    assert np.linalg.norm(b - A @ x) <= 1e-11 * np.linalg.norm(b)
    assert np.linalg.norm(x - x_direct) <= 1e-9 * np.linalg.norm(x_direct)
    assert 5 < it < 200


@pytest.mark.parametrize("p,meshes", [(1, [2, 4, 8]), (2, [2, 4, 8]), (3, [2, 4, 6])])
def test_manufactured_poisson_rate(p, meshes):
    errs, hs = [], []
    for ne in meshes:
        m, d = make(ne, p)
        b = poisson_rhs(m, d)
        u = spla.spsolve(d.assemble(0.0, 1.0).tocsc(), b)
        errs.append(d.l2_error(u, u_manufactured))
        hs.append(1.0 / ne)
    rates = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert rates[-1] >= p + 1 - 0.3, (errs, rates)


def test_manufactured_poisson_error_is_small_at_p4():
    m, d = make(4, 4)
    u = spla.spsolve(d.assemble(0.0, 1.0).tocsc(), poisson_rhs(m, d))
    assert d.l2_error(u, u_manufactured) < 2e-5


def test_ir_reaches_fp64_residual():
    m, d = make(3, 4)
    nu = nu_uniform(m.nelem, d.q, seed=2)
    b = rhs_uniform(m, seed=1)[0]
    a64 = lambda v: d.apply(v, 1e3, 1.0, nu)
    a32 = lambda v: d.apply(v, 1e3, 1.0, nu, dtype=np.float32)
    diag = d.diagonal(1e3, 1.0, nu)
    x, outer, inner, rel = ir_pcg(a64, a32, (1.0 / diag).astype(np.float32), b, rtol=1e-12, inner_rtol=1e-5)
    assert rel <= 1e-12 and 1 <= outer <= 6
    x64, _, _ = pcg(a64, b, 1.0 / diag, rtol=1e-12)
    assert np.linalg.norm(x - x64) <= 1e-10 * np.linalg.norm(x64)
    # the float32 operator alone is accurate only to single precision
    y64, y32 = a64(b), a32(b)
    err32 = np.linalg.norm(y32 - y64) / np.linalg.norm(y64)
    assert 1e-9 < err32 < 1e-5


@pytest.mark.parametrize("alpha", [1e3, 0.0])
def test_adjoint_gradient_vs_finite_differences(alpha):
    m, d = make(2, 2)
    beta = 1.0
    nu = nu_uniform(m.nelem, d.q, seed=2)
    nu_star = nu_uniform(m.nelem, d.q, seed=3)
    b = rhs_uniform(m, seed=1)[0]
    u_t = spla.spsolve(d.assemble(alpha, beta, nu_star).tocsc(), b)
    J, g, u, lam = adjoint_gradient(d, nu, b, u_t, alpha, beta, direct=True)
    eps = 1e-6
    for k in range(4):
        dirn = np.random.default_rng(100 + k).uniform(-1, 1, nu.shape)
        jp = objective(d, nu + eps * dirn, b, u_t, alpha, beta, direct=True)
        jm = objective(d, nu - eps * dirn, b, u_t, alpha, beta, direct=True)
        fd = (jp - jm) / (2 * eps)
        ad = float(np.sum(g * dirn))
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


def test_adjoint_gradient_homogeneity_identity():
    m, d = make(3, 3)
    alpha, beta = 1e3, 0.7
    nu = nu_uniform(m.nelem, d.q, seed=2)
    b = rhs_uniform(m, seed=1)[0]
    u_t = spla.spsolve(d.assemble(alpha, beta, nu_uniform(m.nelem, d.q, seed=3)).tocsc(), b)
    J, g, u, lam = adjoint_gradient(d, nu, b, u_t, alpha, beta, direct=True)
    lhs = float(np.sum(nu * g))
    uf, lf = u.copy(), lam.copy()
    uf[m.ess.astype(bool)] = 0
    lf[m.ess.astype(bool)] = 0
    rhs = -beta * float(lf @ d.apply_unconstrained(uf, 0.0, 1.0, nu))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_planted_gradient_sign_and_scale_fail():
    m, d = make(2, 2)
    nu = nu_uniform(m.nelem, d.q, seed=2)
    b = rhs_uniform(m, seed=1)[0]
    u_t = spla.spsolve(d.assemble(1e3, 1.0, nu_uniform(m.nelem, d.q, seed=3)).tocsc(), b)
    J, g, u, lam = adjoint_gradient(d, nu, b, u_t, 1e3, 1.0, direct=True)
    dirn = np.random.default_rng(100).uniform(-1, 1, nu.shape)
    eps = 1e-6
    fd = (objective(d, nu + eps * dirn, b, u_t, 1e3, 1.0, direct=True)
          - objective(d, nu - eps * dirn, b, u_t, 1e3, 1.0, direct=True)) / (2 * eps)
    for wrong in (-g, 2.0 * g, d.grad_nu(u, u, 1.0)):
        ad = float(np.sum(wrong * dirn))
        assert abs(fd - ad) > 1e-3 * abs(fd)
