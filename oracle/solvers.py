"""Oracle iterative solvers (test infrastructure).

* Jacobi-preconditioned conjugate gradients (the Krylov solver of Section 5 for
  the SPD mass / Poisson / Helmholtz sub-problems of Section 5.3), with the
  preconditioner taken as the exact diagonal of the constrained operator.
  Stopping test on the recursive residual, ||r||_2 <= rtol ||b||_2, x0 = 0 by
  default (the relative-residual convention of Section 7.1).
* Mixed-precision iterative refinement: residual in FP64, correction from an
  FP32 Jacobi-PCG (vectors and operator in float32, dot products accumulated in
  float64), x += ||r|| d in FP64; the inner tolerance is inner_rtol, or half the
  reduction still needed once one FP32 solve can reach it.
* Adjoint gradient of J(nu) = 0.5 ||u(nu) - u_t||^2 with A(nu) u = b:
  lambda solves A lambda = u - u_t (A is symmetric), and
  dJ/dnu_{e,Q} = -lambda^T (dA/dnu_{e,Q}) u, the pointwise integrand of
  Discretization.grad_nu.  K is linear in nu through the quadrature-point factor of
  Section 3.1, which gives that derivative.
"""
from __future__ import annotations

import numpy as np


def pcg(apply, b, dinv, rtol=1e-10, maxit=10000, x0=None, dtype=np.float64, dot_dtype=np.float64,
        nullspace=False, precond=None):
    """Diagonally preconditioned CG.  Returns (x, iters, rel_res_recursive).  ``apply`` maps
    a vector to A v, ``dinv`` is the inverse of the diagonal preconditioner; ``precond``
    (a callable r -> z), if given, replaces the diagonal (e.g. a solve with the LOR
    operator of Section 5.2).

    nullspace=True: the operator has the constant vectors as null space (pure Neumann
    Poisson, Section 5.3); every application of the preconditioner is followed by the
    orthogonalization z <- z - mean(z) 1 against that null space."""
    b = np.asarray(b, dtype=dtype)
    dinv = np.asarray(dinv, dtype=dtype)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=dtype, copy=True)

    def dot(u, v):
        return float(np.dot(u.astype(dot_dtype), v.astype(dot_dtype)))

    bnorm = np.sqrt(dot(b, b))
    if bnorm == 0.0:
        return np.zeros_like(b), 0, 0.0
    r = b - apply(x) if x0 is not None else b.copy()

    user = precond

    def precond(v):
        z = (dinv * v).astype(dtype) if user is None else np.asarray(user(v), dtype=dtype)
        if nullspace:
            z = (z - dtype(np.mean(z.astype(dot_dtype)))).astype(dtype)
        return z

    z = precond(r)
    p = z.copy()
    rho = dot(r, z)
    rr = dot(r, r)
    it = 0
    while np.sqrt(rr) > rtol * bnorm and it < maxit:
        w = apply(p)
        pw = dot(p, w)
        if not pw > 0.0:
            raise FloatingPointError("CG breakdown: p^T A p <= 0")
        alpha = rho / pw
        x = (x + dtype(alpha) * p).astype(dtype)
        r = (r - dtype(alpha) * w).astype(dtype)
        z = precond(r)
        rho_new = dot(r, z)
        rr = dot(r, r)
        beta = rho_new / rho
        rho = rho_new
        p = (z + dtype(beta) * p).astype(dtype)
        it += 1
    return x, it, np.sqrt(rr) / bnorm


def inner_tolerance(rtol, bnorm, rnorm, inner_rtol):
    """Relative tolerance of the next FP32 inner solve of the refinement.  A refinement
    step reduces the residual by the inner solve's tolerance (up to FP32 rounding), so
    a step normally asks for inner_rtol.  The reduction still needed to reach rtol is
    need = rtol ||b|| / ||r||; once one FP32 solve can deliver it (need >= inner_rtol / 10),
    the step asks for need / 2 and the refinement ends with it."""
    need = rtol * bnorm / rnorm if rnorm > 0 else 1.0
    return 0.5 * need if need >= 0.1 * inner_rtol else inner_rtol


def ir_pcg(apply64, apply32, dinv32, b, rtol=1e-10, inner_rtol=1e-5, max_outer=20, inner_maxit=10000):
    """FP64 iterative refinement around an FP32 Jacobi-PCG; each inner tolerance from
    inner_tolerance().

    Returns (x, outer_iters, total_inner_iters, true_rel_res).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0, 0.0
    inner_total = 0
    outer = 0
    r = b.copy()
    rnorm = bnorm
    while rnorm > rtol * bnorm and outer < max_outer:
        rs = (r / rnorm).astype(np.float32)
        itol = inner_tolerance(rtol, bnorm, rnorm, inner_rtol)
        d, it, _ = pcg(apply32, rs, dinv32, rtol=itol, maxit=inner_maxit,
                       dtype=np.float32, dot_dtype=np.float64)
        inner_total += it
        x = x + rnorm * d.astype(np.float64)
        r = b - apply64(x)
        rnorm = np.linalg.norm(r)
        outer += 1
    return x, outer, inner_total, rnorm / bnorm


def adjoint_gradient(disc, nu, b, u_target, alpha, beta, rtol=1e-12, direct=False):
    """J(nu) and dJ/dnu [NE, Q] for J = 0.5 ||u - u_t||^2, A(nu) u = b (constrained Helmholtz)."""
    if direct:
        import scipy.sparse.linalg as spla
        A = disc.assemble(alpha, beta, nu).tocsc()
        lu = spla.splu(A)
        solve = lu.solve
    else:
        dinv = 1.0 / disc.diagonal(alpha, beta, nu)

        def solve(rhs):
            return pcg(lambda v: disc.apply(v, alpha, beta, nu), rhs, dinv, rtol=rtol)[0]
    u = solve(b)
    res = u - u_target
    res[disc.ess] = 0.0
    J = 0.5 * float(res @ res)
    lam = solve(res)
    return J, disc.grad_nu(u, lam, beta), u, lam


def objective(disc, nu, b, u_target, alpha, beta, rtol=1e-13, direct=False):
    """J(nu) alone (for finite differences)."""
    if direct:
        import scipy.sparse.linalg as spla
        u = spla.spsolve(disc.assemble(alpha, beta, nu).tocsc(), b)
    else:
        dinv = 1.0 / disc.diagonal(alpha, beta, nu)
        u = pcg(lambda v: disc.apply(v, alpha, beta, nu), b, dinv, rtol=rtol)[0]
    res = u - u_target
    res[disc.ess] = 0.0
    return 0.5 * float(res @ res)


def neumann_poisson(d, b, nu=None, rtol=1e-10, dinv=None):
    """Pure-Neumann Poisson K(nu) x = b closed by the mean-zero condition int x = 0
    (Section 3, eq. meanZero; Section 5.3).  d: a Discretization without essential DoFs.

    The right-hand side is made orthogonal to the null space (b <- b - mean(b) 1, since
    K 1 = 0), the system is solved by CG with the Jacobi diagonal (or the given inverse
    diagonal) followed by the orthogonalization step, and the constant is fixed by
    int x = (M 1)^T x = 0.  Returns (x, iters, rel_res_recursive)."""
    if d.ess.any():
        raise ValueError("the pure Neumann problem has no essential DoFs")
    b = np.asarray(b, dtype=np.float64)
    b = b - b.mean()
    if dinv is None:
        dinv = 1.0 / d.diagonal(0.0, 1.0, nu)
    x, it, rr = pcg(lambda v: d.apply(v, 0.0, 1.0, nu), b, dinv, rtol=rtol, nullspace=True)
    m1 = d.apply(np.ones(d.ndof), 1.0, 0.0)
    x = x - np.dot(m1, x) / m1.sum()
    return x, it, rr
