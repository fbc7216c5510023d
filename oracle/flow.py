"""Oracle of the velocity-correction projection step (test infrastructure; FP64).

Section 4.2 (projection methods) with equal-order velocity and pressure: every
velocity component and the pressure live in the same continuous Q_p space V_h with the
GLL nodal basis phi_i, on the scalar discretization d (tensor Gauss rule, q points).
The weak vector operators are the plain definitions, evaluated with dense tensors at
the Gauss points (no sum factorization):

    weak_gradient(s)_{c,i}  = sum_e sum_Q w|J| phi_i (grad s)_c
    weak_curl(u)_{c,i}      = sum_e sum_Q w|J| phi_i (curl u)_c
    weak_divergence(V)_i    = sum_e sum_Q w|J| grad phi_i . V

(grad = J^{-T} grad_ref; V and u nodal vector fields [3][N], interpolated at the points).
None of them is constrained: every row is computed.

One step of order k (BDF-k for the implicit terms, EXT-k for the explicit ones;
eq. projKnown, eq. projLinear, eq. pres-poisson, eq. presPoissonBC, eq. meanZero,
eq. proj-helmholtz), for no-slip walls (u = 0 on the whole boundary, the essential
DoFs of d) and a constant viscosity nu:

  1. N^n = -B^{-1} C(u^n): the convection term (eq. nonlinear, rows of boundary DoFs 0,
     oracle.stokes.convection) made nodal with the collocated GLL mass B (Section 5.1);
  2. F* = -sum_{j=1..k} (b_j / dt) u^{n+1-j} + sum_j a_j N^{n+1-j} + f^{n+1}   (nodal);
  3. the rotational term: u* = sum_j a_j u^{n+1-j}, w = B^{-1} weak_curl(u*),
     L* = -nu B^{-1} weak_curl(w)  (nodal curl curl u*);
  4. pressure Poisson: K p = weak_divergence(F* + L*), the Neumann condition of
     eq. presPoissonBC being the natural one of this weak form (u . n = 0 on the walls),
     closed by int p = 0;
  5. Helmholtz: (b_0 / dt) M u + nu K u = M F* - weak_gradient(p) on the free rows,
     u = 0 on the walls.

Returns u^{n+1} and p^{n+1}; the history shifts.  The solves are sparse direct.

Pins (tests/test_oracle_flow.py): the weak operators, the BDF/EXT weights, one step in
hydrostatic balance, the time integration through self-convergence in the step size on
a 4^3, p = 4 mesh (order 1 and order 2 rates; on coarser meshes the run-to-run
differences stall at the mesh's equal-order consistency error), and a manufactured
Navier-Stokes solution with no-slip walls whose velocity and pressure errors fall at
the scheme's order in the step size, while a flipped or unscaled rotational term L*
or a flipped convection term N* leaves the errors large (each term is its own method,
convection_term and rotational_term, so that a test can replace it).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Discretization
from .stokes import convection


def _interp(d, e0, e1, v):
    """Nodal fields v [m][N] at the points: values [C, Q, m] and reference gradients
    [C, Q, m, 3]."""
    dofs = d.elem_dofs[e0:e1]
    ve = np.stack([vc[dofs] for vc in v], axis=1)  # [C, m, l]
    val = np.einsum("Ql,eml->eQm", d.Phi, ve)
    gref = np.einsum("Qld,eml->eQmd", d.dPhi, ve)
    return val, gref


def _phys(inv, gref):
    """(J^{-T} grad_ref v_m)_r = sum_k (J^{-1})_{k r} grad_ref_k: [C, Q, m, r]."""
    return np.einsum("eQkr,eQmk->eQmr", inv, gref)


def weak_gradient(d: Discretization, s):
    s = np.asarray(s, dtype=np.float64).reshape(1, d.ndof)
    y = np.zeros((3, d.ndof))
    for e0 in range(0, d.nelem, d.chunk):
        e1 = min(d.nelem, e0 + d.chunk)
        det, inv, _ = d.geometry(e0, e1)
        _, gref = _interp(d, e0, e1, s)
        g = _phys(inv, gref)[:, :, 0, :]  # [C, Q, r]
        ye = np.einsum("eQ,Ql,eQc->ecl", d.Wq[None, :] * det, d.Phi, g)
        for c in range(3):
            np.add.at(y[c], d.elem_dofs[e0:e1].reshape(-1), ye[:, c].reshape(-1))
    return y


def curl_of(g):
    """curl from the physical gradient tensor g[..., m, r] = d u_m / d x_r."""
    return np.stack([g[..., 2, 1] - g[..., 1, 2],
                     g[..., 0, 2] - g[..., 2, 0],
                     g[..., 1, 0] - g[..., 0, 1]], axis=-1)


def weak_curl(d: Discretization, u):
    u = np.asarray(u, dtype=np.float64).reshape(3, d.ndof)
    y = np.zeros((3, d.ndof))
    for e0 in range(0, d.nelem, d.chunk):
        e1 = min(d.nelem, e0 + d.chunk)
        det, inv, _ = d.geometry(e0, e1)
        _, gref = _interp(d, e0, e1, u)
        cu = curl_of(_phys(inv, gref))  # [C, Q, 3]
        ye = np.einsum("eQ,Ql,eQc->ecl", d.Wq[None, :] * det, d.Phi, cu)
        for c in range(3):
            np.add.at(y[c], d.elem_dofs[e0:e1].reshape(-1), ye[:, c].reshape(-1))
    return y


def weak_divergence(d: Discretization, v):
    v = np.asarray(v, dtype=np.float64).reshape(3, d.ndof)
    y = np.zeros(d.ndof)
    for e0 in range(0, d.nelem, d.chunk):
        e1 = min(d.nelem, e0 + d.chunk)
        det, inv, _ = d.geometry(e0, e1)
        val, _ = _interp(d, e0, e1, v)  # [C, Q, 3]
        gphi = d.phys_grad_basis(inv)  # [C, Q, l, r]
        ye = np.einsum("eQ,eQlr,eQr->el", d.Wq[None, :] * det, gphi, val)
        np.add.at(y, d.elem_dofs[e0:e1].reshape(-1), ye.reshape(-1))
    return y


def bdf_ext(k: int):
    """BDF-k coefficients b_0..b_k (sum_j b_j u^{n+1-j} / dt ~ du/dt at t_{n+1}) and EXT-k
    coefficients a_1..a_k (sum_j a_j u^{n+1-j} ~ u(t_{n+1})), k = 1, 2, 3, for a constant
    step: the unique ones exact for polynomials in t of degree k (BDF) and k - 1 (EXT)."""
    if k == 1:
        return np.array([1.0, -1.0]), np.array([1.0])
    if k == 2:
        return np.array([1.5, -2.0, 0.5]), np.array([2.0, -1.0])
    if k == 3:
        return np.array([11.0 / 6.0, -3.0, 1.5, -1.0 / 3.0]), np.array([3.0, -3.0, 1.0])
    raise ValueError("k = 1, 2 or 3")


class ProjectionStepper:
    """Velocity-correction projection steps on d (essential DoFs = the no-slip walls)."""

    def __init__(self, d: Discretization, dt: float, nu: float, order: int = 3):
        self.d = d
        self.free = Discretization(d.elem_xyz, d.elem_dofs, np.zeros(d.ndof, dtype=bool), d.ndof,
                                   d.p, d.q)
        self.dt, self.nu, self.order = float(dt), float(nu), int(order)
        self.binv = 1.0 / self.free.collocated_mass_diagonal(constrained=False)
        self.M = self.free.assemble(1.0, 0.0, constrained=False)
        K = self.free.assemble(0.0, 1.0, constrained=False)
        m1 = np.asarray(self.M @ np.ones(d.ndof)).reshape(-1, 1)
        # [K m1; m1^T 0]: K p = r with int p = m1^T p = 0 (r is orthogonal to 1)
        self.Kb = spla.splu(sp.bmat([[K, sp.csr_matrix(m1)], [sp.csr_matrix(m1.T), None]]).tocsc())
        self.m1 = m1.reshape(-1)
        self.hlu = {}  # factorized Helmholtz matrix per b_0 / dt
        self.us, self.ns = [], []  # newest first
        self.nstep = 0

    def convection_term(self, u):
        """N = -B^{-1} C(u) (nodal): the explicit convection term of the step."""
        return -self.binv * convection(self.d, u)

    def rotational_term(self, ustar):
        """L* = -nu B^{-1} curl_w(B^{-1} curl_w u*) (nodal -nu curl curl u*, eq. projLinear)."""
        w = self.binv * weak_curl(self.free, ustar)
        return -self.nu * self.binv * weak_curl(self.free, w)

    def step(self, u, f=None):
        """Advance from u = u^n [3][N] (walls 0); f = f^{n+1} [3][N] nodal or None.
        Returns (u^{n+1}, p^{n+1})."""
        d, dt, nu = self.d, self.dt, self.nu
        u = np.asarray(u, dtype=np.float64).reshape(3, d.ndof)
        k = min(self.nstep + 1, self.order)
        b, a = bdf_ext(k)
        self.us.insert(0, u)
        self.ns.insert(0, self.convection_term(u))
        del self.us[k:], self.ns[k:]
        F = sum(a[j] * self.ns[j] - (b[j + 1] / dt) * self.us[j] for j in range(k))
        if f is not None:
            F = F + np.asarray(f, dtype=np.float64).reshape(3, d.ndof)
        ustar = sum(a[j] * self.us[j] for j in range(k))
        L = self.rotational_term(ustar)
        r = weak_divergence(self.free, F + L)
        p = self.Kb.solve(np.concatenate([r - r.mean(), [0.0]]))[:-1]
        R = np.stack([self.M @ F[c] for c in range(3)]) - weak_gradient(self.free, p)
        R[:, d.ess] = 0.0
        alpha = b[0] / dt
        if alpha not in self.hlu:
            self.hlu[alpha] = spla.splu(d.assemble(alpha, nu, constrained=True).tocsc())
        lu = self.hlu[alpha]
        un = np.stack([lu.solve(R[c]) for c in range(3)])
        self.nstep += 1
        return un, p
