"""Oracle of the Stokes block operator (test infrastructure; FP64).

The Taylor-Hood pair of Section 3: velocity in (V_p)^3, pressure in P_{p-1}, both
continuous with nodal tensor-product bases on the GLL points, on the same mapped
hexahedra.  The coupling blocks are the definitions eq. gradient and eq. divergence,
evaluated with dense tensors at the tensor Gauss points (q per direction); there is
no sum factorization:

    G_e[c, l, m] = sum_Q w_Q |J_Q| phi_l(Q) (J_Q^{-T} grad_ref psi_m(Q))_c
    D_e[m, c, l] = sum_Q w_Q |J_Q| psi_m(Q) (J_Q^{-T} grad_ref phi_l(Q))_c

(phi: velocity basis, component c of the vector basis phi_l e_c; psi: pressure basis.)
The block operator of one implicit stage of the unsteady Stokes problem (eq.
unsteadyStokesDiscrete, H = alpha M + beta L(nu) per velocity component) with the
velocity Dirichlet DoFs constrained as for the scalar operators (P zeroes them):

    y_u = P H P u + (I - P) u + P G p,     y_p = -D P u.

Velocity vectors are component-major, [3][nv], every component on the scalar map.

The explicit convection term of the Navier-Stokes problem (eq. nonlinear) on the
velocity space, component c:

    N(u)_{c, i} = sum_e sum_Q w_Q |J_Q| phi_i(Q) sum_d u_d(Q) (J_Q^{-T} grad_ref u_c(Q))_d

i.e. the integral of phi_i ((u . grad) u)_c, evaluated with the same dense tensors and
Gauss points (convection()).  The boundary values of u enter as they are; rows of
essential DoFs are set to 0 (the term is a right-hand side of the constrained solves).
"""
from __future__ import annotations

import numpy as np

from .fem import Discretization, trilinear_shape
from .quadrature import gll, lagrange_values, lagrange_derivs


class StokesDiscretization:
    """Dense evaluation of the Taylor-Hood Stokes blocks on a hex mesh.

    elem_xyz [NE, 8, 3]; vel_dofs [NE, (p+1)^3], vel_ess [nv]; pres_dofs [NE, p^3];
    p = velocity order (pressure order p - 1, p >= 2); q = Gauss points per direction.
    """

    def __init__(self, elem_xyz, vel_dofs, vel_ess, nv, pres_dofs, npres, p, q):
        if p < 2:
            raise ValueError("Taylor-Hood needs p >= 2")
        self.vel = Discretization(elem_xyz, vel_dofs, vel_ess, nv, p, q)
        self.p, self.q = int(p), int(q)
        self.nv, self.np_ = int(nv), int(npres)
        self.pres_dofs = np.asarray(pres_dofs, dtype=np.int64)
        self.nelem = self.vel.nelem
        self.npl = p ** 3  # pressure nodes per element
        pn, _ = gll(p - 1)
        Bp = lagrange_values(pn, self.vel.xi1)  # [q, p]
        Dp = lagrange_derivs(pn, self.vel.xi1)
        # dense pressure basis and reference gradient at the points Q = a + q (b + q c)
        self.Psi = np.einsum("ck,bj,ai->cbakji", Bp, Bp, Bp).reshape(self.vel.nqp, self.npl)
        g0 = np.einsum("ck,bj,ai->cbakji", Bp, Bp, Dp).reshape(self.vel.nqp, self.npl)
        g1 = np.einsum("ck,bj,ai->cbakji", Bp, Dp, Bp).reshape(self.vel.nqp, self.npl)
        g2 = np.einsum("ck,bj,ai->cbakji", Dp, Bp, Bp).reshape(self.vel.nqp, self.npl)
        self.dPsi = np.stack([g0, g1, g2], axis=-1)  # [Q, m, d]

    # ---------------- element blocks ----------------
    def element_blocks(self, e0, e1):
        """G_e [C, 3, nl_v, nl_p] and D_e [C, nl_p, 3, nl_v] for elements e0..e1-1."""
        det, inv, _ = self.vel.geometry(e0, e1)
        wd = self.vel.Wq[None, :] * det  # [C, Q]
        # physical gradients: (J^{-T} g)_c = sum_d (J^{-1})_{d c} g_d
        gpsi = np.einsum("cQdr,Qmd->cQmr", inv, self.dPsi)  # [C, Q, m, c]
        gphi = np.einsum("cQdr,Qld->cQlr", inv, self.vel.dPhi)  # [C, Q, l, c]
        G = np.einsum("eQ,Ql,eQmc->eclm", wd, self.vel.Phi, gpsi)
        D = np.einsum("eQ,Qm,eQlc->emcl", wd, self.Psi, gphi)
        return G, D

    # ---------------- unconstrained blocks ----------------
    def gradient(self, pres):
        """(G p) as [3, nv] (unconstrained)."""
        pres = np.asarray(pres, dtype=np.float64)
        y = np.zeros((3, self.nv))
        vd = self.vel.elem_dofs
        for e0 in range(0, self.nelem, self.vel.chunk):
            e1 = min(self.nelem, e0 + self.vel.chunk)
            G, _ = self.element_blocks(e0, e1)
            ye = np.einsum("eclm,em->ecl", G, pres[self.pres_dofs[e0:e1]])
            for c in range(3):
                np.add.at(y[c], vd[e0:e1].reshape(-1), ye[:, c].reshape(-1))
        return y

    def divergence(self, u):
        """(D u) as [np] (unconstrained); u [3, nv]."""
        u = np.asarray(u, dtype=np.float64).reshape(3, self.nv)
        y = np.zeros(self.np_)
        vd = self.vel.elem_dofs
        for e0 in range(0, self.nelem, self.vel.chunk):
            e1 = min(self.nelem, e0 + self.vel.chunk)
            _, D = self.element_blocks(e0, e1)
            ue = np.stack([u[c][vd[e0:e1]] for c in range(3)], axis=1)  # [C, 3, l]
            ye = np.einsum("emcl,ecl->em", D, ue)
            np.add.at(y, self.pres_dofs[e0:e1].reshape(-1), ye.reshape(-1))
        return y

    # ---------------- constrained block operator ----------------
    def apply(self, u, pres, alpha, beta, nu=None):
        """(y_u [3, nv], y_p [np]) of the constrained block operator."""
        u = np.asarray(u, dtype=np.float64).reshape(3, self.nv)
        ess = self.vel.ess
        uf = u.copy()
        uf[:, ess] = 0.0
        yu = np.stack([self.vel.apply(u[c], alpha, beta, nu) for c in range(3)])
        gp = self.gradient(pres)
        gp[:, ess] = 0.0
        yu = yu + gp
        yp = -self.divergence(uf)
        return yu, yp

    def pressure_mass_rowsums(self):
        """sum_m of the pressure mass matrix rows: int psi_m dx, [np]."""
        out = np.zeros(self.np_)
        for e0 in range(0, self.nelem, self.vel.chunk):
            e1 = min(self.nelem, e0 + self.vel.chunk)
            det, _, _ = self.vel.geometry(e0, e1)
            be = (self.vel.Wq[None, :] * det) @ self.Psi
            np.add.at(out, self.pres_dofs[e0:e1].reshape(-1), be.reshape(-1))
        return out

    def _node_coords(self, order, dofs, count):
        pn, _ = gll(order)
        n = order + 1
        m = np.arange(n ** 3)
        i, j, k = m % n, (m // n) % n, m // (n * n)
        XI = np.stack([pn[i], pn[j], pn[k]], axis=-1)
        N, _ = trilinear_shape(XI)
        out = np.zeros((count, 3))
        xe = np.einsum("evr,mv->emr", self.vel.elem_xyz, N)
        out[np.asarray(dofs).reshape(-1)] = xe.reshape(-1, 3)
        return out

    def pressure_node_coords(self):
        """Physical coordinates of the pressure nodes [np, 3] (trilinear map)."""
        return self._node_coords(self.p - 1, self.pres_dofs, self.np_)

    def velocity_node_coords(self):
        """Physical coordinates of the velocity nodes [nv, 3] (trilinear map)."""
        return self._node_coords(self.p, self.vel.elem_dofs, self.nv)


def convection(d: Discretization, u):
    """N(u) [3, N] on the scalar discretization d (see the module docstring)."""
    u = np.asarray(u, dtype=np.float64).reshape(3, d.ndof)
    y = np.zeros((3, d.ndof))
    for e0 in range(0, d.nelem, d.chunk):
        e1 = min(d.nelem, e0 + d.chunk)
        det, inv, _ = d.geometry(e0, e1)
        wd = d.Wq[None, :] * det  # [C, Q]
        dofs = d.elem_dofs[e0:e1]
        ue = np.stack([u[c][dofs] for c in range(3)], axis=1)  # [C, 3, l]
        uq = np.einsum("Ql,ecl->eQc", d.Phi, ue)  # u at the points [C, Q, 3]
        gref = np.einsum("Qld,ecl->eQcd", d.dPhi, ue)  # grad_ref u_c [C, Q, c, d]
        gphys = np.einsum("eQkr,eQck->eQcr", inv, gref)  # (J^{-T} grad_ref u_c)_r
        adv = np.einsum("eQr,eQcr->eQc", uq, gphys)  # ((u . grad) u)_c
        ye = np.einsum("eQ,Ql,eQc->ecl", wd, d.Phi, adv)
        for c in range(3):
            np.add.at(y[c], dofs.reshape(-1), ye[:, c].reshape(-1))
    y[:, d.ess] = 0.0
    return y
