"""Oracle finite-element operators on mapped Q_p hexahedra (test infrastructure; FP64).

Everything here is the plain definition of the operators of Section 3 and 3.1,
evaluated with dense tensors; there is deliberately no sum factorization, no
per-direction staging and no stored geometric-factor layout.

Definitions followed:

* Basis: phi_ijk(xi) = phi_i(xi_1) phi_j(xi_2) phi_k(xi_3), Lagrange on the p+1
  GLL points (Section 3, Section 3.1).  Local index l = i + n (j + n k).
* Quadrature: tensor Gauss-Legendre with q points per direction; point index
  Q = a + q (b + q c), weight w_a w_b w_c (Section 3.1, eq. localStiffnessQuadrature).
* Geometry: trilinear map through the 8 element vertices, J = dx/dxi.  With this J
  the physical gradient is J^{-T} grad_ref, so the stored factor of Section 3.1 reads
  w |J| J^{-1} J^{-T} (see the reading of the transpose in the design notes).
* Element operator (eq. vectorMass, eq. vectorDiffusion, eq. localStiffnessMapped,
  scalar form), for the Helmholtz combination A = alpha M + beta K(nu) of Section 5.2
  and eq. proj-helmholtz:

      A_e[l, m] = sum_Q w_Q |J_Q| ( alpha phi_l phi_m
                                    + beta nu_Q (J_Q^{-T} grad phi_l) . (J_Q^{-T} grad phi_m) )

  assembled by summing element contributions (Section 3.1), then constrained for
  homogeneous Dirichlet DoFs: A_c = P A P + (I - P), P zeroing essential DoFs.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .quadrature import gauss_legendre, gll, lagrange_values, lagrange_derivs

OP_MASS, OP_DIFFUSION, OP_HELMHOLTZ = 0, 1, 2


def op_coeffs(op: int, alpha: float, beta: float):
    """(alpha, beta) actually used by an operator kind."""
    if op == OP_MASS:
        return 1.0, 0.0
    if op == OP_DIFFUSION:
        return 0.0, 1.0
    return alpha, beta


def trilinear_shape(xi):
    """N[Q, v] and dN[Q, v, d] of the 8 trilinear vertex functions at points xi [Q, 3]."""
    xi = np.asarray(xi, dtype=np.float64)
    nQ = xi.shape[0]
    N = np.ones((nQ, 8))
    dN = np.ones((nQ, 8, 3))
    for v in range(8):
        s = [2 * ((v >> d) & 1) - 1 for d in range(3)]
        f = [(1.0 + s[d] * xi[:, d]) / 2.0 for d in range(3)]
        N[:, v] = f[0] * f[1] * f[2]
        for d in range(3):
            prod = np.full(nQ, s[d] / 2.0)
            for d2 in range(3):
                if d2 != d:
                    prod = prod * f[d2]
            dN[:, v, d] = prod
    return N, dN


class Discretization:
    """Dense-tensor evaluation of the Q_p operators on a given hex mesh.

    elem_xyz [NE, 8, 3], elem_dofs [NE, (p+1)^3], ess [N] (0/1), ndof = N,
    p = order, q = Gauss points per direction.
    """

    def __init__(self, elem_xyz, elem_dofs, ess, ndof, p, q, chunk=None):
        self.elem_xyz = np.asarray(elem_xyz, dtype=np.float64)
        self.elem_dofs = np.asarray(elem_dofs, dtype=np.int64)
        self.ess = np.asarray(ess).astype(bool)
        self.ndof = int(ndof)
        self.p, self.q = int(p), int(q)
        self.n = self.p + 1
        self.nelem = self.elem_xyz.shape[0]
        self.nloc = self.n ** 3
        self.nqp = self.q ** 3
        xi, w = gauss_legendre(self.q)
        nodes, _ = gll(self.p)
        self.xi1, self.w1, self.nodes1 = xi, w, nodes
        Bv = lagrange_values(nodes, xi)  # [q, n]
        Dv = lagrange_derivs(nodes, xi)
        self.B1, self.D1 = Bv, Dv
        # dense 3D basis at the quadrature points
        self.Phi = np.einsum("ck,bj,ai->cbakji", Bv, Bv, Bv).reshape(self.nqp, self.nloc)
        g0 = np.einsum("ck,bj,ai->cbakji", Bv, Bv, Dv).reshape(self.nqp, self.nloc)
        g1 = np.einsum("ck,bj,ai->cbakji", Bv, Dv, Bv).reshape(self.nqp, self.nloc)
        g2 = np.einsum("ck,bj,ai->cbakji", Dv, Bv, Bv).reshape(self.nqp, self.nloc)
        self.dPhi = np.stack([g0, g1, g2], axis=-1)  # [Q, l, d]
        W = np.einsum("c,b,a->cba", w, w, w).reshape(-1)
        self.Wq = W
        XI = np.stack(np.meshgrid(xi, xi, xi, indexing="ij"), axis=-1)  # [a, b, c, 3]
        XI = XI.transpose(2, 1, 0, 3).reshape(-1, 3)  # Q = a + q(b + q c)
        self.XIq = XI
        self.Ntri, self.dNtri = trilinear_shape(XI)
        if chunk is None:
            # keep the dense per-chunk gradient tensors around ~64 MB
            per = self.nqp * self.nloc * 3 * 8
            chunk = max(1, int(64e6 // per))
        self.chunk = chunk
        # geometry-only loops (J, det, coordinates: ~15 values per point)
        self.gchunk = max(1, int(64e6 // (self.nqp * 15 * 8)))

    # ---------------- geometry ----------------
    def geometry(self, e0, e1):
        """detJ [C, Q], invJ [C, Q, 3, 3] (invJ[..., d, r] = (J^{-1})_{d r}), xq [C, Q, 3]."""
        X = self.elem_xyz[e0:e1]  # [C, 8, 3]
        J = np.einsum("cvr,Qvd->cQrd", X, self.dNtri)
        det = np.linalg.det(J)
        inv = np.linalg.inv(J)
        xq = np.einsum("cvr,Qv->cQr", X, self.Ntri)
        return det, inv, xq

    def qpoint_coords(self):
        """Physical quadrature points x(xi_Q) of the trilinear map: [NE, Q, 3]."""
        out = np.empty((self.nelem, self.nqp, 3))
        for e0 in range(0, self.nelem, self.gchunk):
            e1 = min(self.nelem, e0 + self.gchunk)
            out[e0:e1] = np.einsum("cvr,Qv->cQr", self.elem_xyz[e0:e1], self.Ntri)
        return out

    def min_detJ(self):
        m = np.inf
        for e0 in range(0, self.nelem, self.gchunk):
            e1 = min(self.nelem, e0 + self.gchunk)
            det, _, _ = self.geometry(e0, e1)
            m = min(m, det.min())
        return m

    def _nu_chunk(self, nu, e0, e1):
        if nu is None:
            return np.ones((e1 - e0, self.nqp))
        nu = np.asarray(nu, dtype=np.float64).reshape(self.nelem, self.nqp)
        return nu[e0:e1]

    def phys_grad_basis(self, inv):
        """grad phi_l at every point, physical: [C, Q, l, r] = sum_d (J^{-1})_{d r} dPhi[Q, l, d]."""
        return np.einsum("cQdr,Qld->cQlr", inv, self.dPhi)

    # ---------------- element matrices ----------------
    def element_matrices(self, alpha, beta, nu=None, e0=0, e1=None):
        """Dense A_e for elements e0..e1-1: [C, n^3, n^3]."""
        e1 = self.nelem if e1 is None else e1
        det, inv, _ = self.geometry(e0, e1)
        nuc = self._nu_chunk(nu, e0, e1)
        wd = self.Wq[None, :] * det  # [C, Q]
        A = alpha * np.einsum("cQ,Ql,Qm->clm", wd, self.Phi, self.Phi)
        if beta != 0.0:
            gp = self.phys_grad_basis(inv)  # [C, Q, l, r]
            A = A + beta * np.einsum("cQ,cQlr,cQmr->clm", wd * nuc, gp, gp)
        return A

    # ---------------- apply (on the fly, same sums as A_e x_e) ----------------
    def apply_unconstrained(self, x, alpha, beta, nu=None, dtype=np.float64):
        """y = sum_e P_e^T A_e P_e x for the unconstrained operator (x: [N] or [nb, N])."""
        x = np.asarray(x)
        squeeze = x.ndim == 1
        X = np.atleast_2d(x).astype(dtype)
        y = np.zeros(X.shape, dtype=dtype)
        Phi = self.Phi.astype(dtype)
        dPhi = self.dPhi.astype(dtype)
        Wq = self.Wq.astype(dtype)
        for e0 in range(0, self.nelem, self.chunk):
            e1 = min(self.nelem, e0 + self.chunk)
            det, inv, _ = self.geometry(e0, e1)
            det, inv = det.astype(dtype), inv.astype(dtype)
            nuc = self._nu_chunk(nu, e0, e1).astype(dtype)
            dofs = self.elem_dofs[e0:e1]
            wd = Wq[None, :] * det
            for b in range(X.shape[0]):
                xe = X[b][dofs]  # [C, l]
                ye = np.zeros_like(xe)
                if alpha != 0.0:
                    u = xe @ Phi.T  # [C, Q]
                    ye += (dtype(alpha) * wd * u) @ Phi
                if beta != 0.0:
                    gref = np.einsum("Qld,cl->cQd", dPhi, xe)
                    # physical gradient g_r = sum_d (J^{-1})_{d r} gref_d
                    gph = np.einsum("cQdr,cQd->cQr", inv, gref)
                    flux = (dtype(beta) * wd * nuc)[..., None] * gph
                    # back to the reference gradient of the test function
                    fref = np.einsum("cQdr,cQr->cQd", inv, flux)
                    ye += np.einsum("Qld,cQd->cl", dPhi, fref)
                np.add.at(y[b], dofs.reshape(-1), ye.reshape(-1))
        return y[0] if squeeze else y

    def apply(self, x, alpha, beta, nu=None, dtype=np.float64):
        """Constrained operator y = P A P x + (I - P) x."""
        x = np.asarray(x)
        xf = np.array(x, dtype=dtype, copy=True)
        xf[..., self.ess] = 0
        y = self.apply_unconstrained(xf, alpha, beta, nu, dtype=dtype)
        y[..., self.ess] = x[..., self.ess]
        return y

    def element_row(self, e, l, alpha, beta, nu=None):
        """Row l of A_e: sum_Q w|J| (alpha phi_l phi_m + beta nu grad phi_l . grad phi_m) over m."""
        det, inv, _ = self.geometry(e, e + 1)
        nuc = self._nu_chunk(nu, e, e + 1)[0]
        wd = self.Wq * det[0]
        row = alpha * (wd * self.Phi[:, l]) @ self.Phi
        if beta != 0.0:
            gp = np.einsum("Qdr,Qmd->Qmr", inv[0], self.dPhi)  # physical gradients [Q, m, r]
            row = row + beta * np.einsum("Q,Qr,Qmr->m", wd * nuc, gp[:, l, :], gp)
        return row

    def apply_rows(self, rows, x, alpha, beta, nu=None):
        """(A_c x)[rows] for a few rows, summing the element rows that contain each DoF."""
        rows = np.asarray(rows, dtype=np.int64)
        x = np.asarray(x, dtype=np.float64)
        xf = x.copy()
        xf[self.ess] = 0.0
        flat = self.elem_dofs.reshape(-1)
        order = np.argsort(flat, kind="stable")
        sflat = flat[order]
        out = np.zeros(rows.size)
        for t, g in enumerate(rows):
            if self.ess[g]:
                out[t] = x[g]
                continue
            lo, hi = np.searchsorted(sflat, [g, g + 1])
            for pos in order[lo:hi]:
                e, l = divmod(int(pos), self.nloc)
                out[t] += self.element_row(e, l, alpha, beta, nu) @ xf[self.elem_dofs[e]]
        return out

    # ---------------- diagonal ----------------
    def diagonal(self, alpha, beta, nu=None):
        """diag(A_c): sum over elements of the element-matrix diagonals, 1 on essential DoFs."""
        d = np.zeros(self.ndof)
        for e0 in range(0, self.nelem, self.chunk):
            e1 = min(self.nelem, e0 + self.chunk)
            det, inv, _ = self.geometry(e0, e1)
            nuc = self._nu_chunk(nu, e0, e1)
            wd = self.Wq[None, :] * det
            de = alpha * np.einsum("cQ,Ql->cl", wd, self.Phi ** 2)
            if beta != 0.0:
                gp = self.phys_grad_basis(inv)
                de = de + beta * np.einsum("cQ,cQl->cl", wd * nuc, (gp ** 2).sum(-1))
            np.add.at(d, self.elem_dofs[e0:e1].reshape(-1), de.reshape(-1))
        d[self.ess] = 1.0
        return d

    # ---------------- assembled sparse matrix (small cases) ----------------
    def collocated_mass_diagonal(self, constrained=True):
        """Mass matrix integrated with the GLL rule at the nodes themselves (Section 5.1):
        phi_l(xi_m) = delta_lm makes it diagonal, entry g = sum over the elements and their
        local nodes l -> g of w_l |J_e(xi_l)| (w_l the tensor GLL weight).  Essential rows
        are 1 when constrained (the preconditioner of the constrained operator)."""
        nodes, wg = gll(self.p)
        n = self.n
        l = np.arange(self.nloc)
        i, j, k = l % n, (l // n) % n, l // (n * n)
        XI = np.stack([nodes[i], nodes[j], nodes[k]], axis=-1)
        W = wg[i] * wg[j] * wg[k]
        _, dN = trilinear_shape(XI)
        out = np.zeros(self.ndof)
        for e0 in range(0, self.nelem, self.gchunk):
            e1 = min(self.nelem, e0 + self.gchunk)
            J = np.einsum("cvr,lvd->clrd", self.elem_xyz[e0:e1], dN)
            np.add.at(out, self.elem_dofs[e0:e1], W[None, :] * np.linalg.det(J))
        if constrained:
            out[self.ess] = 1.0
        return out

    def assemble(self, alpha, beta, nu=None, constrained=True):
        rows, cols, vals = [], [], []
        for e0 in range(0, self.nelem, self.chunk):
            e1 = min(self.nelem, e0 + self.chunk)
            A = self.element_matrices(alpha, beta, nu, e0, e1)
            dofs = self.elem_dofs[e0:e1]
            rows.append(np.repeat(dofs, self.nloc, axis=1).reshape(-1))
            cols.append(np.tile(dofs, (1, self.nloc)).reshape(-1))
            vals.append(A.reshape(-1))
        M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.ndof, self.ndof)).tocsr()
        if constrained:
            free = sp.diags((~self.ess).astype(np.float64))
            M = (free @ M @ free + sp.diags(self.ess.astype(np.float64))).tocsr()
        return M

    # ---------------- load vector ----------------
    def load(self, f_q):
        """b_l = sum_e sum_Q w |J| f_Q phi_l(Q), essential entries set to 0.  f_q: [NE, Q] or [nb, NE, Q]."""
        f = np.asarray(f_q, dtype=np.float64)
        squeeze = f.ndim == 2
        f = f.reshape(-1, self.nelem, self.nqp)
        b = np.zeros((f.shape[0], self.ndof))
        for e0 in range(0, self.nelem, self.chunk):
            e1 = min(self.nelem, e0 + self.chunk)
            det, _, _ = self.geometry(e0, e1)
            wd = self.Wq[None, :] * det
            dofs = self.elem_dofs[e0:e1].reshape(-1)
            for k in range(f.shape[0]):
                be = (wd * f[k, e0:e1]) @ self.Phi
                np.add.at(b[k], dofs, be.reshape(-1))
        b[:, self.ess] = 0.0
        return b[0] if squeeze else b

    # ---------------- adjoint gradient integrand ----------------
    def grad_nu(self, u, lam, beta):
        """dJ/dnu_{e,Q} = -beta w_Q |J_Q| (J^{-T} grad lam) . (J^{-T} grad u): [NE, Q]."""
        u = np.asarray(u, dtype=np.float64)
        lam = np.asarray(lam, dtype=np.float64)
        g = np.empty((self.nelem, self.nqp))
        for e0 in range(0, self.nelem, self.chunk):
            e1 = min(self.nelem, e0 + self.chunk)
            det, inv, _ = self.geometry(e0, e1)
            dofs = self.elem_dofs[e0:e1]
            gu = np.einsum("cQdr,Qld,cl->cQr", inv, self.dPhi, u[dofs])
            gl = np.einsum("cQdr,Qld,cl->cQr", inv, self.dPhi, lam[dofs])
            g[e0:e1] = -beta * self.Wq[None, :] * det * (gu * gl).sum(-1)
        return g

    # ---------------- error norms ----------------
    def l2_error(self, u, exact, q_err=None):
        """|| u_h - exact ||_{L2(Omega)} with a (q_err)^3 Gauss rule (default p + 4)."""
        q_err = self.p + 4 if q_err is None else q_err
        d = Discretization(self.elem_xyz, self.elem_dofs, self.ess, self.ndof, self.p, q_err)
        u = np.asarray(u, dtype=np.float64)
        s = 0.0
        for e0 in range(0, d.nelem, d.chunk):
            e1 = min(d.nelem, e0 + d.chunk)
            det, _, xq = d.geometry(e0, e1)
            uh = u[d.elem_dofs[e0:e1]] @ d.Phi.T
            ex = exact(xq[..., 0], xq[..., 1], xq[..., 2])
            s += np.sum(d.Wq[None, :] * det * (uh - ex) ** 2)
        return np.sqrt(s)
