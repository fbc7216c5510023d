"""Velocity-correction projection steps (Section 4.2) on the GPU, composed of library calls.

Equal-order velocity and pressure (every velocity component and the pressure in the
same continuous Q_p space, as in the paper's projection method), no-slip walls on the
essential DoFs of the mesh and a constant viscosity nu.  One step of order k (BDF-k for
the implicit terms, EXT-k for the explicit ones; k ramps up 1, 2, ... to `order` over the
first steps):

  1. N^n = -B^{-1} C(u^n): the convection term (eq. nonlinear; rows of wall DoFs 0) made
     nodal with the collocated GLL mass B (Section 5.1);
  2. F* = -sum_j (b_j / dt) u^{n+1-j} + sum_j a_j N^{n+1-j} + f^{n+1}   (eq. projKnown);
  3. the rotational term of eq. projLinear for the extrapolated velocity u*:
     w = B^{-1} curl_w(u*), L* = -nu B^{-1} curl_w(w);
  4. pressure Poisson (eq. pres-poisson with the Neumann condition eq. presPoissonBC,
     natural in the weak form since u . n = 0 on the walls, and eq. meanZero):
     K p = div_w(F* + L*), solved by the orthogonalized Jacobi-PCG (by default with FP32
     inner solves inside FP64 refinement), int p = 0;
  5. Helmholtz (eq. proj-helmholtz): (b_0 / dt) M u + nu K u = M F* - grad_w(p) on the
     free rows, u = 0 on the walls, solved by Jacobi-PCG for the three components at once.

The solves start from the previous step's pressure and from the extrapolated velocity u*.

Every arithmetic step runs in the library's kernels (convection, weak operators, nodal
combinations, applies, solves); this class only orders the calls and keeps the history.
The BDF and EXT weights are computed on the host from their exactness conditions.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (DIFFUSION, HELMHOLTZ, MASS, WEAK_CURL, WEAK_DIVERGENCE, WEAK_GRADIENT, Operator,
               SfemError)


def bdf_ext_weights(k: int):
    """(b_0..b_k, a_1..a_k) for a constant step: sum_j b_j g(t_{n+1-j}) = dt g'(t_{n+1}) for
    every polynomial g of degree <= k, and sum_j a_j g(t_{n+1-j}) = g(t_{n+1}) for degree
    <= k - 1 (t measured in steps from t_{n+1})."""
    if k not in (1, 2, 3):
        raise ValueError("order 1, 2 or 3")
    s = -np.arange(k + 1, dtype=np.float64)  # t_{n+1-j} - t_{n+1}
    Vb = np.vander(s, k + 1, increasing=True).T  # rows: degree m, columns: j
    rb = np.zeros(k + 1)
    rb[1] = 1.0  # d/dt t^m at 0: 1 for m = 1, else 0
    b = np.linalg.solve(Vb, rb)
    Va = np.vander(s[1:], k, increasing=True).T
    ra = np.zeros(k)
    ra[0] = 1.0  # t^m at 0: 1 for m = 0
    a = np.linalg.solve(Va, ra)
    return b, a


class ProjectionStepper:
    """Projection time stepping on one mesh: `vel` (essential DoFs = the walls) holds the
    Helmholtz solve and the convection term, `free` (no essential DoFs) the weak vector
    operators, the mass and the pure-Neumann pressure solve."""

    def __init__(self, elem_xyz, elem_dofs, ndof, p, ess, dt, nu, order=3, rtol=1e-10,
                 pressure_mode=1, device=None):
        self.vel = Operator(elem_xyz, elem_dofs, ndof, p, ess=ess, device=device)
        self.free = Operator(elem_xyz, elem_dofs, ndof, p, device=device)
        self.free.set_coeffs(1.0, 1.0, None)
        self.device = self.free.device
        self.ndof = int(ndof)
        self.dt, self.nu, self.order, self.rtol = float(dt), float(nu), int(order), float(rtol)
        self.pressure_mode = int(pressure_mode)  # 0: FP64 PCG, 1: FP32 inner PCG + FP64 refinement
        if not 1 <= self.order <= 3:
            raise ValueError("order 1, 2 or 3")
        self.B = self.free.collocated_mass()
        self.mask = torch.as_tensor(np.asarray(ess, dtype=np.uint8), device=self.device)
        self.us, self.ns = [], []  # newest first
        self.nstep = 0
        self._alpha = None
        self.p_prev = None
        self.last = {}

    def close(self):
        self.vel.close()
        self.free.close()

    def step(self, u, f=None):
        """Advance from u = u^n [3, ndof] (float64, 0 on the walls); f = f^{n+1} [3, ndof]
        nodal or None.  Returns (u^{n+1}, p^{n+1}); per-solve outcomes in self.last."""
        fr, dt, nu = self.free, self.dt, self.nu
        u = fr._vec(u, torch.float64, "u")
        if u.shape != (3, self.ndof):
            raise ValueError("u must have shape [3, ndof]")
        k = min(self.nstep + 1, self.order)
        b, a = bdf_ext_weights(k)
        n_new = fr.lincomb([-1.0], [self.vel.convection(u)], scale=self.B)
        self.us.insert(0, u.clone())  # the caller may reuse its buffer
        self.ns.insert(0, n_new)
        del self.us[k:], self.ns[k:]
        coefs = [a[j] for j in range(k)] + [-b[j + 1] / dt for j in range(k)]
        terms = self.ns[:k] + self.us[:k]
        if f is not None:
            coefs.append(1.0)
            terms.append(fr._vec(f, torch.float64, "f"))
        F = fr.lincomb(coefs, terms)
        ustar = fr.lincomb([a[j] for j in range(k)], self.us[:k])
        w = fr.lincomb([1.0], [fr.weak_op(WEAK_CURL, ustar)], scale=self.B)
        L = fr.lincomb([-nu], [fr.weak_op(WEAK_CURL, w)], scale=self.B)
        r = fr.weak_op(WEAK_DIVERGENCE, fr.lincomb([1.0, 1.0], [F, L]))
        # initial guesses: the previous pressure, the extrapolated velocity (0 on the walls)
        p, res_p = fr.pcg(r, x=self.p_prev, op=DIFFUSION, rtol=self.rtol, nullspace=True,
                          mode=self.pressure_mode)
        self.p_prev = p
        R = fr.lincomb([1.0, -1.0], [fr.apply(F, op=MASS), fr.weak_op(WEAK_GRADIENT, p)],
                       mask=self.mask)
        alpha = b[0] / dt
        if self._alpha != alpha:
            self.vel.set_coeffs(alpha, nu, None)
            self._alpha = alpha
        un, res_u = self.vel.pcg(R, x=ustar, op=HELMHOLTZ, rtol=self.rtol)
        if not (res_p.converged and res_u.converged):
            raise SfemError(1, f"projection step {self.nstep}: a solve did not converge")
        self.nstep += 1
        self.last = {"order": k, "pressure": res_p, "velocity": res_u}
        return un, p
