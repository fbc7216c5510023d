"""Oracle of the low-order-refined (LOR) operator of Section 5.2 (test infrastructure; FP64).

For the scalar problem A = alpha M + beta K(nu) on the Q_p discretization d, the LOR
operator A_LOR = alpha M_LOR + beta K_LOR is the standard trilinear (Q1) finite element
discretization of the same problem on the refined mesh that splits every element into
the p^3 sub-hexahedra spanned by the tensor products of its p + 1 Gauss-Lobatto-Legendre
points.  Its unknowns are the same nodal values (the GLL nodes are the vertices of the
refined mesh), so A_LOR and A act on the same vectors, and A_LOR has O(1) nonzeros per
row whatever p is.  Section 5.2 states that M_LOR, K_LOR are spectrally equivalent to M,
K with constants independent of h and p, which makes a solver for A_LOR a preconditioner
for A with h- and p-independent iteration counts.

Readings (the paper leaves them open):
  * sub-element geometry: the parent's trilinear map restricted to a sub-box is itself
    trilinear, so each sub-hexahedron is the trilinear element through the physical
    positions of its 8 GLL corner nodes;
  * quadrature: 2 x 2 x 2 Gauss points per sub-hexahedron (the standard Q1 rule, exact on
    parallelepipeds);
  * a per-quadrature-point nu enters as its mean over the parent element's points;
  * essential DoFs are constrained as for A: A_LOR,c = P A_LOR P + (I - P).

The Q1 element matrices are those of `Discretization` at p = 1 (Lagrange basis on the two
GLL points -1, 1 = the trilinear basis) with q = 2, evaluated on the refined mesh.
"""
from __future__ import annotations

import numpy as np

from .fem import Discretization, trilinear_shape
from .quadrature import gll


def refined_mesh(d: Discretization, points=None):
    """Vertices [NE p^3, 8, 3] and vertex DoFs [NE p^3, 8] of the refined mesh; sub-element
    s = e p^3 + i + p (j + p k) spans GLL intervals i, j, k of element e, vertex
    v = a + 2 b + 4 c sits at GLL node (i + a, j + b, k + c).  `points` replaces the GLL
    points (a test hook for planted mistakes)."""
    p, n = d.p, d.n
    pts = gll(p)[0] if points is None else np.asarray(points, dtype=np.float64)
    l = np.arange(n ** 3)
    XI = np.stack([pts[l % n], pts[(l // n) % n], pts[l // (n * n)]], axis=-1)
    N, _ = trilinear_shape(XI)
    node_x = np.einsum("evr,lv->elr", d.elem_xyz, N)  # [NE, n^3, 3] node positions
    ii, jj, kk = np.meshgrid(np.arange(p), np.arange(p), np.arange(p), indexing="ij")
    ii, jj, kk = (a.transpose(2, 1, 0).reshape(-1) for a in (ii, jj, kk))  # i fastest
    corner = np.empty((p ** 3, 8), dtype=np.int64)
    for v in range(8):
        a, b, c = v & 1, (v >> 1) & 1, (v >> 2) & 1
        corner[:, v] = (ii + a) + n * ((jj + b) + n * (kk + c))
    sub_x = node_x[:, corner, :].reshape(-1, 8, 3)
    sub_dofs = d.elem_dofs[:, corner].reshape(-1, 8)
    return sub_x, sub_dofs


def element_mean_nu(d: Discretization, nu):
    """Per-element mean of a per-point nu [NE, Q] (or None: 1)."""
    if nu is None:
        return np.ones(d.nelem)
    return np.asarray(nu, dtype=np.float64).reshape(d.nelem, d.nqp).mean(axis=1)


def lor_discretization(d: Discretization, points=None):
    """The refined Q1 discretization (same DoFs and essential DoFs as d)."""
    sub_x, sub_dofs = refined_mesh(d, points)
    return Discretization(sub_x, sub_dofs, d.ess, d.ndof, 1, 2)


def lor_matrix(d: Discretization, alpha, beta, nu=None, constrained=True, points=None):
    """Assembled A_LOR = alpha M_LOR + beta K_LOR(nu_e) (scipy CSR), nu_e the parent
    element's mean of nu, constrained like A unless constrained=False."""
    q1 = lor_discretization(d, points)
    nu_e = element_mean_nu(d, nu)
    nu_sub = np.repeat(nu_e, d.p ** 3)[:, None] * np.ones((1, q1.nqp))
    return q1.assemble(alpha, beta, nu_sub, constrained=constrained)
