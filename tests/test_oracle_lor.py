"""Pins of the LOR operator oracle (Section 5.2; oracle/lor.py) against what the mathematics
fixes:

* at p = 1 the refined mesh is the mesh itself: on an affine mesh (where both the q = 3
  rule of the Q_p operator and the 2-point rule of the Q1 operator are exact) A_LOR = A;
* the refined mesh's vertices are the GLL nodes of the parent elements, and its
  sub-elements fill the parents: 1^T M_LOR 1 = |Omega| = 1 on a perturbed mesh;
* K_LOR annihilates constants and passes the patch test (linear fields give zero rows at
  interior DoFs) on perturbed trilinear meshes, where the Q1 integrand is polynomial;
* spectral equivalence: the generalized eigenvalues of (A, A_LOR) on the free DoFs stay in
  a fixed band as p grows (p = 2..6), while those of (A, diag A) spread like a power of p;
  a refined mesh on equispaced instead of GLL points loses that bound;
* CG preconditioned by an exact A_LOR solve needs an h-independent number of iterations
  and a number growing only slowly with p, far below diagonally preconditioned CG.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import Discretization, pcg
from oracle.fem import trilinear_shape
from oracle.lor import lor_matrix, refined_mesh
from oracle.quadrature import gll
from workloads import BoxMesh, rhs_uniform


def disc(ne, p, amp=0.1):
    m = BoxMesh(ne, p, amp=amp)
    return m, Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2)


def node_positions(m, p):
    pn, _ = gll(p)
    n = p + 1
    l = np.arange(n ** 3)
    XI = np.stack([pn[l % n], pn[(l // n) % n], pn[l // (n * n)]], axis=-1)
    N, _ = trilinear_shape(XI)
    x = np.zeros((m.ndof, 3))
    x[m.elem_dofs.reshape(-1)] = np.einsum("evr,lv->elr", m.elem_xyz, N).reshape(-1, 3)
    return x


def test_p1_affine_lor_is_the_operator():
    m, d = disc(3, 1, amp=0.0)
    for alpha, beta in ((1.0, 0.0), (0.0, 1.0), (1e3, 0.7)):
        A = d.assemble(alpha, beta).toarray()
        L = lor_matrix(d, alpha, beta).toarray()
        assert np.abs(A - L).max() <= 1e-13 * np.abs(A).max()


def test_refined_mesh_vertices_volume_constants_patch():
    p = 4
    m, d = disc(2, p)
    sub_x, sub_dofs = refined_mesh(d)
    x = node_positions(m, p)
    assert sub_x.shape == (m.nelem * p ** 3, 8, 3)
    assert np.abs(sub_x - x[sub_dofs]).max() <= 1e-15  # vertices are the GLL nodes
    M = lor_matrix(d, 1.0, 0.0, constrained=False)
    ones = np.ones(m.ndof)
    assert abs(ones @ (M @ ones) - 1.0) <= 1e-13
    K = lor_matrix(d, 0.0, 1.0, constrained=False)
    assert np.abs(K @ ones).max() <= 1e-12
    xl = x @ np.array([0.3, -1.1, 0.7]) + 0.2
    r = K @ xl
    interior = ~m.ess.astype(bool)
    assert np.abs(r[interior]).max() <= 1e-12 * np.abs(K).max()
    # O(1) nonzeros per row, independent of p: at most 27 on this structured mesh
    assert np.diff(K.indptr).max() <= 27


def _eig_band(ne, p, alpha, beta, points=None):
    m, d = disc(ne, p)
    A = d.assemble(alpha, beta).toarray()
    L = lor_matrix(d, alpha, beta, points=points).toarray()
    f = ~m.ess.astype(bool)
    A, L = A[np.ix_(f, f)], L[np.ix_(f, f)]
    ev = sla.eigh(A, L, eigvals_only=True)
    evj = sla.eigh(A, np.diag(np.diag(A)), eigvals_only=True)
    return ev.min(), ev.max(), evj.max() / evj.min()


def test_spectral_equivalence_bounded_in_p():
    """(A, A_LOR) on a perturbed 2^3 mesh, Poisson: every eigenvalue in [0.6, 8] for
    p = 2..6 (measured 0.63..7.5), condition number below 12, while the Jacobi one grows
    from ~3 to ~95; Helmholtz (alpha = 1e3): in [0.45, 9]."""
    kap = []
    for p in range(2, 7):
        lo, hi, kj = _eig_band(2, p, 0.0, 1.0)
        assert 0.6 <= lo and hi <= 8.0, (p, lo, hi)
        kap.append((hi / lo, kj))
        lo, hi, _ = _eig_band(2, p, 1e3, 1.0)
        assert 0.45 <= lo and hi <= 9.0, (p, lo, hi)
    assert max(k for k, _ in kap) < 12.0
    assert kap[-1][1] > 80 and kap[-1][1] > 8 * kap[-1][0]


def test_equispaced_refinement_loses_the_bound():
    """Planted mistake: sub-elements on equispaced points (not the GLL points) give a
    condition number that grows much faster with p (29 vs 12 at p = 6)."""
    p = 6
    lo, hi, _ = _eig_band(2, p, 0.0, 1.0, points=np.linspace(-1.0, 1.0, p + 1))
    lo_g, hi_g, _ = _eig_band(2, p, 0.0, 1.0)
    assert hi / lo > 2.0 * hi_g / lo_g


@pytest.mark.parametrize("ne,p", [(2, 3), (4, 3), (6, 3), (3, 2), (3, 4), (3, 6)])
def test_lor_preconditioned_cg_iterations(ne, p):
    """CG to 1e-10 on the Poisson problem with an exact A_LOR solve as preconditioner:
    at most 40 iterations (measured 24..39 for these meshes), against 21..118 for the
    Jacobi-preconditioned CG, which grows with both h^-1 and p."""
    m, d = disc(ne, p)
    lu = spla.splu(lor_matrix(d, 0.0, 1.0).tocsc())
    b = rhs_uniform(m, seed=1)[0]
    x, it, rr = pcg(lambda v: d.apply(v, 0.0, 1.0), b, None, rtol=1e-10, precond=lu.solve)
    _, itj, _ = pcg(lambda v: d.apply(v, 0.0, 1.0), b, 1.0 / d.diagonal(0.0, 1.0), rtol=1e-10)
    assert rr <= 1e-10 and it <= 40, (it, itj)
    if ne * p >= 12:
        assert itj > 1.5 * it, (it, itj)
