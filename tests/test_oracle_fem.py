"""Pins of the oracle operators (Section 3, Section 3.1) against facts fixed by the mathematics.

* 1^T M 1 = |Omega| = 1 on the perturbed unit-cube meshes.
* u^T M v and u^T K v for linear u, v equal closed-form integrals over the unit
  cube: the integrands are polynomial in the reference coordinates of degree
  <= 2q-1 even on trilinear elements, so the tensor Gauss rule is exact.
* Patch test: for u linear, (K u)_i = int grad phi_i . a = 0 at interior DoFs,
  exactly, on perturbed meshes (the integrand grad_ref phi^T adj(J) a is a
  polynomial).  A transposed Jacobian fails this.
* K 1 = 0; K symmetric positive semi-definite with a one-dimensional kernel.
* Mass exactness at q = p + 2 (the integrand phi phi |J| has degree <= 2p + 2 per
  variable), checked against q = p + 6.
* Diagonal by brute force: diag_i = (A e_i)_i.
* Load vector: for linear f, b = M f_nodal.
* Each pin is also shown to reject a planted mistake in a copy of the oracle.
"""
import numpy as np
import pytest

from oracle import Discretization
from workloads import BoxMesh


def disc_for(ne, p, q=None, amp=0.1, seed=0):
    m = BoxMesh(ne, p, amp=amp, seed=seed)
    return m, Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2 if q is None else q)


def nodal(m, f):
    """Nodal values of f(x) at the DoF positions of a box mesh (trilinear image of GLL nodes)."""
    from oracle import gll
    from oracle.fem import trilinear_shape
    nodes, _ = gll(m.p)
    n = m.p + 1
    X = np.stack(np.meshgrid(nodes, nodes, nodes, indexing="ij"), -1).transpose(2, 1, 0, 3).reshape(-1, 3)
    N, _ = trilinear_shape(X)
    xyz = np.einsum("evr,lv->elr", m.elem_xyz, N)
    out = np.empty(m.ndof)
    out[m.elem_dofs.reshape(-1)] = f(xyz.reshape(-1, 3))
    return out


A_VEC = np.array([0.3, -1.1, 0.7])
B_VEC = np.array([-0.5, 0.2, 1.3])
C0, D0 = 0.4, -0.9


def lin(a, c):
    return lambda X: X @ a + c


def exact_mass_linear(a, c, b, d):
    # int_[0,1]^3 (a.x + c)(b.x + d) dx
    s = sum(a[r] * b[r] / 3.0 for r in range(3))
    s += sum(a[r] * b[t] / 4.0 for r in range(3) for t in range(3) if r != t)
    s += (c * b.sum() + d * a.sum()) / 2.0
    return s + c * d


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mass_volume_and_linear_moments(p):
    m, d = disc_for(3, p)
    M = d.assemble(1.0, 0.0, constrained=False)
    one = np.ones(m.ndof)
    assert abs(one @ (M @ one) - 1.0) < 1e-13
    u, v = nodal(m, lin(A_VEC, C0)), nodal(m, lin(B_VEC, D0))
    assert abs(u @ (M @ v) - exact_mass_linear(A_VEC, C0, B_VEC, D0)) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_stiffness_linear_energy_and_constants(p):
    m, d = disc_for(3, p)
    K = d.assemble(0.0, 1.0, constrained=False)
    one = np.ones(m.ndof)
    assert np.abs(K @ one).max() < 1e-13
    u, v = nodal(m, lin(A_VEC, C0)), nodal(m, lin(B_VEC, D0))
    assert abs(u @ (K @ v) - A_VEC @ B_VEC) < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_patch_test_interior(p):
    m, d = disc_for(3, p)
    u = nodal(m, lin(A_VEC, C0))
    Ku = d.apply_unconstrained(u, 0.0, 1.0)
    interior = ~m.ess.astype(bool)
    assert np.abs(Ku[interior]).max() < 1e-13
    # with a constant viscosity c the operator scales by c
    Ku3 = d.apply_unconstrained(u, 0.0, 1.0, nu=np.full((m.nelem, d.nqp), 3.0))
    assert np.allclose(Ku3, 3.0 * Ku, atol=1e-13)


def test_stiffness_spd_structure():
    m, d = disc_for(2, 2)
    K = d.assemble(0.0, 1.0, constrained=False).toarray()
    assert np.abs(K - K.T).max() < 1e-14
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-13 and abs(ev[0]) < 1e-13 and ev[1] > 1e-3
    Ac = d.assemble(1e3, 1.0, nu=np.random.default_rng(5).uniform(0.5, 2, (m.nelem, d.nqp))).toarray()
    assert np.abs(Ac - Ac.T).max() < 1e-12
    assert np.linalg.eigvalsh(Ac)[0] > 0


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mass_exact_at_q_p_plus_2(p):
    m, d2 = disc_for(3, p, q=p + 2)
    _, d6 = disc_for(3, p, q=p + 6)
    _, d1 = disc_for(3, p, q=p + 1)
    M2 = d2.assemble(1.0, 0.0, constrained=False)
    M6 = d6.assemble(1.0, 0.0, constrained=False)
    M1 = d1.assemble(1.0, 0.0, constrained=False)
    scale = np.abs(M6).max()
    assert np.abs(M2 - M6).max() < 1e-14 * max(1.0, scale) * 100
    assert np.abs(M1 - M6).max() > 1e-8 * scale  # under-integration is visible


def test_helmholtz_is_linear_combination():
    m, d = disc_for(2, 3)
    nu = np.random.default_rng(7).uniform(0.5, 2.0, (m.nelem, d.nqp))
    x = np.random.default_rng(8).standard_normal(m.ndof)
    yH = d.apply_unconstrained(x, 7.0, 0.3, nu)
    yM = d.apply_unconstrained(x, 1.0, 0.0, nu)
    yK = d.apply_unconstrained(x, 0.0, 1.0, nu)
    assert np.allclose(yH, 7.0 * yM + 0.3 * yK, rtol=0, atol=1e-13 * np.abs(yH).max())


def test_apply_equals_assembled_matrix():
    m, d = disc_for(3, 2)
    nu = np.random.default_rng(9).uniform(0.5, 2.0, (m.nelem, d.nqp))
    x = np.random.default_rng(10).standard_normal(m.ndof)
    A = d.assemble(1e3, 1.0, nu)
    y = d.apply(x, 1e3, 1.0, nu)
    assert np.abs(y - A @ x).max() <= 1e-13 * np.abs(y).max()
    ess = m.ess.astype(bool)
    assert np.array_equal(y[ess], x[ess])
    rows = np.array([0, 5, 40, 100, m.ndof // 2, m.ndof - 1])
    assert np.allclose(d.apply_rows(rows, x, 1e3, 1.0, nu), y[rows], rtol=1e-13, atol=0)
    # a single row of an element matrix equals that row of the full element matrix
    Ae = d.element_matrices(1e3, 1.0, nu, 5, 6)[0]
    assert np.allclose(d.element_row(5, 7, 1e3, 1.0, nu), Ae[7], rtol=1e-13, atol=1e-13 * np.abs(Ae).max())


def test_diagonal_brute_force():
    m, d = disc_for(4, 2)  # the 4^3, p = 2 Poisson workload: 729 DoFs
    nu = np.random.default_rng(11).uniform(0.5, 2.0, (m.nelem, d.nqp))
    diag = d.diagonal(1e3, 1.0, nu)
    E = np.eye(m.ndof)
    cols = d.apply(E, 1e3, 1.0, nu)  # rows of A_c e_i (A_c symmetric)
    assert np.abs(np.diag(cols) - diag).max() <= 1e-14 * np.abs(diag).max()


def test_load_vector_linear_source():
    m, d = disc_for(3, 3)
    f = lin(A_VEC, C0)
    xq = d.qpoint_coords()
    b = d.load(f(xq.reshape(-1, 3)).reshape(m.nelem, d.nqp))
    M = d.assemble(1.0, 0.0, constrained=False)
    bm = M @ nodal(m, f)
    bm[m.ess.astype(bool)] = 0.0
    assert np.abs(b - bm).max() < 1e-14


def test_qpoint_coords_inside_unit_cube_and_volume():
    m, d = disc_for(3, 2)
    xq = d.qpoint_coords()
    assert xq.min() > 0.0 and xq.max() < 1.0
    assert d.min_detJ() > 0


# ------------------------------------------------------------------------------------
# Planted mistakes: each must be rejected by one of the pins above.
# ------------------------------------------------------------------------------------
class _TransposedJ(Discretization):
    def geometry(self, e0, e1):
        det, inv, xq = super().geometry(e0, e1)
        return det, np.swapaxes(inv, -1, -2), xq


class _DroppedDet(Discretization):
    def geometry(self, e0, e1):
        det, inv, xq = super().geometry(e0, e1)
        return np.ones_like(det) / 8.0 * np.sign(det), inv, xq


class _SwappedDerivs(Discretization):
    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.dPhi = self.dPhi[..., [1, 0, 2]]


def _planted(cls, ne=3, p=3):
    m = BoxMesh(ne, p)
    return m, cls(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2)


def test_planted_transposed_jacobian_fails_patch_test():
    m, d = _planted(_TransposedJ)
    Ku = d.apply_unconstrained(nodal(m, lin(A_VEC, C0)), 0.0, 1.0)
    assert np.abs(Ku[~m.ess.astype(bool)]).max() > 1e-6


def test_planted_dropped_det_fails_volume():
    m, d = _planted(_DroppedDet)
    M = d.assemble(1.0, 0.0, constrained=False)
    one = np.ones(m.ndof)
    assert abs(one @ (M @ one) - 1.0) > 1e-6


def test_planted_swapped_derivative_directions_fail_energy():
    m, d = _planted(_SwappedDerivs)
    K = d.assemble(0.0, 1.0, constrained=False)
    u, v = nodal(m, lin(A_VEC, C0)), nodal(m, lin(B_VEC, D0))
    assert abs(u @ (K @ v) - A_VEC @ B_VEC) > 1e-6


def test_fan_mesh_volume_constants_and_linear_patch():
    """Unstructured fan mesh (3 kite columns x 2 layers): 1^T M 1 equals the exact volume
    3 sin(60 deg), K 1 = 0, and K annihilates the nodal values of a linear field at the
    DoFs off the boundary (patch test)."""
    from oracle.quadrature import gll
    from workloads import FanMesh
    p = 3
    m = FanMesh(p)
    d = Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2)
    one = np.ones(m.ndof)
    assert abs(d.apply_unconstrained(one, 1.0, 0.0).sum() - 3 * np.sin(np.pi / 3)) <= 1e-13
    assert np.abs(d.apply_unconstrained(one, 0.0, 1.0)).max() <= 1e-13
    # physical GLL node positions through each element's trilinear map
    t = (np.asarray(gll(p)[0]) + 1) / 2
    n = p + 1
    X = np.zeros((m.ndof, 3))
    for e in range(m.nelem):
        for l in range(n ** 3):
            a, b, c = t[l % n], t[(l // n) % n], t[l // (n * n)]
            w = np.array([(1 - a) * (1 - b) * (1 - c), a * (1 - b) * (1 - c), (1 - a) * b * (1 - c),
                          a * b * (1 - c), (1 - a) * (1 - b) * c, a * (1 - b) * c, (1 - a) * b * c, a * b * c])
            X[m.elem_dofs[e, l]] = w @ m.elem_xyz[e]
    xl = X @ np.array([0.3, -1.2, 0.7]) + 0.4
    r = d.apply_unconstrained(xl, 0.0, 1.0)
    outer = np.zeros(m.ndof, dtype=bool)
    for e in range(m.nelem):
        loc = m.elem_dofs[e].reshape(n, n, n)  # [k][j][i]
        outer[loc[:, -1, :].ravel()] = True    # j = p: the face R(theta_{s+1}) - corner
        outer[loc[:, :, -1].ravel()] = True    # i = p: the face R(theta_s) - corner
        outer[loc[0].ravel()] = outer[loc[-1].ravel()] = True  # bottom and top layers' caps
    on_cap = (np.abs(X[:, 2]) < 1e-12) | (np.abs(X[:, 2] - 1) < 1e-12)
    interior = ~outer | (~on_cap & (np.linalg.norm(X[:, :2], axis=1) < 1e-12))
    interior &= ~on_cap
    assert interior.sum() >= 2 * (p - 1) ** 3
    assert np.abs(r[interior]).max() <= 1e-12
