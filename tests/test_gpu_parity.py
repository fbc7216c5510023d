"""HIP path vs the CPU oracle, element by element, through the C ABI.

Tolerances (relative 2-norm over all DoFs): FP64 apply / diagonal / load <= 1e-12,
FP32 apply <= 1e-5 against the FP64 oracle, geometric quantities <= 1e-13.
Sizes span several workgroups and ragged tails (3^3 and 5^3 element meshes are not
multiples of the elements per workgroup, and the interior/shared/essential DoF
classes all occur).
"""
import numpy as np
import pytest
import torch

from gpu_common import case, gpu, host, rel, say, nu_c2_gpu, nu_c2_oracle
from workloads import uniform, nu_uniform, normal

pytestmark = pytest.mark.gpu

OPS = {0: (1.0, 0.0), 1: (0.0, 1.0)}


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_apply_fp64_all_ops(p):
    ne = 3 if p >= 5 else 5
    m, d, op = case(ne, p)
    x = uniform(m.ndof, seed=1)
    nu = nu_uniform(m.nelem, d.q, seed=2)
    xg = gpu(x)
    # mass, diffusion (nu = 1), diffusion with nu, helmholtz with nu
    y = host(op.apply(xg, op=0))
    assert rel(y, d.apply(x, 1.0, 0.0)) <= 1e-12
    y = host(op.apply(xg, op=1))
    assert rel(y, d.apply(x, 0.0, 1.0)) <= 1e-12
    op.set_coeffs(1e3, 0.7, gpu(nu))
    y = host(op.apply(xg, op=1))
    assert rel(y, d.apply(x, 0.0, 1.0, nu)) <= 1e-12
    y = host(op.apply(xg, op=2))
    yo = d.apply(x, 1e3, 0.7, nu)
    say(f"  p={p} helmholtz fp64 rel err {rel(y, yo):.2e}")
    assert rel(y, yo) <= 1e-12
    ess = m.ess.astype(bool)
    assert np.array_equal(y[ess], x[ess])


@pytest.mark.parametrize("p", [1, 2, 4, 7, 8])
def test_apply_fp32(p):
    ne = 3 if p >= 5 else 4
    m, d, op = case(ne, p)
    x = uniform(m.ndof, seed=1)
    nu = nu_uniform(m.nelem, d.q, seed=2)
    op.set_coeffs(1e3, 1.0, gpu(nu))
    yo = d.apply(x, 1e3, 1.0, nu)
    y32 = host(op.apply(gpu(x, torch.float32), op=2))
    e = rel(y32, yo)
    say(f"  p={p} helmholtz fp32 rel err {e:.2e}")
    assert e <= 1e-5
    for k in (0, 1):
        a, b = OPS[k]
        assert rel(host(op.apply(gpu(x, torch.float32), op=k)), d.apply(x, a, b, nu if k == 1 else None)) <= 1e-5


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_diagonal(p):
    m, d, op = case(3, p)
    nu = nu_uniform(m.nelem, d.q, seed=2)
    op.set_coeffs(1e3, 1.0, gpu(nu))
    for k, (a, b) in [(0, (1.0, 0.0)), (1, (0.0, 1.0)), (2, (1e3, 1.0))]:
        dg = host(op.diagonal(op=k))
        do = d.diagonal(a, b, nu if k else None)
        assert rel(dg, do) <= 1e-12, (k, rel(dg, do))
    d32 = host(op.diagonal(op=2, dtype=torch.float32))
    assert rel(d32, d.diagonal(1e3, 1.0, nu)) <= 1e-7


def test_diagonal_brute_force_poisson_p2_4e():
    """diag_i = (A e_i)_i on the 4^3, p = 2 workload, all 729 unit vectors in one batch."""
    m, d, op = case(4, 2)
    E = torch.eye(m.ndof, dtype=torch.float64, device="cuda")
    AE = host(op.apply(E, op=1))
    assert rel(np.diag(AE), host(op.diagonal(op=1))) <= 1e-13
    # and the brute-force columns equal the oracle's assembled matrix
    A = d.assemble(0.0, 1.0).toarray()
    assert np.abs(AE - A).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("p", [2, 5])
def test_qpoint_coords_and_load(p):
    m, d, op = case(3, p)
    xq = host(op.qpoint_coords())
    xo = d.qpoint_coords()
    assert np.abs(xq - xo.reshape(-1, 3).T).max() <= 1e-14
    f = uniform(m.nelem * d.nqp, seed=5)
    bg = host(op.load(gpu(f)))
    bo = d.load(f.reshape(m.nelem, d.nqp))
    assert rel(bg, bo) <= 1e-12


@pytest.mark.parametrize("p", [2, 5])
def test_grad_nu_kernel(p):
    m, d, op = case(3, p)
    u, lam = uniform(m.ndof, seed=7), uniform(m.ndof, seed=8)
    op.set_coeffs(1e3, 0.6, None)
    g = host(op.grad_nu(gpu(u), gpu(lam)))
    go = d.grad_nu(u, lam, 0.6).reshape(-1)
    # the integrand uses P u, P lam (essential entries zeroed)
    uf, lf = u.copy(), lam.copy()
    uf[m.ess.astype(bool)] = 0
    lf[m.ess.astype(bool)] = 0
    go = d.grad_nu(uf, lf, 0.6).reshape(-1)
    assert rel(g, go) <= 1e-12


def test_batched_apply_equals_single_bitwise():
    m, d, op = case(4, 3)
    X = np.stack([uniform(m.ndof, seed=s) for s in (1, 2, 3)])
    op.set_coeffs(1e3, 1.0, gpu(nu_uniform(m.nelem, d.q, seed=2)))
    Y = op.apply(gpu(X), op=2)
    for k in range(3):
        assert torch.equal(Y[k], op.apply(gpu(X[k]), op=2))
    Y32 = op.apply(gpu(X, torch.float32), op=2)
    assert torch.equal(Y32[1], op.apply(gpu(X[1], torch.float32), op=2))


def test_per_member_nu_fields():
    m, d, op = case(3, 4)
    nus = np.stack([nu_uniform(m.nelem, d.q, seed=200 + k).reshape(-1) for k in range(4)])
    X = np.stack([uniform(m.ndof, seed=10 + k) for k in range(4)])
    op.set_coeffs(1e3, 1.0, gpu(nus))
    Y = host(op.apply(gpu(X), op=2))
    D = host(op.diagonal(op=2))
    for k in range(4):
        assert rel(Y[k], d.apply(X[k], 1e3, 1.0, nus[k])) <= 1e-12
        assert rel(D[k], d.diagonal(1e3, 1.0, nus[k])) <= 1e-12
    Yk = host(op.apply(gpu(X), op=1))
    assert rel(Yk[2], d.apply(X[2], 0.0, 1.0, nus[2])) <= 1e-12


def test_determinism_bitwise():
    m, d, op = case(5, 4)
    op.set_coeffs(1e3, 1.0, gpu(nu_uniform(m.nelem, d.q, seed=2)))
    x = gpu(normal(m.ndof, seed=1))
    y0 = op.apply(x, op=2)
    for _ in range(3):
        assert torch.equal(op.apply(x, op=2), y0)
    b = gpu(normal(m.ndof, seed=3))
    b[torch.as_tensor(m.ess.astype(bool), device="cuda")] = 0
    x1, r1 = op.pcg(b, rtol=1e-8)
    x2, r2 = op.pcg(b, rtol=1e-8)
    assert torch.equal(x1, x2) and r1.iters == r2.iters


def test_helmholtz_workload_p4_32e_sampled_rows():
    """Full 32^3, p = 4 Helmholtz workload (2.1M DoFs) in the benchmarked configuration:
    sampled rows against the oracle's one-row evaluation."""
    m, d, op = case(32, 4)
    nu_g = nu_c2_gpu(op)
    op.set_coeffs(1e3, 1.0, nu_g)
    x = normal(m.ndof, seed=1)
    y = host(op.apply(gpu(x), op=2))
    nu_o = nu_c2_oracle(d)
    rng = np.random.default_rng(42)
    rows = np.concatenate([rng.integers(0, m.ndof, 40), [0, 1, m.ndof // 2, m.ndof - 1]])
    yo = d.apply_rows(rows, x, 1e3, 1.0, nu_o)
    err = np.abs(y[rows] - yo).max() / np.abs(yo).max()
    say(f"  sampled rows max rel err {err:.2e}")
    assert err <= 1e-12
    # fp32 on the same rows
    y32 = host(op.apply(gpu(x, torch.float32), op=2))
    assert np.abs(y32[rows] - yo).max() / np.abs(yo).max() <= 1e-5


def _shared_interior_mesh():
    """A 2^3, p = 2 mesh whose element 1 reuses element 0's interior node: the
    element-interior node is then shared, which switches the library to its general
    (non-compact) E-vector layout."""
    from workloads import BoxMesh
    m = BoxMesh(2, 2)
    dofs = m.elem_dofs.copy()
    center = 13  # local (1, 1, 1)
    d0, d1 = dofs[0, center], dofs[1, center]
    dofs[1, center] = d0
    last = m.ndof - 1
    dofs[dofs == last] = d1  # relabel the last DoF into the freed index
    ess = m.ess.copy()
    ess[d1] = ess[last]
    return m, dofs, ess[:last], last


def test_general_layout_when_interior_nodes_are_shared():
    from oracle import Discretization
    from paper_1910_03032_amd import Operator
    m, dofs, ess, ndof = _shared_interior_mesh()
    d = Discretization(m.elem_xyz, dofs, ess, ndof, 2, 4)
    op = Operator(m.elem_xyz, dofs, ndof, 2, ess=ess)
    assert op.info()["compact"] == 0
    x = uniform(ndof, seed=1)
    nu = nu_uniform(m.nelem, 4, seed=2)
    op.set_coeffs(1e3, 1.0, gpu(nu))
    assert rel(host(op.apply(gpu(x), op=2)), d.apply(x, 1e3, 1.0, nu)) <= 1e-12
    assert rel(host(op.diagonal(op=2)), d.diagonal(1e3, 1.0, nu)) <= 1e-12
    f = uniform(m.nelem * 64, seed=5)
    assert rel(host(op.load(gpu(f))), d.load(f.reshape(m.nelem, 64))) <= 1e-12
    # the standard box mesh uses the compact layout
    _, _, op2 = case(2, 2)
    assert op2.info()["compact"] == 1


@pytest.mark.parametrize("p", [2, 3])
def test_fan_mesh_multiplicities_3_and_6(p):
    """Unstructured fan mesh (3 kite columns x 2 layers around an axis): axis DoFs are
    shared by 3 or 6 elements, so the assembly plan pads classes 4 and 8.  Every
    operator, the diagonal, the load vector and a solve match the oracle."""
    from oracle import Discretization
    from paper_1910_03032_amd import Operator
    from workloads import FanMesh
    m = FanMesh(p)
    q = p + 2
    say(f"[case] fan mesh p={p} nelem={m.nelem} ndof={m.ndof}")
    d = Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, q)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=m.ess)
    assert op.info()["compact"] == 1
    nu = nu_uniform(m.nelem, q, seed=2)
    op.set_coeffs(3.0, 0.7, gpu(nu))
    x = uniform(m.ndof, seed=1)
    # SFEM_MASS is M, SFEM_DIFFUSION is K(nu), SFEM_HELMHOLTZ is alpha M + beta K(nu)
    for opk, (a, b) in ((0, (1.0, 0.0)), (1, (0.0, 1.0)), (2, (3.0, 0.7))):
        yo = d.apply(x, a, b, nu if opk else None)
        assert rel(host(op.apply(gpu(x), op=opk)), yo) <= 1e-12, opk
        assert rel(host(op.apply(gpu(x, torch.float32), op=opk)), yo) <= 1e-5, opk
        assert rel(host(op.diagonal(op=opk)), d.diagonal(a, b, nu if opk else None)) <= 1e-12, opk
    f = uniform(m.nelem * q ** 3, seed=5)
    assert rel(host(op.load(gpu(f))), d.load(f.reshape(m.nelem, q ** 3))) <= 1e-12
    bvec = uniform(m.ndof, seed=3)
    bvec[m.ess.astype(bool)] = 0
    xs, res = op.pcg(gpu(bvec), rtol=1e-12)
    assert res.converged
    import scipy.sparse.linalg as spla
    xd = spla.spsolve(d.assemble(3.0, 0.7, nu).tocsc(), bvec)
    assert rel(host(xs), xd) <= 1e-9
