"""The Taylor-Hood Stokes block operator on the GPU (through the C ABI) against the
oracle: the full constrained block apply at p = 2..8 element by element, its gradient
and divergence blocks separately, and at the 32^3, p = 4 size the identities that hold
at any size (integration by parts, the gradient of a linear pressure); plus error paths."""
import numpy as np
import pytest
import torch

from gpu_common import gpu, host, rel, say
from oracle import StokesDiscretization
from workloads import TaylorHoodMesh, uniform, nu_uniform

pytestmark = pytest.mark.gpu


def build(ne, p, nu=None, alpha=10.0, beta=0.5, oracle=True):
    from paper_1910_03032_amd import Operator
    m = TaylorHoodMesh(ne, p)
    v = m.vel
    say(f"[stokes] ne={ne} p={p} nv={v.ndof} np={m.npres}")
    op = Operator(v.elem_xyz, v.elem_dofs, v.ndof, p, ess=v.ess)
    op.set_coeffs(alpha, beta, None if nu is None else gpu(nu))
    op.setup_pressure(m.pres_dofs, m.npres)
    S = None
    if oracle:
        S = StokesDiscretization(v.elem_xyz, v.elem_dofs, v.ess, v.ndof, m.pres_dofs, m.npres, p,
                                 p + 2)
    return m, op, S


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_stokes_block_apply_vs_oracle(p):
    ne = 3 if p <= 4 else 2
    m0 = TaylorHoodMesh(ne, p)
    nu = nu_uniform(m0.nelem, p + 2, seed=2)
    m, op, S = build(ne, p, nu=nu)
    u = uniform(3 * m.vel.ndof, seed=5).reshape(3, -1)
    pres = uniform(m.npres, seed=6)
    yu, yp = op.stokes_apply(gpu(u), gpu(pres))
    ou, opp = S.apply(u, pres, 10.0, 0.5, nu)
    eu, ep = rel(host(yu), ou), rel(host(yp), opp)
    say(f"  p={p}: velocity rows {eu:.2e}, pressure rows {ep:.2e}")
    assert eu <= 1e-12 and ep <= 1e-12
    op.close()


@pytest.mark.parametrize("p", [2, 5])
def test_gradient_and_divergence_blocks_separately(p):
    m, op, S = build(3 if p == 2 else 2, p, alpha=0.0, beta=0.0)
    ess = m.vel.ess.astype(bool)
    pres = uniform(m.npres, seed=7)
    yu, yp = op.stokes_apply(gpu(np.zeros((3, m.vel.ndof))), gpu(pres))
    g = S.gradient(pres)
    g[:, ess] = 0.0
    assert rel(host(yu), g) <= 1e-12
    assert np.all(host(yp) == 0.0)
    u = uniform(3 * m.vel.ndof, seed=8).reshape(3, -1)
    yu, yp = op.stokes_apply(gpu(u), gpu(np.zeros(m.npres)))
    uf = u.copy()
    uf[:, ess] = 0.0
    assert rel(host(yp), -S.divergence(uf)) <= 1e-12
    # alpha = beta = 0: free velocity rows are 0, essential rows copy u
    assert np.all(host(yu)[:, ~ess] == 0.0) and np.array_equal(host(yu)[:, ess], u[:, ess])
    op.close()


def test_full_size_identities_p4_32e():
    """32^3, p = 4 (2.1M velocity DoFs per component, 0.9M pressure DoFs): integration by
    parts u.(G p) + p.(D u) = 0 for u vanishing on the boundary, and G of a linear
    pressure equals a_c M 1 on the free rows (M 1 from the library's unconstrained mass
    apply)."""
    m, op, _ = build(32, 4, alpha=0.0, beta=0.0, oracle=False)
    ess = m.vel.ess.astype(bool)
    nv = m.vel.ndof
    u = uniform(3 * nv, seed=9).reshape(3, -1)
    u[:, ess] = 0.0
    pres = uniform(m.npres, seed=10)
    gu, _ = op.stokes_apply(gpu(np.zeros((3, nv))), gpu(pres))
    _, du = op.stokes_apply(gpu(u), gpu(np.zeros(m.npres)))
    lhs = float(np.sum(u * host(gu)))
    rhs = -float(pres @ host(du))  # du = -D u
    say(f"  u.Gp = {lhs:.6e}, p.Du = {rhs:.6e}")
    assert abs(lhs + rhs) <= 1e-12 * (abs(lhs) + abs(rhs))
    # gradient of a linear pressure: nodal values at the pressure GLL nodes mapped by the
    # trilinear element map (the oracle's rules)
    from oracle.quadrature import gll
    from oracle.fem import trilinear_shape
    pn, _ = gll(3)
    l = np.arange(64)
    XI = np.stack([pn[l % 4], pn[(l // 4) % 4], pn[l // 16]], axis=-1)
    N, _ = trilinear_shape(XI)
    xp = np.zeros((m.npres, 3))
    xp[m.pres_dofs.reshape(-1)] = np.einsum("evr,mv->emr", m.vel.elem_xyz, N).reshape(-1, 3)
    a = np.array([0.7, -1.3, 2.1])
    gl, _ = op.stokes_apply(gpu(np.zeros((3, nv))), gpu(xp @ a + 0.25))
    op.close()
    # int phi_i dx: the unconstrained mass applied to 1 (a context without essential DoFs)
    from paper_1910_03032_amd import MASS, Operator
    free = Operator(m.vel.elem_xyz, m.vel.elem_dofs, nv, 4)
    mass1 = host(free.apply(gpu(np.ones(nv)), op=MASS))
    free.close()
    for c in range(3):
        assert rel(host(gl)[c, ~ess], a[c] * mass1[~ess]) <= 1e-12


def test_stokes_errors():
    from paper_1910_03032_amd import Operator, SfemError
    from workloads import BoxMesh
    m1 = BoxMesh(2, 1)
    op1 = Operator(m1.elem_xyz, m1.elem_dofs, m1.ndof, 1, ess=m1.ess)
    with pytest.raises(SfemError, match="SFEM_E_UNSUPPORTED"):
        op1.setup_pressure(np.zeros((m1.nelem, 1), dtype=np.int32), 1)
    op1.close()
    m = TaylorHoodMesh(2, 2)
    v = m.vel
    op = Operator(v.elem_xyz, v.elem_dofs, v.ndof, 2, ess=v.ess)
    op.npres = m.npres
    with pytest.raises(SfemError, match="SFEM_E_STATE"):
        op.stokes_apply(gpu(np.zeros((3, v.ndof))), gpu(np.zeros(m.npres)))
    bad = m.pres_dofs.copy()
    bad[0, 0] = m.npres  # out of range
    with pytest.raises(SfemError, match="SFEM_E_MESH"):
        op.setup_pressure(bad, m.npres)
    op.setup_pressure(m.pres_dofs, m.npres)
    with pytest.raises(SfemError, match="SFEM_E_STATE"):
        op.setup_pressure(m.pres_dofs, m.npres)
    nu2 = np.ones((2, m.nelem * 64))
    op.set_coeffs(1.0, 1.0, gpu(nu2))
    with pytest.raises(SfemError, match="SFEM_E_ARG"):
        op.stokes_apply(gpu(np.zeros((3, v.ndof))), gpu(np.zeros(m.npres)))
    op.close()


@pytest.mark.parametrize("p", [2, 5])
def test_stokes_and_convection_on_fan_mesh(p):
    """Unstructured fan mesh (axis DoFs shared by 3 or 6 elements in both the velocity and
    the pressure maps): the block apply and the convection term match the oracle."""
    from oracle import convection
    from paper_1910_03032_amd import Operator
    from workloads import FanMesh
    m, pm = FanMesh(p), FanMesh(p - 1)
    say(f"[stokes] fan mesh p={p} nv={m.ndof} np={pm.ndof}")
    q = p + 2
    nu = nu_uniform(m.nelem, q, seed=4)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=m.ess)
    op.set_coeffs(2.0, 0.7, gpu(nu))
    op.setup_pressure(pm.elem_dofs, pm.ndof)
    S = StokesDiscretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, pm.elem_dofs, pm.ndof, p, q)
    u = uniform(3 * m.ndof, seed=14).reshape(3, -1)
    pres = uniform(pm.ndof, seed=15)
    yu, yp = op.stokes_apply(gpu(u), gpu(pres))
    ou, opp = S.apply(u, pres, 2.0, 0.7, nu)
    assert rel(host(yu), ou) <= 1e-12 and rel(host(yp), opp) <= 1e-12
    assert rel(host(op.convection(gpu(u))), convection(S.vel, u)) <= 1e-12
    op.close()
