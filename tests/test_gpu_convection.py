"""The convection term N(u) (eq. nonlinear) on the GPU (through the C ABI) against the
oracle at p = 1..8, and at the 32^3, p = 4 size the identity that holds at any size for
linear velocity fields ((u . grad) u = A (A x + b), tested against the mass matrix)."""
import numpy as np
import pytest

from gpu_common import case, gpu, host, rel, say
from oracle import convection
from workloads import uniform

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_convection_vs_oracle(p):
    m, d, op = case(3 if p <= 4 else 2, p)
    u = uniform(3 * m.ndof, seed=21).reshape(3, -1)  # boundary values included
    y = op.convection(gpu(u))
    yo = convection(d, u)
    e = rel(host(y), yo)
    say(f"  p={p}: {e:.2e}")
    assert e <= 1e-12
    assert np.all(host(y)[:, m.ess.astype(bool)] == 0.0)
    op.close()


def _gll_node_coords(m, p):
    from oracle.fem import trilinear_shape
    from oracle.quadrature import gll
    pn, _ = gll(p)
    n = p + 1
    l = np.arange(n ** 3)
    XI = np.stack([pn[l % n], pn[(l // n) % n], pn[l // (n * n)]], axis=-1)
    N, _ = trilinear_shape(XI)
    x = np.zeros((m.ndof, 3))
    x[m.elem_dofs.reshape(-1)] = np.einsum("evr,mv->emr", m.elem_xyz, N).reshape(-1, 3)
    return x


def test_convection_linear_field_full_size_p4_32e():
    from paper_1910_03032_amd import MASS, Operator
    from workloads import BoxMesh
    m = BoxMesh(32, 4)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, 4, ess=m.ess)
    x = _gll_node_coords(m, 4)
    A = np.array([[0.3, -0.2, 0.5], [1.1, -0.4, 0.25], [-0.6, 0.8, 0.9]])
    b = np.array([0.1, -0.2, 0.3])
    u = (x @ A.T + b).T
    adv = ((x @ A.T + b) @ A.T).T
    y = host(op.convection(gpu(u)))
    op.close()
    free = Operator(m.elem_xyz, m.elem_dofs, m.ndof, 4)  # no essential DoFs: plain M
    fr = ~m.ess.astype(bool)
    # two different FP64 evaluations of the same integral (products of interpolated
    # values and gradients at the points vs the mass apply of the interpolated product,
    # whose components are smaller than |A| |u| by cancellation): a few 1e-13 to 1e-12
    for c in range(3):
        ref = host(free.apply(gpu(adv[c]), op=MASS))
        e = rel(y[c, fr], ref[fr])
        say(f"  component {c}: {e:.2e}")
        assert e <= 5e-12
    free.close()
    assert np.all(y[:, ~fr] == 0.0)


def test_convection_errors():
    from paper_1910_03032_amd import SfemError
    m, _, op = case(2, 2)
    u = gpu(uniform(3 * m.ndof, seed=3).reshape(3, -1))
    with pytest.raises(SfemError, match="SFEM_E_ARG"):
        op._check(op._lib.sfem_convection(op._h, u.data_ptr(), u.data_ptr()))
    with pytest.raises(ValueError):
        op.convection(gpu(np.zeros((2, m.ndof))))
    op.close()
