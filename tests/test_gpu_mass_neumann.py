"""Collocated mass preconditioning (Section 5.1) and the pure-Neumann Poisson problem with
the mean-zero condition (Section 3, eq. meanZero; Section 5.3) on the GPU, against the
oracle through the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gpu_common import gpu, host, rel, say
from oracle import Discretization, pcg as oracle_pcg, neumann_poisson
from workloads import BoxMesh, nu_uniform, uniform

pytestmark = pytest.mark.gpu


def _case(ne, p, ess=True, amp=0.1):
    from paper_1910_03032_amd import Operator
    m = BoxMesh(ne, p, amp=amp)
    e = m.ess if ess else np.zeros(m.ndof, np.uint8)
    d = Discretization(m.elem_xyz, m.elem_dofs, e, m.ndof, p, p + 2)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=e if ess else None)
    say(f"[case] ne={ne} p={p} ess={ess} ndof={m.ndof}")
    return m, d, op


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_collocated_mass_diagonal(p):
    for ess in (True, False):
        m, d, op = _case(3, p, ess)
        dg = host(op.collocated_mass())
        do = d.collocated_mass_diagonal(constrained=True)
        assert rel(dg, do) <= 1e-13, (p, ess, rel(dg, do))


@pytest.mark.parametrize("p", [1, 3, 5, 8])
def test_mass_solve_collocated_preconditioner(p):
    """M x = b with the collocated preconditioner: sparse direct solution, the oracle's
    iteration count (within 2) and the spectral-equivalence iteration bound."""
    from paper_1910_03032_amd import MASS, PRECOND_COLLOCATED_MASS
    m, d, op = _case(3, p, ess=False)
    b = uniform(m.ndof, seed=1)
    x, res = op.pcg(gpu(b), op=MASS, rtol=1e-12, check_every=1, precond=PRECOND_COLLOCATED_MASS)
    assert res.converged
    xd = spla.spsolve(d.assemble(1.0, 0.0, constrained=False).tocsc(), b)
    assert rel(host(x), xd) <= 1e-10
    _, it_o, _ = oracle_pcg(lambda v: d.apply(v, 1.0, 0.0), b, 1.0 / d.collocated_mass_diagonal(False),
                            rtol=1e-12)
    say(f"  p={p}: iterations gpu {res.iters[0]} oracle {it_o}")
    assert abs(res.iters[0] - it_o) <= 2
    assert res.iters[0] <= int(np.ceil(0.5 * np.sqrt(27.3) * np.log(2 / 1e-12)))
    # the FP32-inner refinement uses the same preconditioner
    x2, r2 = op.pcg(gpu(b), op=MASS, rtol=1e-10, mode=1, precond=PRECOND_COLLOCATED_MASS)
    assert r2.converged and r2.true_rel_res[0] <= 1e-10


@pytest.mark.parametrize("p", [1, 2, 4, 6])
def test_neumann_poisson_vs_oracle_and_bordered_solve(p):
    from paper_1910_03032_amd import DIFFUSION
    m, d, op = _case(3, p, ess=False)
    nu = nu_uniform(m.nelem, d.q, seed=2)
    op.set_coeffs(0.0, 1.0, gpu(nu))
    b = uniform(m.ndof, seed=1)
    x, res = op.pcg(gpu(b), op=DIFFUSION, rtol=1e-12, check_every=1, nullspace=True)
    assert res.converged and res.true_rel_res[0] <= 1e-11
    xo, it_o, _ = neumann_poisson(d, b, nu, rtol=1e-12)
    say(f"  p={p}: iterations gpu {res.iters[0]} oracle {it_o}")
    assert abs(res.iters[0] - it_o) <= 2
    assert rel(host(x), xo) <= 1e-9
    K = d.assemble(0.0, 1.0, nu, constrained=False).tocsc()
    m1 = d.apply(np.ones(m.ndof), 1.0, 0.0)
    A = sp.bmat([[K, sp.csc_matrix(m1[:, None])], [sp.csc_matrix(m1[None, :]), None]]).tocsc()
    xd = spla.spsolve(A, np.concatenate([b - b.mean(), [0.0]]))[:-1]
    assert rel(host(x), xd) <= 1e-9
    assert abs(np.dot(m1, host(x))) <= 1e-12 * np.linalg.norm(host(x))
    # from an initial guess (with a constant part, which the null space ignores): the same
    # solution in fewer iterations
    x0 = xd + 1e-6 * uniform(m.ndof, seed=9) + 3.0
    x2, res2 = op.pcg(gpu(b), x=gpu(x0), op=DIFFUSION, rtol=1e-12, check_every=1, nullspace=True)
    say(f"  p={p}: from a close initial guess {res2.iters[0]} iterations")
    assert res2.converged and res2.iters[0] < res.iters[0]
    assert rel(host(x2), xd) <= 1e-9
    # FP32 inner solves inside FP64 refinement, orthogonalized the same way
    x3, res3 = op.pcg(gpu(b), op=DIFFUSION, rtol=1e-12, mode=1, nullspace=True)
    say(f"  p={p}: FP32+IR {res3.iters[0]} inner iterations in {res3.outer[0]} refinement steps")
    assert res3.converged and res3.true_rel_res[0] <= 1e-11
    assert rel(host(x3), xd) <= 1e-9
    assert abs(np.dot(m1, host(x3))) <= 1e-12 * np.linalg.norm(host(x3))


def test_neumann_poisson_manufactured_rate_gpu():
    """u = cos(pi x) cos(pi y) cos(pi z) (zero normal derivative, mean zero) from the GPU
    load vector and null-space solve; L2 error (oracle) at rate >= p + 1 - 0.3, p = 2."""
    from paper_1910_03032_amd import DIFFUSION
    p = 2
    errs = []
    for ne in (2, 4, 8):
        m, d, op = _case(ne, p, ess=False)
        op.set_coeffs(0.0, 1.0, None)
        xq = op.qpoint_coords()
        import torch
        f = 3 * np.pi ** 2 * torch.cos(np.pi * xq[0]) * torch.cos(np.pi * xq[1]) * torch.cos(np.pi * xq[2])
        x, res = op.pcg(op.load(f), op=DIFFUSION, rtol=1e-12, nullspace=True)
        assert res.converged
        u = lambda a, b_, c: np.cos(np.pi * a) * np.cos(np.pi * b_) * np.cos(np.pi * c)
        errs.append(d.l2_error(host(x), u))
    rates = np.diff(np.log(errs)) / np.log(0.5)
    say(f"  L2 errors {errs}, rates {rates}")
    assert rates[-1] >= p + 1 - 0.3


def test_nullspace_option_errors():
    from paper_1910_03032_amd import DIFFUSION, HELMHOLTZ, SfemError
    m, d, op = _case(2, 2, ess=True)
    b = gpu(uniform(m.ndof, seed=1))
    with pytest.raises(SfemError):
        op.pcg(b, op=DIFFUSION, nullspace=True)  # essential DoFs present
    m, d, op = _case(2, 2, ess=False)
    b = gpu(uniform(m.ndof, seed=1))
    with pytest.raises(SfemError):
        op.pcg(b, op=HELMHOLTZ, nullspace=True)  # not the diffusion operator
    with pytest.raises(SfemError):
        op.pcg(b, op=DIFFUSION, precond=7)
