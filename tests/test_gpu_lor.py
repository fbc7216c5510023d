"""The LOR preconditioner of Section 5.2 on the GPU (through the C ABI) against the oracle:
the LOR matrix apply and one multigrid V-cycle (same hierarchy: level sizes equal the
oracle's), CG preconditioned by the V-cycle (iteration counts of the oracle's CG with its
V-cycle, solutions against direct solves), iteration counts bounded in h and growing slowly
in p, the pure-Neumann Poisson problem, and the 32^3 p = 4 pressure-Poisson size."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from gpu_common import gpu, host, rel, say
from oracle import Discretization, pcg as oracle_pcg
from oracle.amg import AMG
from oracle.lor import lor_matrix
from workloads import BoxMesh, FanMesh, nu_uniform, rhs_uniform, uniform

pytestmark = pytest.mark.gpu

THETA, COARSE, MAXLEV, NU = 0.02, 200, 12, 1


def sliced_storage(M):
    """The library's storage rule: sliced ELL (64-row slices) for at least 16384 rows of at
    most 48 entries on average that pad by at most half, CSR otherwise."""
    rl = np.diff(M.indptr)
    n = len(rl)
    ns = (n + 63) // 64
    padded = int(np.pad(rl, (0, ns * 64 - n)).reshape(ns, 64).max(axis=1).sum()) * 64
    return n >= 16384 and M.nnz <= 48 * n and 2 * padded <= 3 * M.nnz


def pattern_slices(M):
    """The library's pattern rule: slices of a square matrix whose rows' column offsets
    (col - row) number at most 1/8 more than the slice's longest row."""
    n = M.shape[0]
    if M.shape[1] != n:
        return 0
    rl = np.diff(M.indptr)
    offs = M.indices - np.repeat(np.arange(n), rl)
    count = 0
    for s in range((n + 63) // 64):
        a, b = M.indptr[s * 64], M.indptr[min(n, (s + 1) * 64)]
        ln = int(rl[s * 64:(s + 1) * 64].max())
        count += ln > 0 and len(np.unique(offs[a:b])) <= ln + ln // 8
    return count


def expected_sliced(amg):
    L = len(amg.A)
    flags = []
    for l in range(L):
        f = 0
        if l + 1 < L or l == 0:
            f |= 1 if sliced_storage(amg.A[l]) else 0
            f |= 8 if (f & 1) and pattern_slices(amg.A[l]) > 0 else 0
        if l + 1 < L:
            f |= 2 if sliced_storage(amg.P[l]) else 0
            f |= 4 if sliced_storage(amg.P[l].T.tocsr()) else 0
        flags.append(f)
    return flags


def setup(m, p, ess, alpha, beta, nu=None):
    from paper_1910_03032_amd import Operator
    d = Discretization(m.elem_xyz, m.elem_dofs, ess, m.ndof, p, p + 2)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=ess)
    op.set_coeffs(alpha, beta, None if nu is None else gpu(nu))
    return d, op


CASES = {"poisson_3e_p4": (3, 4), "helmholtz_nu_3e_p3": (3, 3), "neumann_3e_p5": (3, 5),
         "poisson_8e_p4": (8, 4), "helmholtz_nu_7e_p4": (7, 4), "neumann_6e_p5": (6, 5)}


@pytest.mark.parametrize("case", ["poisson_3e_p4", "helmholtz_nu_3e_p3", "neumann_3e_p5", "fan_p3",
                                  "poisson_8e_p4", "helmholtz_nu_7e_p4", "neumann_6e_p5"])
def test_lor_apply_and_vcycle_vs_oracle(case):
    """The small meshes keep every matrix in CSR; from 16384 rows (8^3 and 7^3 at p = 4, 6^3
    at p = 5) the finest operator is in sliced ELL with shared column-offset patterns (the
    box meshes' lexicographic numbering), and the prolongator where its padding stays
    within half (the reported storage matches the rules applied to the oracle's
    hierarchy)."""
    from paper_1910_03032_amd import DIFFUSION, HELMHOLTZ
    if case == "fan_p3":
        m, p = FanMesh(3), 3
        ess, opk, alpha, beta, nu = m.ess, HELMHOLTZ, 1.0, 1.0, None
    else:
        ne, p = CASES[case]
        m = BoxMesh(ne, p)
        ess = np.zeros(m.ndof, dtype=np.uint8) if case.startswith("neumann") else m.ess
        opk = HELMHOLTZ if case.startswith("helmholtz") else DIFFUSION
        alpha, beta = (1e3, 1.0) if opk == HELMHOLTZ else (0.0, 1.0)
        nu = nu_uniform(m.nelem, p + 2, seed=2) if opk == HELMHOLTZ else None
    say(f"[lor] {case} ndof={m.ndof}")
    d, op = setup(m, p, ess, alpha, beta, nu)
    info = op.lor_setup(opk)
    L = lor_matrix(d, alpha, beta, nu)
    amg = AMG(L, theta=THETA, coarse_size=COARSE, max_levels=MAXLEV, nu=NU)
    say(f"  levels {info['rows']} (oracle {[a.shape[0] for a in amg.A]}), setup {info['setup_ms']:.1f} ms")
    assert info["rows"] == [a.shape[0] for a in amg.A]
    say(f"  storage per level (bit 0 operator, 1 prolongator, 2 restriction sliced, 3 patterns): {info['sliced']}")
    assert info["sliced"] == expected_sliced(amg)
    assert (info["sliced"][0] & 9) == (9 if m.ndof >= 16384 else 0)
    x = uniform(m.ndof, seed=5)
    assert rel(host(op.lor_apply(gpu(x), opk)), L @ x) <= 1e-13
    b = uniform(m.ndof, seed=6)
    if not ess.any():
        b = b - b.mean()
    z = host(op.lor_vcycle(gpu(b), opk))
    zo = amg.vcycle(b)
    # the FP32 V-cycle: every product rounds to u = 2^-24 = 6e-8 with up to ~100 terms per
    # row and a few products in sequence per level, so it stays within 1e-4 (~1700 u) of
    # the FP64 one
    from paper_1910_03032_amd import F32
    z32 = host(op.lor_vcycle(gpu(b), opk, prec=F32))
    say(f"  v-cycle vs oracle {rel(z, zo):.2e}, FP32 v-cycle vs oracle {rel(z32, zo):.2e}")
    assert rel(z, zo) <= 1e-11
    assert rel(z32, zo) <= 1e-4
    op.close()


@pytest.mark.parametrize("case", ["poisson_3e_p3", "helmholtz_nu_3e_p4", "neumann_4e_p3"])
def test_lor_pcg_vs_oracle_and_direct(case):
    from paper_1910_03032_amd import DIFFUSION, HELMHOLTZ, PRECOND_LOR
    ne, p = {"poisson_3e_p3": (3, 3), "helmholtz_nu_3e_p4": (3, 4), "neumann_4e_p3": (4, 3)}[case]
    m = BoxMesh(ne, p)
    neumann = case.startswith("neumann")
    ess = np.zeros(m.ndof, dtype=np.uint8) if neumann else m.ess
    opk = HELMHOLTZ if case.startswith("helmholtz") else DIFFUSION
    alpha, beta = (1e3, 1.0) if opk == HELMHOLTZ else (0.0, 1.0)
    nu = nu_uniform(m.nelem, p + 2, seed=2) if opk == HELMHOLTZ else None
    say(f"[lor] pcg {case} ndof={m.ndof}")
    d, op = setup(m, p, ess, alpha, beta, nu)
    b = rhs_uniform(m, seed=1)[0] if not neumann else uniform(m.ndof, seed=1)
    if neumann:
        b = b - b.mean()
    x, res = op.pcg(gpu(b), op=opk, rtol=1e-10, precond=PRECOND_LOR, nullspace=neumann)
    assert res.converged and res.true_rel_res[0] <= 1e-10
    # the FP32 V-cycle inside FP64 CG: the same solution, at most 2 more iterations
    from paper_1910_03032_amd import PRECOND_LOR32
    x32, res32 = op.pcg(gpu(b), op=opk, rtol=1e-10, precond=PRECOND_LOR32, nullspace=neumann)
    say(f"  FP64 v-cycle {res.iters[0]} iterations, FP32 v-cycle {res32.iters[0]}")
    assert res32.converged and res32.true_rel_res[0] <= 1e-10
    assert res32.iters[0] <= res.iters[0] + 2
    amg = AMG(lor_matrix(d, alpha, beta, nu), theta=THETA, coarse_size=COARSE, max_levels=MAXLEV, nu=NU)
    _, it_o, _ = oracle_pcg(lambda v: d.apply(v, alpha, beta, nu), b, None, rtol=1e-10,
                            precond=amg.vcycle, nullspace=neumann)
    say(f"  iterations gpu {res.iters[0]} oracle {it_o}")
    assert abs(res.iters[0] - it_o) <= 2
    A = d.assemble(alpha, beta, nu)
    if neumann:  # bordered system [K m1; m1^T 0]: K x = b with int x = m1^T x = 0
        import scipy.sparse as sp
        m1 = d.apply(np.ones(m.ndof), 1.0, 0.0).reshape(-1, 1)
        Kb = sp.bmat([[A, sp.csr_matrix(m1)], [sp.csr_matrix(m1.T), None]]).tocsc()
        xd = spla.spsolve(Kb, np.concatenate([b, [0.0]]))[:-1]
    else:
        xd = spla.spsolve(A.tocsc(), b)
    assert rel(host(x), xd) <= 1e-8
    assert rel(host(x32), xd) <= 1e-8
    op.close()


def test_lor_iterations_bounded_in_h_and_p():
    """CG with the LOR V-cycle on the Poisson problem to 1e-10: at most 40 iterations on
    2^3..8^3 meshes at p = 3 (Jacobi 23, 59, 118) and at most 65 for p = 2..7 on 3^3
    (Jacobi 21, 93, 143: the V-cycle with Jacobi smoothing approximates the LOR solve less
    well as the sub-elements' aspect ratios grow with p; an exact LOR solve takes 26, 37,
    43)."""
    from paper_1910_03032_amd import DIFFUSION, PRECOND_LOR
    its = {}
    for ne, p in [(2, 3), (4, 3), (8, 3), (3, 2), (3, 5), (3, 7)]:
        m = BoxMesh(ne, p)
        d, op = setup(m, p, m.ess, 0.0, 1.0)
        b = gpu(rhs_uniform(m, seed=1)[0])
        _, r = op.pcg(b, op=DIFFUSION, rtol=1e-10, precond=PRECOND_LOR)
        _, rj = op.pcg(b, op=DIFFUSION, rtol=1e-10)
        assert r.converged and rj.converged
        its[(ne, p)] = (r.iters[0], rj.iters[0])
        op.close()
    say(f"[lor] iterations (lor, jacobi): {its}")
    assert max(its[(ne, 3)][0] for ne in (2, 4, 8)) <= 40
    assert max(its[(3, p)][0] for p in (2, 5, 7)) <= 65
    assert its[(8, 3)][1] > 2 * its[(8, 3)][0]


def test_lor_neumann_poisson_p4_32e():
    """The projection step's pressure-Poisson size (32^3 p = 4, 2.1M DoFs, pure Neumann):
    CG with the LOR V-cycle reaches 1e-10 in under 80 iterations (Jacobi: ~1100) and its
    solution agrees with the Jacobi-preconditioned one."""
    from paper_1910_03032_amd import DIFFUSION, PRECOND_LOR, PRECOND_LOR32
    m = BoxMesh(32, 4)
    free = np.zeros(m.ndof, dtype=np.uint8)
    from paper_1910_03032_amd import Operator
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, 4, ess=free)
    op.set_coeffs(0.0, 1.0, None)
    info = op.lor_setup(DIFFUSION)
    say(f"[lor] 32^3 p=4 levels {info['rows']} nnz {info['nnz']} setup {info['setup_ms']:.0f} ms")
    b = gpu(uniform(m.ndof, seed=1))
    x, r = op.pcg(b, op=DIFFUSION, rtol=1e-10, precond=PRECOND_LOR, nullspace=True, check_every=16)
    say(f"  lor {r}")
    assert r.converged and r.true_rel_res[0] <= 1e-10 and r.iters[0] < 80
    x32, r32 = op.pcg(b, op=DIFFUSION, rtol=1e-10, precond=PRECOND_LOR32, nullspace=True)
    say(f"  lor fp32 v-cycle {r32}")
    assert r32.converged and r32.true_rel_res[0] <= 1e-10 and r32.iters[0] <= r.iters[0] + 2
    xj, rj = op.pcg(b, op=DIFFUSION, rtol=1e-10, nullspace=True, check_every=16)
    say(f"  jacobi {rj}")
    assert rj.converged
    assert float((x - xj).norm() / xj.norm()) <= 1e-6
    assert float((x32 - xj).norm() / xj.norm()) <= 1e-6
    op.close()


def test_lor_error_paths_and_edge_cases():
    """Several nu fields and refinement mode are rejected; p = 1 (the refined mesh is the
    mesh), a nonzero initial guess and a zero right-hand side work."""
    from paper_1910_03032_amd import DIFFUSION, HELMHOLTZ, PRECOND_LOR, SfemError
    m = BoxMesh(3, 1)
    d, op = setup(m, 1, m.ess, 1e3, 1.0)
    b = rhs_uniform(m, seed=1)[0]
    x, r = op.pcg(gpu(b), op=HELMHOLTZ, rtol=1e-12, precond=PRECOND_LOR)
    assert r.converged and rel(host(x), spla.spsolve(d.assemble(1e3, 1.0).tocsc(), b)) <= 1e-9
    x0 = gpu(uniform(m.ndof, seed=9)) * 0.1
    x0[torch.as_tensor(m.ess.astype(bool), device="cuda")] = 0
    x1, r1 = op.pcg(gpu(b), x=x0, op=HELMHOLTZ, rtol=1e-12, precond=PRECOND_LOR)
    assert r1.converged and rel(host(x1), host(x)) <= 1e-9
    z, rz = op.pcg(gpu(np.zeros(m.ndof)), op=HELMHOLTZ, precond=PRECOND_LOR)
    assert rz.converged and float(z.abs().max()) == 0.0
    with pytest.raises(SfemError, match="SFEM_E_ARG"):
        op.pcg(gpu(b), op=HELMHOLTZ, precond=PRECOND_LOR, mode=1)
    from paper_1910_03032_amd import PRECOND_LOR32
    with pytest.raises(SfemError, match="SFEM_E_ARG"):
        op.pcg(gpu(b), op=HELMHOLTZ, precond=PRECOND_LOR32, mode=1)
    with pytest.raises(SfemError, match="SFEM_E_ARG"):
        op.lor_vcycle(gpu(b), HELMHOLTZ, prec=7)
    x32, r32 = op.pcg(gpu(b), op=HELMHOLTZ, rtol=1e-12, precond=PRECOND_LOR32)
    assert r32.converged and rel(host(x32), host(x)) <= 1e-9
    # an iteration cap: SFEM_NOCONV with exactly that many iterations and the last iterate
    # (the iteration queued after the stop changes nothing)
    assert r.iters[0] >= 3
    for cap in range(1, r.iters[0]):
        xc, rc = op.pcg(gpu(b), op=HELMHOLTZ, rtol=1e-12, precond=PRECOND_LOR, maxit=cap)
        assert rc.status == 1 and rc.iters[0] == cap, rc
        assert rc.rel_res[0] > 1e-12
    # the stop is seen one iteration late: the solution equals the one of a cap at the
    # iteration count the converged solve reported
    xk, rk = op.pcg(gpu(b), op=HELMHOLTZ, rtol=1e-12, precond=PRECOND_LOR, maxit=r.iters[0])
    assert rk.iters[0] == r.iters[0] and float((xk - x).abs().max()) == 0.0
    op.close()
    m2 = BoxMesh(2, 2)
    d2, op2 = setup(m2, 2, m2.ess, 1e3, 1.0)
    nus = np.stack([nu_uniform(m2.nelem, 4, seed=200 + k).reshape(-1) for k in range(2)])
    op2.set_coeffs(1e3, 1.0, gpu(nus))
    with pytest.raises(SfemError, match="SFEM_E_ARG"):
        op2.lor_setup(DIFFUSION)
    op2.close()
