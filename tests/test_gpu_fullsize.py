"""Full-size workloads in the configuration the benchmark times, checked where the
oracle can follow: sampled rows of the apply (the oracle evaluates single rows from
dense element matrices), true residuals of the solves recomputed by the library's FP64
operator and confirmed on sampled rows by the oracle, and central finite differences of
the adjoint gradient on 16 random directions."""
import numpy as np
import pytest
import torch

from gpu_common import case, gpu, host, say, nu_c2_gpu, nu_c2_oracle
from workloads import normal, rhs_uniform, nu_uniform

pytestmark = pytest.mark.gpu


def sampled_rows_check(m, d, op, alpha, beta, nu_o, nb=1, seed=42, nrows=24):
    rng = np.random.default_rng(seed)
    rows = np.concatenate([rng.integers(0, m.ndof, nrows), [0, m.ndof // 2, m.ndof - 1]])
    X = np.stack([normal(m.ndof, seed=1 + k) for k in range(nb)])
    Y = host(op.apply(gpu(X if nb > 1 else X[0]), op=2)).reshape(nb, -1)
    Y32 = host(op.apply(gpu(X if nb > 1 else X[0], torch.float32), op=2)).reshape(nb, -1)
    for k in range(nb):
        yo = d.apply_rows(rows, X[k], alpha, beta, nu_o)
        scale = np.abs(yo).max()
        e64 = np.abs(Y[k, rows] - yo).max() / scale
        e32 = np.abs(Y32[k, rows] - yo).max() / scale
        say(f"  member {k}: sampled-row rel err fp64 {e64:.2e} fp32 {e32:.2e}")
        assert e64 <= 1e-12 and e32 <= 1e-5
    return rows


def test_vector_helmholtz_p7_24e():
    """24^3, p = 7, 3 components (4.8M DoFs each): batched apply rows, IR vs FP64 solves."""
    m, d, op = case(24, 7)
    op.set_coeffs(1e3, 1.0, nu_c2_gpu(op))
    nu_o = nu_c2_oracle(d)
    sampled_rows_check(m, d, op, 1e3, 1.0, nu_o, nb=3)
    B = gpu(rhs_uniform(m, seed=1, nbatch=3))
    X64, r64 = op.pcg(B, rtol=1e-10, check_every=16)
    Xir, rir = op.pcg(B, rtol=1e-10, mode=1, check_every=16)
    say(f"  fp64 {r64}\n  ir {rir}")
    assert r64.converged and rir.converged
    assert max(rir.true_rel_res) <= 1e-10 and max(r64.true_rel_res) <= 1e-10
    diff = float((Xir - X64).norm() / X64.norm())
    say(f"  ||x_ir - x_64|| / ||x_64|| = {diff:.2e}")
    assert diff <= 1e-8
    # the oracle confirms the residual of the IR solution on sampled rows
    rows = np.random.default_rng(7).integers(0, m.ndof, 12)
    x = host(Xir[1])
    r = host(B[1])[rows] - d.apply_rows(rows, x, 1e3, 1.0, nu_o)
    assert np.abs(r).max() <= 1e-8 * np.abs(host(B[1])).max()


def test_large_p8_40e():
    """40^3, p = 8 (33M DoFs): apply rows and the FP32+IR solve to 1e-10."""
    m, d, op = case(40, 8)
    op.set_coeffs(1e3, 1.0, nu_c2_gpu(op))
    nu_o = nu_c2_oracle(d)
    sampled_rows_check(m, d, op, 1e3, 1.0, nu_o, nrows=12)
    b = gpu(rhs_uniform(m, seed=1)[0])
    x, res = op.pcg(b, rtol=1e-10, mode=1, check_every=16)
    say(f"  ir {res}")
    assert res.converged and res.true_rel_res[0] <= 1e-10
    rows = np.random.default_rng(9).integers(0, m.ndof, 8)
    r = host(b)[rows] - d.apply_rows(rows, host(x), 1e3, 1.0, nu_o)
    assert np.abs(r).max() <= 1e-8


def test_adjoint_p5_20e_central_differences_16_directions():
    """20^3, p = 5 (1M DoFs), nu ~ U(0.5, 2): <dJ/dnu, d> vs (J(nu + eps d) - J(nu - eps d)) / 2 eps,
    eps = 1e-6, 16 directions, forward solves to 1e-13."""
    from paper_1910_03032_amd.autograd import helmholtz_solve
    m, d, op = case(20, 5)
    alpha, beta = 1e3, 1.0
    q3 = d.nqp
    ess = torch.as_tensor(m.ess.astype(bool), device="cuda")
    b = gpu(rhs_uniform(m, seed=1)[0])
    op.set_coeffs(alpha, beta, gpu(nu_uniform(m.nelem, d.q, seed=3)))
    u_t, _ = op.pcg(b, rtol=1e-13)
    nu = gpu(nu_uniform(m.nelem, d.q, seed=2)).requires_grad_(True)

    def J(nu_):
        u = helmholtz_solve(nu_, b, op, alpha=alpha, beta=beta, rtol=1e-13)
        r = torch.where(ess, torch.zeros_like(u), u - u_t)
        return 0.5 * (r * r).sum()

    J(nu).backward()
    g = nu.grad.detach().clone()
    eps = 1e-6
    worst = 0.0
    for k in range(16):
        dirn = gpu(np.random.default_rng(100 + k).uniform(-1, 1, (m.nelem, q3)))
        with torch.no_grad():
            fd = (J(nu + eps * dirn) - J(nu - eps * dirn)).item() / (2 * eps)
        ad = float((g * dirn).sum())
        worst = max(worst, abs(fd - ad) / abs(ad))
        assert abs(fd - ad) <= 1e-5 * abs(ad), (k, fd, ad)
    say(f"  worst relative FD mismatch over 16 directions: {worst:.2e}")


def test_helmholtz_p4_32e_solves_checked_by_oracle_rows():
    """32^3, p = 4 (2.1M DoFs), b ~ U(-1, 1): the FP64 PCG and the FP32+IR solutions to a
    relative residual of 1e-10 (the benchmark's solves); the residual b - A x on sampled
    rows, with A evaluated by the oracle, is within what the solve tolerance allows for
    one entry (|r_i| <= ||r||_2 <= 1e-10 ||b||_2) plus the rounding of two FP64
    evaluations of A x (1e-12 of the largest |A x| entry), and the two solutions agree to
    the solve tolerance times the conditioning."""
    m, d, op = case(32, 4)
    op.set_coeffs(1e3, 1.0, nu_c2_gpu(op))
    nu_o = nu_c2_oracle(d)
    b = gpu(rhs_uniform(m, seed=1)[0])
    x64, r64 = op.pcg(b, rtol=1e-10, check_every=16)
    xir, rir = op.pcg(b, rtol=1e-10, mode=1, check_every=16)
    say(f"  fp64 {r64}\n  ir {rir}")
    assert r64.converged and rir.converged
    assert r64.true_rel_res[0] <= 1e-10 and rir.true_rel_res[0] <= 1e-10
    rng = np.random.default_rng(11)
    rows = np.concatenate([rng.integers(0, m.ndof, 24), [0, m.ndof // 2, m.ndof - 1]])
    bh = host(b)
    for name, x in (("fp64", x64), ("ir", xir)):
        ax = d.apply_rows(rows, host(x), 1e3, 1.0, nu_o)
        r = bh[rows] - ax
        bound = 1e-10 * np.linalg.norm(bh) + 1e-12 * np.abs(ax).max()
        say(f"  {name}: max sampled-row residual {np.abs(r).max():.2e} (bound {bound:.2e})")
        assert np.abs(r).max() <= bound
    assert float((xir - x64).norm() / x64.norm()) <= 1e-8
