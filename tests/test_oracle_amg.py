"""Pins of the oracle's smoothed-aggregation multigrid (oracle/amg.py), the solver of the LOR
operator, against properties that make it a valid CG preconditioner and a solver of A_LOR:

* aggregation: every non-isolated row in exactly one aggregate, isolated rows (the
  identity rows of essential DoFs) in none, every aggregate joined by strong connections;
* for the pure-Neumann Poisson operator the smoothed prolongator reproduces the constants
  (its near null space) and the coarse operator keeps them in its null space;
* the V-cycle is a symmetric positive definite linear map (u^T M v = v^T M u, v^T M v > 0);
* a hierarchy with a single level solves exactly (the dense pseudo-inverse), also for the
  singular pure-Neumann operator on the orthogonal complement of the constants;
* as a stationary iteration on A_LOR the V-cycle contracts the error (spectral radius of
  I - M A below 0.6), and CG preconditioned by it solves A_LOR to 1e-10 in a few
  iterations, independently of the mesh size.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import Discretization, pcg
from oracle.amg import AMG, aggregate, strength
from oracle.lor import lor_matrix
from workloads import BoxMesh, uniform


def lor(ne, p, neumann=False, alpha=0.0):
    m = BoxMesh(ne, p)
    ess = np.zeros(m.ndof, dtype=np.uint8) if neumann else m.ess
    d = Discretization(m.elem_xyz, m.elem_dofs, ess, m.ndof, p, p + 2)
    return m, lor_matrix(d, alpha, 1.0)


def test_aggregation_partition_and_connectivity():
    m, A = lor(3, 3)
    agg, nagg = aggregate(A, 0.02)
    ess = m.ess.astype(bool)
    assert np.all(agg[ess] == -1) and np.all(agg[~ess] >= 0)
    assert set(np.unique(agg[~ess])) == set(range(nagg))
    S = strength(A, 0.02)
    for a in range(nagg):  # each aggregate is connected through strong links
        members = np.nonzero(agg == a)[0]
        sub = S[members][:, members]
        ncomp, _ = sp.csgraph.connected_components(sub + sub.T, directed=False)
        assert ncomp == 1, a


def test_vcycle_is_symmetric_positive_definite():
    _, A = lor(3, 4)
    amg = AMG(A)
    assert amg.levels >= 2
    u, v = uniform(A.shape[0], seed=1), uniform(A.shape[0], seed=2)
    Mu, Mv = amg.vcycle(u), amg.vcycle(v)
    assert abs(u @ Mv - v @ Mu) <= 1e-12 * abs(u @ Mv)
    for s in range(3, 8):
        w = uniform(A.shape[0], seed=s)
        assert w @ amg.vcycle(w) > 0


@pytest.mark.parametrize("neumann", [False, True])
def test_single_level_is_an_exact_solve(neumann):
    _, A = lor(2, 2, neumann=neumann)
    amg = AMG(A, coarse_size=A.shape[0])
    assert amg.levels == 1
    b = uniform(A.shape[0], seed=3)
    if neumann:
        b = b - b.mean()
    x = amg.vcycle(b)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_vcycle_contracts_the_error():
    _, A = lor(4, 3)
    amg = AMG(A)
    rng = np.random.default_rng(5)
    e = rng.standard_normal(A.shape[0])
    rates = []
    for _ in range(8):  # error propagation e <- (I - M A) e
        e_new = e - amg.vcycle(A @ e)
        rates.append(np.linalg.norm(e_new) / np.linalg.norm(e))
        e = e_new
    assert rates[-1] < 0.6, rates


@pytest.mark.parametrize("ne", [2, 4, 6])
def test_cg_on_lor_with_vcycle_is_h_independent(ne):
    _, A = lor(ne, 3)
    amg = AMG(A)
    b = uniform(A.shape[0], seed=7)
    x, it, rr = pcg(lambda v: A @ v, b, None, rtol=1e-10, precond=amg.vcycle)
    assert rr <= 1e-10 and it <= 16, it


def test_prolongator_reproduces_the_constants():
    """For the pure-Neumann Poisson LOR operator (K 1 = 0) the smoothed prolongator maps the
    coarse constant to the fine constant: P 1 = (I - omega D^-1 K) P0 1 = 1."""
    _, A = lor(3, 3, neumann=True)
    amg = AMG(A)
    P = amg.P[0]
    assert np.abs(P @ np.ones(P.shape[1]) - 1.0).max() <= 1e-12
    # and the coarse operator keeps the constants in its null space
    Ac = amg.A[1]
    assert np.abs(Ac @ np.ones(Ac.shape[0])).max() <= 1e-12 * abs(Ac).max()
