"""Oracle of the algebraic multigrid V-cycle used as the solver of the LOR operator
(test infrastructure; FP64).

Section 5.2 preconditions A with a solver for the sparse LOR matrix A_LOR, which the
paper builds from multigrid with ILU smoothing inside an overlapping Schwarz method.
The library's solver is smoothed-aggregation algebraic multigrid instead (its setup on
the host, every V-cycle step on the GPU); this module is that algorithm written out with
scipy sparse matrices, step by step, for the parity tests.

Setup, level by level (A_0 = A_LOR, CSR with sorted column indices):
  1. isolated rows (no off-diagonal entry: the identity rows of essential DoFs) are
     left out of the coarse space;
  2. strong connections: j != i with |a_ij| >= theta sqrt(|a_ii a_jj|);
  3. aggregation in three passes over the rows in index order: (a) a row that is not
     isolated, not aggregated and whose strong neighbours are all unaggregated starts an
     aggregate with them; (b) each remaining non-isolated row joins the aggregate of its
     first strong neighbour (in column order) that pass (a) aggregated; (c) each row still
     left starts an aggregate with its unaggregated strong neighbours;
  4. tentative prolongator P0[i, agg(i)] = 1; smoothed P = (I - omega D^-1 A) P0 with
     omega = 4 / (3 rho), rho the spectral radius of D^-1 A estimated by `npower` power
     iterations from the vector v_i = 1 + (i mod 7) / 7;
  5. A_{l+1} = P^T A_l P; stop when A_{l+1} has at most `coarse_size` rows or after
     `max_levels` levels.
The coarsest level is solved with the pseudo-inverse of its dense matrix (eigenvalues
below 1e-12 of the largest dropped: the constants of a pure-Neumann problem).

V-cycle for A_l x = b (x_l = 0 at the start of every level): `nu` damped-Jacobi sweeps
x += omega_l D^-1 (b - A x) with omega_l = 4 / (3 rho_l), the residual restricted by P^T,
the coarse correction added through P, `nu` more sweeps (a symmetric preconditioner).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def strength(A, theta):
    """Boolean CSR pattern of the strong off-diagonal connections."""
    A = A.tocsr()
    d = np.abs(A.diagonal())
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    keep = (rows != cols) & (np.abs(A.data) >= theta * np.sqrt(d[rows] * d[cols]))
    return sp.csr_matrix((np.ones(int(keep.sum()), dtype=bool), (rows[keep], cols[keep])), shape=A.shape)


def aggregate(A, theta):
    """Aggregate index per row (-1: isolated row) and the number of aggregates."""
    A = A.tocsr()
    n = A.shape[0]
    offdiag = np.diff(A.indptr) - (A.diagonal() != 0).astype(np.int64)
    isolated = np.array([not np.any((A.indices[A.indptr[i]:A.indptr[i + 1]] != i)
                                    & (A.data[A.indptr[i]:A.indptr[i + 1]] != 0)) for i in range(n)])
    del offdiag
    S = strength(A, theta)
    agg = np.full(n, -1, dtype=np.int64)
    nagg = 0
    nbrs = [S.indices[S.indptr[i]:S.indptr[i + 1]] for i in range(n)]
    for i in range(n):  # pass (a)
        if isolated[i] or agg[i] >= 0:
            continue
        if np.all(agg[nbrs[i]] < 0):
            agg[i] = nagg
            agg[nbrs[i]] = nagg
            nagg += 1
    first = agg.copy()
    for i in range(n):  # pass (b)
        if isolated[i] or agg[i] >= 0:
            continue
        for j in nbrs[i]:
            if first[j] >= 0:
                agg[i] = first[j]
                break
    for i in range(n):  # pass (c)
        if isolated[i] or agg[i] >= 0:
            continue
        agg[i] = nagg
        for j in nbrs[i]:
            if agg[j] < 0:
                agg[j] = nagg
        nagg += 1
    return agg, nagg


def spectral_radius_dinv_a(A, npower=15):
    """Power-iteration estimate of rho(D^-1 A) from v_i = 1 + (i mod 7) / 7."""
    A = A.tocsr()
    dinv = 1.0 / A.diagonal()
    v = 1.0 + (np.arange(A.shape[0]) % 7) / 7.0
    rho = 0.0
    for _ in range(npower):
        w = dinv * (A @ v)
        rho = np.linalg.norm(w) / np.linalg.norm(v)
        v = w / np.linalg.norm(w)
    return rho


class AMG:
    """Smoothed-aggregation hierarchy of A (scipy sparse, SPD or SPSD)."""

    def __init__(self, A, theta=0.02, coarse_size=200, max_levels=12, nu=1, npower=15):
        self.A, self.P, self.rho = [], [], []
        self.nu = nu
        A = sp.csr_matrix(A)
        A.sort_indices()
        while True:
            rho = spectral_radius_dinv_a(A, npower)
            self.A.append(A)
            self.rho.append(rho)
            if A.shape[0] <= coarse_size or len(self.A) == max_levels:
                break
            agg, nagg = aggregate(A, theta)
            if nagg == 0 or nagg >= A.shape[0]:
                break
            rows = np.nonzero(agg >= 0)[0]
            P0 = sp.csr_matrix((np.ones(rows.size), (rows, agg[rows])), shape=(A.shape[0], nagg))
            omega = 4.0 / (3.0 * rho)
            P = (P0 - omega * sp.diags(1.0 / A.diagonal()) @ (A @ P0)).tocsr()
            P.sort_indices()
            self.P.append(P)
            A = (P.T @ A @ P).tocsr()
            A.sort_indices()
        C = self.A[-1].toarray()
        w, V = np.linalg.eigh(C)
        keep = w > 1e-12 * np.abs(w).max()
        self.coarse_inv = (V[:, keep] / w[keep]) @ V[:, keep].T

    @property
    def levels(self):
        return len(self.A)

    def vcycle(self, b, level=0):
        """One V-cycle for A_level x = b from x = 0."""
        A = self.A[level]
        if level == len(self.A) - 1:
            return self.coarse_inv @ b
        dinv = 1.0 / A.diagonal()
        om = 4.0 / (3.0 * self.rho[level])
        x = np.zeros_like(b)
        for _ in range(self.nu):
            x = x + om * dinv * (b - A @ x)
        r = b - A @ x
        xc = self.vcycle(self.P[level].T @ r, level + 1)
        x = x + self.P[level] @ xc
        for _ in range(self.nu):
            x = x + om * dinv * (b - A @ x)
        return x
