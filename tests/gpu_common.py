"""Shared helpers of the GPU tests: one seeded mesh feeds both the oracle and the library."""
import sys

import numpy as np
import torch

from oracle import Discretization
from workloads import BoxMesh, nu_c2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def case(ne, p, seed=0, amp=0.1):
    from paper_1910_03032_amd import Operator
    m = BoxMesh(ne, p, amp=amp, seed=seed)
    d = Discretization(m.elem_xyz, m.elem_dofs, m.ess, m.ndof, p, p + 2)
    say(f"[case] ne={ne} p={p} nelem={m.nelem} ndof={m.ndof}")
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=m.ess)
    return m, d, op


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def nu_c2_gpu(op):
    xq = op.qpoint_coords()
    return nu_c2(xq[0], xq[1], xq[2])


def nu_c2_oracle(d):
    xq = d.qpoint_coords()
    return nu_c2(xq[..., 0], xq[..., 1], xq[..., 2])
