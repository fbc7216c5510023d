"""The allocation-free apply (sfem_apply_noalloc, for callers that cannot allocate) through
the C ABI: its results equal sfem_apply's on two calls in a row, the second with a
smaller input (another context, fewer members, the other precision), while the shared
scratch still holds the first call's values; a call beyond the scratch size is rejected."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import gpu, say
from workloads import BoxMesh, normal, nu_uniform

pytestmark = pytest.mark.gpu


def _ctx(ne, p):
    from paper_1910_03032_amd import Operator
    m = BoxMesh(ne, p)
    op = Operator(m.elem_xyz, m.elem_dofs, m.ndof, p, ess=m.ess)
    op.set_coeffs(1e3, 1.0, gpu(nu_uniform(m.nelem, p + 2, seed=2)))
    return m, op


def _noalloc(op, x, prec):
    y = torch.full_like(x, float("nan"))
    nb = 1 if x.ndim == 1 else x.shape[0]
    op._sync_stream()
    st = op._lib.sfem_apply_noalloc(op._h, 2, prec, nb, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    return st, y


def test_noalloc_apply_equals_apply_twice_second_smaller():
    from paper_1910_03032_amd import F32, F64
    from paper_1910_03032_amd._lib import APPLY_NOALLOC_MAX_BYTES
    m1, op1 = _ctx(12, 4)
    say(f"[noalloc] first call: 12^3 p=4 ndof={m1.ndof} nbatch=3 fp64, "
        f"nentries={op1.info()['nentries']}")
    X1 = gpu(np.stack([normal(m1.ndof, seed=1 + k) for k in range(3)]))
    st, Y1 = _noalloc(op1, X1, F64)
    assert st == 0, op1._lib.sfem_last_error(op1._h)
    ref1 = op1.apply(X1)
    torch.cuda.synchronize()
    assert torch.equal(Y1, ref1)
    m2, op2 = _ctx(5, 3)
    say(f"[noalloc] second call: 5^3 p=3 ndof={m2.ndof} nbatch=1, fp64 then fp32")
    x2 = gpu(normal(m2.ndof, seed=7))
    st, y2 = _noalloc(op2, x2, F64)
    assert st == 0, op2._lib.sfem_last_error(op2._h)
    ref2 = op2.apply(x2)
    torch.cuda.synchronize()
    assert torch.equal(y2, ref2)
    x3 = x2.to(torch.float32)
    st, y3 = _noalloc(op2, x3, F32)
    assert st == 0
    assert torch.equal(y3, op2.apply(x3))
    # the first context again, one member, after the scratch held the second's values
    st, y4 = _noalloc(op1, X1[2].contiguous(), F64)
    assert st == 0 and torch.equal(y4, ref1[2])
    # beyond the scratch: rejected before any launch, y untouched
    nent = op1.info()["nentries"]
    nb = APPLY_NOALLOC_MAX_BYTES // (8 * nent) + 1
    Xb = gpu(np.zeros((nb, m1.ndof)))
    st, yb = _noalloc(op1, Xb, F64)
    assert st == -1 and b"scratch" in op1._lib.sfem_last_error(op1._h)
    assert torch.isnan(yb).all()
    op1.close()
    op2.close()
