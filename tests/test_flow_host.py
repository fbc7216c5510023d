"""Host logic of the projection stepper (no GPU): the BDF/EXT weights the library derives
from their exactness conditions (sfem_bdf_ext_weights, a host computation behind the C
ABI) equal the oracle's table."""
import numpy as np
import pytest


@pytest.mark.parametrize("k", [1, 2, 3])
def test_bdf_ext_weights_match_the_oracle(k):
    from oracle import bdf_ext
    from paper_1910_03032_amd.flow import bdf_ext_weights
    b, a = bdf_ext_weights(k)
    bo, ao = bdf_ext(k)
    assert np.allclose(b, bo, rtol=0, atol=1e-14) and np.allclose(a, ao, rtol=0, atol=1e-14)


def test_bad_order():
    from paper_1910_03032_amd.flow import bdf_ext_weights
    with pytest.raises(ValueError):
        bdf_ext_weights(4)


def test_bdf_ext_weights_c_abi_rejects_bad_arguments():
    import ctypes as C
    from paper_1910_03032_amd import _lib
    lib = _lib.load()
    b, a = (C.c_double * 5)(), (C.c_double * 4)()
    assert lib.sfem_bdf_ext_weights(0, b, a) == -1
    assert lib.sfem_bdf_ext_weights(4, b, a) == -1
    assert lib.sfem_bdf_ext_weights(2, None, a) == -1
