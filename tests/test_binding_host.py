"""Argument checks of the Python binding that run before any library call: arrays whose
sizes differ from what sfem_setup and sfem_pcg read are rejected on the host."""
import numpy as np
import pytest

from paper_1910_03032_amd import Operator, check_mesh_shapes, check_solve_shapes
from workloads import BoxMesh


def test_mesh_shapes_accepted_and_rejected():
    m = BoxMesh(2, 2)
    assert check_mesh_shapes(m.elem_xyz.shape, m.elem_dofs.shape, m.ndof, 2, m.ess.shape) == m.nelem
    assert check_mesh_shapes(m.elem_xyz.shape, (m.elem_dofs.size,), m.ndof, 2) == m.nelem
    with pytest.raises(ValueError, match="elem_dofs"):
        check_mesh_shapes(m.elem_xyz.shape, m.elem_dofs.shape, m.ndof, 3)      # map of order 2
    with pytest.raises(ValueError, match="elem_dofs"):
        check_mesh_shapes(m.elem_xyz[:-1].shape, m.elem_dofs.shape, m.ndof, 2)  # one element short
    with pytest.raises(ValueError, match="elem_xyz"):
        check_mesh_shapes((m.nelem, 4, 3), m.elem_dofs.shape, m.ndof, 2)
    with pytest.raises(ValueError, match="ess"):
        check_mesh_shapes(m.elem_xyz.shape, m.elem_dofs.shape, m.ndof, 2, (m.ndof - 1,))
    assert check_mesh_shapes((0,), (0,), 0, 2) == 0


def test_operator_rejects_bad_sizes_before_loading_the_library():
    m = BoxMesh(2, 2)
    with pytest.raises(ValueError):
        Operator(m.elem_xyz, m.elem_dofs[:, :8], m.ndof, 2, ess=m.ess)
    with pytest.raises(ValueError):
        Operator(m.elem_xyz, m.elem_dofs, m.ndof, 2, ess=m.ess[:-1])


def test_solve_shapes():
    check_solve_shapes((10,), None, 10)
    check_solve_shapes((3, 10), (3, 10), 10)
    with pytest.raises(ValueError, match="x must have"):
        check_solve_shapes((3, 10), (10,), 10)   # the solve would write 3 * 10 values into x
    with pytest.raises(ValueError, match="x must have"):
        check_solve_shapes((10,), (2, 10), 10)
    with pytest.raises(ValueError, match="b must have"):
        check_solve_shapes((2, 3, 10), None, 10)
    with pytest.raises(ValueError, match="b must have"):
        check_solve_shapes((9,), None, 10)
    assert np.prod((3, 10)) == 30
