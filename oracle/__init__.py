"""CPU oracle for the sum-factorized Q_p operators and their solvers.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 reference that
the HIP library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path (the C-ABI
library and its Python binding) never does, and shares no code with it.

Contents:
  quadrature  Gauss-Legendre / Gauss-Lobatto-Legendre rules, Lagrange basis (Section 3.1)
  fem         dense element operators M, K(nu), alpha M + beta K(nu), their diagonal,
              load vector, adjoint-gradient integrand (Section 3, Section 3.1), the
              collocated (GLL-integrated) mass diagonal (Section 5.1)
  stokes      the Taylor-Hood gradient and divergence blocks and the constrained Stokes
              block operator (Section 3, eq. gradient, eq. divergence); the convection
              term N(u) (eq. nonlinear)
  flow        equal-order weak gradient, curl and divergence, BDF-k/EXT-k coefficients
              and the velocity-correction projection step (Section 4.2)
  solvers     diagonally preconditioned CG (optionally orthogonalized against the
              constants, or with a general preconditioner), FP32-inner iterative
              refinement, adjoint gradient, pure-Neumann Poisson with the mean-zero
              condition (Section 5, Section 5.3)
  lor         the low-order-refined operator A_LOR = alpha M_LOR + beta K_LOR on the
              GLL-refined mesh (Section 5.2)

Pins (tests/test_oracle_*.py) tie each part to closed forms and invariants;
nothing here is "parity unpinned".
"""
from .quadrature import gauss_legendre, gll, lagrange_values, lagrange_derivs, legendre_p  # noqa: F401
from .fem import Discretization, OP_MASS, OP_DIFFUSION, OP_HELMHOLTZ, op_coeffs  # noqa: F401
from .solvers import pcg, ir_pcg, adjoint_gradient, objective, neumann_poisson  # noqa: F401
from .stokes import StokesDiscretization, convection  # noqa: F401
from .flow import (weak_gradient, weak_curl, weak_divergence, bdf_ext,  # noqa: F401
                   ProjectionStepper)
