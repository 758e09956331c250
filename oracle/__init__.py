"""CPU FP64 oracle for the Openpipeflow pipe-flow time step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
implementation of what the time step computes, written from the method's
description (Willis, "The Openpipeflow Navier-Stokes solver", SoftwareX 2017):
the Fourier-Fourier-finite-difference discretisation of Eq. (1), 3/2
dealiasing, the pressure-Poisson / influence-matrix formulation and the
second-order predictor-corrector scheme of Section 2.  Only tests,
`__graft_entry__.smoke()` and the benchmark's CPU-baseline leg may import it;
the product (the HIP library and its binding) never does, and shares no code
with it.

Every linear solve here is a dense solve (numpy.linalg.solve): the definition
of the banded LU solves the method uses.  Transforms use numpy's FFT on the
3/2-padded grid, the definition of the dealiased pseudospectral product.
"""
from .grid import (  # noqa: F401
    radial_nodes, lagrange_derivative_weights, fd_matrices, quadrature_weights,
)
from .spectral import (  # noqa: F401
    to_physical, to_spectral, to_pm, from_pm, vorticity, nonlinear,
)
from .solver import Params, Oracle  # noqa: F401
