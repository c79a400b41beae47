"""MI355X-native solver for the 3D Elder density-driven flow problem with uncertain
porosity and permeability (arXiv 1906.01632): Python binding of libedf.so.

The binding only marshals arguments; every step of the time integration runs in
the HIP kernels of the library.  Importing the package does not need a GPU;
creating a Problem does, and fails loudly if libedf.so has not been built.
"""
from ._binding import (EDFError, EXPORTS, PREC_F64, PREC_MIXED, PREC_MIXED_F16,  # noqa: F401
                       SAMPLE_LINEAR_FAIL,
                       SAMPLE_NEWTON_FAIL, SAMPLE_NONFINITE, SAMPLE_OK, Problem, create_problem,
                       default_options, load_library)

try:  # the autograd wrapper needs torch; the C-ABI binding does not
    from .autograd import ElderQoI, salt_mass  # noqa: F401
except ImportError:  # pragma: no cover
    pass
