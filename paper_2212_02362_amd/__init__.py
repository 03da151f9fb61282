"""MI355X (gfx950) library for the smooth-boundary-method strong-form
elasticity solve of Agrawal & Runnels (arXiv:2212.02362): a matrix-free
geometric multigrid of div(psi C grad u) + b = 0 with node displacements and
cell indicators, in hand-written HIP kernels behind the C ABI of
include/sbm.h.  This package only marshals arguments to that library."""
from ._lib import DISPLACEMENT, TRACTION, SbmError, lib  # noqa: F401
from .solver import Solver  # noqa: F401
from .autograd import SBMSolve, compliance_grad  # noqa: F401
from .amr import AmrSolver  # noqa: F401
