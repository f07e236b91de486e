"""MI355X-native FMM-BEM hot path (arXiv 2103.01048, Bempp-Exafmm): the
kernel-independent FMM matrix-vector product (Laplace and Yukawa, single
plans, pairs sharing one tree, batches of molecules, monopole + dipole
sources, the adjoint), the boundary-element matvec of the direct and the two
derivative formulations and an FP64 GMRES, as hand-written HIP kernels for
gfx950 behind the C ABI in include/fmmbem.h.  This package is the thin Python
binding."""
from ._lib import FmmError, lib  # noqa: F401
from .fmm import FMMPlan, eval_pair, eval_pair_md  # noqa: F401
from .bem import BEMOperator, gmres  # noqa: F401,E402
from .autograd import FMMPotential, fmm_potential, solvation_style_energy  # noqa: F401,E402
from . import autotune  # noqa: F401,E402
