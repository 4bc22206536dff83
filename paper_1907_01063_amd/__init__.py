"""MI355X (gfx950) Cholesky factor and reverse-mode adjoint for Gaussian-process
covariance matrices, behind the C ABI of ``include/gpchol.h``.

``gpchol`` is the ctypes binding; ``build`` compiles the HIP library in-tree.
"""
from . import gpchol  # noqa: F401
from .gpchol import GPC_FP64, GPC_MIXED, GpcError, Handle, default_handle  # noqa: F401
from .gp import GPMarginalLogLik, NotPositiveDefiniteError, gp_mll  # noqa: F401
