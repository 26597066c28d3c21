"""MI355X-native temporally blocked 3D 7-point Jacobi (Wittmann et al. 2010).

Thin Python binding over the C-ABI library ``libjacobi.so`` (declared in
``include/jacobi.h``).  Every step of the solver runs in the library's HIP
kernels; this package only marshals arguments and uses PyTorch for device
memory and streams.  There is no CPU fallback: importing the package on a
machine where ``libjacobi.so`` is missing raises ``ImportError``.
"""

from ._lib import lib, LIB_PATH, JacobiError, check  # noqa: F401
from .solver import Jacobi, probe_copy, probe_update, tile_supported  # noqa: F401
from .batch import JacobiBatch  # noqa: F401
from .guess import GuessNet, init_params, param_count  # noqa: F401

__all__ = ["Jacobi", "JacobiBatch", "GuessNet", "param_count", "JacobiError", "lib", "LIB_PATH", "probe_copy",
           "probe_update", "tile_supported"]
