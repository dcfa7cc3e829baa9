"""MI355X (gfx950) implementation of one time step of differentiable cosmological
hydrodynamics (Horowitz & Lukic, arXiv:2502.02294) and its reverse-mode pass.

The compute path is libdiffhydro.so (HIP kernels behind the C ABI of include/diffhydro.h);
this package only marshals arguments.  Importing it loads the library and fails if it is
not built."""

from ._lib import lib as _load

_load()

from .sim import Sim, conservation_noalloc, default_config, default_params  # noqa: E402
from .autograd import DiffHydroFn  # noqa: E402
from .mlp import Mlp  # noqa: E402

__all__ = ["Sim", "conservation_noalloc", "default_config", "default_params", "DiffHydroFn"]
