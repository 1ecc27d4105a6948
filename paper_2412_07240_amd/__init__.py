"""MI355X spectral point-mass filter: HIP library (libpmf.so) + thin binding.

The numerical work runs in hand-written HIP kernels for gfx950 behind the C ABI
of include/pmf.h; ``binding`` only marshals arguments.  Importing the binding
raises ImportError when the library has not been built.
"""
from . import binding
from .binding import *  # noqa: F401,F403
