"""MI355X-native joint symbolic approximation (JABBA, arXiv 2401.00109).

Hand-written HIP kernels for gfx950 behind a C ABI (include/jabba.h); this
package is the Python binding (ctypes; PyTorch only for device memory and
streams) plus the seeded synthetic workload generators.
"""
from . import api  # noqa: F401
from ._lib import LIB_PATH, JabbaError, lib  # noqa: F401
from .api import *  # noqa: F401,F403

__version__ = "0.1.0"
