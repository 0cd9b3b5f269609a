"""MI355X-native hybrid particle-field MD (hPF-MD) timestep.

The compute path is libhpf.so (HIP kernels for gfx950 behind the C ABI in
include/hpf.h); ``hpf`` is its Python binding and ``engine`` strings the
calls into a velocity-Verlet step. Importing the package loads the library
and fails if it has not been built.
"""
from . import hpf  # noqa: F401

hpf.lib()

from . import engine  # noqa: E402,F401

__all__ = ["hpf", "engine"]
