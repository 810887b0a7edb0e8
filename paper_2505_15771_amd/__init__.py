"""MI355X-native HHO elasto-acoustic explicit Runge-Kutta engine (arXiv 2505.15771).

The compute path is libhho.so (hand-written HIP for gfx950 behind the C ABI of
include/hho.h); this package only marshals arguments to it.
"""
from .hho import Batch, Engine, HHOError, Inspect, SdirkEngine, Unstable, load_library  # noqa: F401
