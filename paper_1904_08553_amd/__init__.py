"""MI355X-native Delta-screening incremental dynamic community detection.

The method (Zarayeneh & Kalyanaraman, arXiv 1904.08553) runs in hand-written
HIP kernels for gfx950 behind the C ABI of include/dc.h; ``dc`` is its
ctypes binding and ``workloads`` draws the seeded synthetic inputs.
"""
from . import dc, workloads  # noqa: F401
from .dc import DynamicCommunities, DCError  # noqa: F401
