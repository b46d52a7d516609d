"""MI355X-native hot path of stochastic progressive photon mapping with a
multiple-threaded BVH and a float-only combined-MLCG generator.

The compute runs in libpm.so (hand-written HIP for gfx950 behind a C ABI,
include/pm.h); ``api`` is its ctypes binding and ``scenes`` the seeded input
generators.
"""
from . import scenes  # noqa: F401
