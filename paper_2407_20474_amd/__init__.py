"""MI355X-native enumeration of factorization sets Z(n; g_1..g_d).

The work runs in libzset.so (hand-written HIP for gfx950, C ABI in
include/zset.h); `zset` is its Python binding and `inputs` draws the seeded
synthetic workloads.
"""
from . import zset  # noqa: F401
