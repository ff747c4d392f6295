"""MI355X-native GEER: epsilon-approximate pairwise effective resistance
(Yang & Tang, SIGMOD 2023) with hand-written HIP kernels for gfx950.

``geer`` is the ctypes binding of the C ABI in ``include/geer.h``;
``inputs`` holds the seeded synthetic graph and query generators.
"""

__all__ = ["geer", "inputs"]
