"""MI355X (gfx950) implementation of the 18th-order hyperpower iteration for
outer generalized inverses (Pan, Soleymani, Zhao, arXiv 1604.07893).

All arithmetic runs in hand-written HIP kernels inside ``libhyperpower.so``,
reached through its C ABI (``include/hyperpower.h``). This package only
marshals arguments: ``inputs`` builds seeded synthetic matrices; ``hyperpower``
is the ctypes binding.
"""

__all__ = ["inputs"]
