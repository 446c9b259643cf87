"""MI355X (gfx950) 2-D shallow-water step: HIP kernels behind a C ABI, thin Python binding.

Importing the package loads nothing; ``paper_1711_04471_amd.sw2d`` loads the in-tree
``libsw2d.so`` on first use and raises if it is missing (there is no CPU fallback).
"""

__all__ = ["inputs", "sw2d"]
