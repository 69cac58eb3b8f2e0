"""mcv: the per-iteration sample pass of the adaptive multi-channel VEGAS
integrator (VAMP, arXiv:1811.09711) as HIP kernels for MI355X (gfx950)
behind a C ABI (include/mcv.h).

``from paper_1811_09711_amd import mcv`` loads the binding (and torch, which
provides device memory and streams); the library itself is libmcv.so next to
this file.
"""
__all__ = ["mcv"]
