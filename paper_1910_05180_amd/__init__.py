"""MI355X (gfx950) implementation of the explicit time step of the Sharp
Phase-Field Method (Fleck, Schleifer & Zimbrod, arXiv:1910.05180).

The step, the initial fields and the diagnostics reductions are HIP kernels in
libspfm.so behind the C ABI of include/spfm.h; ``spfm`` is its ctypes binding
and ``inputs`` draws the seeded synthetic workloads.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "spfm"]
