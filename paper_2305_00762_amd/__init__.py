"""MI355X (gfx950) implementation of the MEG7 gradient-based reconstruction
hot path (Chamarthi, arXiv 2305.00762): the per-stage residual and SSP-RK3
update behind the C ABI of include/gbr.h.

Modules
  gbr       ctypes binding of libgbr.so (same names as the C entry points)
  solver    device buffers and SSP-RK3 steps over the C ABI
  problems  seeded synthetic initial data (no scheme arithmetic)
  build     compiles libgbr.so for gfx950
"""
__all__ = ["gbr", "solver", "problems", "build"]
