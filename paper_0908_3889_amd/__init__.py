"""Batched post-Newtonian binary-black-hole inspiral integrator for MI355X
(gfx950).

Submodules (imported on demand, so that the input generator works without
torch or a GPU):
  population  seeded synthetic initial data (no method arithmetic)
  api         torch binding of the C interface (include/pn.h)
  build       hipcc build of libpn.so
"""
__version__ = "0.1"
