"""MI355X (gfx950) sparse D3Q19 lattice-Boltzmann update behind a C ABI.

* ``hlb``       ctypes binding of include/hlb.h (libhlb.so, HIP kernels)
* ``geometry``  seeded synthetic vessel geometries (inputs only)
* ``build``     in-tree build of libhlb.so
"""
from . import hlb  # noqa: F401

__all__ = ["hlb"]
