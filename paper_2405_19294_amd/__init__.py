"""MI355X (gfx950) Wilson-Dirac operator and CG for fermions in higher representations of SU(N).

The compute path is the HIP library libhrw.so (C ABI in include/hrw.h); this
package holds its sources (csrc/), the build script and the ctypes binding.
"""

from . import hrw  # noqa: F401

__all__ = ["hrw"]
