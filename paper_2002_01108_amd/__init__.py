"""MI355X (gfx950) all-at-once heat solver with the block epsilon-circulant
preconditioner of Lin & Ng (arXiv 2002.01108).

The compute path is the HIP library libaao.so (C ABI: include/aao.h); this
package holds its sources (csrc/), the build script and a thin ctypes binding.
"""
from .binding import Solver, AaoError, load  # noqa: F401
