"""libpsl: MI355X (gfx950) hot path of the two-phase PSL search (arXiv 2107.09801).

The compute lives in HIP kernels behind the C-ABI of include/psl.h; this
package holds the kernels' sources (csrc/), the build step (build.py) and a
thin ctypes binding (libpsl.py).
"""
__all__ = ["libpsl", "build"]
