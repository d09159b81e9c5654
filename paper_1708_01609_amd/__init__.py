"""MI355X (gfx950) matched-filter hot path of butterfly filtering (arXiv:1708.01609).

The product is the C-ABI library libbfsearch.so (include/bfsearch.h); this
package holds its HIP sources (csrc/), the build step (build.py) and a thin
ctypes binding (bfsearch.py).  Import the binding explicitly:

    from paper_1708_01609_amd import bfsearch
"""

__all__ = ["bfsearch", "build"]
