"""MI355X (gfx950) implementation of the coupled semi-implicit LBM for Biot's
consolidation model (Lunowa & Wohlmuth, arXiv:2409.11382).

* ``problem``: problem descriptions and seeded synthetic workloads (inputs only).
* ``lbm``: ctypes binding of the HIP library ``libbiotlbm.so`` (C ABI in
  ``include/biotlbm.h``); imported lazily so that ``problem`` needs no GPU stack.
"""

__all__ = ["problem", "lbm"]
