"""MI355X (gfx950) modified Born series Helmholtz solver with on-device domain decomposition.

The solver is the HIP library ``libmbs.so`` behind the C ABI in ``include/mbs.h``;
``paper_2410_02395_amd.mbs`` is its ctypes binding and ``paper_2410_02395_amd.serve``
the continuous-batching request scheduler built on it.
"""

__all__ = ["mbs"]
