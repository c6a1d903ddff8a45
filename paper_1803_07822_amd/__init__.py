"""Curved-space D3Q19 lattice Boltzmann on MI355X (gfx950).

The solver lives in the HIP library ``csrc/`` builds (``liblbm.so``) and is
reached through ``paper_1803_07822_amd.lbm`` (ctypes binding of the C-ABI in
``include/lbm.h``).  Importing the package itself loads nothing, so that the
seeded input generators in ``synth`` stay usable on a machine without the
library; importing ``lbm`` fails loudly when the library is missing.
"""

__all__ = ["lbm", "synth"]
