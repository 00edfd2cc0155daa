"""MI355X-native D3Q19 central-moment lattice Boltzmann library (arXiv 2010.01628).

The compute path is ``liblbm.so``: hand-written HIP kernels for gfx950 behind a
C ABI (``include/lbm.h``).  ``paper_2010_01628_amd.lbm`` is the thin ctypes
binding with the same entry-point names; ``inputs`` builds seeded synthetic
problem fields.  Importing this package does not load the GPU library; the
binding loads it on first use and raises if it is missing.
"""

__all__ = ["lbm", "inputs"]
