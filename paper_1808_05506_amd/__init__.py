"""MI355X (gfx950) Dirac operators on blocks of right-hand sides.

Staggered, Wilson and Brillouin Dirac matrices times a block of N_v vectors
(S. Duerr, LATTICE 2018), their adjoints, the link gradient, the Brillouin
off-axis links and a mixed-precision solver, as hand-written HIP kernels
behind a C ABI (``include/dslash.h``).  This package is the thin ctypes
binding; importing ``paper_1808_05506_amd.dslash`` loads the library and fails
loudly if it has not been built.
"""
__version__ = "0.1.0"
