"""MI355X-native coarse-grid-projection (CGP) QG time step.

Hand-written gfx950 HIP kernels behind the C ABI of include/cgp.h
(libcgp.so, built in-tree by ``python -m paper_1308_3290_amd.build``), with a
thin torch binding in ``paper_1308_3290_amd.api``.  Importing this package
does not load the library; the first API call does, and fails loudly if it
is missing.
"""
__version__ = "0.1.0"
