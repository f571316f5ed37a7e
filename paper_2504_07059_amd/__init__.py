"""MI355X (gfx950) implementation of the EVD multicomponent lattice Boltzmann
method with forcing (arXiv 2504.07059): a HIP library (liblbm_mc.so, C ABI in
include/lbm_mc.h) and its thin Python binding.

Importing the binding loads the library and fails loudly if it is not built.
"""
__all__ = ["lbm", "build"]
