"""MI355X-native modal discontinuous-Galerkin Euler solver (arXiv 1602.09079).

The compute path is the C-ABI library ``libdgmi.so`` (hand-written HIP kernels
for gfx950); this package only marshals arguments to it.  Importing the package
does not load the library: ``paper_1602_09079_amd.dg`` does, and raises if it
has not been built.
"""
