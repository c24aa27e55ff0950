"""Polynomial-filtered subspace extraction on MI355X (gfx950).

Python binding over the C-ABI library ``libpfx.so`` (declared in
``include/pf.h``).  The binding only marshals arguments; every step of an
extraction runs in the library's HIP kernels.
"""
