"""MI355X-native preconditioned FWI gradient (2D acoustic, 8th-order FD).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``libfwi.so``); this package holds its thin ctypes binding, the
``torch.autograd.Function`` for J(v) and the seeded synthetic-input
generators.  Importing the package does not load the library.
"""
__all__ = ["synthetic"]
