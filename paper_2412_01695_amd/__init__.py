"""mkpw: many-k plane-wave Hamiltonian application on AMD Instinct MI355X (gfx950).

The native library (``libmkpw.so``, built from ``csrc/``) exports the C-ABI
declared in ``include/mkpw.h``; ``paper_2412_01695_amd.mkpw`` is the thin
ctypes binding with the same names.  ``synth`` generates the seeded
synthetic inputs.  Importing this package does not load the native library.
"""
__all__ = ["synth"]
