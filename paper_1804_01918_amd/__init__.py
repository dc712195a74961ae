"""D2Q37 Lattice Boltzmann step on AMD Instinct MI355X (gfx950).

The compute path is the native library ``libd2q37`` (hand-written HIP
kernels behind a C ABI declared in ``include/lb.h``); ``lb`` is its thin
ctypes binding. Importing this package loads nothing native: the library is
opened on first use by ``paper_1804_01918_amd.lb``.
"""
__all__ = ["inputs", "lb"]
