"""Shifted COCG Green's-function solver for MI355X (gfx950).

The compute path is the HIP library ``libscocg.so`` behind the C ABI in
``include/scocg.h``; ``binding`` is its ctypes binding.  Nothing is imported
eagerly so that the build step can run without a built library.
"""
__all__ = ["binding", "build"]
