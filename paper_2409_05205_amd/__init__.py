"""Rotation-free HE Conv/FC server path on MI355X (gfx950).

The compute lives in the HIP library libhe.so (C ABI in include/he.h); the
Python modules here only marshal arguments (he), run layer sequences (runtime)
and serve requests (serve).  Import of a submodule that calls the library
fails loudly when the library has not been built.
"""
__all__ = ["he"]
