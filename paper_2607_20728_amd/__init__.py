"""MI355X (gfx950) library for plane-wave analytical BSE excited-state forces.

The compute lives in libbsex.so (C ABI in include/bsex.h); ``bsex`` is its
ctypes binding.  Importing the package does not load the library.
"""
__all__ = ["bsex", "build"]
