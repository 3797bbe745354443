"""Maximum-likelihood shift-and-stack trajectory search on MI355X (gfx950).

The search itself lives in the HIP library libkbmi.so (C ABI in
include/kbmi.h); `lib` is its thin ctypes binding and `synth` draws seeded
synthetic inputs.  Importing the package loads nothing; the library is loaded
on first use and a missing build raises ImportError.
"""
__all__ = ["lib", "synth", "build"]
