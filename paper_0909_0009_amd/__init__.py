"""MI355X-native local-f_NL CMB map generator (gfx950 HIP behind a C ABI).

Submodules are imported lazily: `inputs` (seeded synthetic inputs) needs only
numpy, `fnlsim` (the ctypes binding) needs torch and the built library.
"""
__all__ = ["inputs", "fnlsim", "build"]
