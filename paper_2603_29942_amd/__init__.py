"""MI355X-native Brouwer-Zimmermann minimum-distance engine for codes over F_3 / F_7.

The enumeration runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/bz.h``; ``paper_2603_29942_amd.bz`` is its Python
binding.  Importing this package loads nothing: import ``bz`` explicitly.
"""
__version__ = "0.1.0"
