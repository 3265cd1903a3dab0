"""MI355X-native ARRABIT block eigensolver (augmented Rayleigh-Ritz).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``libarr.so``); :mod:`paper_1507_06078_amd.arr` is its thin ctypes
binding.
"""
