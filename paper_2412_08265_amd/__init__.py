"""MI355X-native IFU datacube forward model (hand-written HIP kernels for gfx950 behind a C ABI).

Importing the package loads nothing native; `paper_2412_08265_amd.ops` loads the HIP library on
first use and raises if it is missing.
"""
__version__ = "0.1.0"
