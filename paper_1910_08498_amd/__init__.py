"""MI355X-native Kaiser-Bessel Fourier-slice insertion (3D Fourier reconstruction).

The compute path is librecon.so (hand-written HIP kernels for gfx950 behind
the C ABI in include/recon.h); `recon` is its Python binding.  Importing the
binding requires the built library.
"""
__all__ = ["recon"]
