"""MI355X-native batched Levenberg-Marquardt fitting of parametric 2D galaxy
light profiles (the fitting problem of arXiv:2404.07780, "galmoss").

The compute path is the HIP library ``libgmfit.so`` (C ABI, gfx950 kernels);
``gmfit`` is its thin Python binding and ``synth`` draws seeded synthetic
inputs.  Importing the package loads nothing; the library is loaded on first
use of ``gmfit``.
"""
__all__ = ["gmfit", "synth"]
