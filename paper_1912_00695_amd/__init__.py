"""MI355X-native acoustic finite-difference wave propagation.

Submodules:
  wave    -- ctypes binding of the HIP library (libwave.so) behind include/wave.h
  inputs  -- seeded synthetic velocity models, wavelets and acquisition geometry
  autograd -- torch.autograd.Function wrapper (velocity and wavelet gradients)

Importing the package loads nothing; the binding loads libwave.so on first use
and raises if it is missing.
"""
__all__ = ["wave", "inputs"]
