"""MI355X-native FFT-preconditioned conjugate-gradient solver for the
periodic linear-elastic cell problem on voxel grids.

Submodules:
  microstructures  seeded synthetic material fields (inputs only)
  binding          ctypes binding of the HIP C-ABI library (libcellfft.so)
  autograd         torch.autograd.Function around the effective stiffness

Importing the package loads nothing native; ``binding`` loads the HIP
library on first import and raises if it is missing.
"""
__all__ = ["microstructures"]
