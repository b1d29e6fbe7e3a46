"""MI355X-native hot path of the hp-version time-stepping spectral Monte Carlo
method (arXiv 2608.22190): per-node Monte Carlo residual estimation and the
Legendre reconstruction, as hand-written HIP kernels behind a C ABI.

Submodules:
  ``workloads`` -- seeded synthetic problem descriptions (inputs only);
  ``hpsmc``     -- ctypes binding of ``libhpsmc.so`` (loads the HIP library);
  ``build``     -- compiles the library for gfx950.
Importing the package itself loads nothing native.
"""
