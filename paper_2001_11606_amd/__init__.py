"""MI355X (gfx950) implicit SPH radiation-diffusion library.

The compute path lives in ``librt.so`` (HIP, built by ``build.py``) behind the
C ABI of ``include/rt.h``; ``rt`` is its ctypes binding and ``driver`` runs
time steps through it.
"""
