"""Adaptive-multigrid GCR for the Wilson-Dirac operator on MI355X (gfx950).

The compute path lives in the HIP library ``libwmg.so`` (C ABI declared in
``include/wmg.h``); :mod:`paper_0912_2186_amd.wmg` is its thin ctypes
binding and :mod:`paper_0912_2186_amd.inputs` holds the seeded synthetic
input generators.  Importing the package itself loads nothing.
"""
