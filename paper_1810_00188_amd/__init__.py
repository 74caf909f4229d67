"""Emission-based reciprocal Monte Carlo (ERMC) radiative heat source on MI355X.

Submodules are imported explicitly:

* ``paper_1810_00188_amd.inputs`` -- seeded synthetic workloads (grids, fields,
  narrow-band correlated-k and Planck tables).  Holds no part of the method.
* ``paper_1810_00188_amd.rmc`` -- ctypes binding of the HIP library ``librmc.so``.

Importing the package itself loads nothing.
"""
