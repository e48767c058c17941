"""Lattice GMRF data assimilation by re-weighted Gaussian belief propagation on MI355X.

The compute path is a HIP library for gfx950 (``csrc/``) behind a C ABI
(``include/gabp.h``); ``gabp`` is its thin Python binding and ``inputs`` the
seeded synthetic workloads.  Import ``paper_2404_12968_amd.gabp`` explicitly:
this package init loads nothing.
"""
