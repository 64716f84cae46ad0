"""MI355X-native double-double hot path for stealthy hyperuniform point patterns.

Collective-coordinate optimisation (Morse, Kim, Steinhardt, Torquato,
arXiv:2304.09139): the energy Phi = sum_{0<|k|<=K} v(k) |n~(k)|^2, its gradient,
the wavevector set and an L-BFGS quench, all computed in double-double on the
GPU by the HIP library ``libss.so``.  Importing this package loads nothing; the
binding in :mod:`paper_2304_09139_amd.ss` loads the library on first use.
"""
