"""MI355X (gfx950) eigensolver for the Hermitian Wilson-Dirac operator: RQI with
gamma5-preserving aggregation multigrid (Bali et al., Lattice 2015, Alg. 1).

The computation lives in the HIP library ``lib/liblqmg.so`` (C ABI in
``include/lqmg.h``); ``lqmg`` is its ctypes binding.
"""
from .lqmg import (Context, LQError, MGParams, PREC_FP64, PREC_MIXED, KT_COARSE, KT_COMBINE, KT_GRAM,  # noqa: F401
                   KT_PROLONG, KT_RESTRICT, KT_SAP, KT_WILSON, coarse_variant, kernel_timer_read,
                   kernel_timer_start, load, library_path)
