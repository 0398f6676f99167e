"""MI355X (gfx950) implementation of the MPR Gibbs random field gap-filling
hot path (Zukovic & Hristopulos, arXiv 1710.03038): a C-ABI library of HIP
kernels (``libmpr.so``, declared in include/mpr.h) and its Python binding.
"""
from .mpr import (ADAPT, BC_OPEN, BC_REPLICATE, FP32, FP64, MODEL_GMRF, MODEL_MPR, NO_OR, SAMPLE_PAIRS, STATE,  # noqa: F401
                  TRACE_E, Field, MPRError, cv_select_q,
                  default_params, lib, match_T, workspace_bytes)
