"""MI355X-native inexact-Krylov linear-response solver (HIP, gfx950).

The compute path lives in ``libikr.so`` (C ABI in ``include/ikr.h``); this
package holds the build script and a thin ctypes binding.
"""
from .binding import (IKR_AGR, IKR_BAL, IKR_D10, IKR_D10N, IKR_D100, IKR_FIXED,
                      IKR_GRT, STRATEGY, IkrError, ResponseSystem, SIGNATURES,
                      chi0_apply, default_opts, dyson_solve, lib, LIB_PATH, profile_enable,
                      profile_query, profile_reset, set_kernel_paths, kernel_paths,
                      PATH_VECTOR_GRAM, PATH_SPLIT_END, PATH_KWIDE, PATH_FIXED)

__all__ = ["ResponseSystem", "IkrError", "default_opts", "dyson_solve", "chi0_apply", "lib", "LIB_PATH",
           "STRATEGY",
           "SIGNATURES", "IKR_AGR", "IKR_BAL", "IKR_GRT", "IKR_D10", "IKR_D100",
           "IKR_D10N", "IKR_FIXED"]
