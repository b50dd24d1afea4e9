"""ctypes declarations of the C ABI in include/ep_tv.h (libeptv.so).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libeptv.so")

EP_TV_OK = 0
EP_TV_W_NOT_CONVERGED = 1
EP_TV_W_WARM_FALLBACK = 2
EP_TV_E_ARG = -1
EP_TV_E_OOM = -2
EP_TV_E_HIP = -3
EP_TV_E_NONFINITE = -4
EP_TV_E_STATE = -5
EP_TV_E_DIVERGED = -6

OP_IDENTITY = 0
OP_BLUR_PERIODIC = 1
OP_DFT_MASK = 2
OP_HADAMARD_MASK = 3
OP_GAUSS_CS = 4
BND_FREE = 0
BND_PERIODIC = 1
PRECOND_AUTO = 0
PRECOND_JACOBI = 1
PRECOND_CIRCULANT = 2
PRIOR_L1 = 0
PRIOR_MOG2 = 1
PRIOR_BG = 2
OPT_GRAPH = 1
OPT_TILE_ROWS = 2
OPT_EM_OPTION = 3
OPT_PERSISTENT = 4
VAR_SPECTRAL = 0
VAR_RBMC = 1

STATUS_NAMES = {0: "OK", 1: "W_NOT_CONVERGED", 2: "W_WARM_FALLBACK", -1: "E_ARG", -2: "E_OOM",
                -3: "E_HIP", -4: "E_NONFINITE", -5: "E_STATE", -6: "E_DIVERGED"}


class EpTvProblem(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("op", ctypes.c_int32), ("boundary", ctypes.c_int32),
                ("blur_taps", ctypes.POINTER(ctypes.c_float)),
                ("blur_h", ctypes.c_int32), ("blur_w", ctypes.c_int32),
                ("dft_mask", ctypes.POINTER(ctypes.c_uint8)),
                ("noise_var", ctypes.c_double), ("lambda0", ctypes.c_double),
                ("damping", ctypes.c_double), ("cg_tol", ctypes.c_double),
                ("cg_max_iters", ctypes.c_int32), ("cg_precond", ctypes.c_int32),
                ("cg_reduce", ctypes.c_double),
                ("prior", ctypes.c_int32), ("var_estimator", ctypes.c_int32),
                ("prior_omega", ctypes.c_double), ("prior_s1sq", ctypes.c_double),
                ("prior_s2sq", ctypes.c_double),
                ("rbmc_samples", ctypes.c_int32), ("noise_map", ctypes.c_int32),
                ("sense_matrix", ctypes.POINTER(ctypes.c_float)), ("sense_rows", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class EpTvStats(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int32), ("cg_iters_last", ctypes.c_int32),
                ("cg_iters_total", ctypes.c_int32), ("clamp_count", ctypes.c_int32),
                ("status", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("a_bar_u", ctypes.c_double),
                ("max_dmu_rel", ctypes.c_double), ("max_dv_rel", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double), ("lik_precision", ctypes.c_double),
                ("cavity_precision_mean", ctypes.c_double), ("cg_rel_residual", ctypes.c_double),
                ("cold_restarts", ctypes.c_int32), ("reserved_", ctypes.c_int32)]


class EpTvTiming(ctypes.Structure):
    _fields_ = [("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int32),
                ("lik_ms", ctypes.c_double), ("lik_updates", ctypes.c_int32),
                ("apply_ms", ctypes.c_double), ("apply_launches", ctypes.c_int32),
                ("precond_ms", ctypes.c_double), ("precond_launches", ctypes.c_int32),
                ("rf_fwd_ms", ctypes.c_double), ("rf_fwd_launches", ctypes.c_int32),
                ("rf_filt_ms", ctypes.c_double), ("rf_filt_launches", ctypes.c_int32),
                ("rf_inv_ms", ctypes.c_double), ("rf_inv_launches", ctypes.c_int32),
                ("fin_ms", ctypes.c_double), ("fin_launches", ctypes.c_int32),
                ("lik_other_ms", ctypes.c_double), ("lik_other_launches", ctypes.c_int32),
                ("dgemm_ms", ctypes.c_double), ("dgemm_launches", ctypes.c_int32),
                ("dgemm_flops", ctypes.c_double)]


class EpTvTuneResult(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("rows", ctypes.c_int32 * 16), ("ms", ctypes.c_double * 16),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


_P = ctypes.c_void_p
_FPP = ctypes.POINTER(ctypes.c_void_p)   # array of device pointers (host array)

# name -> (restype, argtypes); every symbol include/ep_tv.h declares
SIGNATURES = {
    "ep_tv_version": (ctypes.c_char_p, []),
    "ep_tv_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(EpTvProblem), ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_size_t)]),
    "ep_tv_create": (ctypes.c_int, [ctypes.POINTER(EpTvProblem), ctypes.c_int32, _P, ctypes.c_size_t,
                                    _P, ctypes.POINTER(_P)]),
    "ep_tv_set_observation": (ctypes.c_int, [_P, _FPP]),
    "ep_tv_init_cold": (ctypes.c_int, [_P]),
    "ep_tv_set_rbmc_noise": (ctypes.c_int, [_P, _FPP]),
    "ep_tv_set_noise_variance": (ctypes.c_int, [_P, _FPP]),
    "ep_tv_run": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "ep_tv_em_step": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "ep_tv_solve": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _FPP, _FPP,
                                   ctypes.POINTER(EpTvStats)]),
    "ep_tv_marginals": (ctypes.c_int, [_P, _FPP, _FPP]),
    "ep_tv_get_sites": (ctypes.c_int, [_P, _FPP]),
    "ep_tv_set_sites": (ctypes.c_int, [_P, _FPP, ctypes.POINTER(ctypes.c_double)]),
    "ep_tv_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(EpTvStats)]),
    "ep_tv_get_lik_planes": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "ep_tv_tilted_moments": (ctypes.c_int, [ctypes.c_int32, _P, _P, ctypes.c_float, _P, _P, _P, _P]),
    "ep_tv_tilted_moments_prior": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                  ctypes.c_int32, _P, _P, _P, _P, _P, _P]),
    "ep_tv_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ep_tv_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(EpTvTiming)]),
    "ep_tv_init_warm": (ctypes.c_int, [_P, _FPP, _FPP, ctypes.c_double, ctypes.c_double]),
    "ep_tv_set_option": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64]),
    "ep_tv_get_option": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "ep_tv_autotune": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(EpTvTuneResult)]),
    "ep_tv_denoise_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P]),
    "ep_tv_last_error": (ctypes.c_char_p, [_P]),
    "ep_tv_destroy": (None, [_P]),
    # learned warm start (include/ep_tv_net.h)
    "ep_tv_net_param_count": (ctypes.c_int, []),
    "ep_tv_net_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "ep_tv_net_create": (ctypes.c_int, [_P, _P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "ep_tv_net_sync": (ctypes.c_int, [_P]),
    "ep_tv_net_infer": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_double, _P, _P]),
    "ep_tv_net_loss_grad": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_double, _P,
                                           ctypes.POINTER(ctypes.c_double)]),
    "ep_tv_net_adam_step": (ctypes.c_int, [_P, ctypes.c_float]),
    "ep_tv_net_train_step": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_double, ctypes.c_float,
                                            ctypes.POINTER(ctypes.c_double)]),
    "ep_tv_net_adam_count": (ctypes.c_int, [_P]),
    "ep_tv_net_last_error": (ctypes.c_char_p, [_P]),
    "ep_tv_net_destroy": (None, [_P]),
}

_lib = None


def lib():
    """Load libeptv.so once; raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2110_01585_amd.build "
                           "(there is no non-HIP fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
