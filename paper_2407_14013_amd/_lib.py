"""ctypes declarations of the C ABI in include/wcsdp.h and include/wcsdp_linalg.h.

The shared library is built in-tree (paper_2407_14013_amd/libwcsdp.so).  There
is no fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwcsdp.so")

SDP_OK, SDP_EINVAL, SDP_ENOMEM, SDP_EDEVICE, SDP_ENOTCONV, SDP_ENUMERIC, SDP_ESTALL = 0, -1, -2, -3, -4, -5, -6
SDP_ECENTER = -7
WC_DSYMV_NOALLOC_MAX_D = 16384
SDP_ADJOINT_CENTER_TOL = 1e-6
SDP_A_DENSE, SDP_A_ENTRY, SDP_A_SPARSE = 0, 1, 2
SDP_SOLVER_PCG, SDP_SOLVER_MINRES = 0, 1
SDP_PREC_F64, SDP_PREC_F32, SDP_PREC_BF16 = 0, 1, 2
SDP_REFINE_SWEEPS, SDP_REFINE_REPLACE = 0, 1
SDP_K_A_APPLY, SDP_K_AT_APPLY, SDP_K_GEMM, SDP_K_NEWTON, SDP_K_SANDWICH = 0, 1, 2, 3, 4
SDP_K_SAMPLED_YE, SDP_K_SAMPLED_DOTS, SDP_K_SANDWICH_LOWER = 5, 6, 7
SDP_K_COUNT = 8

STATUS_NAMES = {
    0: "SDP_OK",
    -1: "SDP_EINVAL",
    -2: "SDP_ENOMEM",
    -3: "SDP_EDEVICE",
    -4: "SDP_ENOTCONV",
    -5: "SDP_ENUMERIC",
    -6: "SDP_ESTALL",
    -7: "SDP_ECENTER",
}


class SdpProblem(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("m", C.c_int32),
        ("a_kind", C.c_int32),
        ("A", C.c_void_p),
        ("jk", C.c_void_p),
        ("b", C.c_void_p),
        ("C", C.c_void_p),
        ("on_device", C.c_int32),
    ]


class SdpSparseRows(C.Structure):
    _fields_ = [
        ("ptr", C.c_void_p),
        ("row", C.c_void_p),
        ("col", C.c_void_p),
        ("val", C.c_void_p),
        ("on_device", C.c_int32),
    ]


class SdpLpBlock(C.Structure):
    _fields_ = [
        ("l", C.c_int32),
        ("col_ptr", C.c_void_p),
        ("row", C.c_void_p),
        ("val", C.c_void_p),
        ("c", C.c_void_p),
        ("on_device", C.c_int32),
    ]


class SdpOptions(C.Structure):
    _fields_ = [
        ("rank_max", C.c_int32),
        ("rank_fixed", C.c_int32),
        ("beta", C.c_double),
        ("solver", C.c_int32),
        ("inner_tol", C.c_double),
        ("inner_maxit", C.c_int32),
        ("inner_prec", C.c_int32),
        ("max_refine", C.c_int32),
        ("gap_tol", C.c_double),
        ("feas_tol", C.c_double),
        ("max_ipm_iter", C.c_int32),
        ("step_frac", C.c_double),
        ("verbose", C.c_int32),
        ("refine_tol", C.c_double),
        ("sparse_sandwich", C.c_int32),
        ("refine_mode", C.c_int32),
        ("lp_top_max", C.c_int32),
    ]


class SdpInnerStats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32),
        ("refinements", C.c_int32),
        ("converged", C.c_int32),
        ("r", C.c_int32),
        ("tau", C.c_double),
        ("beta", C.c_double),
        ("rel_res", C.c_double),
    ]


class SdpStepStats(C.Structure):
    _fields_ = [
        ("mu", C.c_double),
        ("pobj", C.c_double),
        ("dobj", C.c_double),
        ("relgap", C.c_double),
        ("pinf", C.c_double),
        ("dinf", C.c_double),
        ("alpha_p", C.c_double),
        ("alpha_d", C.c_double),
        ("sigma", C.c_double),
        ("r", C.c_int32),
        ("pcg_pred", C.c_int32),
        ("pcg_corr", C.c_int32),
        ("converged", C.c_int32),
        ("t_scaling_ms", C.c_double),
        ("t_inner_ms", C.c_double),
        ("t_total_ms", C.c_double),
    ]


class SdpAdjointStats(C.Structure):
    _fields_ = [
        ("centring_steps", C.c_int32),
        ("inner_iterations", C.c_int32),
        ("converged", C.c_int32),
        ("centrality", C.c_double),
        ("mu", C.c_double),
    ]


class SdpBatchTune(C.Structure):
    _fields_ = [
        ("rows_per_wave", C.c_int32),
        ("aq_group", C.c_int32),
        ("gemm_tile", C.c_int32),
    ]


class SdpResult(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("iterations", C.c_int32),
        ("pcg_iterations", C.c_int64),
        ("newton_matvecs", C.c_int64),
        ("pobj", C.c_double),
        ("dobj", C.c_double),
        ("relgap", C.c_double),
        ("pinf", C.c_double),
        ("dinf", C.c_double),
        ("mu", C.c_double),
        ("time_ms", C.c_double),
        ("lp_matvecs", C.c_int64),
    ]


def struct_dict(s) -> dict:
    return {name: getattr(s, name) for name, _ in s._fields_}


_lib = None

# (name, restype, argtypes)
_SIGNATURES = [
    ("sdp_default_options", None, [C.POINTER(SdpOptions)]),
    ("sdp_setup", C.c_int32, [C.POINTER(SdpProblem), C.POINTER(SdpOptions), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("sdp_setup_lp", C.c_int32, [C.POINTER(SdpProblem), C.POINTER(SdpLpBlock), C.POINTER(SdpOptions), C.c_void_p,
                                 C.POINTER(C.c_void_p)]),
    ("sdp_setup_ex", C.c_int32, [C.POINTER(SdpProblem), C.POINTER(SdpSparseRows), C.POINTER(SdpLpBlock),
                                 C.POINTER(SdpOptions), C.c_void_p, C.POINTER(C.c_void_p)]),
    ("sdp_destroy", None, [C.c_void_p]),
    ("sdp_last_error", C.c_char_p, [C.c_void_p]),
    ("sdp_aug_dim", C.c_int64, [C.c_void_p]),
    ("sdp_newton_apply", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sdp_newton_apply_prec", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    ("sdp_precond_apply", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sdp_inner_solve", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SdpInnerStats)]),
    ("sdp_inner_solve_lp", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.POINTER(SdpInnerStats)]),
    ("sdp_get_lp_split", C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_void_p, C.c_void_p]),
    ("sdp_ipm_step", C.c_int32, [C.c_void_p, C.POINTER(SdpStepStats)]),
    ("sdp_solve_batched", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(SdpOptions), C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sdp_autotune_batched", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(SdpOptions), C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_double)]),
    ("sdp_adjoint", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(SdpAdjointStats)]),
    ("sdp_solve", C.c_int32, [C.c_void_p, C.POINTER(SdpResult)]),
    ("sdp_get_point", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sdp_set_point", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sdp_get_point_lp", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sdp_set_point_lp", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("sdp_get_scaling", C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("sdp_profile_enable", C.c_int32, [C.c_void_p, C.c_int32]),
    ("sdp_profile_get", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_double)]),
    ("wc_dgemm", C.c_int32, [C.c_void_p, C.c_char, C.c_char, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_void_p,
                             C.c_int32, C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_int32]),
    ("wc_dgemm_sym_lower", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                       C.c_int32, C.c_void_p, C.c_int32]),
    ("wc_dpotrf", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    ("wc_dtrtri", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    ("wc_dlanczos_min_eig", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                         C.POINTER(C.c_double)]),
    ("wc_djacobi_svd", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                   C.c_double, C.c_int32, C.POINTER(C.c_int32)]),
    ("wc_dsymv", C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_int32, C.c_void_p, C.c_double,
                             C.c_void_p]),
    ("wc_dsymv_noalloc", C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_int32, C.c_void_p,
                                     C.c_double, C.c_void_p]),
    ("wc_gemm_lp", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                               C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    ("wc_gemm_lp_sym", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int32,
                                   C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]),
    ("wc_to_lowp", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                               C.c_int32]),
]


def lib():
    """Load libwcsdp.so (once) and declare its signatures."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2407_14013_amd.build` "
                "(there is no CPU fallback)"
            )
        h = C.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def exported_names():
    return [s[0] for s in _SIGNATURES]
