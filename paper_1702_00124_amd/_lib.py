"""ctypes declarations of libwilson_hmc (include/wilson_hmc.h).

Argument marshalling only: every operation runs in the HIP library.  Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwilson_hmc.so")

WL_OK, WL_EINVAL, WL_EUNSUPPORTED, WL_ENOMEM, WL_EHIP, WL_ENOCONV = 0, -1, -2, -3, -4, -5
WL_F64, WL_F32, WL_BF16 = 0, 1, 2
WL_OP_M, WL_OP_MDAG, WL_OP_K, WL_OP_MHAT, WL_OP_MHAT_DAG, WL_OP_J = range(6)
WL_POLY_P, WL_POLY_PJ, WL_POLY_Q, WL_POLY_QDAG = range(4)
WL_TERM_KINV_FULL, WL_TERM_KINV, WL_TERM_RATIO, WL_TERM_POLY, WL_TERM_POLYK_INV = range(5)
WL_HMC_NO_METROPOLIS, WL_HMC_PHI_GIVEN, WL_HMC_CHRONO = 1, 2, 4
WL_INT_LEAPFROG, WL_INT_OMELYAN = 0, 1


class CgParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("inner", C.c_int), ("delta", C.c_double),
                ("chunk", C.c_int), ("use_graph", C.c_int), ("use_x0", C.c_int)]


class CgStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("reliable_updates", C.c_int), ("converged", C.c_int),
                ("true_rel_res", C.c_double)]


class Poly(C.Structure):
    _fields_ = [("degree", C.c_int), ("a", C.c_double), ("b", C.c_double), ("degree_div", C.c_int)]


class Term(C.Structure):
    _fields_ = [("kind", C.c_int), ("kappa", C.c_double), ("mu2", C.c_double), ("poly", Poly), ("cg", CgParams),
                ("kappa_num", C.c_double), ("mu2_num", C.c_double)]


class HmcParams(C.Structure):
    _fields_ = [("beta", C.c_double), ("tau", C.c_double), ("omelyan_lambda", C.c_double),
                ("integrator", C.c_int), ("nterms", C.c_int), ("terms", Term * 8), ("nsteps", C.c_int * 9),
                ("flags", C.c_int), ("chrono_depth", C.c_int)]


class HmcResult(C.Structure):
    _fields_ = [("dH", C.c_double), ("H0", C.c_double), ("H1", C.c_double), ("S0", C.c_double * 9),
                ("S1", C.c_double * 9), ("plaquette", C.c_double), ("accepted", C.c_int),
                ("n_kmat", C.c_longlong), ("cg_iters", C.c_longlong)]


# name -> (restype, argtypes)
P, D, I, SZ, LL = C.c_void_p, C.c_double, C.c_int, C.c_size_t, C.c_longlong
SIGNATURES = {
    "wl_last_error": (C.c_char_p, []),
    "wl_create": (I, [C.POINTER(P), C.POINTER(C.c_int32), C.c_int32, P]),
    "wl_destroy": (I, [P]),
    "wl_set_stream": (I, [P, P]),
    "wl_set_links": (I, [P, P, I]),
    "wl_get_links": (I, [P, P, I]),
    "wl_field_bytes": (I, [P, I, I, C.POINTER(SZ)]),
    "wl_import_spinor": (I, [P, P, P, I, I]),
    "wl_export_spinor": (I, [P, P, P, I, I]),
    "wl_import_full": (I, [P, P, P]),
    "wl_export_full": (I, [P, P, P]),
    "wl_import_su3": (I, [P, P, P]),
    "wl_export_su3": (I, [P, P, P]),
    "wilson_dslash": (I, [P, P, P, I, I, I, I]),
    "apply_K": (I, [P, P, P, D, C.POINTER(D), I, I, I]),
    "apply_K_noalloc": (I, [P, P, P, D, C.POINTER(D), I, I, I]),
    "cg_solve": (I, [P, P, P, D, C.POINTER(D), I, I, C.POINTER(CgParams), C.POINTER(CgStats)]),
    "cg_multishift": (I, [P, P, P, D, C.POINTER(D), I, I, C.POINTER(CgParams), C.POINTER(CgStats)]),
    "poly_filter_apply": (I, [P, P, P, D, D, C.POINTER(Poly), I, I, I]),
    "wl_heatbath": (I, [P, P, C.POINTER(Term), P]),
    "wl_action": (I, [P, C.POINTER(Term), P, C.POINTER(D)]),
    "fermion_force": (I, [P, P, C.POINTER(Term), P, D, C.POINTER(D)]),
    "wl_force_bilinear": (I, [P, P, P, P, D]),
    "wl_gauge_force": (I, [P, P, D, D]),
    "wl_plaquette": (I, [P, C.POINTER(D)]),
    "wl_link_update": (I, [P, P, D]),
    "hmc_trajectory": (I, [P, C.POINTER(HmcParams), P, P, D, C.POINTER(HmcResult)]),
    "wl_counters": (I, [P, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
    "wl_solve_log": (I, [P, I]),
    "wl_solve_log_read": (I, [P, I, C.POINTER(I), C.POINTER(LL), C.POINTER(LL), C.POINTER(LL)]),
    "wl_batch_create": (I, [C.POINTER(P), C.POINTER(P), I]),
    "wl_batch_destroy": (I, [P]),
    "wl_batch_slot_bytes": (I, [P, I, C.POINTER(SZ)]),
    "wl_batch_dslash": (I, [P, P, P, I, I, I]),
    "wl_batch_apply_J": (I, [P, P, P, C.POINTER(D), C.POINTER(D), I]),
    "wl_batch_cg_solve": (I, [P, P, P, C.POINTER(D), C.POINTER(D), C.POINTER(CgParams), C.POINTER(CgStats)]),
    "wl_integrator_schedule": (I, [C.POINTER(I), I, I, D, C.POINTER(I), C.POINTER(I), C.POINTER(D), I,
                                   C.POINTER(I)]),
    "wl_profile": (I, [P, I]),
    "wl_set_hop_config": (I, [P, I, I, I, I, I, I]),
    "wl_get_hop_config": (I, [P, I, I, C.POINTER(I), C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
    "wl_autotune": (I, [P, C.POINTER(D)]),
    "wl_time_hop": (I, [P, I, I, I, C.POINTER(D)]),
    "wl_stream_copy": (I, [P, SZ, I, C.POINTER(D)]),
    "wl_hop_counts": (I, [P, C.POINTER(C.c_longlong)]),
    "wl_profile_read": (I, [P, C.POINTER(D), C.POINTER(C.c_longlong)]),
}

_lib = None


def load() -> C.CDLL:
    """Load libwilson_hmc.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1702_00124_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class WilsonError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc: int) -> int:
    if rc != WL_OK and rc != WL_ENOCONV:
        raise WilsonError(rc, load().wl_last_error().decode())
    return rc
