"""ctypes declarations of the C ABI in include/klecgc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libklecgc.so")

KC_OK = 0
ERRORS = {
    -1: "KC_EINVAL", -2: "KC_ENOMEM", -3: "KC_EHIP", -4: "KC_ERANK",
    -5: "KC_ENOCONV", -6: "KC_ENONFINITE", -7: "KC_EUNSUPPORTED",
}
KC_PREC_F64, KC_PREC_F32_REFINED = 0, 1
KC_KLE_FIELD_EXP, KC_KLE_SNAPSHOT = 0, 1
KC_INIT_GIVEN, KC_INIT_ZERO, KC_INIT_COARSE, KC_INIT_GPC = 0, 1, 2, 3
KC_INIT_RANDOM, KC_INIT_MLP, KC_INIT_MLP_GPC_FALLBACK = 4, 5, 6
KC_SAMPLE_CONVERGED, KC_SAMPLE_MAXITER, KC_SAMPLE_NONFINITE = 0, 1, 2
KC_GPC_HERMITE, KC_GPC_LEGENDRE = 0, 1
KC_MODEL_ADE_P1, KC_MODEL_BURGERS, KC_MODEL_ALLEN_CAHN = 1, 2, 3


class Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32),
        ("T", ctypes.c_double), ("N", ctypes.c_int32), ("J", ctypes.c_int32),
        ("alpha", ctypes.c_double), ("forcing", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double), ("inner_max_iter", ctypes.c_int32),
        ("cgc_rtol", ctypes.c_double), ("cgc_max_iter", ctypes.c_int32),
    ]


class Model(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("n", ctypes.c_int32),
        ("T", ctypes.c_double), ("N", ctypes.c_int32), ("J", ctypes.c_int32),
        ("alpha", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
        ("beta", ctypes.c_double), ("newton_tol", ctypes.c_double), ("newton_max_iter", ctypes.c_int32),
    ]


class KleDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("d", ctypes.c_int32),
        ("corr_len", ctypes.c_double), ("sigma", ctypes.c_double),
        ("L", ctypes.c_int64), ("eps_kl", ctypes.c_double),
    ]


class Task(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("N", ctypes.c_int32), ("face_off", ctypes.c_int64),
                ("state_off", ctypes.c_int64)]


KC_BATCH_GRAPH, KC_BATCH_PROGRESS, KC_BATCH_PERSISTENT = 1, 2, 4
KC_FINE_STREAM64, KC_FINE_RES16, KC_FINE_RES32, KC_FINE_RES64, KC_FINE_RES128, KC_FINE_MG, KC_FINE_RB128 = 0, 1, 2, 3, 4, 5, 6
KC_CGC_STREAM64, KC_CGC_RES16, KC_CGC_RES32, KC_CGC_RES64, KC_CGC_STREAM32, KC_CGC_MG32 = 0, 1, 2, 3, 4, 5


class Tuning(ctypes.Structure):
    _fields_ = [("fine_variant", ctypes.c_int32), ("fine_pcg_rtol", ctypes.c_float),
                ("cgc_variant", ctypes.c_int32), ("cgc_inner_rtol", ctypes.c_float), ("mg_sweeps", ctypes.c_int32),
                ("mg_smoother", ctypes.c_int32)]

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_P = ctypes.POINTER

SIGNATURES = {
    "klecgc_create": (ctypes.c_int, [_P(_vp), ctypes.c_int, _vp]),
    "klecgc_destroy": (None, [_vp]),
    "klecgc_set_stream": (ctypes.c_int, [_vp, _vp]),
    "klecgc_last_error": (ctypes.c_char_p, [_vp]),
    "klecgc_kle_free": (None, [_vp]),
    "klecgc_gpc_free": (None, [_vp]),
    "klecgc_mlp_free": (None, [_vp]),
    "klecgc_version": (ctypes.c_char_p, []),
    "klecgc_last_stats": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
    "klecgc_last_times": (ctypes.c_int, [_vp, _P(ctypes.c_double), _P(ctypes.c_int64)]),
    "klecgc_set_tuning": (ctypes.c_int, [_vp, _i32, _P(Tuning)]),
    "klecgc_get_tuning": (ctypes.c_int, [_vp, _i32, _P(Tuning)]),
    "klecgc_autotune": (ctypes.c_int, [_vp, _P(Problem), _vp, _i64, _P(Tuning), _P(ctypes.c_double)]),
    "serial_fine_propagate": (ctypes.c_int, [_vp, _P(Problem), _vp, _vp, _i64, _vp]),
    "kle_build": (ctypes.c_int, [_vp, _P(KleDesc), _vp, _i64, _P(_vp), _P(_i32)]),
    "kle_synthesize": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "kle_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "gpc_fit": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _P(_vp), _P(_i32)]),
    "gpc_predict": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp]),
    "fine_propagate": (ctypes.c_int, [_vp, _P(Problem), _vp, _vp, _i64, _vp, _vp]),
    "fine_propagate_noalloc": (ctypes.c_int, [_vp, _P(Problem), _vp, _vp, _i64, _vp, _vp]),
    "cgc_diag_solve": (ctypes.c_int, [_vp, _P(Problem), _vp, _vp, _i64, _vp]),
    "coarse_propagate": (ctypes.c_int, [_vp, _P(Problem), _vp, _vp, _i64, _vp]),
    "parareal_solve": (ctypes.c_int, [_vp, _P(Problem), _vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp,
                                      ctypes.c_uint64, _vp, _P(_i32), _P(_i32), _P(ctypes.c_double),
                                      _P(_i32)]),
    "parareal_solve_sequential": (ctypes.c_int, [_vp, _P(Problem), _vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp,
                                                 ctypes.c_uint64, _vp, _P(_i32), _P(_i32), _P(ctypes.c_double)]),
    "parareal_solve_batch": (ctypes.c_int, [_vp, _P(Problem), _P(Task), _i64, _vp, _i32, _vp, _i32,
                                            _P(_i32), _P(_i32), _P(ctypes.c_double), _P(ctypes.c_double)]),
    "model_fine_propagate": (ctypes.c_int, [_vp, _P(Model), _vp, _vp, _i64, _vp]),
    "model_coarse_propagate": (ctypes.c_int, [_vp, _P(Model), _vp, _vp, _i64, _vp]),
    "model_serial_fine": (ctypes.c_int, [_vp, _P(Model), _vp, _vp, _i64, _vp]),
    "model_cgc_solve": (ctypes.c_int, [_vp, _P(Model), _vp, _vp, _vp, _i64, _vp, _P(_i32)]),
    "model_parareal_solve": (ctypes.c_int, [_vp, _P(Model), _vp, _vp, _i64, _i32, _vp, _vp, _vp, ctypes.c_uint64,
                                            _vp, _vp, _P(_i32), _P(_i32), _P(ctypes.c_double),
                                            _P(ctypes.c_double)]),
    "model_parareal_solve_sequential": (ctypes.c_int, [_vp, _P(Model), _vp, _vp, _i64, _i32, _vp, _vp, _vp,
                                                       ctypes.c_uint64, _vp, _vp, _P(_i32), _P(_i32),
                                                       _P(ctypes.c_double), _P(ctypes.c_double)]),
    "mlp_create": (ctypes.c_int, [_vp, _i32, _i32, _i64, _P(_vp), _P(_i64)]),
    "mlp_set_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "mlp_get_params": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mlp_normalize_targets": (ctypes.c_int, [_vp, _vp, _vp, _i64]),
    "mlp_train": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, _i32, ctypes.c_float, ctypes.c_float, _vp,
                                 _P(ctypes.c_float)]),
    "mlp_predict": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp]),
    "mlp_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _P(ctypes.c_double)]),
    "grid_restrict": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, _vp]),
    "mlp_initial_guess": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _vp, _i64, _vp]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libklecgc.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2510_26180_amd.build` "
                          "(the HIP library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
