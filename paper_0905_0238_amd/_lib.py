"""ctypes declarations of libedt (include/edt.h).  Loading fails loudly: there
is no fallback implementation of any entry point."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libedt.so")

EDT_OK, EDT_EINVAL, EDT_ENOMEM, EDT_EHIP, EDT_ESTATE = 0, -1, -2, -3, -4
STATIC_SCRATCH_BYTES = 256 * 1024 * 1024   # EDT_STATIC_SCRATCH_BYTES
INFO_OK, INFO_EMPTY, INFO_NOCONV, INFO_NONFINITE = 0, -1, -2, -3
FP64, FP32, BF16X3, FP16X3 = 0, 1, 2, 3
DATA_C128, DATA_C64 = 0, 1
DATA_TYPES = {"c128": DATA_C128, "c64": DATA_C64}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3}


class Survey(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_mid", C.c_int), ("d_mid", C.c_double), ("n_off", C.c_int),
                ("d_off", C.c_double), ("n_freq", C.c_int), ("freq_hz", C.POINTER(C.c_double)),
                ("eps", C.c_double), ("nz", C.c_int), ("z0", C.c_double), ("dz", C.c_double),
                ("kappa", C.c_double), ("n_line", C.c_int), ("d_line", C.c_double)]


class Layers(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("vel", C.POINTER(C.c_double)), ("zif", C.POINTER(C.c_double))]


class PlanInfo(C.Structure):
    _fields_ = [("n_km", C.c_int64), ("n_pairs", C.c_int64), ("n_rows", C.c_int64),
                ("n_urows", C.c_int64), ("max_rows", C.c_int64), ("n_empty", C.c_int64),
                ("n_items", C.c_int64), ("n_freq", C.c_int), ("n_cls", C.c_int), ("nz", C.c_int),
                ("n_layers", C.c_int), ("chunk_rows", C.c_int), ("gram_band", C.c_int),
                ("table_elems", C.c_size_t),
                ("dev_plan_bytes", C.c_size_t), ("work_bytes", C.c_size_t), ("gram_flops", C.c_double),
                ("n_pairs_all", C.c_int64), ("pair_begin", C.c_int64), ("resid_group", C.c_int),
                ("data_type", C.c_int), ("resident_bytes", C.c_size_t)]


class PlanOpts(C.Structure):
    _fields_ = [("chunk_rows", C.c_int), ("gram_band", C.c_int), ("pair_begin", C.c_int64),
                ("pair_end", C.c_int64), ("data_type", C.c_int), ("hbm_budget", C.c_size_t),
                ("resid_group", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("refine", C.c_int), ("refine_tol", C.c_double), ("max_refine", C.c_int),
                ("escalate", C.c_int), ("data_summed", C.c_int)]


EXPORTS = ["edt_last_error", "edt_plan_create", "edt_survey_pair_rows", "edt_plan_destroy", "edt_plan_query",
           "edt_plan_rowmap", "edt_plan_urows", "edt_plan_schedule", "edt_plan_upload", "edt_green", "edt_assemble", "edt_solve", "edt_solve_static",
           "edt_forward", "edt_adjoint", "edt_tsvd_work_bytes", "edt_tsvd", "edt_kz_disk_radius", "edt_kz_restrict", "edt_shots_fft", "edt_shots_pack", "edt_model", "edt_aperture_work_bytes", "edt_aperture_gram", "edt_timing_enable",
           "edt_timing_read"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libedt.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_0905_0238_amd.build`")
    L = C.CDLL(path)
    vp, dp, ip, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    L.edt_last_error.restype = C.c_char_p
    L.edt_last_error.argtypes = []
    sig = {
        "edt_plan_create": [C.POINTER(Survey), C.POINTER(Layers), C.POINTER(PlanOpts), C.POINTER(vp)],
        "edt_survey_pair_rows": [C.POINTER(Survey), C.POINTER(Layers), i64p, i64p],
        "edt_plan_destroy": [vp],
        "edt_plan_query": [vp, C.POINTER(PlanInfo)],
        "edt_plan_rowmap": [vp, i64p, ip, ip, ip, dp],
        "edt_plan_urows": [vp, i64p, ip, ip],
        "edt_plan_schedule": [vp, C.c_int, i64p, ip, ip],
        "edt_plan_upload": [vp, vp, C.c_size_t, vp],
        "edt_green": [vp, vp, vp, vp, vp],
        "edt_assemble": [vp, vp, vp, vp, C.c_int, vp, vp, vp, vp, vp],
        "edt_solve": [vp, vp, vp, vp, vp, vp, C.c_double, C.POINTER(SolveOpts), vp, vp, vp, vp, vp, vp],
        "edt_solve_static": [vp, vp, vp, vp, vp, vp, C.c_double, C.POINTER(SolveOpts), vp, vp, vp, vp, vp],
        "edt_forward": [vp, vp, vp, vp, vp],
        "edt_adjoint": [vp, vp, vp, vp, vp, vp, vp, C.c_double, vp, vp, vp, vp, vp, vp],
        "edt_tsvd_work_bytes": [vp, C.POINTER(C.c_size_t)],
        "edt_tsvd": [vp, vp, vp, C.c_double, C.c_int, vp, vp, vp, vp, vp, vp, vp],
        "edt_kz_disk_radius": [vp, C.c_double, C.POINTER(C.c_double)],
        "edt_kz_restrict": [vp, C.c_double, vp, vp, vp, vp, vp],
        "edt_shots_fft": [vp, vp, vp],
        "edt_shots_pack": [vp, vp, vp, vp],
        "edt_model": [vp, vp, vp, vp],
        "edt_aperture_work_bytes": [vp, C.POINTER(C.c_size_t)],
        "edt_aperture_gram": [vp, vp, C.c_double, vp, vp, vp, vp],
        "edt_timing_enable": [vp, C.c_int],
        "edt_timing_read": [vp, C.c_int, C.c_char_p, dp, i64p, C.POINTER(C.c_int)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    _lib = L
    return L


def check(status: int, what: str):
    if status != EDT_OK:
        msg = load().edt_last_error().decode(errors="replace")
        raise RuntimeError(f"{what} failed with status {status}: {msg}")
