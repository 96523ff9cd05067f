"""ctypes declarations of the qtthom C ABI (include/qtthom.h).

Argument marshalling only: every computation runs in the HIP library.  The
library is loaded from this package directory; importing this module fails
loudly when it has not been built (``python -m paper_2412_11566_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqtthom.so")
HOSTLIB_PATH = os.path.join(HERE, "libqtthom_host.so")

QTT_OK = 0
QTT_EINVAL = -1
QTT_ENOMEM = -2
QTT_ECAPACITY = -3
QTT_EHIP = -4
QTT_ENOCONV = -5
QTT_ENAN = -6
QTT_EDIVERGED = -7

QTT_INVERSE = 1
QTT_NO_ROUND = 2
QTT_EXACT = 4

QTT_PREC_FP64 = 0
QTT_PREC_FP32 = 1
QTT_PREC_BF16X3 = 2
QTT_GEMM_PATH_BF16X3 = 16

QTT_ORTH_AUTO = 0
QTT_ORTH_HOUSEHOLDER = 1
QTT_ORTH_CHOLQR = 2
QTT_MV_SKETCH = 0
QTT_MV_AMEN = 1
QTT_SCHEME_DIRECT = 0
QTT_SCHEME_STAGGERED = 1

QTT_ZQR_NOALLOC_MAX_ELEMS = 1048576

ERR_NAMES = {QTT_EINVAL: "EINVAL", QTT_ENOMEM: "ENOMEM", QTT_ECAPACITY: "ECAPACITY",
             QTT_EHIP: "EHIP", QTT_ENOCONV: "ENOCONV", QTT_ENAN: "ENAN",
             QTT_EDIVERGED: "EDIVERGED"}


class Problem(C.Structure):
    _fields_ = [("n", C.c_int), ("phase", C.POINTER(C.c_uint8)), ("nphase", C.c_int),
                ("lame", C.POINTER(C.c_double)), ("lame0", C.c_double * 2),
                ("load_mask", C.c_int), ("phase_on_device", C.c_int), ("scheme", C.c_int),
                ("dim", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("delta", C.c_double), ("tol", C.c_double), ("cap", C.c_int),
                ("max_iter", C.c_int), ("precision", C.c_int), ("oversample", C.c_int),
                ("exact", C.c_int), ("seed", C.c_uint64), ("streams", C.c_int),
                ("history", C.POINTER(C.c_double)), ("history_len", C.c_int), ("orth", C.c_int),
                ("matvec", C.c_int), ("rank_buckets", C.c_int)]


class Report(C.Structure):
    _fields_ = [("iterations", C.c_int * 6), ("residual", C.c_double * 6),
                ("max_rank", C.c_int), ("discarded", C.c_double), ("status", C.c_int),
                ("seconds_setup", C.c_double), ("seconds_solve", C.c_double)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I = C.c_int
D = C.c_double
DP = C.POINTER(C.c_double)
IP = C.POINTER(C.c_int)
U64 = C.c_uint64

SIGNATURES = {
    "qtt_create": (I, [I, P, PP]),
    "qtt_destroy": (I, [P]),
    "qtt_last_error": (C.c_char_p, [P]),
    "qtt_sync": (I, [P]),
    "qtt_tt_from_host": (I, [P, I, IP, IP, I, DP, PP]),
    "qtt_tensor_shape": (I, [P, IP, IP, IP, IP, IP, IP]),
    "qtt_tensor_size": (C.c_size_t, [P]),
    "qtt_tensor_to_host": (I, [P, P, DP, C.c_size_t]),
    "qtt_tensor_destroy": (I, [P]),
    "qtt_tensor_create": (I, [P, I, IP, IP, I, PP]),
    "qtt_tensor_wrap": (I, [P, I, IP, IP, I, P, C.c_size_t, PP]),
    "qtt_tensor_core": (I, [P, I, PP, C.POINTER(C.c_size_t)]),
    "qtt_tensor_export": (I, [P, P, P, C.c_size_t]),
    "qtt_const_strain": (I, [P, I, I, DP, PP]),
    "qtt_sfft_build": (I, [P, I, D, PP]),
    "qtt_green_build": (I, [P, I, D, D, D, PP]),
    "qtt_green_build_scheme": (I, [P, I, D, D, D, I, PP]),
    "qtt_from_voxels": (I, [P, C.POINTER(C.c_uint8), I, I, I, DP, DP, D, I, PP, PP]),
    "qtt_from_voxels_dim": (I, [P, C.POINTER(C.c_uint8), I, I, I, DP, DP, D, I, I, PP, PP]),
    "qtt_rank_estimate": (I, [P, C.POINTER(C.c_uint8), I, I, I, D, IP, DP]),
    "qtt_rank_estimate_dim": (I, [P, C.POINTER(C.c_uint8), I, I, I, D, I, IP, DP]),
    "sfft_apply": (I, [P, P, P, PP, I, D, I, U64]),
    "tt_hadamard": (I, [P, P, P, PP, I, D, I, U64]),
    "green_apply": (I, [P, P, P, PP, I, D, I, U64]),
    "tt_amen_apply": (I, [P, P, P, P, P, D, I, I, D, PP, IP, DP]),
    "tt_round": (I, [P, P, D, I, DP]),
    "tt_norm": (I, [P, P, DP]),
    "tt_axpby": (I, [P, D, P, D, P, PP]),
    "tt_mean_apply": (I, [P, P, P, DP]),
    "ls_solve": (I, [P, C.POINTER(Problem), C.POINTER(SolveOpts), DP, C.POINTER(Report), PP]),
    "ls_adjoint": (I, [P, C.POINTER(Problem), C.POINTER(SolveOpts), P, DP, DP,
                       C.POINTER(Report)]),
    "qtt_batch_solve": (I, [P, I, C.POINTER(Problem), C.POINTER(SolveOpts), DP,
                            C.POINTER(Report)]),
    "qtt_prepare": (I, [P, C.POINTER(Problem), D, PP]),
    "qtt_prepared_destroy": (I, [P]),
    "ls_solve_prepared": (I, [P, P, C.POINTER(SolveOpts), DP, C.POINTER(Report), PP]),
    "qtt_zgemm": (I, [P, I, I, I, I, I, DP, P, C.c_long, P, C.c_long, DP, P, C.c_long, I,
                      C.c_long, C.c_long, C.c_long, I]),
    "qtt_zqr": (I, [P, I, I, I, P, P, P, I]),
    "qtt_zjacobi": (I, [P, I, I, P, P, P]),
    "qtt_zqr_noalloc": (I, [P, I, I, I, P, P, P]),
    "qtt_zorth": (I, [P, I, I, I, P, P, C.POINTER(C.c_int), I]),
    "ls_adjoint_prepared": (I, [P, P, C.POINTER(SolveOpts), P, DP, DP, C.POINTER(Report)]),
    "ls_unrolled": (I, [P, C.POINTER(Problem), C.POINTER(SolveOpts), I, I, DP, DP, DP,
                        C.POINTER(Report)]),
    "ls_unrolled_prepared": (I, [P, P, C.POINTER(SolveOpts), I, I, DP, DP, DP,
                                 C.POINTER(Report)]),
    "qtt_stats_enable": (I, [P, I]),
    "qtt_stats_get": (I, [P, I, C.POINTER(C.c_longlong), DP, DP, DP]),
    "qtt_stats_reset": (I, [P]),
    "qtt_stats_get_all": (I, [P, I, C.POINTER(C.c_longlong), DP, DP]),
}

QTT_K_GEMM = 0
QTT_K_QR = 1
QTT_K_JACOBI = 2
QTT_K_APPLY = 3
QTT_K_OTHER = 4
QTT_K_MFMA = 5
QTT_K_MFMA32 = 6
QTT_K_CONTRACT = 7
QTT_K_MFMA_BF16 = 8
KERNEL_FAMILIES = {QTT_K_GEMM: "gemm", QTT_K_QR: "qr", QTT_K_JACOBI: "jacobi",
                   QTT_K_APPLY: "tto_apply", QTT_K_OTHER: "other", QTT_K_MFMA: "gemm_mfma",
                   QTT_K_MFMA32: "gemm_mfma_fp32", QTT_K_CONTRACT: "tto_contract",
                   QTT_K_MFMA_BF16: "gemm_mfma_bf16x3"}

HOST_SIGNATURES = {
    "qtt_host_qn_tto": (I, [I, D, IP, DP, C.c_size_t]),
    "qtt_host_green": (I, [I, D, D, D, I, IP, IP, IP, DP, C.c_size_t, DP]),
    "qtt_host_stiffness": (I, [C.POINTER(C.c_uint8), I, I, DP, DP, D, IP, IP, IP, DP,
                               C.c_size_t]),
}


def _bind(path: str, sigs: dict) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(
            f"qtthom native library missing at {path}; build it with "
            "`python -m paper_2412_11566_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = None
_hostlib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch has
        # already loaded, so both share one runtime and one device context.
        import torch  # noqa: F401
        _lib = _bind(LIB_PATH, SIGNATURES)
    return _lib


def hostlib() -> C.CDLL:
    global _hostlib
    if _hostlib is None:
        _hostlib = _bind(HOSTLIB_PATH, HOST_SIGNATURES)
    return _hostlib
