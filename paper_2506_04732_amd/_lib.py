"""ctypes declarations of libt2s2 (include/t2s2.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libt2s2.so")

T2S2_OK, T2S2_EINVAL, T2S2_ENOMEM, T2S2_ENOTCONV, T2S2_EHIP, T2S2_EFACTOR = 0, 1, 2, 3, 4, 5
SCHEME_PLAIN, SCHEME_SC = 0, 1
PRECISION_FP64, PRECISION_MIXED = 0, 1
MAX_DIM, MAX_HISTORY, PHASES = 16, 128, 5
PHASE_NAMES = ["setup", "local_solve", "split", "interfaces", "residual"]

EXPORTED = [
    "t2s2_last_error", "t2s2_nodes", "t2s2_matrices_1d", "t2s2_problem_create", "t2s2_problem_destroy",
    "t2s2_problem_operator", "t2s2_problem_colloc", "t2s2_tt_matvec", "t2s2_tt_norm",
    "t2s2_tt_residual_norm", "t2s2_tt_round", "t2s2_local_solve", "t2s2_solve", "t2s2_solve_batched", "t2s2_default_options",
    "t2s2_timing_enable", "t2s2_timing_classes", "t2s2_timing_read", "t2s2_timing_class_name",
    "t2s2_mlp_create", "t2s2_mlp_destroy", "t2s2_mlp_param_count", "t2s2_mlp_get_params", "t2s2_mlp_set_params",
    "t2s2_mlp_forward", "t2s2_mlp_backward", "t2s2_mlp_adam_step", "t2s2_mlp_infer_bf16", "t2s2_mlp_train",
    "t2s2_tt_fit_loss", "t2s2_tt_pack", "t2s2_tt_unpack", "t2s2_source_gaussians", "t2s2_source_manufactured",
    "t2s2_debug_iteration_limits", "t2s2_tt_matvec_noalloc", "t2s2_problem_create_reaction",
    "t2s2_mol_create", "t2s2_mol_step", "t2s2_tt_fiber", "t2s2_problem_create_general", "t2s2_source_cross",
    "t2s2_debug_gemm", "t2s2_gemm_tune_source", "t2s2_debug_readback",
]
TIMING_CLASSES = ["gemm_f64", "gemm_c128", "ttm_matvec", "schur_qr", "hessenberg", "jacobi_svd", "cholesky",
                  "trtri", "trevec", "kron_trisolve", "hess_solve", "other"]


class TTStruct(C.Structure):
    _fields_ = [("d", C.c_int), ("n", C.POINTER(C.c_int)), ("ranks", C.POINTER(C.c_int)),
                ("cores", C.POINTER(C.c_void_p))]


class TTMStruct(C.Structure):
    _fields_ = [("d", C.c_int), ("n", C.POINTER(C.c_int)), ("ranks", C.POINTER(C.c_int)),
                ("cores", C.POINTER(C.c_void_p))]


class Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("target", C.c_double), ("max_sweeps", C.c_int), ("kick", C.c_int),
                ("rank_cap", C.c_int), ("init_rank", C.c_int), ("seed", C.c_ulonglong),
                ("check_every", C.c_int), ("verbose", C.c_int), ("precision", C.c_int),
                ("warm_judge", C.c_int), ("overlap", C.c_int)]


class Report(C.Structure):
    _fields_ = [("status", C.c_int), ("sweeps", C.c_int), ("max_rank", C.c_int),
                ("ranks", C.c_int * (MAX_DIM + 1)), ("residual", C.c_double), ("time_ms", C.c_double),
                ("history_len", C.c_int), ("history_residual", C.c_double * MAX_HISTORY),
                ("history_local", C.c_double * MAX_HISTORY), ("history_max_rank", C.c_int * MAX_HISTORY),
                ("history_time_ms", C.c_double * MAX_HISTORY), ("precision", C.c_int),
                ("local_systems", C.c_int), ("refinement_steps", C.c_int), ("fp64_fallbacks", C.c_int),
                ("warm_start_used", C.c_int), ("warm_residual", C.c_double),
                ("cold_residual", C.c_double), ("refinement_capped", C.c_int), ("max_eig_cond", C.c_double),
                ("phase_ms", C.c_double * PHASES)]


class LibraryMissing(RuntimeError):
    pass


_lib = None


def lib() -> C.CDLL:
    """Load libt2s2.so from the package directory; fail loudly if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is missing: run paper_2506_04732_amd.build.build() first")
    # torch's HIP runtime must be the one in the process: libt2s2 resolves
    # libamdhip64.so.7 by soname, so loading torch first makes both share it
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p
    L.t2s2_last_error.restype = C.c_char_p
    L.t2s2_last_error.argtypes = []
    L.t2s2_nodes.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, dp, dp]
    L.t2s2_matrices_1d.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int, dp, dp, dp]
    L.t2s2_problem_create.argtypes = [C.c_int, ip, C.c_double, dp, C.c_int, C.c_int, C.POINTER(vp)]
    L.t2s2_problem_destroy.argtypes = [vp]
    L.t2s2_problem_create_reaction.argtypes = [C.c_int, ip, C.c_double, dp, C.c_double, C.c_int, C.c_int,
                                               C.POINTER(vp)]
    L.t2s2_problem_create_general.argtypes = [C.c_int, ip, ip, C.c_double, dp, ip, C.c_double, C.c_double,
                                              C.c_int, C.c_int, C.POINTER(vp)]
    L.t2s2_mol_create.argtypes = [C.c_int, ip, C.c_double, dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                  C.c_int, C.POINTER(vp)]
    L.t2s2_mol_step.argtypes = [vp, C.POINTER(TTStruct), C.POINTER(TTStruct), C.POINTER(Options),
                                C.POINTER(TTStruct), C.POINTER(Report), vp]
    L.t2s2_problem_operator.argtypes = [vp, C.POINTER(TTMStruct)]
    L.t2s2_problem_colloc.argtypes = [vp, C.c_int, dp]
    L.t2s2_tt_matvec.argtypes = [C.POINTER(TTMStruct), C.POINTER(TTStruct), C.POINTER(TTStruct), vp]
    L.t2s2_tt_matvec_noalloc.argtypes = [C.POINTER(TTMStruct), C.POINTER(TTStruct), C.POINTER(TTStruct), vp]
    L.t2s2_tt_norm.argtypes = [vp, C.POINTER(TTStruct), dp, vp]
    L.t2s2_tt_fiber.argtypes = [vp, C.POINTER(TTStruct), C.c_int, ip, vp, vp]
    L.t2s2_tt_residual_norm.argtypes = [vp, C.POINTER(TTStruct), C.POINTER(TTStruct), dp, vp]
    L.t2s2_tt_round.argtypes = [vp, C.POINTER(TTStruct), C.c_double, C.c_int, vp]
    L.t2s2_local_solve.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, C.c_int, vp]
    L.t2s2_solve.argtypes = [vp, C.POINTER(TTStruct), C.POINTER(TTStruct), C.POINTER(TTStruct),
                             C.POINTER(Options), C.POINTER(TTStruct), C.POINTER(Report), vp]
    ttp = C.POINTER(TTStruct)
    L.t2s2_solve_batched.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(ttp), C.POINTER(ttp), C.POINTER(ttp),
                                     C.POINTER(Options), C.POINTER(ttp), C.POINTER(Report), C.c_int, vp]
    L.t2s2_debug_iteration_limits.argtypes = [C.c_int, C.c_int]
    ll = C.c_longlong
    L.t2s2_debug_gemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, vp, ll,
                                  ll, vp, ll, ll, C.c_double, vp, ll, ll, vp]
    L.t2s2_gemm_tune_source.argtypes = []
    L.t2s2_gemm_tune_source.restype = C.c_char_p
    L.t2s2_debug_readback.argtypes = [vp, vp, ll, vp]
    fp, u64 = C.POINTER(C.c_float), C.c_ulonglong
    L.t2s2_mlp_create.argtypes = [C.c_int, ip, u64, C.POINTER(vp)]
    L.t2s2_mlp_destroy.argtypes = [vp]
    L.t2s2_mlp_destroy.restype = None
    L.t2s2_mlp_param_count.argtypes = [vp, C.POINTER(C.c_longlong)]
    L.t2s2_mlp_get_params.argtypes = [vp, vp, C.c_int, vp]
    L.t2s2_mlp_set_params.argtypes = [vp, vp, vp]
    L.t2s2_mlp_forward.argtypes = [vp, C.c_int, vp, vp, vp]
    L.t2s2_mlp_backward.argtypes = [vp, C.c_int, vp, vp, vp]
    L.t2s2_mlp_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.t2s2_mlp_infer_bf16.argtypes = [vp, C.c_int, vp, vp, vp]
    L.t2s2_mlp_train.argtypes = [vp, C.c_int, vp, vp, C.c_int, ip, C.c_int, C.c_int, C.c_int, C.c_float, u64, fp, vp]
    L.t2s2_tt_fit_loss.argtypes = [C.c_int, C.c_int, ip, C.c_int, vp, vp, vp, vp, vp]
    L.t2s2_tt_pack.argtypes = [C.POINTER(TTStruct), C.c_int, C.c_int, vp, vp]
    L.t2s2_tt_unpack.argtypes = [C.c_int, ip, C.c_int, vp, C.POINTER(TTStruct), vp]
    L.t2s2_source_gaussians.argtypes = [vp, C.c_int, dp, dp, dp, C.POINTER(TTStruct), vp]
    L.t2s2_source_manufactured.argtypes = [vp, C.POINTER(TTStruct), vp]
    L.t2s2_source_cross.argtypes = [vp, C.c_int, dp, C.c_double, C.c_int, C.c_int, u64, C.POINTER(TTStruct), ip, dp,
                                    vp]
    L.t2s2_default_options.argtypes = [C.POINTER(Options)]
    L.t2s2_default_options.restype = None
    L.t2s2_timing_enable.argtypes = [C.c_int]
    L.t2s2_timing_classes.argtypes = [C.c_uint]
    L.t2s2_timing_read.argtypes = [C.c_int, dp, C.POINTER(C.c_longlong), dp, dp]
    L.t2s2_timing_class_name.argtypes = [C.c_int]
    L.t2s2_timing_class_name.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("t2s2_last_error", "t2s2_default_options", "t2s2_timing_class_name", "t2s2_mlp_destroy",
                        "t2s2_gemm_tune_source"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class T2S2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libt2s2 error {code}: {msg}")
        self.code = code


def check(code: int, allow=()) -> int:
    if code != T2S2_OK and code not in allow:
        raise T2S2Error(code, lib().t2s2_last_error().decode())
    return code
