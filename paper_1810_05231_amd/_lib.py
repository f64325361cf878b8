"""ctypes declarations of the C interface in include/proxsdp.h.

Argument marshalling only: every computation happens inside libproxsdp.so.
Importing this module loads the library and raises if it has not been built
(``python -m paper_1810_05231_amd.build`` or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libproxsdp.so")

PROXSDP_OK = 0
PROXSDP_ERR_INVALID = -1
PROXSDP_ERR_WORKSPACE = -2
PROXSDP_ERR_HIP = -3
PROXSDP_ERR_UNSUPPORTED = -4

STATUS_RUNNING = 0
STATUS_CONVERGED = 1
STATUS_MAX_ITERS = 2
STATUS_TIME_LIMIT = 3
STATUS_NUMERICAL = 4
STATUS_EIG_NOT_CONVERGED = 5
STATUS_RANK_LIMIT = 6
STATUS_NAMES = {0: "running", 1: "converged", 2: "max_iters", 3: "time_limit", 4: "numerical",
                5: "eig_not_converged", 6: "rank_limit"}

RANK_TEST_LAMBDA_R = 0
RANK_TEST_LAMBDA_R_PLUS_1 = 1

FP64, FP32, BF16, IMPLICIT = 0, 1, 2, 3

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


class Problem(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("m", C.c_int32), ("p", C.c_int32),
        ("nnz_c", C.c_int64), ("c_i", _i32p), ("c_j", _i32p), ("c_v", _f64p),
        ("nnz_a", C.c_int64), ("a_row", _i32p), ("a_i", _i32p), ("a_j", _i32p), ("a_v", _f64p),
        ("n_r1", C.c_int32), ("r1_row", _i32p), ("r1_sigma", _f64p), ("r1_u", _f64p),
        ("b", _f64p), ("h", _f64p),
    ]


class Options(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("eps_lambda", C.c_double), ("alpha", C.c_double),
        ("window", C.c_int32), ("check_every", C.c_int32), ("r0", C.c_int32),
        ("r_max", C.c_int32), ("full_eig", C.c_int32), ("precision", C.c_int32),
        ("max_iters", C.c_int32), ("time_limit_s", C.c_double), ("row_scaling", C.c_int32),
        ("block", C.c_int32), ("eig_tol", C.c_double), ("max_passes", C.c_int32),
        ("seed", C.c_int32), ("eig_strict", C.c_int32), ("eig_rel", C.c_double), ("graphs", C.c_int32),
        ("rank_test", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("iters", C.c_int32), ("r", C.c_int32), ("k", C.c_int32),
        ("rank_updates", C.c_int32), ("passes", C.c_int32),
        ("lambda_r", C.c_double), ("lambda_r1", C.c_double),
        ("eps_p", C.c_double), ("eps_d", C.c_double), ("rho_p", C.c_double),
        ("rho_d", C.c_double), ("obj", C.c_double), ("dual_obj", C.c_double),
        ("alpha", C.c_double), ("norm_M", C.c_double), ("ritz_res", C.c_double),
        ("time_s", C.c_double), ("gap", C.c_double), ("rank_value", C.c_double),
        ("saved", C.c_int32), ("verify_steps", C.c_int32),
    ]

    def to_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1810_05231_amd/build.py "
                           "(the HIP library is required, there is no fallback)")
    # PyTorch ships its own HIP runtime; it has to be the one in the process
    # before libproxsdp's HIP dependency is resolved, otherwise two runtimes
    # get loaded and the second one finds no device.  Importing torch first
    # makes the library bind to the runtime torch's tensors and streams live in.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    H = C.c_void_p
    sig = {
        "proxsdp_default_options": (C.c_int, [C.POINTER(Options)]),
        "proxsdp_workspace_size": (C.c_int, [C.POINTER(Problem), C.POINTER(Options),
                                             C.POINTER(C.c_size_t)]),
        "proxsdp_create": (C.c_int, [C.POINTER(Problem), C.POINTER(Options), C.c_void_p,
                                     C.c_size_t, C.c_void_p, C.POINTER(H)]),
        "proxsdp_step": (C.c_int, [H, C.c_int32, C.POINTER(Info)]),
        "proxsdp_solve": (C.c_int, [H, C.POINTER(Info)]),
        "proxsdp_get_solution": (C.c_int, [H, C.c_void_p, C.c_void_p, C.c_int32]),
        "proxsdp_get_factors": (C.c_int, [H, _f64p, _f64p, _i32p]),
        "proxsdp_get_state": (C.c_int, [H, _f64p, _f64p, _f64p, _i32p]),
        "proxsdp_set_state": (C.c_int, [H, C.c_int32, _f64p, _f64p, _f64p]),
        "proxsdp_saved_count": (C.c_int, [H, _i32p]),
        "proxsdp_round_hyperplane": (C.c_int, [H, C.c_int32, _f64p, _f64p, C.POINTER(C.c_int8),
                                               _i32p]),
        "proxsdp_get_saved": (C.c_int, [H, C.c_int32, _f64p, _f64p, _f64p, _i32p, _i32p]),
        "proxsdp_destroy": (None, [H]),
        "proxsdp_project_workspace_size": (C.c_int, [C.c_int32, C.c_int32, C.c_int32,
                                                     C.POINTER(C.c_size_t)]),
        "proxsdp_project_psd": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32,
                                          C.c_int32, C.c_double, C.c_void_p, C.c_int64,
                                          _f64p, _f64p, _i32p, C.c_void_p, C.c_size_t,
                                          C.c_void_p]),
        "proxsdp_project_psd_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int32,
                                                  C.c_int32, C.c_double, C.c_void_p, C.c_int64,
                                                  _f64p, _f64p, _i32p, C.c_void_p]),
        "proxsdp_reset": (C.c_int, [H]),
        "proxsdp_profile_enable": (C.c_int, [H, C.c_int32]),
        "proxsdp_profile_read": (C.c_int, [H, _f64p, _i32p, _f64p, _i32p]),
        "proxsdp_profile_totals": (C.c_int, [H, _f64p, C.c_int32]),
        "proxsdp_step_many": (C.c_int, [C.POINTER(H), C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
        "proxsdp_debug_scalars": (C.c_int, [H, _f64p, C.c_int32]),
        "proxsdp_rank_path": (C.c_int, [H, _i32p, _i32p, _i32p, C.c_int32, _i32p]),
        "proxsdp_last_error": (C.c_char_p, []),
        "proxsdp_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class ProxSDPError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib.proxsdp_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with code {code}: {msg}")
        self.code = code


def check(code: int, where: str) -> None:
    if code != PROXSDP_OK:
        raise ProxSDPError(code, where)


def default_options(**over) -> Options:
    o = Options()
    check(lib.proxsdp_default_options(C.byref(o)), "proxsdp_default_options")
    for k, v in over.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, v)
    return o
