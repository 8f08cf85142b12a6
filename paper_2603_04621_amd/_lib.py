"""ctypes view of libdualip.so (include/dualip.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdualip.so")

DL_OK = 0
DL_ERR_INVALID_ARG = 1
DL_ERR_UNSUPPORTED = 2
DL_ERR_OUT_OF_MEMORY = 3
DL_ERR_DEVICE = 4
DL_ERR_NUMERIC = 5
DL_ERR_NOT_CONVERGED = 6
DL_ERR_BUSY = 7
DL_ERR_NOT_FOUND = 8

DL_CSC, DL_CSR = 0, 1
DL_F64, DL_F32, DL_BF16_AC = 0, 1, 2
DL_TRACE_W = 6
DL_PRESET_CUSTOM, DL_PRESET_PAPER, DL_PRESET_NATURAL = 0, 1, 2
DL_NOALLOC_SCRATCH_BYTES = 64 << 20
PRESET = {"custom": DL_PRESET_CUSTOM, "paper": DL_PRESET_PAPER, "natural": DL_PRESET_NATURAL}

STORAGE = {"f64": DL_F64, "f32": DL_F32, "bf16": DL_BF16_AC}

c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_dbl = ctypes.c_double
c_ptr = ctypes.c_void_p


class ProblemDesc(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("nnz", c_i64), ("layout", ctypes.c_int),
                ("ptr", c_ptr), ("idx", c_ptr), ("val", c_ptr), ("c", c_ptr), ("b", c_ptr),
                ("num_blocks", c_i64), ("block_off", c_ptr), ("block_proj", c_ptr),
                ("upper", c_ptr)]


class ProblemOpts(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int), ("row_normalize", c_i32), ("primal_scale", c_i32),
                ("v", c_ptr), ("autotune", c_i32), ("deterministic", c_i32),
                ("lane_cap", c_i32), ("seg_rmax", c_i32), ("wg_min", c_i32),
                ("chunks_per_cu", c_i32)]


class Eval(ctypes.Structure):
    _fields_ = [(k, c_dbl) for k in ("g", "cx", "reg", "P", "rel_gap", "max_infeas")]


class SolveOpts(ctypes.Structure):
    _fields_ = [("gamma0", c_dbl), ("gamma_final", c_dbl), ("n_stages", c_i32),
                ("momentum", c_i32), ("stage_iters", c_i64), ("stage_tol", c_dbl),
                ("tol_rel_gap", c_dbl), ("max_iters", c_i64), ("check_every", c_i64),
                ("max_step", c_dbl), ("init_step", c_dbl), ("adaptive", c_i32),
                ("warm_start", c_i32), ("graph_iters", c_i32), ("time_kernels", c_i32),
                ("trace_host", c_ptr), ("preset", c_i32), ("reserved", c_i32)]


class SolveResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("converged", c_i32), ("stage", c_i32),
                ("iters", c_i64), ("gamma", c_dbl), ("g", c_dbl), ("P", c_dbl),
                ("rel_gap", c_dbl), ("max_infeas", c_dbl), ("seconds", c_dbl),
                ("grad_kernel_ms", c_dbl), ("grad_launches", c_i64),
                ("check_kernel_ms", c_dbl), ("check_launches", c_i64)]


class ProblemInfo(ctypes.Structure):
    _fields_ = [(k, c_i64) for k in ("m", "n", "num_blocks", "lane_groups", "seg_groups",
                                     "wg_blocks", "chunks", "lds_rows", "stream_bytes",
                                     "device_bytes")] + [(k, c_i32) for k in (
                    "storage", "has_box", "lane_cap", "seg_rmax", "chunks_per_cu", "tuned")] + [
                    ("anorm2", c_dbl), ("deterministic", c_i32), ("has_capped", c_i32),
                    ("col_entries", c_i32), ("wg_min", c_i32)]


# every symbol include/dualip.h declares
EXPORTS = [
    "dl_problem_opts_init", "dl_problem_validate", "dl_problem_create", "dl_problem_destroy",
    "dl_dual_grad", "dl_solve_opts_init", "dl_solve_opts_apply_preset", "dl_solve", "dl_batch_solve", "dl_server_create",
    "dl_server_submit", "dl_server_poll", "dl_server_times", "dl_server_destroy",
    "dl_problem_get_info", "dl_time_grad_kernel", "dl_status_str", "dl_last_error",
    "dl_dual_grad_noalloc",
]

_LIB = None


class DualipError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {status_str(status)} ({status}): {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built (no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.dl_problem_opts_init.argtypes = [P(ProblemOpts)]
        L.dl_problem_opts_init.restype = None
        L.dl_problem_validate.argtypes = [P(ProblemDesc), P(ProblemOpts)]
        L.dl_problem_create.argtypes = [P(ProblemDesc), P(ProblemOpts), c_ptr, P(c_ptr)]
        L.dl_problem_destroy.argtypes = [c_ptr]
        L.dl_dual_grad.argtypes = [c_ptr, c_ptr, c_dbl, c_ptr, c_ptr, P(Eval), c_ptr]
        L.dl_dual_grad_noalloc.argtypes = [c_ptr, c_ptr, c_dbl, c_ptr, c_ptr, P(Eval), c_ptr]
        L.dl_solve_opts_init.argtypes = [P(SolveOpts)]
        L.dl_solve_opts_init.restype = None
        L.dl_solve_opts_apply_preset.argtypes = [P(SolveOpts), c_dbl]
        L.dl_solve_opts_apply_preset.restype = ctypes.c_int
        L.dl_solve.argtypes = [c_ptr, P(SolveOpts), c_ptr, P(SolveResult), c_ptr]
        L.dl_batch_solve.argtypes = [P(c_ptr), c_i32, P(SolveOpts), P(c_ptr), P(SolveResult),
                                     c_ptr]
        L.dl_server_create.argtypes = [ctypes.c_size_t, c_i32, P(c_ptr)]
        L.dl_server_submit.argtypes = [c_ptr, P(ProblemDesc), P(ProblemOpts), P(SolveOpts),
                                       P(ctypes.c_uint64)]
        L.dl_server_poll.argtypes = [c_ptr, ctypes.c_uint64, P(c_i32), P(SolveResult), c_ptr]
        L.dl_server_times.argtypes = [c_ptr, ctypes.c_uint64, P(c_dbl), P(c_dbl), P(c_dbl)]
        L.dl_server_destroy.argtypes = [c_ptr]
        L.dl_problem_get_info.argtypes = [c_ptr, P(ProblemInfo)]
        L.dl_time_grad_kernel.argtypes = [c_ptr, c_ptr, c_dbl, c_i32, c_i32, P(c_dbl), c_ptr]
        L.dl_status_str.argtypes = [ctypes.c_int]
        L.dl_status_str.restype = ctypes.c_char_p
        L.dl_last_error.argtypes = []
        L.dl_last_error.restype = ctypes.c_char_p
        for name in ("dl_problem_validate", "dl_problem_create", "dl_problem_destroy",
                     "dl_dual_grad", "dl_dual_grad_noalloc", "dl_solve", "dl_batch_solve", "dl_server_create",
                     "dl_server_submit", "dl_server_poll", "dl_server_times",
                     "dl_server_destroy", "dl_problem_get_info", "dl_time_grad_kernel"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def status_str(s: int) -> str:
    return lib().dl_status_str(int(s)).decode()


def last_error() -> str:
    return lib().dl_last_error().decode()


def check(status: int, where: str, ok=(DL_OK,)) -> int:
    if status not in ok:
        raise DualipError(status, where, last_error())
    return status
