"""ctypes view of the C-ABI in include/fqp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfqp.so")

c_int32 = ctypes.c_int32
c_float = ctypes.c_float
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_size_t = ctypes.c_size_t

# status codes (fqp_status)
SOLVED, FEASIBLE_UNCERTIFIED, MAX_ITER, TIME_LIMIT, PRIMAL_INFEASIBLE, \
    INVALID_INPUT, NUMERICAL_ERROR = range(7)
STATUS_NAMES = {
    SOLVED: "certified", FEASIBLE_UNCERTIFIED: "feasible/non-certified",
    MAX_ITER: "iteration cap", TIME_LIMIT: "timeout",
    PRIMAL_INFEASIBLE: "primal infeasible", INVALID_INPUT: "invalid input",
    NUMERICAL_ERROR: "numerical failure",
}


class Universe(ctypes.Structure):
    _fields_ = [("n", c_int32), ("k", c_int32), ("n_groups", c_int32),
                ("B", c_void_p), ("f", c_void_p), ("d", c_void_p),
                ("group", c_void_p), ("n_half", c_int32), ("half", c_void_p)]


class Book(ctypes.Structure):
    _fields_ = [("m", c_int32), ("mu", c_void_p), ("w0", c_void_p),
                ("lb", c_void_p), ("ub", c_void_p), ("eligible", c_void_p),
                ("gamma", c_void_p), ("kappa", c_void_p), ("tau", c_void_p),
                ("band_lo", c_void_p), ("band_hi", c_void_p),
                ("tax_ptr", c_void_p), ("tax_asset", c_void_p),
                ("tax_brk", c_void_p), ("tax_slope", c_void_p),
                ("warm_state", c_void_p),
                ("lb_asset", c_void_p), ("ub_asset", c_void_p),
                ("half_lo", c_void_p), ("half_hi", c_void_p),
                ("wb", c_void_p), ("eta", c_void_p)]


class Settings(ctypes.Structure):
    _fields_ = [("eps_prim", c_double), ("eps_dual", c_double),
                ("eps_comp", c_double), ("max_iter", c_int32),
                ("check_every", c_int32), ("rho", c_float),
                ("rho_band", c_float), ("alpha", c_float),
                ("polish_rounds", c_int32),
                ("use_graph", c_int32), ("profile", c_int32),
                ("time_limit_ms", c_double), ("precision", c_int32),
                ("first_check", c_int32), ("warm_start", c_int32),
                ("debug_fail_alloc", c_int32), ("tile_rows", c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("w", c_void_p), ("status", c_void_p), ("iters", c_void_p),
                ("r_prim", c_void_p), ("r_dual", c_void_p),
                ("r_comp", c_void_p), ("obj", c_void_p), ("nu", c_void_p),
                ("lam_cap", c_void_p), ("lam_band", c_void_p),
                ("state", c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("iter_launches", c_int32),
                ("polish_calls", c_int32), ("n_solved", c_int32),
                ("iter_kernel_ms", c_double), ("account_iters", c_double),
                ("total_ms", c_double), ("workspace_bytes", c_size_t),
                ("polish_solves", c_int32), ("polish_gated", c_int32),
                ("contract_kernel_ms", c_double), ("phase_ms", c_double * 4),
                ("graph_reused", c_int32), ("workspace_requests", c_int32),
                ("prox_kernel_ms", c_double)]


def state_floats(m: int, n: int, n_rows: int) -> int:
    """Floats of an ADMM state block (fqp_book.warm_state / fqp_result.state);
    n_rows = n_groups + n_half."""
    return m * n + 2 * m * n_rows + m


EXPORTS = ("fqp_default_settings", "fqp_create", "fqp_solve_batch",
           "fqp_adjoint_batch", "fqp_adjoint_batch_noalloc", "fqp_get_stats", "fqp_get_pass_times", "fqp_error_string",
           "fqp_status_string", "fqp_last_error", "fqp_destroy")

_lib = None


def load(path: str = LIB_PATH):
    """Load libfqp.so; raises when it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    lib.fqp_default_settings.argtypes = [ctypes.POINTER(Settings)]
    lib.fqp_default_settings.restype = None
    lib.fqp_create.argtypes = [ctypes.POINTER(c_void_p), ctypes.c_int]
    lib.fqp_create.restype = ctypes.c_int
    lib.fqp_solve_batch.argtypes = [c_void_p, ctypes.POINTER(Universe),
                                    ctypes.POINTER(Book),
                                    ctypes.POINTER(Settings),
                                    ctypes.POINTER(Result), c_void_p]
    lib.fqp_solve_batch.restype = ctypes.c_int
    lib.fqp_adjoint_batch.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p]
    lib.fqp_adjoint_batch.restype = ctypes.c_int
    lib.fqp_adjoint_batch_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p,
                                              c_void_p]
    lib.fqp_adjoint_batch_noalloc.restype = ctypes.c_int
    lib.fqp_get_stats.argtypes = [c_void_p, ctypes.POINTER(Stats)]
    lib.fqp_get_stats.restype = ctypes.c_int
    lib.fqp_get_pass_times.argtypes = [c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(c_double), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.fqp_get_pass_times.restype = ctypes.c_int
    lib.fqp_error_string.argtypes = [ctypes.c_int]
    lib.fqp_error_string.restype = ctypes.c_char_p
    lib.fqp_status_string.argtypes = [ctypes.c_int]
    lib.fqp_status_string.restype = ctypes.c_char_p
    lib.fqp_last_error.argtypes = [c_void_p]
    lib.fqp_last_error.restype = ctypes.c_char_p
    lib.fqp_destroy.argtypes = [c_void_p]
    lib.fqp_destroy.restype = None
    _lib = lib
    return lib
