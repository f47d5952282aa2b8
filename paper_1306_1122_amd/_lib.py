"""ctypes declarations of the C ABI in include/dbie.h (argument marshalling only)."""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libdbie.so")

DBIE_OK, DBIE_E_INVAL, DBIE_E_DEVICE, DBIE_E_WORKSPACE, DBIE_E_UNSUPPORTED = 0, -1, -2, -3, -4
DBIE_FP64, DBIE_FP32C = 0, 1
DBIE_NELDER_MEAD, DBIE_LEVENBERG_MARQUARDT = 0, 1
DBIE_ST_CONVERGED, DBIE_ST_BUDGET, DBIE_ST_DEGENERATE, DBIE_ST_J_ZERO, DBIE_ST_NONFINITE = 0, 1, 2, 3, 4
DBIE_TRACE_FIELD, DBIE_TRACE_CURRENT = 0, 1


class dbie_boundary(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("x0", c_double), ("y0", c_double), ("h", c_double),
                ("B0", c_void_p)]


class dbie_problem(ctypes.Structure):
    _fields_ = [("n_boundaries", c_int32), ("boundaries", POINTER(dbie_boundary)), ("n_points", c_int64),
                ("xyz", c_void_p), ("seg", POINTER(c_int64))]


class dbie_options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("nearfield_radius_h", c_double), ("dv_over_dsigma_h", c_double),
                ("tune", c_int32), ("tune_cache", c_char_p), ("quad_points", c_int32),
                ("pixel_split", c_int32)]


class dbie_solve_opts(ctypes.Structure):
    _fields_ = [("method", c_int32), ("max_trials", c_int32), ("eps", c_double), ("init_step", c_double),
                ("lambda_cap", c_double), ("fp64_accept", c_int32), ("use_graph", c_int32),
                ("lm_radius", c_double), ("lm_damping", c_double)]


class dbie_lambda_grid(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("x0", c_double), ("y0", c_double),
                ("z0", c_double), ("dx", c_double), ("dy", c_double), ("dz", c_double), ("lam", c_void_p)]


# name -> (restype, argtypes)
SIGNATURES = {
    "dbie_default_options": (c_int32, [POINTER(dbie_options)]),
    "dbie_default_solve_opts": (c_int32, [POINTER(dbie_solve_opts)]),
    "dbie_init": (c_int32, [POINTER(c_void_p), POINTER(dbie_problem), POINTER(dbie_options), c_void_p]),
    "dbie_eval_field": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p]),
    "dbie_eval_field_scalar": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_void_p]),
    "dbie_eval_field_noalloc": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p]),
    "dbie_solve_lambda": (c_int32, [c_void_p, c_void_p, POINTER(dbie_solve_opts), c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p]),
    "dbie_grad": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                            c_void_p]),
    "dbie_timing": (c_int32, [c_void_p, c_int32]),
    "dbie_timing_read": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    "dbie_query": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32),
                             POINTER(c_int32), POINTER(c_int32)]),
    "dbie_query_tan": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "dbie_set_tile_shape": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_int32]),
    "dbie_query_persistent": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32)]),
    "dbie_solve_trace": (c_int32, [c_void_p, c_int32]),
    "dbie_query_split": (c_int32, [c_void_p, POINTER(c_int32)]),
    "dbie_query_tuned": (c_int32, [c_void_p, POINTER(c_int32)]),
    "dbie_residual_stats": (c_int32, [c_void_p, c_void_p, c_double, POINTER(c_double), c_void_p]),
    "dbie_workspace_bytes": (c_int64, [c_void_p]),
    "dbie_set_workspace": (c_int32, [c_void_p, c_void_p, c_int64]),
    "dbie_trace_lines": (c_int32, [c_void_p, POINTER(dbie_lambda_grid), POINTER(c_double), c_double, c_int32,
                                   c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    "dbie_solve_trace_read": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int32), c_int32,
                                        POINTER(c_int32), POINTER(c_double)]),
    "dbie_destroy": (None, [c_void_p]),
    "dbie_last_error": (c_char_p, [c_void_p]),
}

_lib = None


def load():
    """Load libdbie.so from the package directory; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError("libdbie.so is not built: run `python -m paper_1306_1122_amd.build` "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(LIBPATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
