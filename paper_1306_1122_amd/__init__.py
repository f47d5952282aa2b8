"""MI355X (gfx950) library for the hot path of DBIE nonlinear force-free field extrapolation
(Wang, Yan & Tan, arXiv:1306.1122): the lambda-dependent half-space kernel sum against the boundary
magnetogram, its frozen-lambda gradient, the residuals f_i and g_i, the per-point lambda search and
the adjoint. The computation lives in libdbie.so (HIP, C ABI in include/dbie.h); this package is its
binding.
"""
from . import _lib
from .autograd import DbieField, dbie_field
from .dbie import (Context, DbieError, Field, dbie_default_options, dbie_default_solve_opts, dbie_destroy,
                   dbie_eval_field, dbie_eval_field_noalloc, dbie_eval_field_scalar, dbie_grad, dbie_init, dbie_last_error, dbie_query, dbie_solve_lambda,
                   dbie_timing, dbie_timing_read, split_gB0, dbie_query_tan, dbie_query_persistent, dbie_set_tile_shape,
                   dbie_solve_trace, dbie_solve_trace_read, dbie_trace_lines, dbie_query_split, dbie_query_tuned,
                   dbie_workspace_bytes, dbie_set_workspace, dbie_residual_stats)

__all__ = ["Context", "DbieError", "Field", "DbieField", "dbie_field", "dbie_init", "dbie_eval_field", "dbie_eval_field_noalloc", "dbie_eval_field_scalar", "dbie_solve_lambda", "dbie_grad",
           "dbie_timing", "dbie_timing_read", "dbie_query", "dbie_destroy", "dbie_last_error",
           "dbie_default_options", "dbie_default_solve_opts", "split_gB0", "dbie_query_tan", "dbie_query_persistent",
           "dbie_set_tile_shape", "dbie_solve_trace", "dbie_solve_trace_read", "dbie_trace_lines", "dbie_query_split", "dbie_query_tuned",
           "dbie_workspace_bytes", "dbie_set_workspace", "dbie_residual_stats"]
