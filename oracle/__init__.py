"""FP64 CPU oracle for the DBIE hot path.

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import, call or run anything in this package. It shares no code with the GPU library.
"""
from .dbie_oracle import (kernel, pixel_centres, field, field_only, field_fd, curl_div, residuals,
                          residual_jacobian, vjp, nelder_mead, NMResult, PointProblem,
                          default_nm_step, solve_point_nm, solve_point_lm, lm_direction, levenberg_marquardt,
                          field_quad9, ST_CONVERGED, ST_BUDGET, ST_DEGENERATE, ST_J_ZERO, ST_NONFINITE)
from .metrics import schrijver_metrics
from .trace import trilinear, dbie_direction, rk4_trace
