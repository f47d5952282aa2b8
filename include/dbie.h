/*
 * dbie.h - C ABI of the MI355X (gfx950) library for the hot path of direct boundary integral
 * equation (DBIE) nonlinear force-free field extrapolation (Wang, Yan & Tan, arXiv:1306.1122).
 *
 * What it computes (Section 2.1 of the paper):
 *   For every evaluation point i above the boundary z = 0 and every component p in {x, y, z},
 *     B_p(i) = sum_k h^2 K(lambda_pi; x_k - x_i, y_k - y_i, z_i) B0_p(k)                (Eq. 16)
 *     K(lambda; dx, dy, z) = z [lambda r sin(lambda r) + cos(lambda r)] / (2 pi r^3)       (Eq. 6)
 *   with r^2 = dx^2 + dy^2 + z^2 and the sum over the pixel centres k of the magnetogram (the field
 *   outside the magnetogram is zero, Eq. 3 and the text around it). The gradient of B_p with respect
 *   to the point is taken at frozen lambda (the zeroth-order expansion of lambda around the point,
 *   Eq. 13, in its exact delta -> 0 limit). From B and grad B follow J = curl B (Eq. 14) and the two
 *   residuals f_i = |J x B| / (|J||B|) (Eq. 8) and g_i = |div B| dV / (|B| dSigma) (Eq. 9). The
 *   lambda search drives them below a threshold (Eq. 12).
 *
 * Conventions for every call:
 *   - Every device buffer is CALLER-OWNED (e.g. allocated as a PyTorch tensor) unless stated. The
 *     library owns only the opaque context and the device memory it allocates in dbie_init.
 *   - All arrays are structure-of-arrays, component-major, C order. "[3][N]" means 3 rows of N.
 *   - Lengths are in one physical unit (pixels or any other); lambda is in inverse length units.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream). Calls enqueue work on
 *     it and return without synchronising, except where stated (dbie_init, dbie_solve_lambda).
 *   - Return codes: DBIE_OK, or a negative DBIE_E_* code with a message in dbie_last_error(ctx).
 *     Argument checks run on the host before anything is enqueued. No call aborts or throws.
 *     Per-point outcomes go into per-point status arrays, never into the return code.
 *   - One context must not be used from two host threads at once.
 *   - A context lives on the HIP device that was current at dbie_init; every call that enqueues
 *     work needs that device current and returns DBIE_E_INVAL otherwise.
 */
#ifndef DBIE_H
#define DBIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DBIE_API __attribute__((visibility("default")))

typedef struct dbie_ctx dbie_ctx;

/* return codes */
enum {
    DBIE_OK = 0,
    DBIE_E_INVAL = -1,       /* invalid argument (message says which) */
    DBIE_E_DEVICE = -2,      /* a HIP call failed */
    DBIE_E_WORKSPACE = -3,   /* device memory could not be allocated */
    DBIE_E_UNSUPPORTED = -4  /* valid request this library does not support */
};

/* precision of the bulk pixel sum */
enum {
    DBIE_FP64 = 0,   /* every pair in FP64 */
    DBIE_FP32C = 1   /* far pairs in FP32 with compensated (cascaded FP64) accumulation; pairs with
                        r < nearfield_radius * h in FP64; residuals in FP64 */
};

/* lambda-update method of dbie_solve_lambda */
enum {
    DBIE_NELDER_MEAD = 0,          /* derivative-free downhill simplex on Phi = f^2 + g^2 (Section 2.1) */
    DBIE_LEVENBERG_MARQUARDT = 1   /* gradient form: LM in mu = lambda^2 with the mu-tangents */
};

/* per-point status */
enum {
    DBIE_ST_CONVERGED = 0,   /* max(f, g) <= eps (Eq. 12) at the returned lambda */
    DBIE_ST_BUDGET = 1,      /* trial budget spent; the best lambda found is returned */
    DBIE_ST_DEGENERATE = 2,  /* |B| = 0: f and g undefined */
    DBIE_ST_J_ZERO = 3,      /* |J| = 0: f set to 0 (only reported by evaluation, not by a solve) */
    DBIE_ST_NONFINITE = 4    /* a non-finite value appeared (input lambda or overflow) */
};

/* One magnetogram: pixel (a, b) has centre (x0 + a h, y0 + b h, 0), a in [0, nx), b in [0, ny).
 * B0 is a DEVICE pointer to double [3][ny][nx] (Bx, By, Bz planes, x fastest). It is copied in
 * dbie_init; the caller may free it afterwards. */
typedef struct {
    int32_t nx, ny;
    double x0, y0, h;
    const double* B0;
} dbie_boundary;

/* The problem: n_boundaries magnetograms (host array `boundaries`) and n_points evaluation points.
 * xyz is a DEVICE pointer to double [3][n_points] (x, y, z rows) with z > 0; it is copied in
 * dbie_init. seg is a HOST array of n_boundaries + 1 non-decreasing offsets with seg[0] = 0 and
 * seg[n_boundaries] = n_points: points [seg[b], seg[b+1]) belong to boundary b. seg may be NULL
 * when n_boundaries == 1. */
typedef struct {
    int32_t n_boundaries;
    const dbie_boundary* boundaries;
    int64_t n_points;
    const double* xyz;
    const int64_t* seg;
} dbie_problem;

typedef struct {
    int32_t precision;           /* DBIE_FP64 or DBIE_FP32C */
    double nearfield_radius_h;   /* FP32C only: pairs with r < this * h are summed in FP64; in [0, 2] */
    double dv_over_dsigma_h;     /* dV / dSigma of Eq. 9 in units of h (1/6: cube of side h) */
    int32_t tune;                /* 1: choose the FP32C tile shapes (points per lane, waves per
                                  * workgroup, rows of the LDS pixel block, grid or persistent form)
                                  * and, when the point tiles alone
                                  * cannot fill the device, the pixel split, by timing the bulk kernel at
                                  * init on the largest tiles at lambda spread over |lambda| < 4 pi / L.
                                  * Choices are reused within the process for contexts of the same
                                  * device architecture, quadrature and size bucket (floor(log2) of the
                                  * point count and of the mean quadrature points per magnetogram). */
    const char* tune_cache;      /* optional path of a text cache of tuned choices, read before timing
                                  * and appended to after (lines: arch quad_points log2N log2pixels tan
                                  * ppl waves tile_pixels persistent split); NULL: none */
    int32_t quad_points;         /* 0: nodal sum over the pixel centres, weight h^2 (Eq. 16).
                                  * 2, 3 or 4: 9-node quadratic elements (Eq. 15), each element
                                  * integral by quad_points x quad_points Gauss-Legendre points; every
                                  * magnetogram then needs odd nx, ny >= 3 (element (m, n) holds the
                                  * nodes 2m..2m+2 x 2n..2n+2). With DBIE_FP32C the elements
                                  * that come closer than nearfield_radius_h * h to a point (3 x 3
                                  * element window) are summed in FP64, every other pair in FP32. */
    int32_t pixel_split;         /* pixel slices per launch (grid z), each summing an even share of
                                  * the magnetogram's blocks into its own partial, added in order by the
                                  * finalize pass. 0 = automatic (about four workgroups per compute
                                  * unit when the point tiles alone are fewer, else 1), 1..32 fixed.
                                  * The slicing changes the FP64 summation grouping only (results
                                  * agree to ~1e-16 relative; bitwise equal for equal slicing). */
} dbie_options;

typedef struct {
    int32_t method;       /* DBIE_NELDER_MEAD or DBIE_LEVENBERG_MARQUARDT */
    int32_t max_trials;   /* budget of evaluations per point (>= 1) */
    double eps;           /* convergence: max(f, g) <= eps (Eq. 12) */
    double init_step;     /* simplex edge (Nelder-Mead); <= 0 means 1 / (longer side of the magnetogram) */
    double lambda_cap;    /* |lambda| <= cap; <= 0 means pi / h */
    int32_t fp64_accept;  /* FP32C contexts: re-evaluate the result in FP64 and set status from it
                             (with B and fg both NULL only the points that converged are re-evaluated,
                             and those that fail the FP64 test become DBIE_ST_BUDGET) */
    int32_t use_graph;    /* 1: replay the rounds from a captured HIP graph (bitwise the same results) */
    double lm_radius;     /* Levenberg-Marquardt trust radius in lambda at the start: every proposal keeps
                             each sqrt(mu_p) within the radius of the accepted point's (and in [0, cap]);
                             the radius doubles on acceptance (up to the cap) and halves on rejection.
                             0 means the simplex edge (init_step, or 1 / the longer side); +inf means no
                             trust region (proposals only clipped to [0, cap^2]); negative or NaN is
                             DBIE_E_INVAL. Not used by Nelder-Mead. */
    double lm_damping;    /* Levenberg-Marquardt initial damping nu0: each step solves
                             (J^T J + nu diag(J^T J)) d = -J^T u, nu is divided by 10 on acceptance and
                             multiplied by 10 on rejection. 0 means 1; negative, NaN or infinite is
                             DBIE_E_INVAL. Not used by Nelder-Mead. */
} dbie_solve_opts;

/* Fill defaults: FP32C, radius 2, dV/dSigma = 1/6, no tuning, nodal sum / Nelder-Mead, 50 trials, eps 1e-4,
 * default step and cap, FP64 acceptance on, graph replay on, LM trust radius = the simplex edge, LM
 * initial damping 1. Return
 * DBIE_OK, or DBIE_E_INVAL for NULL. */
DBIE_API int dbie_default_options(dbie_options* opt);
DBIE_API int dbie_default_solve_opts(dbie_solve_opts* opt);

/* Create a context on the current HIP device. It stages the problem of Section 2.1: the boundary
 * condition B = B0 on z = 0 with the field zero outside the magnetogram (Eq. 3 and the text around
 * it), so that the sums of Eq. 16 run over the given pixels only (with quad_points > 0, over the
 * Gauss points of the Eq. 15 elements, whose weighted field is formed here), and the evaluation
 * points above the boundary. It copies B0 and xyz into library-owned device memory (B0 also as FP32
 * blocks for DBIE_FP32C), validates the points (z > 0 and finite; checked on the device, then
 * synchronised), classifies the near-field pairs and builds the tile schedules (timing shapes when
 * opt->tune). `opt` may be NULL (defaults). On failure *out is NULL. Synchronises `stream`. */
DBIE_API int dbie_init(dbie_ctx** out, const dbie_problem* prob, const dbie_options* opt, void* stream);

/* Evaluate L lambda trials at every point (Eqs. 6, 13, 14, 8, 9).
 *   lambda : device double [L][3][N]            (input)
 *   B      : device double [L][3][N]            (output, required)
 *   dB     : device double [L][9][N] or NULL    (dB[3p+q] = d B_p / d x_q at frozen lambda)
 *   fg     : device double [L][2][N] or NULL    (f_i, g_i; NaN for a DEGENERATE point)
 *   tan    : device double [L][12][N] or NULL   (d/d mu_p, mu = lambda^2, of the rows B_p and
 *                                                dB_p/dx_q: tan[p] and tan[3 + 3p + q])
 * L >= 1. A non-finite lambda gives non-finite outputs for that point only. In an FP32C context the
 * call with tan != NULL runs the tangent variant of the kernel, whose B and dB agree with the call
 * without tangents to FP32 rounding (not bit for bit). */
DBIE_API int dbie_eval_field(dbie_ctx* ctx, const double* lambda, int32_t L, double* B, double* dB,
                             double* fg, double* tan, void* stream);

/* dbie_eval_field for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments, outputs and kernels,
 * but the partial sums of the bulk pass live in a static device array of 64 MiB that the library
 * holds on every device it runs on until the process ends, instead of the context's accumulator.
 * The call allocates nothing (no hipMalloc / hipFree, no events) and records no kernel timing.
 * Limit: L * n_points <= 399457 (21 doubles per point and trial); larger requests return
 * DBIE_E_INVAL with a message. The pixel slices are the context's, or fewer if the array cannot hold
 * them for L trials (results then differ from dbie_eval_field's in FP64 summation order only, ~1e-16
 * relative; bitwise equal otherwise). All calls on one device share the array: calls that overlap
 * on one device (two streams, two host threads, two contexts) race and give wrong results. Nothing in
 * the array has to start at zero: every call writes each partial sum before reading it. */
DBIE_API int dbie_eval_field_noalloc(dbie_ctx* ctx, const double* lambda, int32_t L, double* B, double* dB,
                                     double* fg, double* tan, void* stream);

/* dbie_eval_field with one lambda shared by the three components at each point (lambda_x = lambda_y
 * = lambda_z, e.g. a linear force-free trial): lambda is device double [L][N]; the outputs are those of
 * dbie_eval_field (tan rows are d/d mu of each row for the shared mu = lambda^2). The FP32C bulk sum
 * then computes one sin/cos pair per kernel pair instead of three. */
DBIE_API int dbie_eval_field_scalar(dbie_ctx* ctx, const double* lambda, int32_t L, double* B, double* dB,
                                    double* fg, double* tan, void* stream);

/* Per-point lambda search (Section 2.1, Eqs. 8-12), all points at once, device resident.
 *   lambda_inout : device double [3][N]; start values in, |lambda*| out
 *   B, fg        : device double [3][N] / [2][N] or NULL: field and (f, g) at lambda*
 *   status       : device int32 [N] (DBIE_ST_*), required
 *   trials       : device int32 [N] evaluations used per point, required
 * One trial is one evaluation of (B, grad B) at one lambda triple for one point. Nelder-Mead uses the
 * simplex {lambda0, lambda0 + step e_p}, coefficients 1, 2, 1/2, 1/2; a proposal outside the cap
 * costs a trial and counts as Phi = +inf. LM starts at mu = lambda0^2. The host reads one active-point
 * count per few rounds (synchronising `stream`), and the number of converged points once more before an
 * FP64 confirmation, and returns when every point is done. The rounds
 * between two reads are captured once into a HIP graph per context and configuration and replayed
 * (not while timing or tracing is enabled). With the environment variable DBIE_PROGRESS set, the host
 * reports the round and the active-point count on stderr at those reads, at most every 20 s. */
DBIE_API int dbie_solve_lambda(dbie_ctx* ctx, double* lambda_inout, const dbie_solve_opts* opt,
                               double* B, double* fg, int32_t* status, int32_t* trials, void* stream);

/* Adjoint of dbie_eval_field at one lambda triple per point (L = 1), for a loss with gradients
 * gB = dLoss/dB [3][N] and gdB = dLoss/d(dB) [9][N] (either may be NULL = zero):
 *   glambda   : device double [3][N] or NULL   dLoss/dlambda at frozen B0
 *   gB0       : device double, concatenation over boundaries of [3][ny][nx], or NULL
 *               dLoss/dB0 (the transpose of Eq. 16 and its gradient rows); overwritten
 *   resid_jac : device double [4][3][N] or NULL  d(u)/d(mu), u = (J x B / (|J||B|), sign(div B) g)
 * Deterministic: no floating-point atomics. */
DBIE_API int dbie_grad(dbie_ctx* ctx, const double* lambda, const double* gB, const double* gdB,
                       double* glambda, double* gB0, double* resid_jac, void* stream);

/* Kernel timing with HIP events on the caller's stream (for benchmarks). enable != 0 starts
 * recording around every bulk field-sum launch; dbie_timing_read synchronises, returns the summed
 * milliseconds and the launch count since the last read, and clears them. */
DBIE_API int dbie_timing(dbie_ctx* ctx, int32_t enable);
DBIE_API int dbie_timing_read(dbie_ctx* ctx, double* total_ms, int64_t* launches);

/* Choose the FP32C tile shape (points per lane, waves per workgroup, tile_pixels = 8 x the rows of the
 * LDS pixel block, 16, 32 or 64 (a block spans 16 columns of a nodal magnetogram, 8 of an element
 * grid), and persistent != 0 for a persistent grid that pulls tiles from a device counter) for both
 * the plain pass and the pass with tangents. Only the shapes the library
 * was built with are accepted: (1, 2, 256), (1, 4, 256), (1, 8, 256), (2, 4, 256), (1, 4, 128),
 * (1, 4, 512) (DBIE_E_UNSUPPORTED otherwise; DBIE_E_UNSUPPORTED for an FP64 context). */
DBIE_API int dbie_set_tile_shape(dbie_ctx* ctx, int32_t ppl, int32_t waves, int32_t tile_pixels,
                                 int32_t persistent);

/* Solve tracing (time to solution): with enable != 0, dbie_solve_lambda records a HIP event on its
 * stream at the start, after every round and at its end (after the FP64 acceptance pass).
 * dbie_solve_trace_read synchronises and returns, for the last solve, the elapsed milliseconds at
 * the end of each round (t_ms) and the number of points that converged in each round (converged),
 * for up to max_rounds rounds; *n_rounds = rounds run; *t_end_ms = elapsed milliseconds at the end
 * of the call. Any output pointer may be NULL. DBIE_E_INVAL for max_rounds < 0, and for converged
 * != NULL when the last traced solve returned an error; dbie_set_workspace discards the trace. */
DBIE_API int dbie_solve_trace(dbie_ctx* ctx, int32_t enable);
DBIE_API int dbie_solve_trace_read(dbie_ctx* ctx, double* t_ms, int32_t* converged, int32_t max_rounds,
                                   int32_t* n_rounds, double* t_end_ms);

/* Sizes the context was built with: n_points, total pixels, FP32C tile shape (points per lane,
 * waves per workgroup, tile_pixels as in dbie_set_tile_shape) as chosen by defaults or the tuner.
 * Any pointer may be NULL. */
DBIE_API int dbie_query(const dbie_ctx* ctx, int64_t* n_points, int64_t* n_pixels, int32_t* ppl,
                        int32_t* waves, int32_t* tile_pixels);
/* The tile shape of the FP32C pass with mu-tangents (the LM solver's pass), and whether each pass
 * runs in the persistent form. */
DBIE_API int dbie_query_tan(const dbie_ctx* ctx, int32_t* ppl, int32_t* waves, int32_t* tile_pixels);
DBIE_API int dbie_query_persistent(const dbie_ctx* ctx, int32_t* plain, int32_t* with_tangents);
/* Residual statistics of a reconstruction (the paper quotes the means of f_i and g_i, Eqs. 8-9, over
 * its volume, Section 4): fg is device double [2][N] as written by dbie_eval_field or
 * dbie_solve_lambda; out is host double[4] = {<f>, <g>, number of points with finite f and g,
 * number of points with max(f, g) <= eps (Eq. 12)}, the means over the finite points (NaN if none).
 * Wavefront shuffles and a fixed-order block sum: deterministic. Synchronises `stream`. */
DBIE_API int dbie_residual_stats(dbie_ctx* ctx, const double* fg, double eps, double* out, void* stream);

/* Where the context's FP32C shapes came from: 0 defaults (no tuning), 1 timed by its dbie_init, 2 reused
 * from an earlier context of this process with the same key, 3 read from the tune_cache file. */
DBIE_API int dbie_query_tuned(const dbie_ctx* ctx, int32_t* source);

/* Pixel slices per launch of the bulk sum (dbie_options.pixel_split, the tuner's or the automatic
 * choice). */
DBIE_API int dbie_query_split(const dbie_ctx* ctx, int32_t* slices);

/* Caller-owned work memory (no operation of the paper: device-memory plumbing for callers that manage
 * their own pools). dbie_workspace_bytes returns the bytes one workspace needs for every call on this
 * context with one trial per evaluation (L = 1): dbie_eval_field(_scalar), dbie_solve_lambda with
 * either method and up to 1e6 trials, dbie_grad and dbie_trace_lines (DBIE_E_INVAL for NULL). The
 * figure depends on the tile shape: ask again after dbie_set_tile_shape.
 * dbie_set_workspace hands the context `dev` (device memory, 256-byte aligned, >= that many bytes;
 * else DBIE_E_INVAL / DBIE_E_WORKSPACE); the library frees the work memory it had allocated itself
 * (after synchronising the device) and allocates none after that: a call needing more (L > 1 trials)
 * returns DBIE_E_WORKSPACE. dev = NULL goes back to library-allocated work memory. The buffer stays
 * the caller's: it must outlive its use by the context (until replaced or dbie_destroy), and calls on
 * one context must not overlap. */
DBIE_API int64_t dbie_workspace_bytes(const dbie_ctx* ctx);
DBIE_API int dbie_set_workspace(dbie_ctx* ctx, void* dev, int64_t bytes);

/* Field-line tracing (the paper's field-line figures; current lines from J = curl B, Eq. 14).
 * Lambda at a point comes from trilinear interpolation of a regular grid (coordinates clamped to
 * the grid): node (i, j, k) at (x0 + i dx, y0 + j dy, z0 + k dz), lambda device double [3][nz][ny][nx]
 * (lambda_x, lambda_y, lambda_z planes); nx = ny = nz = 1 gives one constant lambda triple. */
typedef struct {
    int32_t nx, ny, nz;
    double x0, y0, z0;
    double dx, dy, dz;
    const double* lambda;
} dbie_lambda_grid;

enum { DBIE_TRACE_FIELD = 0, DBIE_TRACE_CURRENT = 1 };

/* Trace one line from each point of the context (the seeds) by fourth-order Runge-Kutta in arc length
 * with step ds (length units): dx/ds = sense * v / |v|, v = B (DBIE_TRACE_FIELD) or v = curl B at
 * frozen lambda (DBIE_TRACE_CURRENT), sense = +1 or -1. Every stage evaluates the context's own
 * discretisation and precision at the stage points (geometry and near field re-classified on the
 * device). A line stops, keeping its last point, when one of a step's four stage points would leave
 * box = {x_lo, y_lo, z_lo, x_hi, y_hi, z_hi} (z_lo > 0) or its direction is undefined; a seed
 * outside the box gives a line of one point.
 *   xyz_out : device double [n_steps + 1][3][N]; point k of line i at [k][0..2][i], NaN after the end
 *   count   : device int32 [N], points per line (>= 1)
 * The context's points are moved during the call and restored before it returns, also when it
 * fails; the call synchronises `stream`. Uses the context's workspace (not concurrently with other
 * calls on it). DBIE_E_INVAL for an output of more than 2^34 values ((n_steps + 1) x 3 x N). */
DBIE_API int dbie_trace_lines(dbie_ctx* ctx, const dbie_lambda_grid* lambda_grid, const double* box, double ds,
                              int32_t n_steps, int32_t mode, double sense, double* xyz_out, int32_t* count,
                              void* stream);

/* Free the context and every device allocation the library made for it (not the caller's workspace);
 * the caller makes sure no work enqueued with it is still running. NULL is a no-op. */
DBIE_API void dbie_destroy(dbie_ctx* ctx);

/* Message of the last failure on ctx (or of the last failed dbie_init when ctx is NULL). */
DBIE_API const char* dbie_last_error(const dbie_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DBIE_H */
