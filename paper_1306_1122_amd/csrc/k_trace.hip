// Field-line and current-line tracing through the DBIE field (dbie_trace_lines).
//
// Every line advances by the classical fourth-order Runge-Kutta step in arc length s with the unit
// direction sense * v / |v|, v = B (field lines) or v = curl B at frozen lambda (Eq. 14; current
// lines). Each of the four stages moves the context's points to the stage positions, re-runs the
// per-point geometry and near-field classification, interpolates lambda trilinearly from the given
// grid, and evaluates the field with the context's bulk kernels: the lines are traced through the
// DBIE field itself, not through an interpolated copy of it. All lines advance together; nothing is
// read back to the host inside the loop. A line stops, keeping its last point, when a step would put
// one of its stage points outside the box or its direction is undefined.
#include <algorithm>
#include <cmath>

#include "dbie_solver.h"

namespace dbie {

struct LamGrid {
    int32_t nx, ny, nz;
    double x0, y0, z0, dx, dy, dz;
    const double* lam;
};

struct Box {
    double lo[3], hi[3];
};

__device__ __forceinline__ bool inside(const Box& b, double x, double y, double z) {
    return x >= b.lo[0] && x <= b.hi[0] && y >= b.lo[1] && y <= b.hi[1] && z >= b.lo[2] && z <= b.hi[2];
}

// Trilinear interpolation with the coordinates clamped to the grid; cell index clamped to n - 2.
__device__ __forceinline__ void axis_cell(double x, double x0, double d, int32_t n, int32_t& i, double& f) {
    double t = (x - x0) / d;
    t = fmin(fmax(t, 0.0), (double)(n - 1));
    i = (int32_t)floor(t);
    i = min(i, max(n - 2, 0));
    f = n > 1 ? t - (double)i : 0.0;
}

__device__ __forceinline__ void interp_lambda(const LamGrid& g, double x, double y, double z, double lam[3]) {
    int32_t ix, iy, iz;
    double fx, fy, fz;
    axis_cell(x, g.x0, g.dx, g.nx, ix, fx);
    axis_cell(y, g.y0, g.dy, g.ny, iy, fy);
    axis_cell(z, g.z0, g.dz, g.nz, iz, fz);
    const int32_t ix1 = min(ix + 1, g.nx - 1), iy1 = min(iy + 1, g.ny - 1), iz1 = min(iz + 1, g.nz - 1);
    const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny, sc = sz * g.nz;
    for (int p = 0; p < 3; ++p) {
        const double* G = g.lam + p * sc;
        auto at = [&](int32_t k, int32_t j, int32_t i) { return G[k * sz + j * sy + i]; };
        const double c00 = at(iz, iy, ix) * (1 - fx) + at(iz, iy, ix1) * fx;
        const double c01 = at(iz, iy1, ix) * (1 - fx) + at(iz, iy1, ix1) * fx;
        const double c10 = at(iz1, iy, ix) * (1 - fx) + at(iz1, iy, ix1) * fx;
        const double c11 = at(iz1, iy1, ix) * (1 - fx) + at(iz1, iy1, ix1) * fx;
        lam[p] = (c00 * (1 - fy) + c01 * fy) * (1 - fz) + (c10 * (1 - fy) + c11 * fy) * fz;
    }
}

__global__ void k_trace_init(int64_t N, const double* __restrict__ seeds, Box box, int64_t total,
                             double* __restrict__ out, int32_t* __restrict__ count, int32_t* __restrict__ alive,
                             double* __restrict__ x) {
    // grid-stride: the output (up to 2^34 values) can exceed one launch's 2^32 work-items
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        if (e >= 3 * N) {
            out[e] = __builtin_nan("");
            continue;
        }
        if (e >= N) continue;
        for (int p = 0; p < 3; ++p) {
            x[p * N + e] = seeds[p * N + e];
            out[p * N + e] = seeds[p * N + e];
        }
        count[e] = 1;
        alive[e] = inside(box, seeds[e], seeds[N + e], seeds[2 * N + e]) ? 1 : 0;
    }
}

// Stage st (0..3) positions y = x + c_st ds k_prev (c = 0, 1/2, 1/2, 1); a line whose stage point
// leaves the box is marked to stop (ok = 0) and is evaluated at x instead. Writes the point to
// evaluate and its lambda.
__device__ __forceinline__ void trace_stage(int64_t i, int64_t N, int st, double ds, const Box& box, const LamGrid& g,
                                            const double* __restrict__ x, const double* __restrict__ kprev,
                                            const int32_t* __restrict__ alive, int32_t* __restrict__ ok,
                                            double* __restrict__ pts, double* __restrict__ lam) {
    double y[3];
    int32_t k = st == 0 ? alive[i] : ok[i];
    const double c = st == 3 ? ds : 0.5 * ds;
    for (int p = 0; p < 3; ++p) y[p] = st == 0 ? x[p * N + i] : x[p * N + i] + c * kprev[p * N + i];
    if (!inside(box, y[0], y[1], y[2])) k = 0;
    if (!k)
        for (int p = 0; p < 3; ++p) y[p] = x[p * N + i];
    ok[i] = k;
    for (int p = 0; p < 3; ++p) pts[p * N + i] = y[p];
    double l[3];
    interp_lambda(g, y[0], y[1], y[2], l);
    for (int p = 0; p < 3; ++p) lam[p * N + i] = l[p];
}

// Direction of stage st from the evaluated field: kprev = sense v / |v|; ksum accumulates
// k1 + 2 k2 + 2 k3 + k4 in that order.
__device__ __forceinline__ void trace_dir(int64_t i, int64_t N, int st, double sense, int current,
                                          const double* __restrict__ B, const double* __restrict__ dB,
                                          double* __restrict__ kprev, double* __restrict__ ksum) {
    double v[3];
    if (current) {
        v[0] = dB[7 * N + i] - dB[5 * N + i];
        v[1] = dB[2 * N + i] - dB[6 * N + i];
        v[2] = dB[3 * N + i] - dB[1 * N + i];
    } else {
        for (int p = 0; p < 3; ++p) v[p] = B[p * N + i];
    }
    const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int p = 0; p < 3; ++p) {
        const double d = sense * (v[p] / n);
        kprev[p * N + i] = d;
        if (st == 0) ksum[p * N + i] = d;
        else if (st == 3) ksum[p * N + i] = ksum[p * N + i] + d;
        else ksum[p * N + i] = ksum[p * N + i] + 2.0 * d;
    }
}

// x <- x + ds/6 (k1 + 2 k2 + 2 k3 + k4) for the lines still going; record point `step`.
__device__ __forceinline__ void trace_advance(int64_t i, int64_t N, int32_t step, double ds,
                                              const int32_t* __restrict__ ok, const double* __restrict__ ksum,
                                              int32_t* __restrict__ alive, double* __restrict__ x,
                                              double* __restrict__ out, int32_t* __restrict__ count) {
    double xn[3];
    bool good = ok[i] != 0;
    for (int p = 0; p < 3; ++p) {
        xn[p] = x[p * N + i] + ds / 6.0 * ksum[p * N + i];
        good = good && isfinite(xn[p]);
    }
    alive[i] = good ? 1 : 0;
    if (good) {
        for (int p = 0; p < 3; ++p) {
            x[p * N + i] = xn[p];
            out[((int64_t)step * 3 + p) * N + i] = xn[p];
        }
        count[i] += 1;
    }
}

// The per-line work between two evaluations in one launch, in this order: the direction of stage
// dir_st (>= 0) from the field just evaluated, the advance of step adv_step (> 0) once the step's
// four directions are in, and the positions and lambda of stage stage_st (>= 0) to evaluate next.
// Every line touches only its own entries, so this equals the separate passes.
__global__ void k_trace_fused(int64_t N, int dir_st, int32_t adv_step, int stage_st, double ds, double sense,
                              int current, Box box, LamGrid g, const double* __restrict__ B,
                              const double* __restrict__ dB, double* __restrict__ kprev, double* __restrict__ ksum,
                              int32_t* __restrict__ ok, int32_t* __restrict__ alive, double* __restrict__ x,
                              double* __restrict__ out, int32_t* __restrict__ count, double* __restrict__ pts,
                              double* __restrict__ lam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (dir_st >= 0) trace_dir(i, N, dir_st, sense, current, B, dB, kprev, ksum);
    if (adv_step > 0) trace_advance(i, N, adv_step, ds, ok, ksum, alive, x, out, count);
    if (stage_st >= 0) trace_stage(i, N, stage_st, ds, box, g, x, kprev, alive, ok, pts, lam);
}

}  // namespace dbie

using namespace dbie;

extern "C" int dbie_trace_lines(dbie_ctx* c, const dbie_lambda_grid* lg, const double* box, double ds,
                                int32_t n_steps, int32_t mode, double sense, double* xyz_out, int32_t* count,
                                void* stream) {
    if (!c) return DBIE_E_INVAL;
    if (!lg || !box) return ctx_fail(c, DBIE_E_INVAL, "lambda grid and box are required");
    if (mode != DBIE_TRACE_FIELD && mode != DBIE_TRACE_CURRENT)
        return ctx_fail(c, DBIE_E_INVAL, "mode must be DBIE_TRACE_FIELD or DBIE_TRACE_CURRENT");
    if (!(sense == 1.0 || sense == -1.0)) return ctx_fail(c, DBIE_E_INVAL, "sense must be +1 or -1");
    if (!(ds > 0.0) || !std::isfinite(ds)) return ctx_fail(c, DBIE_E_INVAL, "ds must be positive and finite");
    if (n_steps < 0) return ctx_fail(c, DBIE_E_INVAL, "n_steps < 0");
    for (int d = 0; d < 3; ++d)
        if (!(box[d] < box[3 + d]) || !std::isfinite(box[d]) || !std::isfinite(box[3 + d]))
            return ctx_fail(c, DBIE_E_INVAL, "box needs finite lo < hi");
    if (!(box[2] > 0.0)) return ctx_fail(c, DBIE_E_INVAL, "box z_lo must be > 0 (the field needs z > 0)");
    if (lg->nx < 1 || lg->ny < 1 || lg->nz < 1 || !lg->lambda)
        return ctx_fail(c, DBIE_E_INVAL, "lambda grid needs nx, ny, nz >= 1 and a lambda pointer");
    if (int rc = ctx_check_device(c)) return rc;
    if (!(lg->dx > 0.0 && lg->dy > 0.0 && lg->dz > 0.0))
        return ctx_fail(c, DBIE_E_INVAL, "lambda grid spacing must be positive");
    const int64_t N = ctx_n(c);
    if (N == 0) return DBIE_OK;
    if (!xyz_out || !count) return ctx_fail(c, DBIE_E_INVAL, "xyz_out and count are required");
    // (n_steps + 1) x 3 x N doubles of output; beyond 2^34 values (128 GB) the call is refused
    if (((int64_t)n_steps + 1) * 3 * N > ((int64_t)1 << 34)) return ctx_fail(c, DBIE_E_INVAL, "output too large");
    hipStream_t s = (hipStream_t)stream;
    // workspace: seeds (3N), x (3N), kprev (3N), ksum (3N), lam (3N), B (3N), dB (9N), ok, alive, flag
    const size_t nd = (size_t)N * 27;
    char* w = (char*)ctx_scratch(c, 0, nd * sizeof(double) + (2 * (size_t)N + 64) * sizeof(int32_t));
    if (!w) return ctx_fail(c, DBIE_E_WORKSPACE, "cannot allocate the tracing workspace");
    double* seeds = (double*)w;
    double* x = seeds + 3 * N;
    double* kprev = x + 3 * N;
    double* ksum = kprev + 3 * N;
    double* lam = ksum + 3 * N;
    double* B = lam + 3 * N;
    double* dB = B + 3 * N;
    int32_t* ok = (int32_t*)(w + nd * sizeof(double));
    int32_t* alive = ok + N;
    int32_t* flag = alive + N;
    double* pts = ctx_xyz(c);
    const bool fp64 = ctx_precision(c) == DBIE_FP64;
    const bool cur = mode == DBIE_TRACE_CURRENT;
    const Box bx{{box[0], box[1], box[2]}, {box[3], box[4], box[5]}};
    const LamGrid g{lg->nx, lg->ny, lg->nz, lg->x0, lg->y0, lg->z0, lg->dx, lg->dy, lg->dz, lg->lambda};
    const unsigned gN = (unsigned)((N + 255) / 256);
    const int64_t total = ((int64_t)n_steps + 1) * 3 * N;
#define TR_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) return ctx_fail(c, DBIE_E_DEVICE, hipGetErrorString(e_)); \
    } while (0)
    TR_HIP(hipMemcpyAsync(seeds, pts, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s));
    // the steps move the context's points; on every exit after this they are put back
    auto steps = [&]() -> int {
        const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1 << 20);
        hipLaunchKernelGGL(k_trace_init, dim3((unsigned)blocks), dim3(256), 0, s, N, seeds, bx, total, xyz_out, count,
                           alive, x);
        TR_HIP(hipGetLastError());
        // before each evaluation: the previous stage's direction (or the previous step's last
        // direction and its advance), then the positions of this stage
        auto between = [&](int dir_st, int32_t adv_step, int stage_st) -> int {
            hipLaunchKernelGGL(k_trace_fused, dim3(gN), dim3(256), 0, s, N, dir_st, adv_step, stage_st, ds, sense,
                               cur ? 1 : 0, bx, g, B, dB, kprev, ksum, ok, alive, x, xyz_out, count, pts, lam);
            TR_HIP(hipGetLastError());
            return DBIE_OK;
        };
        for (int32_t step = 1; step <= n_steps; ++step) {
            for (int st = 0; st < 4; ++st) {
                const int dir_st = st > 0 ? st - 1 : (step > 1 ? 3 : -1);
                if (int r = between(dir_st, st == 0 && step > 1 ? step - 1 : 0, st)) return r;
                TR_HIP(ctx_prep_points(c, flag, s));
                if (int r = eval_set(c, lam, fp64, false, nullptr, B, cur ? dB : nullptr, nullptr, nullptr, s)) return r;
            }
        }
        if (n_steps > 0)
            if (int r = between(3, n_steps, -1)) return r;
        return DBIE_OK;
    };
    const int rc = steps();
    // the context's points and geometry back to the seeds
    TR_HIP(hipMemcpyAsync(pts, seeds, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s));
    TR_HIP(ctx_prep_points(c, flag, s));
    TR_HIP(hipStreamSynchronize(s));
    return rc;
#undef TR_HIP
}
