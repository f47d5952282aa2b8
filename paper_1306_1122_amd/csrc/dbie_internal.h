// Internal declarations of the DBIE library (gfx950). Not part of the public ABI.
//
// Units inside the kernels: every length is in pixels of the point's own magnetogram (u = (x-x0)/h,
// v = (y-y0)/h, w = z/h) and lambda is Lambda = lambda h. In these units the Eq. (16) nodal sum of
// the Eq. (6) kernel is scale free:
//   B_p      = (w / 2pi) A0_p,            A0 = sum_k N(t) rho^-3 B0_pk
//   dB_p/dx  = -(w / 2pi h) A1_p,          A1 = sum_k H rho^-5 (a_k - u) B0_pk,   H = t^2 cos t - 3 N(t)
//   dB_p/dy  = -(w / 2pi h) A2_p,          A2 = sum_k H rho^-5 (b_k - v) B0_pk
//   dB_p/dz  = (A0_p + w^2 A3_p)/(2pi h),  A3 = sum_k H rho^-5 B0_pk
// with rho the pixel-unit distance, t = Lambda rho, N(t) = t sin t + cos t (frozen-lambda gradient,
// Eq. 13 in the delta -> 0 limit). The derivatives with respect to mu = lambda^2 need three more sums
//   T0 = sum_k cos(t) rho^-1 B0_pk,  T1 = sum_k N rho^-3 (a_k - u) B0_pk,  T2 = ... (b_k - v) ...
// because dA3/dmu_px = -A0/2:
//   dB_p/dmu = (w h^2 / 4pi) T0,   d(dB_p/dx)/dmu = (w h / 4pi) T1,   d(dB_p/dy)/dmu = (w h / 4pi) T2,
//   d(dB_p/dz)/dmu = (h / 4pi)(T0 - w^2 A0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dbie {

constexpr int kAccField = 12;   // rows 4p + j: A0, A1, A2, A3 of component p
constexpr int kAccTan = 9;      // rows 12 + 3p + j: T0, T1, T2 of component p
constexpr int kAcc = kAccField + kAccTan;
constexpr int kNearWin = 2;     // near-field window half-width in pixels (radius <= 2 h)
constexpr int kNearSide = 2 * kNearWin + 1;
// 9-node elements: the near window is 3 x 3 elements (of side 2 h) around element (floor(u/2),
// floor(v/2)), which holds every element closer than 2 h horizontally; one mask bit per element.
constexpr int kNearWinQ = 1;
constexpr int kNearSideQ = 2 * kNearWinQ + 1;
constexpr int kMaxSplit = 32;   // largest number of FP32C pixel slices per launch
constexpr int kRows = 32;       // FP32C pixel block: kRows x kCols pixels, tile-major in HBM
constexpr int kCols = 8;

struct BoundaryDev {
    int32_t nx, ny;
    int32_t npix;       // nx * ny
    // Quadrature grid of the FP64 path: gcols x grows points at the positions gpos[gpos_off + c]
    // (columns) and gpos[gpos_off + gcols + r] (rows), in pixels from node (0, 0), carrying the
    // weighted field gB[gpl_off + p * gcols * grows + r * gcols + c]. For the nodal rule (Eq. 16) it
    // is the pixel grid itself; for 9-node elements (Eq. 15) the Gauss points of the elements.
    int32_t gcols, grows;
    int64_t gpos_off, gpl_off;
    int32_t G;          // Gauss points per element side; 0 = nodal rule
    // FP32C grid positions (9-node elements only): float4 {integer part, fraction, element index, 0}
    // for the ntx * kCols padded columns, then the nty * kRows padded rows, from gposf_off
    int64_t gposf_off;
    int32_t ntx, nty;   // FP32C blocks along x and y (ceil(gcols / kCols), ceil(grows / kRows))
    int32_t npix_pad;   // ntx * nty * kRows * kCols
    int64_t pix_off;    // offset of this boundary in the FP64 planes (3 planes of npix each)
    int64_t pixf_off;   // offset of this boundary in the FP32 blocks (3 * npix_pad floats)
    double x0, y0, h;
};

// A run of consecutive points of one boundary (entries of the schedule).
struct Tile {
    int64_t start;
    int32_t count;
    int32_t b;
};

// Per-point geometry, computed once in dbie_init (device SoA arrays of length N).
struct Geo {
    double* u;
    double* v;
    double* w;
    float* xi_int;     // floor(u) as float (exact integer)
    float* xi_frac;    // u - floor(u) rounded once to FP32
    float* yi_int;
    float* yi_frac;
    float* wf;         // (float) w
    int32_t* win_a;    // round(u): centre of the near-field window
    int32_t* win_b;
    uint32_t* near_mask;  // bit (i + 2) + 5 (j + 2): pixel (win_a + i, win_b + j) is near (FP64 test)
    int32_t* bidx;
};

// sin and cos of t for |t| < kSincosBound, to about one ulp, without branches: t = k pi + r with
// k = rint(t/pi), |r| <= pi/2, r from a two-constant Cody-Waite reduction (with FMA the first step is
// exact for |k| < 2^20, the second leaves ~1e-27), and polynomials on [-pi/2, pi/2] fitted by least
// squares on Chebyshev nodes in 50-digit arithmetic (sin r = r + r^3 P(r^2), P of degree 7;
// cos r = 1 - r^2/2 + r^4 Q(r^2), Q of degree 6; fit errors below 2e-17 with the coefficients
// rounded to double). k comes from one FMA that adds 1.5 2^52 to t/pi: doubles in that binade are
// one apart, so the sum is t/pi rounded to an integer (ties to even) and its low word holds k in
// two's complement (|t/pi| < 2^51). Returns sin r, cos r and, as a mask of the sign bit, the parity
// of k: sin t = (-1)^k sin r and cos t = (-1)^k cos r, so the callers flip the sign of what
// multiplies them (one XOR).
constexpr double kSincosBound = 524288.0;   // 2^19
constexpr double kRoundMagic = 6755399441055744.0;   // 1.5 2^52
__device__ __forceinline__ uint64_t sincos_halfturn(double t, double* s, double* c) {
    const double kb = __builtin_fma(t, 0.3183098861837907, kRoundMagic);
    const double k = kb - kRoundMagic;
    double r = __builtin_fma(-k, 3.141592653589793, t);
    r = __builtin_fma(-k, 1.2246467991473532e-16, r);
    const double z = r * r;
    double p = __builtin_fma(z, 2.7221623441283363e-15, -7.64308811092882e-13);
    p = __builtin_fma(z, p, 1.6058943534108974e-10);
    p = __builtin_fma(z, p, -2.5052106951355734e-08);
    p = __builtin_fma(z, p, 2.7557319212021904e-06);
    p = __builtin_fma(z, p, -0.00019841269841214533);
    p = __builtin_fma(z, p, 0.00833333333333321);
    p = __builtin_fma(z, p, -0.16666666666666666);
    *s = __builtin_fma(r * z, p, r);
    double q = __builtin_fma(z, 4.615589456771727e-14, -1.1463582501750082e-11);
    q = __builtin_fma(z, q, 2.0876590527674145e-09);
    q = __builtin_fma(z, q, -2.755731702734344e-07);
    q = __builtin_fma(z, q, 2.4801587285345367e-05);
    q = __builtin_fma(z, q, -0.0013888888888827712);
    q = __builtin_fma(z, q, 0.04166666666666578);
    *c = __builtin_fma(z * z, q, __builtin_fma(z, -0.5, 1.0));
    return __builtin_bit_cast(uint64_t, kb) << 63;
}

// 1/sqrt(x) for finite x > 0 (a squared distance, at least w^2 > 0): the hardware estimate refined by
// one third-order Householder step, y (1 + e/2 + 3 e^2 / 8) with e = 1 - x y^2, which takes the
// estimate's relative error d to about (5/16) d^3.
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

// x with its sign bit flipped where `sign` (0 or the sign bit) says so
__device__ __forceinline__ double flip_sign(double x, uint64_t sign) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, x) ^ sign);
}

// sin and cos of t for |t| < kSincosBound from a table of (sin, cos)(j pi/16), j = 0..31: t =
// k pi/16 + r with k = rint(16 t / pi) from one FMA that adds 1.5 2^52 (as in sincos_halfturn: the
// low word of the sum holds k, so k mod 32 is its low five bits), r from a two-constant Cody-Waite
// reduction with FMA (|r| <= pi/32 up to rounding), sin r = r + r^3 P(r^2) with P of degree 2 fitted
// on [0, pi/32] (largest absolute error 1.4e-17), cos r from its Taylor series to r^8 (coefficients
// +-1/n! rounded to double; the first term left out is below 2.3e-17 there), and the addition
// theorems sin t = S cos r + C sin r, cos t = C cos r - S sin r
// with (S, C) = tab[k mod 32]. About one ulp of 1 absolute. `tab` is kSinCos16 copied to LDS by the
// calling kernel; the constants come from csrc/sincos_fit.py (`table`).
static __constant__ double kSinCos16[64] = {
    0.0, 1.0, 0.19509032201612828, 0.9807852804032304,
    0.3826834323650898, 0.9238795325112867, 0.5555702330196022, 0.8314696123025452,
    0.7071067811865476, 0.7071067811865476, 0.8314696123025452, 0.5555702330196022,
    0.9238795325112867, 0.3826834323650898, 0.9807852804032304, 0.19509032201612828,
    1.0, 0.0, 0.9807852804032304, -0.19509032201612828,
    0.9238795325112867, -0.3826834323650898, 0.8314696123025452, -0.5555702330196022,
    0.7071067811865476, -0.7071067811865476, 0.5555702330196022, -0.8314696123025452,
    0.3826834323650898, -0.9238795325112867, 0.19509032201612828, -0.9807852804032304,
    0.0, -1.0, -0.19509032201612828, -0.9807852804032304,
    -0.3826834323650898, -0.9238795325112867, -0.5555702330196022, -0.8314696123025452,
    -0.7071067811865476, -0.7071067811865476, -0.8314696123025452, -0.5555702330196022,
    -0.9238795325112867, -0.3826834323650898, -0.9807852804032304, -0.19509032201612828,
    -1.0, 0.0, -0.9807852804032304, 0.19509032201612828,
    -0.9238795325112867, 0.3826834323650898, -0.8314696123025452, 0.5555702330196022,
    -0.7071067811865476, 0.7071067811865476, -0.5555702330196022, 0.8314696123025452,
    -0.3826834323650898, 0.9238795325112867, -0.19509032201612828, 0.9807852804032304,
};
__device__ __forceinline__ void sincos_table16(double t, const double2* __restrict__ tab, double* s, double* c) {
    const double kb = __builtin_fma(t, 5.092958178940651, kRoundMagic);
    const double k = kb - kRoundMagic;
    double r = __builtin_fma(-k, 0.19634954084936207, t);
    r = __builtin_fma(-k, 7.654042494670958e-18, r);
    const double z = r * r;
    double p = __builtin_fma(z, -0.00019835792424992082, 0.00833333299396471);
    p = __builtin_fma(z, p, -0.16666666666603067);
    const double sr = __builtin_fma(r * z, p, r);
    double q = __builtin_fma(z, 2.48015873015873e-05, -0.001388888888888889);
    q = __builtin_fma(z, q, 0.041666666666666664);
    const double cr = __builtin_fma(z * z, q, __builtin_fma(z, -0.5, 1.0));
    const double2 e = tab[(uint32_t)__builtin_bit_cast(uint64_t, kb) & 31u];
    *s = __builtin_fma(e.y, sr, e.x * cr);
    *c = __builtin_fma(-e.x, sr, e.y * cr);
}

// The FP64 pair: shared arithmetic of pair_fp64 (every row accumulated per pair) and pair_fp64_row
// (the y-moment rows through per-row sums).
template <bool TAN, bool WIDE, bool TAB, bool ROW>
__device__ __forceinline__ void pair_fp64_core(double dx, double dy, double w2q, const double lam[3],
                                               double b0x, double b0y, double b0z, double* acc, double* rs,
                                               const double2* __restrict__ tab) {
    const double r2 = ROW ? __builtin_fma(dx, dx, w2q) : __builtin_fma(dx, dx, __builtin_fma(dy, dy, w2q));
    const double ri = WIDE ? rsqrt(r2) : rsqrt_pos(r2);
    const double r = r2 * ri;
    const double ri2 = ri * ri;
    const double ri3 = ri2 * ri;
    const double ri2n3 = -3.0 * ri2;
    const double b0[3] = {b0x, b0y, b0z};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const double t = lam[p] * r;
        double s, c, bp = b0[p];
        if (WIDE) sincos(t, &s, &c);
        else if (TAB) sincos_table16(t, tab, &s, &c);
        else bp = flip_sign(bp, sincos_halfturn(t, &s, &c));   // (-1)^k carried by B0
        const double n = __builtin_fma(t, s, c);
        const double b3 = ri3 * bp;
        const double nb = n * b3;
        const double hb = b3 * __builtin_fma(ri2n3, n, lam[p] * lam[p] * c);   // H B0 / r^5
        acc[4 * p + 1] = __builtin_fma(hb, dx, acc[4 * p + 1]);
        if (ROW) {
            // the row's y-moments come from these row sums, times dy, once per row
            rs[p] += hb;
            if (TAN) rs[3 + p] += nb;
        } else {
            acc[4 * p + 0] += nb;
            acc[4 * p + 2] = __builtin_fma(hb, dy, acc[4 * p + 2]);
            acc[4 * p + 3] += hb;
        }
        if (TAN) {
            acc[12 + 3 * p + 0] = __builtin_fma(c * ri, bp, acc[12 + 3 * p + 0]);
            acc[12 + 3 * p + 1] = __builtin_fma(nb, dx, acc[12 + 3 * p + 1]);
            if (!ROW) acc[12 + 3 * p + 2] = __builtin_fma(nb, dy, acc[12 + 3 * p + 2]);
        }
        if (ROW && !TAN) acc[4 * p + 0] += nb;
    }
}

// One pair (point, pixel) in FP64, added to the 12 (+9) accumulators of the three components.
// dx = a_k - u, dy = b_k - v, w2 = w^2, all in pixels. Used by the FP64 near-field pass of the
// FP32C path (and the near pairs the FP64 recompute takes out again). WIDE: the device library's
// sincos (any argument); otherwise every |lambda r| must stay below kSincosBound, and TAB takes
// sincos_table16 (its table in the caller's LDS) instead of sincos_halfturn. With t^2 = lambda^2 r^2,
// the gradient term H B0 / r^5 (H = t^2 cos t - 3 N) is formed as (B0 / r^3)((-3 / r^2) N +
// lambda^2 cos t), sharing B0 / r^3 with the field row: two multiplies and one FMA per component,
// -3 / r^2 once per pair.
template <bool TAN, bool WIDE, bool TAB = false>
__device__ __forceinline__ void pair_fp64(double dx, double dy, double w2, const double lam[3],
                                          double b0x, double b0y, double b0z, double* acc,
                                          const double2* __restrict__ tab = nullptr) {
    pair_fp64_core<TAN, WIDE, TAB, false>(dx, dy, w2, lam, b0x, b0y, b0z, acc, nullptr, tab);
}

// The same pair within a row of the grid: q = dy^2 + w^2 of the row; the A3 terms H B0 / r^5 and,
// with tangents, the A0 terms N B0 / r^3 go to the row sums rs[3] (+3), from which the caller adds
// A0, A3, A2 += dy (sum of A3 terms) and T2 += dy (sum of A0 terms) once per row.
template <bool TAN, bool WIDE, bool TAB = false>
__device__ __forceinline__ void pair_fp64_row(double dx, double q, const double lam[3], double b0x, double b0y,
                                              double b0z, double* acc, double* rs,
                                              const double2* __restrict__ tab = nullptr) {
    pair_fp64_core<TAN, WIDE, TAB, true>(dx, 0.0, q, lam, b0x, b0y, b0z, acc, rs, tab);
}

// FP64 pairs of the near-field window (shared by the finalize pass and the FP64 recompute of
// high-phase points) (the bits set in dbie_init's classification).
template <bool TAN, bool WIDE>
__device__ __forceinline__ void add_near(const BoundaryDev& bd, const double* B0, uint32_t mask,
                                         int32_t wa, int32_t wb, double u, double v, double w2,
                                         const double lm[3], double* a) {
    while (mask) {
        const int bit = __builtin_ctz(mask);
        mask &= mask - 1u;
        const int ii = bit % kNearSide - kNearWin, jj = bit / kNearSide - kNearWin;
        const int32_t pa = wa + ii, pb = wb + jj;
        const int64_t k = (int64_t)pb * bd.nx + pa;
        pair_fp64<TAN, WIDE>((double)pa - u, (double)pb - v, w2, lm, B0[k], B0[bd.npix + k],
                       B0[2 * (int64_t)bd.npix + k], a);
    }
}

// 9-node elements: every Gauss point of each element flagged near, at its FP64 position, with the
// FP64 weighted field of the quadrature grid.
template <bool TAN, bool WIDE>
__device__ __forceinline__ void add_near_grid(const BoundaryDev& bd, const double* __restrict__ gpos,
                                              const double* __restrict__ gB, uint32_t mask, int32_t wa,
                                              int32_t wb, double u, double v, double w2, const double lm[3],
                                              double* a) {
    const double* cpos = gpos + bd.gpos_off;
    const double* rpos = cpos + bd.gcols;
    const int64_t ng = (int64_t)bd.gcols * bd.grows;
    const double* W = gB + bd.gpl_off;
    while (mask) {
        const int bit = __builtin_ctz(mask);
        mask &= mask - 1u;
        const int32_t m = wa + bit % kNearSideQ - kNearWinQ, n = wb + bit / kNearSideQ - kNearWinQ;
        for (int q = 0; q < bd.G; ++q) {
            const int32_t r = bd.G * n + q;
            const double dy = rpos[r] - v;
            for (int g = 0; g < bd.G; ++g) {
                const int32_t c = bd.G * m + g;
                const int64_t k = (int64_t)r * bd.gcols + c;
                pair_fp64<TAN, WIDE>(cpos[c] - u, dy, w2, lm, W[k], W[ng + k], W[2 * ng + k], a);
            }
        }
    }
}

// ---- residuals (Eqs. 8, 9, 14) in FP64 -------------------------------------------------------
enum : int32_t { kStConverged = 0, kStBudget = 1, kStDegenerate = 2, kStJZero = 3, kStNonfinite = 4 };

struct Resid {
    double f, g, Phi, rho;
    double u[4];   // (J x B / (|J||B|), sign(div B) g): |u|^2 = Phi
    int32_t status;
};

// J = curl B (Eq. 14), f = |J x B| / (|J||B|) (Eq. 8), g = |div B| c / |B| with c = dV/dSigma
// (Eq. 9). |J| = 0 gives f = 0 (J_ZERO); |B| = 0 is DEGENERATE; non-finite input is NONFINITE;
// both of the latter get Phi = rho = +inf and f = g = NaN.
__device__ __forceinline__ Resid residual_fp64(const double B[3], const double dB[9], double c) {
    Resid R;
    const double J0 = dB[7] - dB[5], J1 = dB[2] - dB[6], J2 = dB[3] - dB[1];
    const double D = dB[0] + dB[4] + dB[8];
    bool fin = isfinite(B[0]) && isfinite(B[1]) && isfinite(B[2]);
#pragma unroll
    for (int k = 0; k < 9; ++k) fin = fin && isfinite(dB[k]);
    const double nB = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const double nJ = sqrt(J0 * J0 + J1 * J1 + J2 * J2);
    R.status = kStBudget;
    if (!fin || nB == 0.0) {
        R.status = fin ? kStDegenerate : kStNonfinite;
        R.f = R.g = __builtin_nan("");
        R.Phi = R.rho = __builtin_inf();
        R.u[0] = R.u[1] = R.u[2] = R.u[3] = 0.0;
        return R;
    }
    if (nJ == 0.0) {
        R.status = kStJZero;
        R.u[0] = R.u[1] = R.u[2] = 0.0;
    } else {
        const double den = nJ * nB;
        R.u[0] = (J1 * B[2] - J2 * B[1]) / den;
        R.u[1] = (J2 * B[0] - J0 * B[2]) / den;
        R.u[2] = (J0 * B[1] - J1 * B[0]) / den;
    }
    R.u[3] = c * D / nB;
    R.f = sqrt(R.u[0] * R.u[0] + R.u[1] * R.u[1] + R.u[2] * R.u[2]);
    R.g = fabs(R.u[3]);
    R.Phi = R.f * R.f + R.g * R.g;
    R.rho = fmax(R.f, R.g);
    return R;
}

// d u / d mu_p (jac[4][3], row-major) by the chain rule: only B_p and the row dB_p/dx_q depend on
// mu_p, and their mu-derivatives are the tangent rows tan[p] and tan[3 + 3p + q].
__device__ __forceinline__ void residual_jacobian_fp64(const double B[3], const double dB[9],
                                                       const double tan[12], double c,
                                                       double jac[12]) {
    const double J[3] = {dB[7] - dB[5], dB[2] - dB[6], dB[3] - dB[1]};
    const double D = dB[0] + dB[4] + dB[8];
    const double nB = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const double nJ = sqrt(J[0] * J[0] + J[1] * J[1] + J[2] * J[2]);
    const double w[3] = {J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2], J[0] * B[1] - J[1] * B[0]};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        double Bd[3] = {0.0, 0.0, 0.0};
        Bd[p] = tan[p];
        double dBd[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        dBd[3 * p + 0] = tan[3 + 3 * p + 0];
        dBd[3 * p + 1] = tan[3 + 3 * p + 1];
        dBd[3 * p + 2] = tan[3 + 3 * p + 2];
        const double Jd[3] = {dBd[7] - dBd[5], dBd[2] - dBd[6], dBd[3] - dBd[1]};
        const double Dd = dBd[0] + dBd[4] + dBd[8];
        const double wd[3] = {Jd[1] * B[2] - Jd[2] * B[1] + J[1] * Bd[2] - J[2] * Bd[1],
                              Jd[2] * B[0] - Jd[0] * B[2] + J[2] * Bd[0] - J[0] * Bd[2],
                              Jd[0] * B[1] - Jd[1] * B[0] + J[0] * Bd[1] - J[1] * Bd[0]};
        const double db = (B[0] * Bd[0] + B[1] * Bd[1] + B[2] * Bd[2]) / nB;
        if (nJ == 0.0) {
            jac[0 * 3 + p] = jac[1 * 3 + p] = jac[2 * 3 + p] = 0.0;
        } else {
            const double da = (J[0] * Jd[0] + J[1] * Jd[1] + J[2] * Jd[2]) / nJ;
            const double den = nJ * nB;
            const double k = (da / nJ + db / nB) / den;
#pragma unroll
            for (int q = 0; q < 3; ++q) jac[q * 3 + p] = wd[q] / den - w[q] * k;
        }
        jac[3 * 3 + p] = c * Dd / nB - c * D * db / (nB * nB);
    }
}

// ---- launchers (each defined next to its kernels) ---------------------------------------------
hipError_t launch_prep(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd, const double* gB,
                       const double* xyz, int64_t N, Geo geo, double near_r2, int check_only_fp64,
                       int32_t* bad_flag, float* pixf, const BoundaryDev* bnd_host, int32_t nb,
                       hipStream_t s);

hipError_t launch_expand_scalar(const double* lam, int32_t L, int64_t N, double* lam3, hipStream_t s);

// The bulk kernels run over a schedule of tiles. Without `idx` a tile is a run of point indices;
// with `idx` it is a run of entries of the active-point list idx (device schedules of the solver).
hipError_t launch_field64(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd,
                          const double* gpos, const double* gB, Geo geo, const double* lam, int64_t N,
                          int32_t L, int32_t S, const int32_t* idx, bool tan, double* acc, hipStream_t s);
// FP32C contexts, after the FP32 bulk pass: recompute in FP64 (and overwrite) the partial sums of the
// points whose largest phase max_p |lambda_p| r_max exceeds phase_max radians (see k_field64.hip).
hipError_t launch_field64_override(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd, const double* B0d,
                                   const double* gpos, const double* gB, Geo geo, const double* lam, int64_t N,
                                   int32_t L, int32_t S, const int32_t* idx, bool tan, double phase_max, double* acc,
                                   hipStream_t s);
// Largest phase max_p |lambda_p| r_max (radians) up to which the FP32C bulk pass keeps its error
// below its 1e-5 relative bar: without and with the mu-tangents (the tangent rows' weights decay
// only as 1/r, so the far pixels, whose phases carry the most FP32 rounding, dominate them).
constexpr double kFp32cPhaseMax = 2.0 * 3.14159265358979323846 * 512.0;
constexpr double kFp32cPhaseMaxTan = 2.0 * 3.14159265358979323846 * 128.0;

// The weighted field of the 9-node element quadrature grid: gB = w_g w_q sum L_a(xi_g) L_b(xi_q) B0
// (lw[3 * g + a] = w_g L_a(xi_g), G points per element side).
hipError_t launch_quad_weights(const BoundaryDev& bd, const double* B0d, const double* lw, int G, double* gB,
                               hipStream_t s);
// Transpose of the interpolation: gradient at the nodes from the gradient at the grid points.
hipError_t launch_quad_transpose(const BoundaryDev& bd, const double* gW, const double* lw, int G, double* gB0,
                                 hipStream_t s);

struct F32Shape {
    int32_t ppl;      // points per lane
    int32_t waves;    // waves per workgroup
    int32_t tp;       // kCols x the rows of the LDS pixel block (nodal blocks are 2 kCols wide)
    int32_t persist;  // 1: persistent grid pulling tiles from a device counter
};

// work: a device int the persistent form uses as its tile counter (cleared by a kernel inside the
// launch). scalar: the three lambda rows of every point are equal (the kernel reads row 0 only).
hipError_t launch_field32c(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd,
                           const float* pixf, const float4* gposf, Geo geo, const double* lam, int64_t N,
                           int32_t L, int32_t S, const int32_t* idx, int32_t* work, bool tan, bool scalar,
                           F32Shape shape, double* acc, hipStream_t s);
bool field32c_shape_supported(F32Shape shape);
int field32c_shapes(F32Shape* out, int max);   // the instantiated shapes; returns their number

// Over idx[0 .. n) (n = *n_dev when n_dev is given, else n_idx), or over every point without idx.
// acc holds S slices of [L][kAcc][N] (the pixel split of the bulk pass), summed here in order; with
// many slices and few points they are first summed in place into slice 0 by a pass with one thread
// per (point, trial, row) (same order, same result).
hipError_t launch_finalize(const BoundaryDev* bnd, const double* B0d, const double* gpos, const double* gB,
                           Geo geo, const double* lam,
                           const int32_t* idx, int64_t n_idx, const int32_t* n_dev, int64_t N, int32_t L,
                           int32_t S, double* acc,
                           bool add_near, bool tan, double dvds, double* B, double* dB, double* fg,
                           double* tanout, hipStream_t s);

// Sums of f, g, finite points and points with max(f, g) <= eps into scratch[0..3] (scratch holds
// 4 + 4 * 256 doubles).
hipError_t launch_fg_stats(int64_t N, const double* fg, double eps, double* scratch, hipStream_t s);

}  // namespace dbie
