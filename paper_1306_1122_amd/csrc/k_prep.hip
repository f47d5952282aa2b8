// Set-up kernels run once by dbie_init: per-point geometry in pixel units, the FP64 near-field
// classification, point validation, and the FP32 pixel planes of the FP32C path.
#include "dbie_internal.h"

namespace dbie {

// One thread per point of the schedule. Computes u, v, w (FP64), the split FP32 coordinates
// (exact integer part + fraction rounded once, so that a_k - u is formed with one rounding in
// FP32), and the near mask: pixel (a, b) of the 5x5 window around (round(u), round(v)) is "near"
// when it exists and rho^2 = (a-u)^2 + (b-v)^2 + w^2 < near_r2, tested here in FP64 once (for 9-node
// elements, whole elements of a 3x3 element window). The FP32 bulk pass skips exactly these pairs
// and the FP64 near pass sums exactly these pairs.
__global__ void k_prep_points(const Tile* __restrict__ tiles, const BoundaryDev* __restrict__ bnd,
                              const double* __restrict__ xyz, int64_t N, Geo geo, double near_r2,
                              int32_t* __restrict__ bad_flag) {
    const Tile t = tiles[blockIdx.x];
    for (int j = threadIdx.x; j < t.count; j += blockDim.x) {
        const int64_t i = t.start + j;
        const BoundaryDev bd = bnd[t.b];
        const double x = xyz[i], y = xyz[N + i], z = xyz[2 * N + i];
        const double u = (x - bd.x0) / bd.h;
        const double v = (y - bd.y0) / bd.h;
        const double w = z / bd.h;
        const bool ok = (z > 0.0) && isfinite(x) && isfinite(y) && isfinite(z) && fabs(u) < 4.0e6 &&
                        fabs(v) < 4.0e6 && w < 4.0e6;
        if (!ok) atomicOr(bad_flag, 1);
        const double uu = ok ? u : 0.0, vv = ok ? v : 0.0, ww = ok ? w : 1.0;
        geo.u[i] = uu;
        geo.v[i] = vv;
        geo.w[i] = ww;
        const double fu = floor(uu), fv = floor(vv);
        geo.xi_int[i] = (float)fu;
        geo.xi_frac[i] = (float)(uu - fu);
        geo.yi_int[i] = (float)fv;
        geo.yi_frac[i] = (float)(vv - fv);
        geo.wf[i] = (float)ww;
        geo.bidx[i] = t.b;
        uint32_t mask = 0u;
        if (bd.G > 0) {
            // 9-node elements: element (m, n) covers nodes 2m..2m+2 x 2n..2n+2; it is near when the
            // distance from the point to that rectangle (with the height) is below the radius
            const int32_t wa = (int32_t)floor(0.5 * uu), wb = (int32_t)floor(0.5 * vv);
            geo.win_a[i] = wa;
            geo.win_b[i] = wb;
            const int32_t ex = (bd.nx - 1) / 2, ey = (bd.ny - 1) / 2;
            if (ww * ww < near_r2) {
                for (int jj = -kNearWinQ; jj <= kNearWinQ; ++jj) {
                    for (int ii = -kNearWinQ; ii <= kNearWinQ; ++ii) {
                        const int32_t m = wa + ii, n = wb + jj;
                        if (m < 0 || m >= ex || n < 0 || n >= ey) continue;
                        const double dx = fmax(0.0, fmax(2.0 * m - uu, uu - (2.0 * m + 2.0)));
                        const double dy = fmax(0.0, fmax(2.0 * n - vv, vv - (2.0 * n + 2.0)));
                        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, ww * ww));
                        if (r2 < near_r2) mask |= 1u << ((ii + kNearWinQ) + kNearSideQ * (jj + kNearWinQ));
                    }
                }
            }
            geo.near_mask[i] = mask;
            continue;
        }
        const int32_t wa = (int32_t)rint(uu), wb = (int32_t)rint(vv);
        geo.win_a[i] = wa;
        geo.win_b[i] = wb;
        if (ww * ww < near_r2) {
            for (int jj = -kNearWin; jj <= kNearWin; ++jj) {
                for (int ii = -kNearWin; ii <= kNearWin; ++ii) {
                    const int32_t a = wa + ii, b = wb + jj;
                    if (a < 0 || a >= bd.nx || b < 0 || b >= bd.ny) continue;
                    const double dx = (double)a - uu, dy = (double)b - vv;
                    const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, ww * ww));
                    if (r2 < near_r2) mask |= 1u << ((ii + kNearWin) + kNearSide * (jj + kNearWin));
                }
            }
        }
        geo.near_mask[i] = mask;
    }
}

// FP32 blocks of one boundary's quadrature grid (the pixels for the nodal rule): block k = (ty, tx)
// holds three planes (Bx, By, Bz) of kRows x kCols floats for grid points (tx kCols + c, ty kRows + r)
// of the weighted field; points beyond the grid hold zero.
__global__ void k_fill_pixf(BoundaryDev bd, const double* __restrict__ gB, float* __restrict__ pixf) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int BP = kRows * kCols;
    if (e >= 3 * (int64_t)bd.npix_pad) return;
    const int64_t k = e / (3 * BP);
    const int rem = (int)(e - k * 3 * BP);
    const int pl = rem / BP, o = rem - pl * BP;
    const int r = o / kCols, c = o - r * kCols;
    const int ty = (int)(k / bd.ntx), tx = (int)(k - (int64_t)ty * bd.ntx);
    const int a = tx * kCols + c, b = ty * kRows + r;
    float v = 0.0f;
    if (a < bd.gcols && b < bd.grows)
        v = (float)gB[bd.gpl_off + (int64_t)pl * bd.gcols * bd.grows + (int64_t)b * bd.gcols + a];
    pixf[bd.pixf_off + e] = v;
}

// lam3[t][p][i] = lam[t][i] for p = x, y, z (one lambda shared by the three components).
__global__ void k_expand_scalar(const double* __restrict__ lam, int64_t LN, int64_t N, double* __restrict__ lam3) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= LN) return;
    const int64_t t = e / N, i = e - t * N;
    const double v = lam[e];
    for (int p = 0; p < 3; ++p) lam3[(t * 3 + p) * N + i] = v;
}

hipError_t launch_expand_scalar(const double* lam, int32_t L, int64_t N, double* lam3, hipStream_t s) {
    const int64_t LN = (int64_t)L * N;
    hipLaunchKernelGGL(k_expand_scalar, dim3((unsigned)((LN + 255) / 256)), dim3(256), 0, s, lam, LN, N, lam3);
    return hipGetLastError();
}

hipError_t launch_prep(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd, const double* gB,
                       const double* xyz, int64_t N, Geo geo, double near_r2, int fp64_only,
                       int32_t* bad_flag, float* pixf, const BoundaryDev* bnd_host, int32_t nb,
                       hipStream_t s) {
    if (n_tiles > 0) {
        hipLaunchKernelGGL(k_prep_points, dim3((unsigned)n_tiles), dim3(256), 0, s, tiles, bnd, xyz, N,
                           geo, near_r2, bad_flag);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!fp64_only) {
        for (int32_t b = 0; b < nb; ++b) {
            const int64_t P = 3 * (int64_t)bnd_host[b].npix_pad;
            hipLaunchKernelGGL(k_fill_pixf, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s,
                               bnd_host[b], gB, pixf);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace dbie

namespace dbie {

// Weighted field at the element Gauss points: column c = G m + g, row r = G n + q of element
// (m, n) whose nodes are a = 2m..2m+2, b = 2n..2n+2.
__global__ void k_quad_weights(BoundaryDev bd, const double* __restrict__ B0d, const double* __restrict__ lw,
                               int G, double* __restrict__ gB) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gn = (int64_t)bd.gcols * bd.grows;
    if (e >= gn) return;
    const int c = (int)(e % bd.gcols), r = (int)(e / bd.gcols);
    const int m = c / G, g = c - m * G, n = r / G, q = r - n * G;
    for (int p = 0; p < 3; ++p) {
        const double* B = B0d + bd.pix_off + (int64_t)p * bd.npix;
        double acc = 0.0;
        for (int be = 0; be < 3; ++be)
            for (int al = 0; al < 3; ++al)
                acc += lw[3 * g + al] * lw[3 * q + be] * B[(int64_t)(2 * n + be) * bd.nx + 2 * m + al];
        gB[bd.gpl_off + p * gn + e] = acc;
    }
}

// gB0 at node (a, b) = sum over the (up to 4) elements holding it and their Gauss points of the
// interpolation weight times the gradient at the point.
__global__ void k_quad_transpose(BoundaryDev bd, const double* __restrict__ gW, const double* __restrict__ lw,
                                 int G, double* __restrict__ gB0) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= bd.npix) return;
    const int a = (int)(k % bd.nx), b = (int)(k / bd.nx);
    const int64_t gn = (int64_t)bd.gcols * bd.grows;
    const int ex = (bd.nx - 1) / 2, ey = (bd.ny - 1) / 2;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int m = max(0, (a - 1) / 2); m <= min(ex - 1, a / 2); ++m) {
        const int al = a - 2 * m;
        if (al < 0 || al > 2) continue;
        for (int n = max(0, (b - 1) / 2); n <= min(ey - 1, b / 2); ++n) {
            const int be = b - 2 * n;
            if (be < 0 || be > 2) continue;
            for (int q = 0; q < G; ++q)
                for (int g = 0; g < G; ++g) {
                    const double wgt = lw[3 * g + al] * lw[3 * q + be];
                    const int64_t e = (int64_t)(G * n + q) * bd.gcols + G * m + g;
                    for (int p = 0; p < 3; ++p) acc[p] += wgt * gW[bd.gpl_off + p * gn + e];
                }
        }
    }
    for (int p = 0; p < 3; ++p) gB0[bd.pix_off + (int64_t)p * bd.npix + k] = acc[p];
}

hipError_t launch_quad_weights(const BoundaryDev& bd, const double* B0d, const double* lw, int G, double* gB,
                               hipStream_t s) {
    const int64_t gn = (int64_t)bd.gcols * bd.grows;
    hipLaunchKernelGGL(k_quad_weights, dim3((unsigned)((gn + 255) / 256)), dim3(256), 0, s, bd, B0d, lw, G, gB);
    return hipGetLastError();
}

hipError_t launch_quad_transpose(const BoundaryDev& bd, const double* gW, const double* lw, int G, double* gB0,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_quad_transpose, dim3((unsigned)((bd.npix + 255) / 256)), dim3(256), 0, s, bd, gW, lw, G,
                       gB0);
    return hipGetLastError();
}

}  // namespace dbie
