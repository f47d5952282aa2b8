// Adjoint of the evaluation (dbie_grad): the transpose of the Eq. (16) nodal sum together with its
// frozen-lambda gradient rows (the gradient with respect to B0), the lambda gradient from the
// mu-tangents, and the residual Jacobian d u / d mu.
//
// Transpose in pixel units (see dbie_internal.h for the forward relations): with per-point weights
//   alpha_p = w gB_p / 2pi + gZ_p / (2pi h),   beta_p = w^2 gZ_p / (2pi h),
//   gx_p = -w gX_p / (2pi h),                  gy_p = -w gY_p / (2pi h)
// (gX, gY, gZ = dLoss/d(dB_p/dx, dy, dz)),
//   gB0_p(k) = sum_i [ N rho^-3 alpha_p + H rho^-5 (beta_p + gx_p (a_k - u_i) + gy_p (b_k - v_i)) ].
// With 9-node elements (Eq. 15) the FP64 transpose runs over the Gauss points (positions a_k, b_k
// of the quadrature grid) and the interpolation transpose then carries it to the nodes.
// Pixels are the outputs; the points of the pixel's magnetogram stream through LDS in tiles. Every
// output is written by exactly one lane: deterministic, no atomics. FP64 in an FP64 context; in an
// FP32C context the far pairs in FP32 (cascaded into FP64) and the near pairs in FP64.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "dbie_solver.h"

namespace dbie {

constexpr int kVjpPts = 64;      // points per LDS tile
constexpr int kVjpCoef = 15;     // Lambda[3], alpha[3], beta[3], gx[3], gy[3]
constexpr double kInv2Pi_v = 0.15915494309189533577;
constexpr int kVjpPix = 4;       // pixels per lane of the FP32C adjoint
constexpr int kVjpPix64 = 2;     // pixels per lane of the FP64 adjoint

struct PixTile {
    int32_t b;
    int32_t start;   // first pixel
};

__global__ void k_vjp_coef(int64_t N, const BoundaryDev* __restrict__ bnd, Geo geo,
                           const double* __restrict__ lam, const double* __restrict__ gB,
                           const double* __restrict__ gdB, double* __restrict__ coef) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const BoundaryDev bd = bnd[geo.bidx[i]];
    const double w = geo.w[i], h = bd.h;
    for (int p = 0; p < 3; ++p) {
        const double b = gB ? gB[p * N + i] : 0.0;
        const double gx = gdB ? gdB[(3 * p + 0) * N + i] : 0.0;
        const double gy = gdB ? gdB[(3 * p + 1) * N + i] : 0.0;
        const double gz = gdB ? gdB[(3 * p + 2) * N + i] : 0.0;
        coef[(0 + p) * N + i] = lam[p * N + i] * h;
        coef[(3 + p) * N + i] = w * kInv2Pi_v * b + gz * kInv2Pi_v / h;
        coef[(6 + p) * N + i] = w * w * gz * kInv2Pi_v / h;
        coef[(9 + p) * N + i] = -w * gx * kInv2Pi_v / h;
        coef[(12 + p) * N + i] = -w * gy * kInv2Pi_v / h;
    }
}

template <int PPX, bool ROWQ>
__global__ __launch_bounds__(256) void k_vjp64(const PixTile* __restrict__ ptiles,
                                               const BoundaryDev* __restrict__ bnd,
                                               const int64_t* __restrict__ seg, Geo geo, int64_t N,
                                               const double* __restrict__ gpos,
                                               const double* __restrict__ coef, double* __restrict__ gW,
                                               int64_t slice_stride) {
    // sc rows: Lambda[3], alpha[3], then -3 beta[3], -3 gx[3], -3 gy[3] and -Lambda^2/3 [3], so that
    // H rho^-5 (beta + ...) is summed as (N - (Lambda^2/3) rho^2 cos t) rho^-5 (-3 beta + ...).
    // Each lane owns PPX pixels (k, k + 256, ...; ROWQ, every grid row a multiple of PPX long: PPX
    // consecutive pixels of one row, whose dy terms are formed once per point): a point's 21 values
    // read from LDS serve them all.
    __shared__ double su[kVjpPts], sv[kVjpPts], sw2[kVjpPts], sc[kVjpCoef + 3][kVjpPts];
    __shared__ int s_wide;
    const PixTile pt = ptiles[blockIdx.x];
    const BoundaryDev bd = bnd[pt.b];
    const int32_t ngrid = bd.gcols * bd.grows;
    double a[PPX], bb[PPX], acc[PPX][3];
#pragma unroll
    for (int j = 0; j < PPX; ++j) {
        const int32_t k = pt.start + (ROWQ ? PPX * (int32_t)threadIdx.x + j : (int32_t)threadIdx.x + j * 256);
        const bool live = k < ngrid;
        a[j] = live ? gpos[bd.gpos_off + k % bd.gcols] : 0.0;
        bb[j] = live ? gpos[bd.gpos_off + bd.gcols + k / bd.gcols] : 0.0;
        acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
    }
    const int64_t s0 = seg[pt.b], s1 = seg[pt.b + 1];
    const int64_t nch = (s1 - s0 + kVjpPts - 1) / kVjpPts;
    const int64_t p0 = s0 + (int64_t)blockIdx.y * nch / gridDim.y * kVjpPts;
    const int64_t p1 = min(s1, s0 + (int64_t)(blockIdx.y + 1) * nch / gridDim.y * kVjpPts);
    for (int64_t i0 = p0; i0 < p1; i0 += kVjpPts) {
        const int n = (int)min<int64_t>(kVjpPts, p1 - i0);
        __syncthreads();
        if (threadIdx.x == 0) s_wide = 0;
        __syncthreads();
        for (int q = threadIdx.x; q < n; q += blockDim.x) {
            const int64_t i = i0 + q;
            const double u = geo.u[i], v = geo.v[i], w = geo.w[i];
            su[q] = u;
            sv[q] = v;
            sw2[q] = w * w;
            // the largest |lambda r| of this point over the grid (positions in [0, nx-1] x [0, ny-1])
            // selects the sin/cos of the chunk: the branch-free reduced form or the library's
            const double dxm = fmax(fabs(u), fabs((double)(bd.nx - 1) - u));
            const double dym = fmax(fabs(v), fabs((double)(bd.ny - 1) - v));
            const double lmax = fmax(fabs(coef[i]), fmax(fabs(coef[N + i]), fabs(coef[2 * N + i])));
            if (!(lmax * sqrt(dxm * dxm + dym * dym + w * w) < kSincosBound)) s_wide = 1;
        }
        for (int q = threadIdx.x; q < (kVjpCoef + 3) * n; q += blockDim.x) {
            const int r = q / n, e = q - r * n;
            if (r < kVjpCoef) {
                const double v = coef[r * N + i0 + e];
                sc[r][e] = r >= 6 ? -3.0 * v : v;
            } else {
                const double l = coef[(r - kVjpCoef) * N + i0 + e];
                sc[r][e] = l * l * (-1.0 / 3.0);
            }
        }
        __syncthreads();
        double part[PPX][3];
#pragma unroll
        for (int j = 0; j < PPX; ++j) part[j][0] = part[j][1] = part[j][2] = 0.0;
        // the chunk's pairs, with the library's sin/cos (WIDE) or the branch-free reduced form
        auto chunk = [&](auto wide_tag) {
            constexpr bool WIDE = decltype(wide_tag)::value;
            for (int e = 0; e < n; ++e) {
                const double ue = su[e], ve = sv[e], w2 = sw2[e];
                double L[3], al[3], be[3], gx[3], gy[3], l3[3];
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    L[p] = sc[p][e];
                    al[p] = sc[3 + p][e];
                    be[p] = sc[6 + p][e];
                    gx[p] = sc[9 + p][e];
                    gy[p] = sc[12 + p][e];
                    l3[p] = sc[kVjpCoef + p][e];
                }
                // ROWQ: the lane's pixels share dy, dy^2 + w^2 and -3 (beta + gy dy), the same values the
                // per-pixel form computes
                double dyq = 0.0, qq = 0.0, cq[3] = {0.0, 0.0, 0.0};
                if (ROWQ) {
                    dyq = bb[0] - ve;
                    qq = __builtin_fma(dyq, dyq, w2);
#pragma unroll
                    for (int p = 0; p < 3; ++p) cq[p] = __builtin_fma(gy[p], dyq, be[p]);
                }
#pragma unroll
                for (int j = 0; j < PPX; ++j) {
                    const double dx = a[j] - ue, dy = ROWQ ? dyq : bb[j] - ve;
                    const double r2 = __builtin_fma(dx, dx, ROWQ ? qq : __builtin_fma(dy, dy, w2));
                    const double ri = WIDE ? rsqrt(r2) : rsqrt_pos(r2);
                    const double r = r2 * ri;
                    const double ri2 = ri * ri;
                    const double ri3 = ri2 * ri;
                    const double ri5 = ri3 * ri2;
#pragma unroll
                    for (int p = 0; p < 3; ++p) {
                        const double t = L[p] * r;
                        double sn, cs;
                        // (the table form of the forward kernel measured slower here: its three LDS
                        // gathers per pair join this kernel's own 5.6 LDS reads per pair)
                        if (WIDE) {
                            sincos(t, &sn, &cs);
                        } else {
                            const uint64_t sg = sincos_halfturn(t, &sn, &cs);   // t = k pi + r: (-1)^k
                            sn = flip_sign(sn, sg);
                            cs = flip_sign(cs, sg);
                        }
                        const double nn = __builtin_fma(t, sn, cs);
                        const double q = __builtin_fma(l3[p] * r2, cs, nn);   // -H / 3
                        const double lin = __builtin_fma(gx[p], dx, ROWQ ? cq[p] : __builtin_fma(gy[p], dy, be[p]));
                        part[j][p] = __builtin_fma(nn * ri3, al[p], __builtin_fma(q * ri5, lin, part[j][p]));
                    }
                }
            }
        };
        if (s_wide != 0) chunk(std::true_type{});
        else chunk(std::false_type{});
#pragma unroll
        for (int j = 0; j < PPX; ++j)
            for (int p = 0; p < 3; ++p) acc[j][p] += part[j][p];
    }
    double* out = gW + (int64_t)blockIdx.y * slice_stride;
#pragma unroll
    for (int j = 0; j < PPX; ++j) {
        const int32_t k = pt.start + (ROWQ ? PPX * (int32_t)threadIdx.x + j : (int32_t)threadIdx.x + j * 256);
        if (k < ngrid) {
            const int64_t o = bd.gpl_off + k;
            for (int p = 0; p < 3; ++p) out[o + (int64_t)p * ngrid] = acc[j][p];
        }
    }
}

// ---- FP32C adjoint --------------------------------------------------------------------------
// Same transpose in FP32, PPX pixels per lane (the point data read from LDS is shared by them),
// FP32 partials per point tile cascaded into FP64. Pairs classified near in dbie_init are skipped
// here (point tiles holding such points take a masked loop) and added in FP64 by k_vjp_near.
constexpr int kVjp32Pts = 64;
constexpr int kVjp32F = 29;   // per point: xi_int, xi_frac, yi_int, yi_frac, w^2, -Lambda^2/3 [3],
                              // Lambda/2pi [3], alpha[3], -3 beta[3], -3 gx[3], -3 gy[3], window a,
                              // window b, mask (as bits), Lambda [3]

// GRID (9-node elements): output j sits at (a + af, b + bf) (integer part + fraction) and belongs to
// element (ea, eb); the near mask is per element of the 3x3 window. ROWQ: the lane's PPX outputs are
// consecutive points of one grid row, so dy, dy^2 + w^2 and -3 (beta + gy dy) are formed once per
// point for all of them.
template <int PPX, bool SLOW, bool GRID, bool FRACT, bool ROWQ>
__device__ __forceinline__ void vjp32_point(const float (*sp)[kVjp32Pts], int e, const float a[PPX],
                                            const float b[PPX], const float af[PPX], const float bf[PPX],
                                            const float ea[PPX], const float eb[PPX], float (&acc)[PPX][3]) {
    const float X = sp[0][e], xf = sp[1][e], Y = sp[2][e], yf = sp[3][e], w2 = sp[4][e];
    float dyq = 0.0f, qq = 0.0f, cq[3] = {0.0f, 0.0f, 0.0f};
    if (ROWQ) {
        dyq = GRID ? (b[0] - Y) + (bf[0] - yf) : (b[0] - Y) - yf;
        qq = fmaf(dyq, dyq, w2);
#pragma unroll
        for (int p = 0; p < 3; ++p) cq[p] = fmaf(sp[20 + p][e], dyq, sp[14 + p][e]);
    }
#pragma unroll
    for (int j = 0; j < PPX; ++j) {
        const float dx = GRID ? (a[j] - X) + (af[j] - xf) : (a[j] - X) - xf;
        const float dy = ROWQ ? dyq : (GRID ? (b[j] - Y) + (bf[j] - yf) : (b[j] - Y) - yf);
        float keep = 1.0f;
        if (SLOW && GRID) {
            const float da = ea[j] - sp[23][e], db = eb[j] - sp[24][e];
            const bool in = fabsf(da) <= (float)kNearWinQ && fabsf(db) <= (float)kNearWinQ;
            const int bit = in ? (int)(da + (float)kNearWinQ) + kNearSideQ * (int)(db + (float)kNearWinQ) : 0;
            if (in && ((__float_as_uint(sp[25][e]) >> bit) & 1u)) keep = 0.0f;
        } else if (SLOW) {
            const float da = a[j] - sp[23][e], db = b[j] - sp[24][e];
            const bool in = fabsf(da) <= (float)kNearWin && fabsf(db) <= (float)kNearWin;
            const int bit = in ? (int)(da + (float)kNearWin) + kNearSide * (int)(db + (float)kNearWin) : 0;
            if (in && ((__float_as_uint(sp[25][e]) >> bit) & 1u)) keep = 0.0f;
        }
        const float r2 = fmaf(dx, dx, ROWQ ? qq : fmaf(dy, dy, w2));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * ri;
        const float ri2 = ri * ri * keep;   // a skipped pair zeroes both terms through 1 / r^2
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            // phase in revolutions; FRACT (a chunk beyond the sin/cos range): minus its nearest
            // integer, formed from the exact product by one FMA
            const float th = sp[8 + p][e] * r;
            const float tr = FRACT ? fmaf(sp[8 + p][e], r, -__builtin_rintf(th)) : th;
            const float sn = __builtin_amdgcn_sinf(tr);
            const float cs = __builtin_amdgcn_cosf(tr);
            // t = Lambda r is never formed: N / r^3 = (Lambda sin t + cos t / r) / r^2, and
            // -H / 3 / r^5 = (N / r^3 + (-Lambda^2 / 3) cos t / r) / r^2; the -3 sits in the staged
            // coefficients of lin
            const float cri = cs * ri;
            const float nr3 = fmaf(sp[26 + p][e], sn, cri) * ri2;
            const float hr5 = fmaf(sp[5 + p][e], cri, nr3) * ri2;
            const float lin = fmaf(sp[17 + p][e], dx, ROWQ ? cq[p] : fmaf(sp[20 + p][e], dy, sp[14 + p][e]));
            acc[j][p] = fmaf(nr3, sp[11 + p][e], fmaf(hr5, lin, acc[j][p]));
        }
    }
}

// Outputs are the quadrature grid points (the pixels for the nodal rule), written to gW at the
// grid's plane offsets. Lane t owns the tile's points t, t + 256, ... or, ROWQ (every grid row a
// multiple of PPX long), the PPX consecutive points PPX t .. PPX t + PPX - 1, which share a row.
template <int PPX, bool GRID, bool ROWQ>
__global__ __launch_bounds__(256) void k_vjp32c(const PixTile* __restrict__ ptiles,
                                                const BoundaryDev* __restrict__ bnd,
                                                const int64_t* __restrict__ seg, const int32_t* __restrict__ perm,
                                                const float4* __restrict__ gposf, Geo geo, int64_t N,
                                                const double* __restrict__ coef, double* __restrict__ gW,
                                                int64_t slice_stride) {
    __shared__ float sp[kVjp32F][kVjp32Pts];
    __shared__ int any_near, any_far;
    const PixTile pt = ptiles[blockIdx.x];
    const BoundaryDev bd = bnd[pt.b];
    const int32_t ngrid = bd.gcols * bd.grows;
    float a[PPX], b[PPX], af[PPX], bf[PPX], ea[PPX], eb[PPX];
    bool live[PPX];
#pragma unroll
    for (int j = 0; j < PPX; ++j) {
        const int32_t k = pt.start + (ROWQ ? PPX * (int32_t)threadIdx.x + j : (int32_t)threadIdx.x + j * 256);
        live[j] = k < ngrid;
        const int32_t kc = live[j] ? k % bd.gcols : 0, kr = live[j] ? k / bd.gcols : 0;
        if (GRID) {
            const float4 pc = gposf[bd.gposf_off + kc];
            const float4 pr = gposf[bd.gposf_off + (int64_t)bd.ntx * kCols + kr];
            a[j] = pc.x;
            af[j] = pc.y;
            ea[j] = pc.z;
            b[j] = pr.x;
            bf[j] = pr.y;
            eb[j] = pr.z;
        } else {
            a[j] = (float)kc;
            b[j] = (float)kr;
            af[j] = bf[j] = ea[j] = eb[j] = 0.0f;
        }
    }
    double tot[PPX][3];
    float part[PPX][3];
#pragma unroll
    for (int j = 0; j < PPX; ++j)
        for (int p = 0; p < 3; ++p) tot[j][p] = 0.0;
    // point slice blockIdx.y of gridDim.y: an even share of the boundary's 64-point chunks
    const int64_t s0 = seg[pt.b], s1 = seg[pt.b + 1];
    const int64_t nch = (s1 - s0 + kVjp32Pts - 1) / kVjp32Pts;
    const int64_t p0 = s0 + (int64_t)blockIdx.y * nch / gridDim.y * kVjp32Pts;
    const int64_t p1 = min(s1, s0 + (int64_t)(blockIdx.y + 1) * nch / gridDim.y * kVjp32Pts);
    for (int64_t i0 = p0; i0 < p1; i0 += kVjp32Pts) {
        const int n = (int)min<int64_t>(kVjp32Pts, p1 - i0);
        __syncthreads();
        if (threadIdx.x == 0) {
            any_near = 0;
            any_far = 0;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int64_t i = perm ? (int64_t)perm[i0 + e] : i0 + e;
            sp[0][e] = geo.xi_int[i];
            sp[1][e] = geo.xi_frac[i];
            sp[2][e] = geo.yi_int[i];
            sp[3][e] = geo.yi_frac[i];
            const float wf = geo.wf[i];
            sp[4][e] = wf * wf;
            for (int p = 0; p < 3; ++p) {
                const double L = coef[(0 + p) * N + i];
                sp[5 + p][e] = (float)(L * L * (-1.0 / 3.0));
                sp[8 + p][e] = (float)(L * 0.15915494309189533577);
                sp[26 + p][e] = (float)L;
                sp[11 + p][e] = (float)coef[(3 + p) * N + i];
                sp[14 + p][e] = (float)(-3.0 * coef[(6 + p) * N + i]);
                sp[17 + p][e] = (float)(-3.0 * coef[(9 + p) * N + i]);
                sp[20 + p][e] = (float)(-3.0 * coef[(12 + p) * N + i]);
            }
            sp[23][e] = (float)geo.win_a[i];
            sp[24][e] = (float)geo.win_b[i];
            const uint32_t m = geo.near_mask[i];
            sp[25][e] = __uint_as_float(m);
            if (m) any_near = 1;
            {
                // the largest |Lambda| r / 2pi of this point over the magnetogram's grid (positions in
                // [0, nx-1] x [0, ny-1]); beyond the hardware sin/cos range the chunk reduces first
                const float uf = sp[0][e] + sp[1][e], vf = sp[2][e] + sp[3][e];
                const float dxm = fmaxf(fabsf(uf), fabsf((float)(bd.nx - 1) - uf)) + 1.0f;
                const float dym = fmaxf(fabsf(vf), fabsf((float)(bd.ny - 1) - vf)) + 1.0f;
                const float rmax = sqrtf(dxm * dxm + dym * dym + sp[4][e]);
                const float lmax = fmaxf(fabsf(sp[8][e]), fmaxf(fabsf(sp[9][e]), fabsf(sp[10][e])));
                if (!(lmax * rmax < 255.0f)) any_far = 1;   // NaN lambda included
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PPX; ++j)
            for (int p = 0; p < 3; ++p) part[j][p] = 0.0f;
        if (any_far) {
            if (any_near)
                for (int e = 0; e < n; ++e) vjp32_point<PPX, true, GRID, true, ROWQ>(sp, e, a, b, af, bf, ea, eb, part);
            else
                for (int e = 0; e < n; ++e) vjp32_point<PPX, false, GRID, true, ROWQ>(sp, e, a, b, af, bf, ea, eb, part);
        } else {
            if (any_near)
                for (int e = 0; e < n; ++e) vjp32_point<PPX, true, GRID, false, ROWQ>(sp, e, a, b, af, bf, ea, eb, part);
            else
                for (int e = 0; e < n; ++e) vjp32_point<PPX, false, GRID, false, ROWQ>(sp, e, a, b, af, bf, ea, eb, part);
        }
#pragma unroll
        for (int j = 0; j < PPX; ++j)
            for (int p = 0; p < 3; ++p) tot[j][p] += (double)part[j][p];
    }
#pragma unroll
    for (int j = 0; j < PPX; ++j) {
        if (!live[j]) continue;
        const int64_t o = bd.gpl_off + pt.start + (ROWQ ? PPX * (int64_t)threadIdx.x + j : (int64_t)threadIdx.x + j * 256);
        double* out = gW + (int64_t)blockIdx.y * slice_stride;
        for (int p = 0; p < 3; ++p) out[o + (int64_t)p * ngrid] = tot[j][p];
    }
}

// gW[e] = sum over the point slices, in order, of their partial outputs.
__global__ void k_vjp_reduce(int64_t n, int32_t S, const double* __restrict__ parts, double* __restrict__ gW) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double a = parts[e];
    for (int32_t y = 1; y < S; ++y) a += parts[(int64_t)y * n + e];
    gW[e] = a;
}

// FP64 near pairs of the adjoint: grid point g (global index over all boundaries) gathers the points
// listed in near_pts[near_ptr[g] .. near_ptr[g+1]) (sorted by point) and adds to its output.
__global__ void k_vjp_near(int64_t npix_total, const int32_t* __restrict__ near_ptr,
                           const int32_t* __restrict__ near_pts, const int32_t* __restrict__ pix_bnd,
                           const BoundaryDev* __restrict__ bnd, const double* __restrict__ gpos, Geo geo,
                           int64_t N, const double* __restrict__ coef, double* __restrict__ gW) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npix_total) return;
    const int32_t s0 = near_ptr[g], s1 = near_ptr[g + 1];
    if (s0 == s1) return;
    const BoundaryDev bd = bnd[pix_bnd[g]];
    const int64_t k = g - bd.gpl_off / 3;
    const int64_t ngrid = (int64_t)bd.gcols * bd.grows;
    const double a = gpos[bd.gpos_off + k % bd.gcols], bb = gpos[bd.gpos_off + bd.gcols + k / bd.gcols];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int32_t q = s0; q < s1; ++q) {
        const int64_t i = near_pts[q];
        const double dx = a - geo.u[i], dy = bb - geo.v[i], w = geo.w[i];
        const double r2 = __builtin_fma(dx, dx, __builtin_fma(dy, dy, w * w));
        const double ri = rsqrt(r2);
        const double r = r2 * ri;
        const double ri2 = ri * ri;
        const double ri3 = ri2 * ri;
        const double ri5 = ri3 * ri2;
        for (int p = 0; p < 3; ++p) {
            const double t = coef[(0 + p) * N + i] * r;
            double sn, cs;
            sincos(t, &sn, &cs);
            const double nn = __builtin_fma(t, sn, cs);
            const double hh = __builtin_fma(t, t * cs, -3.0 * nn);
            const double lin = __builtin_fma(coef[(9 + p) * N + i], dx,
                                             __builtin_fma(coef[(12 + p) * N + i], dy, coef[(6 + p) * N + i]));
            acc[p] = __builtin_fma(nn * ri3, coef[(3 + p) * N + i], __builtin_fma(hh * ri5, lin, acc[p]));
        }
    }
    for (int p = 0; p < 3; ++p) gW[bd.gpl_off + (int64_t)p * ngrid + k] += acc[p];
}

// g_mu_p = gB_p tan[p] + sum_q gdB[3p+q] tan[3+3p+q]; g_lambda = 2 lambda g_mu.
__global__ void k_grad_lambda(int64_t N, const double* __restrict__ lam, const double* __restrict__ gB,
                              const double* __restrict__ gdB, const double* __restrict__ tan,
                              double* __restrict__ glam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int p = 0; p < 3; ++p) {
        double g = gB ? gB[p * N + i] * tan[p * N + i] : 0.0;
        if (gdB)
            for (int q = 0; q < 3; ++q) g += gdB[(3 * p + q) * N + i] * tan[(3 + 3 * p + q) * N + i];
        glam[p * N + i] = 2.0 * lam[p * N + i] * g;
    }
}

__global__ void k_resid_jac(int64_t N, const BoundaryDev* __restrict__ bnd, const int32_t* __restrict__ bidx,
                            double dvds, const double* __restrict__ B, const double* __restrict__ dB,
                            const double* __restrict__ tan, double* __restrict__ jac_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double h = bnd[bidx[i]].h;
    double b[3], d[9], t[12], jac[12];
    for (int p = 0; p < 3; ++p) b[p] = B[p * N + i];
    for (int r = 0; r < 9; ++r) d[r] = dB[r * N + i];
    for (int r = 0; r < 12; ++r) t[r] = tan[r * N + i];
    residual_jacobian_fp64(b, d, t, dvds * h, jac);
    for (int r = 0; r < 12; ++r) jac_out[r * N + i] = jac[r];
}

}  // namespace dbie

using namespace dbie;

namespace dbie {
// Pixel tiles of the two adjoint kernels and the workspace sizes of dbie_grad's gB0 part.
// Pixel tiles of every boundary's grid: 256 * kVjpPix64 grid points each (FP64 kernel) and
// 256 * kVjpPix (FP32C kernel), uploaded once with the point segments.
hipError_t vjp_tables_init(const dbie_ctx* c, void** dev, VjpTables* t) {
    std::vector<PixTile> pt;
    const int32_t nb = ctx_nb(c);
    for (int per : {256 * kVjpPix64, 256 * kVjpPix}) {
        for (int32_t b = 0; b < nb; ++b) {
            const BoundaryDev& bd = ctx_bnd_host(c, b);
            for (int32_t k = 0; k < bd.gcols * bd.grows; k += per) pt.push_back(PixTile{b, k});
        }
        if (per == 256 * kVjpPix64) t->n64 = (int64_t)pt.size();
    }
    t->n32 = (int64_t)pt.size() - t->n64;
    t->seg_off = (pt.size() * sizeof(PixTile) + 255) / 256 * 256;
    const size_t bytes = t->seg_off + (size_t)(nb + 1) * sizeof(int64_t);
    *dev = nullptr;
    hipError_t e = hipMalloc(dev, bytes);
    if (e == hipSuccess) e = hipMemcpy(*dev, pt.data(), pt.size() * sizeof(PixTile), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy((char*)*dev + t->seg_off, ctx_seg(c), (size_t)(nb + 1) * sizeof(int64_t),
                      hipMemcpyHostToDevice);
    t->base = *dev;
    return e;
}

struct GradPlan {
    int32_t S;                  // point slices of the transpose launch
    size_t szc, szg, szp;
    size_t bytes() const { return szc + szg + szp; }
};

static GradPlan grad_plan(const dbie_ctx* c) {
    GradPlan g;
    const int32_t nb = ctx_nb(c);
    const VjpTables vt = ctx_vjp_tables(c);
    const QuadGrid grid = ctx_grid(c);
    // Point slices: the pixel tiles alone are few for small magnetograms (16 workgroups for 128^2 in
    // FP32C); about four workgroups per compute unit, at least one 64-point chunk per slice.
    const size_t tiles = (size_t)(ctx_precision(c) == DBIE_FP64 ? vt.n64 : vt.n32);
    int64_t maxseg = 0;
    for (int32_t b = 0; b < nb; ++b) maxseg = std::max(maxseg, ctx_seg(c)[b + 1] - ctx_seg(c)[b]);
    const int64_t want = (1024 + (int64_t)std::max<size_t>(tiles, 1) - 1) / (int64_t)std::max<size_t>(tiles, 1);
    g.S = (int32_t)std::max<int64_t>(1, std::min<int64_t>({want, 64, (maxseg + 63) / 64}));
    g.szc = ((size_t)std::max<int64_t>(ctx_n(c), 1) * kVjpCoef * sizeof(double) + 255) / 256 * 256;
    g.szg = grid.G ? (size_t)grid.n_total * 3 * sizeof(double) : 0;
    g.szp = g.S > 1 ? (size_t)g.S * grid.n_total * 3 * sizeof(double) : 0;
    return g;
}

size_t grad_workspace_bytes(const dbie_ctx* c) { return grad_plan(c).bytes(); }
}  // namespace dbie

extern "C" int dbie_grad(dbie_ctx* c, const double* lam, const double* gB, const double* gdB, double* glam,
                         double* gB0, double* resid_jac, void* stream) {
    if (!c) return DBIE_E_INVAL;
    const int64_t N = ctx_n(c);
    if (N > 0 && !lam) return ctx_fail(c, DBIE_E_INVAL, "lambda is required");
    if (int rc = ctx_check_device(c)) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int32_t nb = ctx_nb(c);
    const Geo& geo = ctx_geo(c);
    const BoundaryDev* bnd = ctx_bnd(c);
    const unsigned gN = (unsigned)((std::max<int64_t>(N, 1) + 255) / 256);
#define GRAD_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) return ctx_fail(c, DBIE_E_DEVICE, hipGetErrorString(e_)); \
    } while (0)
    if (N > 0 && (glam || resid_jac)) {
        double* w = (double*)ctx_scratch(c, 0, (size_t)N * 24 * sizeof(double));
        if (!w) return ctx_fail(c, DBIE_E_WORKSPACE, "cannot allocate the gradient workspace");
        double* Bw = w;
        double* dBw = w + 3 * N;
        double* tw = w + 12 * N;
        int rc = eval_set(c, lam, ctx_precision(c) == DBIE_FP64, true, nullptr, Bw, dBw, nullptr, tw, s);
        if (rc) return rc;
        if (glam) hipLaunchKernelGGL(k_grad_lambda, dim3(gN), dim3(256), 0, s, N, lam, gB, gdB, tw, glam);
        if (resid_jac)
            hipLaunchKernelGGL(k_resid_jac, dim3(gN), dim3(256), 0, s, N, bnd, geo.bidx, ctx_dvds(c), Bw, dBw,
                               tw, resid_jac);
        GRAD_HIP(hipGetLastError());
    }
    if (gB0) {
        // pixel tiles of every boundary, and the point segments on the device
        const QuadGrid grid = ctx_grid(c);
        const GradPlan gp = grad_plan(c);
        const VjpTables vt = ctx_vjp_tables(c);
        char* w = (char*)ctx_scratch(c, 1, gp.bytes());
        if (!w) return ctx_fail(c, DBIE_E_WORKSPACE, "cannot allocate the adjoint workspace");
        double* coef = (double*)w;
        double* gW = grid.G ? (double*)(w + gp.szc) : gB0;
        // with point slices the transpose kernels write S partial outputs, reduced into gW in order
        const int64_t T3 = grid.n_total * 3;
        double* parts = gp.S > 1 ? (double*)(w + gp.szc + gp.szg) : gW;
        const PixTile* ptd = (const PixTile*)vt.base;
        const PixTile* ptd32 = ptd + vt.n64;
        const int64_t* segd = (const int64_t*)((const char*)vt.base + vt.seg_off);
        if (N > 0)
            hipLaunchKernelGGL(k_vjp_coef, dim3(gN), dim3(256), 0, s, N, bnd, geo, lam, gB, gdB, coef);
        const dim3 g64((unsigned)vt.n64, (unsigned)gp.S), g32((unsigned)vt.n32, (unsigned)gp.S);
        if (ctx_precision(c) == DBIE_FP64) {
            // rows of a multiple of kVjpPix64 points (tiles start at multiples of it): each lane's
            // outputs share one row
            bool rowq = true;
            for (int32_t b = 0; b < ctx_nb(c); ++b) rowq = rowq && ctx_bnd_host(c, b).gcols % kVjpPix64 == 0;
            if (rowq)
                hipLaunchKernelGGL((k_vjp64<kVjpPix64, true>), g64, dim3(256), 0, s, ptd, bnd, segd, geo, N, grid.pos,
                                   coef, parts, T3);
            else
                hipLaunchKernelGGL((k_vjp64<kVjpPix64, false>), g64, dim3(256), 0, s, ptd, bnd, segd, geo, N, grid.pos,
                                   coef, parts, T3);
        } else {
            // rows of a multiple of kVjpPix points (and tiles starting at multiples of it): each lane's
            // outputs share one row
            bool rowq = true;
            for (int32_t b = 0; b < ctx_nb(c); ++b) rowq = rowq && ctx_bnd_host(c, b).gcols % kVjpPix == 0;
            if (grid.G && rowq)
                hipLaunchKernelGGL((k_vjp32c<kVjpPix, true, true>), g32, dim3(256), 0, s, ptd32, bnd, segd,
                                   ctx_perm(c), grid.posf, geo, N, coef, parts, T3);
            else if (grid.G)
                hipLaunchKernelGGL((k_vjp32c<kVjpPix, true, false>), g32, dim3(256), 0, s, ptd32, bnd, segd,
                                   ctx_perm(c), grid.posf, geo, N, coef, parts, T3);
            else if (rowq)
                hipLaunchKernelGGL((k_vjp32c<kVjpPix, false, true>), g32, dim3(256), 0, s, ptd32, bnd, segd,
                                   ctx_perm(c), grid.posf, geo, N, coef, parts, T3);
            else
                hipLaunchKernelGGL((k_vjp32c<kVjpPix, false, false>), g32, dim3(256), 0, s, ptd32, bnd, segd,
                                   ctx_perm(c), grid.posf, geo, N, coef, parts, T3);
        }
        if (gp.S > 1)
            hipLaunchKernelGGL(k_vjp_reduce, dim3((unsigned)((T3 + 255) / 256)), dim3(256), 0, s, T3, gp.S, parts, gW);
        if (ctx_precision(c) != DBIE_FP64) {
            const NearLists nl = ctx_near_lists(c);
            if (nl.n_pairs > 0)
                hipLaunchKernelGGL(k_vjp_near, dim3((unsigned)((nl.npix_total + 255) / 256)), dim3(256), 0, s,
                                   nl.npix_total, nl.ptr, nl.pts, nl.pix_bnd, bnd, grid.pos, geo, N, coef, gW);
        }
        if (grid.G)
            for (int32_t b = 0; b < nb; ++b)
                GRAD_HIP(launch_quad_transpose(ctx_bnd_host(c, b), gW, grid.lw, grid.G, gB0, s));
        GRAD_HIP(hipGetLastError());
    }
    return DBIE_OK;
#undef GRAD_HIP
}
