// FP64 bulk kernel sum (every pair in FP64): the Eq. (16) nodal sum of the Eq. (6) kernel (or the
// Eq. (15) element quadrature, over its grid of Gauss points) and its frozen-lambda gradient rows
// (Eq. 13 limit), optionally with the mu-tangent rows.
//
// Grid: one workgroup per schedule tile (a run of <= tile points of one magnetogram) and one
// grid row per lambda trial. Each lane owns one point; the magnetogram streams through LDS in
// tiles of kTP64 pixels that all lanes read at the same address (LDS broadcast). Sums are cascaded:
// a per-tile partial in FP64, then added to the running FP64 total. Grid z splits the pixel tiles
// into slices (few points: late solver rounds, the acceptance of converged points, field-line seeds),
// each writing its own partial ([S][L][kAcc][N], added in order by the finalize pass). sin and cos
// come from the branch-free reduced form unless some pair of the workgroup's points can exceed its
// argument bound (then, and for NaN lambda, from the device library).
//
// OVR (FP32C contexts, after the FP32 bulk pass): the same sums in FP64 for the points whose phase
// can exceed the FP32 accuracy bound, max_p |lambda_p| r_max > phase_max with r_max the largest
// distance from the point to its magnetogram's quadrature grid. Only those points' partial sums are
// overwritten (every slice); their near-field pairs, which the finalize pass adds in FP64 as for every
// FP32C point, are subtracted here, so that each pair is counted once. It runs with one wavefront per
// workgroup, and a run of 64 points without such a point skips the pair loop.
#include "dbie_internal.h"

namespace dbie {

constexpr int kTP64 = 128;

template <bool TAN, bool OVR>
__global__ __launch_bounds__(256) void k_field64(const Tile* __restrict__ tiles,
                                                 const BoundaryDev* __restrict__ bnd,
                                                 const double* __restrict__ gpos,
                                                 const double* __restrict__ gB, Geo geo,
                                                 const double* __restrict__ lam, int64_t N,
                                                 const int32_t* __restrict__ idx,
                                                 double* __restrict__ acc, const double* __restrict__ B0d,
                                                 double phase_max) {
    constexpr int NA = TAN ? kAcc : kAccField;
    __shared__ double sa[kTP64], sb[kTP64], sx[kTP64], sy[kTP64], sz[kTP64];
    __shared__ double2 stab[32];   // (sin, cos)(j pi / 16) for sincos_table16
    __shared__ int s_wide, s_any;
    if (threadIdx.x < 32) stab[threadIdx.x] = make_double2(kSinCos16[2 * threadIdx.x], kSinCos16[2 * threadIdx.x + 1]);
    const Tile t = tiles[blockIdx.x];
    const int trial = blockIdx.y;
    const BoundaryDev bd = bnd[t.b];
    const double* B0 = gB + bd.gpl_off;
    const double* cpos = gpos + bd.gpos_off;
    const double* rpos = cpos + bd.gcols;
    const int32_t npix = bd.gcols * bd.grows;
    for (int c0 = 0; c0 < t.count; c0 += blockDim.x) {
        const int j = c0 + (int)threadIdx.x;
        const bool live = j < t.count;
        const int64_t e = t.start + (live ? j : 0);
        const int64_t i = idx ? (int64_t)idx[e] : e;
        const double u = geo.u[i], v = geo.v[i], w = geo.w[i];
        const double w2 = w * w;
        double lm[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) lm[p] = lam[((int64_t)trial * 3 + p) * N + i] * bd.h;
        // the largest |lambda r| of the workgroup's pairs (grid positions lie in [0, nx - 1] x
        // [0, ny - 1]) selects the sin/cos: the branch-free reduced form, or the library's for
        // arguments beyond its range (and for NaN lambda)
        bool mine = live;   // OVR: this lane's point is recomputed
        {
            const double dxm = fmax(fabs(u), fabs((double)(bd.nx - 1) - u));
            const double dym = fmax(fabs(v), fabs((double)(bd.ny - 1) - v));
            const double rmax = sqrt(dxm * dxm + dym * dym + w2);
            const double tmax = fmax(fabs(lm[0]), fmax(fabs(lm[1]), fabs(lm[2]))) * rmax;
            if (OVR) mine = live && !(tmax <= phase_max);   // NaN lambda included
            __syncthreads();
            if (threadIdx.x == 0) s_wide = s_any = 0;
            __syncthreads();
            if (mine && !(tmax < kSincosBound)) s_wide = 1;
            if (OVR && mine) s_any = 1;
            __syncthreads();
        }
        const bool wide = s_wide != 0;
        if (OVR && s_any == 0) continue;   // uniform over the workgroup
        double tot[NA];
#pragma unroll
        for (int r = 0; r < NA; ++r) tot[r] = 0.0;
        // pixel slice blockIdx.z of gridDim.z: an even share of the pixel tiles
        const int ntile = (npix + kTP64 - 1) / kTP64;
        const int kt0 = (int)((int64_t)blockIdx.z * ntile / gridDim.z);
        const int kt1 = (int)((int64_t)(blockIdx.z + 1) * ntile / gridDim.z);
        for (int k0 = kt0 * kTP64; k0 < min(npix, kt1 * kTP64); k0 += kTP64) {
            const int kn = min(kTP64, npix - k0);
            __syncthreads();
            for (int k = threadIdx.x; k < kn; k += blockDim.x) {
                const int kk = k0 + k;
                sa[k] = cpos[kk % bd.gcols];
                sb[k] = rpos[kk / bd.gcols];
                sx[k] = B0[kk];
                sy[k] = B0[npix + kk];
                sz[k] = B0[2 * npix + kk];
            }
            __syncthreads();
            double part[NA];
#pragma unroll
            for (int r = 0; r < NA; ++r) part[r] = 0.0;
            // the tile's pixels row by row: dy is the same along a row, so the y-moment rows come
            // from per-row sums (A2 += dy (sum of A3 terms), T2 += dy (sum of A0 terms))
            for (int k = 0; k < kn;) {
                const int kend = min(kn, ((k0 + k) / bd.gcols + 1) * bd.gcols - k0);   // uniform
                const double dy = sb[k] - v;
                const double q = __builtin_fma(dy, dy, w2);
                double rs[TAN ? 6 : 3];
#pragma unroll
                for (int r = 0; r < (TAN ? 6 : 3); ++r) rs[r] = 0.0;
                if (wide)
                    for (; k < kend; ++k) pair_fp64_row<TAN, true>(sa[k] - u, q, lm, sx[k], sy[k], sz[k], part, rs);
                else
                    for (; k < kend; ++k)
                        pair_fp64_row<TAN, false, true>(sa[k] - u, q, lm, sx[k], sy[k], sz[k], part, rs, stab);
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    part[4 * p + 3] += rs[p];
                    part[4 * p + 2] = __builtin_fma(dy, rs[p], part[4 * p + 2]);
                    if (TAN) {
                        part[4 * p + 0] += rs[3 + p];
                        part[12 + 3 * p + 2] = __builtin_fma(dy, rs[3 + p], part[12 + 3 * p + 2]);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < NA; ++r) tot[r] += part[r];
        }
        if (OVR && mine && blockIdx.z == 0) {
            // the finalize pass adds this point's near pairs: take them out of the full sum
            const uint32_t mask = geo.near_mask[i];
            if (mask) {
                double nr[NA];
#pragma unroll
                for (int r = 0; r < NA; ++r) nr[r] = 0.0;
                const bool wn = !(fmax(fabs(lm[0]), fmax(fabs(lm[1]), fabs(lm[2]))) * 64.0 < kSincosBound);
                if (bd.G > 0) {
                    if (wn) add_near_grid<TAN, true>(bd, gpos, gB, mask, geo.win_a[i], geo.win_b[i], u, v, w2, lm, nr);
                    else add_near_grid<TAN, false>(bd, gpos, gB, mask, geo.win_a[i], geo.win_b[i], u, v, w2, lm, nr);
                } else {
                    if (wn) add_near<TAN, true>(bd, B0d + bd.pix_off, mask, geo.win_a[i], geo.win_b[i], u, v, w2, lm, nr);
                    else add_near<TAN, false>(bd, B0d + bd.pix_off, mask, geo.win_a[i], geo.win_b[i], u, v, w2, lm, nr);
                }
#pragma unroll
                for (int r = 0; r < NA; ++r) tot[r] -= nr[r];
            }
        }
        if (OVR ? mine : live) {
#pragma unroll
            for (int r = 0; r < NA; ++r)
                acc[(((int64_t)blockIdx.z * gridDim.y + trial) * kAcc + r) * N + i] = tot[r];
        }
    }
}

hipError_t launch_field64(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd,
                          const double* gpos, const double* gB, Geo geo, const double* lam, int64_t N,
                          int32_t L, int32_t S, const int32_t* idx, bool tan, double* acc, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)n_tiles, (unsigned)L, (unsigned)S);
    if (tan)
        hipLaunchKernelGGL((k_field64<true, false>), grid, dim3(256), 0, s, tiles, bnd, gpos, gB, geo, lam, N, idx,
                           acc, nullptr, 0.0);
    else
        hipLaunchKernelGGL((k_field64<false, false>), grid, dim3(256), 0, s, tiles, bnd, gpos, gB, geo, lam, N, idx,
                           acc, nullptr, 0.0);
    return hipGetLastError();
}

hipError_t launch_field64_override(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd, const double* B0d,
                                   const double* gpos, const double* gB, Geo geo, const double* lam, int64_t N,
                                   int32_t L, int32_t S, const int32_t* idx, bool tan, double phase_max, double* acc,
                                   hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    // one wavefront per workgroup: the tile's points are taken 64 at a time, and a run of 64 without a
    // point beyond the bound costs only its test (points beyond it are few and scattered)
    const dim3 grid((unsigned)n_tiles, (unsigned)L, (unsigned)S);
    if (tan)
        hipLaunchKernelGGL((k_field64<true, true>), grid, dim3(64), 0, s, tiles, bnd, gpos, gB, geo, lam, N, idx,
                           acc, B0d, phase_max);
    else
        hipLaunchKernelGGL((k_field64<false, true>), grid, dim3(64), 0, s, tiles, bnd, gpos, gB, geo, lam, N, idx,
                           acc, B0d, phase_max);
    return hipGetLastError();
}

}  // namespace dbie
