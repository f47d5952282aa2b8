// Per-point finish of an evaluation, in FP64: add the near-field pairs (FP32C path), scale the
// pixel-unit sums to B, grad B and the mu-tangents, and compute the residuals f_i (Eq. 8) and
// g_i (Eq. 9) from J = curl B (Eq. 14).
#include "dbie_internal.h"

namespace dbie {

constexpr double kInv2Pi = 0.15915494309189533577;
constexpr double kInv4Pi = 0.07957747154594766788;

// acc rows -> (B[3], dB[9], tan[12]) in physical units (see the scale relations at the top of
// dbie_internal.h).
template <bool TAN>
__device__ __forceinline__ void scale_sums(const double* a, double w, double h, double B[3],
                                           double dB[9], double tn[12]) {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const double A0 = a[4 * p + 0], A1 = a[4 * p + 1], A2 = a[4 * p + 2], A3 = a[4 * p + 3];
        B[p] = w * kInv2Pi * A0;
        dB[3 * p + 0] = -w * kInv2Pi / h * A1;
        dB[3 * p + 1] = -w * kInv2Pi / h * A2;
        dB[3 * p + 2] = kInv2Pi / h * __builtin_fma(w * w, A3, A0);
        if (TAN) {
            const double T0 = a[12 + 3 * p + 0], T1 = a[12 + 3 * p + 1], T2 = a[12 + 3 * p + 2];
            tn[p] = w * h * h * kInv4Pi * T0;
            tn[3 + 3 * p + 0] = w * h * kInv4Pi * T1;
            tn[3 + 3 * p + 1] = w * h * kInv4Pi * T2;
            tn[3 + 3 * p + 2] = h * kInv4Pi * (T0 - w * w * A0);
        }
    }
}

template <bool TAN, bool NEAR>
__global__ __launch_bounds__(256) void k_finalize(const BoundaryDev* __restrict__ bnd,
                                                  const double* __restrict__ B0d,
                                                  const double* __restrict__ gpos,
                                                  const double* __restrict__ gB, Geo geo,
                                                  const double* __restrict__ lam,
                                                  const int32_t* __restrict__ idx, int64_t n_idx,
                                                  const int32_t* __restrict__ n_dev, int64_t N, int32_t L,
                                                  int32_t S, const double* __restrict__ acc, double dvds,
                                                  double* __restrict__ Bo, double* __restrict__ dBo,
                                                  double* __restrict__ fgo, double* __restrict__ tno) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (n_dev ? (int64_t)*n_dev : n_idx)) return;
    const int64_t i = idx ? (int64_t)idx[j] : j;
    const int64_t trial = blockIdx.y;
    const BoundaryDev bd = bnd[geo.bidx[i]];
    constexpr int NA = TAN ? kAcc : kAccField;
    double a[NA];
#pragma unroll
    for (int r = 0; r < NA; ++r) a[r] = acc[(trial * kAcc + r) * N + i];
    for (int z = 1; z < S; ++z) {
        const double* az = acc + ((int64_t)z * L + trial) * kAcc * N;
#pragma unroll
        for (int r = 0; r < NA; ++r) a[r] += az[r * N + i];
    }
    const double w = geo.w[i];
    if (NEAR) {
        const uint32_t mask = geo.near_mask[i];
        if (mask) {
            double lm[3];
#pragma unroll
            for (int p = 0; p < 3; ++p) lm[p] = lam[(trial * 3 + p) * N + i] * bd.h;
            double nr[NA];
#pragma unroll
            for (int r = 0; r < NA; ++r) nr[r] = 0.0;
            // near pairs lie within a few pixels (a 3 x 3 window of elements at most): |lambda r| is
            // bounded by 64 |lambda| pixels
            const bool wide = !(fmax(fabs(lm[0]), fmax(fabs(lm[1]), fabs(lm[2]))) * 64.0 < kSincosBound);
            if (bd.G > 0) {
                if (wide)
                    add_near_grid<TAN, true>(bd, gpos, gB, mask, geo.win_a[i], geo.win_b[i], geo.u[i], geo.v[i],
                                             w * w, lm, nr);
                else
                    add_near_grid<TAN, false>(bd, gpos, gB, mask, geo.win_a[i], geo.win_b[i], geo.u[i], geo.v[i],
                                              w * w, lm, nr);
            } else {
                if (wide)
                    add_near<TAN, true>(bd, B0d + bd.pix_off, mask, geo.win_a[i], geo.win_b[i], geo.u[i], geo.v[i],
                                        w * w, lm, nr);
                else
                    add_near<TAN, false>(bd, B0d + bd.pix_off, mask, geo.win_a[i], geo.win_b[i], geo.u[i],
                                         geo.v[i], w * w, lm, nr);
            }
#pragma unroll
            for (int r = 0; r < NA; ++r) a[r] += nr[r];
        }
    }
    double B[3], dB[9], tn[12];
    scale_sums<TAN>(a, w, bd.h, B, dB, tn);
#pragma unroll
    for (int p = 0; p < 3; ++p) Bo[(trial * 3 + p) * N + i] = B[p];
    if (dBo) {
#pragma unroll
        for (int r = 0; r < 9; ++r) dBo[(trial * 9 + r) * N + i] = dB[r];
    }
    if (TAN && tno) {
#pragma unroll
        for (int r = 0; r < 12; ++r) tno[(trial * 12 + r) * N + i] = tn[r];
    }
    if (fgo) {
        const Resid R = residual_fp64(B, dB, dvds * bd.h);
        fgo[(trial * 2 + 0) * N + i] = R.f;
        fgo[(trial * 2 + 1) * N + i] = R.g;
    }
}

// The pixel slices of the first `rows` rows summed in place into slice 0, in slice order (the
// finalize pass then reads one slice and gets the same sums). One thread per (point, trial, row):
// with few points and many slices the finalize pass's own loop (S x rows loads per thread, one
// thread per point) has too few threads in flight to hide the memory latency.
__global__ __launch_bounds__(256) void k_reduce_slices(const int32_t* __restrict__ idx, int64_t n_idx,
                                                       const int32_t* __restrict__ n_dev, int64_t N, int32_t L,
                                                       int32_t S, double* __restrict__ acc) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (n_dev ? (int64_t)*n_dev : n_idx)) return;
    const int64_t i = idx ? (int64_t)idx[j] : j;
    const int64_t o = ((int64_t)blockIdx.y * kAcc + blockIdx.z) * N + i;   // (trial, row, point)
    const int64_t slice = (int64_t)L * kAcc * N;
    double a = acc[o];
    for (int z = 1; z < S; ++z) a += acc[z * slice + o];
    acc[o] = a;
}

hipError_t launch_finalize(const BoundaryDev* bnd, const double* B0d, const double* gpos, const double* gB,
                           Geo geo, const double* lam,
                           const int32_t* idx, int64_t n_idx, const int32_t* n_dev, int64_t N, int32_t L,
                           int32_t S, double* acc,
                           bool add_near, bool tan, double dvds, double* B, double* dB, double* fg,
                           double* tanout, hipStream_t s) {
    if (n_idx == 0) return hipSuccess;
    const dim3 grid((unsigned)((n_idx + 255) / 256), (unsigned)L);
    if (S >= 4 && n_idx * L <= ((int64_t)1 << 18)) {
        hipLaunchKernelGGL(k_reduce_slices, dim3(grid.x, grid.y, (unsigned)(tan ? kAcc : kAccField)), dim3(256), 0,
                           s, idx, n_idx, n_dev, N, L, S, acc);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        S = 1;
    }
#define DBIE_FIN(T, NR)                                                                            \
    hipLaunchKernelGGL((k_finalize<T, NR>), grid, dim3(256), 0, s, bnd, B0d, gpos, gB, geo, lam, idx, n_idx, \
                       n_dev, N, L, S, acc, dvds, B, dB, fg, tanout)
    if (tan) {
        if (add_near) DBIE_FIN(true, true);
        else DBIE_FIN(true, false);
    } else {
        if (add_near) DBIE_FIN(false, true);
        else DBIE_FIN(false, false);
    }
#undef DBIE_FIN
    return hipGetLastError();
}

}  // namespace dbie

// ---- residual statistics (dbie_residual_stats) ----------------------------------------------
// Sums over the points of f, g, the count of finite (f, g) and the count with max(f, g) <= eps:
// per thread over a grid stride, then across the wavefront with shuffles, then across the block in
// LDS; one partial per block, added in block order by a single block (fixed order: deterministic).
namespace dbie {

constexpr int kStatBlocks = 256;

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_fg_partial(int64_t N, const double* __restrict__ fg, double eps,
                                                    double* __restrict__ part) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const double f = fg[i], g = fg[N + i];
        if (isfinite(f) && isfinite(g)) {
            s[0] += f;
            s[1] += g;
            s[2] += 1.0;
            if (fmax(f, g) <= eps) s[3] += 1.0;
        }
    }
    __shared__ double red[4][4];   // [wave][quantity]
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int q = 0; q < 4; ++q) {
        const double v = wave_sum(s[q]);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double v = 0.0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) v += red[w][threadIdx.x];
        part[blockIdx.x * 4 + threadIdx.x] = v;
    }
}

__global__ void k_fg_final(int32_t nblk, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x >= 4) return;
    double v = 0.0;
    for (int32_t b = 0; b < nblk; ++b) v += part[b * 4 + threadIdx.x];
    out[threadIdx.x] = v;
}

hipError_t launch_fg_stats(int64_t N, const double* fg, double eps, double* scratch, hipStream_t s) {
    const int32_t nblk = (int32_t)std::min<int64_t>(kStatBlocks, std::max<int64_t>(1, (N + 255) / 256));
    hipLaunchKernelGGL(k_fg_partial, dim3(nblk), dim3(256), 0, s, N, fg, eps, scratch + 4);
    hipLaunchKernelGGL(k_fg_final, dim3(1), dim3(64), 0, s, nblk, scratch + 4, scratch);
    return hipGetLastError();
}

}  // namespace dbie
