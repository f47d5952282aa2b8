// FP32 bulk kernel sum with compensated accumulation (the FP32C path).
//
// Work decomposition: one workgroup per schedule tile (<= PPL * 64 * WAVES consecutive points of one
// magnetogram) and one grid row per lambda trial. Lane l of the workgroup owns points l, l + NT,
// ..., so a wavefront holds 64 consecutive points (spatially coherent). The magnetogram streams
// through LDS in tiles of TP pixels (five planes: a, b, Bx, By, Bz); every lane reads the same
// address (broadcast), four pixels per ds_read_b128.
//
// Arithmetic per pair, all FP32:
//   dx = (a_k - floor(u)) - frac(u)    (the integer difference is exact: one rounding in total)
//   rho^-1 = rsq(dx^2 + dy^2 + w^2), and per component t = Lambda rho, sin/cos in revolutions
//   (range-reduced by fract only when a workgroup's |Lambda| rho / 2pi can exceed the hardware's
//   accurate range of 256 revolutions), N = t sin t + cos t, H = t (t cos t) - 3 N, and the sums
//   A0 += N rho^-3 B0,  A1 += H rho^-3 B0 * dx rho^-2,  A2 likewise with dy,  A3 += H rho^-3 B0 rho^-2.
// Compensation: each pixel tile is summed in FP32 (error ~ TP u), and the tile partials are added
// into FP64 totals, so the error does not grow with the magnetogram size.
// Near field: pairs whose (FP64-classified) distance is below the near radius are skipped here and
// summed in FP64 by the finalize pass. Tiles that cannot contain such a pair for any point of the
// workgroup take the unmasked loop; the test is uniform over the workgroup.
#include <climits>

#include "dbie_internal.h"

namespace dbie {

template <int PPL, bool TAN>
struct PointState {
    float xn[PPL], xf[PPL], yn[PPL], yf[PPL], w2[PPL];
    float lt[PPL][3];   // Lambda (radians per pixel)
    float lr[PPL][3];   // Lambda / 2pi (revolutions per pixel)
    float fa[PPL], fb[PPL];   // near-window centre as floats
    uint32_t msk[PPL];
};

template <int PPL, bool TAN, bool SLOW, bool FRACT>
__device__ __forceinline__ void pixel_step(const PointState<PPL, TAN>& S, float a, float b, float bx,
                                           float by, float bz, float (&acc)[PPL][TAN ? kAcc : kAccField]) {
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const float dx = (a + S.xn[j]) - S.xf[j];
        const float dy = (b + S.yn[j]) - S.yf[j];
        float b0[3] = {bx, by, bz};
        if (SLOW) {
            const float da = a - S.fa[j], db = b - S.fb[j];
            const bool in = fabsf(da) <= (float)kNearWin && fabsf(db) <= (float)kNearWin;
            const int bit = in ? (int)(da + (float)kNearWin) + kNearSide * (int)(db + (float)kNearWin) : 0;
            const bool nr = in && ((S.msk[j] >> bit) & 1u);
            if (nr) b0[0] = b0[1] = b0[2] = 0.0f;
        }
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, S.w2[j]));
        const float ri = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * ri;
        const float ri2 = ri * ri;
        const float ri3 = ri2 * ri;
        const float dxr = dx * ri2;
        const float dyr = dy * ri2;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            // v_sin / v_cos take revolutions and are accurate on [-256, 256]; FRACT reduces first
            const float tr = FRACT ? __builtin_amdgcn_fractf(S.lr[j][p] * r) : S.lr[j][p] * r;
            const float sn = __builtin_amdgcn_sinf(tr);
            const float cs = __builtin_amdgcn_cosf(tr);
            const float t = S.lt[j][p] * r;
            const float n = fmaf(t, sn, cs);
            const float hh = fmaf(t, t * cs, -3.0f * n);
            const float b3 = ri3 * b0[p];
            const float hb = hh * b3;
            if (TAN) {
                const float nb = n * b3;
                acc[j][4 * p + 0] += nb;
                acc[j][12 + 3 * p + 0] = fmaf(cs, ri * b0[p], acc[j][12 + 3 * p + 0]);
                acc[j][12 + 3 * p + 1] = fmaf(nb, dx, acc[j][12 + 3 * p + 1]);
                acc[j][12 + 3 * p + 2] = fmaf(nb, dy, acc[j][12 + 3 * p + 2]);
            } else {
                acc[j][4 * p + 0] = fmaf(n, b3, acc[j][4 * p + 0]);
            }
            acc[j][4 * p + 1] = fmaf(hb, dxr, acc[j][4 * p + 1]);
            acc[j][4 * p + 2] = fmaf(hb, dyr, acc[j][4 * p + 2]);
            acc[j][4 * p + 3] = fmaf(hb, ri2, acc[j][4 * p + 3]);
        }
    }
}

template <int PPL, int TP, bool TAN, bool SLOW, bool FRACT>
__device__ __forceinline__ void tile_loop(const PointState<PPL, TAN>& S, const float4 (*s4)[TP / 4],
                                          float (&part)[PPL][TAN ? kAcc : kAccField]) {
    for (int q = 0; q < TP / 4; ++q) {
        const float4 A = s4[0][q], Bq = s4[1][q], X = s4[2][q], Y = s4[3][q], Z = s4[4][q];
        pixel_step<PPL, TAN, SLOW, FRACT>(S, A.x, Bq.x, X.x, Y.x, Z.x, part);
        pixel_step<PPL, TAN, SLOW, FRACT>(S, A.y, Bq.y, X.y, Y.y, Z.y, part);
        pixel_step<PPL, TAN, SLOW, FRACT>(S, A.z, Bq.z, X.z, Y.z, Z.z, part);
        pixel_step<PPL, TAN, SLOW, FRACT>(S, A.w, Bq.w, X.w, Y.w, Z.w, part);
    }
}

template <int PPL, int WAVES, int TP, bool TAN>
__global__ __launch_bounds__(64 * WAVES) void k_field32c(const Tile* __restrict__ tiles,
                                                         int64_t n_tiles,
                                                         const BoundaryDev* __restrict__ bnd,
                                                         const float* __restrict__ pixf, Geo geo,
                                                         const double* __restrict__ lam, int64_t N,
                                                         const int32_t* __restrict__ idx, int xcd_remap,
                                                         double* __restrict__ acc) {
    constexpr int NT = 64 * WAVES;
    constexpr int NA = TAN ? kAcc : kAccField;
    constexpr int TQ = TP / 4;
    __shared__ float4 s4[5][TQ];
    __shared__ int box[4];
    __shared__ float rev_max;   // bound of |Lambda| r / 2pi over the workgroup's pairs

    // XCD-aware order (static schedules): workgroups are dealt round-robin to the 8 XCDs; give each
    // XCD a contiguous run of the schedule so that its L2 sees few magnetograms. Schedules are padded
    // to a multiple of 8 tiles (empty tiles have count 0), which makes this remap a permutation.
    // Schedules built on the device over an active-point list keep the identity order.
    const int64_t per = (int64_t)gridDim.x / 8;
    const int64_t bx = blockIdx.x;
    const Tile t = tiles[xcd_remap ? (bx & 7) * per + (bx >> 3) : bx];
    if (t.count == 0) return;
    const int64_t trial = blockIdx.y;
    const BoundaryDev bd = bnd[t.b];
    const int tid = threadIdx.x;

    if (tid == 0) {
        box[0] = INT_MAX;
        box[1] = INT_MIN;
        box[2] = INT_MAX;
        box[3] = INT_MIN;
        rev_max = 0.0f;
    }
    __syncthreads();

    PointState<PPL, TAN> S;
    bool live[PPL];
    int64_t pid[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const int q = tid + j * NT;
        live[j] = q < t.count;
        const int64_t e = t.start + (live[j] ? q : 0);
        const int64_t i = idx ? (int64_t)idx[e] : e;
        pid[j] = i;
        S.xn[j] = -geo.xi_int[i];
        S.xf[j] = geo.xi_frac[i];
        S.yn[j] = -geo.yi_int[i];
        S.yf[j] = geo.yi_frac[i];
        const float wv = geo.wf[i];
        S.w2[j] = wv * wv;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const double L = lam[(trial * 3 + p) * N + i] * bd.h;
            S.lt[j][p] = (float)L;
            S.lr[j][p] = (float)(L * 0.15915494309189533577);
        }
        const int32_t wa = geo.win_a[i], wb = geo.win_b[i];
        S.fa[j] = (float)wa;
        S.fb[j] = (float)wb;
        S.msk[j] = live[j] ? geo.near_mask[i] : 0u;
        {
            // farthest pixel centre of the magnetogram from this point
            const float uf = -S.xn[j] + S.xf[j], vf = -S.yn[j] + S.yf[j];
            const float dxm = fmaxf(fabsf(uf), fabsf((float)(bd.nx - 1) - uf)) + 1.0f;
            const float dym = fmaxf(fabsf(vf), fabsf((float)(bd.ny - 1) - vf)) + 1.0f;
            const float rmax = sqrtf(dxm * dxm + dym * dym + S.w2[j]);
            const float lmax = fmaxf(fabsf(S.lr[j][0]), fmaxf(fabsf(S.lr[j][1]), fabsf(S.lr[j][2])));
            const float rv = live[j] ? lmax * rmax : 0.0f;
            // non-negative floats order like their bit patterns; NaN (bits above +inf) forces FRACT
            atomicMax(reinterpret_cast<int*>(&rev_max), __float_as_int(rv));
        }
        if (S.msk[j]) {
            atomicMin(&box[0], wa - kNearWin);
            atomicMax(&box[1], wa + kNearWin);
            atomicMin(&box[2], wb - kNearWin);
            atomicMax(&box[3], wb + kNearWin);
        }
    }
    __syncthreads();
    const int amin = box[0], amax = box[1], bmin = box[2], bmax = box[3];
    const bool any_near = amin <= amax;
    const bool need_fract = !(rev_max < 255.0f);

    double tot[PPL][NA];
    float part[PPL][NA];
#pragma unroll
    for (int j = 0; j < PPL; ++j)
#pragma unroll
        for (int r = 0; r < NA; ++r) tot[j][r] = 0.0;

    const float* P = pixf + bd.pixf_off;
    const int64_t PP = bd.npix_pad;
    const int npix = bd.npix, nx = bd.nx;
    for (int k0 = 0; k0 < npix; k0 += TP) {
        __syncthreads();
        for (int q = tid; q < 5 * TQ; q += NT) {
            const int pl = q / TQ, o = q - pl * TQ;
            s4[pl][o] = reinterpret_cast<const float4*>(P + pl * PP + k0)[o];
        }
        __syncthreads();
        bool slow = false;
        if (any_near) {
            const int klast = min(k0 + TP, npix) - 1;
            const int r0 = k0 / nx, r1 = klast / nx;
            const int c0 = (r0 == r1) ? k0 - r0 * nx : 0;
            const int c1 = (r0 == r1) ? klast - r1 * nx : nx - 1;
            slow = !(r1 < bmin || r0 > bmax || c1 < amin || c0 > amax);
        }
#pragma unroll
        for (int j = 0; j < PPL; ++j)
#pragma unroll
            for (int r = 0; r < NA; ++r) part[j][r] = 0.0f;
        if (!slow) {
            if (need_fract) tile_loop<PPL, TP, TAN, false, true>(S, s4, part);
            else tile_loop<PPL, TP, TAN, false, false>(S, s4, part);
        } else {
            if (need_fract) tile_loop<PPL, TP, TAN, true, true>(S, s4, part);
            else tile_loop<PPL, TP, TAN, true, false>(S, s4, part);
        }
#pragma unroll
        for (int j = 0; j < PPL; ++j)
#pragma unroll
            for (int r = 0; r < NA; ++r) tot[j][r] += (double)part[j][r];
    }
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        if (!live[j]) continue;
#pragma unroll
        for (int r = 0; r < NA; ++r) acc[(trial * kAcc + r) * N + pid[j]] = tot[j][r];
    }
}

// The instantiated shapes (points per lane, waves per workgroup, pixels per LDS tile).
#define DBIE_F32_SHAPES(X) \
    X(1, 4, 256)           \
    X(2, 4, 256)           \
    X(4, 4, 256)           \
    X(2, 4, 128)           \
    X(2, 8, 256)           \
    X(1, 8, 256)

int field32c_shapes(F32Shape* out, int max) {
    int n = 0;
#define DBIE_LIST(P, W, T) \
    if (n < max) out[n] = F32Shape{P, W, T}; \
    ++n;
    DBIE_F32_SHAPES(DBIE_LIST)
#undef DBIE_LIST
    return n;
}

bool field32c_shape_supported(F32Shape s) {
#define DBIE_CHK(P, W, T) \
    if (s.ppl == P && s.waves == W && s.tp == T) return true;
    DBIE_F32_SHAPES(DBIE_CHK)
#undef DBIE_CHK
    return false;
}

hipError_t launch_field32c(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd,
                           const float* pixf, Geo geo, const double* lam, int64_t N, int32_t L,
                           const int32_t* idx, bool tan, F32Shape s, double* acc, hipStream_t st) {
    const int remap = idx ? 0 : 1;
    if (n_tiles == 0) return hipSuccess;
    const dim3 grid((unsigned)n_tiles, (unsigned)L);
#define DBIE_LAUNCH(P, W, T)                                                                           \
    if (s.ppl == P && s.waves == W && s.tp == T) {                                                     \
        if (tan)                                                                                       \
            hipLaunchKernelGGL((k_field32c<P, W, T, true>), grid, dim3(64 * W), 0, st, tiles, n_tiles, \
                               bnd, pixf, geo, lam, N, idx, remap, acc);                                           \
        else                                                                                           \
            hipLaunchKernelGGL((k_field32c<P, W, T, false>), grid, dim3(64 * W), 0, st, tiles,         \
                               n_tiles, bnd, pixf, geo, lam, N, idx, remap, acc);                                  \
        return hipGetLastError();                                                                      \
    }
    DBIE_F32_SHAPES(DBIE_LAUNCH)
#undef DBIE_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace dbie
