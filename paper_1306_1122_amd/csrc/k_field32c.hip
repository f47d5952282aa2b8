// FP32 bulk kernel sum with compensated accumulation (the FP32C path).
//
// Work decomposition: one schedule tile (<= PPL * 64 * WAVES points of one magnetogram) at a time
// per workgroup, one grid row (y) per lambda trial and one grid layer (z) per pixel slice (when the
// point tiles alone cannot fill the chip, slice z sums its share of the pixel blocks into its own
// partial, and the finalize pass adds the slices in order); static schedules are ordered by
// decreasing cost. Lane l of the workgroup owns points l, l + NT, ...
// of the tile, so a wavefront holds 64 consecutive points (the library orders points so that these
// are spatially coherent). The magnetogram streams through LDS in blocks of RB rows (three planes Bx,
// By, Bz; RB = 16, 32 or 64, a tuning parameter) by 16 columns, or 8 on an element grid; HBM holds
// kRows x kCols blocks, tile-major, so a nodal block stages the rows it needs from two adjacent column
// strips; every lane reads the same LDS address (broadcast).
//
// Arithmetic per pair, all FP32. For each block and point the column offsets
//   dx_c = (a0 + c - floor(u)) - frac(u)           (exact integer difference, one rounding)
// are kept in registers; for each row dy = (b0 + r - floor(v)) - frac(v) and q = dy^2 + w^2; then
//   rho^2 = dx_c^2 + q, rho^-1 = rsq(rho^2), and per component t = Lambda rho, sin/cos in
//   revolutions (minus the nearest integer, only when a wavefront's |Lambda| rho / 2pi can exceed the
//   hardware's accurate range of 256 revolutions). t is never formed: since t / rho = Lambda,
//   N rho^-3 = (t sin t + cos t) rho^-3 = rho^-2 (Lambda sin t + cos t rho^-1), and in place of
//   H = t^2 cos t - 3 N the form Q = -H / 3 = N - (Lambda^2 / 3) rho^2 cos t gives
//   Q rho^-3 = N rho^-3 + (-Lambda^2 / 3) cos t rho^-1;
//   A0 += N rho^-3 B0,  A1 += Q rho^-3 B0 * dx rho^-2,  A2 likewise with dy,  A3 += Q rho^-3 B0 rho^-2
//   (the totals of A1..A3 are multiplied by -3 when written), and with tangents
//   T0 += cos t rho^-1 B0, T1 += N rho^-3 B0 dx, T2 += N rho^-3 B0 dy; there the T0 term
//   cos t rho^-1 B0 is shared by N rho^-3 B0 = rho^-2 (Lambda sin t B0 + cos t rho^-1 B0) and by
//   Q rho^-3 B0.
// Rows: dy is the same for the pairs of a block row, so the row's A3 terms (and, with tangents,
// its A0 terms) are summed apart, and A2 += dy (row sum of A3 terms), T2 += dy (row sum of A0 terms)
// once per row: no per-pair products with dy.
// SCALAR: the three components share one lambda, so t, sin, cos, N and Q are computed once per pair.
// Compensation: at most kRows rows of a block (512 pairs per point, 256 on an element grid) are summed
// in FP32, and these partials are added into FP64 totals, so the error does not grow with the
// magnetogram size.
// Near field: pairs whose (FP64-classified) distance is below the near radius are skipped here and
// summed in FP64 by the finalize pass. Blocks that cannot contain such a pair for any point of the
// wavefront take the unmasked loop; the test is uniform over the wavefront.
#include <algorithm>
#include <atomic>
#include <climits>

#include "dbie_internal.h"

namespace dbie {

// Columns of an LDS pixel block: nodal blocks take two adjacent HBM column strips, so that the per-row
// work (dy, q, the row fold) is shared by 16 pairs; element grids keep one strip (their column
// positions are staged per block, eight of them).
template <bool GRID>
constexpr int block_cols() { return GRID ? kCols : 2 * kCols; }
static_assert(block_cols<false>() % 4 == 0 && block_cols<true>() % 4 == 0, "rows are read as float4");

// Where the 21 FP64 totals of the nodal tangent form with one point per lane live: in LDS (one
// column per lane, 168 bytes), so that its 16-column rows fit three waves per SIMD without spilling
// registers to scratch memory.
template <int PPL, bool TAN, bool GRID>
constexpr bool lds_totals() { return TAN && !GRID && PPL == 1; }

template <int PPL, bool TAN>
struct PointState {
    float xn[PPL], xf[PPL], yn[PPL], yf[PPL], w2[PPL];
    float l3[PPL][3];   // -Lambda^2 / 3 (per pixel^2)
    float lr[PPL][3];   // Lambda / 2pi (revolutions per pixel)
    float lm[PPL][3];   // Lambda (radians per pixel)
    float fa[PPL], fb[PPL];   // near-window centre as floats
    uint32_t msk[PPL];
};

// Phase in revolutions (hi = lr r as rounded), reduced to about [-1/2, 1/2] when FRACT: with
// k = rint(hi), one FMA forms lr r - k from the exact product with a single rounding (the product's
// own rounding, half an ulp of |lr r|, up to 1.5e-5 revolutions at the 256-revolution bound, is not
// incurred), leaving r's rounding as the phase error.
template <bool FRACT>
__device__ __forceinline__ float phase_rev(float lr, float r, float hi) {
    if (!FRACT) return hi;
    return fmaf(lr, r, -__builtin_rintf(hi));
}

// Sum of the row's terms: the first pair of a row sets it, the others add to it.
template <bool FIRST>
__device__ __forceinline__ void row_add(float& s, float x) {
    if (FIRST) s = x;
    else s += x;
}

// One pair given dx (pixels), q = dy^2 + w^2 and the field of the pixel. rs: the row sums of the A3
// terms [3] and, with tangents, of the A0 terms [3] (FIRST: the row's first pair).
template <bool TAN, bool FRACT, bool FIRST>
__device__ __forceinline__ void pair32(float dx, float q, const float nl3[3], const float lr[3],
                                       const float lm[3], float bx, float by, float bz, float* acc, float* rs) {
    const float r2 = fmaf(dx, dx, q);
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float ri2 = ri * ri;
    const float dxr = dx * ri2;
    const float b0[3] = {bx, by, bz};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        // v_sin / v_cos take revolutions and are accurate on [-256, 256]; FRACT reduces first
        const float hi = lr[p] * r;
        const float tr = phase_rev<FRACT>(lr[p], r, hi);
        const float sn = __builtin_amdgcn_sinf(tr);
        const float cs = __builtin_amdgcn_cosf(tr);
        float hb;
        if (TAN) {
            // N B0 / r^3 = (Lambda sin t B0 + cos t B0 / r) / r^2 and -H/3 B0 / r^3 = N B0 / r^3 +
            // (-Lambda^2 / 3) cos t B0 / r: both share the T0 term cos t B0 / r
            const float crb = cs * (ri * b0[p]);
            const float nb = fmaf(lm[p] * sn, b0[p], crb) * ri2;
            hb = fmaf(nl3[p], crb, nb);
            row_add<FIRST>(rs[3 + p], nb);
            acc[12 + 3 * p + 0] += crb;
            acc[12 + 3 * p + 1] = fmaf(nb, dx, acc[12 + 3 * p + 1]);
        } else {
            // N / r^3 = (Lambda sin t + cos t / r) / r^2, -H/3 / r^3 = N / r^3 + (-Lambda^2 / 3) cos t / r
            const float cri = cs * ri;
            const float nr3 = fmaf(lm[p], sn, cri) * ri2;
            hb = fmaf(nl3[p], cri, nr3) * b0[p];
            acc[4 * p + 0] = fmaf(nr3, b0[p], acc[4 * p + 0]);
        }
        acc[4 * p + 1] = fmaf(hb, dxr, acc[4 * p + 1]);
        if (FIRST) rs[p] = hb * ri2;
        else rs[p] = fmaf(hb, ri2, rs[p]);
    }
}

// One pair when the three components share one lambda: the sin/cos, N and H are computed once.
template <bool TAN, bool FRACT, bool FIRST>
__device__ __forceinline__ void pair32_scalar(float dx, float q, float nl3, float lr, float lm, float bx,
                                              float by, float bz, float* acc, float* rs) {
    const float r2 = fmaf(dx, dx, q);
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * ri;
    const float ri2 = ri * ri;
    const float dxr = dx * ri2;
    const float hi = lr * r;
    const float tr = phase_rev<FRACT>(lr, r, hi);
    const float sn = __builtin_amdgcn_sinf(tr);
    const float cs = __builtin_amdgcn_cosf(tr);
    const float cri = cs * ri;
    const float nr3 = fmaf(lm, sn, cri) * ri2;   // N / r^3
    const float hr3 = fmaf(nl3, cri, nr3);       // -H / 3 / r^3
    const float b0[3] = {bx, by, bz};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const float hb = hr3 * b0[p];
        if (TAN) {
            const float nb = nr3 * b0[p];
            row_add<FIRST>(rs[3 + p], nb);
            acc[12 + 3 * p + 0] = fmaf(cri, b0[p], acc[12 + 3 * p + 0]);
            acc[12 + 3 * p + 1] = fmaf(nb, dx, acc[12 + 3 * p + 1]);
        } else {
            acc[4 * p + 0] = fmaf(nr3, b0[p], acc[4 * p + 0]);
        }
        acc[4 * p + 1] = fmaf(hb, dxr, acc[4 * p + 1]);
        if (FIRST) rs[p] = hb * ri2;
        else rs[p] = fmaf(hb, ri2, rs[p]);
    }
}

// Rows r0 .. r1 - 1 of a block of RB x block_cols pixels with origin (a0, b0), for all PPL points.
// GRID (9-node elements): the block's columns and rows sit at the positions sC, sR ({integer part,
// fraction, element index}) instead of at a0 + c, b0 + r, and the near mask is per element.
template <int PPL, int RB, bool TAN, bool SLOW, bool FRACT, bool SCALAR, bool GRID>
__device__ __forceinline__ void block_loop(const PointState<PPL, TAN>& S,
                                           const float4 (*sB)[RB][block_cols<GRID>() / 4], const float4* sC,
                                           const float4* sR, float a0, float b0, int r0, int r1,
                                           float (&part)[PPL][TAN ? kAcc : kAccField]) {
    constexpr int KC = block_cols<GRID>();
    float dxc[PPL][KC];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const float base = a0 + S.xn[j];   // exact: integers
#pragma unroll
        for (int c = 0; c < KC; ++c) {
            if (GRID) dxc[j][c] = (sC[c].x + S.xn[j]) + (sC[c].y - S.xf[j]);
            else dxc[j][c] = (base + (float)c) - S.xf[j];
        }
    }
    for (int r = r0; r < r1; ++r) {
        // the row's three planes (broadcast reads of KC / 4 float4 each)
        const float* bxs = reinterpret_cast<const float*>(&sB[0][r][0]);
        const float* bys = reinterpret_cast<const float*>(&sB[1][r][0]);
        const float* bzs = reinterpret_cast<const float*>(&sB[2][r][0]);
        const float brow = b0 + (float)r;
        // GRID: the row's split position (the element index is read only by the masked loop)
        float2 rp = make_float2(0.0f, 0.0f);
        if (GRID) rp = *reinterpret_cast<const float2*>(&sR[r]);
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            const float dy = GRID ? (rp.x + S.yn[j]) + (rp.y - S.yf[j]) : (brow + S.yn[j]) - S.yf[j];
            const float q = fmaf(dy, dy, S.w2[j]);
            float rs[TAN ? 6 : 3];   // the row sums of the A3 terms and, with tangents, of the A0 terms
#pragma unroll
            for (int c = 0; c < KC; ++c) {
                float bx = bxs[c], by = bys[c], bz = bzs[c];
                if (SLOW && GRID) {
                    const float da = sC[c].z - S.fa[j], db = sR[r].z - S.fb[j];
                    const bool in = fabsf(da) <= (float)kNearWinQ && fabsf(db) <= (float)kNearWinQ;
                    const int bit =
                        in ? (int)(da + (float)kNearWinQ) + kNearSideQ * (int)(db + (float)kNearWinQ) : 0;
                    if (in && ((S.msk[j] >> bit) & 1u)) bx = by = bz = 0.0f;
                } else if (SLOW) {
                    const float da = (a0 + (float)c) - S.fa[j], db = brow - S.fb[j];
                    const bool in = fabsf(da) <= (float)kNearWin && fabsf(db) <= (float)kNearWin;
                    const int bit =
                        in ? (int)(da + (float)kNearWin) + kNearSide * (int)(db + (float)kNearWin) : 0;
                    if (in && ((S.msk[j] >> bit) & 1u)) bx = by = bz = 0.0f;
                }
                if (SCALAR) {
                    if (c == 0)
                        pair32_scalar<TAN, FRACT, true>(dxc[j][c], q, S.l3[j][0], S.lr[j][0], S.lm[j][0], bx, by,
                                                        bz, part[j], rs);
                    else
                        pair32_scalar<TAN, FRACT, false>(dxc[j][c], q, S.l3[j][0], S.lr[j][0], S.lm[j][0], bx, by,
                                                         bz, part[j], rs);
                } else {
                    if (c == 0)
                        pair32<TAN, FRACT, true>(dxc[j][c], q, S.l3[j], S.lr[j], S.lm[j], bx, by, bz, part[j], rs);
                    else
                        pair32<TAN, FRACT, false>(dxc[j][c], q, S.l3[j], S.lr[j], S.lm[j], bx, by, bz, part[j], rs);
                }
            }
            // the row's y-moments: A2 += dy (sum of A3 terms), T2 += dy (sum of A0 terms)
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                part[j][4 * p + 3] += rs[p];
                part[j][4 * p + 2] = fmaf(dy, rs[p], part[j][4 * p + 2]);
                if (TAN) {
                    part[j][4 * p + 0] += rs[3 + p];
                    part[j][12 + 3 * p + 2] = fmaf(dy, rs[3 + p], part[j][12 + 3 * p + 2]);
                }
            }
        }
    }
}

// One schedule tile: the sums of its points over every pixel block of their magnetogram.
template <int PPL, int WAVES, int RB, bool TAN, bool SCALAR, bool GRID>
__device__ __forceinline__ void field32c_tile(const Tile t, const BoundaryDev* __restrict__ bnd,
                                              const float* __restrict__ pixf, const float4* __restrict__ gposf,
                                              const Geo& geo, const double* __restrict__ lam, int64_t N,
                                              const int32_t* __restrict__ idx, double* __restrict__ acc,
                                              float4 (*sB)[RB][block_cols<GRID>() / 4], float4* sC, float4* sR,
                                              double* __restrict__ sT) {
    constexpr int NT = 64 * WAVES;
    constexpr int KC = block_cols<GRID>();
    constexpr int KQ = KC / 4;              // float4 per row of a plane of an LDS block
    constexpr int NA = TAN ? kAcc : kAccField;
    constexpr int BQ = kRows * kCols / 4;   // float4 per plane of an HBM block
    constexpr int RQ = kCols / 4;           // float4 per row of a plane
    static_assert(NT >= kCols + RB, "the row positions of a GRID block are staged one per thread");
    if (t.count == 0) return;
    const int64_t trial = blockIdx.y;
    const BoundaryDev bd = bnd[t.b];
    const int tid = threadIdx.x;

    // per-wavefront bounds: the box of the near-field windows of its points and the largest
    // |Lambda| r / 2pi of its pairs
    int amin = INT_MAX, amax = INT_MIN, bmin = INT_MAX, bmax = INT_MIN;
    float rv_w = 0.0f;
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
            S.l3[j][p] = (float)(L * L * (-1.0 / 3.0));
            S.lr[j][p] = (float)(L * 0.15915494309189533577);
            S.lm[j][p] = (float)L;
        }
        const int32_t wa = geo.win_a[i], wb = geo.win_b[i];
        S.fa[j] = (float)wa;
        S.fb[j] = (float)wb;
        S.msk[j] = live[j] ? geo.near_mask[i] : 0u;
        {
            // farthest pixel centre of the (column-padded) magnetogram from this point
            const float uf = -S.xn[j] + S.xf[j], vf = -S.yn[j] + S.yf[j];
            // (grid positions, padding included, lie in [0, nx - 1] x [0, ny - 1])
            const float xe = GRID ? (float)(bd.nx - 1) : (float)((bd.ntx + 1) / 2 * KC - 1);
            const float dxm = fmaxf(fabsf(uf), fabsf(xe - uf)) + 1.0f;
            const float dym = fmaxf(fabsf(vf), fabsf((float)(bd.ny - 1) - vf)) + 1.0f;
            const float rmax = sqrtf(dxm * dxm + dym * dym + S.w2[j]);
            const float lmax = fmaxf(fabsf(S.lr[j][0]), fmaxf(fabsf(S.lr[j][1]), fabsf(S.lr[j][2])));
            const float rv = live[j] ? lmax * rmax : 0.0f;
            rv_w = (rv == rv) ? fmaxf(rv_w, rv) : __builtin_inff();   // NaN lambda forces FRACT
        }
        if (S.msk[j]) {
            // the window box, in pixels (nodal) or in elements (GRID)
            const int hw = GRID ? kNearWinQ : kNearWin;
            amin = min(amin, wa - hw);
            amax = max(amax, wa + hw);
            bmin = min(bmin, wb - hw);
            bmax = max(bmax, wb + hw);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        amin = min(amin, __shfl_xor(amin, off, 64));
        amax = max(amax, __shfl_xor(amax, off, 64));
        bmin = min(bmin, __shfl_xor(bmin, off, 64));
        bmax = max(bmax, __shfl_xor(bmax, off, 64));
        rv_w = fmaxf(rv_w, __shfl_xor(rv_w, off, 64));
    }
    const bool any_near = amin <= amax;
    const bool need_fract = !(rv_w < 255.0f);

    // the FP64 totals: in registers, or (LT) in the lane's own LDS column sT[r * NT + tid]
    constexpr bool LT = lds_totals<PPL, TAN, GRID>();
    double tot[LT ? 1 : PPL][LT ? 1 : NA];
    float part[PPL][NA];
#pragma unroll
    for (int j = 0; j < PPL; ++j)
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            if (LT) sT[r * NT + tid] = 0.0;
            else tot[LT ? 0 : j][LT ? 0 : r] = 0.0;
        }

    const float4* P = reinterpret_cast<const float4*>(pixf + bd.pixf_off);
    // LDS blocks of RB rows (every block holds at least one row) over strips of KC columns (the last
    // nodal strip may hold one HBM strip and zeros); pixel split: slice blockIdx.z of gridDim.z takes
    // an even share of them
    const int nrows = GRID ? bd.grows : bd.ny;
    const int nrb = (nrows + RB - 1) / RB;
    const int nstrip = GRID ? bd.ntx : (bd.ntx + 1) / 2;
    const int nblk_all = nstrip * nrb;
    const int kb0 = (int)((int64_t)blockIdx.z * nblk_all / gridDim.z);
    const int nblk = (int)((int64_t)(blockIdx.z + 1) * nblk_all / gridDim.z);
    for (int k = kb0; k < nblk; ++k) {
        const int ty = k / nstrip, tx = k - ty * nstrip;
        const int a0 = tx * KC, b0 = ty * RB;
        const int rows = min(RB, nrows - b0);
        __syncthreads();
        if (!GRID) {
            // the block's rows from the HBM blocks of column strips 2 tx and 2 tx + 1 that hold them
            // (rows b0 .. b0 + rows - 1 < nrows <= nty * kRows lie inside the padded magnetogram; a
            // strip beyond the last, ntx odd, reads as zeros)
            for (int q = tid; q < 3 * RB * KQ; q += NT) {
                const int pl = q / (RB * KQ), o = q - pl * (RB * KQ);
                const int r = o / KQ, h = o - r * KQ;
                const int st = 2 * tx + h / RQ, hh = h - (h / RQ) * RQ;
                if (r < rows) {
                    const int b = b0 + r, hb = b / kRows;
                    sB[pl][r][h] = st < bd.ntx
                                       ? P[((int64_t)(hb * bd.ntx + st) * 3 + pl) * BQ + (b - hb * kRows) * RQ + hh]
                                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                }
            }
        } else if (RB == kRows) {
            // one HBM block, contiguous
            for (int q = tid; q < 3 * BQ; q += NT) {
                const int pl = q / BQ, o = q - pl * BQ;
                sB[pl][o / RQ][o % RQ] = P[(int64_t)k * 3 * BQ + q];
            }
        } else {
            // the block's rows from the HBM blocks of column strip tx that hold them (rows b0 .. b0 +
            // rows - 1 < nrows <= nty * kRows: every read lies inside the padded magnetogram)
            for (int q = tid; q < 3 * RB * RQ; q += NT) {
                const int pl = q / (RB * RQ), o = q - pl * (RB * RQ);
                const int r = o / RQ, h = o - r * RQ;
                if (r < rows) {
                    const int b = b0 + r, hb = b / kRows;
                    sB[pl][r][h] = P[((int64_t)(hb * bd.ntx + tx) * 3 + pl) * BQ + (b - hb * kRows) * RQ + h];
                }
            }
        }
        if (GRID) {
            const float4* gp = gposf + bd.gposf_off;
            if (tid < kCols) sC[tid] = gp[a0 + tid];
            else if (tid < kCols + rows) sR[tid - kCols] = gp[(int64_t)bd.ntx * kCols + b0 + tid - kCols];
        }
        __syncthreads();
        bool slow = false;
        if (any_near) {
            if (GRID) {
                // the block's element range (padding columns and rows repeat the last element)
                const int ea0 = a0 / bd.G, ea1 = min(a0 + kCols - 1, bd.gcols - 1) / bd.G;
                const int eb0 = b0 / bd.G, eb1 = (b0 + rows - 1) / bd.G;
                slow = !(eb1 < bmin || eb0 > bmax || ea1 < amin || ea0 > amax);
            } else {
                slow = !(b0 + rows - 1 < bmin || b0 > bmax || a0 + KC - 1 < amin || a0 > amax);
            }
        }
        const float fa0 = (float)a0, fb0 = (float)b0;
        // FP32 partials over at most kRows rows of the block (kRows x block_cols pairs per point), each
        // then added into the FP64 totals
        for (int h0 = 0; h0 < rows; h0 += kRows) {
            const int h1 = min(rows, h0 + kRows);
#pragma unroll
            for (int j = 0; j < PPL; ++j)
#pragma unroll
                for (int r = 0; r < NA; ++r) part[j][r] = 0.0f;
            if (!slow) {
                if (need_fract) block_loop<PPL, RB, TAN, false, true, SCALAR, GRID>(S, sB, sC, sR, fa0, fb0, h0, h1, part);
                else block_loop<PPL, RB, TAN, false, false, SCALAR, GRID>(S, sB, sC, sR, fa0, fb0, h0, h1, part);
            } else {
                if (need_fract) block_loop<PPL, RB, TAN, true, true, SCALAR, GRID>(S, sB, sC, sR, fa0, fb0, h0, h1, part);
                else block_loop<PPL, RB, TAN, true, false, SCALAR, GRID>(S, sB, sC, sR, fa0, fb0, h0, h1, part);
            }
#pragma unroll
            for (int j = 0; j < PPL; ++j)
#pragma unroll
                for (int r = 0; r < NA; ++r) {
                    if (LT) sT[r * NT + tid] += (double)part[j][r];
                    else tot[LT ? 0 : j][LT ? 0 : r] += (double)part[j][r];
                }
        }
    }
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        if (!live[j]) continue;
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            // rows A1..A3 were summed as -1/3 of their terms
            const double sc = (r < kAccField && (r & 3) != 0) ? -3.0 : 1.0;
            const double v = LT ? sT[r * NT + tid] : tot[LT ? 0 : j][LT ? 0 : r];
            acc[(((int64_t)blockIdx.z * gridDim.y + trial) * kAcc + r) * N + pid[j]] = sc * v;
        }
    }
}

// Either one workgroup per tile (work == NULL), or persistent: a grid sized to the resident
// workgroups pulls tile indices from the device counter `work` (cleared by a kernel before the
// launch) until the schedule is exhausted; every workgroup reaches the exit test after each tile.
// Occupancy bounds: three waves per SIMD (at most 168 VGPRs) for the nodal one-point-per-lane forms,
// whose 16-column rows would otherwise take two (the tangent form fits by keeping its FP64 totals in
// LDS; with 64-row blocks its LDS allows two workgroups per compute unit, and it runs at two waves
// per SIMD without spills); four for the plain element form.
template <int PPL, int WAVES, int RB, bool TAN, bool SCALAR, bool GRID>
__global__ __launch_bounds__(64 * WAVES, (GRID && !TAN && !SCALAR && PPL == 1) ? 4
                                        : (!GRID && PPL == 1) ? 3 : 1) void k_field32c(const Tile* __restrict__ tiles,
                                                         int64_t n_tiles,
                                                         const BoundaryDev* __restrict__ bnd,
                                                         const float* __restrict__ pixf,
                                                         const float4* __restrict__ gposf, Geo geo,
                                                         const double* __restrict__ lam, int64_t N,
                                                         const int32_t* __restrict__ idx,
                                                         int32_t* __restrict__ work,
                                                         double* __restrict__ acc) {
    __shared__ float4 sB[3][RB][block_cols<GRID>() / 4];
    __shared__ float4 sC[GRID ? kCols : 1], sR[GRID ? RB : 1];
    __shared__ double sT[lds_totals<PPL, TAN, GRID>() ? kAcc * 64 * WAVES : 1];
    if (!work) {
        field32c_tile<PPL, WAVES, RB, TAN, SCALAR, GRID>(tiles[blockIdx.x], bnd, pixf, gposf, geo, lam, N, idx, acc,
                                                         sB, sC, sR, sT);
        return;
    }
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(work, 1);
        __syncthreads();
        const int64_t ti = next;
        __syncthreads();
        if (ti >= n_tiles) break;
        field32c_tile<PPL, WAVES, RB, TAN, SCALAR, GRID>(tiles[ti], bnd, pixf, gposf, geo, lam, N, idx, acc, sB,
                                                         sC, sR, sT);
    }
}

// The instantiated shapes (points per lane, waves per workgroup, rows of the LDS pixel block); the
// shape's pixel count is rows x kCols whatever the block's width.
#define DBIE_F32_SHAPES(X) \
    X(1, 2, 32)            \
    X(1, 4, 32)            \
    X(1, 8, 32)            \
    X(2, 4, 32)            \
    X(1, 4, 16)            \
    X(1, 4, 64)

int field32c_shapes(F32Shape* out, int max) {
    int n = 0;
    for (int persist = 0; persist < 2; ++persist) {
#define DBIE_LIST(P, W, R)                                        \
        if (n < max) out[n] = F32Shape{P, W, R * kCols, persist}; \
        ++n;
        DBIE_F32_SHAPES(DBIE_LIST)
#undef DBIE_LIST
    }
    return n;
}

bool field32c_shape_supported(F32Shape s) {
    if (s.persist != 0 && s.persist != 1) return false;
#define DBIE_CHK(P, W, R) \
    if (s.ppl == P && s.waves == W && s.tp == R * kCols) return true;
    DBIE_F32_SHAPES(DBIE_CHK)
#undef DBIE_CHK
    return false;
}

__global__ void k_clear_work(int32_t* __restrict__ w) { *w = 0; }

constexpr int kMaxDevices = 64;

template <int P, int W, int R, bool T, bool SC, bool GR>
static hipError_t launch_one(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd, const float* pixf,
                             const float4* gposf, Geo geo, const double* lam, int64_t N, int32_t L, int32_t S,
                             const int32_t* idx, int32_t* work, double* acc, hipStream_t st) {
    unsigned gx = (unsigned)n_tiles;
    if (work) {
        // resident workgroups of this kernel on the current device (queried once per device; a
        // concurrent first query stores the same value)
        static std::atomic<int> resident[kMaxDevices];
        int dev = 0;
        (void)hipGetDevice(&dev);
        int r = (dev >= 0 && dev < kMaxDevices) ? resident[dev].load(std::memory_order_relaxed) : 0;
        if (r == 0) {
            int cus = 0, nb = 0;
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_field32c<P, W, R, T, SC, GR>, 64 * W, 0);
            r = std::max(nb, 1) * std::max(cus, 1);
            if (dev >= 0 && dev < kMaxDevices) resident[dev].store(r, std::memory_order_relaxed);
        }
        gx = (unsigned)std::min<int64_t>(n_tiles, (int64_t)r);
        hipLaunchKernelGGL(k_clear_work, dim3(1), dim3(1), 0, st, work);
    }
    hipLaunchKernelGGL((k_field32c<P, W, R, T, SC, GR>), dim3(gx, (unsigned)L, (unsigned)S), dim3(64 * W), 0, st,
                       tiles, n_tiles, bnd, pixf, gposf, geo, lam, N, idx, work, acc);
    return hipGetLastError();
}

template <int P, int W, int R, bool GR>
static hipError_t launch_variant(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd, const float* pixf,
                                 const float4* gposf, Geo geo, const double* lam, int64_t N, int32_t L, int32_t S,
                                 const int32_t* idx, int32_t* w, bool tan, bool scalar, double* acc, hipStream_t st) {
    if (tan) {
        if (scalar) return launch_one<P, W, R, true, true, GR>(tiles, n_tiles, bnd, pixf, gposf, geo, lam, N, L, S, idx, w, acc, st);
        return launch_one<P, W, R, true, false, GR>(tiles, n_tiles, bnd, pixf, gposf, geo, lam, N, L, S, idx, w, acc, st);
    }
    if (scalar) return launch_one<P, W, R, false, true, GR>(tiles, n_tiles, bnd, pixf, gposf, geo, lam, N, L, S, idx, w, acc, st);
    return launch_one<P, W, R, false, false, GR>(tiles, n_tiles, bnd, pixf, gposf, geo, lam, N, L, S, idx, w, acc, st);
}

hipError_t launch_field32c(const Tile* tiles, int64_t n_tiles, const BoundaryDev* bnd,
                           const float* pixf, const float4* gposf, Geo geo, const double* lam, int64_t N,
                           int32_t L, int32_t S, const int32_t* idx, int32_t* work, bool tan, bool scalar,
                           F32Shape s, double* acc, hipStream_t st) {
    if (n_tiles == 0) return hipSuccess;
    if (S < 1) return hipErrorInvalidValue;
    // a persistent launch with L trials or S slices would share one counter between the grid rows
    int32_t* w = (s.persist && L == 1 && S == 1) ? work : nullptr;
#define DBIE_LAUNCH(P, W, R)                                                                               \
    if (s.ppl == P && s.waves == W && s.tp == R * kCols) {                                                 \
        if (gposf) return launch_variant<P, W, R, true>(tiles, n_tiles, bnd, pixf, gposf, geo, lam, N, L, S, idx, w, tan, scalar, acc, st); \
        return launch_variant<P, W, R, false>(tiles, n_tiles, bnd, pixf, gposf, geo, lam, N, L, S, idx, w, tan, scalar, acc, st);         \
    }
    DBIE_F32_SHAPES(DBIE_LAUNCH)
#undef DBIE_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace dbie
