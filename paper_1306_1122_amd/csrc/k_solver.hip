// Device-resident per-point lambda search (Section 2.1, Eqs. 8-12) behind dbie_solve_lambda.
//
// A solve runs in rounds. In every round each active point evaluates one lambda triple (one trial):
//   bulk sum over the active-point list -> finalize (B, grad B [, tangents]) -> update kernel
//   (residuals, convergence test max(f, g) <= eps, and the next proposal) -> stable compaction of the
//   active list and a device-built tile schedule for the next round.
// Nothing crosses to the host inside a round; the host reads one pinned active count every few
// rounds to stop early. The number of rounds never exceeds the trial budget, because every round
// consumes at least one trial of every active point.
//
// Two update rules:
//  * downhill simplex (Nelder-Mead) on Phi = f^2 + g^2 over (lambda_x, lambda_y, lambda_z), the
//    derivative-free form the paper uses (Lagarias et al. formulation: reflection 1, expansion 2,
//    contraction 1/2, shrink 1/2; vertices in fixed slots ordered by (Phi, slot)). Its vertex
//    arithmetic is written in the same operation order as the CPU oracle with FP contraction off.
//  * Levenberg-Marquardt in mu = lambda^2 >= 0 (the gradient form): the 4x3 Jacobian of the residual
//    vector u = (J x B / (|J||B|), sign(div B) g) from the mu-tangents, Marquardt scaling, nu /= 10 on
//    acceptance (Phi falls) and nu *= 10 on rejection, projection into [0, cap^2].
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dbie_solver.h"

namespace dbie {

constexpr int kCompactThreads = 256;
constexpr int kCompactItems = 4;
constexpr int kCompactBlock = kCompactThreads * kCompactItems;
constexpr int32_t kNoEval = -1;

// ------------------------------------------------------------------------------------------------
// stable compaction of the active flags into a sorted index list + device tile schedules
// ------------------------------------------------------------------------------------------------
// The active flags are read in the order `perm` (NULL = identity): list entries keep that order, so
// the device schedules inherit the grouping of the points with near-field pairs.
__device__ __forceinline__ int64_t at_pos(const int32_t* perm, int64_t k) { return perm ? (int64_t)perm[k] : k; }

__global__ void k_compact_count(const int32_t* __restrict__ active, const int32_t* __restrict__ perm, int64_t N,
                                int32_t* __restrict__ bsum) {
    __shared__ int32_t wsum[kCompactThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kCompactBlock;
    int32_t c = 0;
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k) {
        const int64_t i = base + (int64_t)k * kCompactThreads + threadIdx.x;
        c += (i < N && active[at_pos(perm, i)]) ? 1 : 0;
    }
    // wave reduction (DPP / swizzle under the hood)
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kCompactThreads / 64; ++w) t += wsum[w];
        bsum[blockIdx.x] = t;
    }
}

// Exclusive scan of the block counts in one workgroup.
__global__ void k_compact_scan(int32_t* __restrict__ bsum, int32_t nblk, int32_t* __restrict__ total) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (nblk + 1023) / 1024;
    const int s0 = tid * per, s1 = min(nblk, s0 + per);
    int32_t loc = 0;
    for (int k = s0; k < s1; ++k) loc += bsum[k];
    part[tid] = loc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - loc;
    for (int k = s0; k < s1; ++k) {
        const int32_t v = bsum[k];
        bsum[k] = run;
        run += v;
    }
    if (tid == 1023) *total = part[1023];
}

__global__ void k_compact_scatter(const int32_t* __restrict__ active, const int32_t* __restrict__ perm,
                                  int64_t N, const int32_t* __restrict__ boff, int32_t* __restrict__ list) {
    __shared__ int32_t wcnt[kCompactItems][kCompactThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kCompactBlock;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    bool fl[kCompactItems];
    int32_t rk[kCompactItems];
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k) {
        const int64_t i = base + (int64_t)k * kCompactThreads + threadIdx.x;
        fl[k] = i < N && active[at_pos(perm, i)];
        const uint64_t m = __ballot(fl[k]);
        rk[k] = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        if (lane == 0) wcnt[k][wv] = __popcll(m);
    }
    __syncthreads();
    int32_t run = boff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kCompactItems; ++k) {
        int32_t before = run;
        for (int w = 0; w < wv; ++w) before += wcnt[k][w];
        if (fl[k]) {
            const int64_t i = base + (int64_t)k * kCompactThreads + threadIdx.x;
            list[before + rk[k]] = (int32_t)at_pos(perm, i);
        }
        for (int w = 0; w < kCompactThreads / 64; ++w) run += wcnt[k][w];
    }
}

// Active points of each boundary from the ranks at its segment ends (rank(s) = active points with
// index < s = block prefix + the active flags of the block before s), then the tile offsets of both
// schedules. One workgroup; thread b handles segment start b.
__global__ void k_seg_counts(const int32_t* __restrict__ active, const int32_t* __restrict__ perm, int64_t N,
                             const int32_t* __restrict__ boff,
                             const int32_t* __restrict__ total, const int64_t* __restrict__ seg, int32_t nb,
                             int32_t* __restrict__ cnt_b, int32_t* __restrict__ rank, int32_t per32,
                             int32_t per64, int32_t* __restrict__ off32, int32_t* __restrict__ off64) {
    for (int b = threadIdx.x; b <= nb; b += blockDim.x) {
        const int64_t sp = seg[b];
        int32_t r;
        if (sp >= N) {
            r = *total;
        } else {
            const int64_t blk = sp / kCompactBlock;
            r = boff[blk];
            for (int64_t i = blk * kCompactBlock; i < sp; ++i) r += active[at_pos(perm, i)] ? 1 : 0;
        }
        rank[b] = r;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) cnt_b[b] = rank[b + 1] - rank[b];
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t32 = 0, t64 = 0;
        for (int b = 0; b < nb; ++b) {
            off32[b] = t32;
            off64[b] = t64;
            const int32_t c = rank[b + 1] - rank[b];
            t32 += (c + per32 - 1) / per32;
            t64 += (c + per64 - 1) / per64;
        }
        off32[nb] = t32;
        off64[nb] = t64;
    }
}

// Tile k of a schedule: the boundary whose tile range holds k (binary search over off), and the
// run of `per` list entries it covers; slots past the last tile get count 0.
__global__ void k_fill_tiles(const int32_t* __restrict__ cnt_b, const int32_t* __restrict__ off,
                             const int32_t* __restrict__ rank_start, int32_t nb, int32_t per,
                             Tile* __restrict__ tiles, int64_t max_tiles) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= max_tiles) return;
    if (k >= off[nb]) {
        tiles[k] = Tile{0, 0, 0};
        return;
    }
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (off[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    const int32_t j = (int32_t)(k - off[lo]);
    Tile t;
    t.start = (int64_t)rank_start[lo] + (int64_t)j * per;
    t.count = min(per, cnt_b[lo] - j * per);
    t.b = lo;
    tiles[k] = t;
}

// ------------------------------------------------------------------------------------------------
// per-point state
// ------------------------------------------------------------------------------------------------
struct Common {
    double* lam_cur;   // [3][N] the trial to evaluate next
    double* best;      // [3][N] best (or converged) lambda
    double* best_phi;  // [N]
    int32_t* best_st;  // [N] residual status at best (kNoEval: not evaluated)
    int32_t* trials;   // [N]
    int32_t* status;   // [N]
    int32_t* active;   // [N]
    double* Bw;        // [3][N] evaluation outputs of the round
    double* dBw;       // [9][N]
    double* tanw;      // [12][N]
    double* fgw;       // [2][N]
    int32_t* conv;     // [max_rounds] points converging in each round
};

struct NMDev {
    double* V;        // [4][3][N] vertices
    double* F;        // [4][N]
    double* xr;       // [3][N] reflected point of the current iteration
    double* fr;       // [N]
    int32_t* phase;   // [N]
    int32_t* aux;     // [N] order (4 x 2 bits) | k << 8
};

struct LMDev {
    double* mu;       // [3][N] accepted mu
    double* mu_try;   // [3][N] mu being evaluated
    double* Phi;      // [N]
    double* rho;      // [N]
    double* u;        // [4][N]
    double* jac;      // [12][N]
    double* nu;       // [N]
    double* rad;      // [N] trust radius in lambda (+inf: none)
    int32_t* phase;   // [N]
};

struct SolveCfg {
    int32_t method, max_trials;
    double eps, step, cap, dvds, nu0;
    double radius0;   // LM trust radius at the start; 0: the simplex edge; +inf: none
};

__device__ __forceinline__ double cap_of(const SolveCfg& c, const BoundaryDev& bd) {
    return c.cap > 0.0 ? c.cap : 3.14159265358979323846 / bd.h;
}
__device__ __forceinline__ double step_of(const SolveCfg& c, const BoundaryDev& bd) {
    return c.step > 0.0 ? c.step : 1.0 / ((double)max(bd.nx, bd.ny) * bd.h);
}

enum : int32_t { kPInit0 = 0, kPReflect = 4, kPExpand = 5, kPContractOut = 6, kPContractIn = 7, kPShrink = 8 };

struct NMLocal {
    double V[4][3];
    double F[4];
    double xr[3];
    double fr;
    int32_t phase;
    int32_t ord[4];
    int32_t k;
    double P[3];   // the proposal
};

__device__ __forceinline__ void nm_new_iteration(NMLocal& s) {
#pragma clang fp contract(off)
    int o[4] = {0, 1, 2, 3};
    for (int a = 1; a < 4; ++a) {
        const int x = o[a];
        int b = a - 1;
        while (b >= 0 && (s.F[x] < s.F[o[b]] || (s.F[x] == s.F[o[b]] && x < o[b]))) {
            o[b + 1] = o[b];
            --b;
        }
        o[b + 1] = x;
    }
    for (int a = 0; a < 4; ++a) s.ord[a] = o[a];
    for (int p = 0; p < 3; ++p) {
        const double xb = ((s.V[o[0]][p] + s.V[o[1]][p]) + s.V[o[2]][p]) / 3.0;
        s.xr[p] = (1.0 + 1.0) * xb - 1.0 * s.V[o[3]][p];
        s.P[p] = s.xr[p];
    }
    s.phase = kPReflect;
}

__device__ __forceinline__ void nm_start_shrink(NMLocal& s) {
#pragma clang fp contract(off)
    const int lo = s.ord[0];
    for (int a = 1; a < 4; ++a)
        for (int p = 0; p < 3; ++p) s.V[s.ord[a]][p] = s.V[lo][p] + 0.5 * (s.V[s.ord[a]][p] - s.V[lo][p]);
    s.phase = kPShrink;
    s.k = 1;
    for (int p = 0; p < 3; ++p) s.P[p] = s.V[s.ord[1]][p];
}

// Consume the value of the trial just made (T = the previous proposal) and set the next proposal.
__device__ __forceinline__ void nm_advance(NMLocal& s, const double T[3], double phi) {
#pragma clang fp contract(off)
    const int lo = s.ord[0], sh = s.ord[2], hi = s.ord[3];
    if (s.phase < kPReflect) {
        const int k = s.phase;
        s.F[k] = phi;
        if (k < 3) {
            s.phase = k + 1;
            for (int p = 0; p < 3; ++p) s.P[p] = s.V[k + 1][p];
        } else {
            nm_new_iteration(s);
        }
        return;
    }
    if (s.phase == kPReflect) {
        s.fr = phi;
        double xb[3];
        for (int p = 0; p < 3; ++p) xb[p] = ((s.V[lo][p] + s.V[s.ord[1]][p]) + s.V[sh][p]) / 3.0;
        if (phi < s.F[lo]) {
            for (int p = 0; p < 3; ++p) s.P[p] = (1.0 + 1.0 * 2.0) * xb[p] - 1.0 * 2.0 * s.V[hi][p];
            s.phase = kPExpand;
        } else if (phi < s.F[sh]) {
            for (int p = 0; p < 3; ++p) s.V[hi][p] = s.xr[p];
            s.F[hi] = phi;
            nm_new_iteration(s);
        } else if (phi < s.F[hi]) {
            for (int p = 0; p < 3; ++p) s.P[p] = (1.0 + 0.5 * 1.0) * xb[p] - 0.5 * 1.0 * s.V[hi][p];
            s.phase = kPContractOut;
        } else {
            for (int p = 0; p < 3; ++p) s.P[p] = (1.0 - 0.5) * xb[p] + 0.5 * s.V[hi][p];
            s.phase = kPContractIn;
        }
        return;
    }
    if (s.phase == kPExpand) {
        if (phi < s.fr) {
            for (int p = 0; p < 3; ++p) s.V[hi][p] = T[p];
            s.F[hi] = phi;
        } else {
            for (int p = 0; p < 3; ++p) s.V[hi][p] = s.xr[p];
            s.F[hi] = s.fr;
        }
        nm_new_iteration(s);
        return;
    }
    if (s.phase == kPContractOut || s.phase == kPContractIn) {
        const bool acc = (s.phase == kPContractOut) ? (phi <= s.fr) : (phi < s.F[hi]);
        if (acc) {
            for (int p = 0; p < 3; ++p) s.V[hi][p] = T[p];
            s.F[hi] = phi;
            nm_new_iteration(s);
        } else {
            nm_start_shrink(s);
        }
        return;
    }
    // shrink: the k-th non-best vertex (in the iteration's order) was just evaluated
    s.F[s.ord[s.k]] = phi;
    if (s.k < 3) {
        s.k += 1;
        for (int p = 0; p < 3; ++p) s.P[p] = s.V[s.ord[s.k]][p];
    } else {
        nm_new_iteration(s);
    }
}

__device__ __forceinline__ void nm_load(NMLocal& s, const NMDev& d, int64_t i, int64_t N) {
    for (int v = 0; v < 4; ++v) {
        for (int p = 0; p < 3; ++p) s.V[v][p] = d.V[(v * 3 + p) * N + i];
        s.F[v] = d.F[v * N + i];
    }
    for (int p = 0; p < 3; ++p) s.xr[p] = d.xr[p * N + i];
    s.fr = d.fr[i];
    s.phase = d.phase[i];
    const int32_t a = d.aux[i];
    for (int v = 0; v < 4; ++v) s.ord[v] = (a >> (2 * v)) & 3;
    s.k = (a >> 8) & 3;
}

__device__ __forceinline__ void nm_store(const NMLocal& s, const NMDev& d, int64_t i, int64_t N) {
    for (int v = 0; v < 4; ++v) {
        for (int p = 0; p < 3; ++p) d.V[(v * 3 + p) * N + i] = s.V[v][p];
        d.F[v * N + i] = s.F[v];
    }
    for (int p = 0; p < 3; ++p) d.xr[p * N + i] = s.xr[p];
    d.fr[i] = s.fr;
    d.phase[i] = s.phase;
    int32_t a = 0;
    for (int v = 0; v < 4; ++v) a |= s.ord[v] << (2 * v);
    d.aux[i] = a | (s.k << 8);
}

__device__ __forceinline__ bool feasible(const double P[3], double cap) {
    return fabs(P[0]) <= cap && fabs(P[1]) <= cap && fabs(P[2]) <= cap;
}

__device__ __forceinline__ void record_best(const Common& C, int64_t i, int64_t N, const double T[3],
                                            double phi, int32_t st) {
    if (C.best_st[i] == kNoEval || phi < C.best_phi[i]) {
        for (int p = 0; p < 3; ++p) C.best[p * N + i] = T[p];
        C.best_phi[i] = phi;
        C.best_st[i] = st;
    }
}

__device__ __forceinline__ void finish_budget(const Common& C, int64_t i) {
    C.active[i] = 0;
    const int32_t bs = C.best_st[i];
    if (isfinite(C.best_phi[i])) C.status[i] = kStBudget;
    else C.status[i] = (bs == kStDegenerate || bs == kStNonfinite) ? bs : kStNonfinite;
}

// Advance the simplex until a feasible proposal exists or the budget is spent; infeasible proposals
// (|lambda_p| > cap) cost a trial with Phi = +inf, like the oracle.
__device__ void nm_propose(NMLocal& s, const Common& C, int64_t i, int64_t N, int32_t max_trials,
                           double cap) {
    while (!feasible(s.P, cap)) {
        const int32_t tr = ++C.trials[i];
        if (C.best_st[i] == kNoEval) {
            for (int p = 0; p < 3; ++p) C.best[p * N + i] = s.P[p];
            C.best_phi[i] = __builtin_inf();
            C.best_st[i] = kStNonfinite;
        }
        if (tr >= max_trials) {
            finish_budget(C, i);
            return;
        }
        double T[3] = {s.P[0], s.P[1], s.P[2]};
        nm_advance(s, T, __builtin_inf());
    }
    for (int p = 0; p < 3; ++p) C.lam_cur[p * N + i] = s.P[p];
}

__global__ void k_solve_init(SolveCfg cfg, const BoundaryDev* __restrict__ bnd,
                             const int32_t* __restrict__ bidx, int64_t N, const double* __restrict__ lam0,
                             Common C, NMDev nm, LMDev lm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const BoundaryDev bd = bnd[bidx[i]];
    double l0[3];
    bool fin = true;
    for (int p = 0; p < 3; ++p) {
        l0[p] = lam0[p * N + i];
        fin = fin && isfinite(l0[p]);
        C.best[p * N + i] = l0[p];
    }
    C.trials[i] = 0;
    C.best_phi[i] = __builtin_inf();
    C.best_st[i] = kNoEval;
    C.status[i] = kStBudget;
    C.active[i] = fin ? 1 : 0;
    if (!fin) {
        C.status[i] = kStNonfinite;
        return;
    }
    if (cfg.method == DBIE_NELDER_MEAD) {
        NMLocal s;
        const double d = step_of(cfg, bd);
        for (int v = 0; v < 4; ++v)
            for (int p = 0; p < 3; ++p) s.V[v][p] = l0[p] + ((v >= 1 && v - 1 == p) ? d : 0.0);
        for (int v = 0; v < 4; ++v) s.F[v] = __builtin_inf();
        for (int p = 0; p < 3; ++p) s.xr[p] = 0.0;
        s.fr = 0.0;
        s.phase = kPInit0;
        for (int v = 0; v < 4; ++v) s.ord[v] = v;
        s.k = 0;
        for (int p = 0; p < 3; ++p) s.P[p] = s.V[0][p];
        nm_propose(s, C, i, N, cfg.max_trials, cap_of(cfg, bd));
        nm_store(s, nm, i, N);
    } else {
        for (int p = 0; p < 3; ++p) {
            const double m = l0[p] * l0[p];
            lm.mu_try[p * N + i] = m;
            lm.mu[p * N + i] = m;
            C.lam_cur[p * N + i] = sqrt(m);
        }
        lm.phase[i] = 0;
        lm.nu[i] = cfg.nu0;
        lm.rad[i] = cfg.radius0 > 0.0 ? cfg.radius0 : step_of(cfg, bd);
    }
}

__global__ void k_nm_update(SolveCfg cfg, const BoundaryDev* __restrict__ bnd,
                            const int32_t* __restrict__ bidx, int64_t N, const int32_t* __restrict__ list,
                            const int32_t* __restrict__ n_active, const int32_t* __restrict__ round,
                            Common C, NMDev nm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= *n_active) return;
    const int64_t i = list[j];
    const BoundaryDev bd = bnd[bidx[i]];
    double B[3], dB[9], T[3];
    for (int p = 0; p < 3; ++p) {
        B[p] = C.Bw[p * N + i];
        T[p] = C.lam_cur[p * N + i];
    }
    for (int r = 0; r < 9; ++r) dB[r] = C.dBw[r * N + i];
    const Resid R = residual_fp64(B, dB, cfg.dvds * bd.h);
    const int32_t tr = ++C.trials[i];
    if (R.rho <= cfg.eps) {
        for (int p = 0; p < 3; ++p) C.best[p * N + i] = T[p];
        C.best_phi[i] = R.Phi;
        C.best_st[i] = R.status;
        C.status[i] = kStConverged;
        C.active[i] = 0;
        atomicAdd(&C.conv[*round], 1);
        return;
    }
    record_best(C, i, N, T, R.Phi, R.status);
    if (tr >= cfg.max_trials) {
        finish_budget(C, i);
        return;
    }
    NMLocal s;
    nm_load(s, nm, i, N);
    nm_advance(s, T, R.Phi);
    nm_propose(s, C, i, N, cfg.max_trials, cap_of(cfg, bd));
    nm_store(s, nm, i, N);
}

// Solve (A + nu diag(A)) d = -J^T u with diag(A) floored at 1e-12 max diag(A); LU with partial
// pivoting. d = 0 when A has no positive diagonal.
__device__ __forceinline__ void lm_direction(const double jac[12], const double u[4], double nu, double d[3]) {
    double A[3][3], g[3];
    for (int a = 0; a < 3; ++a) {
        g[a] = 0.0;
        for (int q = 0; q < 4; ++q) g[a] += jac[q * 3 + a] * u[q];
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int q = 0; q < 4; ++q) s += jac[q * 3 + a] * jac[q * 3 + b];
            A[a][b] = s;
        }
    }
    const double m = fmax(A[0][0], fmax(A[1][1], A[2][2]));
    d[0] = d[1] = d[2] = 0.0;
    if (!(m > 0.0) || !isfinite(m)) return;
    double M[3][4];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) M[a][b] = A[a][b];
        M[a][a] += nu * fmax(A[a][a], 1e-12 * m);
        M[a][3] = -g[a];
    }
    for (int c = 0; c < 3; ++c) {
        int pr = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[r][c]) > fabs(M[pr][c])) pr = r;
        if (pr != c)
            for (int k = 0; k < 4; ++k) {
                const double t = M[c][k];
                M[c][k] = M[pr][k];
                M[pr][k] = t;
            }
        if (M[c][c] == 0.0) return;
        for (int r = c + 1; r < 3; ++r) {
            const double f = M[r][c] / M[c][c];
            for (int k = c; k < 4; ++k) M[r][k] -= f * M[c][k];
        }
    }
    double x[3];
    for (int r = 2; r >= 0; --r) {
        double s = M[r][3];
        for (int k = r + 1; k < 3; ++k) s -= M[r][k] * x[k];
        x[r] = s / M[r][r];
    }
    if (isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2])) {
        d[0] = x[0];
        d[1] = x[1];
        d[2] = x[2];
    }
}

__global__ void k_lm_update(SolveCfg cfg, const BoundaryDev* __restrict__ bnd,
                            const int32_t* __restrict__ bidx, int64_t N, const int32_t* __restrict__ list,
                            const int32_t* __restrict__ n_active, const int32_t* __restrict__ round,
                            Common C, LMDev lm) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= *n_active) return;
    const int64_t i = list[j];
    const BoundaryDev bd = bnd[bidx[i]];
    const double c = cfg.dvds * bd.h;
    double B[3], dB[9], tn[12], mt[3];
    for (int p = 0; p < 3; ++p) {
        B[p] = C.Bw[p * N + i];
        mt[p] = lm.mu_try[p * N + i];
    }
    for (int r = 0; r < 9; ++r) dB[r] = C.dBw[r * N + i];
    for (int r = 0; r < 12; ++r) tn[r] = C.tanw[r * N + i];
    const Resid R = residual_fp64(B, dB, c);
    const int32_t tr = ++C.trials[i];
    const int32_t phase = lm.phase[i];
    if (phase == 0 && !isfinite(R.Phi)) {
        for (int p = 0; p < 3; ++p) C.best[p * N + i] = sqrt(mt[p]);
        C.status[i] = R.status;
        C.active[i] = 0;
        return;
    }
    if (R.rho <= cfg.eps) {
        for (int p = 0; p < 3; ++p) C.best[p * N + i] = sqrt(mt[p]);
        C.status[i] = kStConverged;
        C.active[i] = 0;
        atomicAdd(&C.conv[*round], 1);
        return;
    }
    double nu = lm.nu[i];
    double rad = lm.rad[i];
    const double cap = cap_of(cfg, bd);
    const bool accept = (phase == 0) || (R.Phi < lm.Phi[i]);
    if (accept) {
        double jac[12];
        residual_jacobian_fp64(B, dB, tn, c, jac);
        for (int p = 0; p < 3; ++p) lm.mu[p * N + i] = mt[p];
        lm.Phi[i] = R.Phi;
        lm.rho[i] = R.rho;
        for (int q = 0; q < 4; ++q) lm.u[q * N + i] = R.u[q];
        for (int r = 0; r < 12; ++r) lm.jac[r * N + i] = jac[r];
        if (phase != 0) {
            nu = nu / 10.0;
            if (!isinf(rad)) rad = fmin(2.0 * rad, cap);
        }
    } else {
        nu = nu * 10.0;
        if (!isinf(rad)) rad = 0.5 * rad;
    }
    lm.nu[i] = nu;
    lm.rad[i] = rad;
    lm.phase[i] = 1;
    double mu[3];
    for (int p = 0; p < 3; ++p) {
        mu[p] = lm.mu[p * N + i];
        C.best[p * N + i] = sqrt(mu[p]);
    }
    if (tr >= cfg.max_trials) {
        C.status[i] = kStBudget;
        C.active[i] = 0;
        return;
    }
    double jac[12], u[4], d[3];
    for (int r = 0; r < 12; ++r) jac[r] = lm.jac[r * N + i];
    for (int q = 0; q < 4; ++q) u[q] = lm.u[q * N + i];
    lm_direction(jac, u, nu, d);
    // the proposal mu + d, clipped per component to where sqrt(mu) lies within rad of the accepted
    // point's and inside [0, cap] (with no trust region: to [0, cap^2])
    const double cap2 = cap * cap;
    for (int p = 0; p < 3; ++p) {
        double m;
        if (isinf(rad)) {
            m = fmin(fmax(mu[p] + d[p], 0.0), cap2);
        } else {
            const double l = sqrt(mu[p]);
            const double lo = fmax(l - rad, 0.0);
            const double hi = fmin(l + rad, cap);
            m = fmin(fmax(mu[p] + d[p], lo * lo), hi * hi);
        }
        lm.mu_try[p * N + i] = m;
        C.lam_cur[p * N + i] = sqrt(m);
    }
}

// |lambda*| to the caller's array, plus status and trials.
__global__ void k_solve_finish(int64_t N, Common C, double* __restrict__ lam_out, int32_t* __restrict__ st,
                               int32_t* __restrict__ trials) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int p = 0; p < 3; ++p) lam_out[p * N + i] = fabs(C.best[p * N + i]);
    st[i] = C.status[i];
    trials[i] = C.trials[i];
}

// FP64 acceptance: CONVERGED iff max(f, g) <= eps in FP64 at the returned lambda.
__global__ void k_solve_accept(int64_t N, const double* __restrict__ fg, double eps, int32_t* __restrict__ st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t s = st[i];
    if (s != kStConverged && s != kStBudget) return;
    const double rho = fmax(fg[i], fg[N + i]);
    st[i] = (rho <= eps) ? kStConverged : kStBudget;
}

// FP64 confirmation of the points that converged in FP32C (re-evaluated alone): CONVERGED stays only
// if max(f, g) <= eps in FP64; fg holds values for those points only.
__global__ void k_solve_confirm(int64_t N, const double* __restrict__ fg, double eps, int32_t* __restrict__ st) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || st[i] != kStConverged) return;
    if (!(fmax(fg[i], fg[N + i]) <= eps)) st[i] = kStBudget;
}

// active[i] = (status[i] == CONVERGED): the list the FP64 confirmation evaluates.
__global__ void k_mark_converged(int64_t N, const int32_t* __restrict__ st, int32_t* __restrict__ active) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) active[i] = st[i] == kStConverged ? 1 : 0;
}

// The round counter read by the update kernels (a device word, so that captured rounds replay).
__global__ void k_round_next(int32_t* __restrict__ round) { *round += 1; }

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------------------------------------
// host side
// ------------------------------------------------------------------------------------------------
namespace {

struct Layout {
    size_t off = 0;
    template <class T>
    size_t take(size_t n) {
        const size_t o = off;
        off += (n * sizeof(T) + 255) / 256 * 256;
        return o;
    }
};

struct SolverBufs {
    Common C;
    NMDev nm;
    LMDev lm;
    int32_t* list;
    int32_t* bsum;
    int32_t* n_active;
    int32_t* round;     // [1] index of the current round
    int32_t* cnt_b;     // [nb] active points per boundary
    int32_t* rank;      // [nb + 1] list offset of each boundary
    int32_t* off32;     // [nb + 1] tile offsets of the FP32C schedule
    int32_t* off64;     // [nb + 1] tile offsets of the FP64 schedule
    int64_t* segd;      // [nb + 1] point segments
    Tile* tiles32;
    Tile* tiles64;
    int64_t max32, max64;
    int32_t nblk;
    int32_t max_rounds;
};

int64_t pad8(int64_t x) { return (x + 7) / 8 * 8; }

}  // namespace

void solver_free(SolverState& s) {
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.ev_in) (void)hipEventDestroy(s.ev_in);
    if (s.ev_out) (void)hipEventDestroy(s.ev_out);
    if (s.rs) (void)hipStreamDestroy(s.rs);
    if (s.block_owned) (void)hipFree(s.block);
    if (s.count_h) (void)hipHostFree(s.count_h);
    s = SolverState{};
}

// The solver block: every per-point array and the device schedules, 256-byte aligned, for N points,
// nb magnetograms, max_rounds trials and per32 points per FP32C tile.
struct SolverOffsets {
    size_t lam, best, bphi, bst, tr, st, act, B, dB, tan, fg, conv, V, F, Xr, Fr, ph, aux;
    size_t mu, mut, phi, rho, u, jac, nu, rad, lph, list, bsum, nact, rnd, cnt, rank, o32, o64, seg, t32, t64;
    int64_t max32, max64;
    int32_t nblk;
    size_t bytes;
};

static SolverOffsets solver_layout(int64_t N, int32_t nb, int32_t max_rounds, int32_t per32) {
    SolverOffsets o;
    o.max32 = pad8((N + per32 - 1) / per32 + nb);
    o.max64 = pad8((N + 255) / 256 + nb);
    o.nblk = (int32_t)((N + kCompactBlock - 1) / kCompactBlock);
    Layout L;
    const size_t n = (size_t)N;
    o.lam = L.take<double>(3 * n), o.best = L.take<double>(3 * n), o.bphi = L.take<double>(n);
    o.bst = L.take<int32_t>(n), o.tr = L.take<int32_t>(n), o.st = L.take<int32_t>(n), o.act = L.take<int32_t>(n);
    o.B = L.take<double>(3 * n), o.dB = L.take<double>(9 * n), o.tan = L.take<double>(12 * n),
    o.fg = L.take<double>(2 * n);
    o.conv = L.take<int32_t>((size_t)max_rounds + 1);
    o.V = L.take<double>(12 * n), o.F = L.take<double>(4 * n), o.Xr = L.take<double>(3 * n),
    o.Fr = L.take<double>(n), o.ph = L.take<int32_t>(n), o.aux = L.take<int32_t>(n);
    o.mu = L.take<double>(3 * n), o.mut = L.take<double>(3 * n), o.phi = L.take<double>(n),
    o.rho = L.take<double>(n), o.u = L.take<double>(4 * n), o.jac = L.take<double>(12 * n),
    o.nu = L.take<double>(n), o.rad = L.take<double>(n), o.lph = L.take<int32_t>(n);
    o.list = L.take<int32_t>(n), o.bsum = L.take<int32_t>((size_t)o.nblk + 1), o.nact = L.take<int32_t>(1),
    o.rnd = L.take<int32_t>(1), o.cnt = L.take<int32_t>((size_t)nb), o.rank = L.take<int32_t>((size_t)nb + 1),
    o.o32 = L.take<int32_t>((size_t)nb + 1), o.o64 = L.take<int32_t>((size_t)nb + 1),
    o.seg = L.take<int64_t>((size_t)nb + 1);
    o.t32 = L.take<Tile>((size_t)o.max32), o.t64 = L.take<Tile>((size_t)o.max64);
    o.bytes = L.off;
    return o;
}

size_t solver_workspace_bytes(const dbie_ctx* c) {
    // every budget the API accepts (<= 1e6 trials) and the smallest instantiated tile (most tiles)
    F32Shape sh[16];
    const int n = std::min(field32c_shapes(sh, 16), 16);
    int32_t per = 1 << 30;
    for (int k = 0; k < n; ++k) per = std::min(per, sh[k].ppl * sh[k].waves * 64);
    return solver_layout(ctx_n(c), ctx_nb(c), 1000000, per).bytes;
}

static int solver_bufs(dbie_ctx* c, int32_t max_rounds, bool lm_mode, SolverBufs& b) {
    SolverState& S = ctx_solver(c);
    const int64_t N = ctx_n(c);
    const int32_t nb = ctx_nb(c);
    const F32Shape sh = get_shape(c, lm_mode);
    const int32_t per32 = sh.ppl * sh.waves * 64;
    const SolverOffsets o = solver_layout(N, nb, max_rounds, per32);
    b.max32 = o.max32;
    b.max64 = o.max64;
    b.nblk = o.nblk;
    b.max_rounds = max_rounds;
    const size_t need = o.bytes;
    void* ws = ctx_ws_region(c, kWsSolver, need);
    if (ws == kWsTooSmall)
        return ctx_fail(c, DBIE_E_WORKSPACE, "the caller's workspace is too small for this solve");
    if (ws) {
        if (S.block && S.block_owned) (void)hipFree(S.block);
        S.block = ws;
        S.bytes = (int64_t)need;
        S.block_owned = false;
    } else if (!S.block || !S.block_owned || S.bytes < (int64_t)need) {
        if (S.block && S.block_owned) (void)hipFree(S.block);
        S.block = nullptr;
        S.bytes = 0;
        if (hipMalloc(&S.block, need) != hipSuccess)
            return ctx_fail(c, DBIE_E_WORKSPACE, "cannot allocate the solver workspace");
        S.bytes = (int64_t)need;
        S.block_owned = true;
    }
    if (!S.count_h) {
        if (hipHostMalloc((void**)&S.count_h, sizeof(int32_t)) != hipSuccess)
            return ctx_fail(c, DBIE_E_WORKSPACE, "cannot allocate pinned host memory");
    }
    char* base = (char*)S.block;
    auto D = [&](size_t off) { return (void*)(base + off); };
    b.C = Common{(double*)D(o.lam), (double*)D(o.best), (double*)D(o.bphi), (int32_t*)D(o.bst), (int32_t*)D(o.tr),
                 (int32_t*)D(o.st), (int32_t*)D(o.act), (double*)D(o.B), (double*)D(o.dB), (double*)D(o.tan),
                 (double*)D(o.fg), (int32_t*)D(o.conv)};
    b.nm = NMDev{(double*)D(o.V), (double*)D(o.F), (double*)D(o.Xr), (double*)D(o.Fr), (int32_t*)D(o.ph),
                 (int32_t*)D(o.aux)};
    b.lm = LMDev{(double*)D(o.mu), (double*)D(o.mut), (double*)D(o.phi), (double*)D(o.rho), (double*)D(o.u),
                 (double*)D(o.jac), (double*)D(o.nu), (double*)D(o.rad), (int32_t*)D(o.lph)};
    b.list = (int32_t*)D(o.list);
    b.bsum = (int32_t*)D(o.bsum);
    b.n_active = (int32_t*)D(o.nact);
    b.round = (int32_t*)D(o.rnd);
    b.cnt_b = (int32_t*)D(o.cnt);
    b.rank = (int32_t*)D(o.rank);
    b.off32 = (int32_t*)D(o.o32);
    b.off64 = (int32_t*)D(o.o64);
    b.segd = (int64_t*)D(o.seg);
    b.tiles32 = (Tile*)D(o.t32);
    b.tiles64 = (Tile*)D(o.t64);
    return DBIE_OK;
}

static hipError_t compact(const SolverBufs& b, const int32_t* perm, int64_t N, int32_t nb, int32_t per32,
                          hipStream_t s) {
    const unsigned nblk = (unsigned)std::max<int32_t>(b.nblk, 1);
    hipLaunchKernelGGL(k_compact_count, dim3(nblk), dim3(kCompactThreads), 0, s, b.C.active, perm, N, b.bsum);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, b.bsum, (int32_t)nblk, b.n_active);
    hipLaunchKernelGGL(k_compact_scatter, dim3(nblk), dim3(kCompactThreads), 0, s, b.C.active, perm, N, b.bsum,
                       b.list);
    hipLaunchKernelGGL(k_seg_counts, dim3(1), dim3(256), 0, s, b.C.active, perm, N, b.bsum, b.n_active, b.segd,
                       nb, b.cnt_b, b.rank, per32, (int32_t)256, b.off32, b.off64);
    hipLaunchKernelGGL(k_fill_tiles, dim3((unsigned)((b.max32 + 255) / 256)), dim3(256), 0, s, b.cnt_b, b.off32,
                       b.rank, nb, per32, b.tiles32, b.max32);
    hipLaunchKernelGGL(k_fill_tiles, dim3((unsigned)((b.max64 + 255) / 256)), dim3(256), 0, s, b.cnt_b, b.off64,
                       b.rank, nb, (int32_t)256, b.tiles64, b.max64);
    return hipGetLastError();
}

}  // namespace dbie

using namespace dbie;

extern "C" int dbie_solve_lambda(dbie_ctx* c, double* lam, const dbie_solve_opts* opt, double* Bout,
                                 double* fgout, int32_t* status, int32_t* trials, void* stream) {
    if (!c) return DBIE_E_INVAL;
    if (!opt) return ctx_fail(c, DBIE_E_INVAL, "solve options are NULL");
    if (opt->method != DBIE_NELDER_MEAD && opt->method != DBIE_LEVENBERG_MARQUARDT)
        return ctx_fail(c, DBIE_E_INVAL, "method must be DBIE_NELDER_MEAD or DBIE_LEVENBERG_MARQUARDT");
    if (opt->max_trials < 1 || opt->max_trials > 1000000)
        return ctx_fail(c, DBIE_E_INVAL, "max_trials must lie in [1, 1e6]");
    if (!(opt->eps >= 0.0) || !std::isfinite(opt->eps)) return ctx_fail(c, DBIE_E_INVAL, "eps must be >= 0");
    if (!std::isfinite(opt->init_step) || !std::isfinite(opt->lambda_cap))
        return ctx_fail(c, DBIE_E_INVAL, "init_step and lambda_cap must be finite");
    if (!(opt->lm_radius >= 0.0)) return ctx_fail(c, DBIE_E_INVAL, "lm_radius must be >= 0 (or +inf)");
    if (!(opt->lm_damping >= 0.0) || !std::isfinite(opt->lm_damping))
        return ctx_fail(c, DBIE_E_INVAL, "lm_damping must be finite and >= 0");
    const int64_t N = ctx_n(c);
    if (int rc = ctx_check_device(c)) return rc;
    if (N > 0 && (!lam || !status || !trials))
        return ctx_fail(c, DBIE_E_INVAL, "lambda_inout, status and trials are required");
    if (N == 0) return DBIE_OK;
    hipStream_t s = (hipStream_t)stream;
    SolverBufs b;
    const bool lmm = opt->method == DBIE_LEVENBERG_MARQUARDT;
    solver_forget_last(c);   // the block may move below
    int rc = solver_bufs(c, opt->max_trials, lmm, b);
    if (rc) return rc;
    const int32_t nb = ctx_nb(c);
    const Geo& geo = ctx_geo(c);
    const BoundaryDev* bnd = ctx_bnd(c);
    const bool fp64 = ctx_precision(c) == DBIE_FP64;
    const F32Shape sh = get_shape(c, lmm);
    const int32_t per32 = sh.ppl * sh.waves * 64;
    SolveCfg cfg{opt->method, opt->max_trials, opt->eps, opt->init_step, opt->lambda_cap, ctx_dvds(c),
                 opt->lm_damping > 0.0 ? opt->lm_damping : 1.0, opt->lm_radius};
    const unsigned gN = (unsigned)((N + 255) / 256);
#define SOLVE_HIP(call)                                                           \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) return ctx_fail(c, DBIE_E_DEVICE, hipGetErrorString(e_)); \
    } while (0)
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((opt->max_trials + 256) / 256)), dim3(256), 0, s, b.C.conv,
                       (int64_t)opt->max_trials + 1, 0);
    hipLaunchKernelGGL(k_solve_init, dim3(gN), dim3(256), 0, s, cfg, bnd, geo.bidx, N, lam, b.C, b.nm, b.lm);
    SOLVE_HIP(hipGetLastError());
    SOLVE_HIP(hipMemcpyAsync(b.segd, ctx_seg(c), (size_t)(nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    const int32_t* perm = fp64 ? nullptr : ctx_perm(c);
    SOLVE_HIP(compact(b, perm, N, nb, per32, s));
    EvalSet set{b.list, b.n_active, b.tiles32, b.max32, b.tiles64, b.max64};
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, b.round, (int64_t)1, 0);
    SOLVE_HIP(hipGetLastError());
    // one round: bulk sum + finalize over the active list, update, compaction, round counter
    auto enqueue_round = [&](hipStream_t q) -> int {
        int r = eval_set(c, b.C.lam_cur, fp64, lmm, &set, b.C.Bw, b.C.dBw, nullptr, lmm ? b.C.tanw : nullptr, q);
        if (r) return r;
        if (lmm)
            hipLaunchKernelGGL(k_lm_update, dim3(gN), dim3(256), 0, q, cfg, bnd, geo.bidx, N, b.list, b.n_active,
                               b.round, b.C, b.lm);
        else
            hipLaunchKernelGGL(k_nm_update, dim3(gN), dim3(256), 0, q, cfg, bnd, geo.bidx, N, b.list, b.n_active,
                               b.round, b.C, b.nm);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = compact(b, perm, N, nb, per32, q);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_round_next, dim3(1), dim3(1), 0, q, b.round);
            e = hipGetLastError();
        }
        return e == hipSuccess ? DBIE_OK : ctx_fail(c, DBIE_E_DEVICE, hipGetErrorString(e));
    };
    int32_t rounds = 0;
    const int32_t check_every = 4;
    // with DBIE_PROGRESS set in the environment, long solves report their round and active count on
    // stderr (at the host's reads of the count, at most every 20 s)
    const bool progress = std::getenv("DBIE_PROGRESS") != nullptr;
    auto last_print = std::chrono::steady_clock::now();
    std::vector<hipEvent_t>& trace = solver_trace_events(c);
    hipEvent_t& trace_end = solver_trace_end(c);
    const bool tracing = solver_tracing(c);
    if (tracing) {
        hipEvent_t e = nullptr;
        SOLVE_HIP(hipEventCreate(&e));
        SOLVE_HIP(hipEventRecord(e, s));
        trace.push_back(e);
    }
    // Graph replay of check_every rounds: captured once per context and solve configuration (all
    // kernel arguments are fixed; the round index lives on the device). Not used while recording
    // events (timing or tracing).
    const bool graphs = opt->use_graph && !tracing && !ctx_timing(c) && opt->max_trials >= check_every;
    hipGraphExec_t exec = nullptr;
    hipStream_t rs = s;   // the stream the rounds run on
    if (graphs) {
        SolverState& S0 = ctx_solver(c);
        if (!S0.rs) {
            SOLVE_HIP(hipStreamCreateWithFlags(&S0.rs, hipStreamNonBlocking));
            SOLVE_HIP(hipEventCreateWithFlags(&S0.ev_in, hipEventDisableTiming));
            SOLVE_HIP(hipEventCreateWithFlags(&S0.ev_out, hipEventDisableTiming));
        }
        rs = S0.rs;
        SOLVE_HIP(hipEventRecord(S0.ev_in, s));
        SOLVE_HIP(hipStreamWaitEvent(rs, S0.ev_in, 0));
        rc = ensure_acc(c, 1);   // no allocation may happen inside the capture
        if (rc) return rc;
        GraphKey key;
        std::memset(&key, 0, sizeof(key));   // compared bytewise, padding included
        key.method = opt->method;
        key.max_trials = opt->max_trials;
        key.fp64 = fp64;
        key.eps = opt->eps;
        key.step = opt->init_step;
        key.cap = opt->lambda_cap;
        key.radius = opt->lm_radius;
        key.damping = opt->lm_damping;
        key.block = ctx_solver(c).block;
        key.stream = rs;
        key.per32 = per32;
        key.perm = perm;
        key.acc = ctx_acc(c);
        key.split = ctx_split(c);
        key.ppl = sh.ppl;
        key.waves = sh.waves;
        key.persist = sh.persist;
        SolverState& S = ctx_solver(c);
        if (S.exec && std::memcmp(&S.key, &key, sizeof(GraphKey)) == 0) {
            exec = S.exec;
        } else {
            if (S.exec) (void)hipGraphExecDestroy(S.exec);
            S.exec = nullptr;
            hipGraph_t g = nullptr;
            SOLVE_HIP(hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal));
            int rc2 = DBIE_OK;
            for (int k = 0; k < check_every && rc2 == DBIE_OK; ++k) rc2 = enqueue_round(rs);
            const hipError_t ee = hipStreamEndCapture(rs, &g);
            if (rc2) {
                if (g) (void)hipGraphDestroy(g);
                return rc2;
            }
            SOLVE_HIP(ee);
            const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            SOLVE_HIP(ei);
            S.exec = exec;
            S.key = key;
        }
    }
    while (rounds < opt->max_trials) {
        const int32_t k = std::min(check_every, opt->max_trials - rounds);
        if (exec && k == check_every) {
            SOLVE_HIP(hipGraphLaunch(exec, rs));
        } else {
            for (int32_t j = 0; j < k; ++j) {
                rc = enqueue_round(rs);
                if (rc) return rc;
                if (tracing) {
                    hipEvent_t e = nullptr;
                    SOLVE_HIP(hipEventCreate(&e));
                    SOLVE_HIP(hipEventRecord(e, s));
                    trace.push_back(e);
                }
            }
        }
        rounds += k;
        if (rounds < opt->max_trials) {
            SOLVE_HIP(hipMemcpyAsync(ctx_solver(c).count_h, b.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, rs));
            SOLVE_HIP(hipStreamSynchronize(rs));
            if (progress && std::chrono::steady_clock::now() - last_print > std::chrono::seconds(20)) {
                last_print = std::chrono::steady_clock::now();
                std::fprintf(stderr, "dbie_solve_lambda: %d of %d rounds, %d points active\n", rounds,
                             opt->max_trials, *ctx_solver(c).count_h);
                std::fflush(stderr);
            }
            if (*ctx_solver(c).count_h == 0) break;
        }
    }
    if (rs != s) {
        SOLVE_HIP(hipEventRecord(ctx_solver(c).ev_out, rs));
        SOLVE_HIP(hipStreamWaitEvent(s, ctx_solver(c).ev_out, 0));
    }
    ctx_solver(c).last_rounds = rounds;
    ctx_solver(c).last_conv = b.C.conv;
    hipLaunchKernelGGL(k_solve_finish, dim3(gN), dim3(256), 0, s, N, b.C, lam, status, trials);
    SOLVE_HIP(hipGetLastError());
    const bool accept64 = !fp64 && opt->fp64_accept;
    if (accept64 && !Bout && !fgout) {
        // only the points that converged in FP32C need the FP64 test: compact them and evaluate
        // those alone
        hipLaunchKernelGGL(k_mark_converged, dim3(gN), dim3(256), 0, s, N, status, b.C.active);
        SOLVE_HIP(hipGetLastError());
        SOLVE_HIP(compact(b, perm, N, nb, per32, s));
        // their number sizes the pixel slices (few points: many slices)
        int32_t* cnt = ctx_solver(c).count_h;
        SOLVE_HIP(hipMemcpyAsync(cnt, b.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SOLVE_HIP(hipStreamSynchronize(s));
        if (*cnt > 0) {
            rc = eval_set(c, lam, true, false, &set, b.C.Bw, b.C.dBw, b.C.fgw, nullptr, s,
                          split_for_points(c, *cnt));
            if (rc) return rc;
            hipLaunchKernelGGL(k_solve_confirm, dim3(gN), dim3(256), 0, s, N, b.C.fgw, opt->eps, status);
            SOLVE_HIP(hipGetLastError());
        }
    } else if (Bout || fgout || accept64) {
        double* Bdst = Bout ? Bout : b.C.Bw;
        double* fgdst = fgout ? fgout : b.C.fgw;
        rc = eval_set(c, lam, fp64 || accept64, false, nullptr, Bdst, b.C.dBw, fgdst, nullptr, s);
        if (rc) return rc;
        if (accept64) {
            hipLaunchKernelGGL(k_solve_accept, dim3(gN), dim3(256), 0, s, N, fgdst, opt->eps, status);
            SOLVE_HIP(hipGetLastError());
        }
    }
    if (tracing) {
        SOLVE_HIP(hipEventCreate(&trace_end));
        SOLVE_HIP(hipEventRecord(trace_end, s));
    }
    return DBIE_OK;
#undef SOLVE_HIP
}
