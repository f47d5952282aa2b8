// Host side of the C ABI declared in include/dbie.h: argument validation, the context (library-owned
// device copies of the problem, per-point geometry, the tile schedules) and the dispatch of the
// kernels onto the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dbie.h"
#include "dbie_internal.h"
#include "dbie_solver.h"

using namespace dbie;

// Work memory of dbie_eval_field_noalloc: the partial sums of its bulk pass ([S][L][kAcc][N] doubles)
// live in this static array instead of the context's accumulator. Every device the library runs on
// holds its own copy until the process ends; all calls on one device share it.
static constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {

thread_local std::string g_init_error;

// Device address of each device's copy of `scratch`, looked up once per device (with that device
// current) by the first dbie_init on it. In host code `scratch` itself is only a stand-in symbol.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t noalloc_scratch(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

constexpr int kTile64 = 256;         // points per workgroup of the FP64 kernels

template <class T>
hipError_t dalloc(T** p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 1;
    return hipMalloc((void**)p, n * sizeof(T));
}

// Gauss-Legendre points and weights on [-1, 1]: Newton's method on P_n from the three-term recurrence
// (n P_n = (2n - 1) x P_{n-1} - (n - 1) P_{n-2}), started at cos(pi (k + 3/4) / (n + 1/2)); the weight
// is 2 / ((1 - x^2) P_n'(x)^2). Points ascending.
void gauss_legendre(int n, double* x, double* w) {
    for (int k = 0; k < n; ++k) {
        double t = std::cos(M_PI * (k + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        x[n - 1 - k] = t;
        w[n - 1 - k] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

}  // namespace

struct dbie_ctx {
    int device = 0;
    dbie_options opt{};
    int32_t nb = 0;
    int64_t N = 0;
    int64_t npix_total = 0;
    std::vector<BoundaryDev> bnd_h;
    std::vector<int64_t> seg;
    BoundaryDev* bnd_d = nullptr;
    double* B0d = nullptr;      // FP64 planes, concatenated per boundary
    // quadrature grid of the FP64 path (BoundaryDev::gcols/grows): positions, and the weighted field
    // (the B0 planes themselves for the nodal rule; a separate allocation for 9-node elements)
    double* gpos = nullptr;
    double* gB = nullptr;
    double* qlw = nullptr;      // 9-node elements: lw[3 g + a] = w_g L_a(xi_g) (device, 3 G doubles)
    float4* gposf = nullptr;    // 9-node elements, FP32C: split grid positions (BoundaryDev::gposf_off)
    int32_t G = 0;              // Gauss points per element side; 0 = nodal rule
    int64_t ngrid_total = 0;
    float* pixf = nullptr;      // FP32 pixel blocks (Bx, By, Bz planes per block), FP32C only
    double* xyz = nullptr;
    Geo geo{};
    void* geo_block = nullptr;  // one allocation holding every geometry array
    int32_t* near_ptr = nullptr;   // adjoint near lists (FP32C): CSR by global grid-point index
    int32_t* near_pts = nullptr;
    int32_t* pix_bnd = nullptr;
    int64_t near_pairs = 0;
    void* vjp_dev = nullptr;    // the adjoint's tile lists and point segments (VjpTables)
    VjpTables vjp{};
    int32_t* perm = nullptr;    // FP32C point order (NULL = identity): per magnetogram, the points
                                // with near-field pairs first, sorted by their window, then the rest
    Tile* tiles64 = nullptr;
    int64_t n_tiles64 = 0;
    Tile* tiles32 = nullptr;     // static schedule of the plain FP32C pass
    int64_t n_tiles32 = 0;
    Tile* tiles32t = nullptr;    // static schedule of the FP32C pass with mu-tangents
    int64_t n_tiles32t = 0;
    std::vector<Tile> tiles32_h, tiles32t_h;   // host copies of the two FP32C schedules
    int32_t split_tuned = 0;     // pixel slices chosen by the tuner (0: none)
    int32_t tuned = 0;           // 0 untuned, 1 timed at init, 2 from this process's cache, 3 from the file
    // untuned shapes: four-wave workgroups (at three resident waves per SIMD, the register count
    // of both nodal FP32C forms, eight-wave workgroups leave a third of the slots empty)
    F32Shape shape{1, 4, kRows * kCols, 0};
    F32Shape shape_tan{1, 4, kRows * kCols, 0};
    int32_t* work = nullptr;    // tile counter of the persistent FP32C form
    int32_t split = 1;          // FP32C pixel slices per launch (grid z); acc holds split x L slices
    int32_t cus = 256;          // compute units of the device
    double* acc = nullptr;      // [split][L][kAcc][N]
    double* noalloc_acc = nullptr;  // this device's static `scratch` (dbie_eval_field_noalloc)
    int64_t acc_L = 0;          // slices x trials the accumulator holds
    bool acc_owned = true;      // false: it lies in the caller's workspace
    char* ws = nullptr;         // caller-owned workspace (dbie_set_workspace), or NULL
    int64_t ws_bytes = 0;
    size_t ws_off[kWsRegions] = {}, ws_size[kWsRegions] = {};
    SolverState solver{};
    void* scratch[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t scratch_bytes[4] = {0, 0, 0, 0};
    bool trace = false;
    std::vector<hipEvent_t> trace_ev;   // solve tracing: start, then one per round
    hipEvent_t trace_end = nullptr;     // end of the traced solve
    // timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<hipEvent_t> ev_pool;
    std::string err;
};

namespace {

int fail(dbie_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_init_error = msg;
    return code;
}

int hip_fail(dbie_ctx* c, hipError_t e, const char* where) {
    return fail(c, DBIE_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define DBIE_HIP(c, call)                                  \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
    } while (0)

// Tiles of per_tile consecutive points of one boundary. With `cost` (pixels per boundary) the tiles
// are ordered by decreasing work (points x pixels; ties by position), so that the workgroups
// dispatched last are the cheapest ones.
std::vector<Tile> build_schedule(const std::vector<int64_t>& seg, int32_t per_tile,
                                 const std::vector<int64_t>* cost = nullptr) {
    std::vector<Tile> t;
    for (size_t b = 0; b + 1 < seg.size(); ++b) {
        for (int64_t s = seg[b]; s < seg[b + 1]; s += per_tile) {
            Tile x;
            x.start = s;
            x.count = (int32_t)std::min<int64_t>(per_tile, seg[b + 1] - s);
            x.b = (int32_t)b;
            t.push_back(x);
        }
    }
    if (cost)
        std::stable_sort(t.begin(), t.end(), [&](const Tile& x, const Tile& y) {
            return (int64_t)x.count * (*cost)[x.b] > (int64_t)y.count * (*cost)[y.b];
        });
    while (t.size() % 8 != 0 || t.empty()) t.push_back(Tile{0, 0, 0});
    return t;
}

hipEvent_t pool_event(dbie_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void free_ctx(dbie_ctx* c) {
    if (!c) return;
    (void)hipFree(c->bnd_d);
    (void)hipFree(c->B0d);
    (void)hipFree(c->gpos);
    if (c->gB != c->B0d) (void)hipFree(c->gB);
    (void)hipFree(c->qlw);
    (void)hipFree(c->gposf);
    (void)hipFree(c->pixf);
    (void)hipFree(c->xyz);
    (void)hipFree(c->geo_block);
    (void)hipFree(c->perm);
    (void)hipFree(c->near_ptr);
    (void)hipFree(c->near_pts);
    (void)hipFree(c->pix_bnd);
    (void)hipFree(c->vjp_dev);
    (void)hipFree(c->tiles64);
    (void)hipFree(c->tiles32);
    (void)hipFree(c->tiles32t);
    (void)hipFree(c->work);
    if (c->acc_owned) (void)hipFree(c->acc);
    solver_free(c->solver);
    for (int k = 0; k < 4; ++k) (void)hipFree(c->scratch[k]);
    for (auto e : c->trace_ev) (void)hipEventDestroy(e);
    if (c->trace_end) (void)hipEventDestroy(c->trace_end);
    for (auto& p : c->ev) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

int set_tiles32(dbie_ctx* c, F32Shape s, bool tan) {
    const int32_t per = s.ppl * s.waves * 64;
    std::vector<int64_t> cost;
    for (const BoundaryDev& b : c->bnd_h) cost.push_back((int64_t)b.ntx * b.nty);
    std::vector<Tile> t = build_schedule(c->seg, per, &cost);
    Tile* d = nullptr;
    DBIE_HIP(c, dalloc(&d, t.size()));
    DBIE_HIP(c, hipMemcpy(d, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice));
    Tile*& dst = tan ? c->tiles32t : c->tiles32;
    (void)hipFree(dst);
    dst = d;
    (tan ? c->n_tiles32t : c->n_tiles32) = (int64_t)t.size();
    (tan ? c->shape_tan : c->shape) = s;
    (tan ? c->tiles32t_h : c->tiles32_h) = std::move(t);
    // Pixel slices: enough workgroups for about four per compute unit when the point tiles alone
    // are fewer (few points: late solver rounds, field-line seeds), else one; or the caller's or the
    // tuner's choice.
    if (c->opt.pixel_split > 0) {
        c->split = c->opt.pixel_split;
    } else if (c->split_tuned > 0) {
        c->split = c->split_tuned;
    } else {
        const int64_t nt = std::max<int64_t>(1, std::min(c->n_tiles32 > 0 ? c->n_tiles32 : INT64_MAX,
                                                         c->n_tiles32t > 0 ? c->n_tiles32t : INT64_MAX));
        const int64_t want = 4 * (int64_t)c->cus;
        c->split = (int32_t)std::min<int64_t>(kMaxSplit, std::max<int64_t>(1, (want + nt - 1) / nt));
    }
    return DBIE_OK;
}

}  // namespace

namespace dbie {

int ensure_acc(dbie_ctx* c, int64_t L) { return ensure_acc_slices(c, L * c->split); }

// room for `need` partial-sum slices of [kAcc][N] (trials x pixel slices)
int ensure_acc_slices(dbie_ctx* c, int64_t need) {
    if (c->acc && c->acc_L >= need) return DBIE_OK;
    if (c->ws) {
        const size_t per = (size_t)kAcc * std::max<int64_t>(c->N, 1) * sizeof(double);
        void* r = ctx_ws_region(c, kWsAcc, (size_t)need * per);
        if (r == kWsTooSmall)
            return fail(c, DBIE_E_WORKSPACE, "the caller's workspace holds the sums of one trial per call");
        c->acc = (double*)r;
        c->acc_L = (int64_t)(c->ws_size[kWsAcc] / per);
        c->acc_owned = false;
        return DBIE_OK;
    }
    if (c->acc_owned) (void)hipFree(c->acc);
    c->acc = nullptr;
    c->acc_L = 0;
    c->acc_owned = true;
    hipError_t e = dalloc(&c->acc, (size_t)(need * kAcc * std::max<int64_t>(c->N, 1)));
    if (e != hipSuccess) return fail(c, DBIE_E_WORKSPACE, "cannot allocate the accumulator workspace");
    c->acc_L = need;
    return DBIE_OK;
}

// Pixel slices for an evaluation of about n points: about four workgroups per compute unit, at
// most kMaxSplit, and no more than the accumulator holds (a caller's workspace) or than 256 MB of
// partial sums allow.
int32_t split_for_points(dbie_ctx* c, int64_t n) {
    const int64_t tiles = std::max<int64_t>(1, (n + 255) / 256);
    int64_t S = std::min<int64_t>(kMaxSplit, (4 * (int64_t)c->cus + tiles - 1) / tiles);
    const int64_t per = (int64_t)kAcc * std::max<int64_t>(c->N, 1) * (int64_t)sizeof(double);
    const int64_t cap = c->ws ? (int64_t)c->ws_size[kWsAcc] / per : std::max<int64_t>(c->acc_L, (256ll << 20) / per);
    return (int32_t)std::max<int64_t>(1, std::min(S, cap));
}

// Bulk sum + finalize for L trials on the given lambda; the building block of every call. S > 0
// overrides the context's pixel slices. acc_in != NULL: partial sums there (room for L x S slices,
// checked by the caller) instead of the context's accumulator, and no timing events.
static int eval_core(dbie_ctx* c, const double* lam, int32_t L, bool fp64, bool tan, const EvalSet* set,
                     double* B, double* dB, double* fg, double* tn, hipStream_t s, bool scalar = false,
                     int32_t S = 0, double* acc_in = nullptr) {
    if (S <= 0) S = c->split;
    double* acc = acc_in;
    if (!acc) {
        int rc = ensure_acc_slices(c, (int64_t)L * S);
        if (rc) return rc;
        acc = c->acc;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing && !acc_in) {
        e0 = pool_event(c);
        e1 = pool_event(c);
        if (e0 && e1) DBIE_HIP(c, hipEventRecord(e0, s));
    }
    const int32_t* idx = set ? set->idx : nullptr;
    if (fp64)
        DBIE_HIP(c, launch_field64(set ? set->tiles64 : c->tiles64, set ? set->n_tiles64 : c->n_tiles64,
                                   c->bnd_d, c->gpos, c->gB, c->geo, lam, c->N, L, S, idx, tan, acc, s));
    else
        DBIE_HIP(c, launch_field32c(set ? set->tiles32 : (tan ? c->tiles32t : c->tiles32),
                                    set ? set->n_tiles32 : (tan ? c->n_tiles32t : c->n_tiles32), c->bnd_d,
                                    c->pixf, c->gposf, c->geo, lam, c->N, L, S, set ? idx : c->perm, c->work, tan,
                                    scalar, tan ? c->shape_tan : c->shape, acc, s));
    if (e0 && e1) {
        DBIE_HIP(c, hipEventRecord(e1, s));
        c->ev.emplace_back(e0, e1);
    }
    // points beyond the FP32 phase bound: their sums again in FP64, in every evaluation whose results
    // the library returns; a solve's rounds (an active set) only steer its search, which the FP64
    // acceptance and the final evaluation check, and skip it
    if (!fp64 && !set)
        DBIE_HIP(c, launch_field64_override(c->tiles64, c->n_tiles64, c->bnd_d, c->B0d, c->gpos, c->gB, c->geo, lam,
                                            c->N, L, S, idx, tan, tan ? kFp32cPhaseMaxTan : kFp32cPhaseMax, acc, s));
    const bool near = !fp64 && c->opt.nearfield_radius_h > 0.0;
    DBIE_HIP(c, launch_finalize(c->bnd_d, c->B0d, c->gpos, c->gB, c->geo, lam, idx, c->N,
                                set ? set->n_dev : nullptr, c->N,
                                L, S, acc, near, tan, c->opt.dv_over_dsigma_h, B, dB, fg, tn, s));
    return DBIE_OK;
}

int eval_set(dbie_ctx* c, const double* lam, bool fp64, bool tan, const EvalSet* set, double* B, double* dB,
             double* fg, double* tn, hipStream_t s, int32_t S) {
    if (fp64 == false && !c->pixf) return fail(c, DBIE_E_UNSUPPORTED, "FP32C evaluation in an FP64 context");
    return eval_core(c, lam, 1, fp64, tan, set, B, dB, fg, tn, s, false, S);
}

const Geo& ctx_geo(const dbie_ctx* c) { return c->geo; }
const BoundaryDev* ctx_bnd(const dbie_ctx* c) { return c->bnd_d; }
const BoundaryDev& ctx_bnd_host(const dbie_ctx* c, int b) { return c->bnd_h[b]; }
int64_t ctx_n(const dbie_ctx* c) { return c->N; }
const int32_t* ctx_perm(const dbie_ctx* c) { return c->perm; }
const int64_t* ctx_seg(const dbie_ctx* c) { return c->seg.data(); }
void* const kWsTooSmall = (void*)&kWsTooSmall;

void* ctx_ws_region(dbie_ctx* c, int region, size_t bytes) {
    if (!c->ws) return nullptr;
    if (region < 0 || region >= kWsRegions || bytes > c->ws_size[region]) return kWsTooSmall;
    return c->ws + c->ws_off[region];
}

void* ctx_scratch(dbie_ctx* c, int slot, size_t bytes) {
    if (slot < 0 || slot >= 4) return nullptr;
    if (c->ws) {
        void* r = ctx_ws_region(c, kWsSlot0 + slot, bytes);
        return r == kWsTooSmall ? nullptr : r;
    }
    if (c->scratch[slot] && c->scratch_bytes[slot] >= bytes) return c->scratch[slot];
    (void)hipFree(c->scratch[slot]);
    c->scratch[slot] = nullptr;
    c->scratch_bytes[slot] = 0;
    if (hipMalloc(&c->scratch[slot], std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
    c->scratch_bytes[slot] = bytes;
    return c->scratch[slot];
}
bool solver_tracing(const dbie_ctx* c) { return c->trace; }
NearLists ctx_near_lists(const dbie_ctx* c) {
    return NearLists{c->ngrid_total, c->near_pairs, c->near_ptr, c->near_pts, c->pix_bnd};
}
bool ctx_timing(const dbie_ctx* c) { return c->timing; }
std::vector<hipEvent_t>& solver_trace_events(dbie_ctx* c) { return c->trace_ev; }
hipEvent_t& solver_trace_end(dbie_ctx* c) { return c->trace_end; }
void solver_forget_last(dbie_ctx* c) {
    for (auto e : c->trace_ev) (void)hipEventDestroy(e);
    c->trace_ev.clear();
    if (c->trace_end) (void)hipEventDestroy(c->trace_end);
    c->trace_end = nullptr;
    c->solver.last_conv = nullptr;
    c->solver.last_rounds = 0;
}
int32_t ctx_nb(const dbie_ctx* c) { return c->nb; }
const double* ctx_B0d(const dbie_ctx* c) { return c->B0d; }
VjpTables ctx_vjp_tables(const dbie_ctx* c) { return c->vjp; }
QuadGrid ctx_grid(const dbie_ctx* c) { return QuadGrid{c->gpos, c->gB, c->qlw, c->G, c->ngrid_total, c->gposf}; }
int ctx_precision(const dbie_ctx* c) { return c->opt.precision; }
double ctx_dvds(const dbie_ctx* c) { return c->opt.dv_over_dsigma_h; }
SolverState& ctx_solver(dbie_ctx* c) { return c->solver; }
int ctx_fail(dbie_ctx* c, int code, const char* msg) { return fail(c, code, msg); }
int ctx_check_device(dbie_ctx* c) {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess || d != c->device)
        return fail(c, DBIE_E_INVAL, "the current HIP device is not the one the context was created on");
    return DBIE_OK;
}
double* ctx_xyz(dbie_ctx* c) { return c->xyz; }
const void* ctx_acc(const dbie_ctx* c) { return c->acc; }
int32_t ctx_split(const dbie_ctx* c) { return c->split; }

// Regions of a caller-owned workspace, each a multiple of 256 bytes: the sums of one trial (all
// pixel slices), the solver block (any method, up to 1e6 trials, any tile shape), and scratch slots
// 0 (dbie_grad's evaluation, dbie_trace_lines), 1 (dbie_grad's gB0 part), 2 (dbie_residual_stats;
// tuning uses it in dbie_init only) and 3 (the expanded lambda of one single-lambda trial).
void ws_sizes(const dbie_ctx* c, size_t sz[kWsRegions]) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t n = (size_t)std::max<int64_t>(c->N, 1);
    sz[kWsAcc] = up((size_t)kAcc * n * (size_t)c->split * sizeof(double));
    sz[kWsSolver] = up(solver_workspace_bytes(c));
    sz[kWsSlot0 + 0] = up(std::max(24 * n * sizeof(double), 27 * n * sizeof(double) + (2 * n + 64) * sizeof(int32_t)));
    sz[kWsSlot0 + 1] = up(grad_workspace_bytes(c));
    sz[kWsSlot0 + 2] = up((4 + 4 * 256) * sizeof(double));   // residual statistics (tuning uses it at init)
    sz[kWsSlot0 + 3] = up(3 * n * sizeof(double));
}
hipError_t ctx_prep_points(dbie_ctx* c, int32_t* flag, hipStream_t s) {
    const double r = (c->opt.precision == DBIE_FP32C) ? c->opt.nearfield_radius_h : 0.0;
    return launch_prep(c->tiles64, c->n_tiles64, c->bnd_d, c->gB, c->xyz, c->N, c->geo, r * r, 1, flag, nullptr,
                       c->bnd_h.data(), c->nb, s);
}

}  // namespace dbie

extern "C" {

int dbie_default_options(dbie_options* o) {
    if (!o) return DBIE_E_INVAL;
    o->precision = DBIE_FP32C;
    o->nearfield_radius_h = 2.0;
    o->dv_over_dsigma_h = 1.0 / 6.0;
    o->tune = 0;
    o->tune_cache = nullptr;
    o->quad_points = 0;
    o->pixel_split = 0;
    return DBIE_OK;
}

int dbie_default_solve_opts(dbie_solve_opts* o) {
    if (!o) return DBIE_E_INVAL;
    o->method = DBIE_NELDER_MEAD;
    o->max_trials = 50;
    o->eps = 1e-4;
    o->init_step = 0.0;
    o->lambda_cap = 0.0;
    o->fp64_accept = 1;
    o->use_graph = 1;
    o->lm_radius = 0.0;
    o->lm_damping = 0.0;
    return DBIE_OK;
}

int dbie_init(dbie_ctx** out, const dbie_problem* prob, const dbie_options* opt, void* stream) {
    if (!out) return fail(nullptr, DBIE_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!prob) return fail(nullptr, DBIE_E_INVAL, "problem is NULL");
    dbie_options o;
    dbie_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != DBIE_FP64 && o.precision != DBIE_FP32C)
        return fail(nullptr, DBIE_E_INVAL, "precision must be DBIE_FP64 or DBIE_FP32C");
    if (!(o.nearfield_radius_h >= 0.0 && o.nearfield_radius_h <= 2.0))
        return fail(nullptr, DBIE_E_INVAL, "nearfield_radius_h must lie in [0, 2]");
    if (!(o.dv_over_dsigma_h > 0.0) || !std::isfinite(o.dv_over_dsigma_h))
        return fail(nullptr, DBIE_E_INVAL, "dv_over_dsigma_h must be positive and finite");
    if (o.pixel_split < 0 || o.pixel_split > kMaxSplit)
        return fail(nullptr, DBIE_E_INVAL, "pixel_split must lie in [0, 32]");
    if (o.quad_points != 0 && (o.quad_points < 2 || o.quad_points > 4))
        return fail(nullptr, DBIE_E_INVAL, "quad_points must be 0 (nodal sum) or 2, 3, 4 (9-node elements)");
    const int32_t nb = prob->n_boundaries;
    if (nb < 1 || !prob->boundaries) return fail(nullptr, DBIE_E_INVAL, "need at least one boundary");
    if (prob->n_points < 0) return fail(nullptr, DBIE_E_INVAL, "n_points < 0");
    if (prob->n_points > ((int64_t)1 << 31) - 1)
        return fail(nullptr, DBIE_E_INVAL, "n_points exceeds 2^31 - 1");
    if (prob->n_points > 0 && !prob->xyz) return fail(nullptr, DBIE_E_INVAL, "xyz is NULL");
    if (nb > 1 && !prob->seg) return fail(nullptr, DBIE_E_INVAL, "seg is required when n_boundaries > 1");
    std::vector<int64_t> seg(nb + 1);
    if (prob->seg) {
        for (int32_t b = 0; b <= nb; ++b) seg[b] = prob->seg[b];
        if (seg[0] != 0 || seg[nb] != prob->n_points)
            return fail(nullptr, DBIE_E_INVAL, "seg must start at 0 and end at n_points");
        for (int32_t b = 0; b < nb; ++b)
            if (seg[b + 1] < seg[b]) return fail(nullptr, DBIE_E_INVAL, "seg is not non-decreasing");
    } else {
        seg[0] = 0;
        seg[1] = prob->n_points;
    }
    for (int32_t b = 0; b < nb; ++b) {
        const dbie_boundary& bd = prob->boundaries[b];
        if (bd.nx < 1 || bd.ny < 1) return fail(nullptr, DBIE_E_INVAL, "boundary with nx or ny < 1");
        if ((int64_t)bd.nx * bd.ny > ((int64_t)1 << 30))
            return fail(nullptr, DBIE_E_INVAL, "boundary larger than 2^30 pixels");
        if (!(bd.h > 0.0) || !std::isfinite(bd.h) || !std::isfinite(bd.x0) || !std::isfinite(bd.y0))
            return fail(nullptr, DBIE_E_INVAL, "boundary h must be positive; x0, y0, h finite");
        if (!bd.B0) return fail(nullptr, DBIE_E_INVAL, "boundary B0 is NULL");
        if (o.quad_points && (bd.nx < 3 || bd.ny < 3 || bd.nx % 2 == 0 || bd.ny % 2 == 0))
            return fail(nullptr, DBIE_E_INVAL, "9-node elements need odd nx, ny >= 3");
    }

    dbie_ctx* c = new dbie_ctx();
    c->opt = o;
    c->opt.tune_cache = nullptr;
    c->nb = nb;
    c->N = prob->n_points;
    c->seg = seg;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetDevice(&c->device);
    {
        void* p = nullptr;
        const hipError_t e = noalloc_scratch(c->device, &p);
        if (e != hipSuccess) {
            free_ctx(c);
            return fail(nullptr, DBIE_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        c->noalloc_acc = (double*)p;
    }
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && cus > 0)
            c->cus = cus;
    }
    int64_t off = 0, offf = 0, goff = 0, gpoff = 0;
    const int G = o.quad_points;
    c->G = G;
    double xg[4], wg[4];
    if (G) gauss_legendre(G, xg, wg);
    std::vector<double> gpos_h;
    std::vector<float> gposf_h;
    for (int32_t b = 0; b < nb; ++b) {
        const dbie_boundary& bd = prob->boundaries[b];
        BoundaryDev d{};
        d.nx = bd.nx;
        d.ny = bd.ny;
        d.npix = bd.nx * bd.ny;
        d.pix_off = off;
        d.pixf_off = offf;
        d.x0 = bd.x0;
        d.y0 = bd.y0;
        d.h = bd.h;
        d.G = G;
        if (G) {
            d.gcols = G * (bd.nx - 1) / 2;
            d.grows = G * (bd.ny - 1) / 2;
            d.gpl_off = goff;
            goff += 3 * (int64_t)d.gcols * d.grows;
        } else {
            d.gcols = bd.nx;
            d.grows = bd.ny;
            d.gpl_off = off;
        }
        // the FP32C blocks tile the quadrature grid (the pixels for the nodal rule)
        d.ntx = (d.gcols + kCols - 1) / kCols;
        d.nty = (d.grows + kRows - 1) / kRows;
        d.npix_pad = d.ntx * d.nty * kRows * kCols;
        d.gpos_off = gpoff;
        gpoff += d.gcols + d.grows;
        // grid positions in pixels from node (0, 0): the nodes, or the Gauss points 2m + 1 + xi_g
        for (int axis = 0; axis < 2; ++axis) {
            const int32_t n = axis ? d.grows : d.gcols;
            for (int32_t k = 0; k < n; ++k)
                gpos_h.push_back(G ? (double)(2 * (k / G) + 1) + xg[k % G] : (double)k);
        }
        if (G && o.precision == DBIE_FP32C) {
            // split FP32 positions of the padded columns and rows; padding repeats the last point
            d.gposf_off = (int64_t)gposf_h.size() / 4;
            for (int axis = 0; axis < 2; ++axis) {
                const int32_t n = axis ? d.grows : d.gcols, npad = axis ? d.nty * kRows : d.ntx * kCols;
                for (int32_t k = 0; k < npad; ++k) {
                    const int32_t kk = std::min(k, n - 1);
                    const double p = (double)(2 * (kk / G) + 1) + xg[kk % G];
                    const double fl = std::floor(p);
                    gposf_h.push_back((float)fl);
                    gposf_h.push_back((float)(p - fl));
                    gposf_h.push_back((float)(kk / G));
                    gposf_h.push_back(0.0f);
                }
            }
        }
        off += 3 * (int64_t)d.npix;
        offf += 3 * (int64_t)d.npix_pad;
        c->bnd_h.push_back(d);
    }
    c->npix_total = off / 3;
    c->ngrid_total = G ? goff / 3 : off / 3;
    auto bail = [&](int rc) {
        std::string m = c->err;
        free_ctx(c);
        g_init_error = m;
        return rc;
    };
    int rc;
#define DBIE_INIT_HIP(call)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return bail(hip_fail(c, e_, #call)); \
    } while (0)
    DBIE_INIT_HIP(dalloc(&c->bnd_d, nb));
    DBIE_INIT_HIP(hipMemcpy(c->bnd_d, c->bnd_h.data(), nb * sizeof(BoundaryDev), hipMemcpyHostToDevice));
    DBIE_INIT_HIP(dalloc(&c->B0d, (size_t)off));
    for (int32_t b = 0; b < nb; ++b)
        DBIE_INIT_HIP(hipMemcpyAsync(c->B0d + c->bnd_h[b].pix_off, prob->boundaries[b].B0,
                                     3 * (size_t)c->bnd_h[b].npix * sizeof(double),
                                     hipMemcpyDeviceToDevice, s));
    DBIE_INIT_HIP(dalloc(&c->gpos, gpos_h.size()));
    DBIE_INIT_HIP(hipMemcpy(c->gpos, gpos_h.data(), gpos_h.size() * sizeof(double), hipMemcpyHostToDevice));
    if (G) {
        // weighted field at the Gauss points: w_g w_q sum_ab L_a(xi_g) L_b(xi_q) B0(node)
        double lw[12];
        for (int g = 0; g < G; ++g) {
            const double x = xg[g];
            lw[3 * g + 0] = wg[g] * 0.5 * x * (x - 1.0);
            lw[3 * g + 1] = wg[g] * (1.0 - x) * (1.0 + x);
            lw[3 * g + 2] = wg[g] * 0.5 * x * (x + 1.0);
        }
        DBIE_INIT_HIP(dalloc(&c->qlw, 3 * (size_t)G));
        DBIE_INIT_HIP(hipMemcpy(c->qlw, lw, 3 * (size_t)G * sizeof(double), hipMemcpyHostToDevice));
        DBIE_INIT_HIP(dalloc(&c->gB, (size_t)goff));
        for (int32_t b = 0; b < nb; ++b)
            DBIE_INIT_HIP(launch_quad_weights(c->bnd_h[b], c->B0d, c->qlw, G, c->gB, s));
    } else {
        c->gB = c->B0d;
    }
    if (!gposf_h.empty()) {
        DBIE_INIT_HIP(dalloc(&c->gposf, gposf_h.size() / 4));
        DBIE_INIT_HIP(hipMemcpy(c->gposf, gposf_h.data(), gposf_h.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    if (o.precision == DBIE_FP32C) {
        DBIE_INIT_HIP(dalloc(&c->pixf, (size_t)offf));
        DBIE_INIT_HIP(dalloc(&c->work, 1));
    }
    const int64_t N = c->N;
    const size_t Nn = (size_t)std::max<int64_t>(N, 1);
    DBIE_INIT_HIP(dalloc(&c->xyz, 3 * Nn));
    if (N > 0)
        DBIE_INIT_HIP(hipMemcpyAsync(c->xyz, prob->xyz, 3 * (size_t)N * sizeof(double),
                                     hipMemcpyDeviceToDevice, s));
    // geometry: 3 double + 5 float + 4 int arrays of N, each 256-byte aligned
    const size_t al = 256;
    auto up = [&](size_t b) { return (b + al - 1) / al * al; };
    const size_t szd = up(Nn * 8), szf = up(Nn * 4);
    DBIE_INIT_HIP(hipMalloc(&c->geo_block, 3 * szd + 9 * szf));
    char* gp = (char*)c->geo_block;
    c->geo.u = (double*)gp; gp += szd;
    c->geo.v = (double*)gp; gp += szd;
    c->geo.w = (double*)gp; gp += szd;
    c->geo.xi_int = (float*)gp; gp += szf;
    c->geo.xi_frac = (float*)gp; gp += szf;
    c->geo.yi_int = (float*)gp; gp += szf;
    c->geo.yi_frac = (float*)gp; gp += szf;
    c->geo.wf = (float*)gp; gp += szf;
    c->geo.win_a = (int32_t*)gp; gp += szf;
    c->geo.win_b = (int32_t*)gp; gp += szf;
    c->geo.near_mask = (uint32_t*)gp; gp += szf;
    c->geo.bidx = (int32_t*)gp; gp += szf;
    {
        std::vector<Tile> t = build_schedule(seg, kTile64);
        DBIE_INIT_HIP(dalloc(&c->tiles64, t.size()));
        DBIE_INIT_HIP(hipMemcpy(c->tiles64, t.data(), t.size() * sizeof(Tile), hipMemcpyHostToDevice));
        c->n_tiles64 = (int64_t)t.size();
        if (o.precision == DBIE_FP64) {
            // pixel slices of the FP64 pass, as for FP32C: about four workgroups per compute unit
            int64_t busy = 0;
            for (const Tile& x : t) busy += x.count > 0;
            c->split = o.pixel_split > 0 ? o.pixel_split
                                         : (int32_t)std::min<int64_t>(kMaxSplit, std::max<int64_t>(1,
                                               (4 * (int64_t)c->cus + std::max<int64_t>(busy, 1) - 1) /
                                                   std::max<int64_t>(busy, 1)));
        }
    }
    DBIE_INIT_HIP(vjp_tables_init(c, &c->vjp_dev, &c->vjp));
    if (o.precision == DBIE_FP32C) {
        rc = set_tiles32(c, c->shape, false);
        if (!rc) rc = set_tiles32(c, c->shape_tan, true);
        if (rc) return bail(rc);
    }
    // the validation flag lives in a scratch slot, so that every exit path frees it with the context
    int32_t* bad = (int32_t*)ctx_scratch(c, 2, sizeof(int32_t));
    if (!bad) return bail(fail(c, DBIE_E_WORKSPACE, "cannot allocate the validation flag"));
    DBIE_INIT_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    const double r = (o.precision == DBIE_FP32C) ? o.nearfield_radius_h : 0.0;
    DBIE_INIT_HIP(launch_prep(c->tiles64, c->n_tiles64, c->bnd_d, c->gB, c->xyz, N, c->geo, r * r,
                              o.precision != DBIE_FP32C, bad, c->pixf, c->bnd_h.data(), nb, s));
    int32_t bad_h = 0;
    DBIE_INIT_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DBIE_INIT_HIP(hipStreamSynchronize(s));
    if (bad_h) return bail(fail(c, DBIE_E_INVAL, "a point has z <= 0, a non-finite coordinate, or lies "
                                                 "more than 4e6 pixels away"));
    if (o.precision == DBIE_FP32C && r > 0.0 && N > 0) {
        // Points with near-field pairs take the masked loop of the FP32C kernel for the pixel tiles
        // their window touches; grouping them (sorted by window) keeps that loop to few wavefronts.
        std::vector<uint32_t> mask(N);
        std::vector<int32_t> wa(N), wb(N);
        DBIE_INIT_HIP(hipMemcpy(mask.data(), c->geo.near_mask, N * sizeof(uint32_t), hipMemcpyDeviceToHost));
        DBIE_INIT_HIP(hipMemcpy(wa.data(), c->geo.win_a, N * sizeof(int32_t), hipMemcpyDeviceToHost));
        DBIE_INIT_HIP(hipMemcpy(wb.data(), c->geo.win_b, N * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::vector<int32_t> perm;
        perm.reserve(N);
        bool identity = true;
        for (int32_t b = 0; b < nb; ++b) {
            std::vector<int32_t> low, high;
            for (int64_t i = seg[b]; i < seg[b + 1]; ++i) (mask[i] ? low : high).push_back((int32_t)i);
            std::stable_sort(low.begin(), low.end(), [&](int32_t x, int32_t y) {
                return wb[x] != wb[y] ? wb[x] < wb[y] : wa[x] < wa[y];
            });
            for (int32_t i : low) perm.push_back(i);
            for (int32_t i : high) perm.push_back(i);
        }
        for (int64_t k = 0; k < N && identity; ++k) identity = perm[k] == (int32_t)k;
        if (!identity) {
            DBIE_INIT_HIP(dalloc(&c->perm, (size_t)N));
            DBIE_INIT_HIP(hipMemcpy(c->perm, perm.data(), N * sizeof(int32_t), hipMemcpyHostToDevice));
        }
        // the near pairs by grid point (pixel, or Gauss point of a 9-node element) for the adjoint
        // (counting sort by grid point; points ascending)
        const int64_t P = c->ngrid_total;
        std::vector<int64_t> ptr(P + 1, 0);
        std::vector<int32_t> pixb(P);
        for (int32_t b = 0; b < nb; ++b)
            for (int64_t k = 0; k < (int64_t)c->bnd_h[b].gcols * c->bnd_h[b].grows; ++k)
                pixb[c->bnd_h[b].gpl_off / 3 + k] = b;
        std::vector<int32_t> pbnd(N);
        for (int32_t b = 0; b < nb; ++b)
            for (int64_t i = seg[b]; i < seg[b + 1]; ++i) pbnd[i] = b;
        // calls f(global grid index) for every grid point of pair bit `bit` of point i
        auto for_pair = [&](int64_t i, int bit, auto&& f) {
            const BoundaryDev& bd = c->bnd_h[pbnd[i]];
            const int64_t base = bd.gpl_off / 3;
            if (G) {
                const int32_t m = wa[i] + bit % kNearSideQ - kNearWinQ, n = wb[i] + bit / kNearSideQ - kNearWinQ;
                for (int q = 0; q < G; ++q)
                    for (int g = 0; g < G; ++g) f(base + (int64_t)(G * n + q) * bd.gcols + G * m + g);
            } else {
                const int32_t pa = wa[i] + bit % kNearSide - kNearWin, pb = wb[i] + bit / kNearSide - kNearWin;
                f(base + (int64_t)pb * bd.nx + pa);
            }
        };
        for (int64_t i = 0; i < N; ++i)
            for (uint32_t m = mask[i]; m; m &= m - 1u) for_pair(i, __builtin_ctz(m), [&](int64_t g) { ++ptr[g + 1]; });
        for (int64_t g = 0; g < P; ++g) ptr[g + 1] += ptr[g];
        c->near_pairs = ptr[P];
        if (c->near_pairs > ((int64_t)1 << 31) - 1)
            return bail(fail(c, DBIE_E_UNSUPPORTED, "more than 2^31 - 1 near-field pairs"));
        if (c->near_pairs > 0) {
            std::vector<int32_t> ptr32(ptr.begin(), ptr.end());
            std::vector<int32_t> fill(ptr32.begin(), ptr32.end() - 1), pts(c->near_pairs);
            for (int64_t i = 0; i < N; ++i)
                for (uint32_t m = mask[i]; m; m &= m - 1u)
                    for_pair(i, __builtin_ctz(m), [&](int64_t g) { pts[fill[g]++] = (int32_t)i; });
            DBIE_INIT_HIP(dalloc(&c->near_ptr, (size_t)P + 1));
            DBIE_INIT_HIP(dalloc(&c->near_pts, (size_t)c->near_pairs));
            DBIE_INIT_HIP(dalloc(&c->pix_bnd, (size_t)P));
            DBIE_INIT_HIP(hipMemcpy(c->near_ptr, ptr32.data(), (P + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
            DBIE_INIT_HIP(hipMemcpy(c->near_pts, pts.data(), c->near_pairs * sizeof(int32_t), hipMemcpyHostToDevice));
            DBIE_INIT_HIP(hipMemcpy(c->pix_bnd, pixb.data(), P * sizeof(int32_t), hipMemcpyHostToDevice));
        }
    }
    if (o.precision == DBIE_FP32C && o.tune) {
        rc = tune_shapes(c, opt ? opt->tune_cache : nullptr, s);
        if (rc) return bail(rc);
        // the tuning lambda (3 doubles per point) is not kept: later calls size these slots
        DBIE_INIT_HIP(hipStreamSynchronize(s));
        for (int k = 2; k < 4; ++k) {
            DBIE_INIT_HIP(hipFree(c->scratch[k]));
            c->scratch[k] = nullptr;
            c->scratch_bytes[k] = 0;
        }
    }
    *out = c;
    return DBIE_OK;
#undef DBIE_INIT_HIP
}

int dbie_eval_field(dbie_ctx* c, const double* lambda, int32_t L, double* B, double* dB, double* fg,
                    double* tan, void* stream) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    if (L < 1) return fail(c, DBIE_E_INVAL, "L must be >= 1");
    if (c->N > 0 && (!lambda || !B)) return fail(c, DBIE_E_INVAL, "lambda and B are required");
    if ((int64_t)L * c->N > ((int64_t)1 << 31) - 1)
        return fail(c, DBIE_E_INVAL, "L * n_points exceeds 2^31 - 1");
    if (int rc = ctx_check_device(c)) return rc;
    if (c->N == 0) return DBIE_OK;
    return eval_core(c, lambda, L, c->opt.precision == DBIE_FP64, tan != nullptr, nullptr, B, dB, fg, tan,
                     (hipStream_t)stream);
}

int dbie_eval_field_noalloc(dbie_ctx* c, const double* lambda, int32_t L, double* B, double* dB, double* fg,
                            double* tan, void* stream) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    if (L < 1) return fail(c, DBIE_E_INVAL, "L must be >= 1");
    if (c->N > 0 && (!lambda || !B)) return fail(c, DBIE_E_INVAL, "lambda and B are required");
    if (int rc = ctx_check_device(c)) return rc;
    if (c->N == 0) return DBIE_OK;
    // pixel slices: the context's, or as many as the static array holds for L trials
    const int64_t slice = (int64_t)kAcc * c->N * (int64_t)sizeof(double);
    const int64_t fit = (int64_t)kNoAllocBytes / slice / L;
    if (fit < 1) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "dbie_eval_field_noalloc: L * n_points = %lld exceeds %lld (%d MiB of static "
                      "work memory, %d doubles per point and trial)", (long long)L * c->N,
                      (long long)(kNoAllocBytes / (kAcc * sizeof(double))), (int)(kNoAllocBytes >> 20), kAcc);
        return fail(c, DBIE_E_INVAL, msg);
    }
    const int32_t S = (int32_t)std::min<int64_t>(c->split, fit);
    return eval_core(c, lambda, L, c->opt.precision == DBIE_FP64, tan != nullptr, nullptr, B, dB, fg, tan,
                     (hipStream_t)stream, false, S, c->noalloc_acc);
}

int dbie_eval_field_scalar(dbie_ctx* c, const double* lambda, int32_t L, double* B, double* dB, double* fg,
                           double* tan, void* stream) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    if (L < 1) return fail(c, DBIE_E_INVAL, "L must be >= 1");
    if (c->N > 0 && (!lambda || !B)) return fail(c, DBIE_E_INVAL, "lambda and B are required");
    if ((int64_t)L * c->N > ((int64_t)1 << 31) - 1)
        return fail(c, DBIE_E_INVAL, "L * n_points exceeds 2^31 - 1");
    if (int rc = ctx_check_device(c)) return rc;
    if (c->N == 0) return DBIE_OK;
    hipStream_t s = (hipStream_t)stream;
    double* lam3 = (double*)ctx_scratch(c, 3, (size_t)L * 3 * c->N * sizeof(double));
    if (!lam3) return fail(c, DBIE_E_WORKSPACE, "cannot allocate the lambda workspace");
    DBIE_HIP(c, launch_expand_scalar(lambda, L, c->N, lam3, s));
    return eval_core(c, lam3, L, c->opt.precision == DBIE_FP64, tan != nullptr, nullptr, B, dB, fg, tan, s, true);
}

int dbie_timing(dbie_ctx* c, int32_t enable) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    c->timing = enable != 0;
    return DBIE_OK;
}

int dbie_timing_read(dbie_ctx* c, double* total_ms, int64_t* launches) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    double tot = 0.0;
    for (auto& p : c->ev) {
        DBIE_HIP(c, hipEventSynchronize(p.second));
        float ms = 0.0f;
        DBIE_HIP(c, hipEventElapsedTime(&ms, p.first, p.second));
        tot += ms;
        c->ev_pool.push_back(p.first);
        c->ev_pool.push_back(p.second);
    }
    if (launches) *launches = (int64_t)c->ev.size();
    c->ev.clear();
    if (total_ms) *total_ms = tot;
    return DBIE_OK;
}

int dbie_query(const dbie_ctx* c, int64_t* n_points, int64_t* n_pixels, int32_t* ppl, int32_t* waves,
               int32_t* tile_pixels) {
    // (the shape of the plain pass; the pass with tangents is reported by dbie_query_tan)
    if (!c) return DBIE_E_INVAL;
    if (n_points) *n_points = c->N;
    if (n_pixels) *n_pixels = c->npix_total;
    if (ppl) *ppl = c->shape.ppl;
    if (waves) *waves = c->shape.waves;
    if (tile_pixels) *tile_pixels = c->shape.tp;
    return DBIE_OK;
}

int dbie_set_tile_shape(dbie_ctx* c, int32_t ppl, int32_t waves, int32_t tile_pixels, int32_t persistent) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    if (c->opt.precision != DBIE_FP32C) return fail(c, DBIE_E_UNSUPPORTED, "tile shapes apply to FP32C contexts");
    if (int rc = ctx_check_device(c)) return rc;
    const F32Shape sh{ppl, waves, tile_pixels, persistent};
    int rc = dbie::set_shape(c, sh, false);
    if (!rc) rc = dbie::set_shape(c, sh, true);
    return rc;
}

int dbie_query_tan(const dbie_ctx* c, int32_t* ppl, int32_t* waves, int32_t* tile_pixels) {
    if (!c) return DBIE_E_INVAL;
    // (whether either pass is persistent is reported by dbie_query_persistent)
    if (ppl) *ppl = c->shape_tan.ppl;
    if (waves) *waves = c->shape_tan.waves;
    if (tile_pixels) *tile_pixels = c->shape_tan.tp;
    return DBIE_OK;
}

int dbie_solve_trace(dbie_ctx* c, int32_t enable) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    c->trace = enable != 0;
    return DBIE_OK;
}

int dbie_solve_trace_read(dbie_ctx* c, double* t_ms, int32_t* converged, int32_t max_rounds,
                          int32_t* n_rounds, double* t_end_ms) {
    if (!c) return fail(nullptr, DBIE_E_INVAL, "ctx is NULL");
    if (max_rounds < 0) return fail(c, DBIE_E_INVAL, "max_rounds < 0");
    const int32_t n = (int32_t)c->trace_ev.size() - 1;   // the first event marks the start
    if (n_rounds) *n_rounds = std::max(n, 0);
    if (t_end_ms) *t_end_ms = 0.0;
    if (t_end_ms && c->trace_end && !c->trace_ev.empty()) {
        DBIE_HIP(c, hipEventSynchronize(c->trace_end));
        float ms = 0.0f;
        DBIE_HIP(c, hipEventElapsedTime(&ms, c->trace_ev[0], c->trace_end));
        *t_end_ms = ms;
    }
    if (n <= 0) return DBIE_OK;
    DBIE_HIP(c, hipEventSynchronize(c->trace_ev.back()));
    const int32_t m = std::min(n, max_rounds);
    for (int32_t r = 0; r < m; ++r) {
        float ms = 0.0f;
        DBIE_HIP(c, hipEventElapsedTime(&ms, c->trace_ev[0], c->trace_ev[r + 1]));
        if (t_ms) t_ms[r] = ms;
    }
    if (converged) {
        if (!c->solver.last_conv) return fail(c, DBIE_E_INVAL, "the last solve did not complete");
        DBIE_HIP(c, hipMemcpy(converged, c->solver.last_conv, m * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return DBIE_OK;
}

int dbie_query_persistent(const dbie_ctx* c, int32_t* plain, int32_t* with_tangents) {
    if (!c) return DBIE_E_INVAL;
    if (plain) *plain = c->shape.persist;
    if (with_tangents) *with_tangents = c->shape_tan.persist;
    return DBIE_OK;
}

int64_t dbie_workspace_bytes(const dbie_ctx* c) {
    if (!c) return DBIE_E_INVAL;
    size_t sz[kWsRegions];
    ws_sizes(c, sz);
    size_t t = 0;
    for (int r = 0; r < kWsRegions; ++r) t += sz[r];
    return (int64_t)t;
}

int dbie_set_workspace(dbie_ctx* c, void* dev, int64_t bytes) {
    if (!c) return DBIE_E_INVAL;
    if (dev && ((uintptr_t)dev % 256 != 0)) return fail(c, DBIE_E_INVAL, "workspace must be 256-byte aligned");
    size_t sz[kWsRegions];
    ws_sizes(c, sz);
    size_t total = 0;
    for (int r = 0; r < kWsRegions; ++r) total += sz[r];
    if (dev && bytes < (int64_t)total) return fail(c, DBIE_E_WORKSPACE, "workspace smaller than dbie_workspace_bytes");
    if (int rc = ctx_check_device(c)) return rc;
    // nothing may still use the buffers being given up
    DBIE_HIP(c, hipDeviceSynchronize());
    solver_forget_last(c);   // the per-round counts lie in the solver block given up here
    if (c->acc_owned) (void)hipFree(c->acc);
    c->acc = nullptr;
    c->acc_L = 0;
    c->acc_owned = true;
    for (int k = 0; k < 4; ++k) {
        if (!c->ws) (void)hipFree(c->scratch[k]);
        c->scratch[k] = nullptr;
        c->scratch_bytes[k] = 0;
    }
    SolverState& S = c->solver;
    if (S.exec) (void)hipGraphExecDestroy(S.exec);
    S.exec = nullptr;
    if (S.block_owned) (void)hipFree(S.block);
    S.block = nullptr;
    S.bytes = 0;
    S.block_owned = false;
    c->ws = (char*)dev;
    c->ws_bytes = dev ? bytes : 0;
    size_t off = 0;
    for (int r = 0; r < kWsRegions; ++r) {
        c->ws_off[r] = off;
        c->ws_size[r] = dev ? sz[r] : 0;
        off += sz[r];
    }
    return DBIE_OK;
}

int dbie_residual_stats(dbie_ctx* c, const double* fg, double eps, double* out, void* stream) {
    if (!c) return DBIE_E_INVAL;
    if (!out) return fail(c, DBIE_E_INVAL, "out is NULL");
    if (!(eps >= 0.0)) return fail(c, DBIE_E_INVAL, "eps must be >= 0");
    if (c->N > 0 && !fg) return fail(c, DBIE_E_INVAL, "fg is NULL");
    if (int rc = ctx_check_device(c)) return rc;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    if (c->N > 0) {
        hipStream_t s = (hipStream_t)stream;
        double* w = (double*)ctx_scratch(c, 2, (4 + 4 * 256) * sizeof(double));
        if (!w) return fail(c, DBIE_E_WORKSPACE, "cannot allocate the statistics workspace");
        DBIE_HIP(c, launch_fg_stats(c->N, fg, eps, w, s));
        DBIE_HIP(c, hipMemcpyAsync(sums, w, sizeof(sums), hipMemcpyDeviceToHost, s));
        DBIE_HIP(c, hipStreamSynchronize(s));
    }
    out[0] = sums[2] > 0 ? sums[0] / sums[2] : std::nan("");
    out[1] = sums[2] > 0 ? sums[1] / sums[2] : std::nan("");
    out[2] = sums[2];
    out[3] = sums[3];
    return DBIE_OK;
}

int dbie_query_tuned(const dbie_ctx* c, int32_t* source) {
    if (!c) return DBIE_E_INVAL;
    if (source) *source = c->tuned;
    return DBIE_OK;
}

int dbie_query_split(const dbie_ctx* c, int32_t* slices) {
    if (!c) return DBIE_E_INVAL;
    if (slices) *slices = c->split;
    return DBIE_OK;
}

void dbie_destroy(dbie_ctx* c) { free_ctx(c); }

const char* dbie_last_error(const dbie_ctx* c) {
    if (!c) return g_init_error.c_str();
    return c->err.c_str();
}

}  // extern "C"

namespace dbie {
int set_shape(dbie_ctx* c, F32Shape s, bool tan) {
    if (!field32c_shape_supported(s)) return fail(c, DBIE_E_UNSUPPORTED, "tile shape not instantiated");
    return set_tiles32(c, s, tan);
}
F32Shape get_shape(const dbie_ctx* c, bool tan) { return tan ? c->shape_tan : c->shape; }

// The FP32C shape tuner. Candidates: every instantiated (points per lane, waves per workgroup) shape,
// in the grid form and the persistent form; then, only where the point tiles alone cannot fill the
// chip, the pixel split (1..32 slices). A candidate is timed on the bulk kernel alone over a prefix
// of its cost-ordered schedule (the largest tiles: 16 workgroups per compute unit, or the whole
// schedule if shorter; one warm-up launch, one timed), at lambda spread over |lambda| < 4 pi / L
// per component (L the longer side of the point's magnetogram) so that the timed loop is the one
// solves run, not the lambda = 0 special case. The fastest in pairs per second wins. Choices are
// kept per process under the key (device architecture, quadrature, pass, size bucket), the bucket
// being floor(log2) of the point count and of the mean quadrature points per magnetogram, and in
// the optional text cache as lines "<arch> <quad_points> <log2 N> <log2 pixels> <tan> <ppl> <waves>
// <tile_pixels> <persistent> <split>".
namespace {

struct TuneChoice {
    F32Shape shape;
    int32_t split;
};
std::mutex g_tune_mu;
std::vector<std::pair<std::string, TuneChoice>> g_tune_cache;

__global__ void k_tune_lambda(const int32_t* __restrict__ bidx, const BoundaryDev* __restrict__ bnd, int64_t N,
                              double* __restrict__ lam) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const BoundaryDev b = bnd[bidx[i]];
    const double lm = 4.0 * 3.14159265358979323846 / ((double)max(b.nx, b.ny) * b.h);
    for (int p = 0; p < 3; ++p) {
        const double u = (double)(3 * i + p) * 0.6180339887498949;
        lam[p * N + i] = lm * (2.0 * (u - floor(u)) - 1.0);
    }
}

std::string tune_key(const dbie_ctx* c, int tan) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
    }
    const int64_t grid = c->G ? c->ngrid_total : c->npix_total;
    const int bn = 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(c->N, 1));
    const int bp = 63 - __builtin_clzll((unsigned long long)std::max<int64_t>(grid / std::max(c->nb, 1), 1));
    char buf[128];
    std::snprintf(buf, sizeof buf, "%s %d %d %d %d", arch.c_str(), c->G, bn, bp, tan);
    return buf;
}

}  // namespace

// Time one candidate (shape sh, and the split c->split_tuned, or the automatic one when that is 0):
// the bulk kernel over the schedule prefix; returns pairs per millisecond (0 with *rc set on failure).
static double time_candidate(dbie_ctx* c, F32Shape sh, bool tan, const double* lam, hipEvent_t e0, hipEvent_t e1,
                             hipStream_t s, int* rc) {
    *rc = set_tiles32(c, sh, tan);
    if (*rc) return 0.0;
    const int32_t S = c->split;
    const std::vector<Tile>& t = tan ? c->tiles32t_h : c->tiles32_h;
    const int64_t n_sub = std::min<int64_t>((int64_t)t.size(), 16 * (int64_t)c->cus);
    double pairs = 0.0;
    for (int64_t k = 0; k < n_sub; ++k) {
        const BoundaryDev& b = c->bnd_h[t[k].b];
        pairs += (double)t[k].count * (double)(c->G ? (int64_t)b.gcols * b.grows : (int64_t)b.nx * b.ny);
    }
    if ((*rc = ensure_acc_slices(c, S))) return 0.0;
    const Tile* dt = tan ? c->tiles32t : c->tiles32;
    hipError_t e = hipSuccess;
    for (int r = 0; r < 2 && e == hipSuccess; ++r) {   // a warm-up launch, then the timed one
        if (r == 1) e = hipEventRecord(e0, s);
        if (e == hipSuccess)
            e = launch_field32c(dt, n_sub, c->bnd_d, c->pixf, c->gposf, c->geo, lam, c->N, 1, S, c->perm, c->work,
                                tan, false, sh, c->acc, s);
    }
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
        *rc = hip_fail(c, e, "tuning events");
        return 0.0;
    }
    return ms > 0.0f ? pairs / (double)ms : 0.0;
}

static int time_shapes(dbie_ctx* c, TuneChoice best[2], hipStream_t s);

int tune_shapes(dbie_ctx* c, const char* cache_path, hipStream_t s) {
    if (c->N == 0) return DBIE_OK;
    TuneChoice found[2];
    int have[2] = {0, 0};   // 3: the file, 2: this process's cache
    std::string key[2] = {tune_key(c, 0), tune_key(c, 1)};
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "r")) {
            char arch[64];
            int G, bn, bp, t, a, b, d, e, sp;
            while (fscanf(f, "%63s %d %d %d %d %d %d %d %d %d", arch, &G, &bn, &bp, &t, &a, &b, &d, &e, &sp) == 10) {
                char k[128];
                std::snprintf(k, sizeof k, "%s %d %d %d %d", arch, G, bn, bp, t);
                const F32Shape sh{a, b, d, e};
                if ((t == 0 || t == 1) && !have[t] && k == key[t] && field32c_shape_supported(sh) && sp >= 1 &&
                    sp <= kMaxSplit) {
                    found[t] = TuneChoice{sh, sp};
                    have[t] = 3;
                }
            }
            fclose(f);
        }
    }
    if (!(have[0] && have[1])) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        have[0] = have[1] = 0;
        for (auto& kv : g_tune_cache)
            for (int tan = 0; tan < 2; ++tan)
                if (kv.first == key[tan]) {
                    found[tan] = kv.second;
                    have[tan] = 2;
                }
    }
    const bool file_lacks = cache_path && !(have[0] == 3 && have[1] == 3);
    TuneChoice best[2];
    if (have[0] && have[1]) {
        best[0] = found[0];
        best[1] = found[1];
        c->tuned = have[0];
    } else {
        const int rc = time_shapes(c, best, s);
        if (rc) return rc;
        c->tuned = 1;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int tan = 0; tan < 2; ++tan) {
            TuneChoice ch{best[tan].shape, best[0].split};
            bool replaced = false;
            for (auto& kv : g_tune_cache)
                if (kv.first == key[tan]) {
                    kv.second = ch;
                    replaced = true;
                }
            if (!replaced) g_tune_cache.emplace_back(key[tan], ch);
        }
    }
    // the split is tuned with the plain pass and shared by both
    c->split_tuned = c->opt.pixel_split > 0 ? 0 : best[0].split;
    int rc = set_tiles32(c, best[0].shape, false);
    if (!rc) rc = set_tiles32(c, best[1].shape, true);
    if (rc) return rc;
    if (file_lacks) {
        if (FILE* f = fopen(cache_path, "a")) {
            for (int tan = 0; tan < 2; ++tan)
                fprintf(f, "%s %d %d %d %d %d\n", key[tan].c_str(), best[tan].shape.ppl, best[tan].shape.waves,
                        best[tan].shape.tp, best[tan].shape.persist, best[0].split);
            fclose(f);
        }
    }
    return DBIE_OK;
}

// Time the candidates (see tune_shapes) on this context; best[0] is the plain pass (with the split),
// best[1] the pass with tangents.
static int time_shapes(dbie_ctx* c, TuneChoice best[2], hipStream_t s) {
    double* lam = (double*)ctx_scratch(c, 3, (size_t)c->N * 3 * sizeof(double));
    if (!lam) return fail(c, DBIE_E_WORKSPACE, "cannot allocate the tuning workspace");
    hipLaunchKernelGGL(k_tune_lambda, dim3((unsigned)((c->N + 255) / 256)), dim3(256), 0, s, c->geo.bidx, c->bnd_d,
                       c->N, lam);
    DBIE_HIP(c, hipGetLastError());
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    DBIE_HIP(c, hipEventCreate(&ev.e0));
    DBIE_HIP(c, hipEventCreate(&ev.e1));
    F32Shape cand[16];
    const int nc = std::min(field32c_shapes(cand, 16), 16);
    for (int tan = 0; tan < 2; ++tan) {
        double rate = -1.0;
        best[tan] = TuneChoice{tan ? c->shape_tan : c->shape, c->split};
        for (int k = 0; k < nc; ++k) {
            int rc = 0;
            c->split_tuned = tan ? best[0].split : 0;
            const double r = time_candidate(c, cand[k], tan != 0, lam, ev.e0, ev.e1, s, &rc);
            if (rc) return rc;
            // the automatic split of this shape (set by set_tiles32) goes with it
            if (r > rate) {
                rate = r;
                best[tan] = TuneChoice{cand[k], c->split};
            }
        }
        // few points: the pixel split, with the chosen shape (the persistent form needs one slice)
        if (tan == 0 && c->opt.pixel_split == 0 && best[0].split > 1) {
            F32Shape sh = best[0].shape;
            sh.persist = 0;
            for (int32_t S = 1; S <= kMaxSplit; S *= 2) {
                int rc = 0;
                c->split_tuned = S;
                const double r = time_candidate(c, sh, false, lam, ev.e0, ev.e1, s, &rc);
                if (rc) return rc;
                if (r > rate) {
                    rate = r;
                    best[0] = TuneChoice{sh, S};
                }
            }
        }
    }
    return DBIE_OK;
}
}  // namespace dbie
