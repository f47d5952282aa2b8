// Internal: the device-resident lambda solver, the adjoint and the shape tuner, and the context
// accessors they use. Not part of the public ABI.
#pragma once

#include <vector>

#include "../../include/dbie.h"
#include "dbie_internal.h"

namespace dbie {

// What a captured solver graph depends on (compared bytewise before a replay).
struct GraphKey {
    int32_t method, max_trials, fp64, per32;
    double eps, step, cap, radius, damping;
    void* block;
    hipStream_t stream;
    const int32_t* perm;
    // what the captured launches bake in besides the solver's own buffers: the accumulator (it is
    // reallocated when a call needs more trials or slices), the pixel split and the tile shape
    const void* acc;
    int32_t split, ppl, waves, persist;
};

// Device buffers owned by a context for dbie_solve_lambda (allocated on first use, grown on need).
struct SolverState {
    hipGraphExec_t exec = nullptr;   // captured rounds, replayed while `key` matches
    GraphKey key{};
    hipStream_t rs = nullptr;        // library stream the captured rounds run on (the caller's stream
                                     // may be the legacy default stream, which cannot be captured)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    void* block = nullptr;       // one allocation for every per-point solver array
    int64_t bytes = 0;
    bool block_owned = false;    // false: the block lies in the caller's workspace
    int32_t* count_h = nullptr;  // pinned host word: active-point count
    int32_t last_rounds = 0;     // rounds of the last solve
    int32_t* last_conv = nullptr;  // device: points converged in each round of the last solve
};

void solver_free(SolverState& s);

// Which points an evaluation covers: an active-point list with a device-resident count and the
// device-built schedules over it (tiles of list entries). NULL set = every point, static schedules.
struct EvalSet {
    const int32_t* idx;
    const int32_t* n_dev;
    const Tile* tiles32;
    int64_t n_tiles32;
    const Tile* tiles64;
    int64_t n_tiles64;
};

// Make sure the accumulator workspace holds L trials (allocates; never called during capture), or
// `slices` partial-sum slices of [kAcc][N].
int ensure_acc(dbie_ctx* c, int64_t L);
int ensure_acc_slices(dbie_ctx* c, int64_t slices);

// Pixel slices for an evaluation of about n points (bounded by the accumulator memory).
int32_t split_for_points(dbie_ctx* c, int64_t n);

// One lambda trial (L = 1) through the bulk kernel and the finalize pass; S > 0 overrides the
// context's pixel slices.
int eval_set(dbie_ctx* c, const double* lam, bool fp64, bool tan, const EvalSet* set, double* B, double* dB,
             double* fg, double* tn, hipStream_t s, int32_t S = 0);

// context accessors (defined in dbie_api.hip)
const Geo& ctx_geo(const dbie_ctx* c);
const BoundaryDev* ctx_bnd(const dbie_ctx* c);
const BoundaryDev& ctx_bnd_host(const dbie_ctx* c, int b);
int64_t ctx_n(const dbie_ctx* c);
const int32_t* ctx_perm(const dbie_ctx* c);   // FP32C point order or NULL (identity)
int32_t ctx_nb(const dbie_ctx* c);
const int64_t* ctx_seg(const dbie_ctx* c);
const double* ctx_B0d(const dbie_ctx* c);
struct QuadGrid {
    const double* pos;   // grid positions (BoundaryDev::gpos_off)
    const double* gB;    // weighted field on the grid (BoundaryDev::gpl_off)
    const double* lw;    // 9-node elements: w_g L_a(xi_g), 3 G doubles; NULL for the nodal rule
    int32_t G;           // Gauss points per element side; 0 = nodal rule
    int64_t n_total;     // grid points over all boundaries
    const float4* posf;  // FP32C split positions (BoundaryDev::gposf_off); NULL for the nodal rule
};
QuadGrid ctx_grid(const dbie_ctx* c);
int ctx_precision(const dbie_ctx* c);
double ctx_dvds(const dbie_ctx* c);
SolverState& ctx_solver(dbie_ctx* c);
int ctx_fail(dbie_ctx* c, int code, const char* msg);
// DBIE_OK when the current HIP device is the context's, else DBIE_E_INVAL with a message.
int ctx_check_device(dbie_ctx* c);
const void* ctx_acc(const dbie_ctx* c);
int32_t ctx_split(const dbie_ctx* c);
double* ctx_xyz(dbie_ctx* c);   // the context's own copy of the points (device [3][N])
// Re-run the per-point geometry and near-field classification on the current ctx_xyz (same kernel
// as dbie_init; invalid points are flagged in *flag and given safe geometry).
hipError_t ctx_prep_points(dbie_ctx* c, int32_t* flag, hipStream_t s);
// Library-owned scratch block `slot` of at least `bytes` (grown on need); NULL on failure.
void* ctx_scratch(dbie_ctx* c, int slot, size_t bytes);   // NULL if it cannot be provided
// Caller-owned workspace (dbie_set_workspace): the region of one consumer, NULL when no workspace is
// set (the library allocates), kWsTooSmall when the region cannot hold `bytes`.
enum { kWsAcc = 0, kWsSolver = 1, kWsSlot0 = 2, kWsRegions = 6 };
extern void* const kWsTooSmall;
void* ctx_ws_region(dbie_ctx* c, int region, size_t bytes);
size_t solver_workspace_bytes(const dbie_ctx* c);
size_t grad_workspace_bytes(const dbie_ctx* c);   // dbie_grad's gB0 part (scratch slot 1)
// The transpose kernels' pixel-tile lists and the point segments, on the device (built in dbie_init):
// n64 tiles of the FP64 kernel, then n32 of the FP32C kernel, then nb + 1 int64 offsets at seg_off.
struct VjpTables {
    const void* base;
    int64_t n64, n32;
    size_t seg_off;
};
hipError_t vjp_tables_init(const dbie_ctx* c, void** dev, VjpTables* t);
VjpTables ctx_vjp_tables(const dbie_ctx* c);
void ws_sizes(const dbie_ctx* c, size_t sz[kWsRegions]);
// Near-field pairs grouped by pixel (global pixel index over all magnetograms), for the adjoint.
struct NearLists {
    int64_t npix_total;      // quadrature grid points over all boundaries (the pixels for the nodal rule)
    int64_t n_pairs;
    const int32_t* ptr;      // [npix_total + 1]
    const int32_t* pts;      // [n_pairs] point indices, ascending per grid point
    const int32_t* pix_bnd;  // [npix_total] magnetogram of each grid point
};
NearLists ctx_near_lists(const dbie_ctx* c);
bool solver_tracing(const dbie_ctx* c);
bool ctx_timing(const dbie_ctx* c);
std::vector<hipEvent_t>& solver_trace_events(dbie_ctx* c);
hipEvent_t& solver_trace_end(dbie_ctx* c);   // recorded at the end of a traced solve
// Drops what the last solve left for dbie_solve_trace_read (its events and per-round counts); called
// before a solve may move the solver block and when the workspace changes.
void solver_forget_last(dbie_ctx* c);
// FP32C tile shapes: one for the plain field pass and one for the pass with mu-tangents.
int set_shape(dbie_ctx* c, F32Shape s, bool tan);
F32Shape get_shape(const dbie_ctx* c, bool tan);

// Time the instantiated FP32C shapes on this problem and keep the fastest (optionally cached).
int tune_shapes(dbie_ctx* c, const char* cache_path, hipStream_t s);

}  // namespace dbie
