// Internal: the device-resident lambda solver, the adjoint and the shape tuner, and the context
// accessors they use. Not part of the public ABI.
#pragma once

#include "../../include/dbie.h"
#include "dbie_internal.h"

namespace dbie {

// Device buffers owned by a context for dbie_solve_lambda / dbie_grad (allocated on first use).
struct SolverState {
    void* block = nullptr;   // one allocation for every per-point solver array
    int64_t n = 0;           // points it was sized for
    int32_t* count_h = nullptr;  // pinned host word: active-point count
};

void solver_free(SolverState& s);

// context accessors (defined in dbie_api.hip)
int ensure_acc(dbie_ctx* c, int64_t L);
int eval_internal(dbie_ctx* c, const double* lam, int32_t L, bool fp64, bool tan, const int32_t* idx,
                  int64_t n_idx, double* B, double* dB, double* fg, double* tn, hipStream_t s);
const Geo& ctx_geo(const dbie_ctx* c);
const BoundaryDev* ctx_bnd(const dbie_ctx* c);
const BoundaryDev& ctx_bnd_host(const dbie_ctx* c, int b);
int64_t ctx_n(const dbie_ctx* c);
int32_t ctx_nb(const dbie_ctx* c);
const double* ctx_B0d(const dbie_ctx* c);
const double* ctx_xyz(const dbie_ctx* c);
int ctx_precision(const dbie_ctx* c);
double ctx_dvds(const dbie_ctx* c);
SolverState& ctx_solver(dbie_ctx* c);
int ctx_fail(dbie_ctx* c, int code, const char* msg);
int set_shape(dbie_ctx* c, F32Shape s);
F32Shape get_shape(const dbie_ctx* c);

// Time the instantiated FP32C shapes on this problem and keep the fastest (optionally cached).
int tune_shapes(dbie_ctx* c, const char* cache_path, hipStream_t s);

}  // namespace dbie
