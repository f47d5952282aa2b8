#include "dbie_solver.h"

namespace dbie {
void solver_free(SolverState& s) {
    (void)hipFree(s.block);
    if (s.count_h) (void)hipHostFree(s.count_h);
    s = SolverState{};
}
int tune_shapes(dbie_ctx*, const char*, hipStream_t) { return DBIE_OK; }
}  // namespace dbie

extern "C" {
int dbie_solve_lambda(dbie_ctx* c, double*, const dbie_solve_opts*, double*, double*, int32_t*, int32_t*,
                      void*) {
    return dbie::ctx_fail(c, DBIE_E_UNSUPPORTED, "not built yet");
}
int dbie_grad(dbie_ctx* c, const double*, const double*, const double*, double*, double*, double*, void*) {
    return dbie::ctx_fail(c, DBIE_E_UNSUPPORTED, "not built yet");
}
}
