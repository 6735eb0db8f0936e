// Entry points whose device paths are being brought up: they validate nothing
// yet and report CT_E_UNSUPPORTED.
#include "ct_internal.h"

using namespace ct;

extern "C" size_t ct_sinkhorn_batched_workspace_size(int32_t, const int64_t*, const int64_t*,
                                                     const ct_sinkhorn_opts*) {
    return 256;
}
extern "C" ct_status ct_sinkhorn_grad_batched(int32_t, const int64_t*, const int64_t*, const float*,
                                              const float*, const float*, const ct_sinkhorn_opts*,
                                              float*, float*, float*, void*, size_t, void*) {
    return fail(CT_E_UNSUPPORTED, "batched path not built yet");
}
extern "C" size_t ct_svgd_workspace_size(int64_t, int32_t) { return 256; }
extern "C" ct_status ct_svgd_grad(const float*, int64_t, int32_t, const ct_gmm*, float, float*,
                                  float*, float*, void*, size_t, void*) {
    return fail(CT_E_UNSUPPORTED, "svgd path not built yet");
}
extern "C" size_t ct_plan_workspace_size(const ct_plan_problem*, const ct_plan_opts*, int64_t) {
    return 256;
}
extern "C" ct_status ct_plan(const ct_plan_problem*, const ct_plan_opts*, const float*, const float*,
                             int64_t, const ct_gmm*, double*, double*, double*, void*, size_t,
                             void*) {
    return fail(CT_E_UNSUPPORTED, "plan not built yet");
}
extern "C" ct_status ct_lqr_track(int64_t, int32_t, int32_t, double, const double*, const double*,
                                  const double*, const double*, const double*, double*, double*) {
    return fail(CT_E_UNSUPPORTED, "lqr not built yet");
}
