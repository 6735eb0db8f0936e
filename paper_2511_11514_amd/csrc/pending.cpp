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
