// ct_probe_alu_rates: issue rates of the instructions that bound the sweep
// kernels, measured on the current device.  The pair cost of a lagged sweep is
// d subtractions + d FMAs + 1 subtraction + 1 exp2 + 1 add; its roofline is the
// reciprocal of the summed issue time of that mix, so the per-instruction rates
// are what the roofline needs (public figures give only the packed-FMA peak).
#include <hip/hip_runtime.h>

#include "ct_internal.h"

namespace ct {

namespace {

constexpr int kChains = 8;     // independent dependency chains per lane
constexpr int kIters = 2048;   // chain steps per launch
constexpr int kProbeBlocks = 2048;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// kind 0: v_add_f32, 1: v_fma_f32, 2: v_exp_f32, 3: v_mfma_f32_16x16x4f32 (4 chains),
// 4: the MFMA chains and the exp chains of kinds 2 and 3 in the same waves.
// The addend c is formed by a vector multiply, so the add chain compiles to
// v_add_f32 with two vector-register operands (the form of the sweep's pair loop, whose adds
// have no scalar operand); adds with a scalar-register operand issue at about
// half that rate on gfx950.
template <int KIND>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_rate(
    float* __restrict__ out, float seed) {
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = seed * (float)(threadIdx.x + k) * 1e-9f - 3.f;
    const float c = seed * 1e-7f;
    const float a = seed * (float)threadIdx.x, b = seed + (float)threadIdx.x;
    f32x4 m0 = {0.f, 0.f, 0.f, 0.f}, m1 = m0, m2 = m0, m3 = m0;
    for (int i = 0; i < kIters; ++i) {
        if (KIND == 0) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = x[k] + c;
        }
        if (KIND == 1) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = __builtin_fmaf(x[k], c, c);
        }
        if (KIND == 2 || KIND == 4) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) x[k] = __builtin_amdgcn_exp2f(x[k]);
        }
        if (KIND == 3 || KIND == 4) {
            m0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, m0, 0, 0, 0);
            m1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, m1, 0, 0, 0);
            m2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, m2, 0, 0, 0);
            m3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, m3, 0, 0, 0);
        }
    }
    float s = m0[0] + m1[1] + m2[2] + m3[3];
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int KIND>
hipError_t time_kind(float* out, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float* ms) {
    hipLaunchKernelGGL(k_rate<KIND>, dim3(kProbeBlocks), dim3(256), 0, st, out, 1.0f);  // warm-up
    hipError_t e = hipEventRecord(e0, st);
    if (e != hipSuccess) return e;
    for (int r = 0; r < 3; ++r)
        hipLaunchKernelGGL(k_rate<KIND>, dim3(kProbeBlocks), dim3(256), 0, st, out, 1.0f);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipEventRecord(e1, st);
    if (e != hipSuccess) return e;
    e = hipEventSynchronize(e1);
    if (e != hipSuccess) return e;
    e = hipEventElapsedTime(ms, e0, e1);
    *ms /= 3.f;
    return e;
}

}  // namespace

}  // namespace ct

using namespace ct;

extern "C" size_t ct_probe_workspace_size(void) { return (size_t)kProbeBlocks * 256 * sizeof(float); }

extern "C" ct_status ct_probe_alu_rates(double* out6, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (!out6) return fail(CT_E_ARG, "out6 is null");
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (ws_bytes < ct_probe_workspace_size())
        return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes,
                    ct_probe_workspace_size());
    hipStream_t st = static_cast<hipStream_t>(stream);
    {
        const ct_status rc = refuse_capture(st, "ct_probe_alu_rates");
        if (rc) return rc;
    }
    int dev = 0, khz = 0, ncu = 0;
    CT_CHECK_HIP(hipGetDevice(&dev));
    CT_CHECK_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev));
    CT_CHECK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (khz <= 0 || ncu <= 0) return fail(CT_E_HIP, "device reports clock %d kHz, %d CUs", khz, ncu);
    float* out = static_cast<float*>(ws);
    hipEvent_t e0, e1;
    CT_CHECK_HIP(hipEventCreate(&e0));
    CT_CHECK_HIP(hipEventCreate(&e1));
    float ms[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    hipError_t e = time_kind<0>(out, st, e0, e1, &ms[0]);
    if (e == hipSuccess) e = time_kind<1>(out, st, e0, e1, &ms[1]);
    if (e == hipSuccess) e = time_kind<2>(out, st, e0, e1, &ms[2]);
    if (e == hipSuccess) e = time_kind<3>(out, st, e0, e1, &ms[3]);
    if (e == hipSuccess) e = time_kind<4>(out, st, e0, e1, &ms[4]);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(CT_E_HIP, "probe launch failed: %s", hipGetErrorString(e));
    const double lanes = (double)kProbeBlocks * 256 * kIters * kChains;   // lane operations per launch
    const double waves = (double)kProbeBlocks * 4;
    const double clk = (double)khz * 1e3 * ncu;                           // CU-clocks per second
    out6[0] = lanes / (ms[0] * 1e-3) / clk;                                // add lanes / clk / CU
    out6[1] = lanes / (ms[1] * 1e-3) / clk;                                // fma lanes / clk / CU
    out6[2] = lanes / (ms[2] * 1e-3) / clk;                                // exp lanes / clk / CU
    out6[3] = waves * kIters * 4 * 1024.0 / (ms[3] * 1e-3) / clk;          // MFMA FMAs / clk / CU
    out6[4] = ms[4] / (ms[2] + ms[3]);                                     // 1: no overlap
    out6[5] = (double)khz * 1e3;
    return CT_OK;
}
