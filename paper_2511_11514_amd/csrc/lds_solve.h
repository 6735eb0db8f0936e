// Device building blocks of the LDS-resident solves (one workgroup: tiny.hip;
// several workgroups exchanging potentials: mesh.hip).
//
// Pairs in the expanded form.  Coordinates arrive centred on the problem's
// origin and scaled by sqrt(kappa); a point's record is (2v', H) with
// H = h - |v'|^2, so that for a query q'
//     e = h_j - |q' - k'_j|^2 - sh = H_j + 2k'_j.q' + C,   C = -|q'|^2 - sh,
// and a pair costs d FMAs, an add, the exp and the accumulate, reading one
// 16-byte record (an LDS broadcast) per key and wave.
#pragma once

#include <hip/hip_runtime.h>

namespace ct {
namespace lds_solve {

constexpr float kLo = 5.421010862427522e-20f;   // 2^-64
constexpr float kHi = 1.8446744073709552e19f;   // 2^64

__device__ __forceinline__ float tex2(float v) { return __builtin_amdgcn_exp2f(v); }

// H_j + 2k'_j.q' for a key record (2k', H) and a query q'
template <int D>
__device__ __forceinline__ float kdot(const float4& k, const float (&q)[3]) {
    float t = k.w;
    if (D == 3) t = __builtin_fmaf(q[2], k.z, t);
    t = __builtin_fmaf(q[1], k.y, t);
    return __builtin_fmaf(q[0], k.x, t);
}

// Lagged sums of R rows over keys [k0, k1): s_r = sum_j 2^(kdot_j + C_r).
// Four accumulation chains per lane; their sums are added in a fixed order.  The
// key records of the next step are read while the current step is evaluated,
// so a wave waits for LDS once per task rather than once per step.
template <int D, int R>
__device__ __forceinline__ void sum_lagged(const float4* kr, int k0, int k1,
                                           const float (&q)[R][3], const float (&C)[R],
                                           float (&s)[R]) {
    constexpr int A = R >= 4 ? 1 : 4 / R;
    constexpr int U = 4;
    float acc[R][A];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int a = 0; a < A; ++a) acc[r][a] = 0.f;
    auto step = [&](const float4 (&k)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r][u % A] += tex2(kdot<D>(k[u], q[r]) + C[r]);
    };
    int j = k0;
    if (j + U <= k1) {
        // two register buffers in turn: read one step ahead into the other
        float4 ka[U], kb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ka[u] = kr[j + u];
        for (;;) {
            if (j + 2 * U > k1) {
                step(ka);
                j += U;
                break;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) kb[u] = kr[j + U + u];
            step(ka);
            j += U;
            if (j + 2 * U > k1) {
                step(kb);
                j += U;
                break;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) ka[u] = kr[j + U + u];
            step(kb);
            j += U;
        }
    }
    for (; j < k1; ++j) {
        const float4 k = kr[j];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][0] += tex2(kdot<D>(k, q[r]) + C[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float t = acc[r][0];
#pragma unroll
        for (int a = 1; a < A; ++a) t += acc[r][a];
        s[r] = t;
    }
}

// Maximum m_r of kdot_j + C_r over keys [k0, k1) and the sum of 2^(kdot_j + C_r - m_r)
// (two passes).  A row whose every key term is -inf gets m = -inf and s = 0.
template <int D, int R>
__device__ __forceinline__ void sum_safe(const float4* kr, int k0, int k1,
                                         const float (&q)[R][3], const float (&C)[R],
                                         float (&m)[R], float (&s)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) m[r] = -__builtin_huge_valf();
    for (int j = k0; j < k1; ++j) {
        const float4 k = kr[j];
#pragma unroll
        for (int r = 0; r < R; ++r) m[r] = fmaxf(m[r], kdot<D>(k, q[r]) + C[r]);
    }
    float c[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        c[r] = C[r] - (m[r] == -__builtin_huge_valf() ? 0.f : m[r]);
        s[r] = 0.f;
    }
    for (int j = k0; j < k1; ++j) {
        const float4 k = kr[j];
#pragma unroll
        for (int r = 0; r < R; ++r) s[r] += tex2(kdot<D>(k, q[r]) + c[r]);
    }
}

// |v'|^2 of a staged point
template <int D>
__device__ __forceinline__ float norm2(const float4& c) {
    if (D == 2) return __builtin_fmaf(c.x, c.x, c.y * c.y);
    return __builtin_fmaf(c.x, c.x, __builtin_fmaf(c.y, c.y, c.z * c.z));
}

}  // namespace lds_solve
}  // namespace ct
