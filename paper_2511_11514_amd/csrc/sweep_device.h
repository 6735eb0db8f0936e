// Device building blocks of the soft-min (log-sum-exp) sweep over a point-pair
// cost, shared by the per-problem sweep kernel and the batched persistent kernel.
//
// The log-domain Sinkhorn update (Sec. II-B, eq. 5 solved by Sinkhorn's
// algorithm) for one query point i against the key points j is
//     T(h)_i = -eps * log sum_j exp(h_j - |x_i - y_j|^2 / eps).
// Everything here works in base 2 with coordinates pre-scaled by sqrt(kappa),
// kappa = log2(e)/eps, so a pair costs
//     e_ij = kh_j - |x'_i - y'_j|^2      and      T_i = -(1/kappa) log2 sum_j 2^e_ij.
//
// Two accumulation modes:
//  * safe   : groups of kGroup keys, running maximum per query, rescale when it
//             grows (one extra exp per group);
//  * lagged : the shift is the query's own current potential (its value after
//             the previous sweep), folded into the cost; no maximum is tracked.
//             A row whose sum leaves [2^-64, 2^64] is recomputed in safe mode
//             by the block that merges it, so the result never depends on the
//             quality of the shift.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>

#include "ct_internal.h"

namespace ct {

__device__ __forceinline__ float ex2(float v) { return __builtin_amdgcn_exp2f(v); }

constexpr float kNegInf = -__builtin_huge_valf();
constexpr float kSumLo = 5.421010862427522e-20f;  // 2^-64
constexpr float kSumHi = 1.8446744073709552e19f;  // 2^64

// Stage keys [j0, j1) of a job into LDS as (x', y', h, 0) or (x', y', z', h);
// slots past j1 get h = -inf so they contribute exp2(-inf) = 0.
template <int D>
__device__ __forceinline__ void stage_tile(float4* tile, const float4* __restrict__ kc,
                                           const float* __restrict__ kh, int j0, int j1) {
    const int j = j0 + (int)threadIdx.x;
    float4 v;
    if (j < j1) {
        const float4 c = kc[j];
        const float h = kh[j];
        v = (D == 2) ? make_float4(c.x, c.y, h, 0.f) : make_float4(c.x, c.y, c.z, h);
    } else {
        v = (D == 2) ? make_float4(0.f, 0.f, kNegInf, 0.f) : make_float4(0.f, 0.f, 0.f, kNegInf);
    }
    tile[threadIdx.x] = v;
}

template <int D>
__device__ __forceinline__ float key_h(const float4& k) {
    return (D == 2) ? k.z : k.w;
}

// Per-thread state of R queries.
template <int D, int R>
struct QueryRegs {
    float q[R][D];   // pre-scaled coordinates
    float sh[R];     // lagged shift (log2 units) or running maximum (safe)
    float s[R];      // sum of 2^(e - sh)
    float b[R][D];   // sum of 2^(e - sh) * (x'_i - y'_j)
};

// Lagged accumulation over n staged keys (n a multiple of 4).
template <int D, int R, bool BARY>
__device__ __forceinline__ void accum_lagged(const float4* tile, int n, QueryRegs<D, R>& Q) {
#pragma unroll 4
    for (int j = 0; j < n; ++j) {
        const float4 k = tile[j];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float dx = Q.q[r][0] - k.x;
            const float dy = Q.q[r][1] - k.y;
            float c;
            float dz = 0.f;
            if (D == 2) {
                c = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, Q.sh[r]));
            } else {
                dz = Q.q[r][2] - k.z;
                c = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, Q.sh[r])));
            }
            const float p = ex2(key_h<D>(k) - c);
            Q.s[r] += p;
            if (BARY) {
                Q.b[r][0] = __builtin_fmaf(p, dx, Q.b[r][0]);
                Q.b[r][1] = __builtin_fmaf(p, dy, Q.b[r][1]);
                if (D == 3) Q.b[r][2] = __builtin_fmaf(p, dz, Q.b[r][2]);
            }
        }
    }
}

// Safe accumulation over n staged keys (n a multiple of kGroup).
template <int D, int R, bool BARY>
__device__ __forceinline__ void accum_safe(const float4* tile, int n, QueryRegs<D, R>& Q) {
    for (int j0 = 0; j0 < n; j0 += kGroup) {
        float e[R][kGroup];
#pragma unroll
        for (int g = 0; g < kGroup; ++g) {
            const float4 k = tile[j0 + g];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float dx = Q.q[r][0] - k.x;
                const float dy = Q.q[r][1] - k.y;
                float c = dy * dy;
                if (D == 3) {
                    const float dz = Q.q[r][2] - k.z;
                    c = __builtin_fmaf(dz, dz, c);
                }
                c = __builtin_fmaf(dx, dx, c);
                e[r][g] = key_h<D>(k) - c;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            float tm = e[r][0];
#pragma unroll
            for (int g = 1; g < kGroup; ++g) tm = fmaxf(tm, e[r][g]);
            const float mn = fmaxf(Q.sh[r], tm);
            const float sc = ex2(Q.sh[r] - mn);
            Q.sh[r] = mn;
            Q.s[r] *= sc;
            if (BARY) {
#pragma unroll
                for (int t = 0; t < D; ++t) Q.b[r][t] *= sc;
            }
#pragma unroll
            for (int g = 0; g < kGroup; ++g) {
                const float p = ex2(e[r][g] - mn);
                Q.s[r] += p;
                if (BARY) {
                    const float4 k = tile[j0 + g];
                    Q.b[r][0] = __builtin_fmaf(p, Q.q[r][0] - k.x, Q.b[r][0]);
                    Q.b[r][1] = __builtin_fmaf(p, Q.q[r][1] - k.y, Q.b[r][1]);
                    if (D == 3) Q.b[r][2] = __builtin_fmaf(p, Q.q[r][2] - k.z, Q.b[r][2]);
                }
            }
        }
    }
}

// Sweep keys [k0, k1) of job J for the block's queries, staging tiles in LDS.
template <int D, int R, bool LAGGED, bool BARY>
__device__ __forceinline__ void sweep_range(const Job& J, int k0, int k1, float4* tile,
                                            QueryRegs<D, R>& Q) {
    for (int t0 = k0; t0 < k1; t0 += kTile) {
        const int t1 = min(t0 + kTile, k1);
        __syncthreads();
        stage_tile<D>(tile, J.kc, J.kh, t0, t1);
        __syncthreads();
        const int cnt = t1 - t0;
        if (LAGGED) {
            accum_lagged<D, R, BARY>(tile, (cnt + 3) & ~3, Q);
        } else {
            accum_safe<D, R, BARY>(tile, (cnt + kGroup - 1) & ~(kGroup - 1), Q);
        }
    }
}

template <int D, int R>
__device__ __forceinline__ void init_queries(const Job& J, int qbase, float kappa, bool lagged,
                                             QueryRegs<D, R>& Q) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = qbase + r * kBlock + (int)threadIdx.x;
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        float sh = lagged ? 0.f : -FLT_MAX;
        if (q < J.nq) {
            c = J.qc[q];
            if (lagged) sh = -J.qpot[q] * kappa;
        }
        Q.q[r][0] = c.x;
        Q.q[r][1] = c.y;
        if (D == 3) Q.q[r][2] = c.z;
        Q.sh[r] = sh;
        Q.s[r] = 0.f;
#pragma unroll
        for (int t = 0; t < D; ++t) Q.b[r][t] = 0.f;
    }
}

// Write the final value of one query row given (shift, sum, offset sums).
template <int D>
__device__ __forceinline__ void finish_row(const Job& J, int q, float m, float s, const float* b,
                                           float kappa, float inv_kappa, float inv_sqrt_kappa) {
    const float lse2 = m + __log2f(s);
    const float t = -lse2 * inv_kappa;
    const float old = J.qpot[q];
    const float nv = J.self_avg ? 0.5f * (old + t) : t;
    J.out_pot[q] = nv;
    if (J.out_h) {
        const float lw = J.qlog2w ? J.qlog2w[q] : J.qlog2w_s;
        J.out_h[q] = __builtin_fmaf(nv, kappa, lw);
    }
    if (J.out_bary) {
        const float inv = -inv_sqrt_kappa / s;
#pragma unroll
        for (int t2 = 0; t2 < D; ++t2) J.out_bary[(size_t)q * D + t2] = b[t2] * inv;
    }
}

// Recompute the flagged rows of this block with a tracked maximum over every key
// of the job, the whole block cooperating on one row at a time.
template <int D, bool BARY>
__device__ void rescue_rows(const Job& J, const int* flist, int nflag, int qbase, float kappa,
                            float inv_kappa, float inv_sqrt_kappa) {
    __shared__ float red[kBlock * (2 + D)];
    for (int f = 0; f < nflag; ++f) {
        const int q = qbase + flist[f];
        const float4 qc = J.qc[q];
        float m = -FLT_MAX, s = 0.f, b[D];
#pragma unroll
        for (int t = 0; t < D; ++t) b[t] = 0.f;
        for (int j = (int)threadIdx.x; j < J.nk; j += kBlock) {
            const float4 k = J.kc[j];
            const float dx = qc.x - k.x, dy = qc.y - k.y;
            float c = dy * dy;
            float dz = 0.f;
            if (D == 3) {
                dz = qc.z - k.z;
                c = __builtin_fmaf(dz, dz, c);
            }
            c = __builtin_fmaf(dx, dx, c);
            const float e = J.kh[j] - c;
            if (e > m) {
                const float sc = ex2(m - e);
                s *= sc;
#pragma unroll
                for (int t = 0; t < D; ++t) b[t] *= sc;
                m = e;
            }
            const float p = ex2(e - m);
            s += p;
            if (BARY) {
                b[0] = __builtin_fmaf(p, dx, b[0]);
                b[1] = __builtin_fmaf(p, dy, b[1]);
                if (D == 3) b[2] = __builtin_fmaf(p, dz, b[2]);
            }
        }
        red[threadIdx.x] = m;
        red[kBlock + threadIdx.x] = s;
#pragma unroll
        for (int t = 0; t < D; ++t) red[(2 + t) * kBlock + threadIdx.x] = b[t];
        __syncthreads();
        if (threadIdx.x == 0) {
            float M = -FLT_MAX;
            for (int i = 0; i < kBlock; ++i) M = fmaxf(M, red[i]);
            float S = 0.f, B[D];
#pragma unroll
            for (int t = 0; t < D; ++t) B[t] = 0.f;
            for (int i = 0; i < kBlock; ++i) {
                const float sc = ex2(red[i] - M);
                S = __builtin_fmaf(red[kBlock + i], sc, S);
#pragma unroll
                for (int t = 0; t < D; ++t) B[t] = __builtin_fmaf(red[(2 + t) * kBlock + i], sc, B[t]);
            }
            finish_row<D>(J, q, M, S, B, kappa, inv_kappa, inv_sqrt_kappa);
            atomicAdd(J.rescued, 1u);
        }
        __syncthreads();
    }
}

// After the block's key range is done: either finish directly (one split) or
// publish partials and let the last block to arrive merge all splits.
template <int D, int R, bool LAGGED, bool BARY>
__device__ __forceinline__ void publish_and_merge(const Job& J, int qb, int split, int qbase,
                                                  QueryRegs<D, R>& Q, float kappa,
                                                  float inv_kappa, float inv_sqrt_kappa) {
    __shared__ int s_last;
    __shared__ int s_nflag;
    __shared__ int s_flist[kBlock * R];
    const int nqpad = J.nqb * kBlock * R;
    if (J.splits > 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int ql = qbase + r * kBlock + (int)threadIdx.x;
            float* P = J.part + ql;
            const size_t stride = (size_t)J.splits * nqpad;
            P[(size_t)split * nqpad] = Q.sh[r];
            P[stride + (size_t)split * nqpad] = Q.s[r];
            if (BARY) {
#pragma unroll
                for (int t = 0; t < D; ++t) P[(2 + t) * stride + (size_t)split * nqpad] = Q.b[r][t];
            }
        }
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned prev = atomicAdd(&J.ticket[qb], 1u);
            s_last = (prev == (unsigned)(J.splits - 1));
        }
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        // merge every split's partials for this block's queries
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int ql = qbase + r * kBlock + (int)threadIdx.x;
            const float* P = J.part + ql;
            const size_t stride = (size_t)J.splits * nqpad;
            float M = -FLT_MAX;
            for (int sp = 0; sp < J.splits; ++sp) M = fmaxf(M, P[(size_t)sp * nqpad]);
            float S = 0.f, B[D];
#pragma unroll
            for (int t = 0; t < D; ++t) B[t] = 0.f;
            for (int sp = 0; sp < J.splits; ++sp) {
                const float sc = LAGGED ? 1.f : ex2(P[(size_t)sp * nqpad] - M);
                S = __builtin_fmaf(P[stride + (size_t)sp * nqpad], sc, S);
                if (BARY) {
#pragma unroll
                    for (int t = 0; t < D; ++t)
                        B[t] = __builtin_fmaf(P[(2 + t) * stride + (size_t)sp * nqpad], sc, B[t]);
                }
            }
            Q.sh[r] = M;
            Q.s[r] = S;
#pragma unroll
            for (int t = 0; t < D; ++t) Q.b[r][t] = B[t];
        }
        if (threadIdx.x == 0) J.ticket[qb] = 0u;
    }
    if (LAGGED) {
        if (threadIdx.x == 0) s_nflag = 0;
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = qbase + r * kBlock + (int)threadIdx.x;
        if (q >= J.nq) continue;
        if (LAGGED && !(Q.s[r] >= kSumLo && Q.s[r] <= kSumHi)) {
            const int idx = atomicAdd(&s_nflag, 1);
            s_flist[idx] = r * kBlock + (int)threadIdx.x;
            continue;
        }
        finish_row<D>(J, q, Q.sh[r], Q.s[r], Q.b[r], kappa, inv_kappa, inv_sqrt_kappa);
    }
    if (LAGGED) {
        __syncthreads();
        const int nflag = s_nflag;
        if (nflag > 0) rescue_rows<D, BARY>(J, s_flist, nflag, qbase, kappa, inv_kappa, inv_sqrt_kappa);
    }
}

}  // namespace ct
