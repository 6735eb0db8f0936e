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
// Work decomposition.  A block has 4 wave64s.  Each lane owns R queries.  The
// 4 waves either own 4 different query groups (WS = 1), or 2 groups with the
// keys halved between wave pairs (WS = 2), or one group with the keys split
// four ways (WS = 4); the WS partial sums are combined through LDS.  Keys are
// 16-byte records (x', y', [z',] h).  In lagged sweeps each wave stages 64 keys
// at a time in a private LDS slot (one coalesced vector load, issued a chunk
// ahead) and reads them back as broadcasts, so a key read serves 64 R pairs and
// the load latency hides behind the previous chunk's work; safe sweeps read
// groups of 8 wave-uniform records through the scalar cache.
//
// Two accumulation modes:
//  * safe   : groups of 8 keys, running maximum per query, rescale when it
//             grows (one extra exp per group);
//  * lagged : the shift is the query's own current potential (its value after
//             the previous sweep), folded into the cost; no maximum is tracked.
//             A row whose sum leaves [2^-64, 2^64] is recomputed in safe mode
//             by the block that merges it, so the result never depends on the
//             quality of the shift.
// Blocks that cover different key ranges of the same queries publish partial
// sums; the last block to arrive (arrival ticket per query block) merges them
// in a fixed order, so results are deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>

#include "ct_internal.h"

namespace ct {

__device__ __forceinline__ float ex2(float v) { return __builtin_amdgcn_exp2f(v); }

constexpr float kNegInf = -__builtin_huge_valf();
constexpr float kSumLo = 5.421010862427522e-20f;  // 2^-64
constexpr float kSumHi = 1.8446744073709552e19f;  // 2^64

template <int D>
__device__ __forceinline__ float rec_h(const float4& k) {
    return (D == 2) ? k.z : k.w;
}

// Per-lane state of R queries.
template <int D, int R>
struct QueryRegs {
    float q[R][D];   // pre-scaled coordinates
    float sh[R];     // lagged shift (log2 units) or running maximum (safe)
    float s[R];      // sum of 2^(e - sh)
    float b[R][D];   // sum of 2^(e - sh) * (x'_i - y'_j)
};

template <int D, int R, bool BARY>
__device__ __forceinline__ void pair_lagged(const float4& k, QueryRegs<D, R>& Q) {
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
        const float p = ex2(rec_h<D>(k) - c);
        Q.s[r] += p;
        if (BARY) {
            Q.b[r][0] = __builtin_fmaf(p, dx, Q.b[r][0]);
            Q.b[r][1] = __builtin_fmaf(p, dy, Q.b[r][1]);
            if (D == 3) Q.b[r][2] = __builtin_fmaf(p, dz, Q.b[r][2]);
        }
    }
}

// Expanded form of the lagged pair, for sweeps without offsets.  Around an origin
// o shared by a wave (its first query), with q' = x'_i - o and k' = y'_j - o,
//     e_ij = h_j - |q' - k'|^2 - sh_i = H_j + 2 q'.k' + C_i,
//     H_j = h_j - |k'|^2 (per key, formed once per wave when the key is staged),
//     C_i = -|q'|^2 - sh_i (per query),
// so a pair costs d FMAs, one add, the exp and the accumulate instead of d
// subtractions, d FMAs, one subtraction, the exp and the accumulate.  The staged
// key record holds (2k', H_j); the query registers hold q' and C_i.  Near pairs,
// the only ones whose terms count, have small |q'| and |k'| when the wave's
// queries lie close together; far pairs round more coarsely, but their terms are
// negligible.  Rows recomputed with a tracked maximum use the difference form.
template <int D, int R>
__device__ __forceinline__ void pair_expanded(const float4& k, QueryRegs<D, R>& Q,
                                              const float (&C)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float t;
        if (D == 2) {
            t = __builtin_fmaf(Q.q[r][1], k.y, k.z);
            t = __builtin_fmaf(Q.q[r][0], k.x, t);
        } else {
            t = __builtin_fmaf(Q.q[r][2], k.z, k.w);
            t = __builtin_fmaf(Q.q[r][1], k.y, t);
            t = __builtin_fmaf(Q.q[r][0], k.x, t);
        }
        Q.s[r] += ex2(t + C[r]);
    }
}

// Key record (x', y', [z',] h) -> (2k', H) around the origin o (see pair_expanded).
template <int D>
__device__ __forceinline__ float4 expand_key(const float4& v, const float (&o)[3]) {
    const float kx = v.x - o[0], ky = v.y - o[1];
    if (D == 2) {
        const float n = __builtin_fmaf(kx, kx, ky * ky);
        return make_float4(2.f * kx, 2.f * ky, v.z - n, 0.f);
    }
    const float kz = v.z - o[2];
    const float n = __builtin_fmaf(kx, kx, __builtin_fmaf(ky, ky, kz * kz));
    return make_float4(2.f * kx, 2.f * ky, 2.f * kz, v.w - n);
}

// Lagged sweep of keys [k0, k1) in the expanded form: the LDS staging of
// sweep_keys with each key transformed by the lane that loads it.
template <int D, int R>
__device__ __forceinline__ void sweep_keys_expanded(const float4* __restrict__ rec, int k0, int k1,
                                                    const float (&o)[3], const float (&C)[R],
                                                    QueryRegs<D, R>& Q) {
    __shared__ float4 kbuf[4][64];
    const int lane = (int)threadIdx.x & 63;
    float4* slot = kbuf[__builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6)];
    if (k0 >= k1) return;
    float4 nxt = rec[min(k0 + lane, k1 - 1)];
    for (int k = k0; k < k1; k += 64) {
        const float4 mine = expand_key<D>(nxt, o);
        __builtin_amdgcn_wave_barrier();
        slot[lane] = mine;
        __builtin_amdgcn_wave_barrier();
        if (k + 64 < k1) nxt = rec[min(k + 64 + lane, k1 - 1)];
        const int n = min(64, k1 - k);
#pragma unroll 2
        for (int j = 0; j < n; j += 8) {
#pragma unroll
            for (int g = 0; g < 8; ++g) pair_expanded<D, R>(slot[j + g], Q, C);
        }
    }
}

// Safe mode over a group of 8 keys.
template <int D, int R, bool BARY>
__device__ __forceinline__ void group_safe(const float4 (&k)[8], QueryRegs<D, R>& Q) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float e[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const float dx = Q.q[r][0] - k[g].x;
            const float dy = Q.q[r][1] - k[g].y;
            float c = dy * dy;
            if (D == 3) {
                const float dz = Q.q[r][2] - k[g].z;
                c = __builtin_fmaf(dz, dz, c);
            }
            c = __builtin_fmaf(dx, dx, c);
            e[g] = rec_h<D>(k[g]) - c;
        }
        float tm = fmaxf(fmaxf(fmaxf(e[0], e[1]), fmaxf(e[2], e[3])),
                         fmaxf(fmaxf(e[4], e[5]), fmaxf(e[6], e[7])));
        const float mn = fmaxf(Q.sh[r], tm);
        const float sc = ex2(Q.sh[r] - mn);
        Q.sh[r] = mn;
        Q.s[r] *= sc;
        if (BARY) {
#pragma unroll
            for (int t = 0; t < D; ++t) Q.b[r][t] *= sc;
        }
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const float p = ex2(e[g] - mn);
            Q.s[r] += p;
            if (BARY) {
                Q.b[r][0] = __builtin_fmaf(p, Q.q[r][0] - k[g].x, Q.b[r][0]);
                Q.b[r][1] = __builtin_fmaf(p, Q.q[r][1] - k[g].y, Q.b[r][1]);
                if (D == 3) Q.b[r][2] = __builtin_fmaf(p, Q.q[r][2] - k[g].z, Q.b[r][2]);
            }
        }
    }
}

// Accumulate keys [k0, k1) (wave-uniform, multiples of 8; the record array is
// padded with h = -inf records up to a multiple of 8).
template <int D, int R, bool LAGGED, bool BARY>
__device__ __forceinline__ void sweep_keys(const float4* __restrict__ rec, int k0, int k1,
                                           QueryRegs<D, R>& Q) {
    if (LAGGED) {
        // 64 keys per wave at a time: one coalesced vector load (the next chunk is
        // loaded while this one is swept), one LDS write, then broadcast reads.
        // LDS operations of one wave complete in order, so a wave-private slot
        // needs no barrier; the wave barriers only keep the compiler from moving
        // the slot's accesses across the write.
        __shared__ float4 kbuf[4][64];
        const int lane = (int)threadIdx.x & 63;
        float4* slot = kbuf[__builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6)];
        if (k0 >= k1) return;
        float4 nxt = rec[min(k0 + lane, k1 - 1)];
        for (int k = k0; k < k1; k += 64) {
            __builtin_amdgcn_wave_barrier();
            slot[lane] = nxt;
            __builtin_amdgcn_wave_barrier();
            if (k + 64 < k1) nxt = rec[min(k + 64 + lane, k1 - 1)];
            const int n = min(64, k1 - k);
#pragma unroll 2
            for (int j = 0; j < n; j += 8) {
#pragma unroll
                for (int g = 0; g < 8; ++g) pair_lagged<D, R, BARY>(slot[j + g], Q);
            }
        }
    } else {
        for (int k = k0; k < k1; k += 8) {
            float4 kk[8];
#pragma unroll
            for (int g = 0; g < 8; ++g) kk[g] = rec[k + g];
            group_safe<D, R, BARY>(kk, Q);
        }
    }
}

template <int D, int R>
__device__ __forceinline__ void load_queries(const Job& J, int qbase, int lane, float kappa,
                                             bool lagged, QueryRegs<D, R>& Q) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = qbase + r * 64 + lane;
        float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
        float sh = lagged ? 0.f : -FLT_MAX;
        if (q < J.nq) {
            c = J.qrec[q];
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

// Combine two partials (m1, s1, b1) += (m2, s2, b2).
template <int D, bool LAGGED, bool BARY>
__device__ __forceinline__ void combine(float& m1, float& s1, float* b1, float m2, float s2,
                                        const float* b2) {
    if (LAGGED) {
        s1 += s2;
        if (BARY)
            for (int t = 0; t < D; ++t) b1[t] += b2[t];
    } else {
        const float mn = fmaxf(m1, m2);
        const float c1 = ex2(m1 - mn), c2 = ex2(m2 - mn);
        m1 = mn;
        s1 = s1 * c1 + s2 * c2;
        if (BARY)
            for (int t = 0; t < D; ++t) b1[t] = b1[t] * c1 + b2[t] * c2;
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
    if (J.out_rec) {
        const float lw = J.qlog2w ? J.qlog2w[q] : J.qlog2w_s;
        float* hp = reinterpret_cast<float*>(J.out_rec + q) + (D == 2 ? 2 : 3);
        *hp = __builtin_fmaf(nv, kappa, lw);
    }
    if (J.out_bary) {
        const float inv = -inv_sqrt_kappa / s;
#pragma unroll
        for (int t2 = 0; t2 < D; ++t2) J.out_bary[(size_t)q * D + t2] = b[t2] * inv;
    }
}

// Recompute the flagged rows with a tracked maximum over every key of the job,
// the whole block cooperating on one row at a time.
template <int D, bool BARY>
__device__ void rescue_rows(const Job& J, const int* flist, int nflag, float kappa,
                            float inv_kappa, float inv_sqrt_kappa) {
    __shared__ float red[kBlock * (2 + D)];
    for (int f = 0; f < nflag; ++f) {
        const int q = flist[f];
        const float4 qc = J.qrec[q];
        float m = -FLT_MAX, s = 0.f, b[D];
#pragma unroll
        for (int t = 0; t < D; ++t) b[t] = 0.f;
        for (int j = (int)threadIdx.x; j < J.nk; j += kBlock) {
            const float4 k = J.krec[j];
            const float dx = qc.x - k.x, dy = qc.y - k.y;
            float c = dy * dy;
            float dz = 0.f;
            if (D == 3) {
                dz = qc.z - k.z;
                c = __builtin_fmaf(dz, dz, c);
            }
            c = __builtin_fmaf(dx, dx, c);
            const float e = rec_h<D>(k) - c;
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

// Shared memory of one sweep work unit.
template <int D, int R>
struct SweepSmem {
    float part[kBlock * R * (2 + D)];  // wave-split partials / merge scratch
    int flist[kBlock * R];             // rows flagged for recomputation
    int nflag;
    int last;
};

// Finish (or flag) the rows held as (m, s, b) by this thread; rows of a lagged
// sweep whose sum is out of range go to the block's rescue list.
template <int D, bool LAGGED>
__device__ __forceinline__ void finish_or_flag(const Job& J, int q, float m, float s, const float* b,
                                               int* flist, int* nflag, float kappa, float inv_kappa,
                                               float inv_sqrt_kappa) {
    if (q >= J.nq) return;
    if (LAGGED && !(s >= kSumLo && s <= kSumHi)) {
        const int idx = atomicAdd(nflag, 1);
        flist[idx] = q;
        return;
    }
    finish_row<D>(J, q, m, s, b, kappa, inv_kappa, inv_sqrt_kappa);
}

// One work unit: queries of query-block qb, keys of split `split`.
//   QW = 4 / WS query groups of 64 R queries per block.
template <int D, int R, int WS, bool LAGGED, bool BARY, bool SEP = false, bool EXP = false>
__device__ __forceinline__ void sweep_unit(const Job& J, int qb, int split, float kappa,
                                           float inv_kappa, float inv_sqrt_kappa,
                                           SweepSmem<D, R>& sm) {
    static_assert(!EXP || (LAGGED && !BARY), "the expanded form serves lagged sweeps without offsets");
    constexpr int QW = 4 / WS;
    constexpr int NC = 2 + D;                  // components of a partial
    constexpr int QB = QW * 64 * R;            // queries per block
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    const int qwave = wave % QW;
    const int kpart = wave / QW;
    const int qblock0 = qb * QB;
    const int qbase = qblock0 + qwave * 64 * R;

    QueryRegs<D, R> Q;
    load_queries<D, R>(J, qbase, lane, kappa, LAGGED, Q);
    {
        const int s0 = split * J.kps;
        const int kpw = J.kps / WS;
        const int k0 = min(J.nkpad, s0 + kpart * kpw);
        const int k1 = min(J.nkpad, k0 + kpw);
        if constexpr (EXP) {
            // origin: the wave's first query (zero if the wave has none)
            float o[3] = {0.f, 0.f, 0.f};
            if (qbase < J.nq) {
                const float4 c0 = J.qrec[qbase];
                o[0] = c0.x;
                o[1] = c0.y;
                o[2] = D == 3 ? c0.z : 0.f;
            }
            float qsave[R][D], C[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float n = 0.f;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    qsave[r][t] = Q.q[r][t];
                    Q.q[r][t] -= o[t];
                    n = __builtin_fmaf(Q.q[r][t], Q.q[r][t], n);
                }
                C[r] = -n - Q.sh[r];
            }
            sweep_keys_expanded<D, R>(J.krec, k0, k1, o, C, Q);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int t = 0; t < D; ++t) Q.q[r][t] = qsave[r][t];
        } else {
            sweep_keys<D, R, LAGGED, BARY>(J.krec, k0, k1, Q);
        }
    }

    if (threadIdx.x == 0) sm.nflag = 0;
    // combine the WS wave partials of each query in LDS (waves with kpart 0 keep the result)
    if (WS > 1) {
        __syncthreads();
        if (kpart > 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float* P = sm.part + (((kpart - 1) * QW + qwave) * R + r) * 64 * NC + lane;
                P[0] = Q.sh[r];
                P[64] = Q.s[r];
                if (BARY)
                    for (int t = 0; t < D; ++t) P[(2 + t) * 64] = Q.b[r][t];
            }
        }
        __syncthreads();
        if (kpart == 0) {
            for (int kp = 1; kp < WS; ++kp) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float* P = sm.part + (((kp - 1) * QW + qwave) * R + r) * 64 * NC + lane;
                    float b2[D];
                    if (BARY)
                        for (int t = 0; t < D; ++t) b2[t] = P[(2 + t) * 64];
                    combine<D, LAGGED, BARY>(Q.sh[r], Q.s[r], Q.b[r], P[0], P[64], b2);
                }
            }
        }
    } else {
        __syncthreads();
    }

    if (J.splits == 1) {
        if (kpart == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                finish_or_flag<D, LAGGED>(J, qbase + r * 64 + lane, Q.sh[r], Q.s[r], Q.b[r],
                                          sm.flist, &sm.nflag, kappa, inv_kappa, inv_sqrt_kappa);
        }
    } else {
        // publish this block's partial, then the last block of the query block merges
        const int nqpad = J.nqb * QB;
        const size_t cstride = (size_t)J.splits * nqpad;
        if (kpart == 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float* P = J.part + (size_t)split * nqpad + qbase + r * 64 + lane;
                if (!LAGGED) P[0] = Q.sh[r];
                P[cstride] = Q.s[r];
                if (BARY)
                    for (int t = 0; t < D; ++t) P[(2 + t) * cstride] = Q.b[r][t];
            }
        }
        // separate-merge mode: a later kernel (k_merge) combines the splits
        if (SEP) return;
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned prev = atomicAdd(&J.ticket[qb], 1u);
            sm.last = (prev == (unsigned)(J.splits - 1));
        }
        __syncthreads();
        if (!sm.last) return;
        __threadfence();
        // all 256 threads merge: TPQ threads per query, splits strided among them
        constexpr int TPQ = (QB >= kBlock) ? 1 : kBlock / QB;
        constexpr int QPT = (QB >= kBlock) ? QB / kBlock : 1;
        const int sub = (int)threadIdx.x / (kBlock / TPQ * 1) % TPQ;
        const int slot = (int)threadIdx.x % (kBlock / TPQ);
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            const int ql = slot + u * (kBlock / TPQ);   // query index within the block
            const int q = qblock0 + ql;
            float m, s, b[D];
            if (LAGGED) m = (q < J.nq) ? -J.qpot[q] * kappa : 0.f;
            else m = -FLT_MAX;
            s = 0.f;
            for (int t = 0; t < D; ++t) b[t] = 0.f;
            for (int sp = sub; sp < J.splits; sp += TPQ) {
                const float* P = J.part + (size_t)sp * nqpad + q;
                float b2[D];
                if (BARY)
                    for (int t = 0; t < D; ++t) b2[t] = P[(2 + t) * cstride];
                combine<D, LAGGED, BARY>(m, s, b, LAGGED ? m : P[0], P[cstride], b2);
            }
            if (TPQ > 1) {
                float* S = sm.part + ((sub * (kBlock / TPQ) + slot) * NC);
                S[0] = m;
                S[1] = s;
                if (BARY)
                    for (int t = 0; t < D; ++t) S[2 + t] = b[t];
                __syncthreads();
                if (sub == 0) {
                    for (int k2 = 1; k2 < TPQ; ++k2) {
                        const float* S2 = sm.part + ((k2 * (kBlock / TPQ) + slot) * NC);
                        float b2[D];
                        if (BARY)
                            for (int t = 0; t < D; ++t) b2[t] = S2[2 + t];
                        combine<D, LAGGED, BARY>(m, s, b, S2[0], S2[1], b2);
                    }
                }
            }
            if (sub == 0)
                finish_or_flag<D, LAGGED>(J, q, m, s, b, sm.flist, &sm.nflag, kappa, inv_kappa,
                                          inv_sqrt_kappa);
        }
        if (threadIdx.x == 0) J.ticket[qb] = 0u;
    }
    if (LAGGED) {
        __syncthreads();
        const int nflag = sm.nflag;
        if (nflag > 0) rescue_rows<D, BARY>(J, sm.flist, nflag, kappa, inv_kappa, inv_sqrt_kappa);
    }
}

// Separate merge of the kMergeRows query rows q0.. of a job: the block's four
// waves take every fourth split in increasing order, their partials meet in LDS
// in wave order (a fixed order, so results are deterministic), wave 0 finishes
// or flags the rows, and flagged rows are recomputed by the whole block.
template <int D, bool LAGGED, bool BARY>
__device__ __forceinline__ void merge_block(const Job& J, int q0, int nqpad, float kappa,
                                            float inv_kappa, float inv_sqrt_kappa) {
    constexpr int NC = 2 + D;
    __shared__ float red[3 * NC * kMergeRows];
    __shared__ int flist[kMergeRows];
    __shared__ int nflag;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    const int q = q0 + lane;
    if (threadIdx.x == 0) nflag = 0;
    const size_t cstride = (size_t)J.splits * nqpad;
    float m = LAGGED ? (q < J.nq ? -J.qpot[q] * kappa : 0.f) : -FLT_MAX;
    float s = 0.f, b[D];
#pragma unroll
    for (int t = 0; t < D; ++t) b[t] = 0.f;
    if (q < J.nq) {
        // unrolled so that the loads of several splits are in flight together; the
        // partials are still combined in split order
#pragma unroll 8
        for (int sp = wave; sp < J.splits; sp += 4) {
            const float* P = J.part + (size_t)sp * nqpad + q;
            float b2[D];
            if (BARY)
                for (int t = 0; t < D; ++t) b2[t] = P[(2 + t) * cstride];
            combine<D, LAGGED, BARY>(m, s, b, LAGGED ? m : P[0], P[cstride], b2);
        }
    }
    if (wave > 0) {
        float* S = red + (wave - 1) * NC * kMergeRows + lane;
        S[0] = m;
        S[kMergeRows] = s;
        if (BARY)
            for (int t = 0; t < D; ++t) S[(2 + t) * kMergeRows] = b[t];
    }
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < 4; ++w) {
            const float* S = red + (w - 1) * NC * kMergeRows + lane;
            float b2[D];
            if (BARY)
                for (int t = 0; t < D; ++t) b2[t] = S[(2 + t) * kMergeRows];
            combine<D, LAGGED, BARY>(m, s, b, S[0], S[kMergeRows], b2);
        }
        finish_or_flag<D, LAGGED>(J, q, m, s, b, flist, &nflag, kappa, inv_kappa, inv_sqrt_kappa);
    }
    if (LAGGED) {
        __syncthreads();
        const int n = nflag;
        if (n > 0) rescue_rows<D, BARY>(J, flist, n, kappa, inv_kappa, inv_sqrt_kappa);
    }
}

}  // namespace ct
