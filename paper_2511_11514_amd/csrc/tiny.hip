// One-workgroup solve of a small Sinkhorn problem: the K iterations of the cross
// and self sweeps (Sec. II-B, eq. 5 solved by Sinkhorn's algorithm; eq. 6's self
// terms) in a single workgroup of 16 waves, with every point, potential and key
// term held in LDS.
//
// At the paper's shortest horizons (a few hundred samples) one iteration is
// tens of thousands of point pairs.  Spread over the GPU, such an iteration is
// bound by synchronisation: a kernel boundary, or a grid barrier, costs
// microseconds because it writes back and invalidates the caches of all eight
// dies.  One compute unit evaluates those pairs in a few microseconds by itself,
// and its waves synchronise through LDS with a block barrier, so the whole solve
// runs without touching global memory between its first load and its last store.
//
// Work of a half-iteration: the jobs (f and p, or g and q) are cut into tasks of
// 64 query rows (one per lane) times one key range; the 16 waves take tasks
// round-robin, each lane summing its row over the task's keys (read from LDS as
// broadcasts) with the row's lagged shift, or, in the first iteration from zero,
// with a running maximum.  After a block barrier every row's partials are
// combined in key-range order (deterministic), the row finished (or, if its
// lagged sum left [2^-64, 2^64], recomputed with a tracked maximum by the thread
// that finishes it), and its new potential and key term written to LDS.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstring>

#include "ct_internal.h"

namespace ct {

namespace {

constexpr float kLo = 5.421010862427522e-20f;   // 2^-64
constexpr float kHi = 1.8446744073709552e19f;   // 2^64

__device__ __forceinline__ float tex2(float v) { return __builtin_amdgcn_exp2f(v); }

// |a - b|^2 + c
template <int D>
__device__ __forceinline__ float sqd(const float4& a, const float4& b, float c = 0.f) {
    const float dx = a.x - b.x, dy = a.y - b.y;
    c = __builtin_fmaf(dy, dy, c);
    if (D == 3) {
        const float dz = a.z - b.z;
        c = __builtin_fmaf(dz, dz, c);
    }
    return __builtin_fmaf(dx, dx, c);
}

// Sum of one row over keys [k0, k1) with the shift folded into the cost.
template <int D>
__device__ __forceinline__ float row_lagged(const float4& qc, float sh, const float4* kc,
                                            const float* kh, int k0, int k1) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int j = k0;
    for (; j + 4 <= k1; j += 4) {
        s0 += tex2(kh[j] - sqd<D>(qc, kc[j], sh));
        s1 += tex2(kh[j + 1] - sqd<D>(qc, kc[j + 1], sh));
        s2 += tex2(kh[j + 2] - sqd<D>(qc, kc[j + 2], sh));
        s3 += tex2(kh[j + 3] - sqd<D>(qc, kc[j + 3], sh));
    }
    for (; j < k1; ++j) s0 += tex2(kh[j] - sqd<D>(qc, kc[j], sh));
    return (s0 + s1) + (s2 + s3);
}

// Maximum and shifted sum of one row over keys [k0, k1) (two passes).
template <int D>
__device__ __forceinline__ void row_safe(const float4& qc, const float4* kc, const float* kh,
                                         int k0, int k1, float& m, float& s) {
    m = -__builtin_huge_valf();
    for (int j = k0; j < k1; ++j) m = fmaxf(m, kh[j] - sqd<D>(qc, kc[j]));
    s = 0.f;
    if (m == -__builtin_huge_valf()) return;
    for (int j = k0; j < k1; ++j) s += tex2(kh[j] - sqd<D>(qc, kc[j]) - m);
}

template <int D>
__global__ __launch_bounds__(kTinyThreads) void k_tiny(TinyArgs A) {
    extern __shared__ float lds[];
    float4* X = reinterpret_cast<float4*>(lds + A.o_x);
    float4* Y = reinterpret_cast<float4*>(lds + A.o_y);
    const int tid = (int)threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const float ninf = -__builtin_huge_valf();

    // load: coordinates, masses, potentials; key terms from the potentials
    for (int i = tid; i < A.T; i += kTinyThreads) {
        X[i] = A.cx[i];
        const float f = A.f[i], p = A.p[i];
        lds[A.o_f + i] = f;
        lds[A.o_p + i] = p;
        lds[A.o_hf + i] = __builtin_fmaf(f, A.kappa, A.log2a);
        lds[A.o_hp + i] = __builtin_fmaf(p, A.kappa, A.log2a);
        lds[A.o_hp + A.T + i] = ninf;
    }
    for (int j = tid; j < A.M; j += kTinyThreads) {
        Y[j] = A.cy[j];
        const float lb = A.log2b[j], g = A.g[j], q = A.q[j];
        lds[A.o_lb + j] = lb;
        lds[A.o_g + j] = g;
        lds[A.o_q + j] = q;
        lds[A.o_hg + j] = __builtin_fmaf(g, A.kappa, lb);
        lds[A.o_hq + j] = __builtin_fmaf(q, A.kappa, lb);
        lds[A.o_hq + A.M + j] = ninf;
    }
    __syncthreads();

    int cur = 0;   // current half of the self key-term ping-pong
    for (int k = 0; k < A.iters; ++k) {
        const bool lagged = !A.safe_only && (A.lagged0 || k > 0);
        for (int h = 0; h < 2; ++h) {
            // the self jobs read the current key terms and write the other half
            const int nj = A.njobs[h];
            // sweep: tasks round-robin over the waves
            for (int t = wave; t < A.ntasks[h]; t += kTinyWaves) {
                const int jj = (nj > 1 && t >= A.job[h][1].task0) ? 1 : 0;
                const TinyJob& J = A.job[h][jj];
                const int local = t - J.task0;
                const int grp = local % J.groups, split = local / J.groups;
                const int row = grp * 64 + lane;
                const int k0 = min(J.keys, split * J.kps), k1 = min(J.keys, k0 + J.kps);
                const float4* kc = reinterpret_cast<const float4*>(lds + J.kc);
                const float* kh = lds + J.kh + (J.avg ? cur * J.keys : 0);
                float m = 0.f, s = 0.f;
                if (row < J.rows) {
                    const float4 qc = reinterpret_cast<const float4*>(lds + J.qc)[row];
                    if (lagged) {
                        m = -lds[J.qpot + row] * A.kappa;
                        s = row_lagged<D>(qc, m, kc, kh, k0, k1);
                    } else {
                        row_safe<D>(qc, kc, kh, k0, k1, m, s);
                    }
                }
                lds[A.o_ps + t * 64 + lane] = s;
                lds[A.o_pm + t * 64 + lane] = m;
            }
            __syncthreads();
            // combine and finish: one thread per row
            for (int jj = 0; jj < nj; ++jj) {
                const TinyJob& J = A.job[h][jj];
                const float* kh = lds + J.kh + (J.avg ? cur * J.keys : 0);
                for (int row = tid; row < J.rows; row += kTinyThreads) {
                    const int grp = row >> 6, ln = row & 63;
                    float m, s = 0.f;
                    if (lagged) {
                        m = lds[A.o_pm + (J.task0 + grp) * 64 + ln];
                        for (int sp = 0; sp < J.splits; ++sp)
                            s += lds[A.o_ps + (J.task0 + sp * J.groups + grp) * 64 + ln];
                    } else {
                        m = ninf;
                        for (int sp = 0; sp < J.splits; ++sp)
                            m = fmaxf(m, lds[A.o_pm + (J.task0 + sp * J.groups + grp) * 64 + ln]);
                        for (int sp = 0; sp < J.splits; ++sp) {
                            const int o = (J.task0 + sp * J.groups + grp) * 64 + ln;
                            const float mk = lds[A.o_pm + o];
                            if (mk != ninf) s += lds[A.o_ps + o] * tex2(mk - m);
                        }
                    }
                    if (lagged && !(s >= kLo && s <= kHi)) {
                        // the row's shift was unusable: recompute with a tracked maximum
                        const float4 qc = reinterpret_cast<const float4*>(lds + J.qc)[row];
                        row_safe<D>(qc, reinterpret_cast<const float4*>(lds + J.kc), kh, 0,
                                    J.keys, m, s);
                        atomicAdd(A.rescued, 1u);
                    }
                    const float t = -(m + __log2f(s)) * A.inv_kappa;
                    const float old = lds[J.qpot + row];
                    const float nv = J.avg ? 0.5f * (old + t) : t;
                    lds[J.qpot + row] = nv;
                    const float lw = J.qlw >= 0 ? lds[J.qlw + row] : A.log2a;
                    lds[J.out_h + (J.avg ? (cur ^ 1) * J.rows : 0) + row] =
                        __builtin_fmaf(nv, A.kappa, lw);
                }
            }
            __syncthreads();
        }
        cur ^= 1;
    }

    // store: potentials and the key terms the final pass reads
    const int hofs = D == 2 ? 2 : 3;
    for (int i = tid; i < A.T; i += kTinyThreads) {
        A.f[i] = lds[A.o_f + i];
        A.p[i] = lds[A.o_p + i];
        reinterpret_cast<float*>(A.xrec_f + i)[hofs] = lds[A.o_hf + i];
        if (A.debias) reinterpret_cast<float*>(A.xrec_p + i)[hofs] = lds[A.o_hp + cur * A.T + i];
    }
    for (int j = tid; j < A.M; j += kTinyThreads) {
        A.g[j] = lds[A.o_g + j];
        A.q[j] = lds[A.o_q + j];
        reinterpret_cast<float*>(A.yrec_g + j)[hofs] = lds[A.o_hg + j];
        if (A.ref_iter) reinterpret_cast<float*>(A.yrec_q + j)[hofs] = lds[A.o_hq + cur * A.M + j];
    }
}

}  // namespace

// Plans the tasks and the LDS layout; false if the problem does not fit.
bool tiny_plan(int T, int M, int d, bool debias, bool ref_iter, TinyArgs& A, size_t& lds_bytes) {
    (void)d;
    std::memset(&A, 0, sizeof(A));
    A.T = T;
    A.M = M;
    A.debias = debias;
    A.ref_iter = ref_iter;
    int off = 0;
    auto take = [&](int n) {
        const int o = off;
        off += (n + 3) & ~3;   // keep float4 arrays 16-byte aligned
        return o;
    };
    A.o_x = take(4 * T);
    A.o_y = take(4 * M);
    A.o_lb = take(M);
    A.o_f = take(T);
    A.o_g = take(M);
    A.o_p = take(T);
    A.o_q = take(M);
    A.o_hf = take(T);
    A.o_hg = take(M);
    A.o_hp = take(2 * T);
    A.o_hq = take(2 * M);
    // jobs: half 0 = f (rows x, keys y) [+ p (rows x, keys x)]; half 1 = g [+ q]
    auto mk = [&](int rows, int keys, int qc, int kc, int kh, int qpot, int out_h, int qlw,
                  int avg) {
        TinyJob j;
        std::memset(&j, 0, sizeof(j));
        j.rows = rows; j.keys = keys; j.qc = qc; j.kc = kc; j.kh = kh; j.qpot = qpot;
        j.out_h = out_h; j.qlw = qlw; j.avg = avg;
        j.groups = (rows + 63) / 64;
        return j;
    };
    A.njobs[0] = A.njobs[1] = 0;
    A.job[0][A.njobs[0]++] = mk(T, M, A.o_x, A.o_y, A.o_hg, A.o_f, A.o_hf, -1, 0);
    if (debias) A.job[0][A.njobs[0]++] = mk(T, T, A.o_x, A.o_x, A.o_hp, A.o_p, A.o_hp, -1, 1);
    A.job[1][A.njobs[1]++] = mk(M, T, A.o_y, A.o_x, A.o_hf, A.o_g, A.o_hg, A.o_lb, 0);
    if (ref_iter) A.job[1][A.njobs[1]++] = mk(M, M, A.o_y, A.o_y, A.o_hq, A.o_q, A.o_hq, A.o_lb, 1);
    // key ranges: enough tasks to give every wave one, at least 64 keys per range
    int ntask_max = 0;
    for (int h = 0; h < 2; ++h) {
        int groups = 0;
        for (int j = 0; j < A.njobs[h]; ++j) groups += A.job[h][j].groups;
        int t = 0;
        for (int j = 0; j < A.njobs[h]; ++j) {
            TinyJob& J = A.job[h][j];
            const int want = std::max(1, kTinyWaves / groups);
            const int cap = std::max(1, (J.keys + 63) / 64);
            J.splits = std::min(want, cap);
            J.kps = (J.keys + J.splits - 1) / J.splits;
            J.task0 = t;
            t += J.groups * J.splits;
        }
        A.ntasks[h] = t;
        ntask_max = std::max(ntask_max, t);
    }
    A.ntask_max = ntask_max;
    A.o_ps = take(64 * ntask_max);
    A.o_pm = take(64 * ntask_max);
    lds_bytes = (size_t)off * sizeof(float);
    return lds_bytes <= kTinyMaxLds;
}

hipError_t launch_tiny(int d, const TinyArgs& A, size_t lds_bytes, hipStream_t s) {
    hipEvent_t e0, e1;
    void* tok = profile_kernel_begin(&e0, &e1);
    const double pairs = (double)A.iters * ((double)A.T * A.M * 2 + (A.debias ? (double)A.T * A.T : 0.0) +
                                            (A.ref_iter ? (double)A.M * A.M : 0.0));
    if (d == 2) {
        if (e0) hipExtLaunchKernelGGL(k_tiny<2>, dim3(1), dim3(kTinyThreads), lds_bytes, s, e0, e1, 0, A);
        else hipLaunchKernelGGL(k_tiny<2>, dim3(1), dim3(kTinyThreads), lds_bytes, s, A);
    } else {
        if (e0) hipExtLaunchKernelGGL(k_tiny<3>, dim3(1), dim3(kTinyThreads), lds_bytes, s, e0, e1, 0, A);
        else hipLaunchKernelGGL(k_tiny<3>, dim3(1), dim3(kTinyThreads), lds_bytes, s, A);
    }
    // kind 30/31: a one-workgroup solve (safe / lagged from its first iteration)
    profile_kernel_end(tok, 30 + A.lagged0, 0, 0, 1, pairs);
    return hipGetLastError();
}

}  // namespace ct
