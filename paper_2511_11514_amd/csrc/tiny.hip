// One-workgroup solve of a small Sinkhorn problem: the K iterations of the cross
// and self sweeps (Sec. II-B, eq. 5 solved by Sinkhorn's algorithm; eq. 6's self
// terms) in a single workgroup of 16 waves, with every point, potential and key
// term held in LDS.
//
// At the paper's shortest horizons (a few hundred samples) one iteration is
// tens of thousands to a few hundred thousand point pairs.  Spread over the GPU,
// such an iteration is bound by synchronisation: a kernel boundary, or a grid
// barrier, costs microseconds because it writes back and invalidates the caches
// of the dies.  One compute unit evaluates those pairs in a few microseconds by
// itself, and its waves synchronise through LDS with a block barrier, so the
// whole solve runs without touching global memory between its first load and
// its last store.
//
// Pairs are evaluated in the expanded form (lds_solve.h).  Each record array
// keeps the key term of one potential: x with f, y with g, and a ping-pong pair
// each for the averaged self updates (x with p, y with q).
//
// Work of a half-iteration: the jobs (f and p, or g and q) are cut into tasks of
// 64·R query rows (R per lane) times one key range, planned by a cost model of
// the compute unit (issue cycles per SIMD, LDS broadcasts, per-task set-up); the
// 16 waves take tasks round-robin.  Lanes sum their rows over the task's keys
// with the rows' lagged shifts, or, in a first iteration from zero, with a
// tracked maximum.  After a block barrier every row's partials are combined in
// key-range order (deterministic), the row finished (or, if its lagged sum left
// [2^-64, 2^64], recomputed with a tracked maximum by the thread that finishes
// it), and its new potential and key term written to LDS.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "ct_internal.h"
#include "lds_solve.h"

namespace ct {

namespace {

using namespace lds_solve;

template <int D, int R>
__global__ __launch_bounds__(kTinyThreads) void k_tiny(TinyArgs A) {
    extern __shared__ float4 lds4[];
    float* lds = reinterpret_cast<float*>(lds4);
    const int tid = (int)threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const float ninf = -__builtin_huge_valf();
    const float kap = A.kappa;

    // load: records (2v', H), norms, potentials
    for (int i = tid; i < A.T; i += kTinyThreads) {
        const float4 c = A.cx[i];
        const float n = norm2<D>(c);
        const float rx = 2.f * c.x, ry = 2.f * c.y, rz = D == 3 ? 2.f * c.z : 0.f;
        const float f = A.f[i];
        lds[A.o_f + i] = f;
        lds[A.o_nx + i] = n;
        lds4[A.o_rf + i] = make_float4(rx, ry, rz, __builtin_fmaf(f, kap, A.log2a) - n);
        if (A.debias) {
            const float p = A.p[i];
            lds[A.o_p + i] = p;
            lds4[A.o_rp + i] = make_float4(rx, ry, rz, __builtin_fmaf(p, kap, A.log2a) - n);
            lds4[A.o_rp + A.T + i] = make_float4(rx, ry, rz, ninf);
        }
    }
    for (int j = tid; j < A.M; j += kTinyThreads) {
        const float4 c = A.cy[j];
        const float n = norm2<D>(c);
        const float rx = 2.f * c.x, ry = 2.f * c.y, rz = D == 3 ? 2.f * c.z : 0.f;
        const float lb = A.log2b[j], g = A.g[j];
        lds[A.o_lb + j] = lb;
        lds[A.o_g + j] = g;
        lds[A.o_ny + j] = n;
        lds4[A.o_rg + j] = make_float4(rx, ry, rz, __builtin_fmaf(g, kap, lb) - n);
        if (A.ref_iter) {
            const float q = A.q[j];
            lds[A.o_q + j] = q;
            lds4[A.o_rq + j] = make_float4(rx, ry, rz, __builtin_fmaf(q, kap, lb) - n);
            lds4[A.o_rq + A.M + j] = make_float4(rx, ry, rz, ninf);
        }
    }
    __syncthreads();

    int cur = 0;   // current half of the self records' ping-pong
    for (int k = 0; k < A.iters; ++k) {
        const bool lagged = !A.safe_only && (A.lagged0 || k > 0);
        for (int h = 0; h < 2; ++h) {
            const int nj = A.njobs[h];
            // sweep: tasks round-robin over the waves
            for (int t = wave; t < A.ntasks[h]; t += kTinyWaves) {
                const int jj = (nj > 1 && t >= A.job[h][1].task0) ? 1 : 0;
                const TinyJob& J = A.job[h][jj];
                const int local = t - J.task0;
                const int grp = local % J.groups, split = local / J.groups;
                const int k0 = min(J.keys, split * J.kps), k1 = min(J.keys, k0 + J.kps);
                const float4* qr = lds4 + J.qrec + (J.avg ? cur * J.rows : 0);
                const float4* kr = lds4 + J.krec + (J.avg ? cur * J.keys : 0);
                float q[R][3], C[R], m[R], s[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // lanes past the last row repeat it; the combine never reads them
                    const int rc = min(grp * 64 * R + r * 64 + lane, J.rows - 1);
                    const float4 v = qr[rc];
                    q[r][0] = 0.5f * v.x;
                    q[r][1] = 0.5f * v.y;
                    q[r][2] = 0.5f * v.z;
                    m[r] = lagged ? -lds[J.qpot + rc] * kap : 0.f;
                    C[r] = -lds[J.qnorm + rc] - m[r];
                }
                if (lagged) sum_lagged<D, R>(kr, k0, k1, q, C, s);
                else sum_safe<D, R>(kr, k0, k1, q, C, m, s);
                float* ps = lds + A.o_ps + t * 64 * R + lane;
                float* pm = lds + A.o_pm + t * 64 * R + lane;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    ps[r * 64] = s[r];
                    if (!lagged) pm[r * 64] = m[r];
                }
            }
            __syncthreads();
            // combine and finish: one thread per row of the half-iteration's jobs.
            // Each thread selects its job's fields from two wave-uniform copies
            // (a per-thread index into the kernel arguments would read them
            // through vector memory).
            const TinyJob& J0 = A.job[h][0];
            const TinyJob& J1 = A.job[h][nj > 1 ? 1 : 0];
            const int rows0 = J0.rows;
            const int nrows = rows0 + (nj > 1 ? J1.rows : 0);
            const int q0 = J0.qrec + (J0.avg ? cur * J0.rows : 0);
            const int q1r = J1.qrec + (J1.avg ? cur * J1.rows : 0);
            const int k0r = J0.krec + (J0.avg ? cur * J0.keys : 0);
            const int k1r = J1.krec + (J1.avg ? cur * J1.keys : 0);
            const int o0 = J0.out_rec + (J0.avg ? (cur ^ 1) * J0.rows : 0);
            const int o1 = J1.out_rec + (J1.avg ? (cur ^ 1) * J1.rows : 0);
            for (int idx = tid; idx < nrows; idx += kTinyThreads) {
                const bool sec = idx >= rows0;
                const int row = sec ? idx - rows0 : idx;
                const int task0 = sec ? J1.task0 : J0.task0;
                const int groups = sec ? J1.groups : J0.groups;
                const int splits = sec ? J1.splits : J0.splits;
                const int qpot = sec ? J1.qpot : J0.qpot;
                const int qnorm = sec ? J1.qnorm : J0.qnorm;
                const int qlw = sec ? J1.qlw : J0.qlw;
                const int avg = sec ? J1.avg : J0.avg;
                const int grp = row / (64 * R);
                const int base = (task0 + grp) * 64 * R + (row - grp * 64 * R);
                const int stride = groups * 64 * R;
                const float* ps = lds + A.o_ps + base;
                const float* pm = lds + A.o_pm + base;
                const float old = lds[qpot + row];
                const float nrm = lds[qnorm + row];
                const float lw = qlw >= 0 ? lds[qlw + row] : A.log2a;
                float m, s = 0.f;
                if (lagged) {
                    m = -old * kap;
                    for (int sp = 0; sp < splits; ++sp) s += ps[sp * stride];
                } else {
                    m = ninf;
                    for (int sp = 0; sp < splits; ++sp) m = fmaxf(m, pm[sp * stride]);
                    for (int sp = 0; sp < splits; ++sp) {
                        const float mk = pm[sp * stride];
                        if (mk != ninf) s += ps[sp * stride] * tex2(mk - m);
                    }
                }
                if (lagged && !(s >= kLo && s <= kHi)) {
                    // the row's shift was unusable: recompute with a tracked maximum
                    const float4 v = lds4[(sec ? q1r : q0) + row];
                    const float qv[1][3] = {{0.5f * v.x, 0.5f * v.y, 0.5f * v.z}};
                    const float C1[1] = {-nrm};
                    float m1[1], s1[1];
                    sum_safe<D, 1>(lds4 + (sec ? k1r : k0r), 0, sec ? J1.keys : J0.keys, qv, C1,
                                   m1, s1);
                    m = m1[0];
                    s = s1[0];
                    atomicAdd(A.rescued, 1u);
                }
                const float tn = -(m + __log2f(s)) * A.inv_kappa;
                const float nv = avg ? 0.5f * (old + tn) : tn;
                lds[qpot + row] = nv;
                lds[4 * ((sec ? o1 : o0) + row) + 3] = __builtin_fmaf(nv, kap, lw) - nrm;
            }
            __syncthreads();
        }
        cur ^= 1;
    }

    // store: potentials and the key terms the final pass reads
    const int hofs = D == 2 ? 2 : 3;
    for (int i = tid; i < A.T; i += kTinyThreads) {
        const float f = lds[A.o_f + i];
        A.f[i] = f;
        reinterpret_cast<float*>(A.xrec_f + i)[hofs] = __builtin_fmaf(f, kap, A.log2a);
        if (A.debias) {
            const float p = lds[A.o_p + i];
            A.p[i] = p;
            reinterpret_cast<float*>(A.xrec_p + i)[hofs] = __builtin_fmaf(p, kap, A.log2a);
        }
    }
    for (int j = tid; j < A.M; j += kTinyThreads) {
        const float g = lds[A.o_g + j], lb = lds[A.o_lb + j];
        A.g[j] = g;
        reinterpret_cast<float*>(A.yrec_g + j)[hofs] = __builtin_fmaf(g, kap, lb);
        if (A.ref_iter) {
            const float q = lds[A.o_q + j];
            A.q[j] = q;
            reinterpret_cast<float*>(A.yrec_q + j)[hofs] = __builtin_fmaf(q, kap, lb);
        }
    }
}

// One candidate plan: rows per lane R and about `mult` tasks per wave in each
// half-iteration.  Fills the jobs, the layout and the modelled cycles.
void tiny_build(int T, int M, int d, bool debias, bool ref_iter, int R, int mult, TinyArgs& A,
                size_t& lds_bytes) {
    std::memset(&A, 0, sizeof(A));
    A.T = T;
    A.M = M;
    A.debias = debias;
    A.ref_iter = ref_iter;
    A.R = R;
    // record arrays (float4 units)
    int r4 = 0;
    A.o_rf = r4; r4 += T;
    A.o_rg = r4; r4 += M;
    A.o_rp = r4; r4 += debias ? 2 * T : 0;
    A.o_rq = r4; r4 += ref_iter ? 2 * M : 0;
    // floats after them
    int off = 4 * r4;
    auto take = [&](int n) {
        const int o = off;
        off += n;
        return o;
    };
    A.o_f = take(T);
    A.o_g = take(M);
    A.o_p = take(debias ? T : 0);
    A.o_q = take(ref_iter ? M : 0);
    A.o_lb = take(M);
    A.o_nx = take(T);
    A.o_ny = take(M);
    auto mk = [&](int rows, int keys, int qrec, int krec, int out_rec, int qnorm, int qpot,
                  int qlw, int avg) {
        TinyJob j;
        std::memset(&j, 0, sizeof(j));
        j.rows = rows; j.keys = keys; j.qrec = qrec; j.krec = krec; j.out_rec = out_rec;
        j.qnorm = qnorm; j.qpot = qpot; j.qlw = qlw; j.avg = avg;
        j.groups = (rows + 64 * R - 1) / (64 * R);
        return j;
    };
    A.njobs[0] = A.njobs[1] = 0;
    A.job[0][A.njobs[0]++] = mk(T, M, A.o_rf, A.o_rg, A.o_rf, A.o_nx, A.o_f, -1, 0);
    if (debias) A.job[0][A.njobs[0]++] = mk(T, T, A.o_rp, A.o_rp, A.o_rp, A.o_nx, A.o_p, -1, 1);
    A.job[1][A.njobs[1]++] = mk(M, T, A.o_rg, A.o_rf, A.o_rg, A.o_ny, A.o_g, A.o_lb, 0);
    if (ref_iter) A.job[1][A.njobs[1]++] = mk(M, M, A.o_rq, A.o_rq, A.o_rq, A.o_ny, A.o_q, A.o_lb, 1);

    // Cost model of one compute unit, in cycles: a wave's pass over one key is
    // R pairs of (d + 2) VALU instructions (2 cycles each for a wave64 on a SIMD)
    // and one exp (8 cycles on the transcendental unit); the four SIMDs each
    // run the tasks of their waves (wave w on SIMD w mod 4, task t on wave
    // t mod 16), and all waves share the LDS, which returns a 16-byte broadcast
    // to a wave in 8 cycles.  A task pays a fixed set-up (row loads, partial
    // stores); a half-iteration pays its combine (one row per thread, a read per
    // key range) and two block barriers.
    const double c_key = (double)R * (2.0 * (d + 2) + 8.0);
    const double c_task = 120.0 + 40.0 * R;
    const double c_lds = 8.0;
    double est = 0.0;
    int ntask_max = 0;
    for (int h = 0; h < 2; ++h) {
        double ptot = 0.0;
        for (int j = 0; j < A.njobs[h]; ++j)
            ptot += (double)A.job[h][j].groups * A.job[h][j].keys;
        const double ntarget = (double)kTinyWaves * mult;
        int t = 0, split_max = 1;
        for (int j = 0; j < A.njobs[h]; ++j) {
            TinyJob& J = A.job[h][j];
            // this job's share of the tasks, spread over its row groups
            const double share = ntarget * (double)J.keys / ptot;
            const int cap = std::max(1, (J.keys + 15) / 16);   // at least 16 keys per range
            const int sp = std::min(cap, std::max(1, (int)std::lround(share)));
            J.kps = (J.keys + sp - 1) / sp;
            J.splits = (J.keys + J.kps - 1) / J.kps;
            J.task0 = t;
            t += J.groups * J.splits;
            split_max = std::max(split_max, J.splits);
        }
        A.ntasks[h] = t;
        ntask_max = std::max(ntask_max, t);
        double simd[4] = {0.0, 0.0, 0.0, 0.0}, lds_cycles = 0.0;
        for (int j = 0; j < A.njobs[h]; ++j) {
            const TinyJob& J = A.job[h][j];
            for (int u = 0; u < J.groups * J.splits; ++u) {
                const int task = J.task0 + u;
                const int k0 = std::min(J.keys, (u / J.groups) * J.kps);
                const int nk = std::min(J.keys, k0 + J.kps) - k0;
                simd[task % 4] += c_task + nk * c_key;
                lds_cycles += nk * c_lds;
            }
        }
        const double sweep = std::max(std::max(std::max(simd[0], simd[1]), std::max(simd[2], simd[3])),
                                      lds_cycles);
        int nrows = 0;
        for (int j = 0; j < A.njobs[h]; ++j) nrows += A.job[h][j].rows;
        const double combine = ((nrows + kTinyThreads - 1) / kTinyThreads) * (80.0 + 16.0 * split_max);
        est += sweep + combine + 200.0;
    }
    A.ntask_max = ntask_max;
    A.o_ps = take(64 * R * ntask_max);
    A.o_pm = take(64 * R * ntask_max);
    A.est_cycles = est;
    lds_bytes = (size_t)off * sizeof(float);
}

}  // namespace

bool tiny_plan(int T, int M, int d, bool debias, bool ref_iter, size_t lds_cap, int r_force,
               TinyArgs& A, size_t& lds_bytes) {
    static const int Rs[] = {1, 2, 4};
    static const int mults[] = {1, 2, 3, 4, 6, 8};
    bool found = false;
    size_t smallest = 0;
    for (int R : Rs) {
        if (r_force && R != r_force) continue;
        for (int mult : mults) {
            TinyArgs C;
            size_t bytes = 0;
            tiny_build(T, M, d, debias, ref_iter, R, mult, C, bytes);
            if (smallest == 0 || bytes < smallest) smallest = bytes;
            if (bytes > lds_cap) continue;
            if (!found || C.est_cycles < A.est_cycles) {
                A = C;
                lds_bytes = bytes;
                found = true;
            }
        }
    }
    if (!found) lds_bytes = smallest;
    return found;
}

template <int D, int R>
static hipError_t launch_tiny_dr(const TinyArgs& A, size_t lds_bytes, hipStream_t s,
                                 hipEvent_t e0, hipEvent_t e1) {
    {
        const hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void*>(&k_tiny<D, R>), lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (e0)
        hipExtLaunchKernelGGL((k_tiny<D, R>), dim3(1), dim3(kTinyThreads), lds_bytes, s, e0, e1, 0, A);
    else
        hipLaunchKernelGGL((k_tiny<D, R>), dim3(1), dim3(kTinyThreads), lds_bytes, s, A);
    return hipGetLastError();
}

template <int D>
static hipError_t launch_tiny_d(const TinyArgs& A, size_t lds_bytes, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1) {
    switch (A.R) {
        case 1: return launch_tiny_dr<D, 1>(A, lds_bytes, s, e0, e1);
        case 2: return launch_tiny_dr<D, 2>(A, lds_bytes, s, e0, e1);
        default: return launch_tiny_dr<D, 4>(A, lds_bytes, s, e0, e1);
    }
}

hipError_t launch_tiny(int d, const TinyArgs& A, size_t lds_bytes, hipStream_t s) {
    hipEvent_t e0, e1;
    void* tok = profile_kernel_begin(&e0, &e1);
    const double pairs = (double)A.iters * ((double)A.T * A.M * 2 + (A.debias ? (double)A.T * A.T : 0.0) +
                                            (A.ref_iter ? (double)A.M * A.M : 0.0));
    const hipError_t e = d == 2 ? launch_tiny_d<2>(A, lds_bytes, s, e0, e1)
                                : launch_tiny_d<3>(A, lds_bytes, s, e0, e1);
    // kind 30/31: a one-workgroup solve (safe / lagged from its first iteration); code: R
    profile_kernel_end(tok, 30 + A.lagged0, 0, A.R, 1, pairs);
    return e;
}

}  // namespace ct
