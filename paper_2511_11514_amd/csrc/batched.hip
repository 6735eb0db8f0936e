// ct_sinkhorn_grad_batched: many independent Sinkhorn-divergence gradients of
// uneven size (the per-problem definitions of sinkhorn.hip).
//
// Two executions of the same schedule of updates:
//  * lockstep (default): per iteration two launches over job tables prepared in
//    the workspace, A = every problem's f update and self updates, B = every
//    problem's g update, then the extrapolation launches F1 and F2; each job is
//    split over keys so that all blocks of a launch sweep about the same number
//    of pairs (lockstep.hip), split jobs merged by a second kernel;
//  * persistent (CT_PERSISTENT): one launch walking a dependency-ordered work
//    list, described next;
//  * exchange (CT_MESH, and by default whenever every problem's points fit in
//    one workgroup's LDS and all their blocks fit on the device at once): one
//    launch of the exchange solve of mesh.hip for every problem (each problem's
//    blocks pass their rows' potentials to each other as versioned words), then
//    the lockstep extrapolation launches.
//
// Work list.  Every problem runs the same stage sequence
//     A_0, B_0, A_1, B_1, ..., A_{K-1}, B_{K-1}, F1, F2
// (A: f update + first halves of the self updates, B: g update + second halves,
// F1: f+ and p+ with offsets, F2: g+ and q+).  A stage of a problem is a set of
// units, one per (job, block of queries), each sweeping all keys of its problem
// (no key splits: the parallelism comes from the number of problems), so a unit
// writes final rows and needs no merge.  Units are numbered stage-major, and
// within a stage problem by problem in decreasing order of work (longest
// processing time first).  Blocks claim units in increasing order from one
// atomic counter; a unit of stage s of problem b waits until problem b has
// completed every unit of its earlier stages (a per-problem completion counter).
// Every unit a block waits for has a smaller number, hence was claimed earlier by
// a running block that itself waits only on smaller numbers: the waits cannot
// form a cycle, and every block leaves when the counter passes the last unit.
//
// The host builds the per-problem table once (ct_sinkhorn_batched_prepare) and
// copies it into the workspace; ct_sinkhorn_grad_batched then only enqueues
// kernels, so it can be captured into a graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "ct_internal.h"
#include "sweep_device.h"

namespace ct {

namespace {
constexpr double kLog2e = 1.4426950408889634;
}

struct BProb {
    int T, M;          // sizes
    int xo, yo;        // first point of the problem in x / y
    int xp, yp;        // first record of the problem in the padded record arrays
    int Tpad, Mpad;
    int nA, nB, nF1, nF2;  // units per stage
    int uA[5], uB[5];      // unit prefix of the stage's jobs (f|p1|q1 and g|p2|q2)
    int uF1[3], uF2[3];    // f+|p+ and g+|q+
    float log2a;
};

struct BHeader {
    int B, K, d, R, WS;
    int debias, need_ref;
    int total_units;
    int TA, TB, TF1, TF2;   // units of one stage over all problems
    int sumTpad, sumMpad, sumT, sumM;
    unsigned long long signature;
};

// Lockstep job tables: kinds A (self ping-pong cur = 0), A (cur = 1), B, F1, F2,
// each with room for three jobs per problem.
constexpr int kLockKinds = 5;
struct LockInfo {
    int njobs[kLockKinds], nblocks[kLockKinds], nmerge[kLockKinds];
    Schedule sc;            // the schedule the tables were planned for
};
// Default lockstep schedule: four queries per lane, keys split over the four
// waves of a block, about eight blocks per CU of equal work per launch; a tuned
// entry under the (d, 1, 0) key of the tuning table replaces it.
constexpr Schedule kLockSchedule{4, 4, 8, 1};

static Schedule lock_schedule(int d) {
    Schedule s;
    if (tuning_lookup(d, 1, 0, s) && (s.R == 1 || s.R == 2 || s.R == 4) && (s.WS == 2 || s.WS == 4))
        return Schedule{s.R, s.WS, s.blocks_per_cu, 1};
    return kLockSchedule;
}

// Device-side view of the prepared workspace.
struct BLayout {
    BHeader* hdr;
    BProb* prob;            // [B] in original order
    int* order;             // [B] LPT order -> problem id
    int* preA;              // [B+1] unit prefix over the LPT order, stage type A
    int* preB;
    int* preF1;
    int* preF2;
    int* xoff;              // [B+1] padded x record offsets (for staging lookups)
    int* yoff;
    Job* ljobs;             // [kLockKinds][3B] lockstep job tables
    int* lblk;              // [kLockKinds][3B] sweep-block prefix ends
    int* lmrg;              // [kLockKinds][3B] merge-block prefix ends
    MeshArgs* mtab;         // [B] exchange-solve arguments per problem
    int* mblk;              // [B] exchange-solve block prefix ends
    float* lpart;           // partial sums of split lockstep jobs (one launch at a time)
    unsigned* done;         // [B] completed units per problem
    unsigned* head;         // [1] next unit
    unsigned* counters;     // [4]
    double* wsum;           // [B]
    float* origin;          // [B][4] per-problem origin subtracted before scaling
    float4 *cx, *cy;        // query coordinates
    float4* xrec[4];        // as in the plain path, per problem at offset xp
    float4* yrec[3];
    float *b, *log2b;
    float *f, *g, *p, *q, *fp, *gp, *pp, *qp;
    float *dy, *ds;
    unsigned long long* xch;   // [4 (sumT + sumM)] versioned words of the exchange solve
    size_t bytes;
    size_t table_bytes;     // bytes of the host-built table (header .. mblk)
};

static BLayout b_layout(void* ws, int B, int64_t sumT, int64_t sumM, int64_t sumTpad,
                        int64_t sumMpad, int d, size_t part_floats) {
    Arena a(ws);
    BLayout L;
    L.hdr = a.take<BHeader>(1);
    L.prob = a.take<BProb>(B);
    L.order = a.take<int>(B);
    L.preA = a.take<int>(B + 1);
    L.preB = a.take<int>(B + 1);
    L.preF1 = a.take<int>(B + 1);
    L.preF2 = a.take<int>(B + 1);
    L.xoff = a.take<int>(B + 1);
    L.yoff = a.take<int>(B + 1);
    L.ljobs = a.take<Job>((size_t)kLockKinds * 3 * B);
    L.lblk = a.take<int>((size_t)kLockKinds * 3 * B);
    L.lmrg = a.take<int>((size_t)kLockKinds * 3 * B);
    L.mtab = a.take<MeshArgs>(B);
    L.mblk = a.take<int>(B);
    L.table_bytes = a.off;
    L.lpart = a.take<float>(part_floats);
    L.done = a.take<unsigned>(B);
    L.head = a.take<unsigned>(1);
    L.counters = a.take<unsigned>(4);
    L.wsum = a.take<double>(B);
    L.origin = a.take<float>((size_t)B * 4);
    L.cx = a.take<float4>(sumT);
    L.cy = a.take<float4>(sumM);
    for (int r = 0; r < 4; ++r) L.xrec[r] = a.take<float4>(sumTpad);
    for (int r = 0; r < 3; ++r) L.yrec[r] = a.take<float4>(sumMpad);
    L.b = a.take<float>(sumM);
    L.log2b = a.take<float>(sumM);
    L.f = a.take<float>(sumT);
    L.g = a.take<float>(sumM);
    L.p = a.take<float>(sumT);
    L.q = a.take<float>(sumM);
    L.fp = a.take<float>(sumT);
    L.gp = a.take<float>(sumM);
    L.pp = a.take<float>(sumT);
    L.qp = a.take<float>(sumM);
    L.dy = a.take<float>((size_t)sumT * d);
    L.ds = a.take<float>((size_t)sumT * d);
    L.xch = a.take<unsigned long long>(4 * ((size_t)sumT + sumM));
    L.bytes = a.off + 256;
    return L;
}

// ------------------------------------------------------------------ staging

__device__ __forceinline__ int find_prob(const int* off, int B, int e) {
    int lo = 0, hi = B - 1;   // largest b with off[b] <= e
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One block per problem: the sum of its reference weights and the common origin
// of its points (mean of every finite coordinate of its T + M points), both in
// double, fixed order.  The origin plays the part it plays in the single-problem
// path: subtracted before the float32 prescale by sqrt(kappa), so points far
// from the coordinate origin keep the low bits of their differences.
__global__ __launch_bounds__(256) void k_bwsum(BLayout L, const float* __restrict__ x,
                                               const float* __restrict__ y,
                                               const float* __restrict__ w, int d) {
    __shared__ double red[5][256];
    const BProb P = L.prob[blockIdx.x];
    double s = 0.0, c[3] = {0.0, 0.0, 0.0}, n = 0.0;
    if (w) {
        for (int j = threadIdx.x; j < P.M; j += 256) s += (double)w[P.yo + j];
    } else {
        s = threadIdx.x == 0 ? (double)P.M : 0.0;
    }
    for (int i = threadIdx.x; i < P.T + P.M; i += 256) {
        const float* pt = i < P.T ? x + (size_t)(P.xo + i) * d : y + (size_t)(P.yo + i - P.T) * d;
        bool ok = true;
        for (int t = 0; t < d; ++t) ok = ok && isfinite(pt[t]);
        if (!ok) continue;
        for (int t = 0; t < d; ++t) c[t] += (double)pt[t];
        n += 1.0;
    }
    red[0][threadIdx.x] = s;
    for (int t = 0; t < 3; ++t) red[1 + t][threadIdx.x] = c[t];
    red[4][threadIdx.x] = n;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) {
        const double cnt = red[4][0] > 0.0 ? red[4][0] : 1.0;
        L.origin[(size_t)blockIdx.x * 4 + threadIdx.x] =
            (int)threadIdx.x < d ? (float)(red[1 + threadIdx.x][0] / cnt) : 0.f;
    }
    if (threadIdx.x == 0) {
        L.wsum[blockIdx.x] = red[0][0];
        L.done[blockIdx.x] = 0u;
        if (blockIdx.x == 0) {
            *L.head = 0u;
            for (int k = 0; k < 4; ++k) L.counters[k] = 0u;
        }
    }
}

__device__ __forceinline__ float4 brec(const float* c, int d, float h) {
    return d == 2 ? make_float4(c[0], c[1], h, 0.f) : make_float4(c[0], c[1], c[2], h);
}

__global__ __launch_bounds__(256) void k_bstage(BLayout L, const float* __restrict__ x,
                                                const float* __restrict__ y,
                                                const float* __restrict__ w, float sqrt_kappa,
                                                float kappa) {
    const BHeader H = *L.hdr;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int d = H.d;
    const float ninf = -__builtin_huge_valf();
    if (e < H.sumTpad) {
        const int b = find_prob(L.xoff, H.B, e);
        const BProb P = L.prob[b];
        const int i = e - P.xp;
        float c[3] = {0.f, 0.f, 0.f};
        if (i < P.T) {
            const int gi = P.xo + i;
            for (int t = 0; t < d; ++t)
                c[t] = (x[(size_t)gi * d + t] - L.origin[(size_t)b * 4 + t]) * sqrt_kappa;
            L.cx[gi] = make_float4(c[0], c[1], c[2], 0.f);
            L.f[gi] = 0.f;
            L.p[gi] = 0.f;
            L.fp[gi] = 0.f;
            L.pp[gi] = 0.f;
            L.xrec[0][e] = brec(c, d, ninf);
            L.xrec[1][e] = brec(c, d, ninf);
            L.xrec[2][e] = brec(c, d, P.log2a);
            L.xrec[3][e] = brec(c, d, ninf);
        } else {
            for (int r = 0; r < 4; ++r) L.xrec[r][e] = brec(c, d, ninf);
        }
    }
    if (e < H.sumMpad) {
        const int b = find_prob(L.yoff, H.B, e);
        const BProb P = L.prob[b];
        const int j = e - P.yp;
        float c[3] = {0.f, 0.f, 0.f};
        if (j < P.M) {
            const int gj = P.yo + j;
            for (int t = 0; t < d; ++t)
                c[t] = (y[(size_t)gj * d + t] - L.origin[(size_t)b * 4 + t]) * sqrt_kappa;
            L.cy[gj] = make_float4(c[0], c[1], c[2], 0.f);
            const float wj = w ? w[gj] : 1.f;
            if (!(wj > 0.f) || !isfinite(wj)) atomicAdd(L.counters, 1u);
            const float bj = (float)((double)wj / L.wsum[b]);
            const float lb = __log2f(bj);
            L.b[gj] = bj;
            L.log2b[gj] = lb;
            L.g[gj] = 0.f;
            L.q[gj] = 0.f;
            L.gp[gj] = 0.f;
            L.qp[gj] = 0.f;
            L.yrec[0][e] = brec(c, d, lb);
            L.yrec[1][e] = brec(c, d, lb);
            L.yrec[2][e] = brec(c, d, ninf);
        } else {
            for (int r = 0; r < 3; ++r) L.yrec[r][e] = brec(c, d, ninf);
        }
    }
}

// ------------------------------------------------------------------ persistent kernel

struct BArgs {
    BLayout L;
    float kappa, inv_kappa, inv_sqrt_kappa;
    int safe_only;
    unsigned wait_polls;   // polls of a dependency counter before the wait gives up
};

// Build the job of unit `local` of stage type `st` (0 A, 1 B, 2 F1, 3 F2) of problem P.
template <int D>
__device__ __forceinline__ void unit_job(const BArgs& A, const BHeader& H, const BProb& P, int st,
                                         int cur, int local, Job& J, int& qb) {
    const BLayout& L = A.L;
    J.rescued = L.counters + 1;
    J.splits = 1;
    J.part = nullptr;
    J.ticket = nullptr;
    J.qlog2w = nullptr;
    J.qlog2w_s = P.log2a;
    J.self_avg = 0;
    J.out_rec = nullptr;
    J.out_bary = nullptr;
    const int QB = 64 * H.R * (4 / H.WS);
    const int* pre = st == 0 ? P.uA : st == 1 ? P.uB : st == 2 ? P.uF1 : P.uF2;
    const int njobs = st < 2 ? 3 : 2;
    int jt = 0;
    while (jt + 1 < njobs && local >= pre[jt + 1]) ++jt;
    qb = local - pre[jt];
    // job kinds: 0 cross from x (f), 1 self x (p), 2 self y (q), 3 cross from y (g)
    int kind, q0 = 0, nq;
    if (st == 0) {
        kind = jt == 0 ? 0 : jt == 1 ? 1 : 2;
        nq = kind == 0 ? P.T : kind == 1 ? P.T / 2 : P.M / 2;
    } else if (st == 1) {
        kind = jt == 0 ? 3 : jt == 1 ? 1 : 2;
        if (kind == 3) nq = P.M;
        else if (kind == 1) { q0 = P.T / 2; nq = P.T - P.T / 2; }
        else { q0 = P.M / 2; nq = P.M - P.M / 2; }
    } else if (st == 2) {
        kind = jt == 0 ? 0 : 1;
        nq = P.T;
    } else {
        kind = jt == 0 ? 3 : 2;
        nq = P.M;
    }
    const bool fin = st >= 2;
    if (kind == 0) {           // queries x vs keys y (g records)
        J.qrec = L.cx + P.xo; J.qpot = L.f + P.xo;
        J.krec = L.yrec[0] + P.yp; J.nk = P.M; J.nkpad = P.Mpad;
        J.out_pot = fin ? L.fp + P.xo : L.f + P.xo;
        J.out_rec = fin ? L.xrec[1] + P.xp : L.xrec[0] + P.xp;
        if (fin) J.out_bary = L.dy + (size_t)P.xo * D;
    } else if (kind == 1) {    // queries x vs keys x (p records)
        J.qrec = L.cx + P.xo; J.qpot = L.p + P.xo;
        J.krec = L.xrec[2 + cur] + P.xp; J.nk = P.T; J.nkpad = P.Tpad;
        if (fin) {
            J.out_pot = L.pp + P.xo;
            J.out_bary = L.ds + (size_t)P.xo * D;
        } else {
            J.self_avg = 1;
            J.out_pot = L.p + P.xo;
            J.out_rec = L.xrec[2 + (cur ^ 1)] + P.xp;
        }
    } else if (kind == 2) {    // queries y vs keys y (q records)
        J.qrec = L.cy + P.yo; J.qpot = L.q + P.yo; J.qlog2w = L.log2b + P.yo;
        J.krec = L.yrec[1 + cur] + P.yp; J.nk = P.M; J.nkpad = P.Mpad;
        if (fin) {
            J.out_pot = L.qp + P.yo;
        } else {
            J.self_avg = 1;
            J.out_pot = L.q + P.yo;
            J.out_rec = L.yrec[1 + (cur ^ 1)] + P.yp;
        }
    } else {                   // queries y vs keys x (f or f+ records)
        J.qrec = L.cy + P.yo; J.qpot = L.g + P.yo; J.qlog2w = L.log2b + P.yo;
        J.krec = (fin ? L.xrec[1] : L.xrec[0]) + P.xp; J.nk = P.T; J.nkpad = P.Tpad;
        J.out_pot = fin ? L.gp + P.yo : L.g + P.yo;
        J.out_rec = fin ? nullptr : L.yrec[0] + P.yp;
    }
    if (q0) {
        J.qrec += q0;
        J.qpot += q0;
        if (J.qlog2w) J.qlog2w += q0;
        J.out_pot += q0;
        if (J.out_rec) J.out_rec += q0;
    }
    J.nq = nq;
    J.nqb = (nq + QB - 1) / QB;
    J.kps = J.nkpad;
}

__device__ __forceinline__ int upper_prefix(const int* pre, int n, int r) {
    int lo = 0, hi = n - 1;   // largest i with pre[i] <= r
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D, int R, int WS>
__global__ __launch_bounds__(kBlock) void k_bpersist(BArgs A) {
    __shared__ SweepSmem<D, R> sm;
    __shared__ int s_unit;
    const BLayout& L = A.L;
    const BHeader H = *L.hdr;
    const int per_iter = H.TA + H.TB;
    for (;;) {
        if (threadIdx.x == 0) s_unit = (int)atomicAdd(L.head, 1u);
        __syncthreads();
        const int u = __builtin_amdgcn_readfirstlane(s_unit);
        __syncthreads();
        if (u >= H.total_units) break;
        // decode: stage type, iteration, problem (LPT order), unit of the problem-stage
        int st, it = 0, r;
        const int* pre;
        if (u < H.K * per_iter) {
            it = u / per_iter;
            r = u - it * per_iter;
            if (r < H.TA) { st = 0; pre = L.preA; }
            else { st = 1; r -= H.TA; pre = L.preB; }
        } else {
            r = u - H.K * per_iter;
            it = H.K;
            if (r < H.TF1) { st = 2; pre = L.preF1; }
            else { st = 3; r -= H.TF1; pre = L.preF2; }
        }
        const int oi = upper_prefix(pre, H.B, r);
        const int b = L.order[oi];
        const int local = r - pre[oi];
        const BProb P = L.prob[b];
        // units this problem must have completed first
        const unsigned need = (unsigned)(it * (P.nA + P.nB) + (st == 1 ? P.nA : 0) +
                                         (st == 3 ? P.nF1 : 0));
        if (threadIdx.x == 0) {
            // bounded wait: the dependency order guarantees progress; the bound only
            // turns a logic error into a flagged result (every output NaN, the
            // expiry reported by ct_sinkhorn_batched_status) instead of a hang
            unsigned spins = 0;
            while (__hip_atomic_load(&L.done[b], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
                if (spins >= A.wait_polls) {
                    atomicOr(L.counters + 2, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                ++spins;
            }
        }
        __syncthreads();
        __threadfence();
        Job J;
        int qb;
        const int cur = (st >= 2 ? H.K : it) & 1;
        unit_job<D>(A, H, P, st, cur, local, J, qb);
        const bool lagged = !A.safe_only && (st >= 2 ? H.K > 0 : it > 0);
        if (st == 2) {
            if (lagged) sweep_unit<D, R, WS, true, true>(J, qb, 0, A.kappa, A.inv_kappa, A.inv_sqrt_kappa, sm);
            else sweep_unit<D, R, WS, false, true>(J, qb, 0, A.kappa, A.inv_kappa, A.inv_sqrt_kappa, sm);
        } else {
            if (lagged) sweep_unit<D, R, WS, true, false>(J, qb, 0, A.kappa, A.inv_kappa, A.inv_sqrt_kappa, sm);
            else sweep_unit<D, R, WS, false, false>(J, qb, 0, A.kappa, A.inv_kappa, A.inv_sqrt_kappa, sm);
        }
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(&L.done[b], 1u);
    }
}

// ------------------------------------------------------------------ reductions

__global__ __launch_bounds__(256) void k_breduce(BLayout L, float kappa, float* grad_x,
                                                 float* grad_w, float* value) {
    __shared__ double red[8][256];
    __shared__ double s_bG;
    const BHeader H = *L.hdr;
    const BProb P = L.prob[blockIdx.x];
    const int d = H.d;
    const float two_a = 2.f / (float)P.T;
    // a tripped wait bound (counters[2]) marks every output of every problem as invalid
    const bool expired = L.counters[2] != 0u;
    const float nan = __builtin_nanf("");
    for (int i = threadIdx.x; i < P.T * d; i += 256) {
        const size_t gi = (size_t)P.xo * d + i;
        const float v = H.debias ? L.ds[gi] - L.dy[gi] : -L.dy[gi];
        grad_x[gi] = expired ? nan : two_a * v;
    }
    if (!value && !grad_w) return;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double invT = 1.0 / P.T;
    for (int i = threadIdx.x; i < P.T; i += 256) {
        const int gi = P.xo + i;
        acc[0] += L.fp[gi] * invT;
        if (H.debias) {
            acc[1] += L.pp[gi] * invT;
            acc[2] += L.p[gi] * invT;
        }
    }
    for (int j = threadIdx.x; j < P.M; j += 256) {
        const int gj = P.yo + j;
        const double bj = L.b[gj];
        acc[3] += bj * L.g[gj];
        if (H.need_ref) {
            acc[4] += bj * L.qp[gj];
            acc[5] += bj * L.q[gj];
        }
        const double G = H.need_ref ? (double)L.gp[gj] - (double)L.qp[gj] : (double)L.gp[gj];
        acc[6] += bj * G;
    }
    for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ot_ab = red[0][0] + red[3][0];
        const double S = H.debias ? ot_ab - 0.5 * (red[1][0] + red[2][0]) - 0.5 * (red[4][0] + red[5][0])
                                  : ot_ab;
        if (value) value[blockIdx.x] = expired ? nan : (float)S;
        s_bG = red[6][0];
    }
    __syncthreads();
    if (grad_w) {
        const double ws = L.wsum[blockIdx.x];
        for (int j = threadIdx.x; j < P.M; j += 256) {
            const int gj = P.yo + j;
            const double G = H.need_ref ? (double)L.gp[gj] - (double)L.qp[gj] : (double)L.gp[gj];
            grad_w[gj] = expired ? nan : (float)((G - s_bG) / ws);
        }
    }
}

// ------------------------------------------------------------------ host side

namespace {

std::mutex g_prep_mu;
struct MeshInfo {
    int blocks;             // 0: no exchange solve (lockstep or persistent launches)
    size_t lds;             // dynamic LDS of the launch (the largest problem's)
    double pairs;           // point pairs of its iterations
    float eps;              // the eps its tables were built for
};
struct Prepared {
    unsigned long long signature;
    LockInfo lock;
    MeshInfo mesh;
};
std::map<const void*, Prepared> g_prepared;   // workspace -> what it was prepared for

unsigned long long signature(int B, const int64_t* To, const int64_t* Mo, const ct_sinkhorn_opts* o,
                             const Schedule& sc) {
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&](unsigned long long v) {
        h ^= v;
        h *= 1099511628211ull;
    };
    mix((unsigned)B);
    for (int b = 0; b <= B; ++b) {
        mix((unsigned long long)To[b]);
        mix((unsigned long long)Mo[b]);
    }
    mix((unsigned)o->d);
    mix((unsigned)o->iters);
    mix(o->flags);
    mix((unsigned)(sc.R * 16 + sc.WS));
    const Schedule ls = lock_schedule(o->d);
    mix((unsigned)(ls.R * 4096 + ls.WS * 256 + ls.blocks_per_cu));
    return h;
}

struct BatchSizes {
    int64_t sumT, sumM, sumTpad, sumMpad;
};

ct_status b_validate(int B, const int64_t* To, const int64_t* Mo, const ct_sinkhorn_opts* o,
                     BatchSizes& S) {
    if (!o) return fail(CT_E_ARG, "opts is null");
    if (B < 1) return fail(CT_E_SHAPE, "B must be >= 1");
    if (!To || !Mo) return fail(CT_E_ARG, "T_off and M_off must be non-null");
    if (o->d != 2 && o->d != 3) return fail(CT_E_SHAPE, "d must be 2 or 3");
    if (!(o->eps > 0.f) || !std::isfinite(o->eps)) return fail(CT_E_ARG, "eps must be finite and > 0");
    if (o->iters < 0) return fail(CT_E_ARG, "iters must be >= 0");
    if (o->flags & ~(uint32_t)(CT_DEBIAS | CT_GRAD_W | CT_VALUE | CT_SAFE_LSE | CT_PERSISTENT |
                               CT_DIFFERENCE | CT_MESH | CT_UNFUSED))
        return fail(CT_E_ARG, "unsupported flags for the batched path");
    {
        const uint32_t ex = o->flags & (CT_PERSISTENT | CT_MESH | CT_UNFUSED);
        if (ex & (ex - 1))
            return fail(CT_E_ARG, "CT_PERSISTENT, CT_MESH and CT_UNFUSED exclude each other");
    }
    if (To[0] != 0 || Mo[0] != 0) return fail(CT_E_SHAPE, "offsets must start at 0");
    S = BatchSizes{0, 0, 0, 0};
    for (int b = 0; b < B; ++b) {
        const int64_t T = To[b + 1] - To[b], M = Mo[b + 1] - Mo[b];
        if (T < 1 || M < 1) return fail(CT_E_SHAPE, "problem %d has T=%lld M=%lld (need >= 1)", b,
                                        (long long)T, (long long)M);
        S.sumTpad += pad_keys((int)std::min<int64_t>(T, 1 << 30));
        S.sumMpad += pad_keys((int)std::min<int64_t>(M, 1 << 30));
    }
    S.sumT = To[B];
    S.sumM = Mo[B];
    if (S.sumTpad > (int64_t(1) << 30) || S.sumMpad > (int64_t(1) << 30))
        return fail(CT_E_SHAPE, "total points must stay below 2^30");
    return CT_OK;
}

Schedule batched_schedule(int d) {
    // tuned entry under the (d, 0, 0) key, else two queries per lane, keys split four ways
    Schedule s;
    if (tuning_lookup(d, 0, 0, s) && s.R <= 4) return Schedule{s.R, s.WS, 0, 0};
    return Schedule{2, 4, 0, 0};
}

// Sizes and record offsets of every problem (the part of BProb the lockstep
// tables need).
std::vector<BProb> base_probs(int B, const int64_t* To, const int64_t* Mo) {
    std::vector<BProb> P(B);
    int xp = 0, yp = 0;
    for (int b = 0; b < B; ++b) {
        std::memset(&P[b], 0, sizeof(BProb));
        P[b].T = (int)(To[b + 1] - To[b]);
        P[b].M = (int)(Mo[b + 1] - Mo[b]);
        P[b].xo = (int)To[b];
        P[b].yo = (int)Mo[b];
        P[b].xp = xp;
        P[b].yp = yp;
        P[b].Tpad = pad_keys(P[b].T);
        P[b].Mpad = pad_keys(P[b].M);
        P[b].log2a = (float)(-std::log2((double)P[b].T));
        xp += P[b].Tpad;
        yp += P[b].Mpad;
    }
    return P;
}

// The job of kind 0 f, 1 p, 2 q, 3 g (fin: extrapolation pass) of problem P,
// with pointers into the device layout L (the host mirror of unit_job, full
// query ranges).
Job lock_job(const BLayout& L, const BProb& P, int kind, int cur, bool fin, int d) {
    Job J;
    std::memset(&J, 0, sizeof(Job));
    J.rescued = L.counters + 1;
    J.qlog2w_s = P.log2a;
    if (kind == 0) {
        J.qrec = L.cx + P.xo; J.qpot = L.f + P.xo;
        J.krec = L.yrec[0] + P.yp; J.nq = P.T; J.nk = P.M;
        J.out_pot = (fin ? L.fp : L.f) + P.xo;
        J.out_rec = (fin ? L.xrec[1] : L.xrec[0]) + P.xp;
        if (fin) J.out_bary = L.dy + (size_t)P.xo * d;
    } else if (kind == 1) {
        J.qrec = L.cx + P.xo; J.qpot = L.p + P.xo;
        J.krec = L.xrec[2 + cur] + P.xp; J.nq = P.T; J.nk = P.T;
        if (fin) {
            J.out_pot = L.pp + P.xo;
            J.out_bary = L.ds + (size_t)P.xo * d;
        } else {
            J.self_avg = 1;
            J.out_pot = L.p + P.xo;
            J.out_rec = L.xrec[2 + (cur ^ 1)] + P.xp;
        }
    } else if (kind == 2) {
        J.qrec = L.cy + P.yo; J.qpot = L.q + P.yo; J.qlog2w = L.log2b + P.yo;
        J.krec = L.yrec[1 + cur] + P.yp; J.nq = P.M; J.nk = P.M;
        if (fin) {
            J.out_pot = L.qp + P.yo;
        } else {
            J.self_avg = 1;
            J.out_pot = L.q + P.yo;
            J.out_rec = L.yrec[1 + (cur ^ 1)] + P.yp;
        }
    } else {
        J.qrec = L.cy + P.yo; J.qpot = L.g + P.yo; J.qlog2w = L.log2b + P.yo;
        J.krec = (fin ? L.xrec[1] : L.xrec[0]) + P.xp; J.nq = P.M; J.nk = P.T;
        J.out_pot = (fin ? L.gp : L.g) + P.yo;
        J.out_rec = fin ? nullptr : L.yrec[0] + P.yp;
    }
    return J;
}

// Build the five lockstep job tables (jobs, sweep-block and merge-block prefix
// ends) into the given arrays ([kLockKinds][3B] each) and their sizes; returns
// the floats of partial sums the largest launch needs.
size_t build_lock(const BLayout& L, const std::vector<BProb>& P, uint32_t flags, int K, int d,
                  const Schedule& sc, Job* jobs, int* blk, int* mrg, LockInfo& info) {
    const int B = (int)P.size();
    const bool debias = flags & CT_DEBIAS;
    const bool want_v = flags & (CT_VALUE | CT_GRAD_W);
    const bool need_ref = debias && want_v;
    const int qpb = 64 * sc.R * (4 / sc.WS);
    const int curF = K & 1;
    size_t part_max = 0;
    for (int k = 0; k < kLockKinds; ++k) {
        std::vector<Job> js;
        for (int b = 0; b < B; ++b) {
            if (k <= 1) {
                js.push_back(lock_job(L, P[b], 0, k, false, d));
                if (debias) js.push_back(lock_job(L, P[b], 1, k, false, d));
                if (need_ref) js.push_back(lock_job(L, P[b], 2, k, false, d));
            } else if (k == 2) {
                js.push_back(lock_job(L, P[b], 3, 0, false, d));
            } else if (k == 3) {
                js.push_back(lock_job(L, P[b], 0, curF, true, d));
                if (debias) js.push_back(lock_job(L, P[b], 1, curF, true, d));
            } else if (want_v) {
                js.push_back(lock_job(L, P[b], 3, curF, true, d));
                if (need_ref) js.push_back(lock_job(L, P[b], 2, curF, true, d));
            }
        }
        double pairs = 0.0;
        for (const Job& j : js) pairs += (double)j.nq * pad_keys(j.nk);
        const double ppb = pairs / ((double)kNumCU * sc.blocks_per_cu);
        int nb = 0, nm = 0;
        size_t part = 0;
        Job* jt = jobs + (size_t)k * 3 * B;
        for (size_t i = 0; i < js.size(); ++i) {
            Job& j = js[i];
            nb += plan_job_target(j, sc, ppb);
            if (j.splits > 1) {
                j.part = L.lpart + part;
                part += (size_t)(2 + d) * j.splits * (size_t)j.nqb * qpb;
                nm += (j.nq + kMergeRows - 1) / kMergeRows;
            }
            jt[i] = j;
            blk[(size_t)k * 3 * B + i] = nb;
            mrg[(size_t)k * 3 * B + i] = nm;
        }
        info.sc = sc;
        info.njobs[k] = (int)js.size();
        info.nblocks[k] = nb;
        info.nmerge[k] = nm;
        part_max = std::max(part_max, part);
    }
    return part_max;
}

// Exchange solve of the whole batch: every problem planned (one block allowed),
// at most kMeshBatchPairs point pairs per iteration each, all blocks resident at
// once.  Fills tab/blk (device pointers of L) and returns false if it does not
// apply.
constexpr double kMeshBatchPairs = 1.5e7;
constexpr unsigned kMeshBatchWaitPolls = 1u << 18;

size_t device_lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    return (size_t)std::max(0, v);
}

bool plan_mesh_batch(const BLayout& L, const std::vector<BProb>& P, const ct_sinkhorn_opts* o,
                     MeshArgs* tab, int* blk, MeshInfo& info) {
    info = MeshInfo{0, 0, 0.0, o->eps};
    const int B = (int)P.size(), d = o->d;
    const bool debias = o->flags & CT_DEBIAS;
    const bool want_v = o->flags & (CT_VALUE | CT_GRAD_W);
    const bool need_ref = debias && want_v;
    const size_t dev_lds = device_lds_per_block();
    if (dev_lds <= sizeof(MeshArgs)) return false;
    const size_t cap = std::min(kTinyMaxLds, dev_lds) - sizeof(MeshArgs);
    const double kappa_d = kLog2e / (double)o->eps;
    const int curF = o->iters & 1;
    unsigned polls = kMeshBatchWaitPolls, extra = 0u;
    // test hooks of the give-up path (read when the batch is prepared)
    if (const char* e = std::getenv("CT_MESH_WAIT_POLLS")) polls = (unsigned)std::strtoul(e, nullptr, 10);
    if (const char* e = std::getenv("CT_MESH_UNSATISFIABLE_WAITS")) extra = std::atoi(e) ? (1u << 20) : 0u;
    int blocks = 0;
    size_t lds_max = 0;
    double pairs = 0.0;
    for (int b = 0; b < B; ++b) {
        const BProb& Q = P[b];
        const double pp = 2.0 * Q.T * Q.M + (debias ? (double)Q.T * Q.T : 0.0) +
                          (need_ref ? (double)Q.M * Q.M : 0.0);
        if (pp > kMeshBatchPairs) return false;
        MeshArgs& A = tab[b];
        size_t lds = 0;
        int G = 0;
        if (!mesh_plan(Q.T, Q.M, d, debias, need_ref, cap, true, A, lds, &G)) return false;
        A.cx = L.cx + Q.xo;
        A.cy = L.cy + Q.yo;
        A.log2b = L.log2b + Q.yo;
        A.f = L.f + Q.xo;
        A.g = L.g + Q.yo;
        A.p = L.p + Q.xo;
        A.q = L.q + Q.yo;
        A.xrec_f = L.xrec[0] + Q.xp;
        A.yrec_g = L.yrec[0] + Q.yp;
        A.xrec_p = L.xrec[2 + curF] + Q.xp;
        A.yrec_q = L.yrec[1 + curF] + Q.yp;
        unsigned long long* x0 = L.xch + 4 * ((size_t)Q.xo + Q.yo);
        A.xch_f = x0;
        A.xch_p = x0 + 2 * (size_t)Q.T;
        A.xch_g = x0 + 4 * (size_t)Q.T;
        A.xch_q = x0 + 4 * (size_t)Q.T + 2 * (size_t)Q.M;
        for (int h = 0; h < 2; ++h)
            for (int j = 0; j < A.njobs[h]; ++j) {
                MeshJob& J = A.job[h][j];
                J.xch = J.yside ? (J.avg ? A.xch_q : A.xch_g) : (J.avg ? A.xch_p : A.xch_f);
            }
        A.gat[0][0].xch = A.xch_g;
        if (A.ngat[0] > 1) A.gat[0][1].xch = A.xch_p;
        A.gat[1][0].xch = A.xch_f;
        if (A.ngat[1] > 1) A.gat[1][1].xch = A.xch_q;
        A.rescued = L.counters + 1;
        A.expired = L.counters + 2;   // the batched outputs' invalid flag
        A.polls = polls;
        A.version_extra = extra;
        A.d = d;
        A.iters = o->iters;
        A.lagged0 = 0;
        A.safe_only = (o->flags & CT_SAFE_LSE) ? 1 : 0;
        A.kappa = (float)kappa_d;
        A.inv_kappa = (float)(1.0 / kappa_d);
        A.log2a = Q.log2a;
        blocks += G;
        blk[b] = blocks;
        lds_max = std::max(lds_max, lds);
        pairs += o->iters * pp;
    }
    if (blocks > mesh_resident_blocks(d, lds_max, true)) return false;
    info.blocks = blocks;
    info.lds = lds_max;
    info.pairs = pairs;
    return true;
}

__global__ __launch_bounds__(256) void k_bfill_ones64(unsigned long long* a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = ~0ull;
}

// Floats of lockstep partial sums for this batch (the planning does not depend
// on where the workspace is).
size_t lock_part_floats(int B, const int64_t* To, const int64_t* Mo, const ct_sinkhorn_opts* o,
                        const BatchSizes& S) {
    const std::vector<BProb> P = base_probs(B, To, Mo);
    const BLayout L0 = b_layout(nullptr, B, S.sumT, S.sumM, S.sumTpad, S.sumMpad, o->d, 0);
    std::vector<Job> jobs((size_t)kLockKinds * 3 * B);
    std::vector<int> blk(jobs.size()), mrg(jobs.size());
    LockInfo info;
    return build_lock(L0, P, o->flags, o->iters, o->d, lock_schedule(o->d), jobs.data(), blk.data(),
                      mrg.data(), info);
}

}  // namespace

}  // namespace ct

using namespace ct;

extern "C" size_t ct_sinkhorn_batched_workspace_size(int32_t B, const int64_t* To, const int64_t* Mo,
                                                     const ct_sinkhorn_opts* o) {
    BatchSizes S;
    if (b_validate(B, To, Mo, o, S)) return 0;
    const size_t pf = lock_part_floats(B, To, Mo, o, S);
    return b_layout(nullptr, B, S.sumT, S.sumM, S.sumTpad, S.sumMpad, o->d, pf).bytes;
}

extern "C" ct_status ct_sinkhorn_batched_prepare(int32_t B, const int64_t* To, const int64_t* Mo,
                                                 const ct_sinkhorn_opts* o, void* ws,
                                                 size_t ws_bytes, void* stream) {
    clear_error();
    BatchSizes S;
    ct_status rc = b_validate(B, To, Mo, o, S);
    if (rc) return rc;
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CT_E_WORKSPACE, "workspace not 256-byte aligned");
    const size_t pf = lock_part_floats(B, To, Mo, o, S);
    BLayout L = b_layout(ws, B, S.sumT, S.sumM, S.sumTpad, S.sumMpad, o->d, pf);
    if (ws_bytes < L.bytes) return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    rc = refuse_capture(static_cast<hipStream_t>(stream), "ct_sinkhorn_batched_prepare");
    if (rc) return rc;
    const Schedule sc = batched_schedule(o->d);
    const int QB = 64 * sc.R * (4 / sc.WS);
    const bool debias = o->flags & CT_DEBIAS;
    const bool want_v = o->flags & (CT_VALUE | CT_GRAD_W);
    const bool need_ref = debias && want_v;
    auto nb = [&](int n) { return (n + QB - 1) / QB; };

    // host image of the table: header, problems, order, prefixes, record offsets
    std::vector<char> img(L.table_bytes, 0);
    BLayout H0 = b_layout(img.data(), B, S.sumT, S.sumM, S.sumTpad, S.sumMpad, o->d, pf);
    BHeader& H = *H0.hdr;
    std::vector<double> cost(B);
    int xp = 0, yp = 0;
    for (int b = 0; b < B; ++b) {
        BProb& P = H0.prob[b];
        std::memset(&P, 0, sizeof P);
        P.T = (int)(To[b + 1] - To[b]);
        P.M = (int)(Mo[b + 1] - Mo[b]);
        P.xo = (int)To[b];
        P.yo = (int)Mo[b];
        P.xp = xp;
        P.yp = yp;
        P.Tpad = pad_keys(P.T);
        P.Mpad = pad_keys(P.M);
        H0.xoff[b] = xp;
        H0.yoff[b] = yp;
        xp += P.Tpad;
        yp += P.Mpad;
        P.log2a = (float)(-std::log2((double)P.T));
        const int a1 = nb(P.T), a2 = debias ? nb(P.T / 2) : 0, a3 = need_ref ? nb(P.M / 2) : 0;
        const int b1 = nb(P.M), b2 = debias ? nb(P.T - P.T / 2) : 0, b3 = need_ref ? nb(P.M - P.M / 2) : 0;
        P.uA[0] = 0; P.uA[1] = a1; P.uA[2] = a1 + a2; P.uA[3] = a1 + a2 + a3;
        P.uB[0] = 0; P.uB[1] = b1; P.uB[2] = b1 + b2; P.uB[3] = b1 + b2 + b3;
        P.nA = P.uA[3];
        P.nB = P.uB[3];
        P.uF1[0] = 0; P.uF1[1] = nb(P.T); P.uF1[2] = nb(P.T) + (debias ? nb(P.T) : 0);
        P.uF2[0] = 0; P.uF2[1] = want_v ? nb(P.M) : 0;
        P.uF2[2] = P.uF2[1] + (need_ref ? nb(P.M) : 0);
        P.nF1 = P.uF1[2];
        P.nF2 = P.uF2[2];
        cost[b] = (double)P.T * P.M + (debias ? 0.5 * P.T * P.T : 0.0) +
                  (need_ref ? 0.5 * (double)P.M * P.M : 0.0);
    }
    H0.xoff[B] = xp;
    H0.yoff[B] = yp;
    std::vector<int> ord(B);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int i, int j) { return cost[i] > cost[j]; });
    H0.preA[0] = H0.preB[0] = H0.preF1[0] = H0.preF2[0] = 0;
    for (int i = 0; i < B; ++i) {
        const BProb& P = H0.prob[ord[i]];
        H0.order[i] = ord[i];
        H0.preA[i + 1] = H0.preA[i] + P.nA;
        H0.preB[i + 1] = H0.preB[i] + P.nB;
        H0.preF1[i + 1] = H0.preF1[i] + P.nF1;
        H0.preF2[i + 1] = H0.preF2[i] + P.nF2;
    }
    H.B = B;
    H.K = o->iters;
    H.d = o->d;
    H.R = sc.R;
    H.WS = sc.WS;
    H.debias = debias;
    H.need_ref = need_ref;
    H.TA = H0.preA[B];
    H.TB = H0.preB[B];
    H.TF1 = H0.preF1[B];
    H.TF2 = H0.preF2[B];
    const double total = (double)H.K * (H.TA + H.TB) + H.TF1 + H.TF2;
    if (total >= 2147483647.0) return fail(CT_E_SHAPE, "too many work units (%.3g)", total);
    H.total_units = (int)total;
    H.sumT = (int)S.sumT;
    H.sumM = (int)S.sumM;
    H.sumTpad = (int)S.sumTpad;
    H.sumMpad = (int)S.sumMpad;
    H.signature = signature(B, To, Mo, o, sc);
    // lockstep tables: device pointers of the real workspace, written into the image
    LockInfo info;
    const std::vector<BProb> BP = base_probs(B, To, Mo);
    build_lock(L, BP, o->flags, o->iters, o->d, lock_schedule(o->d), H0.ljobs, H0.lblk, H0.lmrg,
               info);
    MeshInfo minfo{0, 0, 0.0, o->eps};
    if (!(o->flags & (CT_PERSISTENT | CT_UNFUSED)) && o->iters > 0) {
        const bool ok = plan_mesh_batch(L, BP, o, H0.mtab, H0.mblk, minfo);
        if (!ok) {
            minfo = MeshInfo{0, 0, 0.0, o->eps};
            if (o->flags & CT_MESH)
                return fail(CT_E_UNSUPPORTED, "the exchange solve does not apply to this batch (a "
                                              "problem above %.3g pairs per iteration or beyond one "
                                              "workgroup's LDS, or more blocks than fit at once)",
                            kMeshBatchPairs);
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    CT_CHECK_HIP(hipMemcpyAsync(ws, img.data(), img.size(), hipMemcpyHostToDevice, st));
    CT_CHECK_HIP(hipStreamSynchronize(st));
    std::lock_guard<std::mutex> lk(g_prep_mu);
    g_prepared[ws] = Prepared{H.signature, info, minfo};
    return CT_OK;
}

extern "C" ct_status ct_sinkhorn_grad_batched(int32_t B, const int64_t* To, const int64_t* Mo,
                                              const float* x, const float* y, const float* w,
                                              const ct_sinkhorn_opts* o, float* grad_x,
                                              float* grad_w, float* value, void* ws,
                                              size_t ws_bytes, void* stream) {
    clear_error();
    BatchSizes S;
    ct_status rc = b_validate(B, To, Mo, o, S);
    if (rc) return rc;
    if (!x || !y || !grad_x) return fail(CT_E_ARG, "x, y and grad_x must be non-null");
    if (grad_w && !(o->flags & CT_GRAD_W)) return fail(CT_E_ARG, "grad_w given without CT_GRAD_W");
    if (!grad_w && (o->flags & CT_GRAD_W)) return fail(CT_E_ARG, "CT_GRAD_W needs grad_w");
    if (value && !(o->flags & CT_VALUE)) return fail(CT_E_ARG, "value given without CT_VALUE");
    if (!value && (o->flags & CT_VALUE)) return fail(CT_E_ARG, "CT_VALUE needs value");
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    const size_t pf = lock_part_floats(B, To, Mo, o, S);
    BLayout L = b_layout(ws, B, S.sumT, S.sumM, S.sumTpad, S.sumMpad, o->d, pf);
    if (ws_bytes < L.bytes) return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    const Schedule sc = batched_schedule(o->d);
    LockInfo info;
    MeshInfo minfo;
    {
        std::lock_guard<std::mutex> lk(g_prep_mu);
        auto it = g_prepared.find(ws);
        if (it == g_prepared.end() || it->second.signature != signature(B, To, Mo, o, sc))
            return fail(CT_E_ARG, "workspace not prepared for this batch "
                                  "(call ct_sinkhorn_batched_prepare first)");
        info = it->second.lock;
        minfo = it->second.mesh;
    }
    if (minfo.blocks > 0 && minfo.eps != o->eps)
        return fail(CT_E_ARG, "the batch's exchange-solve tables were prepared for eps=%g (got %g)",
                    (double)minfo.eps, (double)o->eps);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double kappa_d = kLog2e / (double)o->eps;
    hipLaunchKernelGGL(k_bwsum, dim3(B), dim3(256), 0, st, L, x, y, w, o->d);
    CT_CHECK_HIP(hipGetLastError());
    const int64_t n = std::max(S.sumTpad, S.sumMpad);
    hipLaunchKernelGGL(k_bstage, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, L, x, y, w,
                       (float)std::sqrt(kappa_d), (float)kappa_d);
    CT_CHECK_HIP(hipGetLastError());
    if (!(o->flags & CT_PERSISTENT)) {
        // lockstep: two launches per iteration, then the extrapolation launches
        TabLaunch T0;
        std::memset(&T0, 0, sizeof(T0));
        T0.kappa = (float)kappa_d;
        T0.inv_kappa = (float)(1.0 / kappa_d);
        T0.inv_sqrt_kappa = (float)(1.0 / std::sqrt(kappa_d));
        T0.expanded = (o->flags & CT_DIFFERENCE) ? 0 : 1;
        const Schedule lsc = info.sc;
        auto run_kind = [&](int k, bool lagged, bool bary) -> ct_status {
            if (info.njobs[k] == 0) return CT_OK;
            TabLaunch t = T0;
            t.jobs = L.ljobs + (size_t)k * 3 * B;
            t.blk_end = L.lblk + (size_t)k * 3 * B;
            t.mrg_end = L.lmrg + (size_t)k * 3 * B;
            t.njobs = info.njobs[k];
            t.nblocks = info.nblocks[k];
            t.nmerge = info.nmerge[k];
            CT_CHECK_HIP(launch_tab(o->d, lsc, lagged, bary, t, st));
            return CT_OK;
        };
        const bool safe_only = o->flags & CT_SAFE_LSE;
        if (minfo.blocks > 0) {
            // the K iterations of every problem in one launch of the exchange solve
            const int64_t nw = 4 * (S.sumT + S.sumM);
            hipLaunchKernelGGL(k_bfill_ones64, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st,
                               L.xch, nw);
            CT_CHECK_HIP(hipGetLastError());
            CT_CHECK_HIP(launch_mesh_batch(o->d, L.mtab, L.mblk, B, minfo.lds, minfo.blocks,
                                           minfo.pairs, st));
        }
        void* tok = profile_begin(st);
        for (int k = 0; k < (minfo.blocks > 0 ? 0 : o->iters); ++k) {
            const bool lagged = !safe_only && k > 0;
            rc = run_kind(k & 1, lagged, false);
            if (rc) return rc;
            rc = run_kind(2, lagged, false);
            if (rc) return rc;
        }
        const bool lagged_final = !safe_only && o->iters > 0;
        rc = run_kind(3, lagged_final, true);
        if (rc) return rc;
        rc = run_kind(4, lagged_final, false);
        if (rc) return rc;
        if (tok) profile_end(tok, st, 4, 0, lsc.R * 100 + lsc.WS * 10, 0, 0.0);
        hipLaunchKernelGGL(k_breduce, dim3(B), dim3(256), 0, st, L, (float)kappa_d, grad_x, grad_w,
                           value);
        CT_CHECK_HIP(hipGetLastError());
        return CT_OK;
    }
    BArgs A;
    A.L = L;
    A.kappa = (float)kappa_d;
    A.inv_kappa = (float)(1.0 / kappa_d);
    A.inv_sqrt_kappa = (float)(1.0 / std::sqrt(kappa_d));
    A.safe_only = (o->flags & CT_SAFE_LSE) ? 1 : 0;
    A.wait_polls = 1u << 22;
    if (const char* e = std::getenv("CT_PERSISTENT_WAIT_POLLS")) A.wait_polls = (unsigned)std::strtoul(e, nullptr, 10);
    const int grid = kNumCU * 4;
    void* tok = profile_begin(st);
#define CT_BP(D, R, WS) hipLaunchKernelGGL((k_bpersist<D, R, WS>), dim3(grid), dim3(kBlock), 0, st, A)
    if (o->d == 2) {
        if (sc.R == 1) { if (sc.WS == 4) CT_BP(2, 1, 4); else if (sc.WS == 2) CT_BP(2, 1, 2); else CT_BP(2, 1, 1); }
        else if (sc.R == 2) { if (sc.WS == 4) CT_BP(2, 2, 4); else if (sc.WS == 2) CT_BP(2, 2, 2); else CT_BP(2, 2, 1); }
        else { if (sc.WS == 4) CT_BP(2, 4, 4); else if (sc.WS == 2) CT_BP(2, 4, 2); else CT_BP(2, 4, 1); }
    } else {
        if (sc.R == 1) { if (sc.WS == 4) CT_BP(3, 1, 4); else if (sc.WS == 2) CT_BP(3, 1, 2); else CT_BP(3, 1, 1); }
        else if (sc.R == 2) { if (sc.WS == 4) CT_BP(3, 2, 4); else if (sc.WS == 2) CT_BP(3, 2, 2); else CT_BP(3, 2, 1); }
        else { if (sc.WS == 4) CT_BP(3, 4, 4); else if (sc.WS == 2) CT_BP(3, 4, 2); else CT_BP(3, 4, 1); }
    }
#undef CT_BP
    CT_CHECK_HIP(hipGetLastError());
    if (tok) {
        double pairs = 0.0;
        for (int b = 0; b < B; ++b) {
            const double T = (double)(To[b + 1] - To[b]), M = (double)(Mo[b + 1] - Mo[b]);
            const bool debias = o->flags & CT_DEBIAS;
            const bool want_v = o->flags & (CT_VALUE | CT_GRAD_W);
            pairs += o->iters * (2 * T * M + (debias ? T * T : 0) + (debias && want_v ? M * M : 0)) +
                     T * M + (debias ? T * T : 0) + (want_v ? T * M + (debias ? M * M : 0) : 0);
        }
        profile_end(tok, st, 3, 0, sc.R * 100 + sc.WS * 10, grid, pairs);
    }
    hipLaunchKernelGGL(k_breduce, dim3(B), dim3(256), 0, st, L, (float)kappa_d, grad_x, grad_w, value);
    CT_CHECK_HIP(hipGetLastError());
    return CT_OK;
}
