// ct_sinkhorn_grad: debiased Sinkhorn divergence gradient for one problem
// (Sec. II-B, eqs. 5-7).  Staging, the iteration schedule, the final
// extrapolation pass and the reductions; the sweeps themselves are in sweep.hip.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "ct_internal.h"

namespace ct {

constexpr double kLog2e = 1.4426950408889634;

// ------------------------------------------------------------------ kernels

__global__ __launch_bounds__(256) void k_zero3(unsigned* a, int na, unsigned* b, int nb,
                                               unsigned* c, int nc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (a && i < na) a[i] = 0u;
    if (b && i < nb) b[i] = 0u;
    if (c && i < nc) c[i] = 0u;
}

// Fill 64-bit words with all ones (a version no exchange ever awaits).
__global__ __launch_bounds__(256) void k_fill_ones64(unsigned long long* a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = ~0ull;
}

// Sum of the reference weights in double, fixed order (one block).
__global__ __launch_bounds__(1024) void k_wsum(const float* __restrict__ w, int M,
                                               double* __restrict__ out) {
    __shared__ double red[1024];
    double s = 0.0;
    if (w) {
        for (int j = threadIdx.x; j < M; j += 1024) s += (double)w[j];
    } else {
        s = threadIdx.x == 0 ? (double)M : 0.0;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Common origin of both point sets (mean of every coordinate, double, fixed
// order, non-finite values skipped).  The soft-min is translation invariant, but
// the float32 prescale x * sqrt(kappa) is not: far from the coordinate origin it
// would round away the low bits of every difference x_i - y_j.  Subtracting the
// origin first (exact for nearby float32 values) keeps them.
__global__ __launch_bounds__(1024) void k_origin(const float* __restrict__ x, int T,
                                                 const float* __restrict__ y, int M, int d,
                                                 float* __restrict__ out) {
    __shared__ double red[3][1024];
    __shared__ double cnt[1024];
    double s[3] = {0.0, 0.0, 0.0}, n = 0.0;
    // a skipped point adds zeros (no branch), so eight loads can be in flight
#pragma unroll 8
    for (int i = threadIdx.x; i < T + M; i += 1024) {
        const float* p = i < T ? x + (size_t)i * d : y + (size_t)(i - T) * d;
        float v[3] = {0.f, 0.f, 0.f};
        bool ok = true;
        for (int t = 0; t < d; ++t) {
            v[t] = p[t];
            ok = ok && isfinite(v[t]);
        }
        for (int t = 0; t < d; ++t) s[t] += ok ? (double)v[t] : 0.0;
        n += ok ? 1.0 : 0.0;
    }
    for (int t = 0; t < 3; ++t) red[t][threadIdx.x] = s[t];
    cnt[threadIdx.x] = n;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            for (int t = 0; t < 3; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + h];
            cnt[threadIdx.x] += cnt[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        const double c = cnt[0] > 0.0 ? cnt[0] : 1.0;
        out[threadIdx.x] = (int)threadIdx.x < d ? (float)(red[threadIdx.x][0] / c) : 0.f;
    }
}

struct StageArgs {
    const float* x;
    const float* y;
    const float* w;
    const float* pot_in;     // [2T+2M] warm start (f, g, p, q) or null
    int warm, ref_cached;
    int T, M, d, Tpad, Mpad;
    float sqrt_kappa, kappa, log2a;
    const double* wsum;
    const float* origin;     // [3] subtracted before scaling
    float4* cx;              // query coordinates of x
    float4* cy;              // query coordinates of y
    float4* xrec[4];         // key records of x: f (g-sweeps), f+ (g+ sweep), p ping-pong
    float4* yrec[3];         // key records of y: g (f-sweeps), q ping-pong
    float* b;
    float* log2b;
    float *f, *g, *p, *q;
    float *fp, *gp, *pp, *qp; // extrapolated potentials, zeroed here
    unsigned* nonfinite;
};

__device__ __forceinline__ float4 make_rec(const float* c, int d, float h) {
    return d == 2 ? make_float4(c[0], c[1], h, 0.f) : make_float4(c[0], c[1], c[2], h);
}

// Pre-scale coordinates, form the reference masses and the initial key records
// (h = log2 mass + kappa * potential; padding records get h = -inf).
__global__ __launch_bounds__(256) void k_stage(StageArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float ninf = -__builtin_huge_valf();
    if (i < A.Tpad) {
        float c[3] = {0.f, 0.f, 0.f};
        if (i < A.T) {
            bool bad = false;
            for (int t = 0; t < A.d; ++t) {
                const float v = A.x[(size_t)i * A.d + t];
                bad |= !isfinite(v);
                c[t] = (v - A.origin[t]) * A.sqrt_kappa;
            }
            A.cx[i] = make_float4(c[0], c[1], c[2], 0.f);
            const float f0 = A.warm ? A.pot_in[i] : 0.f;
            const float p0 = A.warm ? A.pot_in[(size_t)A.T + A.M + i] : 0.f;
            A.f[i] = f0;
            A.p[i] = p0;
            A.fp[i] = 0.f;
            A.pp[i] = 0.f;
            A.xrec[0][i] = make_rec(c, A.d, ninf);
            A.xrec[1][i] = make_rec(c, A.d, ninf);
            A.xrec[2][i] = make_rec(c, A.d, __builtin_fmaf(p0, A.kappa, A.log2a));
            A.xrec[3][i] = make_rec(c, A.d, ninf);
            if (bad) atomicAdd(A.nonfinite, 1u);
        } else {
            for (int r = 0; r < 4; ++r) A.xrec[r][i] = make_rec(c, A.d, ninf);
        }
    }
    if (i < A.Mpad) {
        float c[3] = {0.f, 0.f, 0.f};
        if (i < A.M) {
            bool bad = false;
            for (int t = 0; t < A.d; ++t) {
                const float v = A.y[(size_t)i * A.d + t];
                bad |= !isfinite(v);
                c[t] = (v - A.origin[t]) * A.sqrt_kappa;
            }
            A.cy[i] = make_float4(c[0], c[1], c[2], 0.f);
            const float wj = A.w ? A.w[i] : 1.f;
            bad |= !(wj > 0.f) || !isfinite(wj);
            const float bj = (float)((double)wj / *A.wsum);
            const float lb = __log2f(bj);
            A.b[i] = bj;
            A.log2b[i] = lb;
            const float g0 = A.warm ? A.pot_in[(size_t)A.T + i] : 0.f;
            const float q0 = (A.warm || A.ref_cached) ? A.pot_in[2 * (size_t)A.T + A.M + i] : 0.f;
            A.g[i] = g0;
            A.q[i] = q0;
            A.gp[i] = 0.f;
            A.qp[i] = 0.f;
            A.yrec[0][i] = make_rec(c, A.d, __builtin_fmaf(g0, A.kappa, lb));
            A.yrec[1][i] = make_rec(c, A.d, __builtin_fmaf(q0, A.kappa, lb));
            A.yrec[2][i] = make_rec(c, A.d, ninf);
            if (bad) atomicAdd(A.nonfinite, 1u);
        } else {
            for (int r = 0; r < 3; ++r) A.yrec[r][i] = make_rec(c, A.d, ninf);
        }
    }
}

// grad_x = 2 a (Ds - Dy)  (debiased) or -2 a Dy; NaN after a barrier of the fused
// solve gave up (*expired).
__global__ __launch_bounds__(256) void k_grad_x(const float* __restrict__ dy,
                                                const float* __restrict__ ds, int n, float two_a,
                                                const unsigned* __restrict__ expired,
                                                float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = ds ? ds[i] - dy[i] : -dy[i];
    out[i] = *expired ? __builtin_nanf("") : two_a * v;
}

struct ReduceArgs {
    int T, M;
    int debias, need_ref;
    float kappa;
    const float* fp;
    const float* g;
    const float* gp;
    const float* p;
    const float* pp;
    const float* q;
    const float* qp;
    const float* b;
    const double* wsum;
    unsigned* counters;         // [0] non-finite inputs, [1] rescued rows, [2] residual (float
                                // bits), [3] 1 once the residual is written, [4] a barrier of
                                // the fused solve gave up
    double* bG;                 // out: <b, G>
    float* value;
    float* aux;
};

// Dual objectives, value, <b,G> and the column residual, in double, fixed order.
__global__ __launch_bounds__(1024) void k_reduce(ReduceArgs A) {
    __shared__ double red[8][1024];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double invT = 1.0 / A.T;
    for (int i = threadIdx.x; i < A.T; i += 1024) {
        acc[0] += A.fp[i] * invT;
        if (A.debias) {
            acc[1] += A.pp[i] * invT;
            acc[2] += A.p[i] * invT;
        }
    }
    for (int j = threadIdx.x; j < A.M; j += 1024) {
        const double bj = A.b[j];
        acc[3] += bj * A.g[j];
        if (A.need_ref) {
            acc[4] += bj * A.qp[j];
            acc[5] += bj * A.q[j];
        }
        const double G = A.need_ref ? (double)A.gp[j] - (double)A.qp[j] : (double)A.gp[j];
        acc[6] += bj * G;
        acc[7] += bj * fabs(exp2(((double)A.g[j] - (double)A.gp[j]) * (double)A.kappa) - 1.0);
    }
    for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ot_ab = red[0][0] + red[3][0];
        const double ot_aa = red[1][0] + red[2][0];
        const double ot_bb = red[4][0] + red[5][0];
        const double S = A.debias ? ot_ab - 0.5 * ot_aa - 0.5 * ot_bb : ot_ab;
        *A.bG = red[6][0];
        if (A.value) *A.value = A.counters[4] ? __builtin_nanf("") : (float)S;
        if (A.aux) {
            A.aux[0] = (float)ot_ab;
            A.aux[1] = A.debias ? (float)ot_aa : 0.f;
            A.aux[2] = A.need_ref ? (float)ot_bb : 0.f;
            A.aux[3] = (float)red[7][0];
        }
        A.counters[2] = __float_as_uint((float)red[7][0]);
        A.counters[3] = 1u;
    }
}

__global__ __launch_bounds__(256) void k_grad_w(const float* __restrict__ gp,
                                                const float* __restrict__ qp, int M,
                                                const double* __restrict__ bG,
                                                const double* __restrict__ wsum,
                                                const unsigned* __restrict__ expired,
                                                float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double G = qp ? (double)gp[j] - (double)qp[j] : (double)gp[j];
    out[j] = *expired ? __builtin_nanf("") : (float)((G - *bG) / *wsum);
}

__global__ void k_counters_out(const unsigned* __restrict__ c, float* __restrict__ aux) {
    if (threadIdx.x == 0) {
        aux[4] = (float)c[1];
        aux[5] = (float)c[0];
        aux[6] = c[4] ? 1.f : 0.f;
        aux[7] = 0.f;
    }
}

// --------------------------------------------------------------- layout

struct SkLayout {
    double* wsum;
    double* bG;
    unsigned* counters;      // [8]: see ReduceArgs
    float4* cx;
    float4* cy;
    float4* xrec[4];         // 0: h from f (keys of g-sweeps), 1: from f+, 2/3: from p (ping-pong)
    float4* yrec[3];         // 0: h from g (keys of f-sweeps), 1/2: from q (ping-pong)
    float* origin;           // [4] common origin subtracted before scaling
    float* b;
    float* log2b;
    float *f, *g, *p, *q;
    float *fp, *gp, *pp, *qp;
    float *dy, *ds;
    float* part[3];          // partial buffers: cross jobs, x self jobs, y self jobs
    unsigned* tick[3];
    size_t ntick;
    unsigned* bar;           // [kFusedBarWords] barrier words of the fused solve
    unsigned long long* xch; // [2 (2T + 2M)] versioned potential words of the exchange solve
    size_t bytes;
};

constexpr int kCounters = 8;

static SkLayout sk_layout(void* ws, int T, int M, int d) {
    Arena a(ws);
    SkLayout L;
    const int Tp = pad_keys(T), Mp = pad_keys(M);
    L.wsum = a.take<double>(1);
    L.bG = a.take<double>(1);
    L.counters = a.take<unsigned>(kCounters);
    L.cx = a.take<float4>(T);
    L.cy = a.take<float4>(M);
    for (int r = 0; r < 4; ++r) L.xrec[r] = a.take<float4>(Tp);
    for (int r = 0; r < 3; ++r) L.yrec[r] = a.take<float4>(Mp);
    L.origin = a.take<float>(4);
    L.b = a.take<float>(M);
    L.log2b = a.take<float>(M);
    L.f = a.take<float>(T);
    L.g = a.take<float>(M);
    L.p = a.take<float>(T);
    L.q = a.take<float>(M);
    L.fp = a.take<float>(T);
    L.gp = a.take<float>(M);
    L.pp = a.take<float>(T);
    L.qp = a.take<float>(M);
    L.dy = a.take<float>((size_t)T * d);
    L.ds = a.take<float>((size_t)T * d);
    L.part[0] = a.take<float>(std::max(job_part_floats_max(d, T, M), job_part_floats_max(d, M, T)));
    L.part[1] = a.take<float>(job_part_floats_max(d, T, T));
    L.part[2] = a.take<float>(job_part_floats_max(d, M, M));
    L.ntick = std::max(job_tickets_max(T), job_tickets_max(M));
    for (int i = 0; i < 3; ++i) L.tick[i] = a.take<unsigned>(L.ntick);
    L.bar = a.take<unsigned>(kFusedBarWords);
    L.xch = a.take<unsigned long long>(4 * ((size_t)T + M));
    L.bytes = a.off + 256;
    return L;
}

static const uint32_t kKnownFlags = CT_DEBIAS | CT_GRAD_W | CT_VALUE | CT_WARM_START |
                                    CT_REF_CACHED | CT_SAFE_LSE | CT_ONE_STREAM | CT_FUSED |
                                    CT_UNFUSED | CT_DIFFERENCE | CT_TINY | CT_MESH;

static ct_status validate(const float* x, int64_t T, const float* y, int64_t M,
                          const ct_sinkhorn_opts* o) {
    if (!o) return fail(CT_E_ARG, "opts is null");
    if (o->d != 2 && o->d != 3) return fail(CT_E_SHAPE, "d must be 2 or 3 (got %d)", o->d);
    if (T < 1 || M < 1) return fail(CT_E_SHAPE, "T and M must be >= 1 (T=%lld, M=%lld)",
                                    (long long)T, (long long)M);
    if (T > (int64_t(1) << 30) || M > (int64_t(1) << 30))
        return fail(CT_E_SHAPE, "T and M must be <= 2^30");
    if (!(o->eps > 0.f) || !std::isfinite(o->eps))
        return fail(CT_E_ARG, "eps must be finite and > 0");
    if (o->iters < 0) return fail(CT_E_ARG, "iters must be >= 0");
    if (o->flags & ~kKnownFlags) return fail(CT_E_ARG, "unknown flag bits 0x%x", o->flags & ~kKnownFlags);
    {
        const uint32_t ex = o->flags & (CT_FUSED | CT_UNFUSED | CT_TINY | CT_MESH);
        if (ex & (ex - 1))
            return fail(CT_E_ARG, "CT_FUSED, CT_UNFUSED, CT_TINY and CT_MESH exclude each other");
    }
    if (!x || !y) return fail(CT_E_ARG, "x and y must be non-null");
    return CT_OK;
}

// Launch-time constants of one problem.
struct SkConsts {
    int d, T, M;
    int expanded;   // lagged sweeps without offsets in the expanded form (unless CT_DIFFERENCE)
    float kappa, inv_kappa, inv_sqrt_kappa, log2a;
};

static SkConsts sk_consts(int T, int M, const ct_sinkhorn_opts* o) {
    const double kappa_d = kLog2e / (double)o->eps;
    SkConsts c;
    c.d = o->d;
    c.T = T;
    c.M = M;
    c.expanded = (o->flags & CT_DIFFERENCE) ? 0 : 1;
    c.kappa = (float)kappa_d;
    c.inv_kappa = (float)(1.0 / kappa_d);
    c.inv_sqrt_kappa = (float)(1.0 / std::sqrt(kappa_d));
    c.log2a = (float)(-std::log2((double)T));
    return c;
}

struct JobSet {
    Job j[kMaxJobs];
    int n = 0;
    void add(const Job& x) {
        if (x.nq > 0) j[n++] = x;
    }
};

static ct_status launch_set(const JobSet& js, const SkConsts& c, const Schedule& sc, bool lagged,
                            bool bary, hipStream_t st) {
    if (js.n == 0) return CT_OK;
    Launch Lc;
    std::memset(&Lc, 0, sizeof(Lc));
    Lc.kappa = c.kappa;
    Lc.inv_kappa = c.inv_kappa;
    Lc.inv_sqrt_kappa = c.inv_sqrt_kappa;
    Lc.expanded = c.expanded;
    int nb = 0;
    for (int i = 0; i < js.n; ++i) {
        Lc.job[i] = js.j[i];
        nb += plan_job(Lc.job[i], sc);
        Lc.blk_end[i] = nb;
    }
    Lc.njobs = js.n;
    CT_CHECK_HIP(launch_sweep(c.d, sc, lagged, bary, Lc, nb, st));
    return CT_OK;
}

// Job builders: queries x against keys y (f-type) or x (p-type); queries y
// against keys x (g-type) or y (q-type).
struct SkJobs {
    const SkLayout& L;
    const SkConsts& c;
    Job base() const {
        Job j;
        std::memset(&j, 0, sizeof(Job));
        j.rescued = L.counters + 1;
        return j;
    }
    Job f(float* out_pot, float4* out_rec, float* out_bary) const {
        Job j = base();
        j.qrec = L.cx; j.qpot = L.f; j.qlog2w_s = c.log2a;
        j.krec = L.yrec[0]; j.nq = c.T; j.nk = c.M;
        j.part = L.part[0]; j.ticket = L.tick[0];
        j.out_pot = out_pot; j.out_rec = out_rec; j.out_bary = out_bary;
        return j;
    }
    Job p(int cur, bool avg, float* out_pot, float4* out_rec, float* out_bary) const {
        Job j = base();
        j.qrec = L.cx; j.qpot = L.p; j.qlog2w_s = c.log2a; j.self_avg = avg;
        j.krec = L.xrec[2 + cur]; j.nq = c.T; j.nk = c.T;
        j.part = L.part[1]; j.ticket = L.tick[1];
        j.out_pot = out_pot; j.out_rec = out_rec; j.out_bary = out_bary;
        return j;
    }
    Job g(const float4* krec, float* out_pot, float4* out_rec) const {
        Job j = base();
        j.qrec = L.cy; j.qpot = L.g; j.qlog2w = L.log2b;
        j.krec = krec; j.nq = c.M; j.nk = c.T;
        j.part = L.part[0]; j.ticket = L.tick[0];
        j.out_pot = out_pot; j.out_rec = out_rec;
        return j;
    }
    Job q(int cur, bool avg, float* out_pot, float4* out_rec) const {
        Job j = base();
        j.qrec = L.cy; j.qpot = L.q; j.qlog2w = L.log2b; j.self_avg = avg;
        j.krec = L.yrec[1 + cur]; j.nq = c.M; j.nk = c.M;
        j.part = L.part[2]; j.ticket = L.tick[2];
        j.out_pot = out_pot; j.out_rec = out_rec;
        return j;
    }
};

// One auxiliary stream per device (default priority, non-blocking), created on first use.
static ct_status aux_stream(hipStream_t* out) {
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    int dev = 0;
    CT_CHECK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it == streams.end()) {
        hipStream_t s;
        CT_CHECK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        it = streams.emplace(dev, s).first;
    }
    *out = it->second;
    return CT_OK;
}

// Auxiliary stream and fork/join events of the two-stream schedule, made once and
// reused by every call (the allocation-free entry point); null members: made and
// destroyed by each call.
struct ForkJoin {
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

// Fused solve (all K iterations in one launch; see fused.hip).  By default it is
// taken when one iteration has at most kFusedAutoPairs point pairs: there the
// per-sweep launches are bound by launch latency, and two grid barriers per
// iteration cost less than the four or five kernel boundaries they replace
// (measured on an MI355X, K = 100, d = 3, T = M: 1.2x at 200-300 samples per side,
// 1.04x at 500; at 1000, 3*10^6 pairs per iteration, the barriers' cross-die
// cache write-backs cost more than the launches, 4.3 against 2.7 ms).  CT_FUSED
// forces it and CT_UNFUSED rules it out.  The grid has at most kFusedMaxBlocks
// blocks and never more than can be resident at once.
constexpr double kFusedAutoPairs = 1048576.0;
constexpr int kFusedMaxBlocks = 512;
constexpr unsigned kFusedWaitPolls = 1u << 20;

static ct_status run_fused(const SkLayout& L, const SkConsts& c, const SkJobs& J,
                           const ct_sinkhorn_opts* o, bool debias, bool ref_iter, bool warm,
                           bool safe_only, hipStream_t st, bool* ran) {
    *ran = false;
    const int T = c.T, M = c.M, d = c.d;
    const bool forced = o->flags & CT_FUSED;
    const double pa = (double)T * M + (debias ? (double)T * T : 0.0);
    const double pb = (double)M * T + (ref_iter ? (double)M * M : 0.0);
    if (!forced && pa + pb > kFusedAutoPairs) return CT_OK;
    int gmax = std::min(fused_resident_blocks(d), kFusedMaxBlocks);
    // test and tuning hook: a cap on the grid
    if (const char* e = std::getenv("CT_FUSED_GRID"))
        gmax = std::min(std::min(fused_resident_blocks(d), kFusedMaxGrid),
                        std::max(1, std::atoi(e)));
    if (gmax < 1) {
        if (forced) return fail(CT_E_UNSUPPORTED, "the fused solve cannot place a block on this device");
        return CT_OK;
    }
    // partial buffers of the layout: cross jobs, trajectory self, reference self
    const size_t cap_cross = std::max(job_part_floats_max(d, T, M), job_part_floats_max(d, M, T));
    const size_t cap_p = job_part_floats_max(d, T, T), cap_q = job_part_floats_max(d, M, M);
    const Schedule fs{kFusedR, kFusedWS, 0, 0};
    FusedLaunch F;
    std::memset(&F, 0, sizeof(F));
    // plan every job for about the same pairs per unit, so that one half-iteration
    // is about one unit per block; coarser units if a job's partials would not fit
    double ppb = std::max(pa, pb) / gmax;
    int units_max = 0;
    for (int attempt = 0;; ++attempt) {
        bool fits = true;
        units_max = 0;
        auto add = [&](FusedPhase& P, Job j, size_t cap) {
            const int u = plan_job_target(j, fs, ppb);
            const size_t need = j.splits > 1 ? (size_t)(2 + d) * j.splits * (size_t)j.nqb * 64 *
                                                   kFusedR * (4 / kFusedWS)
                                             : 0;
            if (need > cap) fits = false;
            P.job[P.njobs] = j;
            P.unit_end[P.njobs] = (P.njobs ? P.unit_end[P.njobs - 1] : 0) + u;
            ++P.njobs;
            units_max = std::max(units_max, P.unit_end[P.njobs - 1]);
        };
        for (int par = 0; par < 2; ++par) {
            FusedPhase& A = F.ph[par][0];
            FusedPhase& B = F.ph[par][1];
            A.njobs = B.njobs = 0;
            add(A, J.f(L.f, L.xrec[0], nullptr), cap_cross);
            if (debias) add(A, J.p(par, true, L.p, L.xrec[2 + (par ^ 1)], nullptr), cap_p);
            add(B, J.g(L.xrec[0], L.g, L.yrec[0]), cap_cross);
            if (ref_iter) add(B, J.q(par, true, L.q, L.yrec[1 + (par ^ 1)]), cap_q);
        }
        if (fits) break;
        if (attempt >= 30) {
            if (forced) return fail(CT_E_UNSUPPORTED, "the fused solve found no plan for T=%d, M=%d", T, M);
            return CT_OK;
        }
        ppb *= 2.0;
    }
    F.iters = o->iters;
    F.lagged0 = warm ? 1 : 0;
    F.safe_only = safe_only ? 1 : 0;
    F.bar = L.bar;
    F.expired = L.counters + 4;
    F.wait_polls = kFusedWaitPolls;
    // test hooks of the give-up path: a poll bound, and waits that no arrival count satisfies
    if (const char* e = std::getenv("CT_FUSED_WAIT_POLLS")) F.wait_polls = (unsigned)std::strtoul(e, nullptr, 10);
    if (const char* e = std::getenv("CT_FUSED_UNSATISFIABLE_WAITS")) F.target_extra = std::atoi(e) ? 1u : 0u;
    F.kappa = c.kappa;
    F.inv_kappa = c.inv_kappa;
    F.inv_sqrt_kappa = c.inv_sqrt_kappa;
    hipLaunchKernelGGL(k_zero3, dim3((kFusedBarWords + 255) / 256), dim3(256), 0, st, L.bar,
                       kFusedBarWords, nullptr, 0, nullptr, 0);
    CT_CHECK_HIP(hipGetLastError());
    CT_CHECK_HIP(launch_fused(d, F, std::min(gmax, units_max), st));
    *ran = true;
    return CT_OK;
}

// One-workgroup solve (all K iterations in one workgroup, everything in LDS; see
// tiny.hip).  By default it is taken, where the exchange solve is not, when one
// iteration has at most kTinyAutoPairs point pairs and the problem fits in the
// LDS a workgroup may take: one compute unit evaluates such an iteration faster
// than the GPU can synchronise across its dies (measured on an MI355X, K = 100,
// d = 3, whole call: 0.59 ms at T = M = 100 against 1.34 for the fused solve and
// 1.41 for per-sweep launches).  CT_TINY forces it (CT_E_UNSUPPORTED when the
// problem does not fit); CT_FUSED, CT_UNFUSED and CT_MESH rule it out.
constexpr double kTinyAutoPairs = 150000.0;

static size_t device_max_lds() {
    static std::mutex mu;
    static std::map<int, size_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 0;
    cache.emplace(dev, (size_t)std::max(0, v));
    return (size_t)std::max(0, v);
}

static ct_status run_tiny(const SkLayout& L, const SkConsts& c, const ct_sinkhorn_opts* o,
                          bool debias, bool ref_iter, bool warm, bool safe_only, hipStream_t st,
                          bool* ran) {
    *ran = false;
    const int T = c.T, M = c.M, d = c.d;
    const bool forced = o->flags & CT_TINY;
    const double pairs = 2.0 * T * M + (debias ? (double)T * T : 0.0) +
                         (ref_iter ? (double)M * M : 0.0);
    if (!forced && pairs > kTinyAutoPairs) return CT_OK;
    TinyArgs A;
    size_t lds = 0;
    const size_t cap = std::min(kTinyMaxLds, device_max_lds());
    // test and tuning hook: query rows per lane (1, 2 or 4) instead of the cost model's choice
    int r_force = 0;
    if (const char* e = std::getenv("CT_TINY_R")) {
        r_force = std::atoi(e);
        if (r_force != 1 && r_force != 2 && r_force != 4) r_force = 0;
    }
    if (!tiny_plan(T, M, d, debias, ref_iter, cap, r_force, A, lds)) {
        if (forced)
            return fail(CT_E_UNSUPPORTED, "T=%d, M=%d needs %zu bytes of LDS; the one-workgroup "
                                          "solve may take %zu", T, M, lds, cap);
        return CT_OK;
    }
    const int cur = o->iters & 1;   // the self record arrays current after K iterations
    A.cx = L.cx;
    A.cy = L.cy;
    A.log2b = L.log2b;
    A.f = L.f;
    A.g = L.g;
    A.p = L.p;
    A.q = L.q;
    A.xrec_f = L.xrec[0];
    A.yrec_g = L.yrec[0];
    A.xrec_p = L.xrec[2 + cur];
    A.yrec_q = L.yrec[1 + cur];
    A.rescued = L.counters + 1;
    A.d = d;
    A.iters = o->iters;
    A.lagged0 = warm ? 1 : 0;
    A.safe_only = safe_only ? 1 : 0;
    A.kappa = c.kappa;
    A.inv_kappa = c.inv_kappa;
    A.log2a = c.log2a;
    CT_CHECK_HIP(launch_tiny(d, A, lds, st));
    *ran = true;
    return CT_OK;
}

// Multi-workgroup exchange solve (all K iterations in one launch of blocks that
// each hold every point in LDS and own at most 64 rows of each point set; see
// mesh.hip).  By default it is taken when it plans (two or more blocks, every
// point in one block's LDS, all blocks resident at once), one iteration has more
// than kMeshMinPairs point pairs (below that the one-workgroup solve is as fast)
// and at most kMeshAutoPairs.  Measured on an MI355X, K = 100, d = 3, T = M,
// cached reference potential, whole call (exchange / one-workgroup / fused /
// per-sweep launches): T = 100: 0.63 / 0.59 / 1.34 / 1.41 ms; 300: 0.87 / 1.94 /
// 1.87 / 2.26; 500: 1.08 / 3.65 / 2.63 / 2.66; 1000: 1.54 / - / 7.0 / 2.70;
// 2000: 2.57 / - / 23.5 / 3.13; 2500 (1.9e7 pairs): 3.20 against 3.16 for per-sweep
// launches, so the default stops below.  CT_MESH forces it (CT_E_UNSUPPORTED when it
// cannot plan); CT_FUSED, CT_UNFUSED and CT_TINY rule it out.
constexpr double kMeshMinPairs = 40000.0;
constexpr double kMeshAutoPairs = 1.5e7;
constexpr unsigned kMeshWaitPolls = 1u << 18;

static ct_status run_mesh(const SkLayout& L, const SkConsts& c, const ct_sinkhorn_opts* o,
                          bool debias, bool ref_iter, bool warm, bool safe_only, hipStream_t st,
                          bool* ran) {
    *ran = false;
    const int T = c.T, M = c.M, d = c.d;
    const bool forced = o->flags & CT_MESH;
    const double pairs = 2.0 * T * M + (debias ? (double)T * T : 0.0) +
                         (ref_iter ? (double)M * M : 0.0);
    if (!forced && (pairs > kMeshAutoPairs || pairs <= kMeshMinPairs)) return CT_OK;
    MeshArgs A;
    size_t lds = 0;
    int blocks = 0;
    const size_t cap = std::min(kTinyMaxLds, device_max_lds());
    const bool planned = mesh_plan(T, M, d, debias, ref_iter, cap, false, A, lds, &blocks);
    if (!planned || blocks > mesh_resident_blocks(d, lds, false)) {
        if (forced)
            return fail(CT_E_UNSUPPORTED, "the exchange solve has no plan for T=%d, M=%d (it needs "
                                          "2 to %d blocks of at most %d rows and every point in "
                                          "%zu bytes of LDS)", T, M, kMeshMaxBlocks, kMeshRows, cap);
        return CT_OK;
    }
    const int cur = o->iters & 1;   // the self record arrays current after K iterations
    A.cx = L.cx;
    A.cy = L.cy;
    A.log2b = L.log2b;
    A.f = L.f;
    A.g = L.g;
    A.p = L.p;
    A.q = L.q;
    A.xrec_f = L.xrec[0];
    A.yrec_g = L.yrec[0];
    A.xrec_p = L.xrec[2 + cur];
    A.yrec_q = L.yrec[1 + cur];
    A.xch_f = L.xch;
    A.xch_p = L.xch + 2 * (size_t)T;
    A.xch_g = L.xch + 4 * (size_t)T;
    A.xch_q = L.xch + 4 * (size_t)T + 2 * (size_t)M;
    for (int h = 0; h < 2; ++h) {
        for (int j = 0; j < A.njobs[h]; ++j) {
            MeshJob& J = A.job[h][j];
            J.xch = J.yside ? (J.avg ? A.xch_q : A.xch_g) : (J.avg ? A.xch_p : A.xch_f);
        }
    }
    A.gat[0][0].xch = A.xch_g;
    if (A.ngat[0] > 1) A.gat[0][1].xch = A.xch_p;
    A.gat[1][0].xch = A.xch_f;
    if (A.ngat[1] > 1) A.gat[1][1].xch = A.xch_q;
    A.rescued = L.counters + 1;
    A.expired = L.counters + 4;
    A.polls = kMeshWaitPolls;
    // test hooks of the give-up path: a poll bound, and waits that no version satisfies
    if (const char* e = std::getenv("CT_MESH_WAIT_POLLS")) A.polls = (unsigned)std::strtoul(e, nullptr, 10);
    if (const char* e = std::getenv("CT_MESH_UNSATISFIABLE_WAITS")) A.version_extra = std::atoi(e) ? (1u << 20) : 0u;
    A.d = d;
    A.iters = o->iters;
    A.lagged0 = warm ? 1 : 0;
    A.safe_only = safe_only ? 1 : 0;
    A.kappa = c.kappa;
    A.inv_kappa = c.inv_kappa;
    A.log2a = c.log2a;
    const int nw = 4 * (T + M);
    hipLaunchKernelGGL(k_fill_ones64, dim3((nw + 255) / 256), dim3(256), 0, st, L.xch, nw);
    CT_CHECK_HIP(hipGetLastError());
    CT_CHECK_HIP(launch_mesh(d, A, lds, blocks, st));
    *ran = true;
    return CT_OK;
}

// Iterate-and-extrapolate for one problem whose arrays are staged in L.
static ct_status run_problem(const SkLayout& L, int T, int M, const ct_sinkhorn_opts* o,
                             hipStream_t st, const ForkJoin* fj) {
    const int d = o->d;
    const bool debias = o->flags & CT_DEBIAS;
    const bool want_v = o->flags & (CT_VALUE | CT_GRAD_W);
    const bool need_ref = debias && want_v;
    const bool ref_iter = need_ref && !(o->flags & CT_REF_CACHED);
    const bool warm = o->flags & CT_WARM_START;
    const bool safe_only = o->flags & CT_SAFE_LSE;
    const SkConsts c = sk_consts(T, M, o);
    const SkJobs J{L, c};
    const Schedule sA = schedule_for(d, T, M);
    const Schedule sB = schedule_for(d, M, T);

    int cur = 0;  // which ping-pong self record array is current
    bool fused = false;
    if (o->iters > 0 && !(o->flags & CT_UNFUSED)) {
        if (!(o->flags & (CT_FUSED | CT_TINY))) {
            ct_status rc = run_mesh(L, c, o, debias, ref_iter, warm, safe_only, st, &fused);
            if (rc) return rc;
        }
        if (!fused && !(o->flags & (CT_FUSED | CT_MESH))) {
            ct_status rc = run_tiny(L, c, o, debias, ref_iter, warm, safe_only, st, &fused);
            if (rc) return rc;
        }
        if (!fused && !(o->flags & (CT_TINY | CT_MESH))) {
            ct_status rc = run_fused(L, c, J, o, debias, ref_iter, warm, safe_only, st, &fused);
            if (rc) return rc;
        }
        if (fused) cur = o->iters & 1;
    }

    // The self problems do not depend on f and g: their K sweeps run on the
    // auxiliary stream (forked from / joined back into `st` with events) while the
    // cross sweeps run on `st`; with CT_ONE_STREAM the same launches are serialised
    // on `st`.
    const bool any_self = !fused && (debias || ref_iter);
    const bool two_streams = any_self && o->iters > 0 && !(o->flags & CT_ONE_STREAM);
    hipStream_t sst = st;
    hipEvent_t fork = nullptr, join = nullptr;
    const bool own_events = !(fj && fj->fork);
    if (two_streams) {
        if (own_events) {
            ct_status rc = aux_stream(&sst);
            if (rc) return rc;
            CT_CHECK_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
            CT_CHECK_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        } else {
            sst = fj->aux;
            fork = fj->fork;
            join = fj->join;
        }
        CT_CHECK_HIP(hipEventRecord(fork, st));
        CT_CHECK_HIP(hipStreamWaitEvent(sst, fork, 0));
    }
    if (any_self) {
        const Schedule sS = schedule_for(d, ref_iter ? M : T, ref_iter ? M : T);
        for (int k = 0; k < o->iters; ++k) {
            const bool lagged = !safe_only && (warm || k > 0);
            JobSet Sf;
            if (debias) Sf.add(J.p(cur, true, L.p, L.xrec[2 + (cur ^ 1)], nullptr));
            if (ref_iter) Sf.add(J.q(cur, true, L.q, L.yrec[1 + (cur ^ 1)]));
            ct_status rc = launch_set(Sf, c, sS, lagged, false, sst);
            if (rc) return rc;
            cur ^= 1;
        }
    }
    for (int k = 0; k < (fused ? 0 : o->iters); ++k) {
        const bool lagged = !safe_only && (warm || k > 0);
        JobSet A, B;
        A.add(J.f(L.f, L.xrec[0], nullptr));
        B.add(J.g(L.xrec[0], L.g, L.yrec[0]));
        ct_status rc = launch_set(A, c, sA, lagged, false, st);
        if (rc) return rc;
        rc = launch_set(B, c, sB, lagged, false, st);
        if (rc) return rc;
    }
    if (two_streams) {
        CT_CHECK_HIP(hipEventRecord(join, sst));
        CT_CHECK_HIP(hipStreamWaitEvent(st, join, 0));
        if (own_events) {
            CT_CHECK_HIP(hipEventDestroy(fork));
            CT_CHECK_HIP(hipEventDestroy(join));
        }
    }
    const bool lagged_final = !safe_only && (warm || o->iters > 0);
    {
        JobSet F;
        F.add(J.f(L.fp, L.xrec[1], L.dy));
        if (debias) F.add(J.p(cur, false, L.pp, nullptr, L.ds));
        ct_status rc = launch_set(F, c, sA, lagged_final, true, st);
        if (rc) return rc;
    }
    if (want_v) {
        JobSet F;
        F.add(J.g(L.xrec[1], L.gp, nullptr));
        if (need_ref) F.add(J.q(ref_iter ? cur : 0, false, L.qp, nullptr));
        ct_status rc = launch_set(F, c, sB, lagged_final, false, st);
        if (rc) return rc;
    }
    return CT_OK;
}

}  // namespace ct

using namespace ct;

extern "C" size_t ct_sinkhorn_workspace_size(int64_t T, int64_t M, const ct_sinkhorn_opts* o) {
    if (!o || (o->d != 2 && o->d != 3) || T < 1 || M < 1 || T > (int64_t(1) << 30) ||
        M > (int64_t(1) << 30))
        return 0;
    return sk_layout(nullptr, (int)T, (int)M, o->d).bytes;
}

namespace ct {

// Host checks of one gradient call's arguments (everything but the workspace).
static ct_status validate_call(const float* x, int64_t T64, const float* y, int64_t M64,
                               const ct_sinkhorn_opts* o, const float* grad_x,
                               const float* grad_w, const float* value, const float* pot) {
    ct_status rc = validate(x, T64, y, M64, o);
    if (rc) return rc;
    if (!grad_x) return fail(CT_E_ARG, "grad_x must be non-null");
    if (grad_w && !(o->flags & CT_GRAD_W)) return fail(CT_E_ARG, "grad_w given without CT_GRAD_W");
    if (!grad_w && (o->flags & CT_GRAD_W)) return fail(CT_E_ARG, "CT_GRAD_W needs grad_w");
    if (value && !(o->flags & CT_VALUE)) return fail(CT_E_ARG, "value given without CT_VALUE");
    if (!value && (o->flags & CT_VALUE)) return fail(CT_E_ARG, "CT_VALUE needs value");
    if (!pot && (o->flags & (CT_WARM_START | CT_REF_CACHED)))
        return fail(CT_E_ARG, "CT_WARM_START / CT_REF_CACHED need pot");
    return CT_OK;
}

// The whole gradient call on the workspace `ws` (both entry points).
static ct_status sinkhorn_grad_impl(const float* x, int64_t T64, const float* y, const float* w,
                                    int64_t M64, const ct_sinkhorn_opts* o, float* grad_x,
                                    float* grad_w, float* value, float* pot, float* pot_plus,
                                    float* aux, void* ws, size_t ws_bytes, void* stream,
                                    const ForkJoin* fj) {
    ct_status rc = validate_call(x, T64, y, M64, o, grad_x, grad_w, value, pot);
    if (rc) return rc;
    const int T = (int)T64, M = (int)M64, d = o->d;
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CT_E_WORKSPACE, "workspace not 256-byte aligned");
    SkLayout L = sk_layout(ws, T, M, d);
    if (ws_bytes < L.bytes)
        return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool debias = o->flags & CT_DEBIAS;
    const bool want_v = o->flags & (CT_VALUE | CT_GRAD_W);
    const bool need_ref = debias && want_v;
    const double kappa_d = kLog2e / (double)o->eps;

    // zero the counters and arrival tickets with a fill kernel (no memset nodes,
    // so the sequence can be captured into a graph)
    {
        const int nt = (int)L.ntick;
        hipLaunchKernelGGL(k_zero3, dim3((nt + 255) / 256), dim3(256), 0, st, L.tick[0], nt,
                           L.tick[1], nt, L.tick[2], nt);
        hipLaunchKernelGGL(k_zero3, dim3(1), dim3(256), 0, st, L.counters, kCounters, nullptr, 0,
                           nullptr, 0);
        CT_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_wsum, dim3(1), dim3(1024), 0, st, w, M, L.wsum);
    CT_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_origin, dim3(1), dim3(1024), 0, st, x, T, y, M, d, L.origin);
    CT_CHECK_HIP(hipGetLastError());
    StageArgs A;
    A.x = x; A.y = y; A.w = w; A.pot_in = pot;
    A.warm = (o->flags & CT_WARM_START) ? 1 : 0;
    A.ref_cached = (o->flags & CT_REF_CACHED) ? 1 : 0;
    A.T = T; A.M = M; A.d = d; A.Tpad = pad_keys(T); A.Mpad = pad_keys(M);
    A.sqrt_kappa = (float)std::sqrt(kappa_d);
    A.kappa = (float)kappa_d;
    A.log2a = (float)(-std::log2((double)T));
    A.wsum = L.wsum; A.origin = L.origin; A.cx = L.cx; A.cy = L.cy; A.b = L.b; A.log2b = L.log2b;
    A.f = L.f; A.g = L.g; A.p = L.p; A.q = L.q;
    for (int r = 0; r < 4; ++r) A.xrec[r] = L.xrec[r];
    for (int r = 0; r < 3; ++r) A.yrec[r] = L.yrec[r];
    A.fp = L.fp; A.gp = L.gp; A.pp = L.pp; A.qp = L.qp;
    A.nonfinite = L.counters;
    const int n = std::max(pad_keys(T), pad_keys(M));
    hipLaunchKernelGGL(k_stage, dim3((n + 255) / 256), dim3(256), 0, st, A);
    CT_CHECK_HIP(hipGetLastError());

    rc = run_problem(L, T, M, o, st, fj);
    if (rc) return rc;

    hipLaunchKernelGGL(k_grad_x, dim3((T * d + 255) / 256), dim3(256), 0, st, L.dy,
                       debias ? L.ds : nullptr, T * d, (float)(2.0 / T), L.counters + 4, grad_x);
    CT_CHECK_HIP(hipGetLastError());
    if (want_v) {
        ReduceArgs R;
        R.T = T; R.M = M; R.debias = debias; R.need_ref = need_ref;
        R.kappa = (float)kappa_d;
        R.fp = L.fp; R.g = L.g; R.gp = L.gp; R.p = L.p; R.pp = L.pp; R.q = L.q; R.qp = L.qp;
        R.b = L.b; R.wsum = L.wsum; R.counters = L.counters; R.bG = L.bG;
        R.value = value; R.aux = aux;
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, R);
        CT_CHECK_HIP(hipGetLastError());
        if (grad_w) {
            hipLaunchKernelGGL(k_grad_w, dim3((M + 255) / 256), dim3(256), 0, st, L.gp,
                               need_ref ? L.qp : nullptr, M, L.bG, L.wsum, L.counters + 4, grad_w);
            CT_CHECK_HIP(hipGetLastError());
        }
    } else if (aux) {
        hipLaunchKernelGGL(k_zero3, dim3(1), dim3(256), 0, st, reinterpret_cast<unsigned*>(aux), 4,
                           nullptr, 0, nullptr, 0);
        CT_CHECK_HIP(hipGetLastError());
    }
    if (aux) {
        hipLaunchKernelGGL(k_counters_out, dim3(1), dim3(64), 0, st, L.counters, aux);
        CT_CHECK_HIP(hipGetLastError());
    }
    if (pot) {
        CT_CHECK_HIP(hipMemcpyAsync(pot, L.f, sizeof(float) * T, hipMemcpyDeviceToDevice, st));
        CT_CHECK_HIP(hipMemcpyAsync(pot + T, L.g, sizeof(float) * M, hipMemcpyDeviceToDevice, st));
        CT_CHECK_HIP(hipMemcpyAsync(pot + T + M, L.p, sizeof(float) * T, hipMemcpyDeviceToDevice, st));
        CT_CHECK_HIP(hipMemcpyAsync(pot + 2 * (size_t)T + M, L.q, sizeof(float) * M,
                                    hipMemcpyDeviceToDevice, st));
    }
    if (pot_plus) {
        float* pp = pot_plus;
        CT_CHECK_HIP(hipMemcpyAsync(pp, L.fp, sizeof(float) * T, hipMemcpyDeviceToDevice, st));
        CT_CHECK_HIP(hipMemcpyAsync(pp + T, L.gp, sizeof(float) * M, hipMemcpyDeviceToDevice, st));
        CT_CHECK_HIP(hipMemcpyAsync(pp + T + M, L.pp, sizeof(float) * T, hipMemcpyDeviceToDevice, st));
        CT_CHECK_HIP(hipMemcpyAsync(pp + 2 * (size_t)T + M, L.qp, sizeof(float) * M,
                                    hipMemcpyDeviceToDevice, st));
    }
    return CT_OK;
}

// ------------------------------------------------- allocation-free variant
// Scratch of ct_sinkhorn_grad_static: one array per device, held until the process
// ends.  Host code never passes `scratch` itself (its host name is a stand-in, not
// a device address): each device's address comes from hipGetSymbolAddress once,
// with that device current, and is kept in g_static below.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct StaticDevice {
    void* ptr = nullptr;   // device address of `scratch` on this device
    ForkJoin fj;           // auxiliary stream and events made at set-up
};

// Per-device set-up on the first call on that device: the scratch address, the
// auxiliary stream and the fork/join events.  Later calls only look them up.
static ct_status static_device(StaticDevice* out) {
    static std::mutex mu;
    static std::map<int, StaticDevice> devs;
    int dev = 0;
    CT_CHECK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = devs.find(dev);
    if (it == devs.end()) {
        StaticDevice sd;
        CT_CHECK_HIP(hipGetSymbolAddress(&sd.ptr, HIP_SYMBOL(scratch)));
        if (!sd.ptr || reinterpret_cast<uintptr_t>(sd.ptr) % 256)
            return fail(CT_E_HIP, "static scratch has no usable device address on device %d", dev);
        ct_status rc = aux_stream(&sd.fj.aux);
        if (rc) return rc;
        CT_CHECK_HIP(hipEventCreateWithFlags(&sd.fj.fork, hipEventDisableTiming));
        CT_CHECK_HIP(hipEventCreateWithFlags(&sd.fj.join, hipEventDisableTiming));
        it = devs.emplace(dev, sd).first;
    }
    *out = it->second;
    return CT_OK;
}

}  // namespace ct

extern "C" ct_status ct_sinkhorn_grad(const float* x, int64_t T64, const float* y, const float* w,
                                      int64_t M64, const ct_sinkhorn_opts* o, float* grad_x,
                                      float* grad_w, float* value, float* pot, float* pot_plus,
                                      float* aux, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    return sinkhorn_grad_impl(x, T64, y, w, M64, o, grad_x, grad_w, value, pot, pot_plus, aux, ws,
                              ws_bytes, stream, nullptr);
}

extern "C" size_t ct_sinkhorn_static_scratch_bytes(void) { return kStaticScratchBytes; }

extern "C" ct_status ct_sinkhorn_grad_static(const float* x, int64_t T64, const float* y,
                                             const float* w, int64_t M64,
                                             const ct_sinkhorn_opts* o, float* grad_x,
                                             float* grad_w, float* value, float* pot,
                                             float* pot_plus, float* aux, void* stream) {
    clear_error();
    ct_status rc = validate_call(x, T64, y, M64, o, grad_x, grad_w, value, pot);
    if (rc) return rc;
    const size_t need = sk_layout(nullptr, (int)T64, (int)M64, o->d).bytes;
    if (need > kStaticScratchBytes)
        return fail(CT_E_WORKSPACE,
                    "problem needs %zu bytes of scratch; the static scratch holds %zu "
                    "(T=%lld, M=%lld, d=%d): use ct_sinkhorn_grad with a workspace",
                    need, kStaticScratchBytes, (long long)T64, (long long)M64, o->d);
    if (profiling())
        return fail(CT_E_UNSUPPORTED, "launch profiling creates events; disable it for this entry point");
    StaticDevice sd;
    rc = static_device(&sd);
    if (rc) return rc;
    return sinkhorn_grad_impl(x, T64, y, w, M64, o, grad_x, grad_w, value, pot, pot_plus, aux,
                              sd.ptr, kStaticScratchBytes, stream, &sd.fj);
}

// ------------------------------------------------------------- autotuning

namespace ct {

// Synthetic staged problem for timing: points from a hash in [0,1]^d, equal
// masses, zero potentials (the timing of a sweep does not depend on the data
// beyond its size).
__device__ __forceinline__ float hash01(unsigned v) {
    v ^= v >> 16;
    v *= 0x7feb352du;
    v ^= v >> 15;
    v *= 0x846ca68bu;
    v ^= v >> 16;
    return (float)(v >> 8) * (1.0f / 16777216.0f);
}

__global__ __launch_bounds__(256) void k_synth(int T, int M, int d, int Tpad, int Mpad,
                                               float sqrt_kappa, float log2a, float log2b,
                                               float4* cx, float4* cy, float4* x0, float4* x1,
                                               float4* x2, float4* x3, float4* y0, float4* y1,
                                               float4* y2, float* f, float* g, float* p, float* q,
                                               float* b, float* lb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float ninf = -__builtin_huge_valf();
    if (i < Tpad) {
        float c[3];
        for (int t = 0; t < 3; ++t) c[t] = hash01(2654435761u * (unsigned)i + 97u * t + 1u) * sqrt_kappa;
        const float h = i < T ? log2a : ninf;
        float4 r = d == 2 ? make_float4(c[0], c[1], h, 0.f) : make_float4(c[0], c[1], c[2], h);
        x0[i] = r; x1[i] = r; x2[i] = r; x3[i] = r;
        if (i < T) {
            cx[i] = make_float4(c[0], c[1], c[2], 0.f);
            f[i] = 0.f;
            p[i] = 0.f;
        }
    }
    if (i < Mpad) {
        float c[3];
        for (int t = 0; t < 3; ++t) c[t] = hash01(40503u * (unsigned)i + 131u * t + 7u) * sqrt_kappa;
        const float h = i < M ? log2b : ninf;
        float4 r = d == 2 ? make_float4(c[0], c[1], h, 0.f) : make_float4(c[0], c[1], c[2], h);
        y0[i] = r; y1[i] = r; y2[i] = r;
        if (i < M) {
            cy[i] = make_float4(c[0], c[1], c[2], 0.f);
            g[i] = 0.f;
            q[i] = 0.f;
            b[i] = exp2f(log2b);
            lb[i] = log2b;
        }
    }
}

}  // namespace ct

extern "C" ct_status ct_autotune_sinkhorn(int64_t T64, int64_t M64, const ct_sinkhorn_opts* o,
                                          void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    static const float dummy = 0.f;
    ct_status rc = validate(&dummy, T64, &dummy, M64, o);
    if (rc) return rc;
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    const int T = (int)T64, M = (int)M64, d = o->d;
    SkLayout L = sk_layout(ws, T, M, d);
    if (ws_bytes < L.bytes) return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = refuse_capture(st, "ct_autotune_sinkhorn");
    if (rc) return rc;
    const double kappa_d = kLog2e / (double)o->eps;
    const int n = std::max(pad_keys(T), pad_keys(M));
    hipLaunchKernelGGL(k_zero3, dim3(((int)L.ntick + 255) / 256), dim3(256), 0, st, L.tick[0],
                       (int)L.ntick, L.tick[1], (int)L.ntick, L.tick[2], (int)L.ntick);
    hipLaunchKernelGGL(k_zero3, dim3(1), dim3(256), 0, st, L.counters, kCounters, nullptr, 0, nullptr, 0);
    hipLaunchKernelGGL(k_synth, dim3((n + 255) / 256), dim3(256), 0, st, T, M, d, pad_keys(T),
                       pad_keys(M), (float)std::sqrt(kappa_d), (float)(-std::log2((double)T)),
                       (float)(-std::log2((double)M)), L.cx, L.cy, L.xrec[0], L.xrec[1], L.xrec[2],
                       L.xrec[3], L.yrec[0], L.yrec[1], L.yrec[2], L.f, L.g, L.p, L.q, L.b, L.log2b);
    CT_CHECK_HIP(hipGetLastError());
    hipEvent_t e0, e1;
    CT_CHECK_HIP(hipEventCreate(&e0));
    CT_CHECK_HIP(hipEventCreate(&e1));
    Schedule cand[kMaxCandidates];
    const int nc = schedule_candidates(cand, kMaxCandidates);
    const SkConsts c = sk_consts(T, M, o);
    const SkJobs J{L, c};
    const bool debias = o->flags & CT_DEBIAS;
    const bool ref_iter = debias && (o->flags & (CT_VALUE | CT_GRAD_W));
    // the launches of the default (two-stream) schedule: cross f, cross g, self p + q
    JobSet sets[3];
    sets[0].add(J.f(L.f, L.xrec[0], nullptr));
    sets[1].add(J.g(L.xrec[0], L.g, L.yrec[0]));
    if (debias) sets[2].add(J.p(0, true, L.p, L.xrec[3], nullptr));
    if (ref_iter) sets[2].add(J.q(0, true, L.q, L.yrec[2]));
    const int keys[3][2] = {{T, M}, {M, T}, {ref_iter ? M : T, ref_iter ? M : T}};
    for (int side = 0; side < 3; ++side) {
        const JobSet& S = sets[side];
        if (S.n == 0) continue;
        float best = 1e30f;
        Schedule bs = cand[0];
        for (int ci = 0; ci < nc; ++ci) {
            ct_status rc2 = launch_set(S, c, cand[ci], true, false, st);  // warm-up
            if (rc2) return rc2;
            CT_CHECK_HIP(hipEventRecord(e0, st));
            const int reps = 3;
            for (int r = 0; r < reps; ++r) {
                rc2 = launch_set(S, c, cand[ci], true, false, st);
                if (rc2) return rc2;
            }
            CT_CHECK_HIP(hipEventRecord(e1, st));
            CT_CHECK_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            CT_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= reps;
            if (ms < best) {
                best = ms;
                bs = cand[ci];
            }
        }
        tuning_record(d, keys[side][0], keys[side][1], bs, (int)(best * 1000.f + 0.5f));
    }
    CT_CHECK_HIP(hipEventDestroy(e0));
    CT_CHECK_HIP(hipEventDestroy(e1));
    return CT_OK;
}

extern "C" ct_status ct_status_sync(const void* ws, float resid_tol, uint32_t* nonfinite,
                                    uint32_t* rescued, float* resid, void* stream) {
    clear_error();
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CT_E_WORKSPACE, "workspace not 256-byte aligned");
    if (!(resid_tol >= 0.f)) return fail(CT_E_ARG, "resid_tol must be >= 0 (0: no convergence check)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    ct_status rc = refuse_capture(st, "ct_status_sync");
    if (rc) return rc;
    // the counters come before every size-dependent buffer of the layout; a stand-in
    // base (never dereferenced) gives their offset
    char* const probe = reinterpret_cast<char*>(uintptr_t(1) << 20);
    const size_t off = static_cast<size_t>(reinterpret_cast<char*>(sk_layout(probe, 1, 1, 2).counters) - probe);
    unsigned c[kCounters] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    CT_CHECK_HIP(hipMemcpyAsync(c, static_cast<const char*>(ws) + off, sizeof(c),
                                hipMemcpyDeviceToHost, st));
    CT_CHECK_HIP(hipStreamSynchronize(st));
    float r;
    std::memcpy(&r, &c[2], sizeof(r));
    if (!c[3]) r = __builtin_nanf("");
    if (nonfinite) *nonfinite = c[0];
    if (rescued) *rescued = c[1];
    if (resid) *resid = r;
    if (c[4])
        return fail(CT_E_DEVICE, "a wait of the last call's fused or exchange solve gave up: "
                                 "its outputs are not valid");
    if (c[0])
        return fail(CT_E_NONFINITE, "the last gradient call saw %u non-finite coordinates or "
                                    "non-positive weights: its outputs are not valid", c[0]);
    if (resid_tol > 0.f && c[3] && !(r <= resid_tol))
        return fail(CT_WARN_NOT_CONVERGED, "column residual %.3g above the tolerance %.3g", r,
                    resid_tol);
    return CT_OK;
}
