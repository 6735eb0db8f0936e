// ct_sinkhorn_grad: debiased Sinkhorn divergence gradient for one problem
// (Sec. II-B, eqs. 5-7).  Staging, the iteration schedule, the final
// extrapolation pass and the reductions; the sweeps themselves are in sweep.hip.
#include <cmath>
#include <cstring>

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

struct StageArgs {
    const float* x;
    const float* y;
    const float* w;
    const float* pot_in;     // [2T+2M] warm start (f, g, p, q) or null
    int warm, ref_cached;
    int T, M, d;
    float sqrt_kappa, kappa, log2a;
    const double* wsum;
    float4* cx;
    float4* cy;
    float* b;
    float* log2b;
    float* f;
    float* g;
    float* p;
    float* q;
    float* h2y_g;            // key terms of y for the f-update: log2 b + kappa g
    float* h2x_p;            // key terms of x for the self update: log2 a + kappa p
    float* h2y_q;            // key terms of y for the reference self update
    float *fp, *gp, *pp, *qp; // extrapolated potentials, zeroed here
    unsigned* nonfinite;
};

// Pre-scale coordinates, form the reference masses and the initial key terms.
__global__ __launch_bounds__(256) void k_stage(StageArgs A) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < A.T) {
        float c[3] = {0.f, 0.f, 0.f};
        bool bad = false;
        for (int t = 0; t < A.d; ++t) {
            const float v = A.x[(size_t)i * A.d + t];
            bad |= !isfinite(v);
            c[t] = v * A.sqrt_kappa;
        }
        A.cx[i] = make_float4(c[0], c[1], c[2], 0.f);
        const float f0 = A.warm ? A.pot_in[i] : 0.f;
        const float p0 = A.warm ? A.pot_in[(size_t)A.T + A.M + i] : 0.f;
        A.f[i] = f0;
        A.p[i] = p0;
        A.h2x_p[i] = __builtin_fmaf(p0, A.kappa, A.log2a);
        A.fp[i] = 0.f;
        A.pp[i] = 0.f;
        if (bad) atomicAdd(A.nonfinite, 1u);
    }
    if (i < A.M) {
        float c[3] = {0.f, 0.f, 0.f};
        bool bad = false;
        for (int t = 0; t < A.d; ++t) {
            const float v = A.y[(size_t)i * A.d + t];
            bad |= !isfinite(v);
            c[t] = v * A.sqrt_kappa;
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
        A.h2y_g[i] = __builtin_fmaf(g0, A.kappa, lb);
        A.h2y_q[i] = __builtin_fmaf(q0, A.kappa, lb);
        A.gp[i] = 0.f;
        A.qp[i] = 0.f;
        if (bad) atomicAdd(A.nonfinite, 1u);
    }
}

// grad_x = 2 a (Ds - Dy)  (debiased) or -2 a Dy.
__global__ __launch_bounds__(256) void k_grad_x(const float* __restrict__ dy,
                                                const float* __restrict__ ds, int n, float two_a,
                                                float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = ds ? ds[i] - dy[i] : -dy[i];
    out[i] = two_a * v;
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
    const unsigned* counters;   // [0] non-finite inputs, [1] rescued rows
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
        if (A.value) *A.value = (float)S;
        if (A.aux) {
            A.aux[0] = (float)ot_ab;
            A.aux[1] = A.debias ? (float)ot_aa : 0.f;
            A.aux[2] = A.need_ref ? (float)ot_bb : 0.f;
            A.aux[3] = (float)red[7][0];
        }
    }
}

__global__ __launch_bounds__(256) void k_grad_w(const float* __restrict__ gp,
                                                const float* __restrict__ qp, int M,
                                                const double* __restrict__ bG,
                                                const double* __restrict__ wsum,
                                                float* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double G = qp ? (double)gp[j] - (double)qp[j] : (double)gp[j];
    out[j] = (float)((G - *bG) / *wsum);
}

__global__ void k_counters_out(const unsigned* __restrict__ c, float* __restrict__ aux) {
    if (threadIdx.x == 0) {
        aux[4] = (float)c[1];
        aux[5] = (float)c[0];
        aux[6] = 0.f;
        aux[7] = 0.f;
    }
}

// --------------------------------------------------------------- layout

struct SkLayout {
    double* wsum;
    double* bG;
    unsigned* counters;      // [4]
    float4* cx;
    float4* cy;
    float* b;
    float* log2b;
    float *f, *g, *p, *q;
    float *fp, *gp, *pp, *qp;
    float *h2y_g, *h2x_f, *h2x_fp;
    float *h2x_p[2], *h2y_q[2];
    float *dy, *ds;
    float *part0, *part1;
    unsigned *tick0, *tick1;
    size_t bytes;
};

static SkLayout sk_layout(void* ws, int T, int M, int d) {
    Arena a(ws);
    SkLayout L;
    L.wsum = a.take<double>(1);
    L.bG = a.take<double>(1);
    L.counters = a.take<unsigned>(4);
    L.cx = a.take<float4>(T);
    L.cy = a.take<float4>(M);
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
    L.h2y_g = a.take<float>(M);
    L.h2x_f = a.take<float>(T);
    L.h2x_fp = a.take<float>(T);
    L.h2x_p[0] = a.take<float>(T);
    L.h2x_p[1] = a.take<float>(T);
    L.h2y_q[0] = a.take<float>(M);
    L.h2y_q[1] = a.take<float>(M);
    L.dy = a.take<float>((size_t)T * d);
    L.ds = a.take<float>((size_t)T * d);
    const size_t p0 = std::max(job_part_floats_max(d, T, M), job_part_floats_max(d, M, T));
    const size_t p1 = std::max(job_part_floats_max(d, T, T), job_part_floats_max(d, M, M));
    L.part0 = a.take<float>(p0);
    L.part1 = a.take<float>(p1);
    L.tick0 = a.take<unsigned>(std::max(job_tickets_max(T), job_tickets_max(M)));
    L.tick1 = a.take<unsigned>(std::max(job_tickets_max(T), job_tickets_max(M)));
    L.bytes = a.off + 256;
    return L;
}

static const uint32_t kKnownFlags =
    CT_DEBIAS | CT_GRAD_W | CT_VALUE | CT_WARM_START | CT_REF_CACHED | CT_SAFE_LSE;

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
    if (!x || !y) return fail(CT_E_ARG, "x and y must be non-null");
    return CT_OK;
}

// Iterate-and-extrapolate for one problem whose arrays are staged in L.
static ct_status run_problem(const SkLayout& L, int T, int M, const ct_sinkhorn_opts* o,
                             hipStream_t st) {
    const int d = o->d;
    const bool debias = o->flags & CT_DEBIAS;
    const bool want_v = o->flags & (CT_VALUE | CT_GRAD_W);
    const bool need_ref = debias && want_v;
    const bool ref_iter = need_ref && !(o->flags & CT_REF_CACHED);
    const bool warm = o->flags & CT_WARM_START;
    const bool safe_only = o->flags & CT_SAFE_LSE;
    const double kappa_d = kLog2e / (double)o->eps;
    const float kappa = (float)kappa_d;
    const float inv_kappa = (float)(1.0 / kappa_d);
    const float inv_sqrt_kappa = (float)(1.0 / std::sqrt(kappa_d));
    const float log2a = (float)(-std::log2((double)T));

    const Schedule sxy = schedule_for(d, T, M);
    const Schedule syx = schedule_for(d, M, T);

    auto base_job = [&](Job& j) {
        std::memset(&j, 0, sizeof(Job));
        j.rescued = L.counters + 1;
    };
    auto launch2 = [&](Job* j0, Job* j1, const Schedule& sc, bool lagged, bool bary) -> ct_status {
        Launch Lc;
        std::memset(&Lc, 0, sizeof(Lc));
        Lc.kappa = kappa;
        Lc.inv_kappa = inv_kappa;
        Lc.inv_sqrt_kappa = inv_sqrt_kappa;
        int nb0 = 0, nb1 = 0;
        if (j0) {
            Lc.job[0] = *j0;
            nb0 = plan_job(Lc.job[0], sc.R, sc.blocks_per_cu);
        }
        if (j1) {
            Lc.job[1] = *j1;
            nb1 = plan_job(Lc.job[1], sc.R, sc.blocks_per_cu);
        }
        if (!j0) {
            Lc.job[0] = Lc.job[1];
            nb0 = nb1;
            nb1 = 0;
        }
        Lc.nblk0 = nb0;
        CT_CHECK_HIP(launch_sweep(d, sc.R, lagged, bary, Lc, nb0 + nb1, st));
        return CT_OK;
    };

    // x-side jobs (queries x) and y-side jobs (queries y)
    auto job_f = [&](Job& j, float* out_pot, float* out_h, float* out_bary) {
        base_job(j);
        j.qc = L.cx; j.qpot = L.f; j.qlog2w_s = log2a; j.self_avg = 0;
        j.kc = L.cy; j.kh = L.h2y_g; j.nq = T; j.nk = M;
        j.part = L.part0; j.ticket = L.tick0;
        j.out_pot = out_pot; j.out_h = out_h; j.out_bary = out_bary;
    };
    auto job_p = [&](Job& j, int cur, bool avg, float* out_pot, float* out_h, float* out_bary) {
        base_job(j);
        j.qc = L.cx; j.qpot = L.p; j.qlog2w_s = log2a; j.self_avg = avg;
        j.kc = L.cx; j.kh = L.h2x_p[cur]; j.nq = T; j.nk = T;
        j.part = L.part1; j.ticket = L.tick1;
        j.out_pot = out_pot; j.out_h = out_h; j.out_bary = out_bary;
    };
    auto job_g = [&](Job& j, const float* kh, float* out_pot, float* out_h) {
        base_job(j);
        j.qc = L.cy; j.qpot = L.g; j.qlog2w = L.log2b; j.self_avg = 0;
        j.kc = L.cx; j.kh = kh; j.nq = M; j.nk = T;
        j.part = L.part0; j.ticket = L.tick0;
        j.out_pot = out_pot; j.out_h = out_h;
    };
    auto job_q = [&](Job& j, int cur, bool avg, float* out_pot, float* out_h) {
        base_job(j);
        j.qc = L.cy; j.qpot = L.q; j.qlog2w = L.log2b; j.self_avg = avg;
        j.kc = L.cy; j.kh = L.h2y_q[cur]; j.nq = M; j.nk = M;
        j.part = L.part1; j.ticket = L.tick1;
        j.out_pot = out_pot; j.out_h = out_h;
    };

    int cur = 0;  // which of the ping-pong self key-term buffers is current
    for (int k = 0; k < o->iters; ++k) {
        const bool lagged = !safe_only && (warm || k > 0);
        Job jf, jp, jg, jq;
        job_f(jf, L.f, L.h2x_f, nullptr);
        if (debias) job_p(jp, cur, true, L.p, L.h2x_p[cur ^ 1], nullptr);
        ct_status rc = launch2(&jf, debias ? &jp : nullptr, sxy, lagged, false);
        if (rc) return rc;
        job_g(jg, L.h2x_f, L.g, L.h2y_g);
        if (ref_iter) job_q(jq, cur, true, L.q, L.h2y_q[cur ^ 1]);
        rc = launch2(&jg, ref_iter ? &jq : nullptr, syx, lagged, false);
        if (rc) return rc;
        cur ^= 1;
    }
    const bool lagged_final = !safe_only && (warm || o->iters > 0);
    {
        Job jf, jp;
        job_f(jf, L.fp, L.h2x_fp, L.dy);
        if (debias) job_p(jp, cur, false, L.pp, nullptr, L.ds);
        ct_status rc = launch2(&jf, debias ? &jp : nullptr, sxy, lagged_final, true);
        if (rc) return rc;
    }
    if (want_v) {
        Job jg, jq;
        job_g(jg, L.h2x_fp, L.gp, nullptr);
        if (need_ref) job_q(jq, cur, false, L.qp, nullptr);
        ct_status rc = launch2(&jg, need_ref ? &jq : nullptr, syx, lagged_final, false);
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

extern "C" ct_status ct_sinkhorn_grad(const float* x, int64_t T64, const float* y, const float* w,
                                      int64_t M64, const ct_sinkhorn_opts* o, float* grad_x,
                                      float* grad_w, float* value, float* pot, float* pot_plus,
                                      float* aux, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    ct_status rc = validate(x, T64, y, M64, o);
    if (rc) return rc;
    if (!grad_x) return fail(CT_E_ARG, "grad_x must be non-null");
    if (grad_w && !(o->flags & CT_GRAD_W)) return fail(CT_E_ARG, "grad_w given without CT_GRAD_W");
    if (!grad_w && (o->flags & CT_GRAD_W)) return fail(CT_E_ARG, "CT_GRAD_W needs grad_w");
    if (value && !(o->flags & CT_VALUE)) return fail(CT_E_ARG, "value given without CT_VALUE");
    if (!value && (o->flags & CT_VALUE)) return fail(CT_E_ARG, "CT_VALUE needs value");
    if (!pot && (o->flags & (CT_WARM_START | CT_REF_CACHED)))
        return fail(CT_E_ARG, "CT_WARM_START / CT_REF_CACHED need pot");
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
        const int nt = (int)std::max(job_tickets_max(T), job_tickets_max(M));
        hipLaunchKernelGGL(k_zero3, dim3((nt + 255) / 256), dim3(256), 0, st, L.counters, 4,
                           L.tick0, nt, L.tick1, nt);
        CT_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_wsum, dim3(1), dim3(1024), 0, st, w, M, L.wsum);
    CT_CHECK_HIP(hipGetLastError());
    StageArgs A;
    A.x = x; A.y = y; A.w = w; A.pot_in = pot;
    A.warm = (o->flags & CT_WARM_START) ? 1 : 0;
    A.ref_cached = (o->flags & CT_REF_CACHED) ? 1 : 0;
    A.T = T; A.M = M; A.d = d;
    A.sqrt_kappa = (float)std::sqrt(kappa_d);
    A.kappa = (float)kappa_d;
    A.log2a = (float)(-std::log2((double)T));
    A.wsum = L.wsum; A.cx = L.cx; A.cy = L.cy; A.b = L.b; A.log2b = L.log2b;
    A.f = L.f; A.g = L.g; A.p = L.p; A.q = L.q;
    A.h2y_g = L.h2y_g; A.h2x_p = L.h2x_p[0]; A.h2y_q = L.h2y_q[0];
    A.fp = L.fp; A.gp = L.gp; A.pp = L.pp; A.qp = L.qp;
    A.nonfinite = L.counters;
    const int n = std::max(T, M);
    hipLaunchKernelGGL(k_stage, dim3((n + 255) / 256), dim3(256), 0, st, A);
    CT_CHECK_HIP(hipGetLastError());

    rc = run_problem(L, T, M, o, st);
    if (rc) return rc;

    hipLaunchKernelGGL(k_grad_x, dim3((T * d + 255) / 256), dim3(256), 0, st, L.dy,
                       debias ? L.ds : nullptr, T * d, (float)(2.0 / T), grad_x);
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
                               need_ref ? L.qp : nullptr, M, L.bG, L.wsum, grad_w);
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
