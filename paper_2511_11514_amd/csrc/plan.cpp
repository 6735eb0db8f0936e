// Host side of the planner (Sec. II-C): the FP64 tracking LQR of eqs. 9-10 and
// the outer loop that alternates GPU flow evaluation with the LQR step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "ct_internal.h"

namespace ct {

namespace {

constexpr int kMaxDim = 8;

// In-place Cholesky factor of an SPD m x m matrix; false if not positive definite.
template <int MM>
inline bool cholesky(double* H, int m_rt) {
    const int m = MM > 0 ? MM : m_rt;
    for (int j = 0; j < m; ++j) {
        double d = H[j * m + j];
        for (int k = 0; k < j; ++k) d -= H[j * m + k] * H[j * m + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        H[j * m + j] = d;
        for (int i = j + 1; i < m; ++i) {
            double s = H[i * m + j];
            for (int k = 0; k < j; ++k) s -= H[i * m + k] * H[j * m + k];
            H[i * m + j] = s / d;
        }
    }
    return true;
}

// Solve (L L^T) X = B for an m x c right-hand side in place.
template <int MM, int CC>
inline void chol_solve(const double* L, double* B, int m_rt, int c_rt) {
    const int m = MM > 0 ? MM : m_rt;
    const int c = CC > 0 ? CC : c_rt;
    for (int col = 0; col < c; ++col) {
        for (int i = 0; i < m; ++i) {
            double s = B[i * c + col];
            for (int k = 0; k < i; ++k) s -= L[i * m + k] * B[k * c + col];
            B[i * c + col] = s / L[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = B[i * c + col];
            for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * B[k * c + col];
            B[i * c + col] = s / L[i * m + i];
        }
    }
}

// Backward Riccati recursion with the affine tracking term, then forward rollout.
// With S = dt Q + P_{t+1}, s = dt Q a_t + p_{t+1}, H = dt R + B'SB (discrete A, B):
//   K_t = H^-1 B'SA, k_t = H^-1 B's,  P_t = A'(SA - SB K_t),  p_t = A'(s - SB k_t),
//   v_t = -K_t z_t + k_t,  z_{t+1} = A z_t + B v_t.
// NN, MM > 0 fix the state and control sizes at compile time (the planner's
// dynamics); 0 takes them from n_rt, m_rt.
template <int NN, int MM>
ct_status lqr_core(int64_t T, int n_rt, int m_rt, double dt, const double* A, const double* B,
                   const double* a, const double* Q, const double* R, double* v, double* z) {
    const int n = NN > 0 ? NN : n_rt;
    const int m = MM > 0 ? MM : m_rt;
    std::vector<double> Ks((size_t)T * m * n), ks((size_t)T * m);
    double P[kMaxDim * kMaxDim] = {0}, p[kMaxDim] = {0};
    double Ad[kMaxDim * kMaxDim], Bd[kMaxDim * kMaxDim], S[kMaxDim * kMaxDim], s[kMaxDim];
    double SB[kMaxDim * kMaxDim], SA[kMaxDim * kMaxDim], H[kMaxDim * kMaxDim];
    double G[kMaxDim * (kMaxDim + 1)], SBK[kMaxDim * kMaxDim], Pn[kMaxDim * kMaxDim];
    for (int64_t t = T - 1; t >= 0; --t) {
        const double* At = A + (size_t)t * n * n;
        const double* Bt = B + (size_t)t * n * m;
        const double* at = a + (size_t)t * n;
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) Ad[i * n + j] = (i == j ? 1.0 : 0.0) + dt * At[i * n + j];
            for (int j = 0; j < m; ++j) Bd[i * m + j] = dt * Bt[i * m + j];
        }
        for (int i = 0; i < n * n; ++i) S[i] = dt * Q[i] + P[i];
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int j = 0; j < n; ++j) acc += Q[i * n + j] * at[j];
            s[i] = dt * acc + p[i];
        }
        // SB = S Bd (n x m), SA = S Ad (n x n)
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k) acc += S[i * n + k] * Bd[k * m + j];
                SB[i * m + j] = acc;
            }
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k) acc += S[i * n + k] * Ad[k * n + j];
                SA[i * n + j] = acc;
            }
        }
        // H = dt R + Bd' S Bd;  G = [Bd' S Ad | Bd' s]  (m x (n+1))
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) {
                double acc = dt * R[i * m + j];
                for (int k = 0; k < n; ++k) acc += Bd[k * m + i] * SB[k * m + j];
                H[i * m + j] = acc;
            }
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k) acc += Bd[k * m + i] * SA[k * n + j];
                G[i * (n + 1) + j] = acc;
            }
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Bd[k * m + i] * s[k];
            G[i * (n + 1) + n] = acc;
        }
        if (!cholesky<MM>(H, m))
            return fail(CT_E_UNSUPPORTED, "Riccati step %lld: dt R + B'SB is not positive definite",
                        (long long)t);
        chol_solve<MM, (NN > 0 ? NN + 1 : 0)>(H, G, m, n + 1);
        double* Kt = Ks.data() + (size_t)t * m * n;
        double* kt = ks.data() + (size_t)t * m;
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < n; ++j) Kt[i * n + j] = G[i * (n + 1) + j];
            kt[i] = G[i * (n + 1) + n];
        }
        // P = Ad' (S Ad - S Bd K) ;  p = Ad' (s - S Bd k)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) {
                double acc = SA[k * n + j];
                for (int l = 0; l < m; ++l) acc -= SB[k * m + l] * Kt[l * n + j];
                SBK[k * n + j] = acc;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double acc = 0.0;
                for (int k = 0; k < n; ++k) acc += Ad[k * n + i] * SBK[k * n + j];
                Pn[i * n + j] = acc;
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) P[i * n + j] = 0.5 * (Pn[i * n + j] + Pn[j * n + i]);
        double r[kMaxDim];
        for (int k = 0; k < n; ++k) {
            double sbk = 0.0;
            for (int l = 0; l < m; ++l) sbk += SB[k * m + l] * kt[l];
            r[k] = s[k] - sbk;
        }
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Ad[k * n + i] * r[k];
            p[i] = acc;
        }
    }
    double zt[kMaxDim] = {0}, zn[kMaxDim];
    if (z)
        for (int i = 0; i < n; ++i) z[i] = 0.0;
    for (int64_t t = 0; t < T; ++t) {
        const double* At = A + (size_t)t * n * n;
        const double* Bt = B + (size_t)t * n * m;
        const double* Kt = Ks.data() + (size_t)t * m * n;
        const double* kt = ks.data() + (size_t)t * m;
        double* vt = v + (size_t)t * m;
        for (int i = 0; i < m; ++i) {
            double acc = kt[i];
            for (int j = 0; j < n; ++j) acc -= Kt[i * n + j] * zt[j];
            vt[i] = acc;
        }
        for (int i = 0; i < n; ++i) {
            double acc = zt[i];
            for (int j = 0; j < n; ++j) acc += dt * At[i * n + j] * zt[j];
            for (int j = 0; j < m; ++j) acc += dt * Bt[i * m + j] * vt[j];
            zn[i] = acc;
        }
        for (int i = 0; i < n; ++i) zt[i] = zn[i];
        if (z)
            for (int i = 0; i < n; ++i) z[(size_t)(t + 1) * n + i] = zt[i];
    }
    return CT_OK;
}

}  // namespace

ct_status lqr_solve(int64_t T, int n, int m, double dt, const double* A, const double* B,
                    const double* a, const double* Q, const double* R, double* v, double* z) {
    if (n == 3 && m == 2) return lqr_core<3, 2>(T, n, m, dt, A, B, a, Q, R, v, z);  // unicycle
    if (n == 4 && m == 2) return lqr_core<4, 2>(T, n, m, dt, A, B, a, Q, R, v, z);  // 2-D point mass
    if (n == 6 && m == 3) return lqr_core<6, 3>(T, n, m, dt, A, B, a, Q, R, v, z);  // 3-D point mass
    return lqr_core<0, 0>(T, n, m, dt, A, B, a, Q, R, v, z);
}

namespace {

struct Dyn {
    int n, m, d;
};

bool dyn_dims(const ct_plan_problem* p, Dyn& D) {
    if (p->dynamics == CT_DYN_DOUBLE_INTEGRATOR) {
        if (p->d != 2 && p->d != 3) return false;
        D = Dyn{2 * p->d, p->d, p->d};
        return true;
    }
    if (p->dynamics == CT_DYN_UNICYCLE) {
        if (p->d != 2) return false;
        D = Dyn{3, 2, 2};
        return true;
    }
    return false;
}

// f(s, u) and its Jacobians (eq. 8).
void dyn_f(int kind, const Dyn& D, const double* s, const double* u, double* f) {
    if (kind == CT_DYN_DOUBLE_INTEGRATOR) {
        for (int i = 0; i < D.d; ++i) {
            f[i] = s[D.d + i];
            f[D.d + i] = u[i];
        }
    } else {
        f[0] = u[0] * std::cos(s[2]);
        f[1] = u[0] * std::sin(s[2]);
        f[2] = u[1];
    }
}

void dyn_jac(int kind, const Dyn& D, const double* s, const double* u, double* A, double* B) {
    std::memset(A, 0, sizeof(double) * D.n * D.n);
    std::memset(B, 0, sizeof(double) * D.n * D.m);
    if (kind == CT_DYN_DOUBLE_INTEGRATOR) {
        for (int i = 0; i < D.d; ++i) {
            A[i * D.n + D.d + i] = 1.0;
            B[(D.d + i) * D.m + i] = 1.0;
        }
    } else {
        A[0 * 3 + 2] = -u[0] * std::sin(s[2]);
        A[1 * 3 + 2] = u[0] * std::cos(s[2]);
        B[0 * 2 + 0] = std::cos(s[2]);
        B[1 * 2 + 0] = std::sin(s[2]);
        B[2 * 2 + 1] = 1.0;
    }
}

void rollout(int kind, const Dyn& D, const double* s0, const double* u, int64_t T, double dt,
             double* s) {
    for (int i = 0; i < D.n; ++i) s[i] = s0[i];
    double f[kMaxDim];
    for (int64_t t = 0; t < T; ++t) {
        dyn_f(kind, D, s + t * D.n, u + t * D.m, f);
        for (int i = 0; i < D.n; ++i) s[(t + 1) * D.n + i] = s[t * D.n + i] + dt * f[i];
    }
}

struct PlanLayout {
    float* x;
    float* flow;
    float* score;   // utility-grid score (CT_FLOW_SVGD_GRID)
    float* value;
    float* pot;
    void* inner;
    size_t inner_bytes;
    size_t bytes;
};

PlanLayout plan_layout(void* ws, const ct_plan_problem* p, const ct_plan_opts* o, int64_t M) {
    Arena a(ws);
    PlanLayout L;
    const int64_t T = p->T;
    L.x = a.take<float>((size_t)T * p->d);
    L.flow = a.take<float>((size_t)T * p->d);
    L.score = o->flow == CT_FLOW_SVGD_GRID ? a.take<float>((size_t)T * p->d) : nullptr;
    L.value = a.take<float>(4);
    L.pot = a.take<float>((size_t)(2 * T + 2 * std::max<int64_t>(M, 0)));
    if (o->flow == CT_FLOW_SINKHORN) {
        ct_sinkhorn_opts so = o->sk;
        so.d = p->d;
        L.inner_bytes = ct_sinkhorn_workspace_size(T, M, &so);
    } else {
        L.inner_bytes = ct_svgd_workspace_size(T, p->d);
    }
    L.inner = a.take<char>(L.inner_bytes);
    L.bytes = a.off + 256;
    return L;
}

ct_status plan_validate(const ct_plan_problem* p, const ct_plan_opts* o, const float* y,
                        int64_t M, const ct_gmm* q, Dyn& D) {
    if (!p || !o) return fail(CT_E_ARG, "problem and opts must be non-null");
    if (!dyn_dims(p, D)) return fail(CT_E_SHAPE, "unsupported dynamics/dimension (%d, d=%d)", p->dynamics, p->d);
    if (p->T < 1 || p->T > (int64_t(1) << 30)) return fail(CT_E_SHAPE, "T must be in [1, 2^30]");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(CT_E_ARG, "dt must be finite and > 0");
    if (!p->s0) return fail(CT_E_ARG, "s0 is null");
    if (o->outer < 1) return fail(CT_E_ARG, "outer must be >= 1");
    if (!std::isfinite(o->step)) return fail(CT_E_ARG, "step must be finite");
    if (!o->Q || !o->R) return fail(CT_E_ARG, "Q and R must be non-null");
    if (o->flow == CT_FLOW_SINKHORN) {
        if (!y || M < 1) return fail(CT_E_ARG, "the Sinkhorn flow needs reference samples");
        if (o->sk.flags &
            ~(uint32_t)(CT_DEBIAS | CT_SAFE_LSE | CT_FUSED | CT_UNFUSED | CT_TINY | CT_MESH))
            return fail(CT_E_ARG, "plan accepts only the CT_DEBIAS, CT_SAFE_LSE, CT_FUSED, "
                                  "CT_UNFUSED, CT_TINY and CT_MESH Sinkhorn flags");
    } else if (o->flow == CT_FLOW_SVGD) {
        if (!q) return fail(CT_E_ARG, "the Stein flow needs a mixture");
    } else if (o->flow == CT_FLOW_SVGD_GRID) {
        if (!o->grid) return fail(CT_E_ARG, "the grid Stein flow needs opts.grid");
    } else {
        return fail(CT_E_ARG, "unknown flow %d", o->flow);
    }
    return CT_OK;
}

}  // namespace
}  // namespace ct

using namespace ct;

extern "C" ct_status ct_lqr_track(int64_t T, int32_t n, int32_t m, double dt, const double* A,
                                  const double* B, const double* a, const double* Q, const double* R,
                                  double* v, double* z) {
    clear_error();
    if (!A || !B || !a || !Q || !R || !v) return fail(CT_E_ARG, "A, B, a, Q, R and v must be non-null");
    if (T < 1) return fail(CT_E_SHAPE, "T must be >= 1");
    if (n < 1 || n > kMaxDim || m < 1 || m > kMaxDim) return fail(CT_E_SHAPE, "n and m must be in [1, 8]");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CT_E_ARG, "dt must be finite and > 0");
    return lqr_solve(T, n, m, dt, A, B, a, Q, R, v, z);
}

extern "C" size_t ct_plan_workspace_size(const ct_plan_problem* p, const ct_plan_opts* o, int64_t M) {
    Dyn D;
    if (!p || !o || !dyn_dims(p, D) || p->T < 1) return 0;
    return plan_layout(nullptr, p, o, M).bytes;
}

extern "C" ct_status ct_plan(const ct_plan_problem* p, const ct_plan_opts* o, const float* y,
                             const float* w, int64_t M, const ct_gmm* q, double* u, double* s,
                             double* hist, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    Dyn D;
    ct_status rc = plan_validate(p, o, y, M, q, D);
    if (rc) return rc;
    if (!u) return fail(CT_E_ARG, "u is null");
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CT_E_WORKSPACE, "workspace not 256-byte aligned");
    PlanLayout L = plan_layout(ws, p, o, M);
    if (ws_bytes < L.bytes) return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = refuse_capture(st, "ct_plan");
    if (rc) return rc;
    const int64_t T = p->T;
    const int d = D.d, n = D.n, m = D.m;
    std::vector<double> traj((size_t)(T + 1) * n), A((size_t)T * n * n), B((size_t)T * n * m);
    std::vector<double> tgt((size_t)T * n, 0.0), v((size_t)T * m), Qn((size_t)n * n, 0.0);
    std::vector<float> xh((size_t)T * d), fh((size_t)T * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Qn[i * n + j] = o->Q[i * d + j];
    for (int it = 0; it < o->outer; ++it) {
        rollout(p->dynamics, D, p->s0, u, T, p->dt, traj.data());
        for (int64_t t = 0; t < T; ++t)
            for (int k = 0; k < d; ++k) xh[t * d + k] = (float)traj[(t + 1) * n + k];
        CT_CHECK_HIP(hipMemcpyAsync(L.x, xh.data(), sizeof(float) * T * d, hipMemcpyHostToDevice, st));
        double obj = 0.0;
        if (o->flow == CT_FLOW_SINKHORN) {
            ct_sinkhorn_opts so = o->sk;
            so.d = d;
            so.flags |= CT_VALUE;
            // the reference self potential does not depend on the trajectory: solve it
            // once and reuse it in later outer iterations
            if (it > 0 && (so.flags & CT_DEBIAS)) so.flags |= CT_REF_CACHED;
            rc = ct_sinkhorn_grad(L.x, T, y, w, M, &so, L.flow, nullptr, L.value, L.pot, nullptr,
                                  nullptr, L.inner, L.inner_bytes, stream);
            if (rc) return rc;
            float val = 0.f;
            CT_CHECK_HIP(hipMemcpyAsync(fh.data(), L.flow, sizeof(float) * T * d, hipMemcpyDeviceToHost, st));
            CT_CHECK_HIP(hipMemcpyAsync(&val, L.value, sizeof(float), hipMemcpyDeviceToHost, st));
            CT_CHECK_HIP(hipStreamSynchronize(st));
            obj = val;
            for (int64_t t = 0; t < T; ++t)
                for (int k = 0; k < d; ++k) tgt[t * n + k] = -(double)T * (double)fh[t * d + k];
        } else {
            if (o->flow == CT_FLOW_SVGD) {
                rc = ct_svgd_grad(L.x, T, d, q, o->svgd_h, L.flow, nullptr, nullptr, L.inner,
                                  L.inner_bytes, stream);
            } else {
                rc = ct_grid_score(L.x, T, d, o->grid, L.score, stream);
                if (rc) return rc;
                rc = ct_svgd_grad_score(L.x, T, d, L.score, o->svgd_h, L.flow, nullptr, L.inner,
                                        L.inner_bytes, stream);
            }
            if (rc) return rc;
            CT_CHECK_HIP(hipMemcpyAsync(fh.data(), L.flow, sizeof(float) * T * d, hipMemcpyDeviceToHost, st));
            CT_CHECK_HIP(hipStreamSynchronize(st));
            double acc = 0.0;
            for (int64_t t = 0; t < T; ++t) {
                double nn = 0.0;
                for (int k = 0; k < d; ++k) {
                    tgt[t * n + k] = fh[t * d + k];
                    nn += (double)fh[t * d + k] * fh[t * d + k];
                }
                acc += std::sqrt(nn);
            }
            obj = acc / (double)T;
        }
        if (hist) hist[it] = obj;
        for (int64_t t = 0; t < T; ++t)
            dyn_jac(p->dynamics, D, traj.data() + t * n, u + t * m, A.data() + (size_t)t * n * n,
                    B.data() + (size_t)t * n * m);
        rc = lqr_solve(T, n, m, p->dt, A.data(), B.data(), tgt.data(), Qn.data(), o->R, v.data(),
                       nullptr);
        if (rc) return rc;
        for (size_t i = 0; i < v.size(); ++i) u[i] += o->step * v[i];
    }
    if (s) rollout(p->dynamics, D, p->s0, u, T, p->dt, s);
    return CT_OK;
}

// ------------------------------------------------------------ seed ensemble

namespace ct {
namespace {

struct EnsembleLayout {
    float* x;       // [S*T][d] trajectory samples of every seed
    float* gx;      // [S*T][d] gradients
    float* y;       // [S*M][d] the reference, once per seed
    float* w;       // [S*M] its weights, or null
    float* value;   // [S]
    void* inner;    // batched Sinkhorn workspace
    size_t inner_bytes;
    size_t bytes;
};

void ensemble_offsets(int32_t S, int64_t T, int64_t M, std::vector<int64_t>& To,
                      std::vector<int64_t>& Mo) {
    To.resize((size_t)S + 1);
    Mo.resize((size_t)S + 1);
    for (int32_t b = 0; b <= S; ++b) {
        To[b] = (int64_t)b * T;
        Mo[b] = (int64_t)b * M;
    }
}

// Run f(b, worker) for the seeds b = 0..S-1 on up to 16 host threads (the seeds
// are independent; each worker owns its scratch).  The first failing seed's
// status and message (kept per thread by fail()) are passed to the caller.
template <typename F>
ct_status for_each_seed(int32_t S, int workers, F&& f) {
    std::vector<ct_status> rc((size_t)S, CT_OK);
    std::vector<std::string> msg((size_t)S);
    auto work = [&](int wk) {
        for (int32_t b = wk; b < S; b += workers) {
            rc[b] = f(b, wk);
            if (rc[b] != CT_OK) msg[b] = ct_last_error();
        }
    };
    if (workers <= 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        th.reserve((size_t)workers);
        for (int wk = 0; wk < workers; ++wk) th.emplace_back(work, wk);
        for (auto& t : th) t.join();
    }
    for (int32_t b = 0; b < S; ++b)
        if (rc[b] != CT_OK) return fail(rc[b], "seed %d: %s", b, msg[b].c_str());
    return CT_OK;
}

EnsembleLayout ensemble_layout(void* ws, const ct_plan_problem* p, const ct_plan_opts* o,
                               int32_t S, int64_t M, bool weighted) {
    Arena a(ws);
    EnsembleLayout L;
    const int64_t T = p->T;
    const int d = p->d;
    L.x = a.take<float>((size_t)S * T * d);
    L.gx = a.take<float>((size_t)S * T * d);
    L.y = a.take<float>((size_t)S * M * d);
    L.w = weighted ? a.take<float>((size_t)S * M) : nullptr;
    L.value = a.take<float>((size_t)S);
    std::vector<int64_t> To, Mo;
    ensemble_offsets(S, T, M, To, Mo);
    ct_sinkhorn_opts so = o->sk;
    so.d = d;
    so.flags &= (uint32_t)(CT_DEBIAS | CT_SAFE_LSE);
    const size_t b0 = ct_sinkhorn_batched_workspace_size(S, To.data(), Mo.data(), &so);
    so.flags |= CT_VALUE;
    const size_t b1 = ct_sinkhorn_batched_workspace_size(S, To.data(), Mo.data(), &so);
    L.inner_bytes = std::max(b0, b1);
    L.inner = a.take<char>(L.inner_bytes);
    L.bytes = a.off + 256;
    return L;
}

}  // namespace
}  // namespace ct

extern "C" size_t ct_plan_ensemble_workspace_size(const ct_plan_problem* p, const ct_plan_opts* o,
                                                  int32_t S, int64_t M, int32_t weighted) {
    Dyn D;
    if (!p || !o || !dyn_dims(p, D) || p->T < 1 || S < 1 || M < 1) return 0;
    return ensemble_layout(nullptr, p, o, S, M, weighted != 0).bytes;
}

extern "C" ct_status ct_plan_ensemble(const ct_plan_problem* p, const ct_plan_opts* o, int32_t S,
                                      const float* y, const float* w, int64_t M, double* u,
                                      double* s, double* value, int32_t* best, void* ws,
                                      size_t ws_bytes, void* stream) {
    clear_error();
    Dyn D;
    ct_status rc = plan_validate(p, o, y, M, nullptr, D);
    if (rc) return rc;
    if (o->flow != CT_FLOW_SINKHORN)
        return fail(CT_E_UNSUPPORTED, "the seed ensemble ranks seeds by the Sinkhorn divergence; "
                                      "it needs the Sinkhorn flow");
    if (S < 1) return fail(CT_E_ARG, "S must be >= 1");
    if (!u || !value || !best) return fail(CT_E_ARG, "u, value and best must be non-null");
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CT_E_WORKSPACE, "workspace not 256-byte aligned");
    rc = refuse_capture(static_cast<hipStream_t>(stream), "ct_plan_ensemble");
    if (rc) return rc;
    const int64_t T = p->T;
    if ((int64_t)S * T > (int64_t(1) << 30) || (int64_t)S * M > (int64_t(1) << 30))
        return fail(CT_E_SHAPE, "S*T and S*M must be <= 2^30");
    EnsembleLayout L = ensemble_layout(ws, p, o, S, M, w != nullptr);
    if (ws_bytes < L.bytes) return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int d = D.d, n = D.n, m = D.m;
    std::vector<int64_t> To, Mo;
    ensemble_offsets(S, T, M, To, Mo);
    // the shared reference, once per seed (the batched form takes one reference per problem)
    for (int32_t b = 0; b < S; ++b) {
        CT_CHECK_HIP(hipMemcpyAsync(L.y + (size_t)b * M * d, y, sizeof(float) * M * d,
                                    hipMemcpyDeviceToDevice, st));
        if (w)
            CT_CHECK_HIP(hipMemcpyAsync(L.w + (size_t)b * M, w, sizeof(float) * M,
                                        hipMemcpyDeviceToDevice, st));
    }
    ct_sinkhorn_opts so = o->sk;
    so.d = d;
    so.flags &= (uint32_t)(CT_DEBIAS | CT_SAFE_LSE);
    rc = ct_sinkhorn_batched_prepare(S, To.data(), Mo.data(), &so, L.inner, L.inner_bytes, stream);
    if (rc) return rc;
    const int workers = (int)std::max<int32_t>(
        1, std::min<int32_t>(S, (int32_t)std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    struct Scratch {
        std::vector<double> traj, A, B, tgt, v;
    };
    std::vector<Scratch> sc((size_t)workers);
    for (auto& w_ : sc) {
        w_.traj.resize((size_t)(T + 1) * n);
        w_.A.resize((size_t)T * n * n);
        w_.B.resize((size_t)T * n * m);
        w_.tgt.assign((size_t)T * n, 0.0);
        w_.v.resize((size_t)T * m);
    }
    std::vector<double> Qn((size_t)n * n, 0.0);
    std::vector<float> xh((size_t)S * T * d), gh((size_t)S * T * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) Qn[i * n + j] = o->Q[i * d + j];
    auto stage_positions = [&]() -> ct_status {
        rc = for_each_seed(S, workers, [&](int32_t b, int wk) -> ct_status {
            std::vector<double>& traj = sc[wk].traj;
            rollout(p->dynamics, D, p->s0, u + (size_t)b * T * m, T, p->dt, traj.data());
            for (int64_t t = 0; t < T; ++t)
                for (int k = 0; k < d; ++k)
                    xh[((size_t)b * T + t) * d + k] = (float)traj[(t + 1) * n + k];
            return CT_OK;
        });
        if (rc) return rc;
        CT_CHECK_HIP(hipMemcpyAsync(L.x, xh.data(), sizeof(float) * S * T * d,
                                    hipMemcpyHostToDevice, st));
        return CT_OK;
    };
    for (int it = 0; it < o->outer; ++it) {
        rc = stage_positions();
        if (rc) return rc;
        // every seed's flow in one persistent launch (the gradient only: the
        // reference self term is not needed for it)
        rc = ct_sinkhorn_grad_batched(S, To.data(), Mo.data(), L.x, L.y, L.w, &so, L.gx, nullptr,
                                      nullptr, L.inner, L.inner_bytes, stream);
        if (rc) return rc;
        CT_CHECK_HIP(hipMemcpyAsync(gh.data(), L.gx, sizeof(float) * S * T * d,
                                    hipMemcpyDeviceToHost, st));
        CT_CHECK_HIP(hipStreamSynchronize(st));
        // every seed's LQR step on the host, seeds spread over threads
        rc = for_each_seed(S, workers, [&](int32_t b, int wk) -> ct_status {
            Scratch& w_ = sc[wk];
            double* ub = u + (size_t)b * T * m;
            rollout(p->dynamics, D, p->s0, ub, T, p->dt, w_.traj.data());
            for (int64_t t = 0; t < T; ++t)
                for (int k = 0; k < d; ++k)
                    w_.tgt[t * n + k] = -(double)T * (double)gh[((size_t)b * T + t) * d + k];
            for (int64_t t = 0; t < T; ++t)
                dyn_jac(p->dynamics, D, w_.traj.data() + t * n, ub + t * m,
                        w_.A.data() + (size_t)t * n * n, w_.B.data() + (size_t)t * n * m);
            const ct_status r = lqr_solve(T, n, m, p->dt, w_.A.data(), w_.B.data(), w_.tgt.data(),
                                          Qn.data(), o->R, w_.v.data(), nullptr);
            if (r) return r;
            for (size_t i = 0; i < w_.v.size(); ++i) ub[i] += o->step * w_.v[i];
            return CT_OK;
        });
        if (rc) return rc;
    }
    // rank the final trajectories by their divergence to the reference
    rc = stage_positions();
    if (rc) return rc;
    ct_sinkhorn_opts sv = so;
    sv.flags |= CT_VALUE;
    rc = ct_sinkhorn_batched_prepare(S, To.data(), Mo.data(), &sv, L.inner, L.inner_bytes, stream);
    if (rc) return rc;
    rc = ct_sinkhorn_grad_batched(S, To.data(), Mo.data(), L.x, L.y, L.w, &sv, L.gx, nullptr,
                                  L.value, L.inner, L.inner_bytes, stream);
    if (rc) return rc;
    std::vector<float> vh((size_t)S);
    CT_CHECK_HIP(hipMemcpyAsync(vh.data(), L.value, sizeof(float) * S, hipMemcpyDeviceToHost, st));
    CT_CHECK_HIP(hipStreamSynchronize(st));
    int32_t bi = 0;
    for (int32_t b = 0; b < S; ++b) {
        value[b] = vh[b];
        if (!std::isfinite(vh[b]))
            return fail(CT_E_HIP, "seed %d: the batched evaluation returned a non-finite value", b);
        if (vh[b] < vh[bi]) bi = b;
    }
    *best = bi;
    if (s)
        for (int32_t b = 0; b < S; ++b)
            rollout(p->dynamics, D, p->s0, u + (size_t)b * T * m, T, p->dt,
                    s + (size_t)b * (T + 1) * n);
    return CT_OK;
}
