// Continuous-utility references (Sec. II-A: the reference may be a utility
// function over the search space; Sec. II-B: the Stein flow needs only its score,
// so it need not be normalised).  The utility is given by its values on the nodes
// of a regular grid over a box; the density is proportional to its multilinear
// interpolant (at the point clamped into the box) plus an additive floor.
//
//   ct_grid_score    grad log(U + rho) at every sample, in float64 (one thread per
//                    sample; the 2^d corner values are gathers from a grid that
//                    stays in L2)
//   ct_grid_samples  the nodes as weighted reference samples for the Sinkhorn flow:
//                    weight (u_j + rho) times the node's trapezoid-rule volume
//                    (exact mass of the interpolant), normalised, zero-weight
//                    nodes dropped, node order kept.  Three launches: per-block
//                    counts and masses, one-block scan, compaction.
#include <cmath>

#include "ct_internal.h"

namespace ct {
namespace {

constexpr int64_t kMaxNodes = int64_t(1) << 28;
constexpr int kGridBlock = 256;

struct GridDev {
    const float* u;
    int d;
    int n[3];
    double lo[3], hi[3];
    double floor;
};

GridDev grid_dev(const ct_grid* g, int d) {
    GridDev G;
    G.u = g->u;
    G.d = d;
    for (int t = 0; t < 3; ++t) {
        G.n[t] = t < d ? g->n[t] : 1;
        G.lo[t] = g->lo[t];
        G.hi[t] = g->hi[t];
    }
    G.floor = g->floor;
    return G;
}

int64_t node_count(const ct_grid* g, int d) {
    int64_t N = 1;
    for (int t = 0; t < d; ++t) N *= g->n[t];
    return N;
}

ct_status grid_validate(const ct_grid* g, int d) {
    if (d != 2 && d != 3) return fail(CT_E_SHAPE, "d must be 2 or 3 (got %d)", d);
    if (!g) return fail(CT_E_ARG, "grid is null");
    if (!g->u) return fail(CT_E_ARG, "grid values are null");
    for (int t = 0; t < d; ++t) {
        if (g->n[t] < 2 || g->n[t] > (1 << 20))
            return fail(CT_E_SHAPE, "grid needs 2..2^20 nodes per axis (axis %d has %d)", t, g->n[t]);
        if (!std::isfinite(g->lo[t]) || !std::isfinite(g->hi[t]) || !(g->hi[t] > g->lo[t]))
            return fail(CT_E_ARG, "grid box must be finite with hi > lo (axis %d)", t);
    }
    if (node_count(g, d) > kMaxNodes) return fail(CT_E_SHAPE, "grid has more than 2^28 nodes");
    if (!(g->floor >= 0.f) || !std::isfinite(g->floor)) return fail(CT_E_ARG, "floor must be finite and >= 0");
    return CT_OK;
}

// ------------------------------------------------------------------ score

template <int D>
__global__ __launch_bounds__(256) void k_grid_score(const float* __restrict__ x, int T, GridDev G,
                                                    float* __restrict__ score) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T) return;
    int c[3] = {0, 0, 0};
    double f[3] = {0, 0, 0}, dsdx[3] = {0, 0, 0};
    bool finite = true;
    for (int t = 0; t < D; ++t) {
        const double v = x[(size_t)i * D + t];
        const double top = (double)(G.n[t] - 1);
        finite &= isfinite(v);
        double s = (v - G.lo[t]) * top / (G.hi[t] - G.lo[t]);
        s = isfinite(s) ? fmin(fmax(s, 0.0), top) : 0.0;
        const int ci = min((int)floor(s), G.n[t] - 2);
        c[t] = ci;
        f[t] = s - (double)ci;
        dsdx[t] = (v >= G.lo[t] && v <= G.hi[t]) ? top / (G.hi[t] - G.lo[t]) : 0.0;
    }
    // corner k has bit t set when it is the upper node of axis t
    const size_t stride1 = (size_t)G.n[0], stride2 = (size_t)G.n[0] * G.n[1];
    const size_t base = (size_t)c[0] + stride1 * c[1] + (D == 3 ? stride2 * c[2] : 0);
    double val = 0.0, grad[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
        const size_t off = (k & 1 ? 1 : 0) + (k & 2 ? stride1 : 0) + (D == 3 && (k & 4) ? stride2 : 0);
        const double u = G.u[base + off];
        double w[3];
#pragma unroll
        for (int t = 0; t < D; ++t) w[t] = (k >> t) & 1 ? f[t] : 1.0 - f[t];
        double all = w[0] * w[1];
        if (D == 3) all *= w[2];
        val += all * u;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            // product of the other axes' weights, with the sign of this axis' slope
            double o = 1.0;
#pragma unroll
            for (int r = 0; r < D; ++r)
                if (r != t) o *= w[r];
            grad[t] += ((k >> t) & 1 ? o : -o) * u;
        }
    }
    const double den = val + G.floor;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const double g = grad[t] * dsdx[t];
        score[(size_t)i * D + t] = !finite ? NAN : (den > 0.0 ? (float)(g / den) : 0.f);
    }
}

// ------------------------------------------------------------------ samples

// Trapezoid mass of node j up to the constant cell volume: (u_j + rho) halved once
// per axis on which the node lies on the box face.  Negative: an invalid node.
__device__ inline double node_mass(const GridDev& G, int64_t j, int* idx) {
    int64_t r = j;
    double m = (double)G.u[j] + G.floor;
    const bool bad = !(G.u[j] >= 0.f) || !isfinite(G.u[j]);
    for (int t = 0; t < G.d; ++t) {
        idx[t] = (int)(r % G.n[t]);
        r /= G.n[t];
        if (idx[t] == 0 || idx[t] == G.n[t] - 1) m *= 0.5;
    }
    return bad ? -1.0 : m;
}

struct SampleWs {
    int* cnt;        // [nb] kept nodes per block
    int* bad;        // [nb] invalid nodes per block
    double* mass;    // [nb] block mass
    int64_t* off;    // [nb] output offset of each block
    double* hdr;     // [4]: total mass, kept count, invalid count
};

__global__ __launch_bounds__(kGridBlock) void k_grid_count(GridDev G, int64_t N, SampleWs W) {
    __shared__ double sm[kGridBlock];
    __shared__ int sc[kGridBlock], sb[kGridBlock];
    const int64_t j = (int64_t)blockIdx.x * kGridBlock + threadIdx.x;
    double m = 0.0;
    int keep = 0, bad = 0;
    if (j < N) {
        int idx[3];
        m = node_mass(G, j, idx);
        bad = m < 0.0;
        keep = m > 0.0;
        if (!keep) m = 0.0;
    }
    sm[threadIdx.x] = m;
    sc[threadIdx.x] = keep;
    sb[threadIdx.x] = bad;
    __syncthreads();
    for (int h = kGridBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sm[threadIdx.x] += sm[threadIdx.x + h];
            sc[threadIdx.x] += sc[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        W.mass[blockIdx.x] = sm[0];
        W.cnt[blockIdx.x] = sc[0];
        W.bad[blockIdx.x] = sb[0];
    }
}

// One block: each thread takes a contiguous run of blocks, the runs' totals are
// scanned in LDS; masses are summed in a fixed order.
__global__ __launch_bounds__(1024) void k_grid_scan(int nb, SampleWs W) {
    __shared__ long long sc[1024];
    __shared__ double sm[1024];
    __shared__ long long sb[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = min(nb, (int)threadIdx.x * per), b1 = min(nb, b0 + per);
    long long c = 0, bad = 0;
    double m = 0.0;
    for (int b = b0; b < b1; ++b) {
        c += W.cnt[b];
        bad += W.bad[b];
        m += W.mass[b];
    }
    sc[threadIdx.x] = c;
    sm[threadIdx.x] = m;
    sb[threadIdx.x] = bad;
    __syncthreads();
    // inclusive Hillis-Steele scan of the counts
    for (int h = 1; h < 1024; h <<= 1) {
        const long long v = (int)threadIdx.x >= h ? sc[threadIdx.x - h] : 0;
        __syncthreads();
        sc[threadIdx.x] += v;
        __syncthreads();
    }
    long long run = sc[threadIdx.x] - c;
    for (int b = b0; b < b1; ++b) {
        W.off[b] = run;
        run += W.cnt[b];
    }
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sm[threadIdx.x] += sm[threadIdx.x + h];
            sb[threadIdx.x] += sb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        W.hdr[0] = sm[0];
        W.hdr[1] = (double)sc[1023];
        W.hdr[2] = (double)sb[0];
    }
}

__global__ __launch_bounds__(kGridBlock) void k_grid_emit(GridDev G, int64_t N, SampleWs W,
                                                          float* __restrict__ y,
                                                          float* __restrict__ w) {
#pragma clang fp contract(off)
    __shared__ int wave_cnt[kGridBlock / 64];
    const int64_t j = (int64_t)blockIdx.x * kGridBlock + threadIdx.x;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    int idx[3] = {0, 0, 0};
    double m = 0.0;
    if (j < N) m = node_mass(G, j, idx);
    const bool keep = m > 0.0;
    const unsigned long long ball = __ballot(keep);
    const int before = __popcll(ball & ((1ull << lane) - 1ull));
    if (lane == 0) wave_cnt[wave] = __popcll(ball);
    __syncthreads();
    if (!keep) return;
    int pos = before;
    for (int v = 0; v < wave; ++v) pos += wave_cnt[v];
    const int64_t o = W.off[blockIdx.x] + pos;
    for (int t = 0; t < G.d; ++t) {
        const double h = (G.hi[t] - G.lo[t]) / (double)(G.n[t] - 1);
        y[o * G.d + t] = (float)(G.lo[t] + (double)idx[t] * h);
    }
    w[o] = (float)(m / W.hdr[0]);
}

struct SampleLayout {
    SampleWs W;
    size_t bytes;
};

SampleLayout sample_layout(void* ws, int64_t N) {
    Arena a(ws);
    SampleLayout L;
    const size_t nb = (size_t)((N + kGridBlock - 1) / kGridBlock);
    L.W.hdr = a.take<double>(4);
    L.W.mass = a.take<double>(nb);
    L.W.off = a.take<int64_t>(nb);
    L.W.cnt = a.take<int>(nb);
    L.W.bad = a.take<int>(nb);
    L.bytes = a.off + 256;
    return L;
}

}  // namespace
}  // namespace ct

using namespace ct;

extern "C" ct_status ct_grid_score(const float* x, int64_t T64, int32_t d, const ct_grid* g,
                                   float* score, void* stream) {
    clear_error();
    ct_status rc = grid_validate(g, d);
    if (rc) return rc;
    if (T64 < 1 || T64 > (int64_t(1) << 30)) return fail(CT_E_SHAPE, "T must be in [1, 2^30]");
    if (!x || !score) return fail(CT_E_ARG, "x and score must be non-null");
    const int T = (int)T64;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const GridDev G = grid_dev(g, d);
    if (d == 2)
        hipLaunchKernelGGL(k_grid_score<2>, dim3((T + 255) / 256), dim3(256), 0, st, x, T, G, score);
    else
        hipLaunchKernelGGL(k_grid_score<3>, dim3((T + 255) / 256), dim3(256), 0, st, x, T, G, score);
    CT_CHECK_HIP(hipGetLastError());
    return CT_OK;
}

extern "C" size_t ct_grid_samples_workspace_size(const ct_grid* g, int32_t d) {
    if (!g || (d != 2 && d != 3)) return 0;
    for (int t = 0; t < d; ++t)
        if (g->n[t] < 2 || g->n[t] > (1 << 20)) return 0;
    const int64_t N = node_count(g, d);
    if (N > kMaxNodes) return 0;
    return sample_layout(nullptr, N).bytes;
}

extern "C" ct_status ct_grid_samples(const ct_grid* g, int32_t d, float* y, float* w, int64_t* M,
                                     void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    ct_status rc = grid_validate(g, d);
    if (rc) return rc;
    if (!y || !w || !M) return fail(CT_E_ARG, "y, w and M must be non-null");
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CT_E_WORKSPACE, "workspace not 256-byte aligned");
    const int64_t N = node_count(g, d);
    SampleLayout L = sample_layout(ws, N);
    if (ws_bytes < L.bytes) return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    hipStream_t st = static_cast<hipStream_t>(stream);
    rc = refuse_capture(st, "ct_grid_samples");
    if (rc) return rc;
    const GridDev G = grid_dev(g, d);
    const int nb = (int)((N + kGridBlock - 1) / kGridBlock);
    hipLaunchKernelGGL(k_grid_count, dim3(nb), dim3(kGridBlock), 0, st, G, N, L.W);
    CT_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, st, nb, L.W);
    CT_CHECK_HIP(hipGetLastError());
    double hdr[4] = {0, 0, 0, 0};
    CT_CHECK_HIP(hipMemcpyAsync(hdr, L.W.hdr, sizeof(hdr), hipMemcpyDeviceToHost, st));
    CT_CHECK_HIP(hipStreamSynchronize(st));
    if (hdr[2] > 0.0) return fail(CT_E_ARG, "utility has %.0f negative or non-finite node values", hdr[2]);
    if (!(hdr[1] > 0.0)) return fail(CT_E_ARG, "utility plus floor is zero on every node");
    if (!std::isfinite(hdr[0])) return fail(CT_E_ARG, "utility mass is not finite");
    hipLaunchKernelGGL(k_grid_emit, dim3(nb), dim3(kGridBlock), 0, st, G, N, L.W, y, w);
    CT_CHECK_HIP(hipGetLastError());
    CT_CHECK_HIP(hipStreamSynchronize(st));
    *M = (int64_t)hdr[1];
    return CT_OK;
}
