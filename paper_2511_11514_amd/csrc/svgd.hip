// ct_svgd_grad: Stein variational flow (Sec. II-B, eq. 4) with the RBF kernel
// and the analytic score of a Gaussian mixture (+ uniform floor).
// ct_svgd_grad_score: the same flow for a score the caller already holds in
// device memory (the flow needs only the score, so any unnormalised target
// works, e.g. a gridded utility through ct_grid_score).
//
//   phi_i = 1/T sum_j k_ij [score_j + (2/h)(x_i - x_j)],  k_ij = exp(-|x_i - x_j|^2 / h)
//
// Kernels:
//   k_gmm_score   score of every sample, in float64 (responsibilities of far-away
//                 points are differences of large log-densities);
//   k_med_hist / k_med_select   exact median of the T(T-1)/2 squared distances
//                 (i < j) by a three-pass radix selection on their float32 bit
//                 patterns (12 + 11 + 8 bits), both middle ranks tracked so an
//                 even count takes the mean of the two middle distances;
//   k_svgd_stage  bandwidth h = med^2 / ln T (or the caller's h), coordinates
//                 pre-scaled by sqrt(log2(e)/h) so k_ij = 2^-|x'_i - x'_j|^2;
//   k_svgd_sum / k_svgd_merge   the T x T sum, split over keys like the Sinkhorn
//                 sweep (keys read as wave-uniform records), fixed-order merge.
#include <cmath>
#include <cstring>

#include "ct_internal.h"

namespace ct {

constexpr int kMaxK = 64;
constexpr int kMedBins = 4096;     // first pass: bits 30..19
constexpr double kLog2eD = 1.4426950408889634;

// ------------------------------------------------------------------ score

struct ScoreArgs {
    const float* x;
    int T, d, K;
    const float* weights;
    const float* means;
    const float* sigmas;
    float floor;
    float* score;      // [T][d] (workspace)
    float* score_out;  // [T][d] user copy or null
};

__global__ __launch_bounds__(256) void k_gmm_score(ScoreArgs A) {
    __shared__ double mu[kMaxK * 3], iv[kMaxK * 3], lc[kMaxK];
    const int d = A.d;
    for (int k = threadIdx.x; k < A.K; k += blockDim.x) {
        double ls = 0.0;
        for (int t = 0; t < d; ++t) {
            const double s = A.sigmas[k * d + t];
            mu[k * 3 + t] = A.means[k * d + t];
            iv[k * 3 + t] = 1.0 / (s * s);
            ls += log(s);
        }
        // log((1 - rho) pi_k) - sum log sigma - (d/2) log(2 pi)
        lc[k] = log((1.0 - (double)A.floor) * (double)A.weights[k]) - ls -
                0.5 * d * 1.8378770664093453;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.T) return;
    double x[3] = {0, 0, 0};
    bool inside = true;
    for (int t = 0; t < d; ++t) {
        x[t] = A.x[(size_t)i * d + t];
        inside &= (x[t] >= 0.0 && x[t] <= 1.0);
    }
    // log-density of each component; the uniform floor has log-mass log(rho) inside the box
    double m = (A.floor > 0.f && inside) ? log((double)A.floor) : -INFINITY;
    for (int k = 0; k < A.K; ++k) {
        double q = 0.0;
        for (int t = 0; t < d; ++t) {
            const double z = x[t] - mu[k * 3 + t];
            q += z * z * iv[k * 3 + t];
        }
        m = fmax(m, lc[k] - 0.5 * q);
    }
    double den = (A.floor > 0.f && inside) ? exp(log((double)A.floor) - m) : 0.0;
    double num[3] = {0, 0, 0};
    for (int k = 0; k < A.K; ++k) {
        double q = 0.0;
        for (int t = 0; t < d; ++t) {
            const double z = x[t] - mu[k * 3 + t];
            q += z * z * iv[k * 3 + t];
        }
        const double r = exp(lc[k] - 0.5 * q - m);
        den += r;
        for (int t = 0; t < d; ++t) num[t] -= r * (x[t] - mu[k * 3 + t]) * iv[k * 3 + t];
    }
    for (int t = 0; t < d; ++t) {
        const float v = (float)(num[t] / den);
        A.score[(size_t)i * d + t] = v;
        if (A.score_out) A.score_out[(size_t)i * d + t] = v;
    }
}

// ------------------------------------------------------------------ median

struct MedState {
    unsigned long long rank[2];  // remaining rank of target A / B inside its prefix
    unsigned prefix[2];          // bits of the target values fixed so far
    float h;                     // bandwidth
    float med;
};

struct MedPass {
    int shift, bits;             // bins = bits >> shift & (2^bits - 1)
    unsigned fixed_mask;         // bits already fixed
};

__device__ __forceinline__ MedPass med_pass(int p) {
    if (p == 0) return MedPass{19, 12, 0u};
    if (p == 1) return MedPass{8, 11, 0x7FF80000u};
    return MedPass{0, 8, 0x7FFFFF00u};
}

__global__ __launch_bounds__(256) void k_med_init(MedState* st, unsigned long long* hist, int T) {
    const unsigned long long n = (unsigned long long)T * (T - 1) / 2;
    for (int i = threadIdx.x; i < 2 * kMedBins; i += blockDim.x) hist[i] = 0ull;
    if (threadIdx.x == 0) {
        st->rank[0] = n ? (n - 1) / 2 : 0;
        st->rank[1] = n / 2;
        st->prefix[0] = st->prefix[1] = 0u;
        st->h = 1.f;
        st->med = 0.f;
    }
}

// Histogram of the squared-distance bit patterns of pairs i < j matching each
// target's prefix.  A block takes 256 rows i against 256 / sub columns j (staged
// in LDS); tiles below the diagonal are skipped.  Narrow column tiles (sub = 4)
// give small problems enough blocks; wide ones amortise the per-block clearing
// and flushing of the histogram when there are many tiles.
__host__ __device__ constexpr int med_sub(int nt) { return nt * (nt + 1) / 2 < 1024 ? 4 : 1; }

template <int D>
__global__ __launch_bounds__(256) void k_med_hist(const float4* __restrict__ c, int T, int pass,
                                                  const MedState* __restrict__ st,
                                                  unsigned long long* __restrict__ hist) {
    __shared__ unsigned h[2][kMedBins];
    __shared__ float4 cj[256];
    const int nt = (T + 255) / 256;
    const int nsub = med_sub(nt), jw = 256 / nsub;
    const int bi = blockIdx.x % nt;
    const int rest = blockIdx.x / nt;
    const int bj = rest / nsub, sub = rest % nsub;
    const int j0 = bj * 256 + sub * jw;
    if (bj < bi || j0 >= T) return;
    const int j1 = min(T, j0 + jw);
    const MedPass P = med_pass(pass);
    const unsigned pa = st->prefix[0], pb = st->prefix[1];
    const bool two = pa != pb;
    const int nb = 1 << P.bits;
    for (int k = threadIdx.x; k < nb; k += 256) {
        h[0][k] = 0u;
        h[1][k] = 0u;
    }
    if ((int)threadIdx.x < j1 - j0) cj[threadIdx.x] = c[j0 + threadIdx.x];
    __syncthreads();
    const int i = bi * 256 + (int)threadIdx.x;
    if (i < T && i < j1 - 1) {
        const float4 xi = c[i];
        for (int j = max(j0, i + 1); j < j1; ++j) {
            const float4 xj = cj[j - j0];
            const float dx = xi.x - xj.x, dy = xi.y - xj.y;
            float cc = dy * dy;
            if (D == 3) {
                const float dz = xi.z - xj.z;
                cc = __builtin_fmaf(dz, dz, cc);
            }
            cc = __builtin_fmaf(dx, dx, cc);
            const unsigned v = __float_as_uint(cc);
            const unsigned bin = (v >> P.shift) & (unsigned)(nb - 1);
            if ((v & P.fixed_mask) == pa) atomicAdd(&h[0][bin], 1u);
            if (two && (v & P.fixed_mask) == pb) atomicAdd(&h[1][bin], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += 256) {
        if (h[0][k]) atomicAdd(&hist[k], (unsigned long long)h[0][k]);
        if (two && h[1][k]) atomicAdd(&hist[kMedBins + k], (unsigned long long)h[1][k]);
    }
}

// Locate each target's bin, extend its prefix, clear the histograms.  Each
// thread holds a run of bins; a block-wide prefix sum of the run totals (wave
// scans, then the wave totals) tells which thread holds the target rank, and
// that thread walks its own bins.
__global__ __launch_bounds__(256) void k_med_select(MedState* st, unsigned long long* hist,
                                                    int pass, int T) {
    __shared__ unsigned long long wsum[4];
    const MedPass P = med_pass(pass);
    const int nb = 1 << P.bits;
    const int per = nb / 256;          // bins per thread (16, 8 or 1)
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const bool two = st->prefix[0] != st->prefix[1];
    for (int t = 0; t < 2; ++t) {
        const unsigned long long* H = hist + ((two && t == 1) ? kMedBins : 0);
        unsigned long long v[16];
        unsigned long long loc = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v[k] = k < per ? H[threadIdx.x * per + k] : 0ull;
            loc += v[k];
        }
        unsigned long long inc = loc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        unsigned long long before = 0;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        const unsigned long long excl = before + inc - loc;
        const unsigned long long r = st->rank[t];
        __syncthreads();               // every thread has read the rank before it changes
        // the owner of the rank (the last thread if the rank exceeds the count)
        if ((r >= excl && r < excl + loc) || (threadIdx.x == 255 && r >= excl + loc)) {
            unsigned long long cum = excl;
            int b = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k == b && k < per - 1 && r >= cum + v[k]) {
                    cum += v[k];
                    b = k + 1;
                }
            }
            st->prefix[t] |= (unsigned)(threadIdx.x * per + b) << P.shift;
            st->rank[t] = r - cum;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && pass == 2) {
        const double v1 = (double)__uint_as_float(st->prefix[0]);
        const double v2 = (double)__uint_as_float(st->prefix[1]);
        const double med = 0.5 * (sqrt(v1) + sqrt(v2));
        st->med = (float)med;
        // a vanishing median (all samples coincide) falls back to h = 1, as for one sample
        st->h = (T > 1 && med > 0.0) ? (float)(med * med / log((double)T)) : 1.f;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * kMedBins; k += blockDim.x) hist[k] = 0ull;
}

// ------------------------------------------------------------------ Stein sum

struct SvgdJob {
    const float4* qc;       // [T] pre-scaled coordinates (queries)
    const float4* krec;     // [Tpad * KR] key records (x', score) padded with zero-weight records
    int T, Tpad, nqb, splits, kps;
    float* part;            // [2D][splits][nqpad]
    const MedState* st;
    float* phi;
    float* h_used;
};

template <int D>
struct KeyRec {
    static constexpr int N = D == 2 ? 1 : 2;  // float4 records per key
};

__global__ __launch_bounds__(256) void k_svgd_stage(const float* __restrict__ x,
                                                    const float* __restrict__ score, int T, int Tpad,
                                                    int d, float h_fixed, MedState* st,
                                                    float4* __restrict__ qc,
                                                    float4* __restrict__ krec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (h_fixed > 0.f && i == 0) st->h = h_fixed;
    const float h = h_fixed > 0.f ? h_fixed : st->h;
    const float s = (float)sqrt(kLog2eD / (double)h);
    if (i >= Tpad) return;
    if (i < T) {
        float c[3] = {0, 0, 0}, sc[3] = {0, 0, 0};
        for (int t = 0; t < d; ++t) {
            c[t] = x[(size_t)i * d + t] * s;
            sc[t] = score[(size_t)i * d + t];
        }
        qc[i] = make_float4(c[0], c[1], c[2], 0.f);
        if (d == 2) {
            krec[i] = make_float4(c[0], c[1], sc[0], sc[1]);
        } else {
            krec[2 * (size_t)i] = make_float4(c[0], c[1], c[2], sc[0]);
            krec[2 * (size_t)i + 1] = make_float4(sc[1], sc[2], 0.f, 0.f);
        }
    } else {
        // padding keys sit far away (their kernel weight underflows to 0) with zero score
        const float far = 1e18f;
        if (d == 2) {
            krec[i] = make_float4(far, far, 0.f, 0.f);
        } else {
            krec[2 * (size_t)i] = make_float4(far, far, far, 0.f);
            krec[2 * (size_t)i + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

// Partial sums A_i = sum_j k_ij score_j and B_i = sum_j k_ij (x'_i - x'_j) over one key range.
template <int D, int R>
__global__ __launch_bounds__(256) void k_svgd_sum(SvgdJob J) {
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    const int qb = (int)blockIdx.x % J.nqb;
    const int split = (int)blockIdx.x / J.nqb;
    const int qbase = (qb * 4 + wave) * 64 * R;
    float q[R][D], a[R][D], b[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int qi = qbase + r * 64 + lane;
        const float4 c = qi < J.T ? J.qc[qi] : make_float4(0.f, 0.f, 0.f, 0.f);
        q[r][0] = c.x;
        q[r][1] = c.y;
        if (D == 3) q[r][2] = c.z;
#pragma unroll
        for (int t = 0; t < D; ++t) a[r][t] = b[r][t] = 0.f;
    }
    const int k0 = min(J.Tpad, split * J.kps);
    const int k1 = min(J.Tpad, k0 + J.kps);
    constexpr int NR = KeyRec<D>::N;
    // keys staged 64 at a time in a wave-private LDS slot (one coalesced load per
    // chunk, issued while the previous chunk is summed; broadcast reads)
    __shared__ float4 kbuf[4][64 * NR];
    float4* slot = kbuf[wave];
    float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0;
    if (k0 < k1) {
        const size_t kk = (size_t)min(k0 + lane, k1 - 1) * NR;
        n0 = J.krec[kk];
        if (D == 3) n1 = J.krec[kk + 1];
    }
    for (int kc = k0; kc < k1; kc += 64) {
        __builtin_amdgcn_wave_barrier();
        slot[lane * NR] = n0;
        if (D == 3) slot[lane * NR + 1] = n1;
        __builtin_amdgcn_wave_barrier();
        if (kc + 64 < k1) {
            const size_t kk = (size_t)min(kc + 64 + lane, k1 - 1) * NR;
            n0 = J.krec[kk];
            if (D == 3) n1 = J.krec[kk + 1];
        }
        const int n = min(64, k1 - kc);
#pragma unroll 4
    for (int kq = 0; kq < n; ++kq) {
        const float4 r0 = slot[kq * NR];
        float4 r1 = make_float4(0.f, 0.f, 0.f, 0.f);
        if (D == 3) r1 = slot[kq * NR + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float dx = q[r][0] - r0.x, dy = q[r][1] - r0.y;
            float c = dy * dy;
            float dz = 0.f;
            if (D == 3) {
                dz = q[r][2] - r0.z;
                c = __builtin_fmaf(dz, dz, c);
            }
            c = __builtin_fmaf(dx, dx, c);
            const float p = __builtin_amdgcn_exp2f(-c);
            if (D == 2) {
                a[r][0] = __builtin_fmaf(p, r0.z, a[r][0]);
                a[r][1] = __builtin_fmaf(p, r0.w, a[r][1]);
            } else {
                a[r][0] = __builtin_fmaf(p, r0.w, a[r][0]);
                a[r][1] = __builtin_fmaf(p, r1.x, a[r][1]);
                a[r][2] = __builtin_fmaf(p, r1.y, a[r][2]);
            }
            b[r][0] = __builtin_fmaf(p, dx, b[r][0]);
            b[r][1] = __builtin_fmaf(p, dy, b[r][1]);
            if (D == 3) b[r][2] = __builtin_fmaf(p, dz, b[r][2]);
        }
    }
    }
    const int nqpad = J.nqb * 256 * R;
    const size_t cs = (size_t)J.splits * nqpad;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        float* P = J.part + (size_t)split * nqpad + qbase + r * 64 + lane;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            P[t * cs] = a[r][t];
            P[(D + t) * cs] = b[r][t];
        }
    }
}

// phi_i = (A_i + (2/h)(1/s) B_i) / T with s = sqrt(log2(e)/h).  A block takes 64
// rows; its four waves take every fourth split and meet in LDS in wave order.
constexpr int kSvMergeRows = 64;

template <int D>
__global__ __launch_bounds__(256) void k_svgd_merge(SvgdJob J, int R) {
    __shared__ float red[3][2 * D][kSvMergeRows];
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int i = (int)blockIdx.x * kSvMergeRows + lane;
    const float h = J.st->h;
    if (blockIdx.x == 0 && threadIdx.x == 0 && J.h_used) *J.h_used = h;
    const int nqpad = J.nqb * 256 * R;
    const size_t cs = (size_t)J.splits * nqpad;
    float a[D], b[D];
    for (int t = 0; t < D; ++t) a[t] = b[t] = 0.f;
    if (i < J.T) {
        for (int sp = wave; sp < J.splits; sp += 4) {
            const float* P = J.part + (size_t)sp * nqpad + i;
            for (int t = 0; t < D; ++t) {
                a[t] += P[t * cs];
                b[t] += P[(D + t) * cs];
            }
        }
    }
    if (wave > 0) {
        for (int t = 0; t < D; ++t) {
            red[wave - 1][t][lane] = a[t];
            red[wave - 1][D + t][lane] = b[t];
        }
    }
    __syncthreads();
    if (wave != 0 || i >= J.T) return;
    for (int w = 0; w < 3; ++w)
        for (int t = 0; t < D; ++t) {
            a[t] += red[w][t][lane];
            b[t] += red[w][D + t][lane];
        }
    const double s = sqrt(kLog2eD / (double)h);
    const float cb = (float)(2.0 / ((double)h * s));
    const float invT = 1.0f / (float)J.T;
    for (int t = 0; t < D; ++t) J.phi[(size_t)i * D + t] = __builtin_fmaf(cb, b[t], a[t]) * invT;
}

// ------------------------------------------------------------------ layout

struct SvLayout {
    MedState* st;
    unsigned long long* hist;
    float* score;
    float4* cmed;      // raw coordinates for the median
    float4* qc;
    float4* krec;
    float* part;
    size_t bytes;
};

constexpr int kSvR = 2;            // queries per lane of the Stein sum
constexpr int kSvBlocksPerCU = 8;

static void svgd_plan(int T, int& nqb, int& splits, int& kps) {
    const int Tpad = pad_keys(T);
    nqb = (T + 256 * kSvR - 1) / (256 * kSvR);
    const int want = std::max(1, (kSvBlocksPerCU * kNumCU + nqb - 1) / nqb);
    splits = std::min(want, std::max(1, Tpad / 64));
    kps = (Tpad + splits - 1) / splits;
    kps = (kps + 31) / 32 * 32;
    splits = (Tpad + kps - 1) / kps;
}

static SvLayout sv_layout(void* ws, int T, int d) {
    Arena a(ws);
    SvLayout L;
    int nqb, splits, kps;
    svgd_plan(T, nqb, splits, kps);
    const int Tpad = pad_keys(T);
    L.st = a.take<MedState>(1);
    L.hist = a.take<unsigned long long>(2 * kMedBins);
    L.score = a.take<float>((size_t)T * d);
    L.cmed = a.take<float4>(T);
    L.qc = a.take<float4>(T);
    L.krec = a.take<float4>((size_t)Tpad * (d == 2 ? 1 : 2));
    L.part = a.take<float>((size_t)2 * d * splits * nqb * 256 * kSvR);
    L.bytes = a.off + 256;
    return L;
}

__global__ __launch_bounds__(256) void k_med_coords(const float* __restrict__ x, int T, int d,
                                                    float4* __restrict__ c) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= T) return;
    float v[3] = {0, 0, 0};
    for (int t = 0; t < d; ++t) v[t] = x[(size_t)i * d + t];
    c[i] = make_float4(v[0], v[1], v[2], 0.f);
}

}  // namespace ct

using namespace ct;

extern "C" size_t ct_svgd_workspace_size(int64_t T, int32_t d) {
    if ((d != 2 && d != 3) || T < 1 || T > (int64_t(1) << 30)) return 0;
    return sv_layout(nullptr, (int)T, d).bytes;
}

namespace ct {
namespace {

ct_status svgd_check(const float* x, int64_t T64, int32_t d, float h, float* phi, void* ws,
                     size_t ws_bytes, SvLayout& L) {
    if (d != 2 && d != 3) return fail(CT_E_SHAPE, "d must be 2 or 3 (got %d)", d);
    if (T64 < 1 || T64 > (int64_t(1) << 30)) return fail(CT_E_SHAPE, "T must be in [1, 2^30]");
    if (!x || !phi) return fail(CT_E_ARG, "x and phi must be non-null");
    if (!std::isfinite(h)) return fail(CT_E_ARG, "h must be finite");
    if (h <= 0.f && T64 > 92681) return fail(CT_E_SHAPE, "median bandwidth supports T <= 92681");
    if (!ws) return fail(CT_E_ARG, "workspace is null");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(CT_E_WORKSPACE, "workspace not 256-byte aligned");
    L = sv_layout(ws, (int)T64, d);
    if (ws_bytes < L.bytes) return fail(CT_E_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, L.bytes);
    return CT_OK;
}

// Bandwidth, staging and the T x T sum for a score already in device memory.
ct_status svgd_flow(const float* x, int T, int d, const float* score, float h, float* phi,
                    float* h_used, const SvLayout& L, hipStream_t st) {
    hipLaunchKernelGGL(k_med_init, dim3(1), dim3(256), 0, st, L.st, L.hist, T);
    CT_CHECK_HIP(hipGetLastError());
    if (h <= 0.f && T > 1) {
        hipLaunchKernelGGL(k_med_coords, dim3((T + 255) / 256), dim3(256), 0, st, x, T, d, L.cmed);
        CT_CHECK_HIP(hipGetLastError());
        const int nt = (T + 255) / 256;
        for (int pass = 0; pass < 3; ++pass) {
            if (d == 2)
                hipLaunchKernelGGL(k_med_hist<2>, dim3(nt * nt * med_sub(nt)), dim3(256), 0, st, L.cmed,
                                   T, pass, L.st, L.hist);
            else
                hipLaunchKernelGGL(k_med_hist<3>, dim3(nt * nt * med_sub(nt)), dim3(256), 0, st, L.cmed,
                                   T, pass, L.st, L.hist);
            CT_CHECK_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_med_select, dim3(1), dim3(256), 0, st, L.st, L.hist, pass, T);
            CT_CHECK_HIP(hipGetLastError());
        }
    }
    const int Tpad = pad_keys(T);
    hipLaunchKernelGGL(k_svgd_stage, dim3((Tpad + 255) / 256), dim3(256), 0, st, x, score, T, Tpad,
                       d, h > 0.f ? h : 0.f, L.st, L.qc, L.krec);
    CT_CHECK_HIP(hipGetLastError());
    SvgdJob J;
    J.qc = L.qc;
    J.krec = L.krec;
    J.T = T;
    J.Tpad = Tpad;
    svgd_plan(T, J.nqb, J.splits, J.kps);
    J.part = L.part;
    J.st = L.st;
    J.phi = phi;
    J.h_used = h_used;
    void* tok = profile_begin(st);
    if (d == 2)
        hipLaunchKernelGGL((k_svgd_sum<2, kSvR>), dim3(J.nqb * J.splits), dim3(256), 0, st, J);
    else
        hipLaunchKernelGGL((k_svgd_sum<3, kSvR>), dim3(J.nqb * J.splits), dim3(256), 0, st, J);
    CT_CHECK_HIP(hipGetLastError());
    if (d == 2)
        hipLaunchKernelGGL(k_svgd_merge<2>, dim3((T + kSvMergeRows - 1) / kSvMergeRows), dim3(256), 0,
                           st, J, kSvR);
    else
        hipLaunchKernelGGL(k_svgd_merge<3>, dim3((T + kSvMergeRows - 1) / kSvMergeRows), dim3(256), 0,
                           st, J, kSvR);
    CT_CHECK_HIP(hipGetLastError());
    if (tok) profile_end(tok, st, 2, 0, kSvR * 100, J.nqb * J.splits, (double)T * T);
    return CT_OK;
}

}  // namespace
}  // namespace ct

extern "C" ct_status ct_svgd_grad(const float* x, int64_t T64, int32_t d, const ct_gmm* q, float h,
                                  float* phi, float* score, float* h_used, void* ws,
                                  size_t ws_bytes, void* stream) {
    clear_error();
    SvLayout L;
    ct_status rc = svgd_check(x, T64, d, h, phi, ws, ws_bytes, L);
    if (rc) return rc;
    if (!q) return fail(CT_E_ARG, "q must be non-null");
    if (q->K < 1 || q->K > kMaxK) return fail(CT_E_ARG, "K must be in [1, %d] (got %d)", kMaxK, q->K);
    if (!q->weights || !q->means || !q->sigmas) return fail(CT_E_ARG, "mixture arrays must be non-null");
    if (!(q->floor >= 0.f && q->floor < 1.f)) return fail(CT_E_ARG, "floor must be in [0, 1)");
    const int T = (int)T64;
    hipStream_t st = static_cast<hipStream_t>(stream);
    ScoreArgs S{x, T, d, q->K, q->weights, q->means, q->sigmas, q->floor, L.score, score};
    hipLaunchKernelGGL(k_gmm_score, dim3((T + 255) / 256), dim3(256), 0, st, S);
    CT_CHECK_HIP(hipGetLastError());
    return svgd_flow(x, T, d, L.score, h, phi, h_used, L, st);
}

extern "C" ct_status ct_svgd_grad_score(const float* x, int64_t T64, int32_t d, const float* score,
                                        float h, float* phi, float* h_used, void* ws,
                                        size_t ws_bytes, void* stream) {
    clear_error();
    SvLayout L;
    ct_status rc = svgd_check(x, T64, d, h, phi, ws, ws_bytes, L);
    if (rc) return rc;
    if (!score) return fail(CT_E_ARG, "score must be non-null");
    return svgd_flow(x, (int)T64, d, score, h, phi, h_used, L, static_cast<hipStream_t>(stream));
}
