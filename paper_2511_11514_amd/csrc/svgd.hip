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
//                 even count takes the mean of the two middle distances; for
//                 large T the same selection runs over the pairs inside a
//                 bracket found on a sample (k_med_sample, then one pass over
//                 the pairs: k_med_bracket_tiles over every pair, or from
//                 T = kBoxMinT k_med_bracket with the points in Morton-cell
//                 order so that bounding boxes of groups of 64 settle most pairs
//                 of groups, k_med_classify), with the full selection as the
//                 fallback;
//   k_svgd_stage  bandwidth h = med^2 / ln T (or the caller's h), coordinates
//                 pre-scaled by sqrt(log2(e)/h) so k_ij = 2^-|x'_i - x'_j|^2;
//   k_svgd_sum / k_svgd_merge   the T x T sum, split over keys like the Sinkhorn
//                 sweep (keys read as wave-uniform records), fixed-order merge.
#include <hip/hip_ext.h>

#include <cmath>
#include <cstddef>
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
    int mode;                    // 0: select over all pairs, 1: over the bracket's candidates
    unsigned long long below;    // pairs below the bracket
    unsigned long long ncand;    // pairs inside the bracket (set by k_med_decide)
    unsigned long long novf;     // of them appended to the shared overflow list
    unsigned nitems;             // pairs of groups listed for the pair-by-pair pass
    int skip0;                   // the candidates share the first pass's bits: it is skipped
};

// Large T: an exact selection over a bracket.  kMedSample pseudo-random pairs
// give the bracket [lo, hi] (their quantiles 1/2 -+ 4 standard errors); one pass
// over all pairs counts those below lo and collects those inside; the targets'
// ranks among the candidates are then selected exactly.  If a target falls
// outside the bracket or the candidates overflow their buffer, the selection
// runs over all pairs instead (same result, three full passes).
constexpr int kMedSample = 1 << 20;
constexpr int kBracketMinT = 11000;
constexpr int kMaxMedianT = 92681;               // T(T-1)/2 pairs fit the selection's counters
constexpr unsigned long long kSampleLo = 522240;   // floor((1/2 - 4 * 0.5 / 1024) * 2^20)
constexpr unsigned long long kSampleHi = 526335;   // ceil((1/2 + 4 * 0.5 / 1024) * 2^20) - 1

__host__ __device__ inline unsigned long long med_pairs(int T) {
    return (unsigned long long)T * (unsigned long long)(T - 1) / 2;
}
__host__ __device__ inline unsigned long long cand_cap(int T) {
    return (unsigned long long)(0.008 * (double)med_pairs(T)) + 65536ull;
}

// The pair-by-pair pass runs kBracketWaves waves; each owns a segment of the
// candidate buffer (so that its appends need no atomic: one global counter
// would serialise them), twice its share of cand_cap(T), and what overflows a
// segment goes to a shared list of cand_cap(T) entries.
constexpr int kBracketBlocks = kNumCU * 8;
constexpr int kBracketWaves = kBracketBlocks * 4;
// From this T on the pass runs over boxes of point groups; below it over every
// pair in tiles, with all candidates in the shared list (no segments).
constexpr int kBoxMinT = 24576;
__host__ __device__ inline unsigned long long cand_seg(int T) {
    return T >= kBoxMinT ? (2 * cand_cap(T) + kBracketWaves - 1) / kBracketWaves : 0ull;
}

struct CandStore {
    float* cand;                 // [kBracketWaves][seg] segments, then [ovf_cap] shared overflow
    unsigned* segcnt;            // [kBracketWaves] entries in each segment
    unsigned long long seg, ovf_cap;
};

template <int D>
__device__ __forceinline__ float sqdist(const float4& a, const float4& b) {
    const float dx = a.x - b.x, dy = a.y - b.y;
    float cc = dy * dy;
    if (D == 3) {
        const float dz = a.z - b.z;
        cc = __builtin_fmaf(dz, dz, cc);
    }
    return __builtin_fmaf(dx, dx, cc);
}

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
        st->mode = 0;
        st->below = 0ull;
        st->ncand = 0ull;
        st->novf = 0ull;
        st->nitems = 0u;
        st->skip0 = 0;
    }
}

// SplitMix64 finaliser (Steele, Lea, Flood 2014) as the sample's index hash.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(64) void k_sample_init(MedState* sst) {
    if (threadIdx.x == 0) {
        sst->rank[0] = kSampleLo;
        sst->rank[1] = kSampleHi;
        sst->prefix[0] = sst->prefix[1] = 0u;
        sst->mode = 0;
    }
}

// Squared distances of kMedSample pseudo-random pairs i != j (T >= 2).
template <int D>
__global__ __launch_bounds__(256) void k_med_sample(const float4* __restrict__ c, int T,
                                                    float* __restrict__ out) {
    const int k = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (k >= kMedSample) return;
    const unsigned long long z = mix64((unsigned long long)k);
    const int i = (int)((z & 0xFFFFFFFFull) % (unsigned long long)T);
    int j = (int)((z >> 32) % (unsigned long long)T);
    if (j == i) j = (j + 1) % T;
    out[k] = sqdist<D>(c[i], c[j]);
}

// Histogram of the squared-distance bit patterns of pairs i < j matching each
// target's prefix.  A block takes 256 rows i against 256 / sub columns j (staged
// in LDS); tiles below the diagonal are skipped.  Narrow column tiles (sub = 4)
// give small problems enough blocks; wide ones amortise the per-block clearing
// and flushing of the histogram when there are many tiles.
__host__ __device__ constexpr int med_sub(int nt) { return nt * (nt + 1) / 2 < 1024 ? 4 : 1; }

// Tile t of the (row tile, column tile) index space: rows bi*256.., columns
// bj*256 + sub*jw..; false for tiles below the diagonal or past the end.
struct MedTile {
    int i0, j0, j1;
};
__device__ __forceinline__ bool med_tile(int t, int T, int nt, MedTile& mt) {
    const int nsub = med_sub(nt), jw = 256 / nsub;
    const int bi = t % nt, rest = t / nt;
    const int bj = rest / nsub, sub = rest % nsub;
    mt.i0 = bi * 256;
    mt.j0 = bj * 256 + sub * jw;
    mt.j1 = min(T, mt.j0 + jw);
    return bj >= bi && mt.j0 < T;
}

// Blocks of the pair kernels below: a grid-stride loop over the tiles, so that
// a launch whose mode does not match exits at once and each block clears and
// flushes its histogram once.
inline int med_grid(int T) {
    const int nt = (T + 255) / 256;
    return std::min(nt * nt * med_sub(nt), kNumCU * 8);
}

template <int D>
__global__ __launch_bounds__(256) void k_med_hist(const float4* __restrict__ c, int T, int pass,
                                                  const MedState* __restrict__ st,
                                                  unsigned long long* __restrict__ hist) {
    __shared__ unsigned h[2][kMedBins];
    __shared__ float4 cj[256];
    if (st->mode != 0) return;
    const int nt = (T + 255) / 256;
    const int ntiles = nt * nt * med_sub(nt);
    const MedPass P = med_pass(pass);
    const unsigned pa = st->prefix[0], pb = st->prefix[1];
    const bool two = pa != pb;
    const int nb = 1 << P.bits;
    for (int k = threadIdx.x; k < nb; k += 256) {
        h[0][k] = 0u;
        h[1][k] = 0u;
    }
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        MedTile mt;
        if (!med_tile(t, T, nt, mt)) continue;
        __syncthreads();              // the previous tile's columns are no longer read
        if ((int)threadIdx.x < mt.j1 - mt.j0) cj[threadIdx.x] = c[mt.j0 + threadIdx.x];
        __syncthreads();
        const int i = mt.i0 + (int)threadIdx.x;
        if (i < T && i < mt.j1 - 1) {
            const float4 xi = c[i];
            for (int j = max(mt.j0, i + 1); j < mt.j1; ++j) {
                const unsigned v = __float_as_uint(sqdist<D>(xi, cj[j - mt.j0]));
                const unsigned bin = (v >> P.shift) & (unsigned)(nb - 1);
                if ((v & P.fixed_mask) == pa) atomicAdd(&h[0][bin], 1u);
                if (two && (v & P.fixed_mask) == pb) atomicAdd(&h[1][bin], 1u);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += 256) {
        if (h[0][k]) atomicAdd(&hist[k], (unsigned long long)h[0][k]);
        if (two && h[1][k]) atomicAdd(&hist[kMedBins + k], (unsigned long long)h[1][k]);
    }
}

// The same histogram over a flat array of n squared distances (the bracket's sample).
__global__ __launch_bounds__(256) void k_flat_hist(const float* __restrict__ v, int n, int pass,
                                                   const MedState* st,
                                                   unsigned long long* __restrict__ hist) {
    __shared__ unsigned h[2][kMedBins];
    const MedPass P = med_pass(pass);
    const unsigned pa = st->prefix[0], pb = st->prefix[1];
    const bool two = pa != pb;
    const int nb = 1 << P.bits;
    for (int k = threadIdx.x; k < nb; k += 256) {
        h[0][k] = 0u;
        h[1][k] = 0u;
    }
    __syncthreads();
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const unsigned u = __float_as_uint(v[k]);
        const unsigned bin = (u >> P.shift) & (unsigned)(nb - 1);
        if ((u & P.fixed_mask) == pa) atomicAdd(&h[0][bin], 1u);
        if (two && (u & P.fixed_mask) == pb) atomicAdd(&h[1][bin], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += 256) {
        if (h[0][k]) atomicAdd(&hist[k], (unsigned long long)h[0][k]);
        if (two && h[1][k]) atomicAdd(&hist[kMedBins + k], (unsigned long long)h[1][k]);
    }
}

constexpr int kCandSlots = 16;
constexpr int kBracketRows = 4;                  // rows per thread: tiles of 1024 x 256

inline int bracket_tile_grid(int T) {
    const int ntr = (T + 256 * kBracketRows - 1) / (256 * kBracketRows), ntc = (T + 255) / 256;
    return std::min(ntr * ntc, kNumCU * 8);
}

// The pairs of one tile of the pass over every pair: count those below the
// bracket, keep those in it (the first kCandSlots per thread in LDS slots, the
// rest straight to the shared candidate list).  CHECK keeps only pairs with
// j > i (diagonal and ragged tiles).
template <int D, int RB, bool CHECK>
__device__ __forceinline__ void bracket_tile_pairs(const float4* cj, int n, int j0, const float4 (&xi)[RB],
                                              const int (&ir)[RB], unsigned lo, unsigned span,
                                              unsigned& bl, unsigned& nin,
                                              float (*slots)[256], MedState* st,
                                              float* __restrict__ cand, unsigned long long cap) {
    for (int jj = 0; jj < n; jj += 8) {
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const int jl = jj + g;
            if (jl < n) {
                const float4 xj = cj[jl];
                const int j = j0 + jl;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const float d2 = sqdist<D>(xi[r], xj);
                    const unsigned u = __float_as_uint(d2);
                    const bool ok = !CHECK || j > ir[r];
                    bl += (ok && u < lo) ? 1u : 0u;
                    if (ok && u - lo <= span) {
                        if (nin < (unsigned)kCandSlots) {
                            slots[nin][threadIdx.x] = d2;
                        } else {
                            const unsigned long long gi = atomicAdd(&st->novf, 1ull);
                            if (gi < cap) cand[gi] = d2;
                        }
                        ++nin;
                    }
                }
            }
        }
    }
}

// The pass over every pair in the original order, for T below kBoxMinT (where
// ordering the points and their boxes costs more than they save): tiles of
// 1024 rows (four per thread) by 256 LDS-staged columns; the candidates go to
// the shared list (cand, cap entries; st->novf counts them), one append per
// block and tile.
template <int D>
__global__ __launch_bounds__(256) void k_med_bracket_tiles(const float4* __restrict__ c, int T,
                                                           const MedState* __restrict__ sst,
                                                           MedState* st, float* __restrict__ cand,
                                                           unsigned long long cap) {
    constexpr int RB = kBracketRows;
    __shared__ float4 cj[256];
    __shared__ float slots[kCandSlots][256];
    __shared__ unsigned wsum[4];
    __shared__ unsigned long long base;
    const int ntr = (T + 256 * RB - 1) / (256 * RB), ntc = (T + 255) / 256;
    const int ntiles = ntr * ntc;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const unsigned lo = sst->prefix[0], hi = sst->prefix[1];
    const unsigned span = hi - lo;                 // u in [lo, hi]  <=>  u - lo <= span
    unsigned long long below = 0ull;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int i0 = (t % ntr) * 256 * RB;
        const int j0 = (t / ntr) * 256;
        const int j1 = min(T, j0 + 256);
        if (j1 - 1 <= i0) continue;               // no column j > any row i of the tile
        __syncthreads();                           // previous tile: columns and slots consumed
        if ((int)threadIdx.x < j1 - j0) cj[threadIdx.x] = c[j0 + threadIdx.x];
        __syncthreads();
        float4 xi[RB];
        int ir[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            ir[r] = i0 + r * 256 + (int)threadIdx.x;
            // rows past the end take j > T, which no column satisfies
            xi[r] = ir[r] < T ? c[ir[r]] : make_float4(0.f, 0.f, 0.f, 0.f);
            if (ir[r] >= T) ir[r] = T;
        }
        unsigned nin = 0u, bl = 0u;
        const int n = j1 - j0;
        // every row valid and below every column of the tile: no pair needs j > i
        const bool off_diag = i0 + 256 * RB <= T && j0 >= i0 + 256 * RB;
        if (off_diag)
            bracket_tile_pairs<D, RB, false>(cj, n, j0, xi, ir, lo, span, bl, nin, slots, st, cand, cap);
        else
            bracket_tile_pairs<D, RB, true>(cj, n, j0, xi, ir, lo, span, bl, nin, slots, st, cand, cap);
        below += bl;
        // block exclusive prefix sum of the kept counts
        const unsigned kept = min(nin, (unsigned)kCandSlots);
        unsigned inc = kept;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        unsigned before = 0u, total = 0u;
        for (int w = 0; w < 4; ++w) {
            before += w < wave ? wsum[w] : 0u;
            total += wsum[w];
        }
        if (threadIdx.x == 0) base = total ? atomicAdd(&st->novf, (unsigned long long)total) : 0ull;
        __syncthreads();
        const unsigned long long off = base + before + inc - kept;
        for (unsigned k = 0; k < kept; ++k)
            if (off + k < cap) cand[off + k] = slots[k][threadIdx.x];
    }
    // pairs below the bracket: a wave sum, then one atomic per wave
    unsigned long long b = below;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b += __shfl_down(b, o, 64);
    if (lane == 0 && b) atomicAdd(&st->below, b);
}

// One pass over all pairs i < j: count the pairs below the bracket [lo, hi]
// found on the sample and collect those inside.  The pass runs over the points
// in a spatial order (cells of a Morton curve), in groups of kBoxPts consecutive
// points with a bounding box each, so that most pairs of groups are settled by
// their boxes alone: a pair of groups whose largest squared distance is below lo
// adds all of its pairs to the count, one whose smallest is above hi adds
// nothing, and only the rest are evaluated pair by pair.  The boxes' squared
// distances take the same rounded operations as a pair's (sqdist), and rounding
// is monotonic, so they bound every pair's float32 value exactly; a box with a
// non-finite coordinate is NaN and its groups are always evaluated.  The
// unordered pairs {i, j} and their values are those of the original order.
constexpr int kBoxPts = 64;                      // points per box: a wave's rows or columns
constexpr int kWaveBuf = 960;                    // candidates a wave holds in LDS (8 blocks per CU)
constexpr int kCells2 = 1 << 15;                 // cell counts: 128 x 128 cells (2-D), 32 x 32 x 32 (3-D)

__global__ __launch_bounds__(256) void k_fill_u32(unsigned* __restrict__ p, int n, unsigned v) {
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i < n) p[i] = v;
}

// Bounding box of all points (one block): box[0] = min, box[1] = max.
__global__ __launch_bounds__(1024) void k_med_box(const float4* __restrict__ c, int T,
                                                  float4* __restrict__ box) {
    __shared__ float red[6][16];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll 8
    for (int i = threadIdx.x; i < T; i += 1024) {
        const float4 p = c[i];
        v[0] = fminf(v[0], p.x); v[1] = fminf(v[1], p.y); v[2] = fminf(v[2], p.z);
        v[3] = fmaxf(v[3], p.x); v[4] = fmaxf(v[4], p.y); v[5] = fmaxf(v[5], p.z);
    }
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        for (int o = 32; o > 0; o >>= 1) {
            const float u = __shfl_down(v[k], o, 64);
            v[k] = k < 3 ? fminf(v[k], u) : fmaxf(v[k], u);
        }
        if (lane == 0) red[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float m = red[k][0];
        for (int w = 1; w < 16; ++w) m = k < 3 ? fminf(m, red[k][w]) : fmaxf(m, red[k][w]);
        reinterpret_cast<float*>(box)[(k < 3 ? 0 : 4) + k % 3] = m;
    }
}

__device__ __forceinline__ unsigned spread2(unsigned v) {    // 7 bits -> even bits of 14
    v &= 0x7Fu;
    v = (v | (v << 4)) & 0x070Fu;
    v = (v | (v << 2)) & 0x3333u;
    return (v | (v << 1)) & 0x5555u;
}
__device__ __forceinline__ unsigned spread3(unsigned v) {    // 5 bits -> every third bit of 15
    v &= 0x1Fu;
    v = (v | (v << 8)) & 0x100Fu;
    v = (v | (v << 4)) & 0x10C3u;
    return (v | (v << 2)) & 0x1249u;
}

// Cell of each point on the Morton curve over the bounding box, and the cell counts.
template <int D>
__global__ __launch_bounds__(256) void k_med_cell(const float4* __restrict__ c, int T,
                                                  const float4* __restrict__ box,
                                                  unsigned* __restrict__ cell,
                                                  unsigned* __restrict__ count) {
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= T) return;
    const float4 p = c[i], lo = box[0], hi = box[1];
    constexpr float side = D == 2 ? 128.f : 32.f;
    auto q = [&](float x, float a, float b) {
        const float s = (x - a) / fmaxf(b - a, 1e-30f) * side;      // NaN: cell 0
        return (unsigned)fminf(fmaxf(s, 0.f), side - 1.f);
    };
    const unsigned k = D == 2 ? spread2(q(p.x, lo.x, hi.x)) | (spread2(q(p.y, lo.y, hi.y)) << 1)
                              : spread3(q(p.x, lo.x, hi.x)) | (spread3(q(p.y, lo.y, hi.y)) << 1) |
                                    (spread3(q(p.z, lo.z, hi.z)) << 2);
    cell[i] = k;
    atomicAdd(&count[k], 1u);
}

// Exclusive prefix sum of the kCells2 cell counts, in place (one block).
__global__ __launch_bounds__(1024) void k_med_cell_scan(unsigned* __restrict__ count) {
    constexpr int per = kCells2 / 1024;
    __shared__ unsigned wsum[16];
    unsigned v[per];
    unsigned loc = 0u;
    const unsigned* src = count + threadIdx.x * per;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = src[k];
        loc += v[k];
    }
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    unsigned inc = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    unsigned run = inc - loc;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int k = 0; k < per; ++k) {
        count[threadIdx.x * per + k] = run;
        run += v[k];
    }
}

// Points in cell order (the order inside a cell is immaterial).
__global__ __launch_bounds__(256) void k_med_cell_scatter(const float4* __restrict__ c, int T,
                                                          const unsigned* __restrict__ cell,
                                                          unsigned* __restrict__ cursor,
                                                          float4* __restrict__ cs) {
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= T) return;
    cs[atomicAdd(&cursor[cell[i]], 1u)] = c[i];
}

// Box of each group of kBoxPts consecutive points (a wave per group): gbox[2g]
// = min, gbox[2g + 1] = max; NaN if a coordinate is not finite.
__global__ __launch_bounds__(256) void k_med_group_box(const float4* __restrict__ cs, int T,
                                                       float4* __restrict__ gbox) {
    const int g = blockIdx.x * 4 + ((int)threadIdx.x >> 6), lane = (int)threadIdx.x & 63;
    const int ng = (T + kBoxPts - 1) / kBoxPts;
    if (g >= ng) return;
    const int i = g * kBoxPts + lane;
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    if (i < T) {
        const float4 p = cs[i];
        v[0] = v[3] = p.x;
        v[1] = v[4] = p.y;
        v[2] = v[5] = p.z;
        bad = !(isfinite(p.x) && isfinite(p.y) && isfinite(p.z));
    }
#pragma unroll
    for (int k = 0; k < 6; ++k)
        for (int o = 32; o > 0; o >>= 1) {
            const float u = __shfl_xor(v[k], o, 64);
            v[k] = k < 3 ? fminf(v[k], u) : fmaxf(v[k], u);
        }
    bad = __any(bad);
    if (lane == 0) {
        const float n = __int_as_float(0x7FC00000);
        gbox[2 * g] = bad ? make_float4(n, n, n, 0.f) : make_float4(v[0], v[1], v[2], 0.f);
        gbox[2 * g + 1] = bad ? make_float4(n, n, n, 0.f) : make_float4(v[3], v[4], v[5], 0.f);
    }
}

// 1: every pair of the two boxes is below lo; 2: every pair is above hi; 0: evaluate.
template <int D>
__device__ __forceinline__ int box_class(const float4& alo, const float4& ahi, const float4& blo,
                                         const float4& bhi, float lof, float hif) {
    const float fx = fmaxf(ahi.x - blo.x, bhi.x - alo.x), fy = fmaxf(ahi.y - blo.y, bhi.y - alo.y);
    const float gx = fmaxf(fmaxf(alo.x - bhi.x, blo.x - ahi.x), 0.f);
    const float gy = fmaxf(fmaxf(alo.y - bhi.y, blo.y - ahi.y), 0.f);
    float cmax = fy * fy, cmin = gy * gy;
    if (D == 3) {
        const float fz = fmaxf(ahi.z - blo.z, bhi.z - alo.z);
        const float gz = fmaxf(fmaxf(alo.z - bhi.z, blo.z - ahi.z), 0.f);
        cmax = __builtin_fmaf(fz, fz, cmax);
        cmin = __builtin_fmaf(gz, gz, cmin);
    }
    const float dmax = __builtin_fmaf(fx, fx, cmax), dmin = __builtin_fmaf(gx, gx, cmin);
    // NaN boxes compare false both ways
    if (dmax < lof) return 1;
    if (dmin > hif) return 2;
    return 0;
}

// Move the n candidates in buf (this wave's LDS buffer) to the wave's segment
// (lc entries there so far), the part that does not fit to the shared overflow
// list (one atomic for the wave).
__device__ __forceinline__ void wave_append(const float* buf, unsigned n, const CandStore& C,
                                            float* segp, unsigned& lc, MedState* st, int lane) {
    // the lanes read what other lanes of the wave wrote
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const unsigned room = lc < (unsigned)C.seg ? (unsigned)C.seg - lc : 0u;
    const unsigned a = min(n, room);
    for (unsigned k = (unsigned)lane; k < a; k += 64) segp[lc + k] = buf[k];
    if (n > a) {
        unsigned long long base = 0ull;
        if (lane == 0) base = atomicAdd(&st->novf, (unsigned long long)(n - a));
        base = __shfl(base, 0, 64);
        float* ovf = C.cand + (size_t)kBracketWaves * C.seg;
        for (unsigned k = a + (unsigned)lane; k < n; k += 64)
            if (base + (k - a) < C.ovf_cap) ovf[base + (k - a)] = buf[k];
    }
    lc += a;
    // the buffer is refilled only after every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One pair per lane: count it if below the bracket; if inside, pack it densely
// into the wave's LDS buffer (a lane's place: nbuf plus the lanes of the mask
// below it).  bl counts per lane; nbuf is wave-uniform; ok = false drops the pair.
__device__ __forceinline__ void bracket_pair(float d2, bool ok, unsigned lo, unsigned span,
                                             unsigned& bl, unsigned& nbuf, float* buf) {
    const unsigned u = __float_as_uint(d2);
    bl += (ok && u < lo) ? 1u : 0u;
    const bool in = ok && u - lo <= span;
    const unsigned long long m = __builtin_amdgcn_ballot_w64(in);
    if (m) {
        const unsigned pos = __builtin_amdgcn_mbcnt_hi(
            (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, nbuf));
        if (in) buf[pos] = d2;
        nbuf += (unsigned)__popcll(m);
    }
}

// One row per lane against the columns [c0, c1) of the staged columns cj
// (column c is point j0 + c), appending the wave's buffer to the global list
// when the next eight columns could overflow it.  CHECK keeps only pairs with
// j > i.  c0 is a multiple of 64 and c1 <= c0 + 64, so reading eight columns
// from any chunk start stays inside the 64 (a column past c1 is skipped).
template <int D, bool CHECK>
__device__ __forceinline__ void bracket_row(const float4* cj, int c0, int c1, int j0, const float4& xi,
                                            int ir, unsigned lo, unsigned span, unsigned& bl,
                                            unsigned& nbuf, float* buf, const CandStore& C,
                                            float* segp, unsigned& lc, MedState* st, int lane) {
    for (int jj = c0; jj < c1; jj += 8) {
        if (nbuf > (unsigned)(kWaveBuf - 8 * 64)) {
            wave_append(buf, nbuf, C, segp, lc, st, lane);
            nbuf = 0u;
        }
        float4 xj[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) xj[g] = cj[jj + g];
        if (jj + 8 <= c1) {
#pragma unroll
            for (int g = 0; g < 8; ++g)
                bracket_pair(sqdist<D>(xi, xj[g]), !CHECK || j0 + jj + g > ir, lo, span, bl, nbuf, buf);
        } else {
#pragma unroll
            for (int g = 0; g < 8; ++g)
                if (jj + g < c1)
                    bracket_pair(sqdist<D>(xi, xj[g]), !CHECK || j0 + jj + g > ir, lo, span, bl, nbuf,
                                 buf);
        }
    }
}

// The pairs of groups (gr <= gc) the boxes do not settle, listed as
// gr | gc << 16, and the pairs the boxes put below the bracket.  Block (x, y):
// gr = y against gc = 256 x + thread; block b = y * gridDim.x + x.  Pass 0
// writes each block's count of listed pairs and of pairs below; pass 1 (after
// k_med_list_scan has turned the counts into offsets) writes the list in block
// order.  No atomics: the list and the counts are the same on every run.
template <int D>
__global__ __launch_bounds__(256) void k_med_classify(const float4* __restrict__ gbox, int T,
                                                      const MedState* __restrict__ sst, int pass,
                                                      unsigned* __restrict__ counts,
                                                      unsigned long long* __restrict__ belows,
                                                      unsigned* __restrict__ list) {
    __shared__ unsigned wsum[4];
    __shared__ unsigned long long wbel[4];
    const int ng = (T + kBoxPts - 1) / kBoxPts;
    const int gr = blockIdx.y, gc = blockIdx.x * 256 + (int)threadIdx.x;
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    const float lof = __uint_as_float(sst->prefix[0]), hif = __uint_as_float(sst->prefix[1]);
    bool keep = false;
    unsigned long long bel = 0ull;
    if (gc >= gr && gc < ng) {
        if (gc == gr) {
            keep = true;
        } else {
            const int c = box_class<D>(gbox[2 * gr], gbox[2 * gr + 1], gbox[2 * gc], gbox[2 * gc + 1],
                                       lof, hif);
            // gr < gc: all kBoxPts rows of gr exist
            if (c == 1) bel = (unsigned long long)kBoxPts * (unsigned long long)min(kBoxPts, T - kBoxPts * gc);
            keep = c == 0;
        }
    }
    const unsigned long long m = __builtin_amdgcn_ballot_w64(keep);
    const unsigned pos = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bel += __shfl_down(bel, o, 64);
    if (lane == 0) {
        wsum[wave] = (unsigned)__popcll(m);
        wbel[wave] = bel;
    }
    __syncthreads();
    unsigned before = 0u, total = 0u;
    unsigned long long btot = 0ull;
    for (int w = 0; w < 4; ++w) {
        before += w < wave ? wsum[w] : 0u;
        total += wsum[w];
        btot += wbel[w];
    }
    if (pass == 0) {
        if (threadIdx.x == 0) {
            counts[b] = total;
            belows[b] = btot;
        }
    } else if (keep) {
        list[counts[b] + before + pos] = (unsigned)gr | ((unsigned)gc << 16);
    }
}

// Exclusive prefix sum of the nb block counts (in place, one block), their
// total as st->nitems, and the pairs below the bracket added to st->below.
__global__ __launch_bounds__(1024) void k_med_list_scan(unsigned* __restrict__ counts,
                                                        const unsigned long long* __restrict__ belows,
                                                        int nb, MedState* st) {
    __shared__ unsigned wsum[16];
    __shared__ unsigned long long wbel[16];
    const int per = (nb + 1023) / 1024;
    const int k0 = (int)threadIdx.x * per, k1 = min(nb, k0 + per);
    unsigned loc = 0u;
    unsigned long long bel = 0ull;
    for (int k = k0; k < k1; ++k) {
        loc += counts[k];
        bel += belows[k];
    }
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
    unsigned inc = loc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) bel += __shfl_down(bel, o, 64);
    if (lane == 63) wsum[wave] = inc;
    if (lane == 0) wbel[wave] = bel;
    __syncthreads();
    unsigned run = inc - loc;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int k = k0; k < k1; ++k) {
        const unsigned c = counts[k];
        counts[k] = run;
        run += c;
    }
    if (threadIdx.x == 0) {
        unsigned total = 0u;
        unsigned long long btot = 0ull;
        for (int w = 0; w < 16; ++w) {
            total += wsum[w];
            btot += wbel[w];
        }
        st->nitems = total;
        st->below += btot;
    }
}

// The listed pairs of groups, pair by pair: one pair of groups per wave at a
// time (its 64 rows one per lane, its 64 columns staged in the wave's LDS), the
// next pair's rows and columns read while this one is evaluated.  The list is
// dealt to the waves in turn (every pair of groups costs about the same); a
// wave reads its list entries 64 at a time, one per lane.  Runs with
// kBracketBlocks blocks: wave w = 4 * blockIdx.x + wave owns candidate segment w and
// writes its count to C.segcnt[w].
template <int D>
__global__ __launch_bounds__(256) void k_med_bracket(const float4* __restrict__ cs,
                                                     const unsigned* __restrict__ list, int T,
                                                     const MedState* __restrict__ sst,
                                                     MedState* st, CandStore C) {
    __shared__ float4 cjw[4][kBoxPts];
    __shared__ float wbuf[4][kWaveBuf];
    const int lane = (int)threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    float* buf = wbuf[wave];
    float4* cw = cjw[wave];
    const unsigned lo = sst->prefix[0], hi = sst->prefix[1];
    const unsigned span = hi - lo;                 // u in [lo, hi]  <=>  u - lo <= span
    const int n = (int)st->nitems;
    const int nw = (int)gridDim.x * 4;
    const int first = (int)blockIdx.x * 4 + wave;
    // the wave's k-th pair of groups is list[first + k nw]; lane l holds entry
    // k = 64 q + l of batch q
    const int nmine = first < n ? (n - first + nw - 1) / nw : 0;
    unsigned bl = 0u, nbuf = 0u, lc = 0u;
    float* segp = C.cand + (size_t)first * C.seg;
    unsigned batch = 0u;
    if (lane < nmine) batch = list[first + lane * nw];
    // wave-uniform: the loops below run on scalar bounds
    unsigned item = __builtin_amdgcn_readfirstlane(__shfl(batch, 0, 64));
    float4 xr = make_float4(0.f, 0.f, 0.f, 0.f), xc = xr;
    if (nmine > 0) {
        xr = cs[min((int)(item & 0xFFFFu) * kBoxPts + lane, T - 1)];
        xc = cs[min((int)(item >> 16) * kBoxPts + lane, T - 1)];
    }
    for (int k = 0; k < nmine; ++k) {
        const int gr = (int)(item & 0xFFFFu), gc = (int)(item >> 16);
        const float4 xi = xr;
        cw[lane] = xc;
        // the lanes read the columns other lanes wrote
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (k + 1 < nmine) {
            if (((k + 1) & 63) == 0) {
                const int q = k + 1 + lane;
                batch = q < nmine ? list[first + q * nw] : 0u;
            }
            item = __builtin_amdgcn_readfirstlane(__shfl(batch, (k + 1) & 63, 64));
            xr = cs[min((int)(item & 0xFFFFu) * kBoxPts + lane, T - 1)];
            xc = cs[min((int)(item >> 16) * kBoxPts + lane, T - 1)];
        }
        const int ncols = min(kBoxPts, T - kBoxPts * gc);
        // rows past the end take j > T, which no column satisfies
        const int ir = min(kBoxPts * gr + lane, T);
        if (gr == gc)
            bracket_row<D, true>(cw, 0, ncols, kBoxPts * gc, xi, ir, lo, span, bl, nbuf, buf, C, segp,
                                 lc, st, lane);
        else
            bracket_row<D, false>(cw, 0, ncols, kBoxPts * gc, xi, ir, lo, span, bl, nbuf, buf, C, segp,
                                  lc, st, lane);
        // the columns are overwritten only after every lane has read them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (nbuf) wave_append(buf, nbuf, C, segp, lc, st, lane);
    if (lane == 0) C.segcnt[first] = lc;
    // pairs below the bracket: a wave sum, then one atomic per wave
    unsigned long long b = bl;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b += __shfl_down(b, o, 64);
    if (lane == 0 && b) atomicAdd(&st->below, b);
}

// Count the candidates (the segments' counts and the overflow appends); use
// them if both targets fall inside the bracket and none was lost.  When the
// bracket's ends agree on the first pass's bits (30..19), so does every
// candidate: the first pass over them would only find that bin, so its prefix
// is set here and the pass skipped.
__global__ __launch_bounds__(1024) void k_med_decide(MedState* st, const MedState* __restrict__ sst,
                                                     int T, const unsigned* __restrict__ segcnt,
                                                     unsigned long long ovf_cap) {
    __shared__ unsigned long long wsum[16];
    unsigned long long c = 0ull;
    for (int w = threadIdx.x; w < kBracketWaves; w += 1024) c += segcnt[w];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const unsigned long long novf = st->novf;
    unsigned long long nc = novf;
    for (int w = 0; w < 16; ++w) nc += wsum[w];
    st->ncand = nc;
    const unsigned long long n = med_pairs(T);
    const unsigned long long ra = n ? (n - 1) / 2 : 0, rb = n / 2;
    const unsigned long long below = st->below;
    const unsigned first = med_pass(1).fixed_mask;           // bits 30..19
    const unsigned lo = sst->prefix[0], hi = sst->prefix[1];
    st->prefix[0] = st->prefix[1] = 0u;
    st->skip0 = 0;
    if (novf <= ovf_cap && below <= ra && rb < below + nc) {
        st->mode = 1;
        st->rank[0] = ra - below;
        st->rank[1] = rb - below;
        if (((lo ^ hi) & first) == 0u) {
            st->prefix[0] = st->prefix[1] = lo & first;
            st->skip0 = 1;
        }
    } else {
        st->mode = 0;
        st->rank[0] = ra;
        st->rank[1] = rb;
    }
}

// The histogram of k_flat_hist over the candidates: each segment's entries, then
// the overflow list's.  Runs only when st->mode == 1.
__global__ __launch_bounds__(256) void k_cand_hist(CandStore C, int pass, const MedState* st,
                                                   unsigned long long* __restrict__ hist) {
    __shared__ unsigned h[2][kMedBins];
    if (st->mode != 1 || (pass == 0 && st->skip0)) return;
    const MedPass P = med_pass(pass);
    const unsigned pa = st->prefix[0], pb = st->prefix[1];
    const bool two = pa != pb;
    const int nb = 1 << P.bits;
    for (int k = threadIdx.x; k < nb; k += 256) {
        h[0][k] = 0u;
        h[1][k] = 0u;
    }
    __syncthreads();
    // Candidates lie inside the bracket, so most of a wave's values share a bin
    // (all of them in the first pass, whose 12 bits are coarser than the
    // bracket): the lanes in the bin of the wave's first active lane add one
    // count together, the others one each.
    const int lane = (int)threadIdx.x & 63;
    auto add = [&](float v) {
        const unsigned u = __float_as_uint(v);
        const unsigned bin = (u >> P.shift) & (unsigned)(nb - 1);
        const unsigned b0 = __builtin_amdgcn_readfirstlane(bin);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (t == 1 && !two) break;
            const bool mine = (u & P.fixed_mask) == (t ? pb : pa);
            const unsigned long long m = __builtin_amdgcn_ballot_w64(mine && bin == b0);
            if (m && lane == __builtin_ctzll(m)) atomicAdd(&h[t][b0], (unsigned)__popcll(m));
            if (mine && bin != b0) atomicAdd(&h[t][bin], 1u);
        }
    };
    for (int w = blockIdx.x; w < kBracketWaves; w += gridDim.x) {
        const float* v = C.cand + (size_t)w * C.seg;
        const unsigned n = C.segcnt[w];
        for (unsigned k = threadIdx.x; k < n; k += 256) add(v[k]);
    }
    const float* ovf = C.cand + (size_t)kBracketWaves * C.seg;
    const unsigned long long no = min(st->novf, C.ovf_cap);
    for (unsigned long long k = (unsigned long long)blockIdx.x * 256 + threadIdx.x; k < no;
         k += (unsigned long long)gridDim.x * 256)
        add(ovf[k]);
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
// Runs only when gate < 0 or st->mode == gate; `finish` turns the final pass's
// values into the median and the bandwidth.
__global__ __launch_bounds__(256) void k_med_select(MedState* st, unsigned long long* hist,
                                                    int pass, int T, int gate, int finish) {
    __shared__ unsigned long long wsum[4];
    if (gate >= 0 && st->mode != gate) return;
    if (gate == 1 && pass == 0 && st->skip0) return;       // prefix set by k_med_decide
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
    if (threadIdx.x == 0 && pass == 2 && finish) {
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

// Mean of the samples (double, fixed order, non-finite coordinates skipped).  The
// kernel weights depend only on differences x_i - x_j, but the float32 scale by
// sqrt(log2(e)/h) is not translation invariant: far from the coordinate origin it
// would round away the low bits of every difference.  Subtracting the mean first
// (exact for nearby float32 values) keeps them.
constexpr int kSvOriginBlocks = 64;

// Partial sums of the mean: block b sums the samples of its contiguous share in
// a fixed order into part[b] = (sum x, sum y, sum z, count); k_svgd_stage adds
// the kSvOriginBlocks partials in block order.
__global__ __launch_bounds__(256) void k_sv_origin(const float* __restrict__ x, int T, int d,
                                                   double* __restrict__ part) {
    __shared__ double red[4][256];
    const int chunk = (T + kSvOriginBlocks - 1) / kSvOriginBlocks;
    const int i0 = (int)blockIdx.x * chunk, i1 = min(T, i0 + chunk);
    double s[3] = {0.0, 0.0, 0.0}, n = 0.0;
    // a skipped sample adds zeros (no branch), so eight loads can be in flight
#pragma unroll 8
    for (int i = i0 + (int)threadIdx.x; i < i1; i += 256) {
        const float* p = x + (size_t)i * d;
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
    red[3][threadIdx.x] = n;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int t = 0; t < 4; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_svgd_stage(const float* __restrict__ x,
                                                    const float* __restrict__ score, int T, int Tpad,
                                                    int d, float h_fixed, MedState* st,
                                                    const double* __restrict__ opart,
                                                    float4* __restrict__ qc,
                                                    float4* __restrict__ krec) {
    // the origin: the mean of k_sv_origin's partials, added in block order
    __shared__ float origin[3];
    if (threadIdx.x < 3) {
        double a = 0.0, n = 0.0;
        for (int b = 0; b < kSvOriginBlocks; ++b) {
            a += opart[4 * b + threadIdx.x];
            n += opart[4 * b + 3];
        }
        origin[threadIdx.x] = (int)threadIdx.x < d ? (float)(a / (n > 0.0 ? n : 1.0)) : 0.f;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (h_fixed > 0.f && i == 0) st->h = h_fixed;
    const float h = h_fixed > 0.f ? h_fixed : st->h;
    const float s = (float)sqrt(kLog2eD / (double)h);
    if (i >= Tpad) return;
    if (i < T) {
        float c[3] = {0, 0, 0}, sc[3] = {0, 0, 0};
        for (int t = 0; t < d; ++t) {
            c[t] = (x[(size_t)i * d + t] - origin[t]) * s;
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
    MedState* sst;     // selection state of the bracket's sample (large T)
    float* samp;       // [kMedSample] sampled squared distances (large T)
    float* cand;       // [kBracketWaves cand_seg(T) + cand_cap(T)] squared distances inside the bracket (large T)
    unsigned* segcnt;  // [kBracketWaves] candidates in each wave's segment (large T)
    unsigned long long* hist;
    float* score;
    float4* cmed;      // raw coordinates for the median
    float4* box;       // [2] bounding box of the points (large T)
    unsigned* cell;    // [T] Morton cell of each point (large T)
    unsigned* ccount;  // [kCells2] cell counts, then their prefix sums (large T)
    float4* cs;        // [T] the points in cell order (large T)
    float4* gbox;      // [2 ceil(T / kBoxPts)] boxes of the groups of cs (large T)
    unsigned* glist;   // [ng (ng + 1) / 2] pairs of groups left to evaluate (large T)
    unsigned* gcount;  // [ng ceil(ng / 256)] per classifying block: listed pairs, then offsets
    unsigned long long* gbelow;  // [same] per classifying block: pairs below the bracket
    double* origin;    // [4 kSvOriginBlocks] partial sums of the mean, subtracted before the bandwidth scale
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
    L.sst = a.take<MedState>(1);
    L.hist = a.take<unsigned long long>(2 * kMedBins);
    // the bracket's buffers exist only where a median can be asked for
    const bool bracket = T >= kBracketMinT && T <= kMaxMedianT;
    L.samp = bracket ? a.take<float>(kMedSample) : nullptr;
    L.cand = bracket ? a.take<float>((size_t)(kBracketWaves * cand_seg(T) + cand_cap(T))) : nullptr;
    L.segcnt = bracket ? a.take<unsigned>(kBracketWaves) : nullptr;
    L.score = a.take<float>((size_t)T * d);
    L.cmed = a.take<float4>(T);
    const bool boxes = bracket && T >= kBoxMinT;
    L.box = boxes ? a.take<float4>(2) : nullptr;
    L.cell = boxes ? a.take<unsigned>(T) : nullptr;
    L.ccount = boxes ? a.take<unsigned>(kCells2) : nullptr;
    L.cs = boxes ? a.take<float4>(T) : nullptr;
    const size_t ngrp = (size_t)((T + kBoxPts - 1) / kBoxPts);
    L.gbox = boxes ? a.take<float4>(2 * ngrp) : nullptr;
    L.glist = boxes ? a.take<unsigned>(ngrp * (ngrp + 1) / 2) : nullptr;
    const size_t nblk = ngrp * ((ngrp + 255) / 256);
    L.gcount = boxes ? a.take<unsigned>(nblk) : nullptr;
    L.gbelow = boxes ? a.take<unsigned long long>(nblk) : nullptr;
    L.origin = a.take<double>(4 * kSvOriginBlocks);
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
    if (h <= 0.f && T64 > kMaxMedianT) return fail(CT_E_SHAPE, "median bandwidth supports T <= %d", kMaxMedianT);
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
        const dim3 tiles(med_grid(T));
        if (T >= kBracketMinT) {
            const unsigned long long cap = cand_cap(T);
            hipLaunchKernelGGL(k_sample_init, dim3(1), dim3(64), 0, st, L.sst);
            if (d == 2)
                hipLaunchKernelGGL(k_med_sample<2>, dim3(kMedSample / 256), dim3(256), 0, st, L.cmed, T, L.samp);
            else
                hipLaunchKernelGGL(k_med_sample<3>, dim3(kMedSample / 256), dim3(256), 0, st, L.cmed, T, L.samp);
            CT_CHECK_HIP(hipGetLastError());
            for (int pass = 0; pass < 3; ++pass) {
                hipLaunchKernelGGL(k_flat_hist, dim3(1024), dim3(256), 0, st, L.samp, kMedSample, pass, L.sst, L.hist);
                hipLaunchKernelGGL(k_med_select, dim3(1), dim3(256), 0, st, L.sst, L.hist, pass, T, -1, 0);
                CT_CHECK_HIP(hipGetLastError());
            }
            CandStore C;
            C.cand = L.cand;
            C.segcnt = L.segcnt;
            C.seg = cand_seg(T);
            C.ovf_cap = cap;
            if (T < kBoxMinT) {
                // every pair in the original order; all candidates in the shared list
                hipLaunchKernelGGL(k_fill_u32, dim3(kBracketWaves / 256), dim3(256), 0, st, L.segcnt, kBracketWaves, 0u);
                float* ovf = L.cand + (size_t)kBracketWaves * C.seg;
                const dim3 tgrid(bracket_tile_grid(T));
                if (d == 2)
                    hipLaunchKernelGGL(k_med_bracket_tiles<2>, tgrid, dim3(256), 0, st, L.cmed, T, L.sst, L.st, ovf, cap);
                else
                    hipLaunchKernelGGL(k_med_bracket_tiles<3>, tgrid, dim3(256), 0, st, L.cmed, T, L.sst, L.st, ovf, cap);
                CT_CHECK_HIP(hipGetLastError());
            } else {
                // the points in Morton-cell order and the boxes of their groups
                const int ng = (T + kBoxPts - 1) / kBoxPts;
                hipLaunchKernelGGL(k_fill_u32, dim3(kCells2 / 256), dim3(256), 0, st, L.ccount, kCells2, 0u);
                hipLaunchKernelGGL(k_med_box, dim3(1), dim3(1024), 0, st, L.cmed, T, L.box);
                if (d == 2)
                    hipLaunchKernelGGL(k_med_cell<2>, dim3((T + 255) / 256), dim3(256), 0, st, L.cmed, T, L.box, L.cell, L.ccount);
                else
                    hipLaunchKernelGGL(k_med_cell<3>, dim3((T + 255) / 256), dim3(256), 0, st, L.cmed, T, L.box, L.cell, L.ccount);
                hipLaunchKernelGGL(k_med_cell_scan, dim3(1), dim3(1024), 0, st, L.ccount);
                hipLaunchKernelGGL(k_med_cell_scatter, dim3((T + 255) / 256), dim3(256), 0, st, L.cmed, T, L.cell, L.ccount, L.cs);
                hipLaunchKernelGGL(k_med_group_box, dim3((ng + 3) / 4), dim3(256), 0, st, L.cs, T, L.gbox);
                CT_CHECK_HIP(hipGetLastError());
                const dim3 cgrid((ng + 255) / 256, ng), bgrid(kBracketBlocks);
                const int nblk = (int)(cgrid.x * cgrid.y);
                for (int pass = 0; pass < 2; ++pass) {
                    if (d == 2)
                        hipLaunchKernelGGL(k_med_classify<2>, cgrid, dim3(256), 0, st, L.gbox, T, L.sst, pass, L.gcount, L.gbelow, L.glist);
                    else
                        hipLaunchKernelGGL(k_med_classify<3>, cgrid, dim3(256), 0, st, L.gbox, T, L.sst, pass, L.gcount, L.gbelow, L.glist);
                    if (pass == 0)
                        hipLaunchKernelGGL(k_med_list_scan, dim3(1), dim3(1024), 0, st, L.gcount, L.gbelow, nblk, L.st);
                }
                if (d == 2)
                    hipLaunchKernelGGL(k_med_bracket<2>, bgrid, dim3(256), 0, st, L.cs, L.glist, T, L.sst, L.st, C);
                else
                    hipLaunchKernelGGL(k_med_bracket<3>, bgrid, dim3(256), 0, st, L.cs, L.glist, T, L.sst, L.st, C);
            }
            hipLaunchKernelGGL(k_med_decide, dim3(1), dim3(1024), 0, st, L.st, L.sst, T, L.segcnt, cap);
            CT_CHECK_HIP(hipGetLastError());
            for (int pass = 0; pass < 3; ++pass) {
                hipLaunchKernelGGL(k_cand_hist, dim3(1024), dim3(256), 0, st, C, pass, L.st, L.hist);
                hipLaunchKernelGGL(k_med_select, dim3(1), dim3(256), 0, st, L.st, L.hist, pass, T, 1, 1);
                CT_CHECK_HIP(hipGetLastError());
            }
        }
        // all pairs (small T, or a bracket that missed): each kernel returns at once otherwise
        for (int pass = 0; pass < 3; ++pass) {
            if (d == 2)
                hipLaunchKernelGGL(k_med_hist<2>, tiles, dim3(256), 0, st, L.cmed, T, pass, L.st, L.hist);
            else
                hipLaunchKernelGGL(k_med_hist<3>, tiles, dim3(256), 0, st, L.cmed, T, pass, L.st, L.hist);
            CT_CHECK_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_med_select, dim3(1), dim3(256), 0, st, L.st, L.hist, pass, T, 0, 1);
            CT_CHECK_HIP(hipGetLastError());
        }
    }
    const int Tpad = pad_keys(T);
    hipLaunchKernelGGL(k_sv_origin, dim3(kSvOriginBlocks), dim3(256), 0, st, x, T, d, L.origin);
    CT_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_svgd_stage, dim3((Tpad + 255) / 256), dim3(256), 0, st, x, score, T, Tpad,
                       d, h > 0.f ? h : 0.f, L.st, L.origin, L.qc, L.krec);
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
    // with profiling on, the sum kernel carries events stamped with its own start and end
    hipEvent_t e0, e1;
    void* tok = profile_kernel_begin(&e0, &e1);
    const dim3 grid(J.nqb * J.splits), block(256);
    if (d == 2) {
        if (e0) hipExtLaunchKernelGGL((k_svgd_sum<2, kSvR>), grid, block, 0, st, e0, e1, 0, J);
        else hipLaunchKernelGGL((k_svgd_sum<2, kSvR>), grid, block, 0, st, J);
    } else {
        if (e0) hipExtLaunchKernelGGL((k_svgd_sum<3, kSvR>), grid, block, 0, st, e0, e1, 0, J);
        else hipLaunchKernelGGL((k_svgd_sum<3, kSvR>), grid, block, 0, st, J);
    }
    CT_CHECK_HIP(hipGetLastError());
    profile_kernel_end(tok, 2, 0, kSvR * 100, J.nqb * J.splits, (double)T * T);
    if (d == 2)
        hipLaunchKernelGGL(k_svgd_merge<2>, dim3((T + kSvMergeRows - 1) / kSvMergeRows), dim3(256), 0,
                           st, J, kSvR);
    else
        hipLaunchKernelGGL(k_svgd_merge<3>, dim3((T + kSvMergeRows - 1) / kSvMergeRows), dim3(256), 0,
                           st, J, kSvR);
    CT_CHECK_HIP(hipGetLastError());
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
