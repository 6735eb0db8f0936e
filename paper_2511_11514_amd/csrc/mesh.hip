// Multi-workgroup LDS-resident solve of a small Sinkhorn problem: the K
// iterations of the cross and self sweeps (Sec. II-B, eq. 5 solved by
// Sinkhorn's algorithm; eq. 6's self terms) in one launch of G workgroups
// without grid barriers.
//
// Every block holds all points (their records) in LDS and owns at most 64 rows
// of each point set: rows [b*xr, (b+1)*xr) of x (the f and p updates) and
// [b*yr, (b+1)*yr) of y (the g and q updates).  A half-iteration of a block:
//   gather  the potentials its keys need from every block (f: the new one; g, p,
//           q: the ones the iteration starts from) into the .w of its records;
//   sweep   its own rows over all keys (tasks of 64 rows times one key range,
//           partials in LDS, as in the one-workgroup solve);
//   combine its rows, keep their new potentials and publish them.
// Potentials travel as 64-bit words (version << 32 | float bits), stored and
// polled with relaxed device-scope atomics: a reader waits until a word carries
// the version it needs, so each value brings its own synchronisation and no
// block writes back or invalidates a cache (a grid barrier's release and
// acquire fences do, and cost several microseconds at every half-iteration).
// Words of version v live in buffer v mod 2: a block can publish version v + 2
// only after it has read version v + 1 of every other block's rows, which each
// of them publishes only after it has read its own inputs of version v, so no
// word is overwritten before every reader has taken it.  The buffers are filled
// with a never-matching version before each launch.
//
// All G blocks must be resident together (the plan keeps G at or below what
// fits).  Every wait is bounded; a wait that gives up sets a flag that makes
// every later wait pass at once, marks the outputs invalid and makes the status
// query report it, so even a broken launch finishes.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "ct_internal.h"
#include "lds_solve.h"

namespace ct {

namespace {

using namespace lds_solve;

__device__ __forceinline__ unsigned long long ldx(const unsigned long long* w) {
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// |v'|^2 from a record's (2v'): a power-of-two scaling of the same FMA chain, so
// the same float as when formed from v' itself.
__device__ __forceinline__ float rec_norm(float x2, float y2, float z2) {
    return 0.25f * __builtin_fmaf(x2, x2, __builtin_fmaf(y2, y2, z2 * z2));
}

// Gather the half-iteration's potentials into the key records.  A thread takes
// up to kMeshGatherPerThread words: their first loads are issued together, then
// each word not yet at the awaited version is polled on its own.
__device__ __forceinline__ void gather(const MeshArgs& A, int h, int k, float* lds) {
    const int tid = (int)threadIdx.x;
    const int ng = A.ngat[h];
    const MeshGather& G0 = A.gat[h][0];
    const MeshGather& G1 = A.gat[h][ng > 1 ? 1 : 0];
    const int n0 = G0.n, ntot = n0 + (ng > 1 ? G1.n : 0);
    const unsigned v0 = (unsigned)(k + G0.lag), v1 = (unsigned)(k + G1.lag);
    const unsigned long long* X0 = G0.xch + (size_t)(v0 & 1u) * G0.n;
    const unsigned long long* X1 = G1.xch + (size_t)(v1 & 1u) * G1.n;
    unsigned long long w[kMeshGatherPerThread];
#pragma unroll
    for (int s = 0; s < kMeshGatherPerThread; ++s) {
        const int e = tid + s * kMeshThreads;
        if (e < ntot) w[s] = e < n0 ? ldx(X0 + e) : ldx(X1 + (e - n0));
    }
#pragma unroll
    for (int s = 0; s < kMeshGatherPerThread; ++s) {
        const int e = tid + s * kMeshThreads;
        if (e >= ntot) break;
        const bool sec = e >= n0;
        const int i = sec ? e - n0 : e;
        const unsigned long long* a = sec ? X1 + i : X0 + i;
        const unsigned want = (sec ? v1 : v0) + A.version_extra;
        unsigned spins = 0;
        while ((unsigned)(w[s] >> 32) != want) {
            if (spins >= A.polls ||
                __hip_atomic_load(A.expired, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                atomicOr(A.expired, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            ++spins;
            w[s] = ldx(a);
        }
        const float v = __uint_as_float((unsigned)w[s]);
        const int lw = sec ? G1.lw : G0.lw;
        const float l = lw >= 0 ? lds[lw + i] : A.log2a;
        float* rec = lds + 4 * ((sec ? G1.rec : G0.rec) + i);
        rec[3] = __builtin_fmaf(v, A.kappa, l) - rec_norm(rec[0], rec[1], rec[2]);
    }
}

__device__ __forceinline__ void publish(unsigned long long* xch, int n, int row, unsigned version,
                                        float v) {
    const unsigned long long word = ((unsigned long long)version << 32) | __float_as_uint(v);
    __hip_atomic_store(xch + (size_t)(version & 1u) * n + row, word, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

extern __shared__ float4 mesh_lds4[];

// Block b of one problem's exchange solve.
template <int D>
__device__ __forceinline__ void mesh_solve(const MeshArgs& A, const int b) {
    float4* lds4 = mesh_lds4;
    float* lds = reinterpret_cast<float*>(lds4);
    const int tid = (int)threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const float ninf = -__builtin_huge_valf();
    const float kap = A.kappa;
    const int x0 = min(A.T, b * A.xr), x1 = min(A.T, x0 + A.xr);
    const int y0 = min(A.M, b * A.yr), y1 = min(A.M, y0 + A.yr);

    // load: every point's record (2v', .w filled by the gathers) and log2 b; the
    // own rows' potentials (indexed from the block's first own row), published as
    // version 0
    for (int i = tid; i < A.T; i += kMeshThreads) {
        const float4 c = A.cx[i];
        const float4 r = make_float4(2.f * c.x, 2.f * c.y, D == 3 ? 2.f * c.z : 0.f, 0.f);
        lds4[A.o_rf + i] = r;
        if (A.debias) lds4[A.o_rp + i] = r;
    }
    for (int j = tid; j < A.M; j += kMeshThreads) {
        const float4 c = A.cy[j];
        const float4 r = make_float4(2.f * c.x, 2.f * c.y, D == 3 ? 2.f * c.z : 0.f, 0.f);
        lds4[A.o_rg + j] = r;
        if (A.ref_iter) lds4[A.o_rq + j] = r;
        lds[A.o_lb + j] = A.log2b[j];
    }
    for (int i = x0 + tid; i < x1; i += kMeshThreads) {
        lds[A.o_f + i - x0] = A.f[i];   // f's version 0 is never awaited: iteration 0 reads version 1
        if (A.debias) {
            const float p = A.p[i];
            lds[A.o_p + i - x0] = p;
            publish(A.xch_p, A.T, i, 0u, p);
        }
    }
    for (int j = y0 + tid; j < y1; j += kMeshThreads) {
        const float g = A.g[j];
        lds[A.o_g + j - y0] = g;
        publish(A.xch_g, A.M, j, 0u, g);
        if (A.ref_iter) {
            const float q = A.q[j];
            lds[A.o_q + j - y0] = q;
            publish(A.xch_q, A.M, j, 0u, q);
        }
    }
    __syncthreads();

    for (int k = 0; k < A.iters; ++k) {
        const bool lagged = !A.safe_only && (A.lagged0 || k > 0);
        for (int h = 0; h < 2; ++h) {
            gather(A, h, k, lds);
            __syncthreads();
            const int nj = A.njobs[h];
            // sweep: the block's rows (one per lane) over one key range per task
            for (int t = wave; t < A.ntasks[h]; t += kMeshWaves) {
                const int jj = (nj > 1 && t >= A.job[h][1].task0) ? 1 : 0;
                const MeshJob& J = A.job[h][jj];
                const int r0 = J.yside ? y0 : x0;
                const int nr = (J.yside ? y1 : x1) - r0;
                if (nr <= 0) continue;
                const int split = t - J.task0;
                const int k0 = min(J.keys, split * J.kps), k1 = min(J.keys, k0 + J.kps);
                // lanes past the last row repeat it; the combine never reads them
                const int lr = min(lane, nr - 1);
                const float4 v = lds4[J.qrec + r0 + lr];
                const float q[1][3] = {{0.5f * v.x, 0.5f * v.y, 0.5f * v.z}};
                float m[1] = {lagged ? -lds[J.qpot + lr] * kap : 0.f};
                const float C[1] = {-rec_norm(v.x, v.y, v.z) - m[0]};
                float s[1];
                if (lagged) sum_lagged<D, 1>(lds4 + J.krec, k0, k1, q, C, s);
                else sum_safe<D, 1>(lds4 + J.krec, k0, k1, q, C, m, s);
                lds[A.o_ps + t * 64 + lane] = s[0];
                if (!lagged) lds[A.o_pm + t * 64 + lane] = m[0];
            }
            __syncthreads();
            // combine and publish: one thread per own row of the half-iteration's jobs
            const MeshJob& J0 = A.job[h][0];
            const MeshJob& J1 = A.job[h][nj > 1 ? 1 : 0];
            const int a0 = J0.yside ? y0 : x0;
            const int a1 = J1.yside ? y0 : x0;
            const int n0 = max(0, (J0.yside ? y1 : x1) - a0);
            const int nrows = n0 + (nj > 1 ? max(0, (J1.yside ? y1 : x1) - a1) : 0);
            for (int idx = tid; idx < nrows; idx += kMeshThreads) {
                const bool sec = idx >= n0;
                const int row = sec ? a1 + (idx - n0) : a0 + idx;
                const int lrow = sec ? idx - n0 : idx;
                const int task0 = sec ? J1.task0 : J0.task0;
                const int splits = sec ? J1.splits : J0.splits;
                const int qpot = sec ? J1.qpot : J0.qpot;
                const int avg = sec ? J1.avg : J0.avg;
                const float* ps = lds + A.o_ps + task0 * 64 + lrow;
                const float* pm = lds + A.o_pm + task0 * 64 + lrow;
                const float old = lds[qpot + lrow];
                float mm, ss = 0.f;
                if (lagged) {
                    mm = -old * kap;
                    for (int sp = 0; sp < splits; ++sp) ss += ps[sp * 64];
                } else {
                    mm = ninf;
                    for (int sp = 0; sp < splits; ++sp) mm = fmaxf(mm, pm[sp * 64]);
                    for (int sp = 0; sp < splits; ++sp) {
                        const float mk = pm[sp * 64];
                        if (mk != ninf) ss += ps[sp * 64] * tex2(mk - mm);
                    }
                }
                if (lagged && !(ss >= kLo && ss <= kHi)) {
                    // the row's shift was unusable: recompute with a tracked maximum
                    const float4 v = lds4[(sec ? J1.qrec : J0.qrec) + row];
                    const float qv[1][3] = {{0.5f * v.x, 0.5f * v.y, 0.5f * v.z}};
                    const float C1[1] = {-rec_norm(v.x, v.y, v.z)};
                    float m1[1], s1[1];
                    sum_safe<D, 1>(lds4 + (sec ? J1.krec : J0.krec), 0, sec ? J1.keys : J0.keys,
                                   qv, C1, m1, s1);
                    mm = m1[0];
                    ss = s1[0];
                    atomicAdd(A.rescued, 1u);
                }
                const float tn = -(mm + __log2f(ss)) * A.inv_kappa;
                const float nv = avg ? 0.5f * (old + tn) : tn;
                lds[qpot + lrow] = nv;
                publish(sec ? J1.xch : J0.xch, (sec ? J1.yside : J0.yside) ? A.M : A.T, row,
                        (unsigned)(k + 1), nv);
            }
        }
    }

    // store the own rows: potentials and the key terms the final pass reads
    const int hofs = D == 2 ? 2 : 3;
    for (int i = x0 + tid; i < x1; i += kMeshThreads) {
        const float f = lds[A.o_f + i - x0];
        A.f[i] = f;
        reinterpret_cast<float*>(A.xrec_f + i)[hofs] = __builtin_fmaf(f, kap, A.log2a);
        if (A.debias) {
            const float p = lds[A.o_p + i - x0];
            A.p[i] = p;
            reinterpret_cast<float*>(A.xrec_p + i)[hofs] = __builtin_fmaf(p, kap, A.log2a);
        }
    }
    for (int j = y0 + tid; j < y1; j += kMeshThreads) {
        const float g = lds[A.o_g + j - y0], lb = lds[A.o_lb + j];
        A.g[j] = g;
        reinterpret_cast<float*>(A.yrec_g + j)[hofs] = __builtin_fmaf(g, kap, lb);
        if (A.ref_iter) {
            const float q = lds[A.o_q + j - y0];
            A.q[j] = q;
            reinterpret_cast<float*>(A.yrec_q + j)[hofs] = __builtin_fmaf(q, kap, lb);
        }
    }
}

template <int D>
__global__ __launch_bounds__(kMeshThreads) void k_mesh(MeshArgs A) {
    mesh_solve<D>(A, (int)blockIdx.x);
}

// Many problems in one launch: blk_end[p] is the end of problem p's blocks.  A
// block finds its problem, copies the problem's arguments into LDS and runs that
// problem's exchange solve as its block (blockIdx.x - start).  Every problem
// exchanges only among its own blocks.
template <int D>
__global__ __launch_bounds__(kMeshThreads) void k_mesh_batch(const MeshArgs* __restrict__ tab,
                                                             const int* __restrict__ blk_end,
                                                             int nprob) {
    __shared__ MeshArgs sA;
    const int bid = (int)blockIdx.x;
    int lo = 0, hi = nprob - 1;   // first problem whose blocks end after bid
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (blk_end[mid] > bid) hi = mid;
        else lo = mid + 1;
    }
    const int start = lo ? blk_end[lo - 1] : 0;
    const unsigned* src = reinterpret_cast<const unsigned*>(tab + lo);
    unsigned* dst = reinterpret_cast<unsigned*>(&sA);
    for (int i = (int)threadIdx.x; i < (int)(sizeof(MeshArgs) / 4); i += kMeshThreads) dst[i] = src[i];
    __syncthreads();
    mesh_solve<D>(sA, bid - start);
}

}  // namespace

bool mesh_plan(int T, int M, int d, bool debias, bool ref_iter, size_t lds_cap, bool allow_single,
               MeshArgs& A, size_t& lds_bytes, int* blocks) {
    std::memset(&A, 0, sizeof(A));
    lds_bytes = 0;
    *blocks = 0;
    const int G = std::max((T + kMeshRows - 1) / kMeshRows, (M + kMeshRows - 1) / kMeshRows);
    if (G < (allow_single ? 1 : 2) || G > kMeshMaxBlocks) return false;
    // the words one thread gathers in a half-iteration
    const int gmax = std::max(M + (debias ? T : 0), T + (ref_iter ? M : 0));
    if (gmax > kMeshGatherPerThread * kMeshThreads) return false;
    A.T = T;
    A.M = M;
    A.debias = debias;
    A.ref_iter = ref_iter;
    A.xr = (T + G - 1) / G;
    A.yr = (M + G - 1) / G;
    int r4 = 0;
    A.o_rf = r4; r4 += T;
    A.o_rg = r4; r4 += M;
    A.o_rp = r4; r4 += debias ? T : 0;
    A.o_rq = r4; r4 += ref_iter ? M : 0;
    int off = 4 * r4;
    auto take = [&](int n) {
        const int o = off;
        off += n;
        return o;
    };
    // own rows only
    A.o_f = take(A.xr);
    A.o_g = take(A.yr);
    A.o_p = take(debias ? A.xr : 0);
    A.o_q = take(ref_iter ? A.yr : 0);
    A.o_lb = take(M);
    auto mk = [&](int yside, int keys, int qrec, int krec, int qpot, int avg) {
        MeshJob j;
        std::memset(&j, 0, sizeof(j));
        j.yside = yside; j.keys = keys; j.qrec = qrec; j.krec = krec; j.qpot = qpot; j.avg = avg;
        return j;
    };
    A.njobs[0] = A.njobs[1] = 0;
    A.job[0][A.njobs[0]++] = mk(0, M, A.o_rf, A.o_rg, A.o_f, 0);
    if (debias) A.job[0][A.njobs[0]++] = mk(0, T, A.o_rf, A.o_rp, A.o_p, 1);
    A.job[1][A.njobs[1]++] = mk(1, T, A.o_rg, A.o_rf, A.o_g, 0);
    if (ref_iter) A.job[1][A.njobs[1]++] = mk(1, M, A.o_rg, A.o_rq, A.o_q, 1);
    // gathers: half 0 needs g and p as the iteration starts; half 1 the new f and q
    auto gt = [&](int n, int rec, int lw, int lag) {
        MeshGather g;
        std::memset(&g, 0, sizeof(g));
        g.n = n; g.rec = rec; g.lw = lw; g.lag = lag;
        return g;
    };
    A.ngat[0] = A.ngat[1] = 0;
    A.gat[0][A.ngat[0]++] = gt(M, A.o_rg, A.o_lb, 0);
    if (debias) A.gat[0][A.ngat[0]++] = gt(T, A.o_rp, -1, 0);
    A.gat[1][A.ngat[1]++] = gt(T, A.o_rf, -1, 1);
    if (ref_iter) A.gat[1][A.ngat[1]++] = gt(M, A.o_rq, A.o_lb, 0);

    // Key ranges: each job gets a share of the 16 waves' tasks in proportion to
    // its keys (at least 16 keys per range); a few multiples of 16 tasks are
    // tried and the one with the least modelled time per SIMD kept (a wave's
    // pass over one key: d + 2 VALU instructions and one exp; a task's set-up).
    const double c_key = 2.0 * (d + 2) + 8.0, c_task = 160.0;
    double est = 0.0;
    int ntask_max = 0;
    for (int h = 0; h < 2; ++h) {
        double ktot = 0.0;
        for (int j = 0; j < A.njobs[h]; ++j) ktot += A.job[h][j].keys;
        double best = 0.0;
        int best_sp[2] = {1, 1};
        for (int mult = 1; mult <= 4; mult *= 2) {
            int sp[2] = {1, 1}, kps[2] = {1, 1}, t = 0;
            double simd[4] = {0.0, 0.0, 0.0, 0.0};
            for (int j = 0; j < A.njobs[h]; ++j) {
                const int keys = A.job[h][j].keys;
                const int cap = std::max(1, (keys + 15) / 16);
                sp[j] = std::min(cap, std::max(1, (int)std::lround(kMeshWaves * mult * keys / ktot)));
                kps[j] = (keys + sp[j] - 1) / sp[j];
                sp[j] = (keys + kps[j] - 1) / kps[j];
                for (int u = 0; u < sp[j]; ++u) {
                    const int k0 = std::min(keys, u * kps[j]);
                    const int nk = std::min(keys, k0 + kps[j]) - k0;
                    simd[(t + u) % 4] += c_task + nk * c_key;
                }
                t += sp[j];
            }
            const double cyc = std::max(std::max(simd[0], simd[1]), std::max(simd[2], simd[3]));
            if (mult == 1 || cyc < best) {
                best = cyc;
                best_sp[0] = sp[0];
                best_sp[1] = sp[1];
            }
        }
        int t = 0;
        for (int j = 0; j < A.njobs[h]; ++j) {
            MeshJob& J = A.job[h][j];
            J.kps = (J.keys + best_sp[j] - 1) / best_sp[j];
            J.splits = (J.keys + J.kps - 1) / J.kps;
            J.task0 = t;
            t += J.splits;
        }
        A.ntasks[h] = t;
        ntask_max = std::max(ntask_max, t);
        est += best;
    }
    A.ntask_max = ntask_max;
    A.o_ps = take(64 * ntask_max);
    A.o_pm = take(64 * ntask_max);
    A.est_cycles = est;
    lds_bytes = (size_t)off * sizeof(float);
    if (lds_bytes > lds_cap) return false;
    *blocks = G;
    return true;
}

hipError_t ensure_dynamic_lds(const void* fn, size_t bytes) {
    if (bytes <= (size_t(64) << 10)) return hipSuccess;
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, size_t> set;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    size_t& cur = set[std::make_pair(dev, fn)];
    if (bytes <= cur) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) cur = bytes;
    return e;
}

static const void* mesh_kernel(int d, bool batch) {
    if (batch)
        return d == 2 ? reinterpret_cast<const void*>(&k_mesh_batch<2>)
                      : reinterpret_cast<const void*>(&k_mesh_batch<3>);
    return d == 2 ? reinterpret_cast<const void*>(&k_mesh<2>)
                  : reinterpret_cast<const void*>(&k_mesh<3>);
}

int mesh_resident_blocks(int d, size_t lds_bytes, bool batch) {
    static std::mutex mu;
    static std::map<std::pair<int, std::pair<int, size_t>>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const auto key = std::make_pair(dev * 2 + (batch ? 1 : 0), std::make_pair(d, lds_bytes));
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    const void* fn = mesh_kernel(d, batch);
    if (ensure_dynamic_lds(fn, lds_bytes) != hipSuccess)
        per_cu = 0;
    else if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kMeshThreads, lds_bytes) !=
             hipSuccess)
        per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    const int n = std::max(0, per_cu) * std::max(0, cus);
    cache.emplace(key, n);
    return n;
}

hipError_t launch_mesh(int d, const MeshArgs& A, size_t lds_bytes, int blocks, hipStream_t s) {
    hipEvent_t e0, e1;
    void* tok = profile_kernel_begin(&e0, &e1);
    const double pairs = (double)A.iters * ((double)A.T * A.M * 2 + (A.debias ? (double)A.T * A.T : 0.0) +
                                            (A.ref_iter ? (double)A.M * A.M : 0.0));
    {
        const hipError_t e = ensure_dynamic_lds(mesh_kernel(d, false), lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (d == 2) {
        if (e0) hipExtLaunchKernelGGL((k_mesh<2>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, e0, e1, 0, A);
        else hipLaunchKernelGGL((k_mesh<2>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, A);
    } else {
        if (e0) hipExtLaunchKernelGGL((k_mesh<3>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, e0, e1, 0, A);
        else hipLaunchKernelGGL((k_mesh<3>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, A);
    }
    const hipError_t e = hipGetLastError();
    // kind 40/41: a multi-workgroup exchange solve (safe / lagged from its first iteration)
    profile_kernel_end(tok, 40 + A.lagged0, 0, 0, blocks, pairs);
    return e;
}

hipError_t launch_mesh_batch(int d, const MeshArgs* tab, const int* blk_end, int nprob,
                             size_t lds_bytes, int blocks, double pairs, hipStream_t s) {
    hipEvent_t e0, e1;
    void* tok = profile_kernel_begin(&e0, &e1);
    {
        // set when the batch was planned (so not during a graph capture of the run)
        const hipError_t e = ensure_dynamic_lds(mesh_kernel(d, true), lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (d == 2) {
        if (e0) hipExtLaunchKernelGGL((k_mesh_batch<2>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, e0, e1, 0, tab, blk_end, nprob);
        else hipLaunchKernelGGL((k_mesh_batch<2>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, tab, blk_end, nprob);
    } else {
        if (e0) hipExtLaunchKernelGGL((k_mesh_batch<3>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, e0, e1, 0, tab, blk_end, nprob);
        else hipLaunchKernelGGL((k_mesh_batch<3>), dim3(blocks), dim3(kMeshThreads), lds_bytes, s, tab, blk_end, nprob);
    }
    const hipError_t e = hipGetLastError();
    // kind 42: the exchange solve of a whole batch in one launch
    profile_kernel_end(tok, 42, 0, 0, blocks, pairs);
    return e;
}

}  // namespace ct
