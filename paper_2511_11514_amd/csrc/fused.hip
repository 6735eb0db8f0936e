// Fused solve of one small Sinkhorn problem: the K iterations of the cross and
// self sweeps (Sec. II-B, eq. 5 solved by Sinkhorn's algorithm; eq. 6's self
// terms) in a single launch.
//
// At the paper's short horizons (a few hundred trajectory samples) one
// iteration is a few hundred thousand point pairs, a few microseconds of work
// for the whole GPU, so the per-iteration launches of the general path are
// bound by launch latency, not by arithmetic.  Here every block stays resident
// for the whole solve and walks the same (query block x key split) work units
// as the general path's sweep kernel, with the split partials merged by the last
// block to arrive (arrival tickets); a grid-wide barrier separates the two
// halves of an iteration, because each half reads the potentials the other one
// wrote.
//
// Barrier (grid_barrier below): every block fences its writes and arrives at a
// two-level counter tree in the workspace.  The launch never has more blocks
// than can be resident at once, so every wait ends; the poll count is still
// bounded, and a wait that gives up sets a flag (the outputs are then marked
// invalid and the status query reports it) and lets every later wait through at
// once, so even a broken launch finishes instead of hanging.  A one-block launch
// (small problems) needs no counters at all.
#include <hip/hip_ext.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "ct_internal.h"
#include "sweep_device.h"

namespace ct {

// Barrier number k (1, 2, ...) of the launch.  One block: a block barrier.  Else
// two levels, so that no counter takes more than kFusedGroup (or group-count)
// atomic arrivals per barrier and no word is polled by more than kFusedGroup
// blocks: a block adds an arrival to its group's counter; the group's last
// arrival (the one that sees k * group size - 1 before its add) adds one to the
// top counter, waits until every group has arrived and then writes k into its
// group's release word, which the other blocks of the group wait for.  Counts are
// cumulative over the launch (a block cannot reach barrier k + 1 before every
// block has arrived at k).  Every wait is bounded; a wait that gives up sets
// *expired, and every later wait passes at once.
__device__ __forceinline__ bool wait_at_least(unsigned* w, unsigned target, unsigned* expired,
                                              unsigned polls) {
    unsigned spins = 0;
    while (__hip_atomic_load(w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (spins >= polls ||
            __hip_atomic_load(expired, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
            atomicOr(expired, 1u);
            return false;
        }
        __builtin_amdgcn_s_sleep(4);
        ++spins;
    }
    return true;
}

__device__ __forceinline__ void grid_barrier(const FusedLaunch& L, unsigned k) {
    const unsigned G = gridDim.x;
    if (G == 1) {
        __syncthreads();
        return;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned g = blockIdx.x / kFusedGroup;
        const unsigned ngroups = (G + kFusedGroup - 1) / kFusedGroup;
        const unsigned gsize = min((unsigned)kFusedGroup, G - g * kFusedGroup);
        unsigned* grp = L.bar + g * kFusedLine;
        unsigned* rel = L.bar + (kFusedMaxGroups + g) * kFusedLine;
        unsigned* top = L.bar + 2 * kFusedMaxGroups * kFusedLine;
        const unsigned old = atomicAdd(grp, 1u);
        if (old == k * gsize - 1u) {
            atomicAdd(top, 1u);
            wait_at_least(top, k * ngroups + L.target_extra, L.expired, L.wait_polls);
            __hip_atomic_store(rel, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            wait_at_least(rel, k, L.expired, L.wait_polls);
        }
    }
    __syncthreads();
    __threadfence();
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_fused(FusedLaunch L) {
    __shared__ SweepSmem<D, kFusedR> sm;
    const unsigned G = gridDim.x;
    unsigned nbar = 0;
    for (int k = 0; k < L.iters; ++k) {
        const bool lagged = !L.safe_only && (L.lagged0 || k > 0);
        for (int h = 0; h < 2; ++h) {
            const FusedPhase& P = L.ph[k & 1][h];
            const int units = P.unit_end[P.njobs - 1];
            for (int u = (int)blockIdx.x; u < units; u += (int)G) {
                const int j = (P.njobs > 1 && u >= P.unit_end[0]) ? 1 : 0;
                const Job& J = P.job[j];
                const int local = u - (j ? P.unit_end[0] : 0);
                // the previous unit's LDS (key slots, partials, flags) is free again
                __syncthreads();
                if (lagged)
                    sweep_unit<D, kFusedR, kFusedWS, true, false, false>(
                        J, local % J.nqb, local / J.nqb, L.kappa, L.inv_kappa, L.inv_sqrt_kappa, sm);
                else
                    sweep_unit<D, kFusedR, kFusedWS, false, false, false>(
                        J, local % J.nqb, local / J.nqb, L.kappa, L.inv_kappa, L.inv_sqrt_kappa, sm);
            }
            grid_barrier(L, ++nbar);
        }
    }
}

int fused_resident_blocks(int d) {
    static std::mutex mu;
    static std::map<int, int> cache;   // key: device * 4 + d
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev * 4 + d);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    hipError_t e = d == 2
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<2>, kBlock, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused<3>, kBlock, 0);
    if (e != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int n = std::max(0, per_cu) * std::max(0, cus);
    cache.emplace(dev * 4 + d, n);
    return n;
}

hipError_t launch_fused(int d, const FusedLaunch& L, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    double pairs = 0.0;
    for (int par = 0; par < 2; ++par)
        for (int h = 0; h < 2; ++h)
            for (int j = 0; j < L.ph[par][h].njobs; ++j)
                pairs += (double)L.ph[par][h].job[j].nq * L.ph[par][h].job[j].nk;
    pairs *= 0.5 * L.iters;   // both parities were summed
    hipEvent_t e0, e1;
    void* tok = profile_kernel_begin(&e0, &e1);
    if (d == 2) {
        if (e0) hipExtLaunchKernelGGL(k_fused<2>, dim3(nblocks), dim3(kBlock), 0, s, e0, e1, 0, L);
        else hipLaunchKernelGGL(k_fused<2>, dim3(nblocks), dim3(kBlock), 0, s, L);
    } else {
        if (e0) hipExtLaunchKernelGGL(k_fused<3>, dim3(nblocks), dim3(kBlock), 0, s, e0, e1, 0, L);
        else hipLaunchKernelGGL(k_fused<3>, dim3(nblocks), dim3(kBlock), 0, s, L);
    }
    // kind 20/21: a fused solve (safe / lagged from its first iteration)
    profile_kernel_end(tok, 20 + L.lagged0, 0, kFusedR * 100 + kFusedWS * 10, nblocks, pairs);
    return hipGetLastError();
}

}  // namespace ct
