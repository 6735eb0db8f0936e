// Lockstep sweep launches over a job table in device memory: one launch carries
// the same update of many independent problems (the batched path runs two such
// launches per iteration), each job split over keys so that every block sweeps
// about the same number of pairs; split jobs are merged by a second kernel.
// The per-unit work is sweep_unit / merge_block of sweep_device.h.
#include <algorithm>
#include <cmath>

#include "ct_internal.h"
#include "sweep_device.h"

namespace ct {

// Smallest j with end[j] > b (entries may repeat: jobs without blocks).
__device__ __forceinline__ int owner(const int* end, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (end[mid] > b) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

template <int D, int R, int WS, bool LAGGED, bool BARY, bool EXP = false>
__global__ __launch_bounds__(kBlock) void k_sweep_tab(TabLaunch L) {
    __shared__ SweepSmem<D, R> sm;
    const int bid = (int)blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(owner(L.blk_end, L.njobs, bid));
    const Job J = L.jobs[j];
    const int local = bid - (j ? L.blk_end[j - 1] : 0);
    const int qb = local % J.nqb;
    const int split = local / J.nqb;
    sweep_unit<D, R, WS, LAGGED, BARY, true, EXP>(J, qb, split, L.kappa, L.inv_kappa,
                                                  L.inv_sqrt_kappa, sm);
}

template <int D, bool LAGGED, bool BARY>
__global__ __launch_bounds__(kBlock) void k_merge_tab(TabLaunch L, int qpb) {
    const int bid = (int)blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(owner(L.mrg_end, L.njobs, bid));
    const Job J = L.jobs[j];
    const int q0 = (bid - (j ? L.mrg_end[j - 1] : 0)) * kMergeRows;
    merge_block<D, LAGGED, BARY>(J, q0, J.nqb * qpb, L.kappa, L.inv_kappa, L.inv_sqrt_kappa);
}

int plan_job_target(Job& j, const Schedule& s, double pairs_per_block) {
    const int qpb = 64 * s.R * (4 / s.WS);
    j.nkpad = pad_keys(j.nk);
    j.nqb = (j.nq + qpb - 1) / qpb;
    const double per_qb = (double)qpb * j.nkpad;
    const int want = (int)std::min(1e9, std::ceil(per_qb / std::max(pairs_per_block, 1.0)));
    const int max_splits = std::max(1, j.nkpad / (64 * s.WS));   // at least 64 keys per wave
    int splits = std::max(1, std::min(want, max_splits));
    int kps = (j.nkpad + splits - 1) / splits;
    const int gran = kKeyPad * s.WS;
    kps = (kps + gran - 1) / gran * gran;
    splits = (j.nkpad + kps - 1) / kps;
    j.splits = splits;
    j.kps = kps;
    return j.nqb * splits;
}

template <int D, int R, int WS>
static hipError_t tab_drw(bool lagged, bool bary, const TabLaunch& L, hipStream_t s) {
    const dim3 g(L.nblocks), b(kBlock);
    if (lagged) {
        if (bary) hipLaunchKernelGGL((k_sweep_tab<D, R, WS, true, true>), g, b, 0, s, L);
        else if (L.expanded) hipLaunchKernelGGL((k_sweep_tab<D, R, WS, true, false, true>), g, b, 0, s, L);
        else hipLaunchKernelGGL((k_sweep_tab<D, R, WS, true, false>), g, b, 0, s, L);
    } else {
        if (bary) hipLaunchKernelGGL((k_sweep_tab<D, R, WS, false, true>), g, b, 0, s, L);
        else hipLaunchKernelGGL((k_sweep_tab<D, R, WS, false, false>), g, b, 0, s, L);
    }
    return hipGetLastError();
}

template <int D>
static hipError_t tab_d(const Schedule& sc, bool lagged, bool bary, const TabLaunch& L,
                        hipStream_t s) {
    if (sc.WS == 2) {
        if (sc.R == 1) return tab_drw<D, 1, 2>(lagged, bary, L, s);
        if (sc.R == 2) return tab_drw<D, 2, 2>(lagged, bary, L, s);
        return tab_drw<D, 4, 2>(lagged, bary, L, s);
    }
    if (sc.R == 1) return tab_drw<D, 1, 4>(lagged, bary, L, s);
    if (sc.R == 2) return tab_drw<D, 2, 4>(lagged, bary, L, s);
    return tab_drw<D, 4, 4>(lagged, bary, L, s);
}

template <int D>
static hipError_t tab_merge(int qpb, bool lagged, bool bary, const TabLaunch& L, hipStream_t s) {
    const dim3 g(L.nmerge), b(kBlock);
    if (lagged) {
        if (bary) hipLaunchKernelGGL((k_merge_tab<D, true, true>), g, b, 0, s, L, qpb);
        else hipLaunchKernelGGL((k_merge_tab<D, true, false>), g, b, 0, s, L, qpb);
    } else {
        if (bary) hipLaunchKernelGGL((k_merge_tab<D, false, true>), g, b, 0, s, L, qpb);
        else hipLaunchKernelGGL((k_merge_tab<D, false, false>), g, b, 0, s, L, qpb);
    }
    return hipGetLastError();
}

// Schedules supported by the lockstep launches: R in {1, 2, 4}, WS in {2, 4}
// (other requests fall back to R = 4, WS = 4 inside tab_d).
hipError_t launch_tab(int d, const Schedule& sc, bool lagged, bool bary, const TabLaunch& L,
                      hipStream_t s) {
    if (L.nblocks <= 0) return hipSuccess;
    hipError_t e = d == 2 ? tab_d<2>(sc, lagged, bary, L, s) : tab_d<3>(sc, lagged, bary, L, s);
    if (e != hipSuccess || L.nmerge <= 0) return e;
    const int qpb = 64 * sc.R * (4 / sc.WS);
    return d == 2 ? tab_merge<2>(qpb, lagged, bary, L, s) : tab_merge<3>(qpb, lagged, bary, L, s);
}

}  // namespace ct
