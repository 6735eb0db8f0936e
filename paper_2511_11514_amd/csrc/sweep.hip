// The per-problem sweep kernel: one or two soft-min jobs per launch, each split
// into (query block x key range) work units; see sweep_device.h.
#include <hip/hip_ext.h>

#include <algorithm>

#include "ct_internal.h"
#include "sweep_device.h"

namespace ct {

template <int D, int R, int WS, bool LAGGED, bool BARY, bool SEP, bool EXP = false>
__global__ __launch_bounds__(kBlock) void k_sweep(Launch L) {
    __shared__ SweepSmem<D, R> sm;
    const int bid = (int)blockIdx.x;
    int j = 0;
    while (j + 1 < L.njobs && bid >= L.blk_end[j]) ++j;
    const Job& J = L.job[j];
    const int local = bid - (j ? L.blk_end[j - 1] : 0);
    const int qb = local % J.nqb;
    const int split = local / J.nqb;
    sweep_unit<D, R, WS, LAGGED, BARY, SEP, EXP>(J, qb, split, L.kappa, L.inv_kappa,
                                                 L.inv_sqrt_kappa, sm);
}

// Merge kernel of the separate-merge mode: blocks of kMergeRows query rows per job
// (jobs with a single split were finished by the sweep itself).
template <int D, bool LAGGED, bool BARY>
__global__ __launch_bounds__(kBlock) void k_merge(Launch L, int R, int WS) {
    const int bid = (int)blockIdx.x;
    int j = 0, start = 0;
    for (;;) {
        const Job& Jj = L.job[j];
        const int nb = Jj.splits > 1 ? (Jj.nq + kMergeRows - 1) / kMergeRows : 0;
        if (bid < start + nb || j + 1 == L.njobs) break;
        start += nb;
        ++j;
    }
    const Job& J = L.job[j];
    const int nqpad = J.nqb * 64 * R * (4 / WS);
    merge_block<D, LAGGED, BARY>(J, (bid - start) * kMergeRows, nqpad, L.kappa, L.inv_kappa,
                                 L.inv_sqrt_kappa);
}

int plan_job(Job& j, const Schedule& s) {
    const int qpb = 64 * s.R * (4 / s.WS);
    j.nkpad = pad_keys(j.nk);
    j.nqb = (j.nq + qpb - 1) / qpb;
    const int target = s.blocks_per_cu * kNumCU;
    const int want = std::max(1, (target + j.nqb - 1) / j.nqb);
    // at least 64 keys per wave
    const int unit = 64 * s.WS;
    const int max_splits = std::max(1, j.nkpad / unit);
    int splits = std::min(want, max_splits);
    int kps = (j.nkpad + splits - 1) / splits;
    const int gran = kKeyPad * s.WS;
    kps = (kps + gran - 1) / gran * gran;
    splits = (j.nkpad + kps - 1) / kps;
    j.splits = splits;
    j.kps = kps;
    return j.nqb * splits;
}

size_t job_part_floats(int d, int nq, int nk, const Schedule& s) {
    Job j{};
    j.nq = nq;
    j.nk = nk;
    plan_job(j, s);
    if (j.splits <= 1) return 0;
    return (size_t)(2 + d) * j.splits * (size_t)j.nqb * 64 * s.R * (4 / s.WS);
}

int schedule_candidates(Schedule* out, int max) {
    static const int Rs[] = {1, 2, 4, 8};
    static const int WSs[] = {1, 2, 4};
    static const int Bs[] = {1, 2, 4, 8, 16};
    int n = 0;
    for (int sep = 0; sep < 2; ++sep)
        for (int R : Rs)
            for (int ws : WSs)
                for (int b : Bs)
                    if (n < max) out[n++] = Schedule{R, ws, b, sep};
    return n;
}

size_t job_part_floats_max(int d, int nq, int nk) {
    Schedule c[kMaxCandidates];
    const int n = schedule_candidates(c, kMaxCandidates);
    size_t m = 0;
    for (int i = 0; i < n; ++i) m = std::max(m, job_part_floats(d, nq, nk, c[i]));
    return m;
}

size_t job_tickets_max(int nq) { return (size_t)(nq + 63) / 64; }

// Launch a kernel; with profiling events, through hipExtLaunchKernelGGL so that
// the events carry the kernel's own start and end.
template <typename K, typename... A>
static void launch_k(K kernel, int nb, hipStream_t s, hipEvent_t e0, hipEvent_t e1, A... args) {
    if (e0)
        hipExtLaunchKernelGGL(kernel, dim3(nb), dim3(kBlock), 0, s, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, dim3(nb), dim3(kBlock), 0, s, args...);
}

template <int D, int R, int WS, bool SEP>
static hipError_t launch_drws(bool lagged, bool bary, const Launch& L, int nb, hipStream_t s,
                              hipEvent_t e0, hipEvent_t e1) {
    if (lagged) {
        if (bary) launch_k(k_sweep<D, R, WS, true, true, SEP>, nb, s, e0, e1, L);
        else if (L.expanded) launch_k(k_sweep<D, R, WS, true, false, SEP, true>, nb, s, e0, e1, L);
        else launch_k(k_sweep<D, R, WS, true, false, SEP>, nb, s, e0, e1, L);
    } else {
        if (bary) launch_k(k_sweep<D, R, WS, false, true, SEP>, nb, s, e0, e1, L);
        else launch_k(k_sweep<D, R, WS, false, false, SEP>, nb, s, e0, e1, L);
    }
    return hipGetLastError();
}

template <int D, int R, int WS>
static hipError_t launch_drw(bool sep, bool lagged, bool bary, const Launch& L, int nb,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return sep ? launch_drws<D, R, WS, true>(lagged, bary, L, nb, s, e0, e1)
               : launch_drws<D, R, WS, false>(lagged, bary, L, nb, s, e0, e1);
}

static int merge_blocks(const Launch& L) {
    int nb = 0;
    for (int j = 0; j < L.njobs; ++j)
        if (L.job[j].splits > 1) nb += (L.job[j].nq + kMergeRows - 1) / kMergeRows;
    return nb;
}

template <int D>
static hipError_t launch_merge(int R, int WS, bool lagged, bool bary, const Launch& L, int nb,
                               hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (lagged) {
        if (bary) launch_k(k_merge<D, true, true>, nb, s, e0, e1, L, R, WS);
        else launch_k(k_merge<D, true, false>, nb, s, e0, e1, L, R, WS);
    } else {
        if (bary) launch_k(k_merge<D, false, true>, nb, s, e0, e1, L, R, WS);
        else launch_k(k_merge<D, false, false>, nb, s, e0, e1, L, R, WS);
    }
    return hipGetLastError();
}

template <int D, int R>
static hipError_t launch_dr(int WS, bool sep, bool lagged, bool bary, const Launch& L, int nb,
                            hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (WS) {
        case 1: return launch_drw<D, R, 1>(sep, lagged, bary, L, nb, s, e0, e1);
        case 2: return launch_drw<D, R, 2>(sep, lagged, bary, L, nb, s, e0, e1);
        default: return launch_drw<D, R, 4>(sep, lagged, bary, L, nb, s, e0, e1);
    }
}

template <int D>
static hipError_t launch_d(const Schedule& sc, bool lagged, bool bary, const Launch& L, int nb,
                           hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const bool sep = sc.sep != 0;
    switch (sc.R) {
        case 1: return launch_dr<D, 1>(sc.WS, sep, lagged, bary, L, nb, s, e0, e1);
        case 2: return launch_dr<D, 2>(sc.WS, sep, lagged, bary, L, nb, s, e0, e1);
        case 4: return launch_dr<D, 4>(sc.WS, sep, lagged, bary, L, nb, s, e0, e1);
        default: return launch_dr<D, 8>(sc.WS, sep, lagged, bary, L, nb, s, e0, e1);
    }
}

// One sweep: the sweep kernel, then (separate-merge schedules) the merge kernel.
// With profiling on, each kernel gets its own event pair stamped with the
// kernel's start and end: kind4[0] is 0/1 for a safe/lagged sweep and 10/11 for
// its merge.
hipError_t launch_sweep(int d, const Schedule& sc, bool lagged, bool bary, const Launch& L,
                        int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    double pairs = 0.0;
    for (int j = 0; j < L.njobs; ++j) pairs += (double)L.job[j].nq * L.job[j].nk;
    // code: R, WS and merge kind of the schedule; +1000 for the expanded form
    const int code = sc.R * 100 + sc.WS * 10 + sc.sep + (lagged && !bary && L.expanded ? 1000 : 0);
    hipEvent_t e0, e1;
    void* tok = profile_kernel_begin(&e0, &e1);
    hipError_t e = d == 2 ? launch_d<2>(sc, lagged, bary, L, nblocks, s, e0, e1)
                          : launch_d<3>(sc, lagged, bary, L, nblocks, s, e0, e1);
    profile_kernel_end(tok, lagged, bary, code, nblocks, pairs);
    if (e != hipSuccess || !sc.sep) return e;
    const int nm = merge_blocks(L);
    if (nm == 0) return hipSuccess;
    tok = profile_kernel_begin(&e0, &e1);
    e = d == 2 ? launch_merge<2>(sc.R, sc.WS, lagged, bary, L, nm, s, e0, e1)
               : launch_merge<3>(sc.R, sc.WS, lagged, bary, L, nm, s, e0, e1);
    profile_kernel_end(tok, 10 + lagged, bary, code, 0, 0.0);
    return e;
}

}  // namespace ct
