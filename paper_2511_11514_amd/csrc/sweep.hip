// The per-problem sweep kernel: one or two soft-min jobs per launch, each split
// into (query block x key range) work units; see sweep_device.h.
#include <algorithm>

#include "ct_internal.h"
#include "sweep_device.h"

namespace ct {

template <int D, int R, bool LAGGED, bool BARY>
__global__ __launch_bounds__(kBlock) void k_sweep(Launch L) {
    __shared__ float4 tile[kTile];
    const int bid = (int)blockIdx.x;
    const bool second = bid >= L.nblk0;
    const Job& J = second ? L.job[1] : L.job[0];
    const int local = second ? bid - L.nblk0 : bid;
    const int qb = local % J.nqb;
    const int split = local / J.nqb;
    const int qbase = qb * kBlock * R;
    QueryRegs<D, R> Q;
    init_queries<D, R>(J, qbase, L.kappa, LAGGED, Q);
    const int k0 = split * J.kps;
    const int k1 = min(J.nk, k0 + J.kps);
    sweep_range<D, R, LAGGED, BARY>(J, k0, k1, tile, Q);
    publish_and_merge<D, R, LAGGED, BARY>(J, qb, split, qbase, Q, L.kappa, L.inv_kappa,
                                          L.inv_sqrt_kappa);
}

int plan_job(Job& j, int R, int blocks_per_cu) {
    const int qpb = kBlock * R;
    j.nqb = (j.nq + qpb - 1) / qpb;
    const int target = blocks_per_cu * kNumCU;
    int want = std::max(1, (target + j.nqb - 1) / j.nqb);
    const int max_splits = std::max(1, (j.nk + kTile - 1) / kTile);
    int splits = std::min(want, max_splits);
    int kps = (j.nk + splits - 1) / splits;
    kps = (kps + kGroup - 1) / kGroup * kGroup;
    splits = (j.nk + kps - 1) / kps;
    j.splits = splits;
    j.kps = kps;
    return j.nqb * splits;
}

size_t job_part_floats(int d, int nq, int nk, int R, int blocks_per_cu) {
    Job j{};
    j.nq = nq;
    j.nk = nk;
    plan_job(j, R, blocks_per_cu);
    if (j.splits <= 1) return 0;
    return (size_t)(2 + d) * j.splits * (size_t)j.nqb * kBlock * R;
}

static const int kRs[] = {1, 2, 4, 8};
static const int kBpc[] = {1, 2, 4, 8, 16};

size_t job_part_floats_max(int d, int nq, int nk) {
    size_t m = 0;
    for (int R : kRs)
        for (int b : kBpc) m = std::max(m, job_part_floats(d, nq, nk, R, b));
    return m;
}

size_t job_tickets_max(int nq) { return (size_t)(nq + kBlock - 1) / kBlock; }

template <int D, int R>
static hipError_t launch_dr(bool lagged, bool bary, const Launch& L, int nb, hipStream_t s) {
    if (lagged) {
        if (bary)
            hipLaunchKernelGGL((k_sweep<D, R, true, true>), dim3(nb), dim3(kBlock), 0, s, L);
        else
            hipLaunchKernelGGL((k_sweep<D, R, true, false>), dim3(nb), dim3(kBlock), 0, s, L);
    } else {
        if (bary)
            hipLaunchKernelGGL((k_sweep<D, R, false, true>), dim3(nb), dim3(kBlock), 0, s, L);
        else
            hipLaunchKernelGGL((k_sweep<D, R, false, false>), dim3(nb), dim3(kBlock), 0, s, L);
    }
    return hipGetLastError();
}

template <int D>
static hipError_t launch_d(int R, bool lagged, bool bary, const Launch& L, int nb, hipStream_t s) {
    switch (R) {
        case 1: return launch_dr<D, 1>(lagged, bary, L, nb, s);
        case 2: return launch_dr<D, 2>(lagged, bary, L, nb, s);
        case 4: return launch_dr<D, 4>(lagged, bary, L, nb, s);
        default: return launch_dr<D, 8>(lagged, bary, L, nb, s);
    }
}

hipError_t launch_sweep(int d, int R, bool lagged, bool bary, const Launch& L, int nblocks,
                        hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    return d == 2 ? launch_d<2>(R, lagged, bary, L, nblocks, s)
                  : launch_d<3>(R, lagged, bary, L, nblocks, s);
}

}  // namespace ct
