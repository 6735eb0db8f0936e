// Internal declarations shared by the HIP sources of libct.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ct.h"

namespace ct {

// ---------------------------------------------------------------- errors
ct_status fail(ct_status code, const char* fmt, ...);
void clear_error();

#define CT_CHECK_HIP(call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return ::ct::fail(CT_E_HIP, "%s failed: %s", #call,          \
                                                hipGetErrorString(e_));                     \
    } while (0)

// --------------------------------------------------------------- geometry
constexpr int kBlock = 256;      // threads per block (4 wave64s)
constexpr int kTile = 256;       // keys staged in LDS per tile (one per thread)
constexpr int kGroup = 8;        // keys per tracked-maximum group (safe mode)
constexpr int kNumCU = 256;      // MI355X compute units
constexpr int kMaxSplitBlocksPerCU = 16;

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Arena {
    char* base;
    size_t off = 0;
    explicit Arena(void* p) : base(static_cast<char*>(p)) {}
    template <class T>
    T* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// ------------------------------------------------------- sweep job layout
// One "job" is a soft-min sweep of a query point set against a key point set:
//   out_i = -(1/kappa) log2 sum_j 2^(kh_j - |qc_i - kc_j|^2)
// where coordinates are pre-scaled by sqrt(kappa), kappa = log2(e)/eps, and
// kh_j = log2(mass_j) + kappa * potential_j is the key's log-weight term.
struct Job {
    const float4* qc;      // [nq] pre-scaled query coordinates (x', y', z', 0)
    const float* qpot;     // [nq] the query points' current potential (shift / averaging)
    const float* qlog2w;   // [nq] log2 mass of the query points, or null: qlog2w_s
    float qlog2w_s;
    int self_avg;          // 1: out = (old + T)/2 (self problems), 0: out = T
    const float4* kc;      // [nk] pre-scaled key coordinates
    const float* kh;       // [nk] key terms
    int nq, nk;
    int nqb, splits, kps;  // query blocks, key splits, keys per split
    float* part;           // [(2 + D) * splits * nqpad] partial (shift, sum, offsets)
    unsigned* ticket;      // [nqb] arrival counters (zero between launches)
    float* out_pot;        // [nq] new potential (may alias qpot)
    float* out_h;          // [nq] key term of the query points for the next sweep, or null
    float* out_bary;       // [nq][D] mean offset under the row plan (unscaled), or null
    unsigned* rescued;     // counter of rows recomputed with a tracked maximum
};

struct Launch {
    Job job[2];
    int nblk0;             // blocks of job 0; the rest belong to job 1
    float kappa, inv_kappa, inv_sqrt_kappa;
};

struct Schedule {
    int R;                 // queries per lane (1, 2, 4, 8)
    int blocks_per_cu;     // target blocks per CU per job
};

// Fill nqb/splits/kps of `j` for the schedule; returns the number of blocks.
int plan_job(Job& j, int R, int blocks_per_cu);
// Floats of partial storage a job needs under this schedule.
size_t job_part_floats(int d, int nq, int nk, int R, int blocks_per_cu);
// Worst case over every schedule the tuner may pick.
size_t job_part_floats_max(int d, int nq, int nk);
size_t job_tickets_max(int nq);

// Launch one sweep kernel (one or two jobs).
hipError_t launch_sweep(int d, int R, bool lagged, bool bary, const Launch& L, int nblocks,
                        hipStream_t s);

// Tuning table lookup (falls back to a size heuristic).
Schedule schedule_for(int d, int64_t nq, int64_t nk);
void tuning_record(int d, int64_t nq, int64_t nk, int R, int bpc, int us);

}  // namespace ct
