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
// CT_E_CAPTURE (with a message naming `what`) if `st` is being captured into a graph.
ct_status refuse_capture(hipStream_t st, const char* what);

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
//   out_i = -(1/kappa) log2 sum_j 2^(h_j - |x'_i - y'_j|^2)
// where coordinates are pre-scaled by sqrt(kappa), kappa = log2(e)/eps, and
// h_j = log2(mass_j) + kappa * potential_j is the key's log-weight term.
// Key records are float4 (x', y', h, 0) for d = 2 and (x', y', z', h) for d = 3,
// padded with h = -inf records up to nkpad (a multiple of kKeyPad).
constexpr int kKeyPad = 32;
// Query rows per block of the separate merge kernels (one per lane of a wave;
// the block's four waves share the splits).
constexpr int kMergeRows = 64;

struct Job {
    const float4* qrec;    // [nq] pre-scaled query coordinates (never written)
    const float* qpot;     // [nq] the query points' current potential (shift / averaging)
    const float* qlog2w;   // [nq] log2 mass of the query points, or null: qlog2w_s
    float qlog2w_s;
    int self_avg;          // 1: out = (old + T)/2 (self problems), 0: out = T
    const float4* krec;    // [nkpad] key records
    int nq, nk, nkpad;
    int nqb, splits, kps;  // query blocks, key splits, keys per split
    float* part;           // [(2 + D) * splits * nqpad] partials (shift, sum, offsets)
    unsigned* ticket;      // [nqb] arrival counters (zero between launches)
    float* out_pot;        // [nq] new potential (may alias qpot)
    float4* out_rec;       // [nq] records of the query points as keys of a later sweep: h written
    float* out_bary;       // [nq][D] mean offset under the row plan (unscaled), or null
    unsigned* rescued;     // counter of rows recomputed with a tracked maximum
};

constexpr int kMaxJobs = 4;

struct Launch {
    Job job[kMaxJobs];
    int blk_end[kMaxJobs]; // job j owns blocks [blk_end[j-1], blk_end[j])
    int njobs;
    int expanded;          // 1: lagged sweeps without offsets use the expanded pair form
    float kappa, inv_kappa, inv_sqrt_kappa;
};

struct Schedule {
    int R;                 // queries per lane (1, 2, 4, 8)
    int WS;                // waves of a block splitting the keys (1, 2, 4)
    int blocks_per_cu;     // target blocks per CU per job
    int sep;               // 1: key splits merged by a separate kernel, 0: by the last block
};

inline int pad_keys(int n) { return (n + kKeyPad - 1) / kKeyPad * kKeyPad; }

// Fill nqb/splits/kps of `j` for the schedule; returns the number of blocks.
int plan_job(Job& j, const Schedule& s);
// Floats of partial storage a job needs under this schedule.
size_t job_part_floats(int d, int nq, int nk, const Schedule& s);
// Worst case over every schedule the tuner may pick.
size_t job_part_floats_max(int d, int nq, int nk);
size_t job_tickets_max(int nq);
// Candidate schedules of the tuner.
constexpr int kMaxCandidates = 128;
int schedule_candidates(Schedule* out, int max);

// Launch one sweep kernel (one or two jobs).
hipError_t launch_sweep(int d, const Schedule& sc, bool lagged, bool bary, const Launch& L,
                        int nblocks, hipStream_t s);

// Lockstep launches over a job table in device memory (the batched path): job j
// owns sweep blocks [blk_end[j-1], blk_end[j]) and merge blocks
// [mrg_end[j-1], mrg_end[j]) (none when it has a single key split).
struct TabLaunch {
    const Job* jobs;
    const int* blk_end;
    const int* mrg_end;
    int njobs;
    int nblocks, nmerge;
    int expanded;          // 1: lagged sweeps without offsets use the expanded pair form
    float kappa, inv_kappa, inv_sqrt_kappa;
};
// Plan nqb/splits/kps of `j` so that one block sweeps about `pairs_per_block` pairs.
int plan_job_target(Job& j, const Schedule& s, double pairs_per_block);
// Sweep kernel (separate-merge mode) then, if any job is split, the merge kernel.
hipError_t launch_tab(int d, const Schedule& sc, bool lagged, bool bary, const TabLaunch& L,
                      hipStream_t s);

// Fused solve of one small problem: all K iterations in one launch of co-resident
// blocks, a grid-wide barrier after each half-iteration.  Half-iteration 0 holds
// the f update and the trajectory self update p, half-iteration 1 the g update and
// the reference self update q (the self chains are independent of the cross one,
// so each rides in the half that balances the work).  The self jobs swap their
// ping-pong record arrays every iteration, hence one job set per parity.
struct FusedPhase {
    Job job[2];
    int unit_end[2];       // job j owns units [unit_end[j-1], unit_end[j])
    int njobs;             // 1 or 2
};
struct FusedLaunch {
    FusedPhase ph[2][2];   // [iteration parity][half]
    int iters;
    int lagged0;           // 1: the first iteration already has a usable shift (warm start)
    int safe_only;         // 1: every sweep tracks its maximum
    unsigned* bar;         // [kFusedBarWords] barrier words (zero at launch): per group of
                           // kFusedGroup blocks an arrival count and a release word, one
                           // arrival count of the groups; each on its own 128-byte line
    unsigned* expired;     // set when a barrier wait gave up (zero at launch)
    unsigned wait_polls;   // polls of the arrival counter before a wait gives up
    unsigned target_extra; // 0; 1 makes every wait unsatisfiable (tests of the give-up path)
    float kappa, inv_kappa, inv_sqrt_kappa;
};
// Schedule of the fused kernel: R = 1 query per lane, the keys split across the
// four waves of a block (64 queries per block).
constexpr int kFusedR = 1;
constexpr int kFusedWS = 4;
// Barrier layout: blocks form groups of kFusedGroup; a block arrives at its group's
// counter, the group's last arrival at the top counter, and the groups' last arrivals
// release their groups.  At most kFusedMaxGrid blocks.
constexpr int kFusedGroup = 16;
constexpr int kFusedMaxGrid = 2048;
constexpr int kFusedMaxGroups = kFusedMaxGrid / kFusedGroup;
constexpr int kFusedLine = 32;   // words per counter (one 128-byte line each)
constexpr int kFusedBarWords = (2 * kFusedMaxGroups + 1) * kFusedLine;
// Blocks of the fused kernel that can be resident at once on the current device
// (0 if the occupancy query fails).
int fused_resident_blocks(int d);
hipError_t launch_fused(int d, const FusedLaunch& L, int nblocks, hipStream_t s);

// One-workgroup solve of a small problem with everything in LDS (tiny.hip).
constexpr int kTinyThreads = 1024;                 // 16 waves
constexpr int kTinyWaves = kTinyThreads / 64;
constexpr size_t kTinyMaxLds = size_t(160) << 10;  // bytes of LDS the solve may take (also
                                                   // capped by the device's per-block limit)
// One soft-min job of a half-iteration.  Offsets are in float4 units for record
// arrays and in float units for everything else.
struct TinyJob {
    int rows, keys;        // query rows, key points
    int qrec, krec;        // record arrays of the rows / keys ([2][n] ping-pong for self jobs)
    int out_rec;           // record array whose .w takes the rows' new key terms
    int qnorm;             // |q'|^2 of the rows
    int qpot;              // current potential of the rows (shift, averaging)
    int qlw;               // log2 mass of the rows, or -1: the constant log2a
    int avg;               // 1: new = (old + T)/2 (self problems; records ping-pong)
    int groups, splits, kps;  // 64R-row groups, key ranges, keys per range
    int task0;             // first task index of the job within its half-iteration
};
struct TinyArgs {
    const float4* cx;      // [T] staged coordinates of x (global)
    const float4* cy;      // [M] staged coordinates of y
    const float* log2b;    // [M]
    float *f, *g, *p, *q;  // [T], [M], [T], [M] starting values in, last iterates out
    float4* xrec_f;        // [T] records of x: h from f written at the end
    float4* yrec_g;        // [M] records of y: h from g
    float4* xrec_p;        // [T] records of x: h from p (the final pass's current array)
    float4* yrec_q;        // [M] records of y: h from q
    unsigned* rescued;
    int T, M, d, iters, lagged0, safe_only, debias, ref_iter;
    int R;                 // query rows per lane
    float kappa, inv_kappa, log2a;
    TinyJob job[2][2];     // [half-iteration][job]
    int njobs[2], ntasks[2];
    // LDS offsets: record arrays (float4 units), then floats
    int o_rf, o_rg, o_rp, o_rq;
    int o_f, o_g, o_p, o_q, o_lb, o_nx, o_ny, o_ps, o_pm;
    int ntask_max;
    double est_cycles;     // the plan's modelled cycles per iteration
};
// Plans the tasks, the rows per lane (r_force: 1, 2 or 4, or 0 for the cost
// model's choice) and the LDS layout (fills everything but the pointers and the
// iteration options); false if no plan fits in lds_cap bytes.
bool tiny_plan(int T, int M, int d, bool debias, bool ref_iter, size_t lds_cap, int r_force,
               TinyArgs& A, size_t& lds_bytes);
hipError_t launch_tiny(int d, const TinyArgs& A, size_t lds_bytes, hipStream_t s);

// Raise a kernel's dynamic-LDS limit on the current device to at least `bytes`
// (beyond the default 64 KiB); never lowers it, so launches planned for larger
// problems stay valid.
hipError_t ensure_dynamic_lds(const void* fn, size_t bytes);

// Several workgroups, each holding every point in LDS and owning at most 64 rows
// of each point set, exchanging their rows' potentials through versioned words
// in global memory instead of grid barriers (mesh.hip).
constexpr int kMeshThreads = 1024;                 // 16 waves
constexpr int kMeshWaves = kMeshThreads / 64;
constexpr int kMeshRows = 64;                      // rows of one point set per block, at most
constexpr int kMeshMaxBlocks = 64;
constexpr int kMeshGatherPerThread = 8;            // words one thread gathers per half-iteration
// One soft-min job of a half-iteration over the block's own rows.  Offsets are
// in float4 units for record arrays and in float units for everything else;
// record arrays are indexed by the global row, potential arrays by the row's
// place among the block's own rows.
struct MeshJob {
    int yside;             // rows of y (g, q) rather than of x (f, p)
    int keys;              // key points
    int qrec, krec;        // record arrays of the rows / keys
    int qpot;              // potential of the block's own rows (from its first own row)
    int avg;               // 1: new = (old + T)/2 (self problems)
    int splits, kps;       // key ranges, keys per range
    int task0;             // first task index of the job within its half-iteration
    unsigned long long* xch;   // [2][rows] versioned words of the rows' new potentials
};
// One potential gathered into the .w of a record array at the start of a
// half-iteration: version = iteration + lag.
struct MeshGather {
    const unsigned long long* xch;   // [2][n]
    int n;                 // points
    int rec;               // record array that takes H = h - |v'|^2 (|v'|^2 from its (2v'))
    int lw;                // log2 mass, or -1: the constant log2a
    int lag;               // 0: the version the iteration starts from, 1: the next one
};
struct MeshArgs {
    const float4* cx;      // [T] staged coordinates of x (global)
    const float4* cy;      // [M] staged coordinates of y
    const float* log2b;    // [M]
    float *f, *g, *p, *q;  // starting values in, last iterates out (own rows of each block)
    float4* xrec_f;        // [T] records of x: h from f written at the end
    float4* yrec_g;        // [M] records of y: h from g
    float4* xrec_p;        // [T] records of x: h from p (the final pass's current array)
    float4* yrec_q;        // [M] records of y: h from q
    unsigned long long *xch_f, *xch_g, *xch_p, *xch_q;   // [2][T], [2][M], [2][T], [2][M]
    unsigned* rescued;
    unsigned* expired;     // set when a gather gave up waiting
    unsigned polls;        // poll bound of one gathered word
    unsigned version_extra;   // added to the awaited versions (0; a test hook makes waits unsatisfiable)
    int T, M, d, iters, lagged0, safe_only, debias, ref_iter;
    int xr, yr;            // own rows per block of x and of y
    float kappa, inv_kappa, log2a;
    MeshJob job[2][2];     // [half-iteration][job]
    int njobs[2], ntasks[2];
    MeshGather gat[2][2];
    int ngat[2];
    // LDS offsets: record arrays (float4 units), then floats
    int o_rf, o_rg, o_rp, o_rq;
    int o_f, o_g, o_p, o_q, o_lb, o_ps, o_pm;
    int ntask_max;
    double est_cycles;     // the plan's modelled cycles per iteration (compute only)
};
// Plans blocks, tasks and the LDS layout (fills everything but the pointers and
// the iteration options); false if the problem needs a single block (unless
// allow_single), more than kMeshMaxBlocks blocks, or more than lds_cap bytes of
// LDS per block.  Returns the grid size in *blocks.
bool mesh_plan(int T, int M, int d, bool debias, bool ref_iter, size_t lds_cap, bool allow_single,
               MeshArgs& A, size_t& lds_bytes, int* blocks);
// Blocks of the exchange kernel (single problem, or the batch kernel) that fit
// on the device at once with this much dynamic LDS each.
int mesh_resident_blocks(int d, size_t lds_bytes, bool batch);
hipError_t launch_mesh(int d, const MeshArgs& A, size_t lds_bytes, int blocks, hipStream_t s);
// All problems of a batch in one launch: tab[p] (device) holds problem p's
// arguments, blk_end[p] (device) the end of its blocks; lds_bytes is the largest
// problem's dynamic LDS.
hipError_t launch_mesh_batch(int d, const MeshArgs* tab, const int* blk_end, int nprob,
                             size_t lds_bytes, int blocks, double pairs, hipStream_t s);

// Per-launch event timing (ct_profile_enable); no-ops when disabled.
bool profiling();
void* profile_begin(hipStream_t s);
void profile_end(void* tok, hipStream_t s, int lagged, int bary, int code, int blocks, double pairs);
// Events for one kernel launched with hipExtLaunchKernelGGL, which stamps them
// with the kernel's own start and end (no dispatch gap): *e0, *e1 stay null when
// profiling is off.  profile_kernel_end stores the record's description.
void* profile_kernel_begin(hipEvent_t* e0, hipEvent_t* e1);
void profile_kernel_end(void* tok, int lagged, int bary, int code, int blocks, double pairs);

// Tuning table lookup (falls back to a size heuristic).
Schedule schedule_for(int d, int64_t nq, int64_t nk);
void tuning_record(int d, int64_t nq, int64_t nk, const Schedule& s, int us);
// Exact lookup by size classes (no fallback).
bool tuning_lookup(int d, int qclass, int kclass, Schedule& out);

}  // namespace ct
