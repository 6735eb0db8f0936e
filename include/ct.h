/*
 * ct.h - C ABI of the coverage-flow library (libct.so).
 *
 * The library evaluates the reference flow that pulls the T samples of a robot
 * trajectory toward a target spatial distribution (Sun, Kwon, Murphey,
 * "Scalable Coverage Trajectory Synthesis on GPUs as Statistical Inference",
 * Sec. II), on one AMD MI355X (gfx950) with hand-written HIP kernels:
 *
 *   ct_sinkhorn_grad          gradient of the debiased Sinkhorn divergence
 *                             (Sec. II-B, eqs. 5-7) w.r.t. the trajectory samples
 *                             and the reference weights, and its value;
 *   ct_status_sync            device-detected conditions of the last gradient call
 *                             (non-finite inputs, rescued rows, convergence);
 *   ct_sinkhorn_grad_batched  the same for many independent problems of uneven
 *                             size (lockstep launches or one persistent kernel);
 *   ct_svgd_grad              Stein variational flow (Sec. II-B, eq. 4) with an
 *                             RBF kernel and an analytic Gaussian-mixture score;
 *   ct_svgd_grad_score        the same flow for any score in device memory;
 *   ct_grid_score, ct_grid_samples  a reference given as a continuous utility on
 *                             a grid (Sec. II-A): its score for the Stein flow,
 *                             its weighted nodes for the Sinkhorn flow;
 *   ct_lqr_track              linear-quadratic flow matching (Sec. II-C, eqs. 8-10),
 *                             a sequential FP64 host solve;
 *   ct_plan                   the outer planning loop (Sec. II-A eqs. 2-3 with
 *                             Sec. II-C): flow on the GPU, LQR on the host;
 *   ct_plan_ensemble          many seeds of that loop in lockstep, their flows
 *                             in one batched launch, the best seed reported.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Point sets are row-major float32 arrays [N][d] (point after point), d = 2 or 3.
 * - Pointers marked "device" are HIP device (or managed) memory; "host" ones are
 *   ordinary host memory.  The caller owns every buffer.  GPU entry points never
 *   allocate: they use the caller's workspace `ws` (device, 256-byte aligned,
 *   at least the size returned by the matching *_workspace_size call).  Its
 *   contents need not be initialised and are clobbered.
 * - GPU entry points are asynchronous on `stream` (a hipStream_t; NULL = the
 *   null stream): they enqueue kernels and return without synchronising, except
 *   ct_sinkhorn_batched_prepare, ct_grid_samples, ct_plan and ct_plan_ensemble,
 *   which are synchronous.  Those, ct_status_sync, ct_autotune_sinkhorn and
 *   ct_probe_alu_rates return CT_E_CAPTURE, enqueueing nothing, when `stream` is
 *   being captured into a graph.  Two calls that share a workspace must be
 *   ordered on one stream.
 * - Arguments are validated on the host before anything is enqueued; an invalid
 *   call returns a negative status, enqueues nothing and leaves a message for
 *   ct_last_error() (per thread).
 * - The arithmetic is float32 on the GPU and float64 on the host (LQR).
 */
#ifndef CT_H
#define CT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ct_status;

#define CT_OK 0
#define CT_WARN_NOT_CONVERGED 1 /* ct_status_sync: column residual above the caller's tolerance */
#define CT_E_ARG (-1)         /* null pointer, out-of-range scalar or bad flag */
#define CT_E_SHAPE (-2)       /* sizes inconsistent or unsupported (d, T, M, B) */
#define CT_E_NONFINITE (-3)   /* ct_status_sync: the device saw non-finite inputs or non-positive
                                 weights, so the last call's outputs are not valid */
#define CT_E_WORKSPACE (-4)   /* ws too small or misaligned */
#define CT_E_HIP (-5)         /* a HIP runtime call failed (message has the HIP error) */
#define CT_E_UNSUPPORTED (-6) /* feature not available for this input */
#define CT_E_CAPTURE (-7)     /* a synchronous entry point was called while its stream is being
                                 captured into a graph (nothing was enqueued) */
#define CT_E_DEVICE (-8)      /* ct_status_sync: a bounded wait inside a kernel (the grid barrier
                                 of the fused solve) gave up, so the last call's outputs are not
                                 valid (they are NaN) */

/* Message of the last failing call on this thread ("" if none). */
const char* ct_last_error(void);
/* Library version string. */
const char* ct_version(void);

/* ------------------------------------------------------------------------- */
/* Sinkhorn divergence gradient (Sec. II-B, eqs. 5-7)                          */
/* ------------------------------------------------------------------------- */

/* Option flags (bitwise or). */
#define CT_DEBIAS 1u      /* S = OT(a,b) - OT(a,a)/2 - OT(b,b)/2 (eq. 6); else S = OT(a,b) */
#define CT_GRAD_W 2u      /* compute dS/dw */
#define CT_VALUE 4u       /* compute S */
#define CT_WARM_START 8u  /* start from the potentials in `pot` instead of zeros */
#define CT_REF_CACHED 16u /* `pot` holds a converged reference self potential q: skip its iterations */
#define CT_SAFE_LSE 32u   /* track the running maximum in every sweep (no lagged shift) */
#define CT_ONE_STREAM 64u /* serialise every sweep on `stream` (default: the self-problem sweeps
                             run on a library-owned auxiliary stream of the current device, forked
                             from and joined back into `stream` with events, so they overlap the
                             cross sweeps; the fork/join is graph-capture compatible) */
#define CT_PERSISTENT 128u /* batched path only: one persistent launch walking a dependency-
                            ordered work list instead of lockstep launches per iteration */
#define CT_FUSED 256u   /* run all K iterations in one launch of co-resident blocks with a
                           grid-wide barrier after each half-iteration (f and p, then g and q),
                           instead of one launch per sweep; meant for small problems (short
                           horizons), whose per-iteration launches are bound by launch latency */
#define CT_UNFUSED 512u /* one launch per sweep (none of CT_FUSED, CT_TINY, CT_MESH) */
#define CT_TINY 2048u   /* run all K iterations in one workgroup with every point and potential
                           in LDS (no synchronisation beyond the workgroup); CT_E_UNSUPPORTED
                           when the problem does not fit in the LDS of one workgroup (about
                           48 to 80 bytes per point of x and y, depending on the self terms). */
#define CT_MESH 4096u   /* run all K iterations in one launch of 2 to 64 workgroups, each with
                           every point in LDS and at most 64 rows of x and of y of its own;
                           the workgroups exchange their rows' new potentials through
                           versioned words in device memory (relaxed device-scope atomics),
                           with no grid barrier; CT_E_UNSUPPORTED when it cannot plan (T and
                           M both at most 64, more than 4096 of either, or the points do not
                           fit in one workgroup's LDS).  Without any of CT_FUSED,
                           CT_UNFUSED, CT_TINY and CT_MESH (at most one may be given) the
                           library picks, by the point pairs of one iteration: the
                           one-workgroup solve up to 4e4, the exchange solve up to 1.5e7 where
                           it plans, else the one-workgroup solve up to 1.5e5, the fused
                           solve up to 1.05e6, and per-sweep launches beyond. */
#define CT_DIFFERENCE 1024u /* per-sweep launches: evaluate the lagged sweeps' exponent in the
                               difference form h_j - |x'_i - y'_j|^2 - shift (d subtractions, d
                               FMAs, one subtraction per pair).  Default: the expanded form
                               around an origin shared by a wave, h_j - |k'|^2 + 2 q'.k'
                               - |q'|^2 - shift with q' = x'_i - o, k' = y'_j - o (d FMAs and
                               one add per pair); likewise the batched lockstep launches.  The
                               extrapolation pass, the first (tracked-maximum) sweep, rescued
                               rows, the fused and one-workgroup solves and the batched
                               persistent kernel always use the difference form. */

typedef struct ct_sinkhorn_opts {
    int32_t d;      /* 2 or 3 */
    int32_t iters;  /* Sinkhorn iterations K >= 0 (0: only the final extrapolation pass) */
    float eps;      /* entropic weight (the paper's omega), > 0, in squared-distance units */
    uint32_t flags; /* CT_* flags above */
} ct_sinkhorn_opts;

/* Workspace bytes needed by ct_sinkhorn_grad for these sizes and options. */
size_t ct_sinkhorn_workspace_size(int64_t T, int64_t M, const ct_sinkhorn_opts* o);

/*
 * Debiased Sinkhorn divergence S between the trajectory samples x_1..x_T (equal
 * masses a_i = 1/T: eq. 1 at equal time steps) and the reference samples
 * y_1..y_M with masses b_j = w_j / sum(w) (eq. 5 with the squared-norm cost and
 * relative-entropy regulariser, eq. 6), solved by log-domain Sinkhorn sweeps:
 * K Gauss-Seidel iterations f <- T_b(g), g <- T_a(f) for the cross problem and
 * K averaged iterations p <- (p + T_a(p))/2, q <- (q + T_b(q))/2 for the self
 * problems, all from zero (or `pot` with CT_WARM_START), followed by one
 * extrapolation pass f+ = T_b(g), p+ = T_a(p), g+ = T_a(f+), q+ = T_b(q), where
 * T_b(g)_i = -eps log sum_j b_j exp((g_j - |x_i - y_j|^2)/eps).
 *
 * Outputs (eq. 7 by the envelope theorem):
 *   grad_x[i] = dS/dx_i = 2 a_i (Ds_i - Dy_i), with Dy_i (Ds_i) the mean of
 *               y_j - x_i (x_k - x_i) under the row-normalised cross (self) plan;
 *               without CT_DEBIAS, -2 a_i Dy_i.  The planner's flow is -T*grad_x.
 *   grad_w[j] = dS/dw_j = (G_j - <b,G>) / sum(w), G = g+ - q+ (g+ without debias).
 *   value     = <a,f+> + <b,g> - (<a,p+> + <a,p>)/2 - (<b,q+> + <b,q>)/2.
 *
 *   x       device [T][d]       trajectory samples
 *   y       device [M][d]       reference samples
 *   w       device [M] or NULL  reference weights > 0 (NULL: all equal)
 *   grad_x  device [T][d]       out
 *   grad_w  device [M] or NULL  out (requires CT_GRAD_W)
 *   value   device [1] or NULL  out (requires CT_VALUE)
 *   pot     device [2T+2M] or NULL  f[T], g[M], p[T], q[M]: last iterates out;
 *                               starting iterates in with CT_WARM_START (and q in
 *                               with CT_REF_CACHED).  Required for those flags.
 *   pot_plus device [2T+2M] or NULL  f+, g+, p+, q+ out (g+, q+ only when
 *                               CT_VALUE or CT_GRAD_W; p+, q+ only with CT_DEBIAS)
 *   aux     device [8] or NULL  out: [0] OT(a,b), [1] OT(a,a), [2] OT(b,b),
 *                               [3] column-marginal L1 residual sum_j |colsum_j - b_j|
 *                               of the plan (f+, g) (entries 0-3 need CT_VALUE or
 *                               CT_GRAD_W, else 0), [4] number of rows whose lagged
 *                               shift was unusable and that were recomputed with a
 *                               tracked maximum, [5] number of non-finite inputs or
 *                               non-positive weights, [6] 1 if a grid barrier of
 *                               the fused solve or a wait of the exchange solve
 *                               gave up (outputs NaN), [7] zero
 * Errors: CT_E_ARG (null x/y/grad_x/ws, eps <= 0 or non-finite, iters < 0, grad_w
 * without CT_GRAD_W, pot missing for CT_WARM_START/CT_REF_CACHED, unknown flag,
 * more than one of CT_FUSED, CT_UNFUSED, CT_TINY and CT_MESH), CT_E_UNSUPPORTED
 * (CT_TINY for a problem that does not fit in one workgroup's LDS, CT_MESH for one it
 * cannot plan),
 * CT_E_SHAPE (d not 2/3, T < 1, M < 1, T or M > 2^30), CT_E_WORKSPACE, CT_E_HIP.
 */
ct_status ct_sinkhorn_grad(const float* x, int64_t T, const float* y, const float* w, int64_t M,
                           const ct_sinkhorn_opts* o, float* grad_x, float* grad_w, float* value,
                           float* pot, float* pot_plus, float* aux, void* ws, size_t ws_bytes,
                           void* stream);

/*
 * Allocation-free variant of ct_sinkhorn_grad, for callers that cannot allocate
 * device memory or create HIP objects around the call (code being captured into
 * a HIP graph, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, definitions, outputs and errors as ct_sinkhorn_grad, minus the
 * workspace: the call uses a static device array of
 * ct_sinkhorn_static_scratch_bytes() bytes (64 MiB) that the library holds on
 * every device it runs on until the process ends.  The first call on a device
 * looks up that array's device address and creates the library's auxiliary
 * stream and two events for that device; later calls create, allocate and free
 * nothing.  The caller still owns x, y, w and every output.
 *   Errors: as ct_sinkhorn_grad; CT_E_WORKSPACE when the problem needs more
 *   scratch than the array holds (ct_sinkhorn_workspace_size(T, M, o) >
 *   ct_sinkhorn_static_scratch_bytes(), e.g. T = 4096 with M = 16384), with
 *   nothing enqueued; CT_E_UNSUPPORTED while ct_profile_enable is on (its
 *   per-launch events would be created by the call).
 *   Every call on one device shares that device's array, and the array keeps
 *   the last call's contents (each call clears what must start at zero): two
 *   calls that may overlap on one device (different streams, or different host
 *   threads) race and give undefined results; order them on one stream.
 */
size_t ct_sinkhorn_static_scratch_bytes(void);
ct_status ct_sinkhorn_grad_static(const float* x, int64_t T, const float* y, const float* w,
                                  int64_t M, const ct_sinkhorn_opts* o, float* grad_x,
                                  float* grad_w, float* value, float* pot, float* pot_plus,
                                  float* aux, void* stream);

/*
 * Status words that the last ct_sinkhorn_grad call on `ws` left in its workspace,
 * read after waiting for `stream` (the one synchronising query of the Sinkhorn
 * path; ct_sinkhorn_grad itself never waits).  The residual is the column
 * marginal error of eq. 5's constraint for the plan of (f+, g),
 * sum_j |sum_i pi_ij - b_j| (aux[3]); it is written only by calls with CT_VALUE
 * or CT_GRAD_W (the pass that yields g+).
 *   ws         device, a workspace last used by ct_sinkhorn_grad (256-byte aligned)
 *   resid_tol  tolerance of the residual, >= 0 (0: no convergence check)
 *   nonfinite  host [1] or NULL  out: non-finite input coordinates plus non-positive
 *              or non-finite weights (the count that aux[5] reports)
 *   rescued    host [1] or NULL  out: rows whose lagged shift was unusable and that
 *              were recomputed with a tracked maximum (aux[4])
 *   resid      host [1] or NULL  out: the residual, NaN when the call computed none
 * Returns CT_E_DEVICE when a grid barrier of the fused solve gave up (its outputs
 * are NaN); else CT_E_NONFINITE when nonfinite > 0; else CT_WARN_NOT_CONVERGED (positive)
 * when resid_tol > 0 and a computed residual exceeds it (or is NaN); else CT_OK.
 * CT_E_ARG for a null ws or a negative tolerance, CT_E_WORKSPACE for a misaligned
 * ws, CT_E_CAPTURE while `stream` is being captured, CT_E_HIP.
 */
ct_status ct_status_sync(const void* ws, float resid_tol, uint32_t* nonfinite, uint32_t* rescued,
                         float* resid, void* stream);

/*
 * Many independent problems b = 0..B-1 of uneven size (the batched form of
 * ct_sinkhorn_grad, same definitions and options for every problem).  Three
 * executions of the K iterations:
 *   exchange (CT_MESH; the default when it applies): one launch for the whole
 *     batch, each problem given the blocks of its exchange solve (see CT_MESH:
 *     every point of the problem in each block's LDS, at most 64 own rows of x and
 *     of y per block, potentials passed between the problem's blocks as versioned
 *     words); it applies when every problem has at most 1.5e7 point pairs per
 *     iteration and fits one workgroup's LDS and all the blocks fit on the device
 *     at once (decided by ct_sinkhorn_batched_prepare; CT_E_UNSUPPORTED there for
 *     CT_MESH when it does not apply);
 *   lockstep (CT_UNFUSED, and the default otherwise): two launches per iteration
 *     (every problem's f and self updates, then every problem's g update) over
 *     job tables prepared in the workspace, each job split over keys so that all
 *     blocks sweep about the same number of pairs;
 *   persistent (CT_PERSISTENT): one kernel that walks a dependency-ordered work
 *     list.
 * The extrapolation pass and the reductions follow as lockstep launches in every
 * execution.
 *   T_off, M_off  host [B+1]  prefix offsets: problem b owns x rows
 *                             T_off[b]..T_off[b+1]-1 and y rows M_off[b]..M_off[b+1]-1
 *                             (every problem needs T_b >= 1, M_b >= 1)
 *   x, y, w, grad_x, grad_w   concatenations in that order (w may be NULL)
 *   value         device [B] or NULL (requires CT_VALUE)
 * Flags: CT_DEBIAS, CT_GRAD_W, CT_VALUE, CT_SAFE_LSE, CT_PERSISTENT, CT_MESH, CT_UNFUSED
 * (at most one of the last three), CT_DIFFERENCE (others:
 * CT_E_ARG).
 * The workspace must first be prepared for this batch (same B, offsets, d, iters,
 * flags) by ct_sinkhorn_batched_prepare, which builds the work list on the host
 * and copies it into `ws`; ct_sinkhorn_grad_batched itself only enqueues kernels
 * (no copies, no host synchronisation), so it may be captured into a graph and
 * replayed as long as the workspace stays prepared.  Returns CT_E_ARG for a
 * workspace not prepared for this batch.  If a wait of the persistent kernel on
 * another problem's progress expires (an internal error, never expected: its
 * work order guarantees progress, and the bound, 2^22 polls of about 0.1 us, only
 * turns such an error into a result instead of a hang), every grad_x, grad_w and
 * value entry of the call is NaN.  The environment variable
 * CT_PERSISTENT_WAIT_POLLS, read at each call, replaces the bound (0: a wait
 * expires at its first unsatisfied poll), to test that path.  The exchange
 * execution's waits are bounded likewise (2^18 polls per word) with the same
 * outcome; CT_MESH_WAIT_POLLS and CT_MESH_UNSATISFIABLE_WAITS, read when the batch
 * is prepared, replace the bound and make every wait unsatisfiable, to test that
 * path.  The exchange execution's tables hold kappa: a call with another eps than
 * the prepared one returns CT_E_ARG.
 */
size_t ct_sinkhorn_batched_workspace_size(int32_t B, const int64_t* T_off, const int64_t* M_off,
                                          const ct_sinkhorn_opts* o);
ct_status ct_sinkhorn_batched_prepare(int32_t B, const int64_t* T_off, const int64_t* M_off,
                                      const ct_sinkhorn_opts* o, void* ws, size_t ws_bytes,
                                      void* stream);
ct_status ct_sinkhorn_grad_batched(int32_t B, const int64_t* T_off, const int64_t* M_off,
                                   const float* x, const float* y, const float* w,
                                   const ct_sinkhorn_opts* o, float* grad_x, float* grad_w,
                                   float* value, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------- */
/* Stein variational flow (Sec. II-B, eq. 4)                                   */
/* ------------------------------------------------------------------------- */

/*
 * Target density: a Gaussian mixture with diagonal covariances, optionally mixed
 * with a uniform density of mass `floor` on the unit box [0,1]^d:
 *   q(x) = (1 - floor) sum_k pi_k N(x; mu_k, diag sigma_k^2) + floor 1[x in [0,1]^d].
 * Only its score grad log q is used (Sec. II-B: the Stein flow needs only the score).
 */
typedef struct ct_gmm {
    int32_t K;            /* components, 1..64 */
    const float* weights; /* device [K]  pi_k > 0 */
    const float* means;   /* device [K][d] */
    const float* sigmas;  /* device [K][d]  > 0 */
    float floor;          /* uniform mass in [0, 1) */
} ct_gmm;

/* Workspace of ct_svgd_grad / ct_svgd_grad_score: O(T) bytes, plus, for 11000 <= T <= 92681
 * (median bandwidth over a sampled bracket), 4 MiB of samples and 4 bytes per 125 pairs for the
 * bracket's candidates; from T = 24576 on also 4 bytes per pair of 64-point groups and another
 * 8 bytes per 125 pairs (each wave of the pass owns a segment of twice its share of the
 * candidates): 245 MB in all at T = 65536 (d = 3), 458 MB at T = 92681. */
size_t ct_svgd_workspace_size(int64_t T, int32_t d);

/*
 * phi_i = 1/T sum_j k_ij [ score(x_j) + (2/h)(x_i - x_j) ],  k_ij = exp(-|x_i - x_j|^2 / h)
 * (eq. 4; the j = i term included).  With h <= 0 the bandwidth is the median
 * heuristic h = med^2 / ln T, med the median of the T(T-1)/2 distances
 * |x_i - x_j| (i < j; mean of the two middle ones for an even count; h = 1 for
 * T = 1), found by an exact radix selection on the device.
 *   x       device [T][d]
 *   q       host struct with device arrays (see ct_gmm)
 *   phi     device [T][d] out
 *   score   device [T][d] or NULL  out: grad log q(x_i)
 *   h_used  device [1] or NULL     out: the bandwidth used
 * Errors: CT_E_ARG (null x/q/phi/ws, K out of range, floor outside [0,1), h not
 * finite), CT_E_SHAPE (d, T < 1 or T > 2^30), CT_E_WORKSPACE, CT_E_HIP.
 */
ct_status ct_svgd_grad(const float* x, int64_t T, int32_t d, const ct_gmm* q, float h, float* phi,
                       float* score, float* h_used, void* ws, size_t ws_bytes, void* stream);

/*
 * The Stein flow phi of ct_svgd_grad for a score the caller supplies (Sec. II-B:
 * the flow uses the target only through grad log q, so q may be unnormalised).
 *   score   device [T][d]  grad log q(x_i), read only
 * Same workspace (ct_svgd_workspace_size), bandwidth rule, outputs and errors as
 * ct_svgd_grad (CT_E_ARG for a null score instead of the mixture checks).  Given
 * the score that ct_svgd_grad computes for a mixture, the result is identical.
 */
ct_status ct_svgd_grad_score(const float* x, int64_t T, int32_t d, const float* score, float h,
                             float* phi, float* h_used, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------- */
/* Continuous-utility references on a grid (Sec. II-A)                        */
/* ------------------------------------------------------------------------- */

/*
 * A utility map: values u_j >= 0 on the nodes of a regular grid over the box
 * [lo, hi] (n[t] >= 2 nodes on axis t; node index j_t at
 * lo_t + j_t (hi_t - lo_t) / (n_t - 1)).  The reference density is proportional
 * to U(x) + floor, with U the multilinear interpolant of the node values at x
 * clamped into the box (constant along an axis outside it).  At most 2^20 nodes
 * per axis and 2^28 in all.
 */
typedef struct ct_grid {
    int32_t n[3];   /* nodes per axis (n[2] unused when d = 2) */
    float lo[3];    /* box lower corner (finite) */
    float hi[3];    /* box upper corner (finite, hi > lo) */
    const float* u; /* device, node values, axis 0 fastest: u[j0 + n0 (j1 + n1 j2)] */
    float floor;    /* additive floor >= 0, in the units of u */
} ct_grid;

/*
 * score[i] = grad log(U + floor) at x_i, in float64 rounded to float32: the
 * gradient of the multilinear piece of the cell holding x_i (a point on a face
 * shared by two cells takes the upper cell, the last cell on the box's upper
 * face); zero along an axis on which x_i lies outside the box; zero where
 * U + floor = 0; NaN for a non-finite x_i.  Scaling u and floor by one constant
 * leaves it unchanged.  Node values are not checked (negative ones give
 * meaningless scores).  No workspace.
 *   x      device [T][d]
 *   g      host struct with a device array
 *   score  device [T][d] out
 * Errors: CT_E_ARG (null x/score/g/u, box not finite or hi <= lo, floor < 0 or not
 * finite), CT_E_SHAPE (d not 2/3, T < 1 or > 2^30, node counts out of range).
 */
ct_status ct_grid_score(const float* x, int64_t T, int32_t d, const ct_grid* g, float* score,
                        void* stream);

/*
 * The utility as weighted reference samples for the Sinkhorn flow: every node
 * with weight (u_j + floor) times its trapezoid-rule volume (the cell volume,
 * halved once for each axis on which the node lies on the box face; the rule is
 * exact for the interpolant's mass), normalised to sum 1 in float64; nodes of
 * zero weight are dropped; order is node order.  Synchronous (the count M is
 * returned on the host).
 *   y   device [N][d] out, N = n0 n1 (n2): the first M rows are written
 *   w   device [N] out: the first M entries are written
 *   M   host [1] out: number of samples
 *   ws  workspace of ct_grid_samples_workspace_size(g, d) bytes
 * Errors: as ct_grid_score, plus CT_E_ARG for null y/w/M/ws, a negative or
 * non-finite node value, or a utility that is zero everywhere (with floor 0).
 */
size_t ct_grid_samples_workspace_size(const ct_grid* g, int32_t d);
ct_status ct_grid_samples(const ct_grid* g, int32_t d, float* y, float* w, int64_t* M, void* ws,
                          size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------- */
/* Linear-quadratic flow matching (Sec. II-C, eqs. 8-10), host FP64            */
/* ------------------------------------------------------------------------- */

/*
 * Forward-Euler discretisation of eqs. 9-10 at step dt:
 *   z_0 = 0,  z_{t+1} = (I + dt A_t) z_t + dt B_t v_t,   t = 0..T-1
 *   minimise sum_t dt |a_t - z_{t+1}|^2_Q + dt |v_t|^2_R
 * solved exactly by the backward Riccati recursion with the affine tracking
 * term and a forward rollout.  Sequential, O(T n^3).
 *   A host [T][n][n]  continuous-time Jacobians df/ds along the trajectory (eq. 8)
 *   B host [T][n][m]  df/du
 *   a host [T][n]     reference flow, the target of z_{t+1}
 *   Q host [n][n], R host [m][m]  symmetric, Q >= 0, R > 0
 *   v host [T][m] out;  z host [T+1][n] out or NULL
 * Errors: CT_E_ARG (null pointers, dt <= 0), CT_E_SHAPE (T < 1, n or m outside
 * 1..8), CT_E_UNSUPPORTED (a Riccati step is not positive definite).
 */
ct_status ct_lqr_track(int64_t T, int32_t n, int32_t m, double dt, const double* A, const double* B,
                       const double* a, const double* Q, const double* R, double* v, double* z);

/* ------------------------------------------------------------------------- */
/* Outer planning loop (Sec. II-A eqs. 2-3, Sec. II-C)                         */
/* ------------------------------------------------------------------------- */

#define CT_DYN_DOUBLE_INTEGRATOR 0 /* state (p, v) in R^{2d}, control acceleration in R^d */
#define CT_DYN_UNICYCLE 1          /* state (p_x, p_y, heading), control (speed, turn rate); d = 2 */
#define CT_FLOW_SINKHORN 0
#define CT_FLOW_SVGD 1
#define CT_FLOW_SVGD_GRID 2        /* Stein flow toward a utility grid (opts.grid) */

typedef struct ct_plan_problem {
    int32_t dynamics; /* CT_DYN_* */
    int32_t d;        /* position dimension (2 or 3; 2 for the unicycle) */
    int64_t T;        /* control steps = trajectory samples */
    double dt;        /* > 0 */
    const double* s0; /* host [n] initial state */
} ct_plan_problem;

typedef struct ct_plan_opts {
    int32_t flow;        /* CT_FLOW_* */
    int32_t outer;       /* outer iterations >= 1 */
    double step;         /* control update u <- u + step v* */
    const double* Q;     /* host [d][d]: weight of the position block */
    const double* R;     /* host [m][m] */
    ct_sinkhorn_opts sk; /* Sinkhorn settings (flow = CT_FLOW_SINKHORN) */
    float svgd_h;        /* Stein bandwidth, <= 0 for the median heuristic */
    const ct_grid* grid; /* Stein target for CT_FLOW_SVGD_GRID, else unused (may be NULL) */
} ct_plan_opts;

size_t ct_plan_workspace_size(const ct_plan_problem* p, const ct_plan_opts* o, int64_t M);

/*
 * Each outer iteration: roll the dynamics forward with Euler steps from s0 under
 * u; take the positions of s_1..s_T as the trajectory samples; evaluate the
 * reference flow on the GPU (Sinkhorn: -T dS/dx_i; Stein: phi_i, with the
 * mixture's score for CT_FLOW_SVGD or the utility grid's (ct_grid_score) for
 * CT_FLOW_SVGD_GRID); linearise the dynamics along (s_t, u_t) (eq. 8); solve
 * ct_lqr_track with the flow as the target of the position block; update
 * u <- u + step v*.  Synchronous.  A utility map reaches the Sinkhorn flow as the
 * samples of ct_grid_samples.
 *   y, w    device reference samples/weights (Sinkhorn flow; w may be NULL)
 *   q       host struct (CT_FLOW_SVGD), else NULL
 *   u       host [T][m] controls, in/out
 *   s       host [T+1][n] out: final rollout (after the last update), or NULL
 *   hist    host [outer] out: S (Sinkhorn) or mean |phi_i| (Stein) at the start
 *           of each outer iteration, or NULL
 */
ct_status ct_plan(const ct_plan_problem* p, const ct_plan_opts* o, const float* y, const float* w,
                  int64_t M, const ct_gmm* q, double* u, double* s, double* hist, void* ws,
                  size_t ws_bytes, void* stream);

/*
 * Seed ensemble.  Different initial controls reach different, equally good
 * optima of the planning problem (Sec. III-C, the results), which several seeds can
 * exploit for robustness.  ct_plan_ensemble runs S planners that share the
 * problem p (dynamics, s0, T, dt), the options o and the reference samples, but
 * start from their own controls, in lockstep: every outer iteration rolls out
 * all seeds on the host, evaluates their S Sinkhorn flows in one persistent
 * launch (ct_sinkhorn_grad_batched, gradient only) and solves the S LQR problems
 * on the host (spread over up to 16 threads; each seed's result does not depend
 * on the thread), exactly as S independent ct_plan calls would.  After the last
 * iteration the divergence of every final trajectory to the reference is
 * evaluated in one more batched launch, and the seed with the smallest is
 * reported.
 *   S      seeds, >= 1 (S*T and S*M at most 2^30)
 *   y, w   device [M][d], [M] or NULL: the shared reference (as in ct_plan)
 *   u      host [S][T][m]  in: initial controls of every seed; out: final controls
 *   s      host [S][T+1][n] or NULL  out: final state trajectories
 *   value  host [S]  out: S(final trajectory of seed b, reference)
 *   best   host [1]  out: index of the smallest value (lowest index on ties)
 * Sinkhorn flow only (CT_E_UNSUPPORTED for the Stein flow, which has no
 * objective to rank seeds by).  Synchronous.  The workspace holds every seed's
 * samples, gradients and a copy of the reference per seed:
 * ct_plan_ensemble_workspace_size(p, o, S, M, w != NULL) bytes.  Errors as
 * ct_plan, plus CT_E_HIP if a batched evaluation returns a non-finite value.
 */
size_t ct_plan_ensemble_workspace_size(const ct_plan_problem* p, const ct_plan_opts* o, int32_t S,
                                       int64_t M, int32_t weighted);
ct_status ct_plan_ensemble(const ct_plan_problem* p, const ct_plan_opts* o, int32_t S,
                           const float* y, const float* w, int64_t M, double* u, double* s,
                           double* value, int32_t* best, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------- */
/* Autotuning of the sweep kernels' tile and split schedule                    */
/* ------------------------------------------------------------------------- */

/*
 * Times the candidate schedules of the Sinkhorn sweep kernel (queries per lane,
 * key-splitting waves per block, blocks per CU, merge by a separate kernel or by
 * the last block) for the three launch sets of this problem shape (cross f, cross g, self p + q) on
 * `stream` (synchronously), and records the fastest of each in the process-wide
 * tuning table, keyed by (d, size class of the query set, size class of the key
 * set).  Later ct_sinkhorn_grad calls of those classes use them.  `ws` must hold
 * ct_sinkhorn_workspace_size(T, M, o) bytes.  Must not be called while `stream`
 * is being captured.
 */
ct_status ct_autotune_sinkhorn(int64_t T, int64_t M, const ct_sinkhorn_opts* o, void* ws,
                               size_t ws_bytes, void* stream);
/* Number of tuned entries, and entry i written to out8 (host, 8 ints) as
 * (d, query-set size class, key-set size class, queries per lane, key-splitting
 * waves per block, blocks per CU, separate merge 0/1, time in microseconds of
 * one sweep); a size class is ceil(log2(n)).  CT_E_ARG for an index out of range
 * or a null out8. */
int32_t ct_tuning_count(void);
ct_status ct_tuning_entry(int32_t i, int32_t* out8);
/* Save / load the tuning table as text, one entry per line with the eight fields
 * of ct_tuning_entry in that order ('#' starts a comment line).  Loading merges
 * into the table; a malformed line fails with CT_E_ARG. */
ct_status ct_tuning_save(const char* path);
ct_status ct_tuning_load(const char* path);
void ct_tuning_clear(void);

/* ------------------------------------------------------------------------- */
/* Launch timing                                                               */
/* ------------------------------------------------------------------------- */

/*
 * While enabled, every sweep kernel of ct_sinkhorn_grad (and the merge kernel
 * after it) is launched with hipExtLaunchKernelGGL and a pair of HIP events that
 * the runtime stamps with the kernel's own start and end on its stream, as is the
 * T x T sum of the Stein flow (kind4[0] = 2, pairs = T^2); the batched launches
 * are bracketed by event records instead.  Two events
 * per launch (do not enable while capturing a graph; the event bookkeeping slows
 * the host enqueue).  Record i gives (kind4 = {0 / 1 for a tracked-maximum /
 * lagged-shift sweep, or 10 / 11 for the merge kernel that follows it; offsets
 * pass 0/1; 100 * queries per lane + 10 * key-splitting waves + separate merge;
 * blocks}, the launch's point pairs (0 for a merge), its elapsed ms);
 * ct_profile_read waits for the record's end event.
 */
ct_status ct_profile_enable(int32_t on);
int32_t ct_profile_count(void);
ct_status ct_profile_read(int32_t i, int32_t* kind4, double* pairs, float* ms);
void ct_profile_clear(void);

/* ------------------------------------------------------------------------- */
/* Issue-rate probe (measurement support for the sweep roofline)                */
/* ------------------------------------------------------------------------- */

/*
 * The sweeps are bound by plain vector-ALU issue: per point pair d subtractions,
 * d FMAs, one more subtraction, one v_exp_f32 and one add.  Public figures give
 * only the packed-FMA peak, so the per-instruction rates are measured here: five
 * timed launches on `stream` (synchronous; not while capturing) of 2048 blocks x
 * 256 threads, each lane running 8 independent chains of 2048 steps.  out6 (host)
 * receives lanes per clock per CU of v_add_f32 [0], v_fma_f32 [1] and v_exp_f32
 * [2]; FMAs per clock per CU of v_mfma_f32_16x16x4f32 [3]; the time of MFMA and
 * exp chains issued by the same waves divided by the sum of their separate times
 * [4] (1: the matrix cores and the vector ALU do not overlap, 0.5: they fully
 * overlap); and the clock used, the device's reported peak, in Hz [5].
 * ws: device scratch of ct_probe_workspace_size() bytes (clobbered).
 */
size_t ct_probe_workspace_size(void);
ct_status ct_probe_alu_rates(double* out6, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CT_H */
