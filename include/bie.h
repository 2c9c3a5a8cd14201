/*
 * bie.h -- C ABI of the MI355X space-time BIEM convolution library.
 *
 * The library evaluates, at every time step n, the space-time convolution of
 * the discretized elastodynamic kernel with the slip-rate history,
 *
 *     T_{i,n} = sum_{m=0}^{M-1} sum_{j=1}^{N} K_{ij,m} D_{j,n-m}        (Eq. 4)
 *
 * for the 2D anti-plane (mode III) problem of Sec. 2.1: N straight boundary
 * elements with piecewise-constant slip rate in space and time, traction
 * collocated at the element midpoints x_i and at t_n = (n + eps_t) dt, and
 * K_{ij,m} the integral of the continuous kernel over (t_{m-1}, t_m).  The
 * slip rate is zero before step 0 (quiescent past).
 *
 * Two forms sit behind the same step/run calls:
 *   - the plain form: the dense N x N x M kernel tensor (bie_build_kernel);
 *   - the FDP=H form of Secs. 3-5 and Apps. B, C.2, E, H: the fast domain
 *     partitioning of lag time into Domain F (wavefronts) and Domain S
 *     (statics plus the 2D transient), a block cluster tree with dense
 *     near-field windows and ACA low-rank far-field blocks, and the averaged-
 *     reduced-time (ART) ring-buffer arithmetic of Eqs. 52, 56 and 59
 *     (bie_compress_fdph).
 *
 * Conventions
 *   - Every function returns an int status: BIE_OK (0) or a negative code.
 *     bie_last_error() returns a message for the last failure on the calling
 *     thread.  No C++ exception crosses the ABI.
 *   - Pointers named *_host are host memory, read during the call only.
 *     Pointers named *_dev are device memory on the current HIP device; the
 *     caller owns them.  `stream` is a hipStream_t passed as void* (NULL =
 *     the default stream).  Step and run calls are asynchronous on `stream`.
 *     An FDP=H operator also launches on a second stream of its own (default
 *     priority), forked from `stream` and joined back to it within every
 *     step or time block, so that its work stays ordered on `stream`.
 *   - The library allocates no device memory.  Building an operator is a
 *     host plan (bie_plan_dense, bie_plan_fdph), for the FDP=H form a window
 *     scan in a caller scratch buffer (bie_plan_windows), then the operator
 *     inside one caller workspace of bie_workspace_size bytes
 *     (bie_build_kernel, bie_compress_fdph).  Every device array the
 *     operator reads or writes lives in that workspace, which the caller
 *     keeps allocated and untouched until bie_destroy.  Scratch and
 *     workspace pointers must be 256-byte aligned.
 *   - An operator is not thread safe; calls on one operator must be ordered
 *     on one stream.  A plan is read-only after bie_plan_windows and may
 *     build several operators.
 *   - Slip-rate and traction arrays are FP64, time-major: D[n][j], T[n][i].
 *   - Timing, probes, exports and debug scans: bie_diag.h.
 */
#ifndef BIE_H
#define BIE_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BIE_OK            0
#define BIE_EINVAL       -1   /* invalid argument or unsupported setting */
#define BIE_ECAUSALITY   -2   /* discretized causality violated (App. D.1) */
#define BIE_ENOMEM       -3   /* host allocation failed */
#define BIE_EHIP         -4   /* a HIP runtime call failed */
#define BIE_ESTATE       -5   /* call not valid in the operator's or plan's state */
#define BIE_EWORKSPACE   -6   /* workspace or scratch null, misaligned or too small */
#define BIE_ENOTCONV     -7   /* ACA+ reached a block's full rank above eps_aca and the
                                 exact fallback of Sec. 6.2 is disabled
                                 (BIE_FLAG_NO_ACA_FALLBACK) */

/* operator kinds */
#define BIE_KIND_DENSE    1
#define BIE_KIND_FDPH     2

/* storage precision of the FDP=H operator */
#define BIE_FP64          0   /* everything in FP64 */
#define BIE_MIXED_FP32    1   /* near windows and low-rank factors stored in FP32,
                                 widened and summed in FP64; FP64 histories,
                                 rings, self terms and accumulators */
#define BIE_MIXED_BF16    2   /* as BIE_MIXED_FP32 with the low-rank factors
                                 stored in BF16 (widened on load) */

/*
 * Problem statement (Sec. 2.1): geometry, medium, time step.
 *   n_elem   N, number of boundary elements
 *   n_lags   M, number of kernel lags kept (= steps of a full run)
 *   xa_host, xb_host   [N][2] end points of each element; the collocation
 *            point is the midpoint and the element normal is the tangent
 *            (xb - xa)/|xb - xa| rotated by +90 degrees; slip is the jump
 *            u(+normal) - u(-normal).
 *   mu, beta shear modulus and S-wave speed
 *   dt       time step; eps_t collocation offset, t_n = (n + eps_t) dt.  The
 *            FDP=H form requires eps_t = 1 (Sec. 4.3).
 *   mode     BIE_MODE_ANTIPLANE (0): one slip component (mode III), T and D
 *            rows hold N values.  BIE_MODE_INPLANE (1): plane strain (P-SV,
 *            the in-plane medium of App. A) on a straight fault, two
 *            components per element, rows hold N pairs (shear slip rate,
 *            opening rate) -> (shear traction, normal traction); on a
 *            straight fault the 2 x 2 kernel is diagonal.  Plain form only.
 *   alpha    P-wave speed (in-plane; > beta), ignored for anti-plane
 */
#define BIE_MODE_ANTIPLANE 0
#define BIE_MODE_INPLANE   1
typedef struct bie_problem {
    int32_t n_elem;
    int32_t n_lags;
    const double *xa_host;
    const double *xb_host;
    double mu;
    double beta;
    double dt;
    double eps_t;
    int32_t mode;           /* BIE_MODE_* */
    int32_t reserved;       /* 0 */
    double alpha;           /* P-wave speed (BIE_MODE_INPLANE) */
} bie_problem;

/*
 * FDP=H parameters.
 *   eta        admissibility diam < eta * dist (Eq. 8)
 *   leaf_size  a block whose receiver or source cluster has at most this
 *              many elements is an inadmissible (near-field) leaf
 *   n_c        2D broadening of Domain F, in steps (Sec. 4.3, App. H)
 *   eps_aca    stopping tolerance of ACA+ (Sec. 6.1.1)
 *   eps_q      relative bound of the static cut-off rule (App. A.1)
 *   eps_st     absolute bound, in units of mu/(2 beta), of the same rule
 *   precision  BIE_FP64, BIE_MIXED_FP32 or BIE_MIXED_BF16
 *   flags      BIE_FLAG_* options
 *   seed       seed of the random reference pivots of ACA+
 *   eps_qtr    relative bound of the transient staircase (with
 *              BIE_FLAG_QUANTIZE_TRANSIENT; the paper runs Quantization with
 *              relative bounds up to 0.1 together with an absolute bound)
 */
typedef struct bie_fdph_params {
    double eta;
    int32_t leaf_size;
    int32_t n_c;
    double eps_aca;
    double eps_q;
    double eps_st;
    int32_t precision;
    int32_t flags;          /* BIE_FLAG_* */
    uint64_t seed;
    double eps_qtr;         /* relative bound of the transient staircase (BIE_FLAG_QUANTIZE_TRANSIENT) */
    int32_t n_rhs;          /* slip-rate histories (scenarios) that share the operator: 1, 2 or 4
                               (0 reads as 1); rows of D and T then hold n_rhs blocks of N values */
    int32_t time_block;     /* steps of a prescribed-slip run (bie_run, bie_run_graph) whose near
                               field shares one pass over the windows: 1 (0 reads as 1) or
                               BIE_TIME_BLOCK; one scenario only */
} bie_fdph_params;

/* Steps of a time block (bie_fdph_params.time_block). */
#define BIE_TIME_BLOCK 16

/* flags of bie_fdph_params:
 * BIE_FLAG_QUANTIZE_TRANSIENT  staircase 2D transient waveform (App. A.1 applied
 *   to h^tr, App. B.3): consecutive lags of h^tr within min(eps_qtr |h^|,
 *   eps_st mu/(2 beta) / |K^tr at the pivot|) of one value share it, and the
 *   step keeps the running sums of the runs (Eq. A.3). */
#define BIE_FLAG_QUANTIZE_TRANSIENT 1
/* BIE_FLAG_NO_ACA_FALLBACK  a block that ACA+ cannot compress to eps_aca
 *   before its full rank makes bie_plan_fdph fail with BIE_ENOTCONV instead
 *   of being kept exactly (the fallback rule of Sec. 6.2). */
#define BIE_FLAG_NO_ACA_FALLBACK 2
/* BIE_FLAG_HOST_ACA  ACA+ runs on the host inside bie_plan_fdph (OpenMP over
 *   blocks) instead of on the device inside bie_plan_windows: for checks of a
 *   plan's factors without a GPU, and as the reference of the device path. */
#define BIE_FLAG_HOST_ACA 4

/* Operator statistics (bie_query). */
typedef struct bie_stats {
    int32_t kind;               /* BIE_KIND_* */
    int32_t n_elem;
    int32_t n_lags;
    int32_t precision;
    int64_t steps_done;         /* steps applied since build/reset */
    int64_t n_adm;              /* admissible leaves */
    int64_t n_inadm;            /* inadmissible leaves */
    int64_t near_pairs;         /* receiver-source pairs in inadmissible leaves */
    int64_t near_lags;          /* sum of the near windows W_ij */
    int64_t rank_sum[3];        /* sum of ranks over admissible leaves: F, S, transient */
    int64_t rank_max[3];
    int64_t aca_fallbacks;      /* blocks kept at full rank */
    int64_t device_bytes;       /* workspace bytes the operator uses */
    double  bytes_per_step;     /* algorithmic bytes of one steady-state step */
    double  near_bytes_per_step;/* of which: near-field windows and histories */
    double  flops_per_step;     /* 2 x multiply-adds of one steady-state step */
    double  setup_seconds;      /* wall time of plan, window scan and build */
    int64_t aca_sweeps;         /* full residual sweeps of ACA+ after its random
                                   references stalled (blocks whose residual sits
                                   in few rows or columns) */
    int64_t scratch_bytes;      /* per-step partial sums (part of the workspace;
                                   the static array of bie_run_static holds them) */
    int64_t aca_host_blocks;    /* blocks that reached the device rank cap of
                                   ACA+ and were factored again on the host */
    double  aca_seconds;        /* time of ACA+: on the device, the kernel's
                                   device time plus the unpacking of its factors
                                   and any host refactoring; on the host, wall time */
    int64_t time_block;         /* steps per pass over the near windows in
                                   bie_run / bie_run_graph (1: none) */
} bie_stats;

typedef struct bie_op bie_op;
typedef struct bie_plan bie_plan;

/*
 * Plan of the plain form (Eq. 4): checks the problem and fixes the layout of
 * the dense N x N x M kernel tensor (FP64).  Host only.
 * Errors: BIE_EINVAL (invalid problem, tensor beyond one dispatch), BIE_ENOMEM.
 */
int bie_plan_dense(const bie_problem *prob, bie_plan **plan_out);

/*
 * Plan of the FDP=H form (Secs. 3-5, Apps. B.1, B.3, C.2, E, H), host only:
 * the cluster tree and block cluster tree, the ART integers and the
 * discretized-causality check (App. D.1), the degenerate waveforms (Eq. 50)
 * and 2D transient waveforms, the ACA+ factors (Sec. 6.1.1, FP64) of the
 * Domain-F amplitude (Eq. 51), Domain-S static and transient matrices of
 * every admissible leaf, the far-field ring layout, and the near-field tiles
 * of the inadmissible leaves.
 *   probs, count  one problem, or `count` independent problems (faults of
 *           any sizes that do not interact) in one operator, each with its
 *           own trees; all must share mu, beta, dt and eps_t.  D and T rows
 *           then hold sum_k n_elem_k values, problem k at offset
 *           sum_{k'<k} n_elem_k'; the lag count is max_k n_lags_k and at a
 *           step n >= n_lags_k problem k's entries of T_n are zero.
 *   params  FDP=H parameters.  n_rhs = 2 or 4 slip-rate histories
 *           (scenarios) on the same fault(s) share the kernels: every row of
 *           D and T holds n_rhs blocks of values (scenario r at r * values),
 *           each scenario keeps its own histories and rings, and the near
 *           field reads each window value once for all of them.
 * The near-field windows W_ij (App. E cut-off) are not known yet: call
 * bie_plan_windows before bie_workspace_size.
 * Errors: BIE_EINVAL, BIE_ECAUSALITY (min over an admissible leaf of
 * dm_i + mbar_j < 1), BIE_ENOTCONV, BIE_ENOMEM.
 */
int bie_plan_fdph(const bie_problem *probs, int32_t count, const bie_fdph_params *params, bie_plan **plan_out);

/* Bytes of device scratch bie_plan_windows needs (0 for a plain plan: the
 * call is then a no-op).  Errors: BIE_EINVAL (null pointer). */
int bie_plan_scratch_size(const bie_plan *plan, int64_t *bytes_out);

/*
 * Scans the near-field windows W_ij of an FDP=H plan on the device: for
 * every near pair, one past the last lag m < M where |K_ij,m - K^S_ij dt|
 * exceeds min(eps_q |K^S_ij dt|, eps_st mu/(2 beta)) (App. E with the
 * cut-off rule of Apps. A.1, H.1), evaluated from the closed-form kernel in
 * FP64.  scratch_dev: device memory of at least bie_plan_scratch_size bytes,
 * 256-byte aligned, free again when the call returns (it blocks).  Completes
 * the plan's layout.  Errors: BIE_EINVAL, BIE_EWORKSPACE, BIE_EHIP.
 */
int bie_plan_windows(bie_plan *plan, void *scratch_dev, int64_t scratch_bytes, void *stream);

/* Bytes of the device workspace an operator of this plan needs.
 * Errors: BIE_EINVAL (null pointer), BIE_ESTATE (FDP=H windows not scanned). */
int bie_workspace_size(const bie_plan *plan, int64_t *bytes_out);

/* Statistics of the operator a plan builds (as bie_query; steps_done 0).
 * Errors: BIE_EINVAL, BIE_ESTATE (FDP=H windows not scanned). */
int bie_plan_query(const bie_plan *plan, bie_stats *stats_out);

/* Frees a plan (host memory only; operators built from it stay valid). */
void bie_plan_free(bie_plan *plan);

/*
 * Plain form (Eq. 4): builds the operator inside ws_dev (at least
 * bie_workspace_size bytes, 256-byte aligned): K_{ij,m} for m < n_lags from
 * the closed-form step response, evaluated on the device.  Blocks until the
 * tensor is built.  Errors: BIE_EINVAL (not a plain plan), BIE_EWORKSPACE,
 * BIE_EHIP.
 */
int bie_build_kernel(const bie_plan *plan, void *ws_dev, int64_t ws_bytes, void *stream, bie_op **op_out);

/*
 * FDP=H form: builds the operator of a plan whose windows were scanned inside
 * ws_dev (at least bie_workspace_size bytes, 256-byte aligned): the factors
 * in the storage precision of params->precision, the waveforms and index
 * lists, the chunk-major near-field windows (filled on the device from the
 * closed form), and the zeroed histories and rings.  Blocks until ready.
 * Errors: BIE_EINVAL (not an FDP=H plan), BIE_ESTATE (windows not scanned),
 * BIE_EWORKSPACE, BIE_EHIP.
 */
int bie_compress_fdph(const bie_plan *plan, void *ws_dev, int64_t ws_bytes, void *stream, bie_op **op_out);

/*
 * One time step: consumes D_n (d_n_dev, N doubles) as the slip rate of the
 * next step n and writes T_n (t_n_dev, N doubles).  Asynchronous.  The plain
 * form keeps convolving the last M lags past step M; an FDP=H operator's
 * runs end at its (largest) lag count M, and later steps are refused.
 * Errors: BIE_EINVAL (null pointer; FDP=H: step n >= M), BIE_ESTATE
 * (operator not built, or a predicted step awaits its commit), BIE_EHIP.
 */
int bie_step(bie_op *op, const double *d_n_dev, double *t_n_dev, void *stream);

/*
 * `steps` consecutive steps: D_dev and T_dev are [steps][N] (time-major).
 * Equivalent to `steps` calls of bie_step.  With time blocks, each whole
 * block of BIE_TIME_BLOCK steps takes its near field in one pass over the
 * windows: the same terms, summed in another order by the matrix-core kernel
 * (results agree with single steps to rounding; bit for bit with the
 * lane-per-lag kernel, for finite slip rates).  Asynchronous.
 * Errors: as bie_step, and BIE_EINVAL for a negative count or (FDP=H) steps
 * past the lag count, checked before any step is issued.
 */
int bie_run(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream);

/*
 * As bie_run, with up to 32 consecutive steps captured as one HIP graph and
 * the graph launched once per 32 steps (a remainder of fewer steps runs as
 * bie_run runs it; time blocks fall at the same steps as in bie_run): the
 * step index lives in a device counter that the last node of every captured
 * step advances, so every launch continues where the previous one stopped.
 * Results are identical to bie_run.  Use for long runs of cheap steps, where per-kernel
 * launch overhead matters.  The graph of a call is kept: a later call with
 * the same D_dev and T_dev from the same step (after bie_reset, say) replays
 * it without capturing again; any other call first waits for it to finish
 * and captures a new one; bie_autotune drops it (it holds the previous
 * launch configuration).  The kernel timer (bie_timing) does not see graph
 * launches.  Asynchronous.
 * Errors: BIE_EINVAL (as bie_run), BIE_ESTATE (operator not built), BIE_EHIP.
 */
int bie_run_graph(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream);

/*
 * For callers that cannot allocate device memory at run time (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): as
 * bie_run, with the per-step partial sums (of the dense lag chunks, or of the
 * near-field work items of the FDP=H form) in a static device array of the
 * library, BIE_STATIC_SCRATCH_BYTES per GPU, held until the process ends,
 * instead of the operator's workspace.  Calls no allocating routine.  Every
 * step writes each partial sum it later reads, so nothing needs clearing.
 * All calls on one GPU share its array: calls that overlap on one GPU (other
 * streams, other threads, other operators) race.  Takes one step per pass
 * (no time blocks): the tractions of bie_run on an operator without time
 * blocks, bit for bit (with time blocks, equal to rounding).
 * Errors: as bie_run, and BIE_EINVAL when the operator's partial sums exceed
 * the array (plain form: ncomp * n_chunks * N doubles; FDP=H: n_rhs times the
 * near-field partial slots; the message gives the size).
 */
#define BIE_STATIC_SCRATCH_BYTES (32ll << 20)
int bie_run_static(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream);

/*
 * Autotuner of the FDP=H near-field kernel: times each launch configuration
 * (source-loop unroll 8 or 16; window loads of 8 or 16 bytes per lane (4 or
 * 8 for FP32 in 64-lag chunks); 4, 3 or 2 workgroups per compute unit; work
 * items in build order, grouped so that items staging the same source
 * histories share one XCD, or largest first) `reps` times on the operator's
 * own data, at a
 * step index with every lag chunk active, and keeps the fastest for the
 * following steps; an operator with time blocks keeps two configurations,
 * both tuned here: that of its time blocks (bie_run, bie_run_graph: the
 * matrix-core or the lane-per-lag kernel), which `out` describes, and that of
 * single steps (bie_step, coupled steps).  Leaves the operator's state
 * unchanged; blocks until done.  Results of later steps are identical for every configuration of
 * one load width; another width, or the matrix-core kernel of time blocks,
 * sums each receiver's lags in another order (the same terms, so they agree
 * to rounding).
 *   out (optional)  the chosen configuration and its time per launch
 * Errors: BIE_EINVAL (not an FDP=H operator, reps < 1), BIE_EHIP.
 */
typedef struct bie_tune {
    int32_t unroll;          /* source-loop unroll of the chosen configuration */
    int32_t lds_pad;         /* unused LDS bytes per workgroup (occupancy cap) */
    int32_t item_order;      /* 0: build order, 1: grouped by sources per XCD,
                                2: largest work items first */
    int32_t candidates;      /* configurations timed */
    int32_t load_bytes;      /* window bytes each lane loads at once (4, 8 or 16) */
    int32_t mfma;            /* 1: the time blocks' near field runs on the matrix
                                cores (16 steps per pass), one lag chunk per work
                                item; 2: the same with up to four consecutive lag
                                chunks of a tile per work item (one partial sum per
                                receiver and step for them); 0: lane-per-lag kernel */
    double  best_ms;         /* time per launch of the chosen configuration */
    double  default_ms;      /* time per launch of the configuration before the call */
} bie_tune;
int bie_autotune(bie_op *op, int32_t reps, bie_tune *out, void *stream);

/*
 * Advances the operator by `steps` steps of zero slip rate, discarding their
 * tractions (the quiescent-history extension of Eq. 4).  The plain form only
 * clears the history slots and moves its step counter; the FDP=H form runs
 * its per-step kernels on an internal zero input.  Asynchronous.
 * Errors: BIE_EINVAL (null operator, negative count, FDP=H steps past the
 * lag count), BIE_EHIP.
 */
int bie_advance(bie_op *op, int64_t steps, void *stream);

/* Clears the history and state (back to step 0; a pending prediction is
 * dropped).  Asynchronous.  Errors: BIE_EINVAL (null operator), BIE_ESTATE
 * (operator not built), BIE_EHIP. */
int bie_reset(bie_op *op, void *stream);

/* Fills *stats_out (host).  Errors: BIE_EINVAL (null pointer). */
int bie_query(const bie_op *op, bie_stats *stats_out);

/*
 * Checkpoint and resume of a time-marching run.  The state of an operator is
 * everything a step reads that earlier steps wrote: the step counter and the
 * slip-rate history the convolution of Eq. 4 runs over (plain form: the
 * history ring; FDP=H form: the near-field history and running slip sum, the
 * recent-history ring of the Domain-F filters, the representative-stress
 * rings of Eqs. 56 and 59 with their Domain-S and transient counterparts,
 * the staircase running sums and the FP64 running Domain-S stress).
 *
 * bie_state_bytes gives the size of a saved state (a 256-byte header, then
 * each array on a 256-byte boundary).  bie_save_state copies the state into
 * dst_dev (device memory of at least that many bytes, 256-byte aligned, owned
 * by the caller) in the order of `stream` and returns when the copy is done.
 * bie_load_state restores a saved state into an operator built from the same
 * problem(s) and parameters (the header's shape and setup fingerprint must
 * match), with the same stream semantics, and sets the step counter to the
 * saved one; the steps that follow give the same tractions, bit for bit, as
 * they did after the save.  A predicted step must be committed first.
 * Errors: BIE_EINVAL (null pointer, misaligned or too small buffer, a state
 * saved from an operator of another shape), BIE_ESTATE (operator not built,
 * predicted step pending), BIE_EHIP.
 */
int bie_state_bytes(const bie_op *op, int64_t *bytes_out);
int bie_save_state(bie_op *op, void *dst_dev, int64_t capacity, void *stream);
int bie_load_state(bie_op *op, const void *src_dev, int64_t capacity, void *stream);

/*
 * Coupled stepping: the step of Eq. 4 split at its first lag, for boundary
 * conditions that fix D_n from T_n (friction, Sec. 6.2).  With the first lag
 * diagonal, T_n = P_n + K_ii,0 D_n, where the prediction
 *   P_n = sum_{m >= 1} K_m D_{n-m}
 * uses the history only.  bie_step_predict writes P_n (device [N]) for the
 * current step without advancing; bie_step_commit then takes that step's
 * slip rate D_n (device [N]) into the history and advances by one step.
 * predict + commit equals bie_step up to rounding.  In the FDP=H form the
 * far-field gathers of step n never read what step n scatters (discretized
 * causality, min dm_i + mbar_j >= 1, checked at setup), so commit only adds
 * D_n's first FIR tap (and its Domain-S and transient terms) to the rings.
 * bie_first_lag writes K_ii,0 (device [N]; negative: radiation damping).
 * Available when the first lag couples each element only to itself: no
 * collocation point within beta eps_t dt (less a relative 1e-9) of another
 * element of its problem (anti-plane mode only).  An element grazed by that
 * front at the limit distance up to rounding (neighbours on a curved trace at
 * beta dt = dx/2) has a first-lag entry below 1e-7 |K_ii,0|: the coupled step
 * leaves such entries out (T_n = P_n + K_ii,0 D_n).  A predict without its commit leaves the operator
 * mid-step: the next predict of the same step is allowed, bie_step is not.
 * Errors: BIE_EINVAL (null arguments, in-plane mode, several scenarios
 * (n_rhs > 1), first lag not diagonal, commit without a predict, step past
 * the lag count), BIE_EHIP.
 */
int bie_step_predict(bie_op *op, double *p_n_dev, void *stream);
int bie_step_commit(bie_op *op, const double *d_n_dev, void *stream);
int bie_first_lag(const bie_op *op, double *k0_dev, void *stream);

/*
 * Dynamic rupture (Sec. 6.2 boundary conditions; App. A.2.3 law): `steps`
 * coupled steps of predict, a per-element friction solve, and commit.
 *   fr        friction law (host):
 *               BIE_LAW_EXP_WEAKENING: strength (t_th - t_dy) exp(-slip/d_c) + t_dy
 *               BIE_LAW_STATIC_DYNAMIC: strength t_dy once ruptured
 *   t0_dev    [N] initial shear traction (device, read)
 *   slip_dev  [N] slip (device, read and updated)
 *   state_dev [N] int32 1 = ruptured (device, read and updated)
 *   D_dev     [steps][N] slip rate out; T_dev [steps][N] shear traction out
 *             (t0 plus the convolution)
 * Per element and step: t* = t0 + P_n; an element not ruptured with t* < t_th
 * keeps D = 0; otherwise it is ruptured and D >= 0 solves
 * t* + K_ii,0 D = strength(slip + dt D) (D = 0 when t* <= strength(slip):
 * it sticks); slip += dt D.  The exponential law's root is bracketed in
 * (0, (t* - t_dy)/|K_ii,0|] and found by Newton steps kept in the bracket,
 * to the rounding level of the equation.
 * Errors: as bie_step_predict, and BIE_EINVAL for an unknown law, t_dy >
 * t_th, d_c <= 0 (exponential law), steps past the lag count.
 */
#define BIE_LAW_STATIC_DYNAMIC 0
#define BIE_LAW_EXP_WEAKENING  1
typedef struct bie_friction {
    int32_t law;
    int32_t reserved;        /* zero */
    double  t_th;            /* yield traction */
    double  t_dy;            /* dynamic (fully weakened) traction */
    double  d_c;             /* slip-weakening distance (exponential law) */
} bie_friction;
int bie_rupture_run(bie_op *op, const bie_friction *fr, const double *t0_dev, double *slip_dev,
                    int32_t *state_dev, double *D_dev, double *T_dev, int64_t steps, void *stream);

/* Frees the operator's host resources (streams, events, graphs) after waiting
 * for the device; the workspace stays the caller's to free. */
void bie_destroy(bie_op *op);

/* Message of the last error on this thread ("" if none). */
const char *bie_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BIE_H */
