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
 *   - Operators own the device memory they allocate at build time and free
 *     it in bie_destroy().  An operator is not thread safe; calls on one
 *     operator must be ordered on one stream.
 *   - Slip-rate and traction arrays are FP64, time-major: D[n][j], T[n][i].
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
#define BIE_ENOMEM       -3   /* device or host allocation failed */
#define BIE_EHIP         -4   /* a HIP runtime call failed */
#define BIE_ESTATE       -5   /* call not valid in the operator's state */

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
    int32_t reserved;       /* zero */
} bie_fdph_params;

/* flags of bie_fdph_params:
 * BIE_FLAG_QUANTIZE_TRANSIENT  staircase 2D transient waveform (App. A.1 applied
 *   to h^tr, App. B.3): consecutive lags of h^tr within min(eps_qtr |h^|,
 *   eps_st mu/(2 beta) / |K^tr at the pivot|) of one value share it, and the
 *   step keeps the running sums of the runs (Eq. A.3). */
#define BIE_FLAG_QUANTIZE_TRANSIENT 1

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
    int64_t device_bytes;       /* device memory owned by the operator */
    double  bytes_per_step;     /* algorithmic bytes of one steady-state step */
    double  near_bytes_per_step;/* of which: near-field windows and histories */
    double  flops_per_step;     /* 2 x multiply-adds of one steady-state step */
    double  setup_seconds;      /* wall time of the build call */
} bie_stats;

typedef struct bie_op bie_op;

/*
 * Plain form (Eq. 4): evaluates K_{ij,m} for m < n_lags from the closed-form
 * step response on the device and keeps the dense N x N x M tensor (FP64).
 * Blocks until the tensor is built.  Errors: BIE_EINVAL, BIE_ENOMEM, BIE_EHIP.
 */
int bie_build_kernel(const bie_problem *prob, void *stream, bie_op **op_out);

/*
 * FDP=H form (Secs. 3-5, Apps. B.1, B.3, C.2, E, H): builds the cluster tree
 * and block cluster tree, the ART integers, the degenerate waveforms, the
 * ACA+ factors of the Domain-F amplitude, Domain-S static and 2D transient
 * matrices of every admissible leaf, and the near-field windows of every
 * inadmissible leaf.  Blocks until the operator is ready.
 * Several scenarios (params->n_rhs = 2 or 4: slip-rate histories on the same
 * fault) share the kernels: every step row of D and T then holds n_rhs
 * blocks of N values (scenario r at r * N), each scenario keeps its own
 * histories and rings, and the near field reads each window value once for
 * all of them.
 * Errors: BIE_EINVAL, BIE_ECAUSALITY (min over an admissible leaf of
 * dm_i + mbar_j < 1), BIE_ENOMEM, BIE_EHIP.
 */
int bie_compress_fdph(const bie_problem *prob, const bie_fdph_params *params,
                      void *stream, bie_op **op_out);

/*
 * Batched FDP=H form: `count` independent problems (faults of any sizes that
 * do not interact) in one operator, so that each step of all of them is one
 * set of launches.  Each problem gets its own cluster tree and block cluster
 * tree, built as bie_compress_fdph does; no block couples two problems.
 *   probs    [count] problems; all must share mu, beta, dt and eps_t
 *   params   shared FDP=H parameters
 * The operator's element space is the concatenation of the problems in
 * order: D and T rows of bie_step/bie_run hold sum_k n_elem_k values, problem
 * k at offset sum_{k'<k} n_elem_k'.  Its lag count is max_k n_lags_k.  At a
 * step n >= n_lags_k problem k's run is over: its entries of T_n are written
 * as zero and its kernels skip their work.
 * Errors: as bie_compress_fdph, and BIE_EINVAL when count < 1, when a
 * problem is invalid or when the media or time steps differ.
 */
int bie_compress_fdph_batched(const bie_problem *probs, int32_t count,
                              const bie_fdph_params *params, void *stream,
                              bie_op **op_out);

/*
 * One time step: consumes D_n (d_n_dev, N doubles) as the slip rate of the
 * next step n and writes T_n (t_n_dev, N doubles).  Asynchronous.
 * Errors: BIE_EINVAL (null pointer), BIE_ESTATE (operator not built, or a
 * predicted step awaits its commit), BIE_EHIP.
 */
int bie_step(bie_op *op, const double *d_n_dev, double *t_n_dev, void *stream);

/*
 * `steps` consecutive steps: D_dev and T_dev are [steps][N] (time-major).
 * Equivalent to `steps` calls of bie_step.  Asynchronous.
 * Errors: as bie_step, and BIE_EINVAL for a negative count.
 */
int bie_run(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream);

/*
 * As bie_run, with up to 32 consecutive steps captured as one HIP graph and
 * the graph launched once per 32 steps (a remainder of fewer steps runs as
 * eager launches): the step index lives in a device counter that the last
 * node of every captured step advances, so every launch continues where the
 * previous one stopped.  Results are
 * identical to bie_run.  Use for long runs of cheap steps, where per-kernel
 * launch overhead matters.  The graph of a call is kept: a later call with
 * the same D_dev and T_dev from the same step (after bie_reset, say) replays
 * it without capturing again; any other call first waits for it to finish
 * and captures a new one.  The kernel timer (bie_timing) does not see graph
 * launches.  Asynchronous.
 * Errors: BIE_EINVAL, BIE_ESTATE (operator not built), BIE_EHIP.
 */
int bie_run_graph(bie_op *op, const double *D_dev, double *T_dev, int64_t steps, void *stream);

/*
 * Autotuner of the FDP=H near-field kernel: times each launch configuration
 * (source-loop unroll 8 or 16; window loads of 8 or 16 bytes per lane (4 or
 * 8 for FP32 in 64-lag chunks); 4, 3 or 2 workgroups per compute unit; work
 * items in build order or grouped so that items staging the same source
 * histories share one XCD) `reps` times on the operator's own data, at a
 * step index with every lag chunk active, and keeps the fastest for the
 * following steps.  Leaves the operator's state unchanged; blocks until
 * done.  Results of later steps are identical for every configuration of
 * one load width; another width sums each receiver's lags in another order
 * (the same terms, so they agree to rounding).
 *   out (optional)  the chosen configuration and its time per launch
 * Errors: BIE_EINVAL (not an FDP=H operator, reps < 1), BIE_EHIP.
 */
typedef struct bie_tune {
    int32_t unroll;          /* source-loop unroll of the chosen configuration */
    int32_t lds_pad;         /* unused LDS bytes per workgroup (occupancy cap) */
    int32_t item_order;      /* 0: build order, 1: grouped by sources per XCD */
    int32_t candidates;      /* configurations timed */
    int32_t load_bytes;      /* window bytes each lane loads at once (4, 8 or 16) */
    int32_t reserved;        /* zero */
    double  best_ms;         /* time per launch of the chosen configuration */
    double  default_ms;      /* time per launch of the configuration before the call */
} bie_tune;
int bie_autotune(bie_op *op, int32_t reps, bie_tune *out, void *stream);

/*
 * Advances the operator by `steps` steps of zero slip rate, discarding their
 * tractions (the quiescent-history extension of Eq. 4).  The plain form only
 * clears the history slots and moves its step counter; the FDP=H form runs
 * its per-step kernels on an internal zero input.  Asynchronous.
 * Errors: BIE_EINVAL (null operator, negative count), BIE_EHIP.
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
 * Copies integer setup data of an FDP=H operator to host buffers, for
 * checking against an independent implementation.  `what` selects:
 *   BIE_EXPORT_NEAR    rows of 3 int64: receiver, source, window W_ij
 *   BIE_EXPORT_LEAVES  rows of 5 int64: admissible (1/0), receiver-cluster
 *                      size, source-cluster size, smallest receiver index,
 *                      smallest source index
 *   BIE_EXPORT_ART     rows of 6 int64 per admissible (leaf, source, receiver
 *                      slot): leaf id, source j, mbar_j, dm_j, receiver i
 *                      (or -1), dm_i  -- one row per source and per receiver
 *   BIE_EXPORT_TRANS   rows of 4 int64 per admissible leaf: leaf id, pivot
 *                      source, transient length, number of staircase runs
 *                      (0 unless BIE_FLAG_QUANTIZE_TRANSIENT)
 * Writes at most `capacity` rows to buf_host and the total row count to
 * *rows_out (call with capacity 0 to size the buffer).
 */
#define BIE_EXPORT_NEAR   1
#define BIE_EXPORT_LEAVES 2
#define BIE_EXPORT_ART    3
#define BIE_EXPORT_TRANS  4
int bie_fdph_export(const bie_op *op, int32_t what, int64_t *buf_host,
                    int64_t capacity, int64_t *rows_out);

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

/*
 * Kernel timing of the operator's dominant kernel (the dense sum of the plain
 * form; the near-field window convolution of the FDP=H form).  While enabled,
 * every step records a pair of HIP events around that kernel on the step's
 * stream (at most 16384 pairs; later steps are not recorded).  Enabling
 * clears earlier records.  bie_timing_read waits for the last recorded event
 * and returns the summed elapsed milliseconds and the number of launches.
 * Errors: BIE_EINVAL (null operator), BIE_EHIP.
 */
int bie_timing(bie_op *op, int32_t enable);
int bie_timing_read(const bie_op *op, double *ms_total_out, int64_t *launches_out);

/*
 * Measurement utility (not part of the method): streams `bytes` of device
 * memory at buf_dev once with 16-byte non-temporal loads (the access of the
 * near-field and dense kernels) and returns the elapsed milliseconds of that
 * one launch, timed with HIP events on `stream` (blocks until done).  `bytes`
 * must be a positive multiple of 16; buf_dev 16-byte aligned; its contents
 * are only read.  Gives the HBM read rate the streaming kernels can reach.
 * Errors: BIE_EINVAL, BIE_EHIP.
 */
int bie_hbm_read_probe(const void *buf_dev, int64_t bytes, double *ms_out, void *stream);

/* Frees the operator and its device memory (after the stream is idle). */
void bie_destroy(bie_op *op);

/* Message of the last error on this thread ("" if none). */
const char *bie_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BIE_H */
