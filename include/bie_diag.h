/*
 * bie_diag.h -- diagnostics of the BIEM convolution library (include/bie.h):
 * kernel timing, an HBM read probe, exports of integer setup data, a scan
 * of the tractions for non-finite values, and checks of the ACA+
 * compression.  None of these is part of the method; they serve
 * measurement, tests and debugging.  Same conventions as bie.h.
 */
#ifndef BIE_DIAG_H
#define BIE_DIAG_H

#include "bie.h"

#ifdef __cplusplus
extern "C" {
#endif

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
 * Debug scan of the tractions (failure detection): with
 * BIE_DEBUG_SCAN_FINITE set, every step also scans its T_n for NaN or Inf
 * and records the first offending (step * row values + index) in a word of
 * the operator's workspace (a few microseconds per step).  Setting the flag
 * clears the record.  bie_debug_status waits for `stream` and returns that
 * position, or -1 when every scanned traction was finite.
 * Errors: BIE_EINVAL (null pointer), BIE_ESTATE (operator not built),
 * BIE_EHIP.
 */
#define BIE_DEBUG_SCAN_FINITE 1
int bie_set_debug(bie_op *op, int32_t flags, void *stream);
int bie_debug_status(const bie_op *op, int64_t *first_bad_out, void *stream);

/*
 * ACA+ (Sec. 6.1.1, the compression bie_plan_fdph applies to every
 * admissible block) on a caller matrix, host only: A_host is nr x ns,
 * row-major.  Returns the rank reached, whether the block was kept exactly
 * (rank = min(nr, ns)), the number of full residual sweeps, and the relative
 * Frobenius error |A - U V^T| / |A| of the result (0 for a zero matrix).
 * Errors: BIE_EINVAL.
 */
int bie_diag_aca(int32_t nr, int32_t ns, const double *A_host, double eps, uint64_t seed, int32_t *rank_out,
                 int32_t *fallback_out, int32_t *sweeps_out, double *rel_err_out);

/*
 * Exact low-rank errors of an FDP=H plan's blocks (host, evaluates every
 * entry of every admissible block): rows of 8 doubles per block -- leaf,
 * piece (0 Domain F, 1 Domain S, 2 transient), component, rows, columns,
 * rank, |A - U V^T|_F / |A|_F with the FP64 factors, and the same with the
 * factors rounded to BF16.  Writes at most `capacity` rows and the block count
 * to *rows_out (capacity 0 sizes the buffer).  Errors: BIE_EINVAL.
 */
int bie_plan_block_errors(const bie_plan *plan, double *buf_host, int64_t capacity, int64_t *rows_out);

/*
 * Causal-band entries of each lag of a plain-form plan (per component):
 * buf_host[m] = sum over receivers i of the band width at lag m, for
 * m < min(capacity, M) -- the kernel values a step reads at that lag.
 * Errors: BIE_EINVAL (null pointer, not a plain-form plan).
 */
int bie_plan_dense_lag_entries(const bie_plan *plan, int64_t *buf_host, int64_t capacity);

#ifdef __cplusplus
}
#endif

#endif /* BIE_DIAG_H */
