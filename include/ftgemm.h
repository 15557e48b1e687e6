/*
 * ftgemm.h -- C ABI of the online fault-tolerant GEMM library for AMD MI355X
 * (gfx950).
 *
 * The library computes C = alpha * A * B + beta * C with algorithm-based fault
 * tolerance fused into the GEMM main loop, following Wu et al., "Anatomy of
 * High-Performance GEMM with Online Fault Tolerance on GPUs" (ICS'23,
 * arXiv:2305.01024):
 *   - checksum encodings e^T A (column checksums of A) and B e (row checksums
 *     of B), section 2.2, Eq. 1-2, carried as the reference checksums of the
 *     product (Eq. 3);
 *   - the outer-product online form (section 2.2, Eq. 4): the checksum
 *     relation is maintained after every k-step update, so each output tile
 *     is checked during the k-loop and at its end (threadblock-level ABFT,
 *     section 4.2.3);
 *   - a single faulty accumulator element per tile and check interval (the
 *     single-event-upset model of section 4.1) is located at the intersection
 *     of the offending row and column and corrected from the checksum
 *     (section 4.2.1, section 5.3).
 * The detection threshold, which the paper fixes in advance without a value
 * (section 2.2), is the analytic FP32 roundoff bound
 *     tau_row_i = c * 2u (K' + n_J + 1) * ||a_i[0:K']|| * sum_{j in J} ||b_j[0:K']||
 *     tau_col_j = c * 2u (K' + m_I + 1) * ||b_j[0:K']|| * sum_{i in I} ||a_i[0:K']||
 * with u = 2^-24, K' the k indices accumulated so far, (m_I, n_J) the valid
 * extent of the tile and c the tolerance factor (default 2).
 *
 * Conventions (BLAS, column-major, no transposes): A is m x k with leading
 * dimension lda >= max(1, m); B is k x n with ldb >= max(1, k); C is m x n with
 * ldc >= max(1, m).  A, B and C are device pointers on the handle's device,
 * owned by the caller.  Every call is asynchronous on the given HIP stream
 * unless a report is requested (then it synchronises that stream).
 *
 * Return codes: FTGEMM_OK (0); FTGEMM_UNCORRECTABLE (1, success with a
 * warning: at least one tile saw more than one fault in a check interval, C
 * may be wrong there and the events say where; with FTGEMM_FT_RECOMPUTE:
 * a recomputed tile flagged again); FTGEMM_NONFINITE_INPUT (2, success with
 * a warning: A or B holds Inf or NaN, the tiles reading it were reported and
 * not checked); negative values are errors listed in enum ftgemm_status.  A handle is not thread-safe; use one handle
 * per stream.
 */
#ifndef FTGEMM_H
#define FTGEMM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ftgemm_ctx* ftgemm_t;

/* FTGEMM_C64: double complex, (re, im) binary64 pairs (ftgemm_run_z64). */
enum ftgemm_dtype { FTGEMM_F32 = 0, FTGEMM_BF16 = 1, FTGEMM_F8E4M3 = 2, FTGEMM_F64 = 3, FTGEMM_C64 = 4 };

/* ft_level: 0 = plain GEMM (fault tolerance compiled out of the kernel);
 * 1 = detect only, one check of the accumulated tile at the end of the
 *     k-loop (the offline, detect-only scheme of section 5.5);
 * 2 = online detect + locate + correct, checks every check interval.
 * FTGEMM_FT_RECOMPUTE may be OR-ed into level 1 or 2 (ftgemm_run only): a
 * tile that ends possibly wrong (level 1: any flagged check; level 2: an
 * uncorrectable pattern) does not write C; a second launch on the same
 * stream recomputes exactly those tiles, with the same level and no fault
 * injection, and writes them.  Section 5.5 recomputes the whole product
 * when its offline (detect-only) scheme flags an error; here only the
 * flagged tiles are recomputed.
 * It adds one small launch per call (it reads a device counter and exits
 * when nothing is queued) and needs no host synchronisation or memset, so
 * with report == NULL the pair of launches can be captured into a HIP graph
 * once the handle's queue is large enough for the shape (the first call of
 * a larger shape allocates it). */
enum ftgemm_level { FTGEMM_FT_OFF = 0, FTGEMM_FT_DETECT = 1, FTGEMM_FT_CORRECT = 2, FTGEMM_FT_RECOMPUTE = 0x10 };

enum ftgemm_status {
    FTGEMM_OK = 0,
    FTGEMM_UNCORRECTABLE = 1,
    FTGEMM_NONFINITE_INPUT = 2,  /* success with a warning: A or B holds Inf/NaN; the tiles that read
                                    it were reported (FTGEMM_EV_NONFINITE), not checked, and their C
                                    is what IEEE arithmetic gives.  FTGEMM_UNCORRECTABLE takes
                                    precedence when both apply. */
    FTGEMM_INVALID = -1,       /* invalid argument; report->bad_arg names it */
    FTGEMM_UNSUPPORTED = -2,   /* dtype, level or device not supported */
    FTGEMM_HIP_ERROR = -3,     /* a HIP runtime call failed */
    FTGEMM_NO_MEMORY = -4,     /* device or host allocation failed */
    FTGEMM_LOG_OVERFLOW = -5   /* more events than the report can hold; counts stay exact */
};

enum ftgemm_event_kind {
    FTGEMM_EV_CORRECTED = 1,      /* one row and one column flagged: element rebuilt */
    FTGEMM_EV_CHECKSUM_ROW = 2,   /* one row flagged, no column: row checksum re-based */
    FTGEMM_EV_CHECKSUM_COL = 3,   /* one column flagged, no row: column checksum re-based */
    FTGEMM_EV_UNCORRECTABLE = 4,  /* any other pattern: checksums re-based, C left as computed */
    FTGEMM_EV_DETECTED = 5,       /* detect-only level: any flagged pattern */
    FTGEMM_EV_NONFINITE = 6       /* the check tile's operands hold Inf or NaN: the bound and the
                                     references are not finite, so rounding cannot be told from a
                                     fault (the single-event-upset model of section 4.1 covers
                                     faults in the computation on finite data).  Logged once per
                                     check tile, at the first check whose k prefix holds the value,
                                     with row = col = -1; nothing is located, corrected or
                                     re-based there and the tile is not recomputed. */
};

enum ftgemm_fault_kind { FTGEMM_FAULT_ADD = 0, FTGEMM_FAULT_XOR = 1 };

/* One detection event.  (tile_m, tile_n) is the check tile, row/col are
 * relative to it (row index within the m range of the check tile, column
 * index within its n range; -1 where nothing was flagged); value_before/after are
 * the accumulator element before and after correction (alpha/beta not yet
 * applied). */
typedef struct {
    int32_t problem, tile_m, tile_n, kstep, row, col, kind, n_rows, n_cols, pad_;
    float value_before, value_after, r_row, r_col, tau_row, tau_col;
} ftgemm_event_t;

/* A fault site for the injection hook: after the accumulator update of k-step
 * `kstep`, element (row, col) of check tile (tile_m, tile_n) of problem `problem`
 * gets `+= payload` (FTGEMM_FAULT_ADD) or has bit (int)payload flipped
 * (FTGEMM_FAULT_XOR). */
typedef struct {
    int32_t tile_m, tile_n, kstep, row, col, kind;
    float payload;
    int32_t problem;
} ftgemm_fault_t;

/* An applied fault: the site, the accumulator value before/after (rounded to
 * float), the residuals and thresholds of its row and column at the first
 * check that saw it (check_step; -1 if no check ran after it), and delta =
 * after - before in binary64 (exact for binary32 accumulators; the binary64
 * difference for binary64 ones). */
typedef struct {
    int32_t problem, tile_m, tile_n, kstep, row, col, kind, check_step;
    float old_v, new_v, r_row, r_col, tau_row, tau_col;
    double delta;
} ftgemm_fault_log_t;

/* Kernel configuration: compute tile m_tile x n_tile (one workgroup), k-step
 * k_step, a check every check_interval k-steps (and after the last), and the
 * check tile check_m x check_n: the block of C whose row and column sums are
 * compared with its own reference checksums and in which one fault per check
 * interval can be corrected.  The check tile is either the compute tile
 * (threadblock-level ABFT, section 4.2.3; 0 x 0 also selects it) or, for the
 * FP32 128x128 tile (2 x 2 wavefronts), the 64x64 sub-tile of one wavefront
 * (warp-level ABFT, section 4.2.2: per-wavefront encodings e^T A_w and B_w e
 * and reference checksums).  Events and fault sites address
 * check tiles: tile_m, tile_n count check tiles of C, row and col are
 * relative to the check tile.  The library reports the check shape it used
 * (never 0). */
typedef struct {
    int32_t m_tile, n_tile, k_step, check_interval;
    int32_t check_m, check_n;
} ftgemm_config_t;

typedef struct {
    uint64_t checks;          /* check-tile checks performed, counted on the device (the
                                 recompute launch's included) */
    uint64_t detected;        /* checks that flagged anything */
    uint64_t corrected;       /* FTGEMM_EV_CORRECTED events */
    uint64_t uncorrectable;   /* FTGEMM_EV_UNCORRECTABLE events */
    uint64_t checksum_only;   /* FTGEMM_EV_CHECKSUM_ROW/COL events */
    uint64_t nonfinite_input; /* FTGEMM_EV_NONFINITE events: check tiles whose operands hold Inf/NaN */
    uint32_t n_events;        /* events written to `events` (<= cap_events) */
    uint32_t cap_events;      /* set by the caller: capacity of `events` */
    ftgemm_event_t* events;   /* caller-owned host array, may be NULL */
    ftgemm_config_t config;   /* configuration the call used */
    int32_t bad_arg;          /* 1-based position of an invalid argument, else 0 */
    float tol_used;           /* threshold factor c the call used */
    int32_t bad_problem;      /* ftgemm_batched: index of the invalid problem, else -1 */
    uint32_t recomputed;      /* FTGEMM_FT_RECOMPUTE: tiles recomputed by the second launch */
    uint32_t recompute_failed;/* ... of which the recomputation flagged again (C written as computed) */
    int32_t pad_;
} ftgemm_report_t;

/* Create a handle on `device` for operands of type `dtype`.  Allocates the
 * device event log and counters.  FTGEMM_F32: A, B are float.  FTGEMM_BF16:
 * A, B are bfloat16 codes (uint16, same column-major layout); products and
 * accumulation are FP32, checksums and the check run in FP32 on the exactly
 * decoded values (section 4.2.3).  Returns FTGEMM_UNSUPPORTED for a dtype
 * with no compiled kernel or a device that is not gfx950. */
int ftgemm_create(ftgemm_t* handle, int dtype, int device);
int ftgemm_destroy(ftgemm_t handle);

/* Per-tensor dequantisation scales for BF16/FP8 operands (default 1; the
 * low-precision operand types extend section 6's list of further data types):
 * the product is computed as (scale_a * A) (scale_b * B).  The scales are
 * applied in the epilogue as alpha * scale_a * scale_b, after the checks,
 * so powers of two keep the result bit-identical to scaling the operands.
 * Ignored for FP32.  Returns FTGEMM_INVALID unless both are > 0. */
int ftgemm_set_scales(ftgemm_t handle, float scale_a, float scale_b);

/* Force a kernel configuration for later calls (NULL: automatic selection).
 * Returns FTGEMM_UNSUPPORTED if no kernel variant has that tile and check
 * shape.  A wavefront check tile applies to ft_level 1 and 2; at level 0
 * the configuration runs the plain kernel of its compute tile.  Automatic
 * selection picks compute-tile checks only. */
int ftgemm_set_config(ftgemm_t handle, const ftgemm_config_t* config);

/* Host-only: the configuration automatic selection picks for a shape. */
int ftgemm_select_config(int dtype, int64_t m, int64_t n, int64_t k, int ft_level,
                         ftgemm_config_t* config);

/* Host-only argument check used by ftgemm_run.  Returns FTGEMM_OK or
 * FTGEMM_INVALID with *bad_arg set to the 1-based position of the offending
 * ftgemm_run argument (2 = m, 3 = n, 4 = k, 7 = lda, 9 = ldb, 12 = ldc,
 * 13 = ft_level, 14 = tol).  ft_level is 0, 1 or 2, optionally with
 * FTGEMM_FT_RECOMPUTE on 1 or 2. */
int ftgemm_validate(int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb, int64_t ldc,
                    int ft_level, float tol, int32_t* bad_arg);

/* C = alpha * A * B + beta * C with fault tolerance level `ft_level`.
 * tol <= 0 selects the default threshold factor c = 2; tol > 0 sets c.
 * beta == 0: C is not read.  k == 0 or alpha == 0: C = beta * C.
 * With report != NULL the call synchronises `stream` and fills the report
 * (events up to report->cap_events).  Returns a status code. */
int ftgemm_run(ftgemm_t handle, int64_t m, int64_t n, int64_t k, float alpha,
               const void* A, int64_t lda, const void* B, int64_t ldb, float beta,
               float* C, int64_t ldc, int ft_level, float tol, hipStream_t stream,
               ftgemm_report_t* report);

/* The same ABFT without the fusion, for measuring what fusing saves
 * (sections 5.2-5.4 compare the fused kernels with ABFT applied around a GEMM):
 * 256 x 256 check tiles, a check every check_k k indices (0 = 256); the
 * encodings, the reference update per chunk and the check (which reads C
 * back from memory and locates / corrects / logs exactly as the fused
 * kernels do) are separate launches around the plain FP32 kernel run on one
 * k-chunk at a time.  FP32 handles only; alpha must be 1 and beta 0
 * (FTGEMM_UNSUPPORTED otherwise).  Fault sites of ftgemm_set_injection apply
 * to C after the GEMM of chunk `kstep` (row/col within the 256 x 256 tile).
 * Events carry the chunk index as kstep.  The chunk GEMMs use the
 * configuration ftgemm_tune found for (m, n, check_k) at level 0, if any.
 * Uses a handle-owned workspace of ceil(m/256) * (k + n) + ceil(n/256) * (k + m)
 * + m + n + ceil(m/256) * ceil(n/256) floats, grown on demand. */
int ftgemm_run_nonfused(ftgemm_t handle, int64_t m, int64_t n, int64_t k, float alpha,
                        const void* A, int64_t lda, const void* B, int64_t ldb, float beta,
                        float* C, int64_t ldc, int check_k, float tol, hipStream_t stream,
                        ftgemm_report_t* report);

/* ftgemm_run for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  No
 * handle: the call runs on the current device, with operands of type `dtype`
 * (FTGEMM_F32, FTGEMM_BF16 or FTGEMM_F8E4M3; per-tensor scales of low-
 * precision operands go into alpha), the automatic configuration and no fault
 * injection; every other argument, the levels, the report and the return
 * codes are those of ftgemm_run.  The call allocates nothing: its counters,
 * event log (1024 events; FTGEMM_LOG_OVERFLOW past that, with the counts
 * exact) and recompute queue live in a static device array of 128.5 KiB that
 * each device holds until the process ends.  FTGEMM_FT_RECOMPUTE on a shape
 * of more than 16384 output tiles returns FTGEMM_NO_MEMORY.  All calls on a
 * device share that array: calls that overlap on one device (several
 * streams, several host threads) race and must be serialised by the caller.
 * The first call on a device takes the array's device address (no
 * allocation); with report == NULL a call launches only kernels, so it can be
 * captured into a HIP graph. */
int ftgemm_run_noalloc(int dtype, int64_t m, int64_t n, int64_t k, float alpha, const void* A, int64_t lda,
                       const void* B, int64_t ldb, float beta, float* C, int64_t ldc, int ft_level, float tol,
                       hipStream_t stream, ftgemm_report_t* report);

/* C = alpha * A * B + beta * C in binary64 for a handle created with
 * FTGEMM_F64 (ftgemm_run refuses such a handle: its C is float).  A, B, C
 * are double, column-major, device pointers as in ftgemm_run; products,
 * accumulation, encodings, reference checksums and the check are binary64,
 * and the threshold takes u = 2^-53 (section 6 names further data types,
 * double-precision complex among them, as future work).  The products run on
 * the FP64 matrix cores.  One compiled configuration: 128 x 128 tiles,
 * k-step 16, a check every 16 k-steps (256 k) unless a configuration is
 * forced; ft_level 0, 1 or 2 (FTGEMM_FT_RECOMPUTE is not supported:
 * FTGEMM_UNSUPPORTED).  tol <= 0 selects c = 2.  Events and the fault log
 * carry their values rounded to float; the fault log also carries the applied
 * offset `delta` in binary64.  Injected FTGEMM_FAULT_XOR sites flip
 * bit (int)payload of the 64-bit value (0..63).  Same return codes, report
 * and bad_arg positions as ftgemm_run. */
int ftgemm_run_f64(ftgemm_t handle, int64_t m, int64_t n, int64_t k, double alpha,
                   const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                   double* C, int64_t ldc, int ft_level, double tol, hipStream_t stream,
                   ftgemm_report_t* report);

/* C = alpha * A * B + beta * C in double complex for a handle created with
 * FTGEMM_C64: A (m x k), B (k x n) and C (m x n) are column-major arrays of
 * (re, im) binary64 pairs, device pointers as in ftgemm_run, with leading
 * dimensions counted in complex elements; alpha and beta point to host
 * (re, im) pairs.  Section 6 names double-precision complex among the data
 * types for future work.  The product runs as two binary64 FT products: with
 * the inner index of each complex product split in two real ones,
 * Re(AB) = A' B' and Im(AB) = A'' B', where A' interleaves (Re A, -Im A),
 * A'' interleaves (Im A, Re A) and B' is B's own storage read as a real
 * 2k x n matrix; the checksum relations of the two products are the real
 * and imaginary parts of the complex ones, so every component of C is
 * checked, located and corrected on its own (a complex element is two real
 * accumulator values; the single-event-upset model of section 4.1 applies to
 * each).  Threshold: u = 2^-53 and 2K' products per component, with
 * complex 2-norms (K' complex k indices accumulated).  A configuration's
 * k_step counts real inner indices (2 per complex k).  Events and fault
 * sites carry the component in `problem` (0 real part, 1 imaginary part);
 * tile, k-step, row and column are those of the real products.  The
 * handle's workspace grows on demand to 4 m k + 2 m n doubles (A', A'' and
 * the two real accumulators; alpha and beta are applied by a final pass).
 * ft_level 0, 1 or 2 (FTGEMM_FT_RECOMPUTE: FTGEMM_UNSUPPORTED).  Return codes
 * and report as ftgemm_run. */
int ftgemm_run_z64(ftgemm_t handle, int64_t m, int64_t n, int64_t k, const double* alpha,
                   const void* A, int64_t lda, const void* B, int64_t ldb, const double* beta,
                   void* C, int64_t ldc, int ft_level, double tol, hipStream_t stream,
                   ftgemm_report_t* report);

/* One problem of a batched call: C = alpha * (scale_a A) (scale_b B) +
 * beta * C, column-major as in ftgemm_run, with its own dtype (FTGEMM_F32,
 * FTGEMM_BF16 or FTGEMM_F8E4M3), sizes, scales and device pointers
 * (96 bytes). */
typedef struct {
    int32_t dtype;
    int32_t reserved_;        /* must be 0 */
    int64_t m, n, k, lda, ldb, ldc;
    float alpha, beta, scale_a, scale_b;
    const void* A;
    const void* B;
    float* C;
} ftgemm_problem_t;

/* Many independent FT-GEMMs in one persistent launch (section 4.2.3 ABFT per
 * output tile, applied to every tile of every problem).  Each problem gets
 * its tile shape from the batched tile variants (FP32 128x128 or 64x64, BF16
 * 128x128, FP8 128x128) by the cost model of ftgemm_tune_batched, and a check
 * every 256 k.
 * The workgroups of a persistent grid walk a cost-ordered list of (problem,
 * tile) items.  Events carry the problem index.  The per-problem plan is
 * built on the host and kept in the handle: a call with the same problem
 * list as the previous batched call on this handle copies nothing and
 * allocates nothing, so with report == NULL it can be captured into a HIP
 * graph (a different list under stream capture returns FTGEMM_INVALID with
 * bad_arg 3).  An invalid problem returns FTGEMM_INVALID with bad_arg 3 and
 * its index in report->bad_problem. */
int ftgemm_batched(ftgemm_t handle, int count, const ftgemm_problem_t* probs, int ft_level, float tol,
                   hipStream_t stream, ftgemm_report_t* report);

/* The configuration the handle's current batched plan uses for problem p
 * (zeros for a problem with no tiles or only the C = beta C update). */
int ftgemm_batched_config(ftgemm_t handle, int p, ftgemm_config_t* config);

/* Autotuner, in place of the paper's kernel-template generator: times every
 * compiled tile variant of the handle's dtype (at ft_level 1 and 2 both check
 * granularities, compute tile and wavefront tile), each with the check intervals
 * of 1, 2, 4, ... k-steps up to max_k_between_checks (0 = 256) columns of k,
 * on operands of shape (m, n, k) allocated for the purpose (filled with
 * zeros, freed before return): one warm-up round, then five interleaved
 * rounds, median per candidate.  The default configuration of ftgemm_run is
 * kept unless a candidate is at least 2% faster.  The result is kept in the
 * handle for this shape and ft_level; later ftgemm_run calls with the same
 * shape and level use it unless a configuration is forced.  *best receives
 * it.  Synchronises `stream`. */
int ftgemm_tune(ftgemm_t handle, int64_t m, int64_t n, int64_t k, int ft_level, int max_k_between_checks,
                hipStream_t stream, ftgemm_config_t* best);

/* Tuned configurations held by the handle, for persisting them: copy up to
 * cap entries into out (shape and level in the first four int64 of each
 * entry: m, n, k, ft_level; then the configuration); *n receives the count.
 * ftgemm_add_tuned inserts one entry (replacing one for the same key). */
typedef struct {
    int64_t m, n, k, ft_level;
    ftgemm_config_t config;
} ftgemm_tuned_t;
int ftgemm_get_tuned(ftgemm_t handle, ftgemm_tuned_t* out, int cap, int* n);
int ftgemm_add_tuned(ftgemm_t handle, const ftgemm_tuned_t* entry);

/* Cost model of ftgemm_batched: the batched tile variants' throughput, in
 * multiply-adds per second, measured by one timed batched launch per variant
 * on 64 problems of 512 x 512 x 512 with operands allocated for the purpose.
 * Without it the model uses built-in relative rates.  rates (may be NULL)
 * receives the measured value per variant (4 entries: FP32 128x128,
 * FP32 64x64, BF16 128x128, FP8 128x128).  Synchronises `stream`. */
int ftgemm_tune_batched(ftgemm_t handle, hipStream_t stream, double* rates);

/* Fault injection hook (section 5.3: errors placed in the accumulator
 * registers to stand for bit flips, a set number per threadblock spread over
 * the k loop at the check distance; section 4.1 fixes the single-upset model
 * they follow).  Compiled into dedicated kernel instantiations; the
 * production kernels contain no injection code.  `faults` is a host array
 * of n sites, copied to the device (the handle owns the copy); n == 0
 * disables injection.  Sites must be sorted by (problem, tile_m, tile_n,
 * kstep); at most 32 per compute tile (all its check tiles together).
 * Returns FTGEMM_INVALID for a negative n, a NULL array with n > 0, a
 * negative coordinate, an unknown kind or a bit index beyond the accumulator
 * (31, or 63 for FP64 and FP64 complex); the order is not checked. */
int ftgemm_set_injection(ftgemm_t handle, const ftgemm_fault_t* faults, int n);

/* Copy the applied-fault log of the last call into `out` (host array of cap
 * entries, caller-owned); *n receives the number of entries copied.  The log
 * is what section 5.3 validates against: each applied fault with the residuals
 * and thresholds of the first check that saw it.  Returns
 * FTGEMM_LOG_OVERFLOW if more faults were applied than were copied (the
 * device log holds 16384 entries; `cap` may be smaller). */
int ftgemm_get_injection_log(ftgemm_t handle, ftgemm_fault_log_t* out, int cap, int* n);

const char* ftgemm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* FTGEMM_H */
