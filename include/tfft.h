/*
 * tfft.h -- C ABI of the fault-tolerant batched FFT library for MI355X (gfx950).
 *
 * The library computes a batched one-dimensional complex-to-complex discrete
 * Fourier transform (TurboFFT paper, arXiv 2405.02520, Section II: forward
 * y_j = sum_n x_n w_N^{jn}, w_N = exp(-2 pi i/N); inverse with w_N^{-jn} and
 * a 1/N factor) and protects it with the paper's two-sided checksum
 * (Section III, Eq. (4)-(5)): each group of G signals is encoded before the
 * transform with the per-position vector c = (e^T W)^T and the batch vectors
 * w1 = 1, w2 = (1..G); after it with e; a mismatch beyond a rounding-scaled
 * threshold is detected, the quotient of the two residuals locates the
 * corrupted signal, and the divergence between the transform of the combined
 * input and the combined output is added back to it (Section III-B).
 *
 * Conventions for every entry point:
 *  - Status codes are ints (enum tfft_status); nothing throws across the ABI.
 *  - Device buffers are owned by the caller, hold `batch` contiguous signals of
 *    `n` interleaved complex values (re, im) each, row-major [batch][n], and
 *    must be 16-byte aligned.  Input and output are either the same buffer
 *    (in place; see tfft_exec_forward) or do not overlap at all.
 *  - A plan owns its tables, workspace and report buffers; it is bound to the
 *    device current when it was created and must not be executed on two
 *    streams at once.  hip_stream may be NULL (the null stream).
 *  - Execution is asynchronous on the given stream; tfft_get_report
 *    synchronises that stream.
 */
#ifndef TFFT_H
#define TFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TFFT_VERSION 1
#define TFFT_MAX_PASSES 3

typedef struct tfft_plan_s *tfft_plan;

/* Element type: complex64 (two binary32) or complex128 (two binary64). */
enum tfft_dtype { TFFT_C64 = 0, TFFT_C128 = 1 };

/* Fault-tolerance mode of one execution.
 *  OFF     transform only.
 *  DETECT  transform + two-sided checksum; flagged groups are reported (and
 *          located by the residual quotient) but outputs are left as computed.
 *  CORRECT as DETECT, then the located signal of each flagged group is
 *          rewritten from the transform of the group's combined input
 *          (delayed, batched correction, Section III-B).                     */
enum tfft_ft_mode { TFFT_FT_OFF = 0, TFFT_FT_DETECT = 1, TFFT_FT_CORRECT = 2 };

enum tfft_status {
    TFFT_OK = 0,
    TFFT_UNCORRECTABLE = 1,  /* output written; some flagged group could not be located */
    TFFT_E_INVALID = -1,     /* bad argument */
    TFFT_E_UNSUPPORTED = -2, /* valid request this build does not implement */
    TFFT_E_NOMEM = -3,       /* device or host allocation failed */
    TFFT_E_HIP = -4,         /* a HIP runtime call failed */
    TFFT_E_STATE = -5,       /* call out of order (e.g. report before any exec) */
    TFFT_E_SCRATCH = -6      /* tfft_exec_noalloc: the execution needs more than the
                                static scratch (TFFT_SCRATCH_BYTES) */
};

/* Plan flags. */
enum tfft_flags {
    TFFT_INVERSE_UNSCALED = 1u << 0, /* exec_inverse omits the 1/N factor */
    TFFT_PERSISTENT = 1u << 1,       /* ragged plans only: every class's passes run in one
                                        persistent kernel launch draining a work queue */
    TFFT_PERSIST_INTERLEAVE = 1u << 2, /* with TFFT_PERSISTENT: the work items of a block of
                                         signals take every n-th checksum group instead of a
                                         range of them (tfft_ragged_tune chooses either) */
    TFFT_PERSIST_ONE_QUEUE = 1u << 3   /* with TFFT_PERSISTENT: one work queue for all
                                         workgroups instead of one per XCD (tfft_ragged_tune
                                         chooses either) */
};

/* Record actions. */
enum tfft_action {
    TFFT_ACT_DETECTED = 1,      /* flagged; DETECT mode */
    TFFT_ACT_CORRECTED = 2,     /* flagged, located and rewritten */
    TFFT_ACT_BENIGN = 3,        /* flagged, data consistent (fault hit the checksum) */
    TFFT_ACT_UNCORRECTABLE = 4  /* flagged, not locatable (outside one fault per group) */
};

/* Location method of a record.  TFFT_LOC_THREAD: the thread-level scheme
 * found the fault inside one radix butterfly; in a one-pass plan record.sub
 * then holds that butterfly's stage, and the ratio is k + 1 for its wrong
 * output k.  TFFT_LOC_SUBSIGNAL: the one-sided scheme flagged one sub-signal
 * of a multi-pass plan's pass (record.sub), recomputed alone. */
enum tfft_locate {
    TFFT_LOC_NONE = 0,
    TFFT_LOC_QUOTIENT = 1,
    TFFT_LOC_PER_SIGNAL = 2,
    TFFT_LOC_THREAD = 3,
    TFFT_LOC_SUBSIGNAL = 4
};

/* Granularity of the checksum (TurboFFT Sec. IV-B and the overhead
 * comparison of Sec. V).
 *   BLOCK  - two-sided checksum over a group of G signals, one residual pair
 *            per group reduced over the workgroup (the default);
 *   SIGNAL - one-sided: one residual per signal (per sub-signal in the
 *            passes of multi-pass plans; transform encoding only), reduced
 *            over its threads; a flagged (sub-)signal is recomputed in
 *            binary64;
 *   THREAD - two-sided checks of every radix butterfly inside the thread that
 *            computes it (two transform encodings e and (k+1) e locate the
 *            wrong output); a flagged butterfly is recomputed in registers.
 *            Protects the butterflies only, not the data between them nor
 *            the inter-pass twiddles of multi-pass plans. */
enum tfft_scheme { TFFT_SCHEME_BLOCK = 0, TFFT_SCHEME_SIGNAL = 1, TFFT_SCHEME_THREAD = 2 };

/* Options for tfft_plan_create_with.  Zero fields take the defaults. */
typedef struct {
    uint32_t flags;  /* enum tfft_flags */
    int32_t group;   /* signals per checksum group G (a power of two, 1..64); 0 = default */
    double kappa;    /* threshold factor; 0 = default (16 for complex64, 96 for complex128,
                        calibrated on fault-free runs) */
    int32_t passes;  /* 0 = automatic; 1, 2 or 3 forces the number of passes (n <= 2^12
                        for 1, 2^8 <= n <= 2^20 for 2, n >= 2^12 for 3); another
                        length gives E_UNSUPPORTED */
    int32_t grid_scale; /* 0 = default; else workgroups per launch = default * 2^grid_scale
                           (-3..3), a tuning knob */
    int32_t scheme;  /* enum tfft_scheme */
    int32_t chunk;   /* multi-pass plans: run the batch in chunks of this many signals (a
                        multiple of 64), each chunk's passes through one workspace slot of
                        chunk * n elements; 0 = the whole batch at once.  Faults, records
                        and group numbers are those of the whole batch. */
    int32_t split;   /* multi-pass plans: 0 = the default split N = M_1..M_P (shortest
                        first); 1 = the alternative (two passes: the longer first; three
                        passes: the middle length first), a tuning knob */
    int32_t reserved[3];
} tfft_options;

/* Description of a plan (tfft_plan_info). */
typedef struct {
    int64_t n, batch;
    int32_t dtype, passes;
    int32_t pass_len[TFFT_MAX_PASSES];     /* transform length of each pass, product = n */
    int32_t group[TFFT_MAX_PASSES];        /* checksum group size of each pass           */
    int32_t elems_per_thread[TFFT_MAX_PASSES];
    int32_t tile_signals[TFFT_MAX_PASSES]; /* sub-signals held in LDS by one workgroup   */
    int32_t stages[TFFT_MAX_PASSES];
    int32_t radices[TFFT_MAX_PASSES][8];   /* butterfly radix of each stage of each pass */
    int64_t groups[TFFT_MAX_PASSES];       /* checksum groups per pass                   */
    size_t workspace_bytes;
    double kappa;
} tfft_plan_desc;

/* Counters of the last execution. */
typedef struct {
    int64_t groups_checked; /* groups whose checksums were compared (all passes) */
    int64_t detected;       /* flagged groups                                    */
    int64_t corrected;
    int64_t uncorrectable;
    int64_t benign;
    int64_t n_records;      /* records available (<= capacity)                   */
    int64_t dropped;        /* flagged groups beyond the record capacity         */
} tfft_counts;

/* One flagged group.
 * Checksum groups: in a one-pass plan, group g of G = group[0] members holds
 * signals g*G .. g*G+G-1 (member b = signal g*G + b; the last group may be
 * partial).  In pass p of a multi-pass plan (tile C = tile_signals[p],
 * G = group[p], rb = G / C), the sub-transforms are numbered per signal as
 * in tfft_fault (sub = o * S_p + i in a strided pass, sub = output row r in
 * the last pass); an "outer unit" is one block o of one signal (strided
 * passes, unit = signal * (N / L_p) + o) or one signal (last pass), and a
 * "strip" is C consecutive sub-transforms i (strided) or rows r (last) of a
 * unit.  With n_strips = S_p / C (strided) or (N / M_P) / C (last), group g
 * holds members b = 0..G-1: unit (g / n_strips) * rb + b / C, sub-transform
 * (g % n_strips) * C + b % C of that unit; members whose unit lies beyond the
 * batch do not exist (a partial last group). */
typedef struct {
    int64_t signal;   /* batch index of the affected signal (group's first signal if not located) */
    int64_t sub;      /* multi-pass plans: sub-transform of the located member inside the signal
                         (see tfft_fault); one-pass plans: 0 */
    int64_t group;    /* checksum group index within the pass */
    int32_t pass;     /* 0-based pass */
    int32_t member;   /* located member within the group, -1 if none */
    int32_t action;   /* enum tfft_action */
    int32_t method;   /* enum tfft_locate */
    double residual;  /* |d1| = |R1 - L1| */
    double threshold; /* tau */
    double ratio_re, ratio_im; /* d2 / d1 */
} tfft_record;

/* Kinds of injected faults: an additive value (the paper's register offset)
 * or one flipped bit (the paper's bit-flip protocol, Section II-A). */
enum tfft_fault_mode { TFFT_FAULT_ADD = 0, TFFT_FAULT_FLIP_RE = 1, TFFT_FAULT_FLIP_IM = 2 };

/* Test instrument: one fault in a register of the transform of signal
 * `signal` in pass `pass` (an additive value or one flipped bit):
 *   stage >= 0: to output `index` of butterfly stage `stage` (position in that
 *               stage's output array, after the stage's butterflies);
 *   stage == -1: to final output value `index` of the pass (after the
 *               inter-pass twiddle, conjugation and scale), before the
 *               post-transform checksum.
 * For one-pass plans index = position.  For a plan of P passes with lengths
 * M_1..M_P, pass p transforms N / M_p sub-signals of each signal and
 * index = sub * M_p + position, where for p < P sub = o * S_p + i (block o of
 * L_p = M_p...M_P elements, offset i < S_p = L_p / M_p inside the stride) and
 * for the last pass sub is the output row r (outputs r + (N / M_P) k).  This
 * models a compute fault (paper Section II-A) inside the protected region. */
typedef struct {
    int64_t signal;
    int32_t pass;
    int32_t stage;
    int64_t index;
    double dre, dim;  /* TFFT_FAULT_ADD: value added */
    int32_t mode;     /* enum tfft_fault_mode */
    int32_t bit;      /* TFFT_FAULT_FLIP_*: bit of the IEEE representation of the
                         real or imaginary part (0 = least significant; < 32 for
                         complex64, < 64 for complex128) */
} tfft_fault;

/* Create a plan for `batch` transforms of length `n` (a power of two,
 * 2 <= n <= 2^24) of element type `dtype`.  Chooses one pass for n <= 2^12,
 * two passes up to 2^19 (complex64) / 2^20 (complex128) and three above
 * (n = M_1 M_2 [M_3], the tiled FFT of Section IV-A.1, last pass stored
 * transposed); generates every twiddle and
 * checksum vector in binary64 on the host and rounds it once; allocates the
 * tables, the workspace (multi-pass plans: n * batch elements; three-pass
 * plans also use the output buffer between passes) and the report.
 * *out receives the plan, or NULL on error.  E_INVALID for bad arguments,
 * E_NOMEM / E_HIP on allocation failure. */
int tfft_plan_create(tfft_plan *out, int64_t n, int64_t batch, int dtype, uint32_t flags);
int tfft_plan_create_with(tfft_plan *out, int64_t n, int64_t batch, int dtype, const tfft_options *opt);

/* Free a plan and everything it owns.  NULL is accepted. */
int tfft_plan_destroy(tfft_plan p);

/* Forward transform of the plan's batch, d_in -> d_out, on hip_stream.
 * ft_mode is enum tfft_ft_mode.  Resets the report.  d_in == d_out transforms
 * in place; in CORRECT mode that needs a two-pass plan (the correction of a
 * pass re-reads that pass's inputs, which in place survive only when they are
 * in the workspace) or the THREAD scheme, else E_UNSUPPORTED.  Returns
 * E_INVALID for NULL, misaligned or partially overlapping buffers or a bad
 * mode, E_HIP if a launch fails, else OK (the outcome of the checks is read
 * with tfft_get_report). */
int tfft_exec_forward(tfft_plan p, const void *d_in, void *d_out, int ft_mode, void *hip_stream);

/* Inverse transform (w_N^{-jn}; times 1/N unless TFFT_INVERSE_UNSCALED). */
int tfft_exec_inverse(tfft_plan p, const void *d_in, void *d_out, int ft_mode, void *hip_stream);

/* Size of the library's static device scratch: one array of this many bytes
 * per device the library runs on, held until the process ends. */
#define TFFT_SCRATCH_BYTES (64u << 20)

/* Allocation-free execution, for callers that cannot allocate device memory
 * while they run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same transform, checks and outcome as
 * tfft_exec_forward (inverse == 0) or tfft_exec_inverse (inverse != 0) on the
 * same plan and buffers, but the execution's report counters, records and
 * multi-pass workspace live in the library's static device scratch of
 * TFFT_SCRATCH_BYTES instead of the plan's buffers; the call allocates
 * nothing (no hipMalloc, no hipFree, no allocating library routine).  The
 * caller passes the input and output buffers as for tfft_exec_forward.
 * Returns E_SCRATCH when the report and workspace of the plan need more than
 * TFFT_SCRATCH_BYTES (about 64 B per checksum group plus, for multi-pass
 * plans, n * batch elements, or n * chunk with tfft_options.chunk), else as
 * tfft_exec_forward.  Every call on one device shares that device's scratch
 * and leaves the last call's contents there: tfft_get_report on this plan
 * reads the scratch and is valid until the next tfft_exec_noalloc on the
 * same device, and calls that overlap in time on one device (two streams,
 * two threads) race. */
int tfft_exec_noalloc(tfft_plan p, const void *d_in, void *d_out, int ft_mode, int inverse, void *hip_stream);

/* Copy out the report of the last execution: counters into *counts (may be
 * NULL) and up to `cap` records, sorted by (signal, pass, group, sub), into
 * recs (may be NULL when cap == 0).  Synchronises the stream of the last execution.
 * Returns UNCORRECTABLE if any flagged group was left uncorrected in CORRECT
 * mode, E_STATE before the first execution, else OK. */
int tfft_get_report(tfft_plan p, tfft_counts *counts, tfft_record *recs, int64_t cap);

/* Test hook: install `n` fault specifications applied by every following
 * execution (n = 0 clears them).  The specs are validated against the plan
 * (signal, pass, stage and index in range) and copied; E_INVALID otherwise.
 * Waits for the plan's last execution (its stream) before replacing the
 * tables it reads. */
int tfft_set_faults(tfft_plan p, const tfft_fault *specs, int64_t n);

/* Fill *info with the plan's decomposition and sizes. */
int tfft_plan_info(tfft_plan p, tfft_plan_desc *info);

/* The description tfft_plan_info would give for a plan created with these
 * arguments, computed on the host without creating the plan (no device call,
 * no allocation): validation as tfft_plan_create_with (E_INVALID /
 * E_UNSUPPORTED), the pass decomposition N = M_1..M_P of the tiled FFT
 * (Section IV-A.1), thread radix, tile and stage radices of every pass, the
 * checksum groups and the workspace size. */
int tfft_plan_describe(int64_t n, int64_t batch, int dtype, const tfft_options *opt, tfft_plan_desc *info);

/* Host generators of the tables a plan uploads (no device call):
 *  tfft_host_root: out[0] + i out[1] = w_n^t = exp(-2 pi i t / n) in binary64,
 *    for any integer t and n >= 1, the twiddle of the DFT matrix (Section II;
 *    the paper precomputes twiddles, Section IV-A.3).  The angle is reduced
 *    exactly in integers to a quadrant and libm sees only [0, pi/4].
 *  tfft_host_checksum_vector: the precomputed checksum vector
 *    c = scale * (e^T W)^T with e_k = w_3^k, for a length-m DFT matrix W
 *    (w_m^{-kn} when inverse != 0), Section II-C Eq. (1)-(2); out[2n],
 *    out[2n+1] = c_n for n < m (2m doubles, caller-owned).  m a power of two,
 *    2..2^24.
 * E_INVALID for a NULL out or an argument outside those ranges. */
int tfft_host_root(int64_t t, int64_t n, double *out);
int tfft_host_checksum_vector(int64_t m, int inverse, double scale, double *out);

/* Measurement instrument.  With timing enabled (enable != 0), every
 * execution records HIP events on its stream immediately before and after
 * each kernel launch; tfft_get_timings synchronises that stream and writes
 * the durations of the last execution in milliseconds: pass_ms[p] for the
 * transform kernel of pass p and correct_ms[p] for its correction launch
 * (0 when not launched); each array holds TFFT_MAX_PASSES entries, either may
 * be NULL.
 * E_STATE if timing was off for the last execution. */
int tfft_set_timing(tfft_plan p, int enable);
int tfft_get_timings(tfft_plan p, double *pass_ms, double *correct_ms);

/* ------------------------------------------------------------------------
 * Ragged batches: `count` signals of power-of-two lengths lengths[i]
 * (2..2^24) stored at element offsets offsets[i] of the input and output
 * buffers, signal i occupying [offsets[i], offsets[i] + lengths[i]) of each
 * (signals must not overlap each other).  Signals of one length form a class
 * that is transformed by one plan addressing the signals through a device
 * offset table (no repacking).  Records and faults use the index i.
 * ------------------------------------------------------------------------ */
typedef struct tfft_ragged_s *tfft_ragged;

/* Create a ragged plan on the current device.  lengths[count] and
 * offsets[count] are host arrays (copied; the caller keeps ownership);
 * dtype as for tfft_plan_create; opt as for tfft_plan_create_with (applied
 * to every class), may be NULL.  E_INVALID: count < 1, a length that is not a
 * power of two in 2..2^24, a negative offset, overlapping signals, a bad
 * dtype or option; E_NOMEM / E_HIP as for plans.  *out is NULL on failure.
 *
 * With TFFT_PERSISTENT in opt->flags (lengths 64..2^24, else E_UNSUPPORTED)
 * every pass of every class runs in one persistent kernel launch: its
 * workgroups take work items (a range of at most 64 checksum groups of one
 * pass of one class) from a device queue, run them, correct the groups they
 * flagged (CORRECT mode) and release them; an item of pass p > 0 starts once
 * every item of pass p - 1 covering the same block of 64 signals of its
 * class is released.  One report serves all classes.  In place is not
 * supported in this mode (E_INVALID).  With TFFT_PERSIST_INTERLEAVE as well,
 * the items of a block of signals take every n-th of its checksum groups
 * (n = the number of items) instead of a range, so that the workgroups
 * running them side by side work on neighbouring strips of the data.  The
 * items sit in 8 queues, one per XCD (TFFT_PERSIST_ONE_QUEUE: a single
 * one), every item of a block of signals in the same queue; a workgroup
 * serves its own XCD's queue first and the others once it is drained. */
int tfft_ragged_create(tfft_ragged *out, int64_t count, const int64_t *lengths, const int64_t *offsets, int dtype,
                       const tfft_options *opt);
/* Free the plans, graphs and streams of r (NULL-safe). */
int tfft_ragged_destroy(tfft_ragged r);

/* Transform every signal (forward, or inverse when inverse != 0) from the
 * device buffer d_in to d_out, each at least max(offsets[i] + lengths[i])
 * elements, 16-byte aligned, not overlapping each other; elements outside
 * every signal are left untouched in d_out.  ft_mode as for
 * tfft_exec_forward.  With use_graph != 0 all launches of all classes are
 * captured once into a HIP graph (per buffers, mode, direction and stream;
 * the classes run on parallel branches) and replayed as one graph launch;
 * hip_stream must then be a non-null stream.  Asynchronous; E_INVALID for
 * NULL or misaligned pointers, E_HIP for a failed launch or capture. */
int tfft_ragged_exec(tfft_ragged r, const void *d_in, void *d_out, int ft_mode, int inverse, int use_graph,
                     void *hip_stream);

/* Merged report of the last execution (records carry the ragged index i). */
int tfft_ragged_get_report(tfft_ragged r, tfft_counts *counts, tfft_record *recs, int64_t cap);

/* Test hook; specs[k].signal is the ragged index. */
int tfft_ragged_set_faults(tfft_ragged r, const tfft_fault *specs, int64_t n);

/* Autotuner (the semi-empirical choice of per-size parameters, TurboFFT
 * Sec. IV-B.3 and Table I, made by measurement), timing candidates on the
 * given buffers with fault tolerance CORRECT, `reps` executions each after
 * one warm-up.  Per-class plans: for each length class, the candidate plans
 * (pass count, checksum group size, workgroups per launch), fastest kept.
 * Persistent plans: coordinate descent over the classes, largest first, on
 * the time of the whole persistent launch: per class the pass count, the
 * split of the stages over the passes and the checksum group size (classes
 * up to 4096 points keep one pass), then the tiles per work item.
 * Overwrites d_out.  Synchronous on hip_stream; drops captured graphs; the
 * new class plans get the injected faults of the old ones. */
int tfft_ragged_tune(tfft_ragged r, const void *d_in, void *d_out, void *hip_stream, int reps);

/* Classes of the ragged plan: their count in *classes and, for the first
 * `cap` classes, length, number of signals and the chosen plan's
 * description (arrays may be NULL). */
int tfft_ragged_info(tfft_ragged r, int64_t *classes, int64_t *lengths, int64_t *counts, tfft_plan_desc *descs,
                     int64_t cap);

/* Measurement instrument: copy `bytes` from d_src to d_dst (device buffers,
 * 16-byte aligned, not overlapping) with a plain streaming kernel that moves
 * data the way the pass kernels do (16-byte non-temporal loads and stores,
 * several in flight per thread, many workgroups); the bandwidth it reaches
 * is the attainable HBM ceiling quoted next to the peak.  Asynchronous on
 * hip_stream.  E_INVALID for NULL, misaligned or overlapping buffers. */
int tfft_stream_copy(void *d_dst, const void *d_src, size_t bytes, void *hip_stream);

/* Static text for a status code. */
const char *tfft_status_string(int status);

/* TFFT_VERSION of the library. */
int tfft_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TFFT_H */
