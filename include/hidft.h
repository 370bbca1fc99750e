/*
 * hidft.h -- C ABI of the homogeneous-support DFT library for AMD MI355X (gfx950).
 *
 * Problem (arXiv 2211.15299, Sec. II, "Structured-DFT algorithm"): a signal
 * f in C^N, N = 2^M, has a known frequency support J (|J| = k): (Ff)(m) = 0
 * for m outside J, with (Ff)(m) = sum_n f(n) exp(-2 pi i m n / N).  The
 * algorithm is given J (in binary) and access to entries of f, may preprocess
 * J, and must return the k coefficients {(Ff)(j)}_{j in J} exactly.
 *
 * When J is homogeneous (Sec. VI, Def. homogeneous: the congruence tree of J
 * has exactly log2 k pivots), the library reads f on the k points of the
 * pivoted sampling pattern I_r (Sec. VII, Def. pivoted sampling pattern) and
 * computes the coefficients with the radix-2 recursion of Lemma 3 / Algorithm 1
 * in O(k log k) operations per signal (Theorem 1, Corollary 1).
 *
 * Two layers:
 *   planner  (host, C++): hidft_analyze, hidft_plan_create and the getters.
 *            Validates J, finds the pivots, derives I_r, the plan orders of
 *            Corollary 2 and the twiddle schedule; uploads device tables.
 *   executor (device, HIP): hidft_execute and its variants map samples to
 *            coefficients for a batch of signals on a HIP stream.
 *
 * Numbers.  Samples and coefficients are complex64: interleaved
 * (float re, float im) pairs, 8 bytes per value, 8-byte aligned.  Index sets
 * are uint64.  Arithmetic is FP32 on the device; twiddles are evaluated in
 * FP64 on the device from exact integer exponents and rounded once to FP32.
 *
 * Streams are passed as `void*` holding a hipStream_t (NULL = the legacy
 * default stream).  Device pointers are plain HIP device addresses on the
 * device that was current when the plan was created.
 *
 * Errors.  Every call returns hidft_status; nothing throws across the ABI.
 * Argument, index and homogeneity errors are detected synchronously on the
 * host before any device work is queued.  Device faults surface as HIP errors
 * at the caller's next synchronisation.  hidft_last_error() returns a
 * thread-local message describing the most recent failure on this thread.
 */
#ifndef HIDFT_H_
#define HIDFT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hidft_status {
  HIDFT_OK = 0,
  HIDFT_ERR_INVALID_ARGUMENT = 1,   /* null pointer, bad size, stride, alignment, device */
  HIDFT_ERR_INDEX_OUT_OF_RANGE = 2, /* some j >= N = 2^M */
  HIDFT_ERR_DUPLICATE_INDEX = 3,    /* J lists an index twice */
  HIDFT_ERR_SIZE_NOT_POW2 = 4,      /* k is not a power of two (cannot be homogeneous) */
  HIDFT_ERR_NOT_HOMOGENEOUS = 5,    /* k = 2^s but J has more than s pivots */
  HIDFT_ERR_OUT_OF_MEMORY = 6,      /* host or device allocation failed */
  HIDFT_ERR_DEVICE = 7,             /* a HIP runtime call failed */
  HIDFT_ERR_UNSUPPORTED = 8         /* valid request outside what the library executes */
} hidft_status;

/* Opaque plan: immutable after creation; safe to execute concurrently from
 * several host threads and streams.  Destroying a plan while executions that
 * use it are still in flight is the caller's error: synchronise first. */
typedef struct hidft_plan_s* hidft_plan;

/* Limits of the library. */
#define HIDFT_MAX_LOG2_N 63u        /* N = 2^M with M <= 63 */
#define HIDFT_MAX_LOG2_K_HOST 26u   /* planner (HOST_ONLY plans): k <= 2^26 */
#define HIDFT_MAX_LOG2_K_DEVICE 14u /* executor: one signal is staged whole in LDS */
#define HIDFT_MAX_LOG2_K_LARGE 22u  /* hidft_execute / _ws: larger k in passes through a workspace */

/* Plan flags. */
#define HIDFT_PLAN_HOST_ONLY 0x1u   /* derive the schedule on the host only: no
                                       device tables, no HIP calls; execute
                                       calls on such a plan are refused. */

/*
 * hidft_analyze -- pivots and the homogeneity verdict of J.
 *
 * Sec. VI, Remark 2 (pivot as gcd): level e is a pivot iff 2^e is the largest
 * power of two dividing j1 - j2 for some j1 != j2 in J; Def. homogeneous:
 * exactly log2 |J| pivots (Prop. 1: never fewer).
 *
 *   log2_n          M, with N = 2^M, 0 <= M <= 63.
 *   J[k]            host array of distinct indices in [0, N), any order.
 *   pivots          host output, capacity 64 entries: pivot levels ascending.
 *                   May be NULL.
 *   n_pivots        host output: number of pivots.  May be NULL.
 *   is_homogeneous  host output: 1 if k = 2^s and there are exactly s pivots.
 *                   May be NULL.
 * Returns HIDFT_OK for any valid J, homogeneous or not (the verdict is in
 * *is_homogeneous); INDEX_OUT_OF_RANGE / DUPLICATE_INDEX / INVALID_ARGUMENT
 * otherwise.  Host only; O(k log k).
 */
hidft_status hidft_analyze(uint32_t log2_n, const uint64_t* J, uint64_t k,
                           uint32_t* pivots, uint32_t* n_pivots,
                           int32_t* is_homogeneous);

/*
 * hidft_plan_create -- plan the transform for (N, J).
 *
 * Validates J (range, duplicates, k = 2^s, homogeneity), finds the pivots
 * r_1 < ... < r_s, derives the sample set I_r (Sec. VII, Def. pivoted sampling
 * pattern), the frequency order q(j) = sum_u bit_{r_u}(j) 2^{u-1} of
 * Corollary 2, and the k-1 butterfly twiddles of Lemma 3
 * (stage u, q_lo < 2^{u-1}: exp(-i pi m / 2^{r_u}), m = j mod 2^{r_u} for the
 * j in J whose first u-1 pivot bits spell q_lo).
 * Unless HIDFT_PLAN_HOST_ONLY is set, allocates the device tables on the
 * current device, generates the twiddles there in FP64 (rounded once to FP32)
 * on `stream`, and waits for that work before returning.
 *
 *   log2_n, J, k  as for hidft_analyze; J is copied, the caller keeps it.
 *   flags         0 or HIDFT_PLAN_HOST_ONLY.
 *   stream        hipStream_t used for the table upload (ignored if HOST_ONLY).
 *   out           receives the plan; set to NULL on failure.
 * Errors: INVALID_ARGUMENT, INDEX_OUT_OF_RANGE, DUPLICATE_INDEX,
 * SIZE_NOT_POW2, NOT_HOMOGENEOUS, UNSUPPORTED (device plan with
 * k > 2^HIDFT_MAX_LOG2_K_LARGE, or k > 2^HIDFT_MAX_LOG2_K_HOST),
 * OUT_OF_MEMORY, DEVICE.  A device plan with k > 2^HIDFT_MAX_LOG2_K_DEVICE
 * runs only through hidft_execute and hidft_execute_ws (the other execute
 * calls, the group and the autotuner return UNSUPPORTED for it).
 */
hidft_status hidft_plan_create(uint32_t log2_n, const uint64_t* J, uint64_t k,
                               uint32_t flags, void* stream, hidft_plan* out);

/* Releases host and device memory of the plan.  NULL is accepted. */
hidft_status hidft_plan_destroy(hidft_plan plan);

/* Sizes of the plan: M, k and s = log2 k (any output may be NULL). */
hidft_status hidft_plan_get_info(hidft_plan plan, uint32_t* log2_n, uint64_t* k,
                                 uint32_t* n_pivots);

/* The pivot vector r (ascending), s = log2 k entries, into host memory. */
hidft_status hidft_plan_get_pivots(hidft_plan plan, uint32_t* pivots);

/*
 * The sample set I_r, ascending, k entries, into host memory.  Sample
 * position p of the execute calls holds f(sample_idx[p]).
 * Sec. VII: I_r = { sum_u b_u 2^{M-1-r_u} : b in {0,1}^s }, |I_r| = k.
 */
hidft_status hidft_plan_get_samples(hidft_plan plan, uint64_t* sample_idx);

/*
 * The integer schedule, for exact checks against an independent derivation.
 *   freq_pos[k]       q(J[t]) for the caller's order of J (Corollary 2 order).
 *   tw_num[k-1]       m of each twiddle, stage-major, q_lo-minor
 *                     (stage u = 1..s, q_lo = 0..2^{u-1}-1).
 *   tw_log2den[k-1]   r_u of each twiddle: the value is exp(-i pi m / 2^{r_u}).
 * Any output may be NULL.  Host memory.
 */
hidft_status hidft_plan_get_schedule(hidft_plan plan, uint32_t* freq_pos,
                                     uint64_t* tw_num, uint8_t* tw_log2den);

/*
 * The FP32 twiddles as generated on the device, copied to host memory in the
 * schedule's order (2*(k-1) floats: re, im).  Synchronous.  Device plans only.
 */
hidft_status hidft_plan_get_twiddles(hidft_plan plan, float* twiddles);

/* Device bytes held by the plan (tables), for memory-based admission. */
hidft_status hidft_plan_device_bytes(hidft_plan plan, size_t* bytes);

/*
 * hidft_execute -- batched transform, one plan shared by all signals.
 *
 * For b < batch: d_coefs[b*ld_out + t] = (F f_b)(J[t]) for t < k, where
 * d_samples[b*ld_in + p] = f_b(sample_idx[p]) for p < k (ascending I_r).
 * Coefficients follow the caller's order of J and the DFT of Sec. II exactly
 * (no normalisation).  Computes (N/k) F(J, I_r) f_I by s = log2 k radix-2
 * stages (Lemma 3), which equals (Ff)_J for f in B^J (Sec. VII-B, Lemma 1).
 * One fused kernel launch: each signal is read once from HBM, transformed in
 * LDS and registers, and written once.
 *
 * k > 2^HIDFT_MAX_LOG2_K_DEVICE (up to 2^HIDFT_MAX_LOG2_K_LARGE): the stages
 * run in three passes through a workspace of hidft_plan_workspace_bytes
 * (Corollary 2: the recursion splits at any level): the top s1 = s - s2
 * stages (s1 <= 9) on the 2^s2 columns of each signal, the other s2 stages
 * (s2 = 12 up to k = 2^20, else s - 9) on each of the 2^s1 subtrees with the
 * fused kernel's per-signal code, then a placement into the caller's order
 * of J, scaled by N/k.  The stage arithmetic and order are those of one pass.  Here
 * hidft_execute takes the workspace from the stream-ordered allocator
 * (hipMallocAsync / hipFreeAsync on `stream`); hidft_execute_ws takes it
 * from the caller instead and allocates nothing.
 *
 *   d_samples  device, complex64, batch rows of ld_in >= k values.
 *   d_coefs    device, complex64, batch rows of ld_out >= k values.
 *              May equal d_samples (in place) when ld_out == ld_in; any other
 *              overlap is INVALID_ARGUMENT.
 *   batch      number of signals; 0 is a no-op.
 *   stream     hipStream_t; the call is asynchronous on it.
 * Errors: INVALID_ARGUMENT (null plan or pointer, misaligned pointer,
 * ld < k, bad overlap, current device differs from the plan's, HOST_ONLY
 * plan), DEVICE (launch failure).
 */
hidft_status hidft_execute(hidft_plan plan, const void* d_samples, int64_t ld_in,
                           void* d_coefs, int64_t ld_out, uint64_t batch,
                           void* stream);

/*
 * Workspace of hidft_execute_ws for `batch` signals: 0 for
 * k <= 2^HIDFT_MAX_LOG2_K_DEVICE (one pass, no workspace), else
 * batch * k * 8 bytes (one complex64 intermediate per point).  Any plan
 * (also HOST_ONLY).  Errors: INVALID_ARGUMENT (NULL, or a size that
 * overflows).
 */
hidft_status hidft_plan_workspace_bytes(hidft_plan plan, uint64_t batch, size_t* bytes);

/*
 * hidft_execute_ws -- hidft_execute with the caller's workspace: the same
 * result, bit for bit, and no allocation.  d_work: device, 8-byte aligned,
 * at least hidft_plan_workspace_bytes(plan, batch) bytes, not overlapping
 * the samples or coefficients (d_samples may still equal d_coefs as for
 * hidft_execute); its contents are overwritten.  For
 * k <= 2^HIDFT_MAX_LOG2_K_DEVICE d_work is not used (may be NULL).
 * Errors: those of hidft_execute, and INVALID_ARGUMENT for a missing,
 * small, misaligned or overlapping workspace.
 */
hidft_status hidft_execute_ws(hidft_plan plan, const void* d_samples, int64_t ld_in,
                              void* d_coefs, int64_t ld_out, uint64_t batch, void* d_work,
                              size_t work_bytes, void* stream);

/*
 * Execution variants of the fused transform (hidft_execute_config).
 *
 * precision -- arithmetic of the first group of stages (radix 16: stages
 *   1..4 of Lemma 3, the recursion levels of the four lowest pivots, which
 *   form one fixed 16 x 16 matrix per plan; radix 32: stages 1..5, one
 *   32 x 32 matrix applied as four 16 x 16 blocks); every other stage is FP32:
 *   HIDFT_PREC_FP32   FP32 butterflies (the default).
 *   HIDFT_PREC_F16X2  matrix cores: samples and matrix split into two FP16
 *                     terms (samples scaled per column by a power of two),
 *                     three products summed in FP32.
 *   HIDFT_PREC_BF16X3 matrix cores: three-term BF16 split, six products
 *                     summed in FP32.
 *   The matrix is computed in FP64 on the device at plan creation and split
 *   there.  The matrix-core precisions need k >= 16 (radix 32: k >= 2^13
 *   and the short group last).
 * schedule -- where the short group of stages goes when 4 does not divide
 *   s = log2 k (the transform runs in groups of four stages):
 *   HIDFT_SCHED_DEFAULT      SHORT_LAST (measured the faster grouping).
 *   HIDFT_SCHED_SHORT_FIRST  the first group is short.
 *   HIDFT_SCHED_SHORT_LAST   the first group is a full four stages and the
 *                            last one is short (required by the matrix-core
 *                            precisions when 4 does not divide s).
 *   HIDFT_SCHED_TUNED        the whole variant (schedule, radix, blocks per
 *                            CU) that hidft_autotune recorded for this
 *                            device, size, precision and batch class; DEFAULT
 *                            with the given radix and blocks_per_cu if none.
 *   The schedules compute the same stages in a different grouping; results
 *   agree to rounding.
 * radix -- stages per group (and points per thread): 0 = default (16),
 *   16, or 32 (k >= 2^13 only: 13 = 3 + 5 + 5 stages, 14 = 4 + 5 + 5 with
 *   SHORT_FIRST, 5 + 5 + 3 and 5 + 5 + 4 with SHORT_LAST, the only grouping
 *   of the matrix-core precisions at radix 32).  Like the schedule, changes
 *   the grouping only.
 * blocks_per_cu -- for k <= 2^12 (persistent launches): at most this many
 *   resident workgroups per compute unit, 0 = as many as fit.  Ignored for
 *   larger k (one workgroup per signal).  Does not change results.
 */
#define HIDFT_PREC_FP32 0u
#define HIDFT_PREC_F16X2 1u
#define HIDFT_PREC_BF16X3 2u

#define HIDFT_SCHED_DEFAULT 0u
#define HIDFT_SCHED_SHORT_FIRST 1u
#define HIDFT_SCHED_SHORT_LAST 2u
#define HIDFT_SCHED_TUNED 3u

typedef struct hidft_exec_config {
  uint32_t precision;
  uint32_t schedule;
  uint32_t radix;
  uint32_t blocks_per_cu;
} hidft_exec_config;

/*
 * hidft_execute_config -- hidft_execute with an explicit execution variant.
 *
 * Same contract as hidft_execute (Lemma 3, Sec. VII-B); `config` (host,
 * read during the call only) selects precision, schedule and launch shape.
 * hidft_execute is this call with {FP32, DEFAULT, 0, 0}.
 * Errors: as hidft_execute, plus INVALID_ARGUMENT for a NULL config or an
 * unknown precision, schedule or radix, and UNSUPPORTED for a matrix-core
 * precision with k < 16, or with SHORT_FIRST when the radix's stage count
 * (4 or 5) does not divide s, and for radix 32 with k < 2^13.
 */
hidft_status hidft_execute_config(hidft_plan plan, const hidft_exec_config* config,
                                  const void* d_samples, int64_t ld_in, void* d_coefs,
                                  int64_t ld_out, uint64_t batch, void* stream);

/*
 * hidft_autotune -- pick the fastest execution variant by measurement.
 *
 * No counterpart in the paper: every variant computes the same transform
 * (Lemma 3, Algorithm 1) with another grouping of its stages or launch shape.
 *
 * Runs every variant of `precision` for this plan (both schedules where they
 * differ, radix 16 and 32 where both exist, 0..3 blocks per CU for
 * persistent sizes) on the caller's buffers, as hidft_execute_config would:
 * two warm-up launches, then `reps` timed launches between two HIP events on
 * `stream`, in two interleaved rounds (the better round counts).  Blocks until
 * the measurements are done.  The winner goes to *best (and its mean launch
 * time in microseconds to *best_us, which may be NULL) and into the
 * process-wide tuning table under (device architecture and CU count,
 * s = log2 k, precision, batch class floor(log2 batch)), replacing an older
 * entry; HIDFT_SCHED_TUNED reads it back.
 *
 *   d_samples, ld_in, d_coefs, ld_out, batch  as for hidft_execute; the
 *       samples are read and the coefficient rows are overwritten (they
 *       hold the transform of the samples on return).  The buffers must be
 *       distinct.
 *   reps   timed launches per variant and round, > 0.
 * Errors: as hidft_execute_config, plus INVALID_ARGUMENT for batch == 0,
 * reps == 0, equal buffers or a NULL `best`; DEVICE for event failures.
 */
hidft_status hidft_autotune(hidft_plan plan, uint32_t precision, const void* d_samples,
                            int64_t ld_in, void* d_coefs, int64_t ld_out, uint64_t batch,
                            uint32_t reps, void* stream, hidft_exec_config* best,
                            double* best_us);

/* The tuning table entry for (plan's device, plan's s, precision, class of
 * batch): *found = 1 and *config set, or *found = 0.  Host only. */
hidft_status hidft_tune_lookup(hidft_plan plan, uint32_t precision, uint64_t batch,
                               hidft_exec_config* config, int* found);

/* Empties the process-wide tuning table. */
hidft_status hidft_tune_clear(void);

/*
 * Saves the tuning table to a text file (header line "hidft-tune 1", then one
 * entry per line: device tag, s, precision, batch class, schedule, radix,
 * blocks per CU, measured microseconds), or merges such a file into the table
 * (entries of the file replace equal keys).  INVALID_ARGUMENT if the file
 * cannot be opened or written, lacks the header or has a malformed entry (the
 * table is then unchanged).
 */
hidft_status hidft_tune_save(const char* path);
hidft_status hidft_tune_load(const char* path);

/*
 * hidft_execute_plain -- the plain per-signal GPU method (baseline).
 *
 * Same contract and results as hidft_execute, computed the textbook way:
 * one kernel launch per signal, one workgroup, the samples permuted into the
 * recursion order of Algorithm 1 in LDS, then one radix-2 stage of Lemma 3 per
 * LDS barrier.  Exists to measure the batched and fused forms against.
 */
hidft_status hidft_execute_plain(hidft_plan plan, const void* d_samples, int64_t ld_in,
                                 void* d_coefs, int64_t ld_out, uint64_t batch,
                                 void* stream);

/*
 * Grouped execution: an uneven batch (instances with different N, J and k) in
 * one persistent kernel launch.
 *
 * Each instance is hidft_execute's transform of its own (N, J) (Lemma 3,
 * Algorithm 1, Sec. VII-B); Sec. II's families of index sets are what such a
 * batch draws from.  The packing and the single launch have no counterpart in
 * the paper.
 *
 * One work item is a plan and `batch` rows of samples and coefficients, with
 * the same contract as hidft_execute for that plan.  hidft_group_create
 * validates every item as hidft_execute would, expands the items into
 * instances (one per row), orders them by size, packs instances of equal size
 * -- k >= 2^13 into wide packs of up to 2^14 points, smaller ones into narrow
 * packs of up to 2^12 points (when the wide packs leave the persistent grid a
 * partial last round, that round's packs are split into packs of fewer
 * instances until every block has one; narrow packs likewise up to four per
 * block), schedules the narrow packs over the quarters of the blocks, and
 * uploads the resulting descriptor list (pointers to rows, plan tables and
 * scales, and the schedule) to the current device, waiting for the upload on
 * `stream`.  hidft_group_execute then runs the whole group as one kernel
 * launch on `stream`, asynchronously: each block of the persistent grid runs
 * its wide packs, then splits into four quarters that run their narrow
 * packs.  It may be called any number of times (the samples may change
 * between calls; the pointers may not), also from a captured graph.
 *
 * Ownership: the group copies the items; the plans and buffers they name must
 * outlive every execution of the group.  Outputs of different instances must
 * not overlap (not checked); an instance may run in place.
 * Errors: as hidft_execute for each item (the message names the item), plus
 * INVALID_ARGUMENT for n_items == 0 or more than 2^31 instances, and
 * OUT_OF_MEMORY / DEVICE for the descriptor upload.
 */
typedef struct hidft_work {
  hidft_plan plan;          /* device plan (not HOST_ONLY) */
  const void* d_samples;    /* batch rows of ld_in >= k complex64 samples */
  int64_t ld_in;
  void* d_coefs;            /* batch rows of ld_out >= k complex64 coefficients */
  int64_t ld_out;
  uint64_t batch;           /* rows; 0 contributes nothing */
} hidft_work;

typedef struct hidft_group_s* hidft_group;

hidft_status hidft_group_create(const hidft_work* items, uint64_t n_items, void* stream,
                                hidft_group* out);
hidft_status hidft_group_execute(hidft_group group, void* stream);
hidft_status hidft_group_destroy(hidft_group group);  /* NULL accepted; synchronise first */
/* Instances, packs and device bytes of the descriptor list (outputs may be NULL). */
hidft_status hidft_group_get_info(hidft_group group, uint64_t* n_instances,
                                  uint64_t* n_packs, size_t* device_bytes);

/*
 * Launch configuration of a group (the schedule and pack layout of the one
 * grouped launch; the arithmetic of each stage is the same in all of them).
 *   schedule  HIDFT_SCHED_DEFAULT or _SHORT_LAST: for sizes 2^s with s > 4
 *             and 4 not dividing s, the short radix group runs last;
 *             _SHORT_FIRST: first.  The results of an instance equal
 *             hidft_execute_config's with the same schedule, bit for bit.
 *   order     HIDFT_GROUP_ORDER_LARGEST_FIRST: packs by size, largest first,
 *             so the persistent blocks take them in that order;
 *             _ALTERNATE: the blocks take, in alternate rounds, the largest
 *             and the smallest packs left (a block whose first pack is long
 *             gets a short second one).  The order changes no result.
 * hidft_group_set_config re-packs the group's instances and uploads the new
 * descriptor list on `stream` (waiting for it); it must not overlap an
 * execution of the group.  hidft_group_autotune times every configuration
 * (two warm-up and `reps` timed launches each, in two interleaved rounds,
 * the better round counting), leaves the group in the fastest one and
 * returns it with its mean launch time.  The group's samples are
 * transformed by the timed launches (its outputs are overwritten).
 * Errors: INVALID_ARGUMENT (NULL, unknown schedule or order, reps == 0,
 * another current device), DEVICE for upload or timing failures.
 */
#define HIDFT_GROUP_ORDER_LARGEST_FIRST 0u
#define HIDFT_GROUP_ORDER_ALTERNATE 1u
typedef struct hidft_group_config {
  uint32_t schedule;  /* HIDFT_SCHED_DEFAULT, _SHORT_FIRST or _SHORT_LAST */
  uint32_t order;     /* HIDFT_GROUP_ORDER_* */
} hidft_group_config;

hidft_status hidft_group_set_config(hidft_group group, const hidft_group_config* config,
                                    void* stream);
hidft_status hidft_group_get_config(hidft_group group, hidft_group_config* config);
hidft_status hidft_group_autotune(hidft_group group, uint32_t reps, void* stream,
                                  hidft_group_config* best, double* best_us);

/*
 * Request server (continuous batching).
 *
 * Each request is hidft_execute's transform of its (N, J) (Lemma 3,
 * Algorithm 1, Sec. VII-B), with the plan as the paper's preprocessing
 * (Sec. II).  Batching, admission and the plan cache have no counterpart in
 * the paper.
 *
 * Clients submit requests -- (N = 2^log2_n, J, k host samples on I_r in
 * ascending order) -- from any thread and later collect results.  The server:
 *   * keeps the plans of recently seen supports resident on the device in a
 *     cache keyed by (N, J) whose device bytes never exceed cfg.plan_bytes:
 *     resident plans, a plan being created and evicted plans not yet freed
 *     all count.  A request whose plan is not resident waits while a planner
 *     thread creates it; when the plan does not fit, the planner evicts least
 *     recently used plans that no request holds, and if all are held, keeps
 *     the request (and those queued behind it) waiting until requests retire.
 *     Plan creation and the freeing of evicted plans happen on the planner
 *     thread only, never on a client's or the scheduler's;
 *   * admits requests with resident plans, in arrival order, into batches: a
 *     batch slot takes requests while its region (cfg.data_bytes /
 *     cfg.slots, half for samples, half for coefficients) and cfg.max_batch
 *     allow;
 *   * runs each batch as one grouped launch (see hidft_group_create) on the
 *     slot's own stream.  A slot's regions are pinned host memory mapped for
 *     the device: the kernel reads the samples and writes the coefficients
 *     over the host link, with no copies.  Up to cfg.slots batches are in
 *     flight at once, and requests that arrive while others are on the
 *     device fill the next free slot.
 * A request's coefficients do not depend on which other requests share its
 * batch (each instance runs the same per-signal code).
 *
 * hidft_server_submit: validates the request synchronously (errors as
 * hidft_plan_create for a support that is not resident; OUT_OF_MEMORY if k
 * samples and k coefficients exceed a slot's region, or the plan's tables
 * alone exceed cfg.plan_bytes), queues it and returns its id.  Makes no HIP
 * call and does not change the calling thread's device.  A failure after
 * submission (the device plan cannot be created) completes the request with
 * that status.  host_samples (k complex64) must stay readable and host_coefs
 * (k complex64) writable until the request's result has been polled.
 * Thread-safe.
 * hidft_server_submit_many: hidft_server_submit for n requests in one call;
 * statuses[i] and ids[i] (0 when refused) per request, *n_accepted (may be
 * NULL) the number accepted.
 * hidft_server_poll: moves up to `cap` finished results into `out`, waiting
 * up to wait_us microseconds for the first one; *n receives the count.
 * hidft_server_drain: waits until every submitted request has finished.
 * hidft_server_destroy: refuses new requests, finishes queued work, then
 * frees everything (plans included).
 */
typedef struct hidft_server_s* hidft_server;

typedef struct hidft_server_config {
  size_t data_bytes;   /* pinned host bytes (mapped for the device) for request samples
                          and coefficients, all slots */
  size_t plan_bytes;   /* device bytes of the plan cache: a hard limit (> 0) */
  uint32_t slots;      /* batches in flight, each with its own stream */
  uint32_t max_batch;  /* requests per batch */
} hidft_server_config;

typedef struct hidft_server_request {
  uint32_t log2_n;
  const uint64_t* J;
  uint64_t k;
  const void* host_samples;
  void* host_coefs;
} hidft_server_request;

typedef struct hidft_server_result {
  uint64_t id;
  int32_t status;      /* hidft_status of the request */
  uint32_t batch_size; /* requests in the batch that served it (0 if it failed before) */
  double latency_us;   /* from submit to the coefficients being in host_coefs */
} hidft_server_result;

typedef struct hidft_server_stats {
  uint64_t submitted, completed, rejected, batches;
  uint64_t plan_hits, plan_misses, plan_evictions;
  uint64_t max_inflight_batches;  /* most batches on the device at once */
  uint64_t plans_resident;
  size_t plan_bytes_resident;     /* device bytes counted against plan_bytes now */
  size_t slot_bytes;              /* one slot's sample + coefficient region
                                     (pinned host memory mapped for the device) */
  size_t plan_bytes_peak;         /* most device bytes ever counted (<= plan_bytes) */
  uint64_t waiting_for_plan;      /* requests queued for a plan now */
  uint64_t plan_waits;            /* plans that had to wait for held plans to retire */
  uint64_t failed;                /* requests completed with an error after submission */
} hidft_server_stats;

hidft_status hidft_server_create(const hidft_server_config* cfg, hidft_server* out);
hidft_status hidft_server_submit(hidft_server server, uint32_t log2_n, const uint64_t* J,
                                 uint64_t k, const void* host_samples, void* host_coefs,
                                 uint64_t* id);
hidft_status hidft_server_submit_many(hidft_server server, const hidft_server_request* reqs,
                                      uint64_t n, uint64_t* ids, int32_t* statuses,
                                      uint64_t* n_accepted);
hidft_status hidft_server_poll(hidft_server server, hidft_server_result* out, uint32_t cap,
                               uint32_t* n, int32_t wait_us);
hidft_status hidft_server_drain(hidft_server server);
hidft_status hidft_server_get_stats(hidft_server server, hidft_server_stats* stats);
hidft_status hidft_server_destroy(hidft_server server);

/*
 * hidft_execute_inverse -- the inverse map: coefficients on J to samples on I_r.
 *
 * For b < batch: d_samples[b*ld_out + p] = f_b(sample_idx[p]), the samples on
 * I_r (ascending) of the signal f_b in B^J whose DFT on J is
 * d_coefs[b*ld_in + t] (caller's order of J):
 * f_I = F^{-1}(I_r, J) c (Sec. II, Sec. IV item 1; Eq. submatrix-method).
 * Since F(J, I_r) F(J, I_r)^H = k Id (Lemma 1), this is (1/N) F(J, I_r)^H c,
 * computed as the adjoint of the radix-2 stages of hidft_execute (reverse
 * order, conjugated twiddles), O(k log k) per signal, one kernel launch.
 * Same plans, layouts, alignment, overlap and error rules as hidft_execute,
 * with the roles of the two buffers exchanged.  Above 2^HIDFT_MAX_LOG2_K_DEVICE
 * points, the adjoint of hidft_execute's passes, in reverse order, through a
 * workspace taken from the stream-ordered allocator; hidft_execute_inverse_ws
 * takes it from the caller (hidft_plan_workspace_bytes, the rules of
 * hidft_execute_ws) and allocates nothing.
 */
hidft_status hidft_execute_inverse(hidft_plan plan, const void* d_coefs, int64_t ld_in,
                                   void* d_samples, int64_t ld_out, uint64_t batch,
                                   void* stream);
hidft_status hidft_execute_inverse_ws(hidft_plan plan, const void* d_coefs, int64_t ld_in,
                                      void* d_samples, int64_t ld_out, uint64_t batch,
                                      void* d_work, size_t work_bytes, void* stream);

/*
 * Shift-and-Sample (Sec. IX, Algorithm 2) and the Hi-DFT of part-homogeneous
 * supports (Sec. VII-B, Def. Hi-DFT, Eq. aliasing-homogeneous-tree).
 *
 * J (any k distinct indices) is r-part-homogeneous when it has no pivot at a
 * level <= r_max outside r (Sec. VI, Def. part-homogeneous).  The nodes of
 * its congruence tree at level r_max + 1 (classes of J modulo 2^{r_max+1})
 * then sit at distinct slots q = sum_u bit_{r_u}(node) 2^{u-1} of the
 * 2^s-point Hi-DFT over I_r, s = |r|, and that Hi-DFT of f in B^J gives, at
 * the slot of node v, (2^s/N) mu_J(v, Ff): the sum of the coefficients of the
 * node (its induced weight).  Shift-and-Sample samples f on I_r + j for
 * j < mu* (the largest node), computes the mu* Hi-DFTs (batched fused
 * kernel) and solves one mu(v) x mu(v) dual Vandermonde system per node for
 * its coefficients (Eq. alg1_system), in FP64 on the GPU.  Sample complexity
 * mu* 2^s; cost per Lemma 4.
 *
 * Accuracy of the leaf solves (the paper treats arithmetic as exact).  With
 * V_v the mu(v) x mu(v) system of node v and D_v the mu* x mu(v) matrix of all
 * its shifted rows, the FP32 errors of the Hi-DFT outputs reach the
 * coefficients amplified by at most A = max_v |V_v^{-1}|_2 max_v |D_v|_2 (2-norms,
 * FP64 on the host at plan creation: Gauss-Jordan inverse and power
 * iteration, nodes of equal shape analysed once).  The plan's relative error
 * bound is A (2 + s)/2 u + u, u = 2^-24: (2 + s)/2 u models the FP32 Hi-DFT at
 * 2^s points (measured 1.75 u at 2^6, 2.5 u at 2^14), the last u the rounding
 * of the result.  Plans that solve must keep it within HIDFT_SAS_MAX_REL_ERR.
 *
 * hidft_sas_create: pivots == NULL chooses r: the first t pivots of J (J is
 * part-homogeneous at any such prefix) minimising Lemma 4's cost
 * 1.5 t 2^t mu* + 6 sum_v mu(v)^2 under 2^t <= 2^14 (2^22 when mu* = 1),
 * mu* <= 32 and an error bound <= HIDFT_SAS_MAX_REL_ERR (UNSUPPORTED, naming
 * the best bound, if no prefix qualifies; r = every pivot gives mu* = 1 and
 * qualifies whenever J has at most 22 pivots).  Else r is validated
 * (ascending in [0, M); part-homogeneity: NOT_HOMOGENEOUS; 2^s <= 2^14, or
 * 2^s <= 2^22 with mu* = 1: UNSUPPORTED) and, unless
 * HIDFT_SAS_WEIGHTS_ONLY is set, refused with UNSUPPORTED when mu* > 32 or the
 * error bound exceeds HIDFT_SAS_MAX_REL_ERR (the message names the condition
 * number and the bound).  A HIDFT_SAS_WEIGHTS_ONLY plan serves
 * hidft_sas_weights only: it holds no leaf-solve tables, and
 * hidft_sas_execute refuses it (UNSUPPORTED).  Device tables are built on the
 * current device (synchronously on `stream`) unless HIDFT_PLAN_HOST_ONLY.
 * flags: 0 or any of HIDFT_PLAN_HOST_ONLY, HIDFT_SAS_TWO_PASS,
 * HIDFT_SAS_WEIGHTS_ONLY.
 * hidft_sas_get_accuracy: the largest condition number |V_v|_2 |V_v^{-1}|_2
 * over the nodes, the amplification A and the relative error bound (each
 * +infinity when mu* > 32, where they are not analysed); outputs may be NULL.
 * hidft_sas_get_samples: mu* 2^s sample positions, row j = (I_r + j) mod N
 * in ascending order of I_r: the layout of one signal's samples for execute.
 * hidft_sas_get_nodes: node index of each J[t], and the slot of each node.
 * hidft_sas_execute: d_samples rows (ld_in >= mu* 2^s) -> d_coefs rows
 * (ld_out >= k, caller's order of J).  d_work: device workspace of
 * hidft_sas_workspace_bytes(batch) bytes (mu* n_nodes complex64 values per
 * signal), 8-byte aligned, owned by the caller (no allocation happens in the
 * call); when that size is 0 d_work may be NULL.  It is 0 when mu* = 1 (the
 * Hi-DFT output is the answer) with 2^s <= 2^14 -- above, the Hi-DFT runs in
 * the passes of hidft_execute_ws and needs 2^s complex64 values per signal --
 * and when the plan runs as one kernel: for 2^s <= 2^13 and mu* = 2..4,
 * when the node values fit in LDS (at 2^10 and 2^11 points, with all mu*
 * shifted transforms of a signal in one block, over the transform area;
 * otherwise beside it, with at most 8 elements per thread), the shifted
 * Hi-DFTs gather their node values into LDS and the leaf solves read them
 * there (bit-identical results, no workspace traffic), unless the plan was
 * created with HIDFT_SAS_TWO_PASS.  Inputs,
 * outputs and the workspace must not overlap (INVALID_ARGUMENT).
 * The leaf solves: each node's dual Vandermonde matrix is inverted once, in
 * FP64 on the device, at plan creation (the plan holds sum_v mu(v)^2
 * complex128 values); per signal each coefficient is one row of that inverse
 * times the node's mu(v) values, accumulated in FP64.  They inherit the
 * conditioning of the node's Vandermonde matrix (nodes e^{2 pi i l/N} on the
 * unit circle), which the accuracy bound above accounts for.
 * Supports with additive structure (Sec. IX-B, Lemma 5): passing every pivot
 * of J (from hidft_analyze) as r gives mu* = 1 -- each node at level
 * r_max + 1 holds one element -- so the call is the Hi-DFT on all pivots,
 * 2^n samples for n pivots (up to n = 22), with trivial leaf solves.  For a
 * proper GAP of dimension d, 2^n <= n^d 2^d k (the bound in the proof of
 * Lemma 5).
 * hidft_sas_weights (2^s <= 2^14): d_samples rows of 2^s samples on I_r (ascending) ->
 * 2^s induced weights mu_J(v, Ff) in slot order (0 at slots with no node, up
 * to rounding); with r truncated to its first s-n pivots this is the Hi-DFT
 * at height n.
 */
typedef struct hidft_sas_s* hidft_sas;
#define HIDFT_SAS_MAX_MU 32u
#define HIDFT_SAS_TWO_PASS 0x2u  /* hidft_sas_create flag: always run the
                                    shifted Hi-DFTs and the leaf solves as two
                                    launches through the caller's workspace */
#define HIDFT_SAS_WEIGHTS_ONLY 0x4u  /* hidft_sas_create flag: a plan for
                                        hidft_sas_weights alone (no leaf
                                        solves, no accuracy or mu* limit) */
#define HIDFT_SAS_MAX_REL_ERR 1e-5   /* error bound a solving plan must meet */

hidft_status hidft_sas_create(uint32_t log2_n, const uint64_t* J, uint64_t k,
                              const uint32_t* pivots, uint32_t n_pivots, uint32_t flags,
                              void* stream, hidft_sas* out);
hidft_status hidft_sas_destroy(hidft_sas plan);
hidft_status hidft_sas_get_info(hidft_sas plan, uint32_t* n_pivots, uint32_t* mu_max,
                                uint64_t* n_nodes, uint64_t* samples_per_signal, double* cost);
hidft_status hidft_sas_get_accuracy(hidft_sas plan, double* cond, double* amplification,
                                    double* rel_err_bound);
hidft_status hidft_sas_get_pivots(hidft_sas plan, uint32_t* pivots);
hidft_status hidft_sas_get_samples(hidft_sas plan, uint64_t* sample_idx);
hidft_status hidft_sas_get_nodes(hidft_sas plan, uint32_t* node_of_t, uint32_t* slot_of_node);
hidft_status hidft_sas_workspace_bytes(hidft_sas plan, uint64_t batch, size_t* bytes);
hidft_status hidft_sas_execute(hidft_sas plan, const void* d_samples, int64_t ld_in,
                               void* d_coefs, int64_t ld_out, uint64_t batch, void* d_work,
                               void* stream);
hidft_status hidft_sas_weights(hidft_sas plan, const void* d_samples, int64_t ld_in,
                               void* d_weights, int64_t ld_out, uint64_t batch, void* stream);

/*
 * hidft_sas_execute_noalloc -- hidft_sas_execute without a workspace argument,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * Same transform, arguments (minus d_work), validation and results as
 * hidft_sas_execute, bit for bit.  Plans that need no workspace (mu* = 1, the
 * one-kernel form) run exactly as there.  Otherwise the shifted Hi-DFT
 * outputs go to the library's own device scratch of HIDFT_SAS_SCRATCH_BYTES
 * (one static array per GPU, held until the process ends), and the batch runs
 * in chunks of as many signals as fit it (mu* n_nodes complex64 values per
 * signal, at most 32 * 2^14 * 8 B = 4 MiB; 2^s values above 2^14 samples,
 * so up to 2^21), in stream order on `stream`.  The
 * call allocates nothing: no hipMalloc, no hipFree, no allocating library
 * routine.  The scratch is written in full before it is read, so it needs no
 * clearing.  Every call on a GPU shares that GPU's scratch: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller.
 * Errors: as hidft_sas_execute; UNSUPPORTED if one signal's outputs exceed
 * the scratch; DEVICE if the scratch's address cannot be obtained.
 */
#define HIDFT_SAS_SCRATCH_BYTES (16u << 20)
hidft_status hidft_sas_execute_noalloc(hidft_sas plan, const void* d_samples, int64_t ld_in,
                                       void* d_coefs, int64_t ld_out, uint64_t batch,
                                       void* stream);

/* Human-readable name of a status code (static storage). */
const char* hidft_status_string(hidft_status status);

/* Message of the most recent failure on the calling thread ("" if none). */
const char* hidft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HIDFT_H_ */
