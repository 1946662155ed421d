/*
 * pf.h - C-ABI of the butterfly-interaction bootstrap particle filter on
 * MI355X (gfx950).
 *
 * Method: Heine, Whiteley, Cemgil, "Parallelising Particle Filters with
 * Butterfly Interactions" (arXiv 1812.01502).
 *
 *  - The filter is Algorithm 1 (particle filter) of Section 1.1 for the hidden
 *    Markov model of eq. HMM: X_0 ~ pi_0, X_n | X_{n-1} ~ f(X_{n-1}, .),
 *    Y_n | X_n ~ g(X_n, .). The observations are fixed inputs (Section 1.3).
 *  - The particle count is N = mM with the interaction pattern A_1..A_S of
 *    eq. A matrices (Section 1.2, Assumption A1). Here the pattern is given
 *    as a radix r: the particle index is written in mixed radix (digits of
 *    radix r from the least significant end, the top digit taking what is
 *    left) and stage k lets the particles that differ only in digit k
 *    interact (Lemma 1 for r = 2; Remark 1 allows any such family).
 *  - One time step t runs one stage, k = t mod S (the stage-wise scheme of
 *    Section 1.2 with the rotation proposed in Section 6.4): log-weight with
 *    y_t, resample inside each group with probability proportional to the
 *    weights (Algorithm 3), carry the group-mean weight (eq. V_defn_proofs),
 *    gather the ancestors, propagate with f.
 *  - r >= N is the plain bootstrap filter with global multinomial resampling
 *    (Algorithms 1 and 2).
 *
 * Conventions
 *  - Every function returns a pf_status (0 = PF_OK, < 0 = error) and never
 *    aborts or throws. After a device error a handle is poisoned: later
 *    calls return PF_E_STATE until pf_destroy.
 *  - Numeric failure: the reduction of every step checks its partial sums on
 *    the device. A step whose weights are not usable (a non-finite sum, e.g.
 *    from a non-finite device observation or state, or no positive weight)
 *    gets an estimate record with valid = 0, adds nothing to the
 *    log-normaliser and sets a sticky per-filter flag on the device: every
 *    later record is invalid too. Calls that synchronise (pf_estimate,
 *    pf_history) then return PF_E_NUMERIC (their output is still written),
 *    and pf_step / pf_run return PF_E_NUMERIC without work until pf_reset,
 *    pf_set_state or pf_load clears the flag. The handle is not poisoned.
 *  - All pointers marked "host" are ordinary host memory, read or written
 *    before the call returns. Pointers marked "device" are HIP device
 *    memory on the handle's device.
 *  - A handle owns all its device buffers. Model arrays are copied at
 *    create time; the caller keeps ownership of what it passes.
 *  - Work is enqueued on the HIP stream given at create time (NULL = the
 *    default stream). Calls that return data to the host synchronise that
 *    stream. A handle is not thread-safe; distinct handles are independent.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by
 *    `seed`, counter (particle pair, step, block, stream_id). Results depend
 *    only on (model, N, radix, resampler, dtype, seed, stream_id, y), not on
 *    launch shapes.
 */
#ifndef PF_H
#define PF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_MAX_DIM 16

typedef enum {
  PF_OK = 0,
  PF_E_INVALID = -1,     /* bad argument (size, pointer, radix, dimension) */
  PF_E_UNSUPPORTED = -2, /* valid but not supported by this build */
  PF_E_OOM = -3,         /* device allocation failed */
  PF_E_HIP = -4,         /* a HIP runtime call failed */
  PF_E_NUMERIC = -5,     /* non-finite observation or weights */
  PF_E_STATE = -6        /* handle poisoned by an earlier error */
} pf_status;

typedef enum { PF_MODEL_LG = 0, PF_MODEL_SV = 1 } pf_model_kind;
typedef enum { PF_RESAMPLE_MULTINOMIAL = 0, PF_RESAMPLE_SYSTEMATIC = 1 } pf_resampler;
/* Storage type of the particle states. F32 and BF16 compute in FP32 with
 * FP32 log-weights; F64 computes and stores in FP64. The running
 * log-normaliser is always FP64. */
typedef enum { PF_DTYPE_F32 = 0, PF_DTYPE_BF16 = 1, PF_DTYPE_F64 = 2 } pf_dtype;

/* Model (host memory, copied at create). Section 1.1, eq. HMM.
 * LG  (kind = PF_MODEL_LG), all matrices row-major d x d, vectors length d:
 *       x_0 = m0 + P0_chol z,  x_n = A x_{n-1} + Q_chol z,
 *       y_n = H x_n + R_chol e,  z, e ~ N(0, I_d);
 *     Q_chol, R_chol, P0_chol lower-triangular with positive diagonal.
 *     g(x, y) is the N(H x, R) density, normalising constant included.
 * SV  (kind = PF_MODEL_SV, d = 1):
 *       x_0 ~ N(0, sigma^2 / (1 - phi^2)),  x_n = phi x_{n-1} + sigma z,
 *       y_n = beta exp(x_n / 2) e.                                        */
typedef struct {
  int32_t kind;
  int32_t d;                /* 1 <= d <= PF_MAX_DIM (SV: 1) */
  const double* A;
  const double* Q_chol;
  const double* H;
  const double* R_chol;
  const double* m0;
  const double* P0_chol;
  double phi, sigma, beta;  /* SV only; |phi| < 1, sigma > 0, beta > 0 */
} pf_model;

typedef struct {
  uint64_t n_particles;  /* N: power of two, 2 <= N <= 2^30 */
  uint64_t radix;        /* r: power of two >= 2; r >= N selects the global path */
  int32_t resampler;     /* pf_resampler */
  int32_t state_dtype;   /* pf_dtype */
  uint64_t seed;         /* Philox key */
  uint32_t stream_id;    /* Philox counter word 3 (identity of the filter) */
  uint32_t history;      /* per-step estimate records kept on device (0 -> 1) */
  uint32_t keep_ancestors; /* nonzero: record each step's ancestor indices */
  uint32_t full_cycle;     /* nonzero: every time step runs all S stages of
                              Algorithm 3 (full augmented resampling; the
                              output is unweighted, Lemma 3(c)); zero: one
                              stage per step, k = t mod S */
  uint32_t island;         /* M > 0: the island filter of Section 4
                              (Algorithm 4, AIRPF) instead of the butterfly
                              filter: N / M islands of M consecutive
                              particles, M a power of two, 2 <= M <= N / 2
                              (M <= 4096; radix is ignored, full_cycle must
                              be 0). A step weights, resamples within every
                              island (Algorithm 5, `resampler` applies),
                              runs the log2(N / M) island stages of
                              Algorithm 6 (whole islands copied) and
                              mutates; the output is unweighted. */
  uint32_t island_swap;    /* island filter only. 0: the no-swap rule of
                              Algorithm 7 (a pair of islands whose draws
                              would exchange their samples keeps them);
                              nonzero: plain Algorithm 6. */
  double ess_threshold;    /* theta in (0, 1]: ESS-gated stages (Section
                              1.2, the fully adapted scheme, with the
                              rotating start of Section 6.4). A step
                              weights, then runs butterfly stages k, k + 1,
                              ... (mod S) only while the effective sample
                              size (sum w)^2 / (N sum w^2) of the current
                              weights is below theta, at most S; k is the
                              stage after the last one run by an earlier
                              step (0 at first). The estimate record's
                              `stage` is the number of stages run. Needs FP32
                              states, radix <= 64 and below N, N >= 512, no
                              full_cycle, island or keep_ancestors.
                              0: off. */
} pf_config;

/* Estimate of one completed step t (the weighted cloud
 * before resampling, i.e. the filtering law of x_t given y_0..y_t). */
typedef struct {
  uint32_t t;              /* step index the record belongs to */
  uint32_t stage;          /* butterfly stage k = t mod S used by the step
                              (S: a full-cycle step ran every stage; island
                              filter: the number of island stages; ESS-gated
                              stages: the number of stages the step ran) */
  uint32_t radix;          /* radix r_k of that stage (full cycle: the radix;
                              island filter: the island size M) */
  uint32_t valid;          /* 1 if the step has run and its weights were
                              usable; 0 if it has not run, or after a
                              numeric failure (see Conventions) */
  double log_normaliser;   /* running log p-hat(y_0..y_t), FP64 */
  double ess;              /* (sum w)^2 / (N sum w^2), in [1/N, 1] */
  double max_log_weight;   /* max_i l_i of the step */
  double next_offset;      /* max of the new log-weights (subtracted next step) */
  double mean[PF_MAX_DIM]; /* weighted mean of x_t */
  double var[PF_MAX_DIM];  /* weighted variance of x_t */
} pf_estimate_t;

typedef struct {
  uint64_t n_particles;
  uint32_t d;
  uint32_t n_stages;        /* S */
  uint32_t radices[32];     /* r_0..r_{S-1} */
  uint32_t global_path;     /* 1 if r >= N */
  uint32_t state_dtype;
  uint64_t device_bytes;    /* device memory held by the handle */
  uint32_t t;               /* completed steps */
  uint32_t tile_elems[32];  /* particles per workgroup tile, per stage */
} pf_info_t;

typedef struct pf_handle pf_handle;

/* Create a filter and run the initialisation of Algorithm 1 (x_0 ~ pi_0,
 * unit weights) on `hip_stream` (a hipStream_t, or NULL). On success *out
 * owns the handle. Errors: PF_E_INVALID (N not a power of two, radix < 2
 * or not a power of two, d out of range, NULL pointers, non-finite or
 * non-positive-definite parameters), PF_E_UNSUPPORTED (a stage radix the
 * device kernels cannot tile), PF_E_OOM, PF_E_HIP. */
pf_status pf_create(const pf_model* model, const pf_config* cfg, void* hip_stream,
                    pf_handle** out);

/* Release every device buffer of the handle. NULL is accepted. */
pf_status pf_destroy(pf_handle* h);

/* Re-run the initialisation (t = 0, log-normaliser 0) with the same seed. */
pf_status pf_reset(pf_handle* h);

/* One time step (Algorithm 1 loop body with one butterfly stage) using the
 * observation `y_host` (host, d doubles). Asynchronous. Errors:
 * PF_E_NUMERIC for a non-finite observation, PF_E_STATE if poisoned. */
pf_status pf_step(pf_handle* h, const double* y_host);

/* `n_steps` consecutive time steps reading observation j from
 * `y_dev + j * y_stride` (device; elements of the compute type: float for
 * F32/BF16 states, double for F64; y_stride >= d). With use_graph != 0 the
 * launches are captured in a HIP graph and replayed once. Asynchronous.
 * A non-finite device observation makes its step a numeric failure (see
 * Conventions). */
pf_status pf_run(pf_handle* h, const void* y_dev, uint32_t n_steps, uint64_t y_stride,
                 int32_t use_graph);

/* Estimate of the last completed step (synchronises the stream). `out`
 * host, caller-owned. PF_E_STATE if no step has run. */
pf_status pf_estimate(pf_handle* h, pf_estimate_t* out);

/* The last min(n_max, history, steps run) records, oldest first (host
 * output; synchronises). *n_out receives the count. */
pf_status pf_history(pf_handle* h, pf_estimate_t* out, uint32_t n_max, uint32_t* n_out);

/* Current particle cloud (synchronises): x_host receives d planes of N
 * values in the storage type (plane j = component j of every particle),
 * logw_host receives N log-weights normalised so that their max is 0
 * (float, or double for F64 states); either may be NULL. *t_out (may be
 * NULL) receives the number of completed steps and *log_norm (may be NULL)
 * the running log-normaliser. */
pf_status pf_get_state(pf_handle* h, void* x_host, void* logw_host, uint32_t* t_out,
                       double* log_norm);

/* Overwrite the particle cloud (host input, same layouts as pf_get_state)
 * and set the step counter and log-normaliser. Used to start a step from a
 * given cloud. logw_host may be NULL (all zero). */
pf_status pf_set_state(pf_handle* h, const void* x_host, const void* logw_host, uint32_t t,
                       double log_norm);

/* Checkpoint (host memory). pf_save writes the filter's complete state:
 * a versioned header (configuration, model fingerprint, step counter,
 * running log-normaliser, log-weight offset), the d state planes, the raw
 * log-weights and the estimate record of the last step. With buf == NULL
 * only *len_out (the size needed) is set. cap < size -> PF_E_INVALID.
 * Synchronises. The blob is plain bytes, owned by the caller. */
pf_status pf_save(pf_handle* h, void* buf, uint64_t cap, uint64_t* len_out);

/* Restore a pf_save blob into a handle created with the same model, N,
 * radix, resampler and dtype (seed and stream_id may differ: the
 * continuation then draws other random numbers). Afterwards the handle
 * continues exactly as the saved one would have: same states, weights,
 * step counter and log-normaliser. Mismatch, truncation or corruption ->
 * PF_E_INVALID with the handle unchanged. */
pf_status pf_load(pf_handle* h, const void* buf, uint64_t len);

/* Ancestor index a(i) (into the previous cloud) of every particle of the
 * last step (host output, N uint32; synchronises). Requires
 * cfg.keep_ancestors, else PF_E_STATE. In full-cycle mode: the ancestors of
 * the last stage (into the cloud after the previous stage). */
pf_status pf_get_ancestors(pf_handle* h, uint32_t* anc_host);

/* Sizes and plan of the handle (host output). */
pf_status pf_info(pf_handle* h, pf_info_t* out);

/* Wait for all work of the handle (hipStreamSynchronize). */
pf_status pf_sync(pf_handle* h);

/* ------------------------------------------------------------------------
 * Batched filters: n independent filters (each its own model, N, radix,
 * resampler, seed and stream_id) advanced together. Every filter computes
 * exactly what a single pf_handle with the same configuration computes
 * (same states and log-weights bit for bit; estimates up to the summation
 * order of the reductions). Filters are grouped by (state dimension, model
 * kind); one step is one kernel launch per group plus one reduction launch
 * per group, with no host data besides two device pointers, so pf_batch_run
 * can capture many steps in one HIP graph.
 * Restrictions: FP32 states, 512 <= N <= 2^30, stage radices <= 64 (no
 * global path), no ancestor recording. A slot may be vacant (n_particles =
 * 0) and re-bound to another filter at any time (pf_batch_rebind).
 * ------------------------------------------------------------------------ */
typedef struct pf_batch pf_batch;

/* One autotuner trial: a (pairs per thread, radix) candidate of a class,
 * the measured time of one batched step, and whether it was chosen. */
typedef struct {
  uint32_t class_index;
  uint32_t dim;             /* compiled state dimension of the class */
  uint32_t model_kind;      /* 0 dense LG, 1 LG with diagonal noise, 2 SV */
  uint32_t pairs_per_thread;/* tile of 512 x pairs_per_thread particles */
  uint32_t radix;
  uint32_t chosen;
  float ms_per_step;
  uint32_t reserved;
} pf_batch_tune_t;

/* Create n filters from models[i] and cfgs[i] (host arrays, copied) and run
 * every initialisation (Algorithm 1). cfgs[i].radix = 0 asks the autotuner
 * to choose the radix of that filter: per class it times one batched step
 * for each tile size and radix in {2, ..., 64} and keeps, at the fastest
 * tile size, the largest radix within 10 % of the fastest time (see
 * pf_batch_tuning). cfgs[i].history and the dtype other than F32 are not
 * supported (history is 1). Errors as pf_create; the message of a failed
 * create is pf_batch_last_error(NULL).
 * hip_stream: the stream every call enqueues on (NULL: the null stream).
 * With a non-null stream the batch also creates three streams of its own
 * (default priority, released by pf_batch_destroy): pf_batch_step and
 * pf_batch_run spread the classes of filters over them, forked from and
 * joined back to hip_stream by events within the call, so work enqueued on
 * hip_stream after a call sees all of it (also inside a captured graph). */
pf_status pf_batch_create(const pf_model* models, const pf_config* cfgs, uint32_t n,
                          void* hip_stream, pf_batch** out);

/* Release every device buffer. NULL is accepted. */
pf_status pf_batch_destroy(pf_batch* b);

/* One time step of every active filter. y_dev (device, float): the packed
 * observations, filter i's d_i values at offset sum_{j<i} d_j. active_dev
 * (device, n bytes, or NULL for all): filters with 0 do not step (their
 * state, counter and record are untouched). Asynchronous. */
pf_status pf_batch_step(pf_batch* b, const float* y_dev, const uint8_t* active_dev);

/* n_steps batched steps, step j reading y_dev + j * y_stride (y_stride >=
 * sum d_i), the same active mask for all; with use_graph != 0 captured in
 * one HIP graph and replayed once. Asynchronous. */
pf_status pf_batch_run(pf_batch* b, const float* y_dev, uint32_t n_steps, uint64_t y_stride,
                       const uint8_t* active_dev, int32_t use_graph);

/* Estimate record of the last step of every filter (host output, n
 * records; a filter that has not stepped has valid = 0, and so has a filter
 * whose weights became unusable at that step or earlier: a numeric failure
 * of one filter, e.g. a non-finite observation, leaves the others
 * unaffected; pf_batch_reset or pf_batch_set_state clears it).
 * Synchronises. */
pf_status pf_batch_estimates(pf_batch* b, pf_estimate_t* out);

/* Plan of filter f (radices, tile size, completed steps). */
pf_status pf_batch_filter_info(pf_batch* b, uint32_t f, pf_info_t* out);

/* Autotuner trials (host output, up to n_max; out may be NULL to count). */
pf_status pf_batch_tuning(pf_batch* b, pf_batch_tune_t* out, uint32_t n_max, uint32_t* n_out);

/* State of filter f (host, layouts as pf_get_state with float storage). */
pf_status pf_batch_get_state(pf_batch* b, uint32_t f, float* x_host, float* logw_host,
                             uint32_t* t_out, double* log_norm);

/* Overwrite the state of filter f (as pf_set_state). */
pf_status pf_batch_set_state(pf_batch* b, uint32_t f, const float* x_host, const float* logw_host,
                             uint32_t t, double log_norm);

/* Re-initialise filter f with a new seed and stream_id (t = 0), e.g. to
 * give its slot to a new stream. Synchronises. */
pf_status pf_batch_reset(pf_batch* b, uint32_t f, uint64_t seed, uint32_t stream_id);

/* Wait for all work of the batch. */
pf_status pf_batch_sync(pf_batch* b);

/* Copy the estimate record of every filter (n records, as
 * pf_batch_estimates) into `out` asynchronously: the copy is enqueued on
 * the batch's stream after the work enqueued so far, and the call returns
 * at once. `out` is host memory the caller owns; it must be page-locked
 * (hipHostMalloc, or a framework's pinned buffer) for the copy to overlap,
 * and must not be read before the stream (or an event recorded on it after
 * this call) has completed. Lets a serving loop collect estimates without
 * stalling the device. */
pf_status pf_batch_estimates_async(pf_batch* b, pf_estimate_t* out);

/* Re-bind `count` slots of a batch (slots[i], distinct) to other filters
 * in one call: slot slots[i] takes models[i] and cfgs[i] (host arrays) -
 * any model, state dimension, N, radix (0: 64, capped at N / 2; no
 * autotuning), resampler, seed and stream_id that pf_batch_create accepts -
 * or becomes vacant with cfgs[i].n_particles = 0 (no particle memory, never
 * steps, records valid = 0; its model is not read). pf_batch_create accepts
 * vacant slots the same way. The slots' previous device buffers are
 * released first (a slot bound at create time keeps its share of the
 * create-time pools until pf_batch_destroy); the new filters are allocated
 * through the batch's allocator and initialised (Algorithm 1; t = 0). The
 * packed observation layout follows the slots' current dimensions (vacant
 * slots take none). Synchronises the batch's stream once. Every other
 * filter continues exactly as before. Errors: as pf_batch_create for a
 * slot's configuration (nothing is changed); PF_E_OOM when a filter does
 * not fit: that slot is left vacant, the others are bound. */
pf_status pf_batch_rebind(pf_batch* b, uint32_t count, const uint32_t* slots, const pf_model* models,
                          const pf_config* cfgs);

/* Last error message of the batch ("" if none); NULL: the last failed
 * pf_batch_create of this thread. */
const char* pf_batch_last_error(const pf_batch* b);

/* Device memory of handles and batches. By default every device buffer of a
 * handle or batch (state planes, log-weights, reduction records, control
 * block, estimate records, scratch of the global and island paths) comes
 * from hipMalloc and goes back with hipFree. pf_set_allocator installs a
 * pair of callbacks instead, e.g. a framework's caching allocator:
 *   alloc(bytes, ctx) returns device memory on the current device of at
 *   least `bytes` bytes, aligned to 256 bytes, or NULL when it has none;
 *   free_(ptr, ctx) takes back a pointer alloc returned.
 * Process-wide and thread-safe. The setting applies to handles and batches
 * created afterwards; each keeps the allocator it was created with and frees
 * every buffer with it (pf_destroy / pf_batch_destroy, or a failed create,
 * after synchronising its stream). alloc = free_ = NULL restores
 * hipMalloc/hipFree. The callbacks are called only from pf_create and
 * pf_batch_create (alloc) and from pf_destroy, pf_batch_destroy and failed
 * creates (free_), on the calling thread; they must stay valid until every
 * handle using them is destroyed.
 * Errors: PF_E_INVALID when exactly one of alloc and free_ is NULL. A NULL
 * from alloc makes the create fail with PF_E_OOM, a misaligned pointer with
 * PF_E_INVALID (the pointer is handed back to free_ first). */
pf_status pf_set_allocator(void* (*alloc)(size_t bytes, void* ctx), void (*free_)(void* ptr, void* ctx),
                           void* ctx);

/* pf_run without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc). It runs what pf_create followed by pf_run and
 * pf_history computes, for the butterfly path with rotating stages only
 * (radix < N; no full_cycle, island, ess_threshold or keep_ancestors;
 * cfg->history is ignored), on state buffers the caller owns:
 *   x_dev     (device, in/out) d planes of N values in the storage type,
 *             plane j = component j of every particle (as pf_get_state);
 *   logw_dev  (device, in/out) N log-weights (float; double for F64
 *             states), any common offset (all zero for a fresh cloud);
 *   y_dev     (device) observation j at y_dev + j * y_stride, in the
 *             compute type (float; double for F64), y_stride >= d;
 *   est_dev   (device, out) n_steps records, record j for step t0 + j; the
 *             log-normaliser accumulates from 0 at the first step of the
 *             call.
 * Step t0 + j uses stage (t0 + j) mod S and the random numbers of that
 * step, so from the cloud pf_create initialises (pf_get_state at t = 0)
 * and t0 = 0 it computes the same states, log-weights and records as
 * pf_create + pf_run of the same configuration, bit for bit. The steps
 * update x_dev and logw_dev in place. Every other buffer (control block,
 * model parameters, the per-tile reduction records of one step) lives in one
 * static device array of 1 MiB per device (kept until the process ends);
 * its address is looked up once per device. Calls that overlap on one device
 * (other streams or threads) share that array and race: serialise them.
 * Asynchronous on hip_stream; calls no allocation routine (device memory
 * comes only from the caller and the static array; the model parameters
 * reach the device as kernel arguments). Errors, with the message in
 * pf_last_error(NULL): PF_E_INVALID (arguments as pf_create, NULL buffers,
 * y_stride < d), PF_E_UNSUPPORTED (a configuration outside the above, or N
 * and d whose reduction records exceed the static array: e.g. above about
 * 2^25 particles at d = 1, 2^22 at d = 8), PF_E_HIP. */
pf_status pf_run_noalloc(const pf_model* model, const pf_config* cfg, void* x_dev, void* logw_dev,
                         const void* y_dev, uint32_t n_steps, uint64_t y_stride, uint32_t t0,
                         pf_estimate_t* est_dev, void* hip_stream);

/* Static description of a status code. */
const char* pf_status_string(pf_status s);

/* Last error message of the handle (never NULL; "" if none). With h == NULL
 * the message of the last failed pf_create of this thread. */
const char* pf_last_error(const pf_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* PF_H */
