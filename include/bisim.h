/*
 * bisim.h — C ABI of the MI355X (gfx950) strong-bisimulation library.
 *
 * The library computes the relational coarsest partition of a labelled
 * transition system: the coarsest refinement of an initial partition pi_0
 * whose induced relation is a strong bisimulation (section 2, the BCRP and
 * RCPP problem statements; Definition 2).  It runs the labelled PRAM
 * refinement of section 4 (Algorithm 3) on the GPU: preprocessing
 * (section 4.1: per-state action slots, Algorithm 4's split by outgoing
 * action sets), then repeated iterations of
 *     select splitter C  ->  mark (state, action) slots whose transition
 *     targets C  ->  tag states whose marks differ from their block leader's
 *     ->  elect the smallest tagged state per block as the new leader  ->
 *     relabel tagged states and update the unstable set,
 * until no block is unstable.
 *
 * Concurrent writes are resolved by priority (section 2.1's priority CRCW
 * rule): the splitter is the smallest unstable block label and the new leader
 * of a split-off part is its smallest state.  Under that rule every block
 * label is the smallest member of its block, so results are canonical
 * (block id = smallest member) and the iteration count is deterministic.
 *
 * Conventions
 *   - Pointers documented as "device" are GPU global-memory pointers on the
 *     device that is current when the call is made; "host" pointers are CPU
 *     memory.  Nothing crosses the ABI as an exception.
 *   - All work is enqueued on the hip_stream given at load time (NULL = the
 *     default stream).  Calls that return results to the host synchronise
 *     that stream.
 *   - The caller owns every buffer it passes.  Input buffers may be freed once
 *     the loading call has returned.  A handle owns its device working set
 *     until it is freed.
 *   - On error a negative status is returned, outputs are unspecified, a
 *     failed load leaves *out == NULL, and bisim_last_error() describes the
 *     failure.  A handle stays usable after a failed call on it.
 *   - A handle must not be used from two threads at once.
 */
#ifndef BISIM_H
#define BISIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bisim_status;
#define BISIM_OK 0
#define BISIM_E_INVALID -1     /* NULL pointer where one is required, n < 0, m < 0,
                                  num_actions < 1, unknown option */
#define BISIM_E_RANGE -2       /* src/dst outside [0,n), label outside [0,K),
                                  init_partition value outside [0,n) */
#define BISIM_E_NOMEM -3       /* device or host allocation failed */
#define BISIM_E_DEVICE -4      /* HIP runtime error */
#define BISIM_E_ITERCAP -5     /* iteration count exceeded 3n - |pi_pre| + 1, the bound of
                                  section 4.2's complexity theorem plus the final pass;
                                  reachable only through the test hook below */
#define BISIM_E_UNSUPPORTED -6 /* sizes beyond the documented limits, or an option the
                                  input does not allow */

typedef struct bisim_lts bisim_lts;

typedef struct {
  int64_t iterations;  /* executions of the while-loop body, counting the final pass
                          that finds no splitter (Table 1's #It) */
  int64_t blocks;      /* blocks of the result */
  int64_t pre_blocks;  /* blocks after preprocessing (the partition the loop starts from) */
  int64_t mark_length; /* total number of (state, action) mark slots (section 4.1) */
  double t_pre_ms;     /* lts_load device time: validation, preprocessing, layout */
  double t_alg_ms;     /* refinement-loop device time of the last coarsest_partition */
} bisim_stats;

/*
 * lts_load — validate an LTS and build its device working set
 * (section 4.1 preprocessing).
 *   src, label, dst   device, m entries each: transition i is
 *                     src[i] -label[i]-> dst[i]; any order, duplicates and
 *                     self-loops allowed (section 2, Definition 1).
 *   n                 number of states, 0 <= n < 2^31 - 1.
 *   m                 number of transitions, 0 <= m < 2^32 - 1.
 *   num_actions       K >= 1; labels lie in [0, K).
 *   init_partition    device, n entries, or NULL for pi_0 = {S}.  States with
 *                     equal values share an initial block; values must lie in
 *                     [0, n) (block labels are state indices, section 3.2).
 *                     A Kripke structure is num_actions = 1 plus the
 *                     partition by atomic propositions.
 *   hip_stream        hipStream_t to enqueue on, or NULL.
 *   out               host; receives the handle, or NULL on failure.
 * Errors: BISIM_E_INVALID, BISIM_E_RANGE, BISIM_E_NOMEM, BISIM_E_DEVICE,
 * BISIM_E_UNSUPPORTED.
 */
bisim_status lts_load(const int32_t* src, const int32_t* label, const int32_t* dst, int32_t n,
                      int64_t m, int32_t num_actions, const int32_t* init_partition,
                      void* hip_stream, bisim_lts** out);

/*
 * coarsest_partition — run the refinement loop (Algorithm 3) from the
 * preprocessed partition to the fixpoint and write the result.
 *   block_id   device, n entries: block_id[s] = smallest state bisimilar to s
 *              (within the same initial block).
 *   st         host, nullable: statistics of this run.
 * May be called repeatedly on one handle; every call restarts from the
 * preprocessed partition and gives identical results.
 * Errors: BISIM_E_INVALID, BISIM_E_DEVICE, BISIM_E_ITERCAP.
 */
bisim_status coarsest_partition(bisim_lts* h, int32_t* block_id, bisim_stats* st);

/* lts_free — release a handle and its device memory (NULL is a no-op). */
void lts_free(bisim_lts* h);

/*
 * coarsest_partition_noalloc — lts_load + coarsest_partition + lts_free in
 * one call that allocates no device or pinned host memory, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Loading and refinement run the same
 * kernels as the handle-based calls (plain splitter policy, Algorithm 3,
 * default engine), with all their working memory taken from one static
 * device region of BISIM_NOALLOC_SCRATCH_BYTES per GPU, held from the first
 * call on that GPU until the process ends.
 *   src, label, dst, n, m, num_actions, init_partition, hip_stream
 *                 as for lts_load (device pointers; inputs are only read).
 *   block_id      device, n entries: the result, as for coarsest_partition.
 *   st            host, nullable: statistics (t_pre_ms = loading time).
 * Size limit: the call needs at most about 16m + 100n + 8K bytes plus a few
 * KiB (an exact upper bound is computed from n, m and K before any work);
 * inputs beyond BISIM_NOALLOC_SCRATCH_BYTES are rejected with
 * BISIM_E_UNSUPPORTED before anything is enqueued.
 * The region keeps the last call's contents; every buffer is initialised by
 * the call that uses it.  All calls on one GPU share the region: calls that
 * overlap on one GPU (other host threads, other streams) race and must not
 * be made.  Returns after synchronising hip_stream.
 * Errors: BISIM_E_INVALID, BISIM_E_RANGE, BISIM_E_UNSUPPORTED, BISIM_E_DEVICE,
 * BISIM_E_ITERCAP.
 */
#define BISIM_NOALLOC_SCRATCH_BYTES (64ll << 20)
bisim_status coarsest_partition_noalloc(const int32_t* src, const int32_t* label,
                                        const int32_t* dst, int32_t n, int64_t m,
                                        int32_t num_actions, const int32_t* init_partition,
                                        int32_t* block_id, bisim_stats* st, void* hip_stream);

/* bisim_last_error — text for the last failure on the calling thread; valid
   until the next library call on that thread.  Never NULL. */
const char* bisim_last_error(void);

/*
 * bisim_set_option — per-handle settings.
 *   BISIM_OPT_ENGINE        0 = automatic (default: engine 2 for LTSs under
 *                           200,000 states, the learned policy, Algorithm 2,
 *                           traced or limited runs; otherwise the fastest of
 *                           engines 2 and 3 at a few grid sizes, timed on the
 *                           LTS's first 96 iterations once per device and size
 *                           class and cached in the file BISIM_TUNE_CACHE, else
 *                           $HOME/.cache/bisim_tune.txt), 1 = one cooperative persistent
 *                           launch per fixpoint (grid barriers between
 *                           phases), 2 = one kernel per phase, launched in
 *                           batches with a device-side done flag, each
 *                           scanning all states, 3 = three kernels per
 *                           iteration over member lists (a refinable
 *                           partition): work per iteration follows the
 *                           splitter's members and in-transitions and the
 *                           states they touch, not n; Algorithm 3 with the
 *                           plain policy only (else BISIM_E_UNSUPPORTED at
 *                           coarsest_partition); about 96 more bytes of
 *                           device memory per state, allocated on first use.
 *   BISIM_OPT_COUNT_WORK    0 (default) or 1: engine 3 accumulates work totals
 *                           over the run (bisim_get_work).
 *   BISIM_OPT_FIRST_SPLITTER  -1 (default) or a block label of the
 *                           preprocessed partition to use as the first
 *                           splitter instead of the smallest (test hook, used
 *                           to replay Figure 1).
 *   BISIM_OPT_ITER_LIMIT    0 (default: 3n - |pi_pre| + 1) or a smaller cap
 *                           (test hook for the BISIM_E_ITERCAP path).
 *   BISIM_OPT_GRID          0 (default: fill the device) or a workgroup count
 *                           for the persistent engine / per-phase kernels.
 * Errors: BISIM_E_INVALID.
 */
#define BISIM_OPT_ENGINE 1
#define BISIM_OPT_FIRST_SPLITTER 2
#define BISIM_OPT_ITER_LIMIT 3
#define BISIM_OPT_GRID 4
#define BISIM_OPT_PROFILE_EVERY 5 /* 0 (default) or P: with the per-phase engine, time the
                                     phase kernels of every P-th iteration (at most 256
                                     iterations per run) with events bound to the end of
                                     each kernel; a phase's time is the distance between
                                     the ends of consecutive kernels of the stream */
#define BISIM_OPT_COUNT_WORK 7
#define BISIM_OPT_ALGORITHM 6     /* 3 (default): the labelled algorithm (Algorithm 3, with
                                     section 4.1's preprocessing); 2: the algorithm for the
                                     relational coarsest partition problem (section 3.2,
                                     Algorithm 2) — one-action LTSs (Kripke structures)
                                     only (else BISIM_E_UNSUPPORTED): it starts from the
                                     leader-normalised pi_0 without preprocessing, keeps
                                     one mark per state, and does not make the splitter
                                     unstable again after a split.  Same result, its own
                                     iteration count; the plain policy only.
                                     BISIM_ALGORITHM_SIGNATURE: multi-way signature
                                     refinement, the signature-based splitting of the
                                     systems the paper compares against (section 5), an
                                     in-house baseline: from pi_pre, every round regroups
                                     the states by (block, {(action, block of target)})
                                     until a round changes nothing; iterations = rounds.
                                     Set hashes, checked at the fixpoint with a second
                                     independent hash (BISIM_E_DEVICE if three seeds
                                     fail); no splitter policy or trace
                                     (BISIM_E_UNSUPPORTED), m < 2^31 and (distinct
                                     actions per state) * n < 2^32 (else
                                     BISIM_E_UNSUPPORTED).  Device memory: 20 bytes per
                                     transition and 48 per state, plus the radix sort's
                                     scratch (about 9 bytes per transition and 13 per
                                     state) and, up to 4M states, a grouping table of
                                     24 to 48 bytes per state; a run of more than four
                                     rounds adds 37 bytes per transition and 4 per state
                                     (the transitions laid out by source) and up to 32
                                     bytes per transition of a state with more than 64
                                     (a duplicate table).  The handle keeps this memory from
                                     its first signature or hybrid run until lts_free, so
                                     later runs allocate nothing.
                                     BISIM_ALGORITHM_HYBRID: signature rounds while they
                                     split many blocks, then Algorithm 3 (multi-way
                                     splitting combined with the linear bound, left as
                                     future work in section 6): the rounds stop at the
                                     fixpoint, or after two consecutive rounds that each
                                     add fewer than 64 blocks, and Algorithm 3 (plain
                                     policy) continues from the partition reached with
                                     every block unstable.  iterations = rounds +
                                     Algorithm 3 iterations; limits and errors as for
                                     BISIM_ALGORITHM_SIGNATURE. */
#define BISIM_ALGORITHM_RCPP 2
#define BISIM_ALGORITHM_LABELLED 3
#define BISIM_ALGORITHM_SIGNATURE 100
#define BISIM_ALGORITHM_HYBRID 101
bisim_status bisim_set_option(bisim_lts* h, int32_t option, int64_t value);

/*
 * bisim_get_phase_times — after a run with BISIM_OPT_PROFILE_EVERY > 0:
 * average kernel execution time in ms (avg_ms, host, 4 entries) over the
 * sampled iterations that had a splitter, and the number of samples per
 * phase (samples, host, 4 entries).  Engine 2: select+relabel+mark and
 * compare+elect (the learned policy: select+mark, compare+elect, relabel,
 * re-score); engine 3: select+mark, compare+elect (+ the next splitter's
 * prefetch), split (relabel, swaps, ranges); unused entries are 0.
 * Errors: BISIM_E_INVALID.
 */
bisim_status bisim_get_phase_times(bisim_lts* h, double* avg_ms, int64_t* samples);

/*
 * bisim_get_work — work totals of the last run with BISIM_OPT_COUNT_WORK set
 * (engine 3): out (host, 8 entries) = members of the splitters, their
 * in-transitions, touched states, listed member segments, members visited
 * of leader-touched blocks that have an untouched member, split states,
 * split blocks, iterations in which something split.  Zeros for other
 * engines.
 * Errors: BISIM_E_INVALID.
 */
bisim_status bisim_get_work(bisim_lts* h, int64_t* out);

/*
 * bisim_get_run_config — engine (1, 2 or 3) and workgroup count of the last
 * coarsest_partition on h (what BISIM_OPT_ENGINE = 0 resolved to); 0s before
 * the first run.  Errors: BISIM_E_INVALID.
 */
bisim_status bisim_get_run_config(bisim_lts* h, int32_t* engine, int32_t* grid);

/*
 * bisim_set_trace — record, for each iteration k < cap of subsequent
 * coarsest_partition calls:
 *   trace_C[k]        the splitter label (-1 for the final pass);
 *   trace_nsplit[k]   the number of states split off (nullable);
 *   trace_work[4k..]  (nullable) the members of the splitter, its
 *                     in-transitions, the states they touch, and whether a
 *                     touched state was a block leader (0/1) — the
 *                     data-dependent terms of the iteration's memory traffic.
 * All device buffers with cap (trace_work: 4 * cap) entries.  cap = 0
 * disables tracing.
 * Errors: BISIM_E_INVALID.
 */
bisim_status bisim_set_trace(bisim_lts* h, int32_t* trace_C, int64_t* trace_nsplit,
                             int64_t* trace_work, int64_t cap);

/*
 * bisim_get_preprocessed — copy the preprocessed partition pi_pre
 * (section 4.1, Algorithm 4: pi_0 split by outgoing action sets, canonical)
 * into block_id (device, n entries), and optionally nr_marks (device, n
 * entries: number of distinct outgoing actions per state).
 * Errors: BISIM_E_INVALID, BISIM_E_DEVICE.
 */
bisim_status bisim_get_preprocessed(bisim_lts* h, int32_t* block_id, int32_t* nr_marks);

/*
 * bisim_get_preprocess_method — how lts_load computed pi_pre and the action
 * ranks (section 4.1): *method (host) = 0 for Algorithm 4's rounds, one per
 * action; 1 for the one-pass kernels (more than 64 actions and at most 64
 * outgoing transitions per state: each state's distinct actions ranked and
 * its action set hashed in one pass, states grouped by (pi_0 block, hash),
 * every group checked exactly against its smallest state, the rounds run if
 * the check fails).  Both give the same partition, ranks and counts.  Test
 * hook: with the environment variable BISIM_ONEPASS_COLLIDE=1 at lts_load,
 * every state's key collides, so the check fails (unless all states agree)
 * and the rounds run.
 * Errors: BISIM_E_INVALID.
 */
bisim_status bisim_get_preprocess_method(bisim_lts* h, int32_t* method);

/* ------------------------------------------------------------------------ */
/* Batched refinement: many independent LTSs in one launch                   */
/* ------------------------------------------------------------------------ */
/*
 * The refinement of each instance is the same Algorithm 3 run as above (same
 * preprocessing, splitter order and iteration count as a single-instance
 * run of that instance); instances are refined concurrently, one workgroup
 * per instance, with per-instance fixpoint detection.
 */
typedef struct bisim_batch bisim_batch;

typedef struct {
  int64_t max_iterations;   /* largest per-instance #It */
  int64_t sum_iterations;   /* sum of per-instance #It */
  int64_t lds_instances;    /* instances refined with LDS-resident state */
  int64_t global_instances; /* instances refined with state in global memory */
  int32_t workgroup_size;   /* threads per workgroup used */
  int32_t grid;             /* workgroups launched */
  double t_pre_ms;          /* lts_batch_load device time */
  double t_alg_ms;          /* device time of the last coarsest_partition_batch */
  int64_t work[2][8];       /* work totals of the last run over all instances:
                               [0] LDS-resident instances: iterations, splitter
                               members, their in-transitions, touched states, -,
                               split states, -, instances;
                               [1] member-list instances: iterations, splitter
                               members, their in-transitions, touched states,
                               touched leaders listed, members of their blocks
                               visited, split states, split blocks */
} bisim_batch_stats;

/*
 * lts_batch_load — validate and preprocess `count` LTSs stored back to back.
 *   count           number of instances, >= 1.
 *   n_off, m_off    host, count + 1 entries each, non-decreasing from 0:
 *                   instance k owns states [n_off[k], n_off[k+1]) of the
 *                   concatenation and transitions [m_off[k], m_off[k+1]).
 *                   Totals: n_off[count] < 2^31 - 1, m_off[count] < 2^32 - 1.
 *   src, label, dst device, m_off[count] entries: instance-local ids
 *                   (src, dst in [0, n_k), label in [0, num_actions[k])).
 *   num_actions     host, count entries, each >= 1.
 *   init_partition  device, n_off[count] entries of instance-local values in
 *                   [0, n_k), or NULL for pi_0 = {S_k} in every instance.
 *   hip_stream, out as for lts_load.
 * Errors: BISIM_E_INVALID, BISIM_E_RANGE, BISIM_E_NOMEM, BISIM_E_DEVICE,
 * BISIM_E_UNSUPPORTED (a state with more than 64 distinct outgoing actions).
 */
bisim_status lts_batch_load(int32_t count, const int64_t* n_off, const int64_t* m_off,
                            const int32_t* src, const int32_t* label, const int32_t* dst,
                            const int32_t* num_actions, const int32_t* init_partition,
                            void* hip_stream, bisim_batch** out);

/*
 * coarsest_partition_batch — refine every instance to its fixpoint.
 *   block_id    device, n_off[count] entries: instance-local canonical ids
 *               (block_id[n_off[k] + s] = smallest state of instance k
 *               bisimilar to s).
 *   iterations  host, nullable, count entries: each instance's #It.
 *   st          host, nullable.
 * Errors: BISIM_E_INVALID, BISIM_E_DEVICE, BISIM_E_ITERCAP.
 */
bisim_status coarsest_partition_batch(bisim_batch* b, int32_t* block_id, int64_t* iterations,
                                      bisim_batch_stats* st);

/* lts_batch_free — release a batch handle (NULL is a no-op). */
void lts_batch_free(bisim_batch* b);

/*
 * bisim_batch_set_option — per-batch settings.
 *   BISIM_BOPT_WG_SIZE     0 (default) or 256: the one size the kernel is built for.
 *   BISIM_BOPT_GRID        0 (default: autotuned) or a workgroup count.
 *   BISIM_BOPT_LDS_LIMIT   0 (default: the device's per-workgroup LDS) or a
 *                          smaller byte budget; instances whose state does
 *                          not fit are refined from global memory.
 *   BISIM_BOPT_TUNE        1 = re-run the autotuner on the next call even if
 *                          a cached choice exists.
 * Errors: BISIM_E_INVALID.
 */
#define BISIM_BOPT_WG_SIZE 1
#define BISIM_BOPT_GRID 2
#define BISIM_BOPT_LDS_LIMIT 3
#define BISIM_BOPT_TUNE 4
bisim_status bisim_batch_set_option(bisim_batch* b, int32_t option, int64_t value);

/* ------------------------------------------------------------------------ */
/* Learned splitter priority                                                 */
/* ------------------------------------------------------------------------ */
/*
 * Algorithm 3 is correct for any choice of the unstable splitter C (the
 * concurrent write of section 3.2 may be won by any block; Theorem 1 and the
 * labelled argument of section 4.2 do not depend on it), so the splitter
 * order can be chosen to cut the iteration count without changing the
 * result.  The learned policy scores each unstable block with a small network
 *     y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3,   hidden width 64,
 * (trained to predict log(1 + number of blocks the splitter would split)),
 * quantises the score into 16 priority levels, floor(3y) clamped to 0..15,
 * and picks C = the smallest label of the highest non-empty level.  Features
 * x (19 values; the first 18 log1p-scaled):
 *     x[0]      block size
 *     x[1..8]   outgoing transitions of the members, by label mod 8
 *     x[9..16]  incoming transitions of the members, by label mod 8
 *     x[17]     iterations since the block was created or last split
 *     x[18]     1 if the block has been the splitter since it was created or
 *               last split, else 0.
 * Parameters are fp32 masters with bf16 copies used by the forward pass
 * (inputs also rounded to bf16, fp32 accumulation).  Levels are refreshed for
 * both blocks of every split and for the splitter in each iteration, and for
 * all unstable blocks every R iterations.
 */
typedef struct bisim_mlp bisim_mlp;

/* parameter count for `in_features` inputs (1..32), or -1 */
int64_t mlp_num_params(int32_t in_features);

/*
 * mlp_create — a network on the current device.
 *   init_fp32   host, mlp_num_params(in_features) values in the order
 *               W1 (row-major [64][F]), b1 [64], W2 ([64][64]), b2 [64],
 *               w3 [64], b3; or NULL for He-normal weights (seeded by `seed`)
 *               and zero biases.
 * Errors: BISIM_E_INVALID, BISIM_E_NOMEM, BISIM_E_DEVICE.
 */
bisim_status mlp_create(int32_t in_features, const float* init_fp32, uint64_t seed,
                        bisim_mlp** out);
void mlp_free(bisim_mlp* w);
/* copy the fp32 master parameters to host memory (mlp_num_params floats) */
bisim_status mlp_get_params(const bisim_mlp* w, float* host_fp32);

/*
 * mlp_forward — y[r] = network(x[r]) for r < rows.
 *   x device fp32 [rows][F] (row-major); y device fp32 [rows].
 * The forward pass computes with bf16 inputs: each x value is rounded to
 * bf16 (nearest even) in the kernel, so fp32 features (what the refinement
 * engines and the training-data collector produce) need no separate
 * conversion pass; mlp_forward_bf16 takes inputs already in bf16.
 * Synchronises hip_stream.  Errors: BISIM_E_INVALID, BISIM_E_DEVICE.
 */
bisim_status mlp_forward(const bisim_mlp* w, const float* x, int64_t rows, float* y,
                         void* hip_stream);

/*
 * mlp_forward_bf16 — as mlp_forward with x device bf16 [rows][F] (IEEE
 * bfloat16 bit patterns, row-major); y device fp32 [rows].  Results equal
 * mlp_forward's on the fp32 values of the same bf16 numbers.
 * Synchronises hip_stream.  Errors: BISIM_E_INVALID, BISIM_E_DEVICE.
 */
bisim_status mlp_forward_bf16(const bisim_mlp* w, const void* x_bf16, int64_t rows, float* y,
                              void* hip_stream);

/*
 * mlp_train_step — one full-batch step on rows (x, target):
 * loss = mean over rows of (y - target)^2; gradients w.r.t. the bf16
 * parameter copies; then an Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * learning rate lr; lr = 0 computes gradients only) on the fp32 masters and
 * a refresh of the bf16 copies.
 *   x device fp32 [rows][F]; target device fp32 [rows];
 *   loss_out host, nullable: the loss before the update;
 *   grad_out device, nullable: the gradient (mlp_num_params floats).
 * Synchronises hip_stream.  Errors: BISIM_E_INVALID, BISIM_E_DEVICE.
 */
bisim_status mlp_train_step(bisim_mlp* w, const float* x, const float* target, int64_t rows,
                            float lr, float* loss_out, float* grad_out, void* hip_stream);

/*
 * bisim_set_splitter_policy — 0: the smallest unstable label (default);
 * 1: the learned score (`w` must have 19 inputs and outlive the handle's
 * runs).  rescore_every: full re-scoring period R (>= 1).
 * Errors: BISIM_E_INVALID.
 */
bisim_status bisim_set_splitter_policy(bisim_lts* h, int32_t policy, const bisim_mlp* w,
                                       int32_t rescore_every);

/*
 * bisim_collect_training — run the plain policy to the fixpoint and, before
 * every `sample_every`-th iteration, evaluate up to `max_cands` unstable
 * blocks (evenly spaced in label order): their 19 features (as above) and
 * the counterfactual target log(1 + number of blocks that would split if
 * that block were the splitter now).
 *   feat device fp32 [cap][19]; target device fp32 [cap];
 *   meta device int32 [cap][2], nullable: (iteration, block label) per row;
 *   rows host: rows written (<= cap).
 * Supports states with at most 64 distinct outgoing actions and
 * n <= 16384.  Errors: BISIM_E_INVALID, BISIM_E_UNSUPPORTED, BISIM_E_DEVICE.
 */
bisim_status bisim_collect_training(bisim_lts* h, int64_t sample_every, int32_t max_cands,
                                    float* feat, float* target, int32_t* meta, int64_t cap,
                                    int64_t* rows);

/* ------------------------------------------------------------------------ */
/* Measurement                                                               */
/* ------------------------------------------------------------------------ */
/*
 * bisim_device_copy — copy `bytes` (a multiple of 16, 16-byte aligned device
 * pointers) with a plain streaming kernel and report its device time in ms
 * (ms_out, host, nullable).  Used to measure the bandwidth the device
 * sustains and to calibrate memory-traffic counters; not part of the method.
 * Errors: BISIM_E_INVALID, BISIM_E_DEVICE.
 */
bisim_status bisim_device_copy(void* dst, const void* src, int64_t bytes, void* hip_stream,
                               double* ms_out);

#ifdef __cplusplus
}
#endif

#endif /* BISIM_H */
