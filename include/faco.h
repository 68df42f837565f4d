/*
 * faco.h -- C ABI of the MI355X Focused ACO (FACO) library.
 *
 * Method: R. Skinderowicz, "Improving Ant Colony Optimization Efficiency for
 * Solving Large TSP Instances" (Applied Soft Computing 2022, arXiv 2203.02228).
 *
 * Problem (Sec. 2.1): n cities 0..n-1 with symmetric positive costs; find a
 * minimum-cost Hamiltonian cycle.  Here the cost is TSPLIB EUC_2D,
 * nint(sqrt(dx^2 + dy^2)), on integer coordinates.  The result is a
 * permutation of 0..n-1 (the tour) and its integer cost.
 *
 * One call of faco_run_iterations advances the main loop of Alg. 2: every ant
 * builds a focused tour (Eq. (1) choice over candidate/backup lists until
 * min_new_edges edges differ from the source solution, remainder copied from
 * the source), improves it with the checklist local search of Alg. 3 (plus
 * Or-opt), then the colony picks the iteration best, updates the global best
 * and the trail limits (Sec. 4.5), chooses the next source and applies the
 * bounded pheromone update of Eq. (2).
 *
 * All state lives in device memory owned by the library.  Every call returns
 * FACO_OK (0) or a negative FACO_E* code; the message is available from
 * faco_last_error().  Distinct handles may be used from distinct host threads
 * concurrently; one handle must not be used by two threads at once.
 */
#ifndef FACO_H
#define FACO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FACO_OK 0
#define FACO_EINVAL (-1)  /* invalid argument                           */
#define FACO_EDUP (-2)    /* two cities share coordinates (zero cost)   */
#define FACO_ENOMEM (-3)  /* device or host allocation failed           */
#define FACO_EDEVICE (-4) /* HIP runtime / kernel launch error          */

/* local-search bits of faco_params.ls_flags */
#define FACO_LS_2OPT 1u  /* 2-opt moves of Alg. 3                         */
#define FACO_LS_OROPT 2u /* Or-opt segment insertion (not in the paper)   */
#define FACO_LS_SWEEP 4u /* re-examine every listed node until none improves */
#define FACO_LS_INIT_3OPT 8u /* the initial solution's search also tries 3-opt
                                (Sec. 4.3: nearest neighbour improved with
                                2-opt and 3-opt); ants never use it        */

/* Parameters (Table 1 of the paper; names follow it). */
typedef struct faco_params {
  int32_t cl_size;       /* candidate-list length (paper: 16); >= 2          */
  int32_t bl_size;       /* backup-list length (paper: 64); 0..64            */
  int32_t n_ants;        /* ants per iteration; 1..4096                       */
  int32_t min_new_edges; /* new edges before copying (paper: 8); >= 0        */
  float rho;             /* pheromone retention of Eq. (2); [0, 1)            */
  float reserved0;       /* must be 0                                         */
  double p_best;         /* Sec. 4.5 limit parameter; (0, 1); e.g. 0.05       */
  double p_source_gbest; /* probability that the source is the global best
                            (paper: 0.01, Sec. 5.3); [0, 1]                   */
  uint64_t seed;         /* Philox4x64-10 key word 0                          */
  uint32_t ls_flags;     /* FACO_LS_* bits                                    */
  int32_t oropt_max_seg; /* longest Or-opt segment; 1..3                      */
  int32_t min_new_edges_max; /* Alg. 2 calls calc_num_new_edges() once per ant;
                            0 (or min_new_edges): the constant min_new_edges
                            of Table 1; above min_new_edges: each ant draws its
                            threshold uniformly from [min_new_edges,
                            min_new_edges_max] (Philox counter (iteration,
                            ant, 0, 3))                                      */
  int32_t reserved1;     /* must be 0                                         */
} faco_params;

typedef struct faco_instance faco_instance;

/*
 * Build an instance (Alg. 2 before the main loop): candidate lists (cl_size
 * nearest cities by exact squared distance, ties by id) and backup lists (the
 * next bl_size), heuristic eta = 1/d, the initial solution (nearest neighbour
 * from city 0 improved by the local search over all cities), the trail limits,
 * tau = tau_max everywhere, source = initial solution.
 *   xy         host pointer, n rows of (x, y) int32, row-major; each
 *              coordinate in [0, 2^26) (squared lengths below 2^53, exact
 *              in binary64).  Copied; the caller keeps ownership.
 *   n          number of cities, 4 .. 262144 (2^18).
 *   p          parameters, copied.
 *   hip_stream hipStream_t to run on (NULL = the default stream).  The handle
 *              keeps using this stream for all later calls.
 *   out        receives the new handle on success.
 * Runs asynchronously on the stream but returns after setup has finished.
 * Errors: FACO_EINVAL, FACO_EDUP, FACO_ENOMEM, FACO_EDEVICE.
 */
int faco_build_instance(const int32_t *xy, int32_t n, const faco_params *p,
                        void *hip_stream, faco_instance **out);

/*
 * Enqueue `iterations` more iterations of Alg. 2's main loop on the handle's
 * stream and return without waiting.  The iteration counter persists, so two
 * calls of a and b iterations give exactly the state of one call of a + b.
 * Errors: FACO_EINVAL (iterations < 0 or NULL handle), FACO_EDEVICE.
 */
int faco_run_iterations(faco_instance *h, int32_t iterations);

/*
 * Wait for the handle's stream and copy the global-best tour (n int32 into
 * the caller's host buffer, exactly as stored: tour_out[0] is not rotated)
 * and its cost.  Either pointer may be NULL.
 * Errors: FACO_EINVAL; FACO_EDEVICE on a HIP error, or when the device
 * recorded a fault (FACO_DBG_FAULT; the outputs are still written).
 */
int faco_get_best_tour(faco_instance *h, int32_t *tour_out,
                       int64_t *length_out);

/*
 * Release all device state of the handle.  NULL is allowed.  Waits for the
 * handle's stream; the device blocks then go to a per-device cache of the
 * library (at most 32 GiB; beyond it they are freed) and later builds and
 * batch tables reuse them, because hipFree would wait for all work queued on
 * the device, every other stream's included.
 */
void faco_destroy_instance(faco_instance *h);

/*
 * Move the handle to another stream: later calls on it (iterations, batch
 * ordering, reads, destroy) run on and wait for `hip_stream` (NULL = the
 * default stream), after the handle's work already queued on its previous
 * stream.  A server that builds on a builder stream and then runs a solve on
 * its batch stream moves it there, so that the solve's batches and reads
 * never wait for other builds queued later on the builder stream.
 * Errors: FACO_EINVAL (NULL handle), FACO_EDEVICE.
 */
int faco_set_stream(faco_instance *h, void *hip_stream);

/* Last error message of the handle, or of the calling thread if h is NULL.
 * The string stays valid until the next call on the same handle/thread. */
const char *faco_last_error(const faco_instance *h);

/*
 * Advance several instances by `iterations` each in shared launches: one
 * kernel launch per phase covers the ants of every instance.  Each instance
 * ends in exactly the state a solo faco_run_iterations would give it.
 *   hs          host array of `count` handles, all distinct.
 *   hip_stream  stream for the shared launches (NULL = default); the call
 *               orders itself after each handle's own stream and the handles'
 *               later calls after it.
 * Returns after enqueue.  Errors: FACO_EINVAL, FACO_ENOMEM, FACO_EDEVICE.
 */
int faco_run_batch(faco_instance *const *hs, int32_t count, int32_t iterations,
                   void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): faco_run_batch
 * without allocation.  The same launches and results as faco_run_batch, but
 * the instance and ant tables live in a fixed array of 256 KiB that each
 * device holds until the process ends, no graph is captured and no event is
 * created; each iteration is launched directly.
 *   Limits: at most 256 instances and 16384 ants (all instances together)
 *   per call, else FACO_EINVAL.  Every handle must have been built on
 *   hip_stream (the call adds no cross-stream ordering) and on the current
 *   device, else FACO_EINVAL.
 *   Calls on one device share the array: calls that overlap on the device
 *   (different streams, or different host threads without ordering) race and
 *   must not be made; calls in order on one stream are safe.
 * Returns after enqueue.  Errors: FACO_EINVAL, FACO_EDEVICE.
 */
int faco_run_batch_noalloc(faco_instance *const *hs, int32_t count, int32_t iterations,
                           void *hip_stream);

/* How faco_run_batch launches a batch (execution shape only: no setting
 * changes a result). */
typedef struct faco_batch_config {
  int32_t persistent;         /* 1: one persistent launch runs every iteration
                                 of every instance; each instance's ants of
                                 the next iteration start as soon as its own
                                 colony and pheromone update is done
                                 (device-side phase counters per instance),
                                 largest tours first.  0: one launch per
                                 phase over all instances, one iteration
                                 captured as a HIP graph and replayed.
                                 Instances with verification on run per
                                 phase.                                     */
  int32_t team_waves;         /* waves per ant: 0 = by size (as for a lone
                                 instance, counting the batch's longest tour
                                 and all its ants), else 1, 4 or 8          */
  int32_t ants_per_block;     /* one-wave ants per workgroup: 1, 2 or 4,
                                 lowered when their LDS would not fit a CU  */
  int32_t queue_lds_capacity; /* LDS part of each ant's work queue: 0 = as
                                 built, else 64..16384                       */
  int32_t big_percent;        /* 0: one batch.  1..100: that share of the
                                 instances, longest tours first, runs as a
                                 sub-batch of its own (per phase, waves per
                                 ant big_team_waves) on a second stream
                                 beside the rest; the call stays ordered on
                                 hip_stream                                 */
  int32_t big_team_waves;     /* 1, 4 or 8 when big_percent > 0              */
} faco_batch_config;

/* The process-wide default configuration of faco_run_batch (initially per
 * phase, sizes by the library's rule, one ant per workgroup, queues as
 * built).  Setting it forgets the configurations faco_autotune_batch
 * stored.  Errors: FACO_EINVAL. */
int faco_set_batch_config(const faco_batch_config *config);
int faco_get_batch_config(faco_batch_config *config);

/* Autotuner: times faco_run_batch over `trial_iterations` iterations with
 * each candidate configuration (per phase with 1/4/8 waves per ant, 1/2 ants
 * per workgroup for one-wave ants, LDS queue capacity as built or 2048;
 * persistent with 4/8-wave teams; the largest 10/15/20/30% of the instances
 * split off with 4- or 8-wave teams) on twins of the handles built from their
 * own inputs (the handles do not advance).  Each candidate first runs one
 * untimed iteration (first launches, streams, tables); then, in each of
 * three rounds (one if trial_iterations < 3) a third of trial_iterations
 * apart by 5x that many untimed iterations, every device block of the twins
 * is copied aside and copied back before each candidate's trial, so that all
 * candidates of a round run the same iterations from the same state (the
 * copy takes device memory the size of the twins); keeps the fastest total,
 * and stores it
 * for the batch's size class (the longest tour's power of two): later
 * faco_run_batch calls use the stored configuration of their own class,
 * else of the nearest stored one.  best_out (may be NULL) receives it.  Synchronises hip_stream.
 * Errors: FACO_EINVAL, FACO_ENOMEM, FACO_EDEVICE. */
int faco_autotune_batch(faco_instance *const *hs, int32_t count, int32_t trial_iterations,
                        void *hip_stream, faco_batch_config *best_out);

/* Ants per workgroup of the default configuration (1, 2 or 4).
 * Errors: FACO_EINVAL. */
int faco_set_batch_ants_per_block(int32_t ants_per_block);

/* Waves per ant in the ant kernels, for instances built after the call and
 * for faco_run_batch launches after it (process-wide): 1, 4 or 8, or 0 for a
 * choice by size (1 below 2048 cities; else 8 up to 256 ants, 4 up to 512,
 * 1 beyond; a batch counts its largest tour and all its ants).  Wave 0 of an
 * ant makes every decision; the others share its wide steps (speculative
 * source-following windows of 64 steps per wave, the array rewrites of 2-opt
 * and Or-opt moves, sweep tests).  An execution-shape choice that never
 * changes results.  Errors: FACO_EINVAL. */
int faco_set_team_waves(int32_t team_waves);

/* Capacity (entries) of the LDS part of each ant's work queue of listed
 * cities, for instances built after the call (process-wide): 0 for the
 * default 16384, else 64..16384; an instance uses min(n, capacity).  A queue
 * that outgrows it continues in global memory.  An execution-shape choice
 * that never changes results.  Errors: FACO_EINVAL. */
int faco_set_queue_lds_capacity(int32_t capacity);

/* How the local search of faco_run_iterations holds each ant's tour, for
 * instances built after the call (process-wide).  Sec. 4.4: a 2-opt flip on
 * an array rewrites O(n) elements.  With segment lists the tour is the array
 * of the last materialisation read through up to max_records records in LDS
 * (a storage range, its orientation, the array position of its first
 * element); a move splits at most three records and rewrites the records
 * inside its range, and when the records run short the tour is written out
 * in array order (materialised) and cut again into segments of
 * 2^length_log2 cities.  Array positions, and so every rule that depends on
 * them, are exactly those of the flat arrays: results never change.
 *   mode: 0 (the default) or 1 flat arrays, 2 segment lists.
 *   length_log2: 0 for the smallest power of two >= 64 that cuts the tour
 *         into at most 512 segments, else 1..24.
 *   max_records: 0 for 2048, else 8..2048; it must exceed the tour's
 *         segment count by 4 (checked at build: FACO_EINVAL).
 * Segment lists take 24 n bytes more per ant (a second array buffer and a
 * record label per city).  faco_run_batch and the initial solution always
 * use flat arrays.  Errors: FACO_EINVAL. */
int faco_set_tour_segments(int32_t mode, int32_t length_log2, int32_t max_records);

/* Debug / test dumps of the state after the last completed iteration.  Sync,
 * then copy `bytes` bytes into the host buffer `out`; `bytes` must equal the
 * size given below, otherwise FACO_EINVAL. */
enum {
  FACO_DBG_ANT_ROUTES = 0,   /* int32 [n_ants][n]; all -1 before iteration 1 */
  FACO_DBG_ANT_LENGTHS = 1,  /* int64 [n_ants]                               */
  FACO_DBG_PHEROMONE = 2,    /* float [n][k_eff]                             */
  FACO_DBG_SOURCE = 3,       /* int32 [n]                                    */
  FACO_DBG_LIMITS = 4,       /* float [3]: tau_min, tau_max, last delta      */
  FACO_DBG_COUNTERS = 5,     /* int64 [n_ants][FACO_NCNT]                    */
  FACO_DBG_CAND_LISTS = 6,   /* int32 [n][k_eff]                             */
  FACO_DBG_BACKUP_LISTS = 7, /* int32 [n][bl_eff]                            */
  FACO_DBG_HEURISTIC = 8,    /* float [n][k_eff]                             */
  FACO_DBG_INFO = 9,         /* int64 [8]: iterations, k_eff, bl_eff, last
                                iteration-best ant, last source was gbest,
                                initial length, gbest length, source length  */
  FACO_DBG_INIT_COUNTERS = 10, /* int64 [FACO_NCNT] of the initial solution  */
  FACO_DBG_COUNTER_TOTALS = 11, /* int64 [n_ants][FACO_NCNT], summed over all
                                   iterations since the build                 */
  FACO_DBG_PHASE_TICKS = 12, /* int64 [n_ants][32] summed since the build;
                               device wall-clock ticks (100 MHz): [0]
                               construction, [1] move evaluation, [2] move
                               application, [3] sweeps, [4] whole ant, [8]
                               speculative windows, [9] one-step choices,
                               [10] copies, [11] backup/nearest choices; call
                               counts: [5] windows, [6] one-step choices, [7]
                               copies, [12] evaluation rounds, [13] ticks
                               in Or-opt evaluation, [14] rounds that
                               evaluated Or-opt, [15] ticks in the array
                               rewrites of moves (part of [2]); segment
                               lists: [16] materialisations, [17] ticks in
                               them, [18] cities relabelled by splits, [19]
                               splits, [20] records passed by moves, [21]
                               ticks of the leader's part of moves, [22]
                               ticks of the team's part; sweeps: [24] ticks
                               in the move tests, [25] ticks in listing the
                               improvable cities, [26] cities tested;
                               [23], [27..31] zero                       */
  FACO_DBG_TEAM_WAVES = 13, /* int32 [1]: waves per ant of this instance   */
  FACO_DBG_FAULT = 14,      /* int64 [4]: FACO_FAULT_* bits found on the
                               device, the first fault's ant (-1: initial
                               solution or global best) and iteration, and
                               the number of tours verified so far           */
  FACO_DBG_RECOMPUTED_LENGTHS = 15, /* int64 [n_ants + 1]: runs the tour-length
                               verification now (Alg. 2's select_shortest
                               relies on the lengths) and returns every ant's
                               tour length recomputed from its stored route
                               and the coordinates, then the global best's;
                               -1 for an ant route that is not a permutation;
                               0 for the ants before the first iteration.
                               A mismatch with the tracked lengths sets a
                               fault.                                         */
  FACO_DBG_TOUR = 16,       /* int64 [3]: segment lists in use (0/1), their
                               segment length, the record limit              */
  FACO_DBG_INIT_TICKS = 17  /* int64 [32]: the initial solution's tick slots
                               and call counts, as FACO_DBG_PHASE_TICKS for
                               one ant (slot 4: the whole kernel; set with the
                               3-opt initial search too, which runs after)   */
};
/* device faults (FACO_DBG_FAULT; faco_get_best_tour then returns
 * FACO_EDEVICE) */
#define FACO_FAULT_LS_STALL 1    /* local search stopped early: cities a sweep
                                    listed had no move in the evaluation    */
#define FACO_FAULT_LENGTH 2      /* recomputed length != tracked length      */
#define FACO_FAULT_PERMUTATION 4 /* an ant route is not a permutation        */
#define FACO_FAULT_BATCH_STALL 8 /* a persistent batch saw no progress       */
/* per-ant counters (same meaning as the oracle's) */
enum {
  FACO_CNT_ACO_STEPS = 0,
  FACO_CNT_COPIED,
  FACO_CNT_BACKUP,
  FACO_CNT_FALLBACK,
  FACO_CNT_NEW_EDGES,
  FACO_CNT_LS_POPS,
  FACO_CNT_MOVES_2OPT,
  FACO_CNT_MOVES_OROPT,
  FACO_CNT_MOVED_ELEMS,
  FACO_CNT_SWEEPS,
  FACO_CNT_CHECKLIST0,
  FACO_CNT_LS_GAIN,
  FACO_CNT_MOVES_3OPT,   /* 3-opt moves (initial solution only)          */
  FACO_NCNT
};
int faco_debug_get(faco_instance *h, int32_t what, void *out, size_t bytes);

/* Device bytes the instance holds (coordinates, lists, pheromone, tours,
 * per-ant scratch), for admission by footprint.  Pure arithmetic; valid
 * without a GPU.  Returns 0 for invalid arguments. */
uint64_t faco_footprint_bytes(int32_t n, const faco_params *p);

/* Tour-length verification in every iteration (Alg. 2's select_shortest
 * compares the tracked lengths): when enabled, each iteration of
 * faco_run_iterations and faco_run_batch also recomputes every ant's tour
 * length and the global best's from the stored tours and the coordinates
 * (exact int64 sums), checks each ant route against its inverse, and records
 * a fault on any mismatch (FACO_DBG_FAULT; faco_get_best_tour then fails).
 * Off by default.  Errors: FACO_EINVAL. */
int faco_set_verify(faco_instance *h, int32_t enable);

/* Kernel timing.  When enabled, each phase launch of faco_run_iterations is
 * bracketed by HIP events on the handle's stream (enable > 1 also creates
 * the events of that many iterations at once, so that none is created while
 * the timed iterations are enqueued; events are reused after
 * faco_phase_times).  faco_phase_times syncs and
 * returns, per phase (0 = ants: construction + local search, 1 = colony
 * update, 2 = source materialisation, 3 = pheromone update), the summed
 * milliseconds in ms_out[phase] and the launch count in launches[phase]. */
int faco_set_timing(faco_instance *h, int32_t enable);
int faco_phase_times(faco_instance *h, double *ms_out /* [4] */,
                     int64_t *launches /* [4] */);

#ifdef __cplusplus
}
#endif
#endif
