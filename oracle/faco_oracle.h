/*
 * faco_oracle.h -- plain, slow CPU oracle for Focused ACO (FACO).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP path of
 * the package.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no source with the GPU library.
 *
 * Paper: R. Skinderowicz, "Improving Ant Colony Optimization Efficiency for
 * Solving Large TSP Instances", Applied Soft Computing 2022 (arXiv 2203.02228).
 * Alg. 2 (FACO main loop), Alg. 3 (2-opt with checklist), Eq. (1) (choice
 * rule), Eq. (2) (bounded pheromone update), Sec. 4.5 (trail limits),
 * Table 1 (parameters).
 */
#ifndef FACO_ORACLE_H
#define FACO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ls_flags bits */
#define ORC_LS_2OPT 1u
#define ORC_LS_OROPT 2u
#define ORC_LS_SWEEP 4u
#define ORC_LS_INIT_3OPT 8u /* initial solution: 3-opt too (Sec. 4.3) */

/* Philox counter "purpose" word */
#define ORC_PURPOSE_ROULETTE 0u
#define ORC_PURPOSE_START 1u
#define ORC_PURPOSE_SOURCE 2u
#define ORC_PURPOSE_NEW_EDGES 3u

/* per-ant counters */
enum {
  ORC_CNT_ACO_STEPS = 0, /* select_next_node calls                     */
  ORC_CNT_COPIED,        /* nodes appended by the copy-from-source step */
  ORC_CNT_BACKUP,        /* choices taken from the backup list          */
  ORC_CNT_FALLBACK,      /* choices taken by the global nearest scan    */
  ORC_CNT_NEW_EDGES,     /* counted new edges (closing edge excluded)   */
  ORC_CNT_LS_POPS,       /* checklist pops                              */
  ORC_CNT_MOVES_2OPT,    /* applied 2-opt moves                         */
  ORC_CNT_MOVES_OROPT,   /* applied Or-opt moves                        */
  ORC_CNT_MOVED_ELEMS,   /* array positions rewritten by moves          */
  ORC_CNT_SWEEPS,        /* sweeps over the touched set                 */
  ORC_CNT_CHECKLIST0,    /* checklist length handed to the LS           */
  ORC_CNT_LS_GAIN,       /* total LS gain                               */
  ORC_CNT_MOVES_3OPT,    /* applied 3-opt moves (initial solution)      */
  ORC_NCNT
};

typedef struct {
  int32_t cl_size;       /* candidate-list length (16 in Table 1)        */
  int32_t bl_size;       /* backup-list length (64 in Table 1)           */
  int32_t n_ants;
  int32_t min_new_edges; /* min_new_edges of Alg. 2                      */
  float rho;             /* retention factor of Eq. (2)                  */
  float _pad0;
  double p_best;         /* Sec. 4.5 trail-limit parameter               */
  double p_source_gbest; /* probability the source is the global best    */
  uint64_t seed;         /* Philox key word 0                            */
  uint32_t ls_flags;     /* ORC_LS_* bits                                */
  int32_t oropt_max_seg; /* longest Or-opt segment                       */
  int32_t min_new_edges_max; /* calc_num_new_edges() range top; <= min_new_edges:
                                the constant min_new_edges              */
  int32_t _pad1;
} orc_params;

typedef struct orc_instance orc_instance;

/* Build: lists, heuristic, initial solution, limits, pheromone, source.
 * Returns NULL on invalid input (n<4, bad params, duplicate points). */
orc_instance *orc_build(const int32_t *xy, int32_t n, const orc_params *p,
                        int32_t n_threads);
void orc_free(orc_instance *h);

/* Run `iterations` more iterations of Alg. 2's main loop. */
void orc_run(orc_instance *h, int32_t iterations);

/* state accessors (all copy out) */
int64_t orc_best(const orc_instance *h, int32_t *tour /* n */);
int64_t orc_source(const orc_instance *h, int32_t *tour /* n */);
void orc_ant_routes(const orc_instance *h, int32_t *out /* A*n */);
void orc_ant_lengths(const orc_instance *h, int64_t *out /* A */);
void orc_ant_counters(const orc_instance *h, int64_t *out /* A*ORC_NCNT */);
void orc_init_counters(const orc_instance *h, int64_t *out /* ORC_NCNT */);
void orc_pheromone(const orc_instance *h, float *out /* n*k_eff */);
void orc_heuristic(const orc_instance *h, float *out /* n*k_eff */);
void orc_lists(const orc_instance *h, int32_t *cl /* n*k_eff */,
               int32_t *bl /* n*bl_eff */);
/* limits[0]=tau_min, [1]=tau_max, [2]=delta of the last deposit */
void orc_limits(const orc_instance *h, float *limits);
/* info[0]=iterations done, [1]=k_eff, [2]=bl_eff, [3]=last iteration-best
 * ant, [4]=last source was gbest (0/1), [5]=initial tour length,
 * [6]=gbest length, [7]=source length */
void orc_info(const orc_instance *h, int64_t *info);

/* Replace the source solution (tests only). */
void orc_set_source(orc_instance *h, const int32_t *tour);
/* Overwrite the pheromone (tests only). */
void orc_set_pheromone(orc_instance *h, const float *tau);

/* Construct one ant's tour at iteration t with the current state (no LS).
 * Writes route (n), checklist (up to n) and its length; returns tour length. */
int64_t orc_construct(const orc_instance *h, uint64_t t, uint64_t ant,
                      int32_t *route, int32_t *checklist, int32_t *n_check,
                      int64_t *counters);

/* calc_num_new_edges() of Alg. 2 for ant `ant` at iteration t. */
int32_t orc_min_new_edges(const orc_instance *h, uint64_t t, uint64_t ant);

/* Local search on an arbitrary tour (route in/out); returns total gain. */
int64_t orc_local_search(const orc_instance *h, int32_t *route,
                         const int32_t *checklist, int32_t n_check,
                         uint32_t flags, int64_t *counters);

/* Nearest-neighbour tour from city 0 (before its local search). */
int64_t orc_nearest_neighbour(const orc_instance *h, int32_t *route /* n */);

/* Gain of the best move from node a on the tour (0 if none). */
int64_t orc_best_move_gain(const orc_instance *h, const int32_t *route,
                           int32_t a, uint32_t flags);

/* primitives */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]);
int32_t orc_dist(const int32_t *xy, int32_t i, int32_t j);
int32_t orc_nint_sqrt(int64_t d2); /* nint(sqrt(d2)), d2 >= 0 */
int64_t orc_tour_length(const int32_t *xy, int32_t n, const int32_t *route);

#ifdef __cplusplus
}
#endif
#endif
