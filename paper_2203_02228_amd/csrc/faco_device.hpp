// faco_device.hpp -- device-side instance view and per-instance state.
#pragma once
#include <stdint.h>

namespace faco {

// Scalars that change every iteration, kept on the device so that a whole
// run of iterations is enqueued without host round trips.
struct DevState {
  int64_t iter;      // completed iterations
  int64_t gb_len;    // global-best cost
  int64_t src_len;   // cost of the current source solution
  int64_t init_len;  // cost of the initial solution
  float tau_min, tau_max, delta, pad0;
  int32_t ib;        // iteration-best ant of the last iteration
  int32_t src_gb;    // 1 if the last source choice took the global best
  int32_t improved;  // 1 if the last iteration improved the global best
  int32_t dup;       // set by the list kernel when two cities coincide
  int64_t init_cnt[13];
  int64_t init_ticks[32];  // the initial solution's tick slots (an ant's [kTicks])
  // Faults found on the device (FAULT_* bits; the first one's ant and
  // iteration), and the number of tours the verification kernel has checked.
  int32_t fault, fault_ant;
  int64_t fault_iter;
  int64_t verified;
};

enum : int32_t {
  // a sweep listed cities with improving moves, but their evaluation found
  // no move (the two move tests disagree): the local search stopped early
  FAULT_LS_STALL = 1,
  // a recomputed tour length differs from the incrementally tracked one
  FAULT_LENGTH = 2,
  // an ant's route is not a permutation (route and pos disagree)
  FAULT_PERMUTATION = 4,
  // a persistent batched launch saw no progress for a long time and left
  // before this instance completed its iterations
  FAULT_BATCH_STALL = 8,
};

// Device view of one instance (kernel argument).  Layouts:
//   xy        int2 [n]           (x, y)
//   cl, eta,
//   tau       [n][k]             row-major, k = effective candidate-list length
//   bll       [n][bl]            backup lists
//   routes,
//   pos, ring [A][n]             ant tours, their inverses, LS checklist rings
//   cnt       int64 [A][12]      per-ant counters of the last iteration
//   cnt_acc   int64 [A][12]      the same summed over all iterations
struct Inst {
  int32_t n, k, bl, A, m;
  int32_t m_hi;       // calc_num_new_edges() range top (<= m: the constant m)
  int32_t verify;     // 1: each iteration recomputes and checks tour lengths
  int32_t lcap;       // capacity of the LDS part of an ant's work queue
  float rho;
  uint32_t ls_flags;
  int32_t oropt_max;
  uint64_t seed;
  double p_gb;   // probability the source is the global best
  double p_root; // p_best^(1/n)
  // Cities are relabelled internally along a Hilbert curve of the
  // coordinates (spatially close cities get close labels, so a tour segment's
  // cities share cache lines).  Every rule that depends on a city's number
  // uses its original number: orig_of[internal], int_of[original].
  const int32_t *orig_of;
  const int32_t *int_of;
  const int2 *xy;     // [n] coordinates by internal label
  const int4 *wbox;   // [(n + 31) / 32] bounding box (min x, min y, max x, max y) of labels 32 i ..
  const int32_t *cl;
  const int32_t *bll;
  const float *eta;
  const int32_t *cl_d;  // [n][k] cost of every candidate slot
  float *tau;
  int32_t *src_route, *src_pos, *gb_route;
  int2 *src_adj;      // [n] (successor, predecessor) of each city in the source
  // Candidate rows in SOURCE order (row p = candidates of the city at source
  // position p), rewritten by the pheromone kernel every iteration; laid out
  // by srow() in blocks of 64 positions:
  int32_t *scl;       // candidate city
  float *sw;          // tau * eta (Eq. (1) weight)
  int32_t *ssp;       // source position of the candidate
  int32_t *sd;        // cost of the candidate edge
  int32_t *src_d;     // [n] cost of the source edge from position i to i + 1
  int2 *src_xy;       // [n] coordinates of the city at source position i
  int32_t *routes, *pos, *ring;
  int2 *rxy;          // [A][n] coordinates of routes[a][p] (tour order)
  int64_t *lens, *cnt, *cnt_acc;
  int64_t *ticks;     // [A][kTicks] wall-clock ticks and call counts per phase, summed
  // Segment-list ant tours (the local search of the single-instance kernel
  // with seg_on): between materialisations the ant's tour is the storage
  // arrays (route, pos, rxy of buffer `live`) read through segment records,
  // each a storage range, its orientation and the array position of its
  // first element, so a move rewrites records instead of elements.
  int32_t seg_on;     // 1: the local search runs on segment lists
  int32_t seg_shift;  // log2 of the segment length after a materialisation
  int32_t seg_max;    // records in use that trigger a materialisation
  int32_t *r2, *p2;   // [A][n] second storage buffer: route, pos
  int2 *x2;           // [A][n] second storage buffer: coordinates
  int2 *sgid;         // [A][n] (epoch, segment) of a city whose segment was split off
  int32_t *sepoch;    // [A] last epoch of each ant
  int32_t *rsel;      // [A] buffer holding each ant's final tour (0: routes, 1: r2)
  // tour-length verification: partial sums and route faults of the tours
  // being checked (ants 0..A-1, then the global best), the last results
  int64_t *vsum;      // [A + 1], zero between verifications
  int32_t *vbad;      // [A + 1], zero between verifications
  int64_t *vout;      // [A + 1] recomputed lengths (-1: not a permutation)
  DevState *st;
};

enum {
  CNT_ACO_STEPS = 0,
  CNT_COPIED,
  CNT_BACKUP,
  CNT_FALLBACK,
  CNT_NEW_EDGES,
  CNT_LS_POPS,
  CNT_MOVES_2OPT,
  CNT_MOVES_OROPT,
  CNT_MOVED_ELEMS,
  CNT_SWEEPS,
  CNT_CHECKLIST0,
  CNT_LS_GAIN,
  CNT_MOVES_3OPT,
  NCNT
};

constexpr uint32_t LS_2OPT = 1u, LS_OROPT = 2u, LS_SWEEP = 4u, LS_INIT_3OPT = 8u;
constexpr int kMaxCl = 32;
constexpr int kMaxBl = 64;
constexpr int kMaxOrSeg = 3;
// tick and count slots per ant (FACO_DBG_PHASE_TICKS)
constexpr int kTicks = 32;
static_assert(sizeof(((DevState *)nullptr)->init_ticks) == sizeof(int64_t) * kTicks,
              "the initial solution keeps an ant's tick slots");
// capacity of the segment record table of a segment-list tour
constexpr int kSegCap = 2048;

// Final tour of ant a (its route and positions), wherever its local search
// left it.
__device__ __forceinline__ const int32_t *ant_route(const Inst &I, int a) {
  return (I.rsel[a] ? I.r2 : I.routes) + (size_t)a * (size_t)I.n;
}
__device__ __forceinline__ const int32_t *ant_pos(const Inst &I, int a) {
  return (I.rsel[a] ? I.p2 : I.pos) + (size_t)a * (size_t)I.n;
}

// Element (position p, slot s) of a source-ordered table with k slots: 64
// consecutive positions form a block, slot-major inside it, so the lanes of
// a window (consecutive positions, one slot per load) read adjacent words.
// A table holds ceil(n / 64) * 64 * k elements.
__device__ __forceinline__ size_t srow(int p, int s, int k) {
  return ((size_t)(p >> 6) * (size_t)k + (size_t)s) * 64u + (size_t)(p & 63);
}

// Control of a persistent batched launch: one BatchCtl per instance (the
// ticket of the next ant task, ants of the current iteration done,
// iterations completed in the launch, ants per iteration) and one BatchRun.
struct BatchCtl {
  int64_t ticket;
  int32_t done, epoch, ants, pad;
};
struct BatchRun {
  int32_t count, iterations;
  int32_t finished;  // instances that completed all their iterations
  int32_t progress;  // ant tasks completed (stall detection)
};

// Default capacity of the LDS part of an ant's work queue (listed cities).
constexpr int kLdsRingMax = 16384;

}  // namespace faco
