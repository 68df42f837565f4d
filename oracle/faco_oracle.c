/*
 * faco_oracle.c -- plain, slow CPU oracle for Focused ACO (FACO).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the HIP library.
 *
 * Everything follows the paper's steps in the paper's order, on plain arrays:
 *   - the tour is an array route[0..n-1] with its inverse pos[];
 *   - the visited set is a byte per node;
 *   - distances are recomputed from coordinates (TSPLIB EUC_2D) every time.
 * Readings of points the paper leaves open are marked "reading:".
 *
 * Arithmetic environment: compiled with -ffp-contract=off, no fast-math;
 * float is IEEE binary32, double binary64, round to nearest even.
 */
#include "faco_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Distances.  The paper's problem statement (Sec. 2.1) only asks for
 * positive symmetric costs; its instances are TSPLIB/TSP-Art instances with
 * integer lengths.  reading: cost = TSPLIB EUC_2D, nint(sqrt(dx^2+dy^2)),
 * coordinates in [0, 2^26) so that dx^2 + dy^2 < 2^53. */

static inline int64_t sqd(const int32_t *xy, int32_t i, int32_t j) {
  int64_t dx = (int64_t)xy[2 * i] - (int64_t)xy[2 * j];
  int64_t dy = (int64_t)xy[2 * i + 1] - (int64_t)xy[2 * j + 1];
  return dx * dx + dy * dy;
}

/* nint(sqrt(d2)) for an integer d2 >= 0, by integer arithmetic: r = floor of
 * the square root (r^2 <= d2 < (r+1)^2, found from a floating-point start and
 * settled with exact int64 products), then r + 1 when d2 > r^2 + r, i.e. when
 * sqrt(d2) > r + 1/2 (sqrt(d2) is never a half-integer). */
static inline int32_t nint_sqrt(int64_t d2) {
  int64_t r = (int64_t)sqrt((double)d2);
  while (r > 0 && r * r > d2) --r;
  while ((r + 1) * (r + 1) <= d2) ++r;
  return (int32_t)(r + (d2 > r * r + r ? 1 : 0));
}

static inline int32_t dist(const int32_t *xy, int32_t i, int32_t j) {
  return nint_sqrt(sqd(xy, i, j));
}

int32_t orc_nint_sqrt(int64_t d2) { return nint_sqrt(d2); }

int32_t orc_dist(const int32_t *xy, int32_t i, int32_t j) {
  return dist(xy, i, j);
}

int64_t orc_tour_length(const int32_t *xy, int32_t n, const int32_t *route) {
  int64_t s = 0;
  for (int32_t i = 0; i < n; ++i) s += dist(xy, route[i], route[(i + 1) % n]);
  return s;
}

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  The paper does not say how random numbers are
 * drawn; reading: counter-based draws keyed by (seed, 0) with counter
 * (iteration, ant, step, purpose), so every draw is addressable. */

static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ull;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ull;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ull;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73Bull;

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2],
                       uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

static uint64_t draw(uint64_t seed, uint64_t t, uint64_t ant, uint64_t step,
                     uint64_t purpose) {
  uint64_t ctr[4] = {t, ant, step, purpose};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  orc_philox4x64_10(ctr, key, out);
  return out[0];
}

/* U = top 24 bits / 2^24, an exact binary32 in [0,1). */
static inline float unit24(uint64_t x) {
  return (float)(uint32_t)(x >> 40) * 0x1p-24f;
}

/* U{0, n-1} (Alg. 2 start node): floor(x * n / 2^64). */
static inline int32_t uniform_node(uint64_t x, int32_t n) {
  return (int32_t)(((unsigned __int128)x * (uint64_t)n) >> 64);
}

/* ------------------------------------------------------------------------ */

struct orc_instance {
  int32_t n, k, bl, A, m;
  orc_params p;
  int32_t n_threads;
  int32_t *xy;
  int32_t *cl;  /* n*k: k nearest by (d^2, id), Sec. 4.1 */
  int32_t *bll; /* n*bl: the next bl nearest (backup list), Sec. 4.1 */
  float *eta;   /* n*k: 1/d per candidate slot, Eq. (1) */
  float *tau;   /* n*k: partial pheromone memory, Sec. 4.2 */
  double p_root; /* p_best^(1/n), Sec. 4.5 */
  float tau_min, tau_max, delta;
  int32_t *src_route, *src_pos;
  int64_t src_len;
  int32_t *gb_route;
  int64_t gb_len, init_len;
  int64_t iter;
  int32_t last_ib, last_src_gb;
  int32_t *routes; /* A*n */
  int64_t *lens;   /* A */
  int64_t *cnt;    /* A*ORC_NCNT */
  int64_t init_cnt[ORC_NCNT];
};

/* ------------------------------------------------------------------------ */
/* Candidate and backup lists (Sec. 4.1): cl(i) = the k nearest nodes,
 * bl(i) = the next bl nearest.  reading: "nearest" orders by the exact squared
 * Euclidean distance, ties by node id. */

static int key_less(int64_t da, int32_t a, int64_t db, int32_t b) {
  return da < db || (da == db && a < b);
}

static void build_lists(orc_instance *h) {
  const int32_t n = h->n, k = h->k, bl = h->bl, K = k + bl;
#pragma omp parallel for schedule(dynamic, 64) num_threads(h->n_threads)
  for (int32_t i = 0; i < n; ++i) {
    int64_t *kd = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    int32_t *kj = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    int32_t cnt = 0;
    for (int32_t j = 0; j < n; ++j) {
      if (j == i) continue;
      int64_t d = sqd(h->xy, i, j);
      if (cnt == K && !key_less(d, j, kd[K - 1], kj[K - 1])) continue;
      int32_t q = (cnt < K) ? cnt++ : K - 1;
      while (q > 0 && key_less(d, j, kd[q - 1], kj[q - 1])) {
        kd[q] = kd[q - 1];
        kj[q] = kj[q - 1];
        --q;
      }
      kd[q] = d;
      kj[q] = j;
    }
    for (int32_t s = 0; s < k; ++s) {
      h->cl[(size_t)i * k + s] = kj[s];
      int32_t dd = dist(h->xy, i, kj[s]);
      h->eta[(size_t)i * k + s] = (float)(1.0 / (double)dd);
    }
    for (int32_t s = 0; s < bl; ++s) h->bll[(size_t)i * bl + s] = kj[k + s];
    free(kd);
    free(kj);
  }
}

/* ------------------------------------------------------------------------ */
/* Trail limits (Sec. 4.5): tau_max = 1/(cost_gb (1 - rho)),
 * tau_min = tau_max (1 - p) / ((avg - 1) p) with p = p_best^(1/n) and
 * avg = cl_size.  reading: computed in binary64, clamped so tau_min <= tau_max,
 * then rounded to binary32. */

static void update_limits(orc_instance *h) {
  double tmax = 1.0 / ((double)h->gb_len * (1.0 - (double)h->p.rho));
  double num = 1.0 - h->p_root;
  double den = (double)(h->k - 1) * h->p_root;
  double tmin = tmax * num / den;
  if (tmin > tmax) tmin = tmax;
  h->tau_max = (float)tmax;
  h->tau_min = (float)tmin;
}

static void set_source(orc_instance *h, const int32_t *route, int64_t len) {
  memcpy(h->src_route, route, sizeof(int32_t) * (size_t)h->n);
  for (int32_t i = 0; i < h->n; ++i) h->src_pos[route[i]] = i;
  h->src_len = len;
}

static inline int32_t src_succ(const orc_instance *h, int32_t u) {
  int32_t q = h->src_pos[u] + 1;
  return h->src_route[q == h->n ? 0 : q];
}
static inline int32_t src_pred(const orc_instance *h, int32_t u) {
  int32_t q = h->src_pos[u] - 1;
  return h->src_route[q < 0 ? h->n - 1 : q];
}

/* ------------------------------------------------------------------------ */
/* Next-node choice (Eq. (1) over the candidate list, then the backup list,
 * then the best heuristic value; Sec. 4.3 text after Alg. 2).
 * reading: alpha = beta = 1, so the weight is tau*eta (one binary32 multiply);
 * the cumulative sum runs over the candidate slots in list order in binary32;
 * r = U*S; the chosen slot is the first whose cumulative sum exceeds r, or the
 * last unvisited slot if none does (r rounded up to S).  The backup list is
 * used "aggressively": its first unvisited node.  The last resort is the
 * unvisited node of largest eta = smallest distance, i.e. smallest (d^2, id).
 * mode 0: roulette; mode 1: greedy (first unvisited candidate), used for the
 * nearest-neighbour initial tour. */

static int32_t select_next(const orc_instance *h, int32_t u,
                           const uint8_t *visited, uint64_t t, uint64_t ant,
                           uint64_t step, int mode, int64_t *cnt) {
  const int32_t k = h->k;
  const int32_t *row = h->cl + (size_t)u * k;
  if (mode == 0) {
    const float *trow = h->tau + (size_t)u * k;
    const float *erow = h->eta + (size_t)u * k;
    float cum[64];
    float total = 0.0f;
    int32_t last = -1;
    for (int32_t s = 0; s < k; ++s) {
      if (!visited[row[s]]) {
        float w = trow[s] * erow[s];
        total = total + w;
        last = s;
      }
      cum[s] = total;
    }
    if (last >= 0) {
      float U = unit24(draw(h->p.seed, t, ant, step, ORC_PURPOSE_ROULETTE));
      float r = U * total;
      for (int32_t s = 0; s < k; ++s)
        if (cum[s] > r) return row[s];
      return row[last];
    }
  } else {
    for (int32_t s = 0; s < k; ++s)
      if (!visited[row[s]]) return row[s];
  }
  const int32_t *brow = h->bll + (size_t)u * h->bl;
  for (int32_t s = 0; s < h->bl; ++s)
    if (!visited[brow[s]]) {
      if (cnt) cnt[ORC_CNT_BACKUP]++;
      return brow[s];
    }
  if (cnt) cnt[ORC_CNT_FALLBACK]++;
  int32_t best = -1;
  int64_t bd = 0;
  for (int32_t j = 0; j < h->n; ++j) {
    if (visited[j]) continue;
    int64_t d = sqd(h->xy, u, j);
    if (best < 0 || d < bd) {
      best = j;
      bd = d;
    }
  }
  return best;
}

/* ------------------------------------------------------------------------ */
/* Focused construction (Alg. 2, inner loop; Sec. 4.3).
 * Random start node, ACO steps until new_edges >= min_new_edges, then the
 * remainder is copied from the source solution.
 * reading of the copy: walk the source forward from v while the nodes are
 * unvisited; if that appends nothing, walk backward from v instead; then go
 * back to the ACO rule.  An edge (u,v) is "in the source" when v is u's
 * successor or predecessor there (symmetric TSP).  The closing edge is not
 * counted. */

/* calc_num_new_edges() (Alg. 2): the threshold of one ant's construction,
 * called once per ant before it starts.  The paper names the function but
 * states no rule; its experiments use the constant of Table 1.
 * reading: with min_new_edges_max <= min_new_edges the constant
 * min_new_edges; otherwise each ant draws its own threshold uniformly from
 * [min_new_edges, min_new_edges_max]: lo + floor(x * (hi - lo + 1) / 2^64)
 * with x the Philox word of counter (t, ant, 0, purpose 3). */
static int32_t calc_num_new_edges(const orc_instance *h, uint64_t t, uint64_t ant) {
  const int32_t lo = h->m, hi = h->p.min_new_edges_max;
  if (hi <= lo) return lo;
  const uint64_t x = draw(h->p.seed, t, ant, 0, ORC_PURPOSE_NEW_EDGES);
  const uint64_t span = (uint64_t)hi - (uint64_t)lo + 1u;
  return lo + (int32_t)(((unsigned __int128)x * span) >> 64);
}

int32_t orc_min_new_edges(const orc_instance *h, uint64_t t, uint64_t ant) {
  return calc_num_new_edges(h, t, ant);
}

static int64_t construct(const orc_instance *h, uint64_t t, uint64_t ant,
                         int32_t *route, uint8_t *visited, int32_t *chk,
                         int32_t *nchk, int64_t *cnt) {
  const int32_t n = h->n;
  const int32_t min_new_edges = calc_num_new_edges(h, t, ant);
  memset(visited, 0, (size_t)n);
  int32_t r0 = uniform_node(draw(h->p.seed, t, ant, 0, ORC_PURPOSE_START), n);
  route[0] = r0;
  visited[r0] = 1;
  int32_t k = 1, new_edges = 0, nc = 0;
  int64_t len = 0;
  uint64_t step = 0;
  while (k < n) {
    int32_t u = route[k - 1];
    int32_t v = select_next(h, u, visited, t, ant, step, 0, cnt);
    ++step;
    route[k++] = v;
    visited[v] = 1;
    len += dist(h->xy, u, v);
    if (v != src_succ(h, u) && v != src_pred(h, u)) {
      ++new_edges;
      chk[nc++] = v;
    }
    if (new_edges >= min_new_edges) {
      int32_t prev = v, c = src_succ(h, v), appended = 0;
      while (!visited[c]) {
        route[k++] = c;
        visited[c] = 1;
        len += dist(h->xy, prev, c);
        prev = c;
        c = src_succ(h, c);
        ++appended;
      }
      if (appended == 0) {
        c = src_pred(h, v);
        while (!visited[c]) {
          route[k++] = c;
          visited[c] = 1;
          len += dist(h->xy, prev, c);
          prev = c;
          c = src_pred(h, c);
          ++appended;
        }
      }
      if (cnt) cnt[ORC_CNT_COPIED] += appended;
    }
  }
  len += dist(h->xy, route[n - 1], route[0]);
  if (cnt) {
    cnt[ORC_CNT_ACO_STEPS] += (int64_t)step;
    cnt[ORC_CNT_NEW_EDGES] += new_edges;
  }
  *nchk = nc;
  return len;
}

/* Nearest-neighbour tour from node 0 (initial solution, Sec. 4.3): the same
 * fallback chain with the greedy rule, no source, no copy. */
static int64_t nearest_neighbour_tour(const orc_instance *h, int32_t *route,
                                      uint8_t *visited) {
  const int32_t n = h->n;
  memset(visited, 0, (size_t)n);
  route[0] = 0;
  visited[0] = 1;
  int64_t len = 0;
  for (int32_t k = 1; k < n; ++k) {
    int32_t u = route[k - 1];
    int32_t v = select_next(h, u, visited, 0, 0, 0, 1, NULL);
    route[k] = v;
    visited[v] = 1;
    len += dist(h->xy, u, v);
  }
  return len + dist(h->xy, route[n - 1], route[0]);
}

/* ------------------------------------------------------------------------ */
/* Local search (Alg. 3, Sec. 4.4): a FIFO checklist, best improvement over
 * the candidate list of the popped node, succ and pred variants, strict
 * improvement, flip, append the four endpoints, stop when the list is empty
 * or n changes were made.
 * Additions beyond Alg. 3 (readings):
 *   - Or-opt (segment insertion, not in the paper): tried only when no
 *     improving 2-opt move starts at the popped node;
 *   - sweep: when the list empties, every node ever listed is re-examined in
 *     ascending id and the ones with an improving move are re-listed.
 * A node already on the list is not appended again. */

typedef struct {
  int32_t *route, *pos;
  int32_t n;
} tour_t;

static inline int32_t t_succ(const tour_t *T, int32_t x) {
  int32_t q = T->pos[x] + 1;
  return T->route[q == T->n ? 0 : q];
}
static inline int32_t t_pred(const tour_t *T, int32_t x) {
  int32_t q = T->pos[x] - 1;
  return T->route[q < 0 ? T->n - 1 : q];
}

typedef struct {
  int kind; /* 0 none, 1 2-opt, 2 or-opt, 3 3-opt */
  int64_t gain;
  int32_t w, x, y, z;                 /* 2-opt: remove (w,x),(y,z) */
  int32_t f, l, p, q, a, o, b, e, L; /* or-opt */
  int32_t t[6], dir;                 /* 3-opt: t1..t6, orientation */
} move_t;

static void eval_2opt(const orc_instance *h, const tour_t *T, int32_t a,
                      move_t *mv) {
  const int32_t *nn = h->cl + (size_t)a * h->k;
  int32_t a_s = t_succ(T, a), a_p = t_pred(T, a);
  int64_t d_as = dist(h->xy, a, a_s), d_ap = dist(h->xy, a_p, a);
  for (int32_t s = 0; s < h->k; ++s) {
    int32_t b = nn[s];
    int64_t d_ab = dist(h->xy, a, b);
    if (d_as > d_ab) {
      int32_t b_s = t_succ(T, b);
      int64_t g = d_as + dist(h->xy, b, b_s) - d_ab - dist(h->xy, a_s, b_s);
      if (g > mv->gain) {
        mv->gain = g;
        mv->kind = 1;
        mv->w = a;
        mv->x = a_s;
        mv->y = b;
        mv->z = b_s;
      }
    }
  }
  for (int32_t s = 0; s < h->k; ++s) {
    int32_t b = nn[s];
    int64_t d_ab = dist(h->xy, a, b);
    if (d_ap > d_ab) {
      int32_t b_p = t_pred(T, b);
      int64_t g = d_ap + dist(h->xy, b_p, b) - d_ab - dist(h->xy, a_p, b_p);
      if (g > mv->gain) {
        mv->gain = g;
        mv->kind = 1;
        mv->w = a_p;
        mv->x = a;
        mv->y = b_p;
        mv->z = b;
      }
    }
  }
}

/* Or-opt (reading; the paper has none).  A segment of L <= oropt_max_seg
 * consecutive nodes with a at one end (forward: a first; backward: a last),
 * with outer neighbours p (before) and q (after), is moved between b in cl(a)
 * and e in {succ(b), pred(b)} (both outside the segment) so that a becomes
 * adjacent to b and the far end o adjacent to e.  Only b with d(a,b) shorter
 * than the removed edge at a are tried.  Order: forward L=1..Lmax, then
 * backward L=2..Lmax; b in list order; e = succ(b) before pred(b). */
static void eval_oropt(const orc_instance *h, const tour_t *T, int32_t a,
                       move_t *mv) {
  const int32_t n = h->n;
  int32_t Lmax = h->p.oropt_max_seg;
  if (Lmax > n - 3) Lmax = n - 3;
  const int32_t *nn = h->cl + (size_t)a * h->k;
  for (int dir = 0; dir < 2; ++dir) {
    for (int32_t L = (dir == 0 ? 1 : 2); L <= Lmax; ++L) {
      int32_t f, l;
      if (dir == 0) {
        f = a;
        l = a;
        for (int32_t i = 1; i < L; ++i) l = t_succ(T, l);
      } else {
        l = a;
        f = a;
        for (int32_t i = 1; i < L; ++i) f = t_pred(T, f);
      }
      int32_t p = t_pred(T, f), q = t_succ(T, l);
      int32_t o = (dir == 0) ? l : f;
      int64_t d_rem_a = (dir == 0) ? dist(h->xy, p, a) : dist(h->xy, a, q);
      int64_t g_rem =
          (int64_t)dist(h->xy, p, f) + dist(h->xy, l, q) - dist(h->xy, p, q);
      int32_t fpos = T->pos[f];
      for (int32_t s = 0; s < h->k; ++s) {
        int32_t b = nn[s];
        if ((T->pos[b] - fpos + n) % n < L) continue;
        int64_t d_ab = dist(h->xy, a, b);
        if (!(d_ab < d_rem_a)) continue;
        for (int side = 0; side < 2; ++side) {
          int32_t e = (side == 0) ? t_succ(T, b) : t_pred(T, b);
          if ((T->pos[e] - fpos + n) % n < L) continue;
          int64_t g = g_rem + dist(h->xy, b, e) - d_ab - dist(h->xy, o, e);
          if (g > mv->gain) {
            mv->gain = g;
            mv->kind = 2;
            mv->f = f;
            mv->l = l;
            mv->p = p;
            mv->q = q;
            mv->a = a;
            mv->o = o;
            mv->b = b;
            mv->e = e;
            mv->L = L;
          }
        }
      }
    }
  }
}

/* 3-opt.  The paper improves its initial solution with 2-opt and 3-opt
 * following Bentley (Sec. 4.3, after Alg. 2) without defining the move set.
 * reading: the pure 3-opt reconnection (no segment reversed), searched from
 * t1 = a over the candidate lists with positive partial gains (the rule
 * that keeps neighbour-list searches complete), in both orientations.
 * Orientation succ: t2 = succ(t1); t3 in cl(t2), t3 != t1, with
 * g1 = d(t1,t2) - d(t2,t3) > 0; t4 = succ(t3), t4 != t1; t5 in cl(t4) with
 * g2 = g1 + d(t3,t4) - d(t4,t5) > 0 and t5 on the path t2..t3 before t3;
 * t6 = succ(t5); gain = g2 + d(t5,t6) - d(t6,t1).  The tour
 * t1 [t2..t5] [t6..t3] t4 becomes t1 [t6..t3] [t2..t5] t4: the two blocks
 * exchange places and keep their orientation.  Orientation pred: the same
 * with pred for succ.  Best improvement, strict >; order: succ then pred,
 * t3 in list order, t5 in list order. */
static int32_t t_step(const tour_t *T, int32_t x, int dir) {
  return dir == 0 ? t_succ(T, x) : t_pred(T, x);
}
/* positions from `from` to x along the orientation */
static int32_t t_offset(const tour_t *T, int32_t from, int32_t x, int dir) {
  const int32_t n = T->n;
  return dir == 0 ? (T->pos[x] - T->pos[from] + n) % n : (T->pos[from] - T->pos[x] + n) % n;
}

static void eval_3opt(const orc_instance *h, const tour_t *T, int32_t a,
                      move_t *mv) {
  for (int dir = 0; dir < 2; ++dir) {
    const int32_t t1 = a, t2 = t_step(T, t1, dir);
    const int64_t d12 = dist(h->xy, t1, t2);
    const int32_t *nn2 = h->cl + (size_t)t2 * h->k;
    for (int32_t s = 0; s < h->k; ++s) {
      const int32_t t3 = nn2[s];
      const int64_t g1 = d12 - dist(h->xy, t2, t3);
      if (g1 <= 0 || t3 == t1) continue;
      const int32_t t4 = t_step(T, t3, dir);
      if (t4 == t1) continue;
      const int32_t off3 = t_offset(T, t2, t3, dir);
      const int64_t d34 = dist(h->xy, t3, t4);
      const int32_t *nn4 = h->cl + (size_t)t4 * h->k;
      for (int32_t r = 0; r < h->k; ++r) {
        const int32_t t5 = nn4[r];
        const int64_t g2 = g1 + d34 - dist(h->xy, t4, t5);
        if (g2 <= 0) continue;
        if (t_offset(T, t2, t5, dir) >= off3) continue;
        const int32_t t6 = t_step(T, t5, dir);
        const int64_t g = g2 + dist(h->xy, t5, t6) - dist(h->xy, t6, t1);
        if (g > mv->gain) {
          mv->gain = g;
          mv->kind = 3;
          mv->dir = dir;
          mv->t[0] = t1;
          mv->t[1] = t2;
          mv->t[2] = t3;
          mv->t[3] = t4;
          mv->t[4] = t5;
          mv->t[5] = t6;
        }
      }
    }
  }
}

static void best_move(const orc_instance *h, const tour_t *T, int32_t a,
                      uint32_t flags, move_t *mv) {
  mv->kind = 0;
  mv->gain = 0;
  if (flags & ORC_LS_2OPT) eval_2opt(h, T, a, mv);
  if (mv->kind == 0 && (flags & ORC_LS_OROPT)) eval_oropt(h, T, a, mv);
  if (mv->kind == 0 && (flags & ORC_LS_INIT_3OPT)) eval_3opt(h, T, a, mv);
}

/* reverse the cyclic array range of length L starting at position s */
static void reverse_range(tour_t *T, int32_t s, int32_t L) {
  const int32_t n = T->n;
  for (int32_t i = 0; i < L / 2; ++i) {
    int32_t p1 = (s + i) % n, p2 = (s + L - 1 - i) % n;
    int32_t x = T->route[p1], y = T->route[p2];
    T->route[p1] = y;
    T->route[p2] = x;
    T->pos[y] = p1;
    T->pos[x] = p2;
  }
}

/* "Flip a section of route between x and y" (Alg. 3).  reading: reverse the
 * path x..y when it holds at most n/2 nodes, otherwise the complementary path
 * z..w; both give the same cycle. */
static int64_t apply_2opt(tour_t *T, const move_t *mv) {
  const int32_t n = T->n;
  int32_t L1 = (T->pos[mv->y] - T->pos[mv->x] + n) % n + 1;
  if (2 * L1 <= n) {
    reverse_range(T, T->pos[mv->x], L1);
    return L1;
  }
  reverse_range(T, T->pos[mv->z], n - L1);
  return n - L1;
}

/* Or-opt realisation: the segment and the shorter of the two blocks between
 * its old place and the insertion edge exchange places; the block keeps its
 * orientation, the segment is written in the orientation the move asks for. */
static int64_t apply_oropt(tour_t *T, const move_t *mv, int32_t *tmp) {
  const int32_t n = T->n, L = mv->L;
  int32_t x1, x2;
  if (t_succ(T, mv->b) == mv->e) {
    x1 = mv->b;
    x2 = mv->e;
  } else {
    x1 = mv->e;
    x2 = mv->b;
  }
  int32_t seg[64];
  int32_t fpos = T->pos[mv->f];
  for (int32_t i = 0; i < L; ++i) seg[i] = T->route[(fpos + i) % n];
  /* inserted sequence in forward order: a..o if x1 == b, else o..a */
  int rev = (x1 == mv->b) ? (mv->a != mv->f) : (mv->a == mv->f);
  int32_t ins[64];
  for (int32_t i = 0; i < L; ++i) ins[i] = rev ? seg[L - 1 - i] : seg[i];
  int32_t D1 = (T->pos[x1] - T->pos[mv->q] + n) % n + 1;
  int32_t D2 = (T->pos[mv->p] - T->pos[x2] + n) % n + 1;
  if (D1 <= D2) {
    int32_t qpos = T->pos[mv->q];
    for (int32_t i = 0; i < D1; ++i) tmp[i] = T->route[(qpos + i) % n];
    for (int32_t i = 0; i < D1; ++i) {
      int32_t ps = (fpos + i) % n;
      T->route[ps] = tmp[i];
      T->pos[tmp[i]] = ps;
    }
    for (int32_t i = 0; i < L; ++i) {
      int32_t ps = (fpos + D1 + i) % n;
      T->route[ps] = ins[i];
      T->pos[ins[i]] = ps;
    }
    return D1 + L;
  }
  int32_t base = T->pos[x2];
  for (int32_t i = 0; i < D2; ++i) tmp[i] = T->route[(base + i) % n];
  for (int32_t i = 0; i < L; ++i) {
    int32_t ps = (base + i) % n;
    T->route[ps] = ins[i];
    T->pos[ins[i]] = ps;
  }
  for (int32_t i = 0; i < D2; ++i) {
    int32_t ps = (base + L + i) % n;
    T->route[ps] = tmp[i];
    T->pos[tmp[i]] = ps;
  }
  return D2 + L;
}

/* 3-opt realisation: in array order the range covered by the two blocks
 * ([t2..t5][t6..t3] for orientation succ, [t3..t6][t5..t2] for pred) is
 * rewritten with the second block first; both keep their orientation and
 * nothing outside the range moves. */
static int64_t apply_3opt(tour_t *T, const move_t *mv, int32_t *tmp) {
  const int32_t n = T->n;
  const int32_t *t = mv->t;
  int32_t s, L1, L2;
  if (mv->dir == 0) {
    s = T->pos[t[1]];
    L1 = (T->pos[t[4]] - s + n) % n + 1;
    L2 = (T->pos[t[2]] - T->pos[t[5]] + n) % n + 1;
  } else {
    s = T->pos[t[2]];
    L1 = (T->pos[t[5]] - s + n) % n + 1;
    L2 = (T->pos[t[1]] - T->pos[t[4]] + n) % n + 1;
  }
  for (int32_t i = 0; i < L1 + L2; ++i) tmp[i] = T->route[(s + i) % n];
  for (int32_t i = 0; i < L2; ++i) {
    int32_t ps = (s + i) % n;
    T->route[ps] = tmp[L1 + i];
    T->pos[tmp[L1 + i]] = ps;
  }
  for (int32_t i = 0; i < L1; ++i) {
    int32_t ps = (s + L2 + i) % n;
    T->route[ps] = tmp[i];
    T->pos[tmp[i]] = ps;
  }
  return L1 + L2;
}

typedef struct {
  int32_t *ring, *tmp, *pos;
  uint8_t *inq, *touched, *visited;
  int32_t *chk;
} scratch_t;

static void scratch_alloc(scratch_t *S, int32_t n) {
  S->ring = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  S->tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  S->pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  S->chk = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  S->inq = (uint8_t *)calloc((size_t)n, 1);
  S->touched = (uint8_t *)calloc((size_t)n, 1);
  S->visited = (uint8_t *)calloc((size_t)n, 1);
}
static void scratch_free(scratch_t *S) {
  free(S->ring);
  free(S->tmp);
  free(S->pos);
  free(S->chk);
  free(S->inq);
  free(S->touched);
  free(S->visited);
}

static int64_t local_search(const orc_instance *h, int32_t *route,
                            const int32_t *chk, int32_t nchk, uint32_t flags,
                            scratch_t *S, int64_t *cnt) {
  const int32_t n = h->n;
  tour_t T = {route, S->pos, n};
  for (int32_t i = 0; i < n; ++i) S->pos[route[i]] = i;
  int32_t head = 0, tail = 0, count = 0;
#define PUSH(x)                      \
  do {                               \
    int32_t _x = (x);                \
    if (!S->inq[_x]) {               \
      S->inq[_x] = 1;                \
      S->touched[_x] = 1;            \
      S->ring[tail] = _x;            \
      tail = (tail + 1 == n) ? 0 : tail + 1; \
      ++count;                       \
    }                                \
  } while (0)
  for (int32_t i = 0; i < nchk; ++i) PUSH(chk[i]);
  if (cnt) cnt[ORC_CNT_CHECKLIST0] += nchk;
  int64_t changes = 0, gain = 0;
  move_t mv;
  for (;;) {
    while (count > 0 && changes < n) {
      int32_t a = S->ring[head];
      head = (head + 1 == n) ? 0 : head + 1;
      --count;
      S->inq[a] = 0;
      if (cnt) cnt[ORC_CNT_LS_POPS]++;
      best_move(h, &T, a, flags, &mv);
      if (mv.kind == 1) {
        int64_t r = apply_2opt(&T, &mv);
        PUSH(mv.w);
        PUSH(mv.x);
        PUSH(mv.y);
        PUSH(mv.z);
        if (cnt) {
          cnt[ORC_CNT_MOVES_2OPT]++;
          cnt[ORC_CNT_MOVED_ELEMS] += r;
        }
      } else if (mv.kind == 2) {
        int64_t r = apply_oropt(&T, &mv, S->tmp);
        PUSH(mv.p);
        PUSH(mv.q);
        PUSH(mv.b);
        PUSH(mv.e);
        PUSH(mv.f);
        PUSH(mv.l);
        if (cnt) {
          cnt[ORC_CNT_MOVES_OROPT]++;
          cnt[ORC_CNT_MOVED_ELEMS] += r;
        }
      } else if (mv.kind == 3) {
        int64_t r = apply_3opt(&T, &mv, S->tmp);
        for (int i = 0; i < 6; ++i) PUSH(mv.t[i]);
        if (cnt) {
          cnt[ORC_CNT_MOVES_3OPT]++;
          cnt[ORC_CNT_MOVED_ELEMS] += r;
        }
      } else {
        continue;
      }
      ++changes;
      gain += mv.gain;
    }
    if (!(flags & ORC_LS_SWEEP) || changes >= n) break;
    if (cnt) cnt[ORC_CNT_SWEEPS]++;
    int32_t pushed = 0;
    for (int32_t x = 0; x < n; ++x) {
      if (!S->touched[x]) continue;
      best_move(h, &T, x, flags, &mv);
      if (mv.kind != 0) {
        PUSH(x);
        ++pushed;
      }
    }
    if (pushed == 0) break;
  }
#undef PUSH
  /* leave the scratch flags clear for the next call */
  for (int32_t i = 0; i < n; ++i) {
    S->inq[i] = 0;
    S->touched[i] = 0;
  }
  if (cnt) cnt[ORC_CNT_LS_GAIN] += gain;
  return gain;
}

/* ------------------------------------------------------------------------ */
/* Colony update and Eq. (2) (Alg. 2, after the ants): iteration best (lowest
 * ant index on equal length), global best on strict improvement with new
 * limits, source = global best with probability p_source_gbest else the
 * iteration best (Sec. 5.3), then evaporation and deposit on the source.
 * reading: one clamp per slot, tau' = clamp(rho*tau + delta*[edge in source]),
 * delta = 1/cost(source), on every candidate slot (i, j) whose edge is in the
 * source, using the limits of the next iteration. */

static void colony_update(orc_instance *h, uint64_t t) {
  const int32_t n = h->n, k = h->k;
  int32_t ib = 0;
  for (int32_t a = 1; a < h->A; ++a)
    if (h->lens[a] < h->lens[ib]) ib = a;
  const int32_t *ibr = h->routes + (size_t)ib * n;
  if (h->lens[ib] < h->gb_len) {
    memcpy(h->gb_route, ibr, sizeof(int32_t) * (size_t)n);
    h->gb_len = h->lens[ib];
    update_limits(h);
  }
  uint64_t x = draw(h->p.seed, t, ~0ull, 0, ORC_PURPOSE_SOURCE);
  int use_gb = (double)(uint32_t)(x >> 40) < h->p.p_source_gbest * 16777216.0;
  if (use_gb)
    set_source(h, h->gb_route, h->gb_len);
  else
    set_source(h, ibr, h->lens[ib]);
  h->last_ib = ib;
  h->last_src_gb = use_gb;
  h->delta = (float)(1.0 / (double)h->src_len);
  for (int32_t i = 0; i < n; ++i) {
    int32_t sn = src_succ(h, i), pn = src_pred(h, i);
    for (int32_t s = 0; s < k; ++s) {
      int32_t j = h->cl[(size_t)i * k + s];
      float t1 = h->p.rho * h->tau[(size_t)i * k + s];
      float t2 = (j == sn || j == pn) ? t1 + h->delta : t1;
      if (t2 > h->tau_max) t2 = h->tau_max;
      if (t2 < h->tau_min) t2 = h->tau_min;
      h->tau[(size_t)i * k + s] = t2;
    }
  }
}

/* ------------------------------------------------------------------------ */

orc_instance *orc_build(const int32_t *xy, int32_t n, const orc_params *p,
                        int32_t n_threads) {
  if (!xy || !p || n < 4 || p->cl_size < 2 || p->bl_size < 0 ||
      p->n_ants < 1 || p->min_new_edges < 0 || !(p->rho >= 0.0f) ||
      !(p->rho < 1.0f) || !(p->p_best > 0.0) || !(p->p_best < 1.0) ||
      p->oropt_max_seg < 1 || p->oropt_max_seg > 64 || (p->ls_flags & ~15u) ||
      (p->min_new_edges_max > 0 && p->min_new_edges_max < p->min_new_edges))
    return NULL;
  for (int32_t i = 0; i < 2 * n; ++i)
    if (xy[i] < 0 || xy[i] >= (1 << 26)) return NULL;
  orc_instance *h = (orc_instance *)calloc(1, sizeof(orc_instance));
  h->n = n;
  h->p = *p;
  h->k = p->cl_size < n - 1 ? p->cl_size : n - 1;
  h->bl = p->bl_size < n - 1 - h->k ? p->bl_size : n - 1 - h->k;
  h->A = p->n_ants;
  h->m = p->min_new_edges;
  h->n_threads = n_threads > 0 ? n_threads : 1;
  h->xy = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n);
  memcpy(h->xy, xy, sizeof(int32_t) * 2 * (size_t)n);
  h->cl = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * h->k);
  h->bll = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n * h->bl + 1));
  h->eta = (float *)malloc(sizeof(float) * (size_t)n * h->k);
  h->tau = (float *)malloc(sizeof(float) * (size_t)n * h->k);
  h->src_route = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  h->src_pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  h->gb_route = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  h->routes = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * h->A);
  h->lens = (int64_t *)calloc((size_t)h->A, sizeof(int64_t));
  h->cnt = (int64_t *)calloc((size_t)h->A * ORC_NCNT, sizeof(int64_t));

  build_lists(h);
  /* duplicate points give a zero distance: rejected */
  for (int32_t i = 0; i < n; ++i)
    if (sqd(h->xy, i, h->cl[(size_t)i * h->k]) == 0) {
      orc_free(h);
      return NULL;
    }

  /* initial solution: nearest neighbour + LS over all nodes (2-opt, Or-opt
   * when enabled, and 3-opt with ORC_LS_INIT_3OPT) */
  scratch_t S;
  scratch_alloc(&S, n);
  int32_t *all = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t i = 0; i < n; ++i) all[i] = i;
  int64_t len = nearest_neighbour_tour(h, h->gb_route, S.visited);
  uint32_t init_flags =
      ORC_LS_2OPT | ORC_LS_SWEEP | (p->ls_flags & (ORC_LS_OROPT | ORC_LS_INIT_3OPT));
  len -= local_search(h, h->gb_route, all, n, init_flags, &S, h->init_cnt);
  free(all);
  scratch_free(&S);
  h->gb_len = len;
  h->init_len = len;
  h->p_root = pow(p->p_best, 1.0 / (double)n);
  update_limits(h);
  for (size_t i = 0; i < (size_t)n * h->k; ++i) h->tau[i] = h->tau_max;
  set_source(h, h->gb_route, h->gb_len);
  h->iter = 0;
  h->last_ib = -1;
  h->delta = 0.0f;
  return h;
}

void orc_free(orc_instance *h) {
  if (!h) return;
  free(h->xy);
  free(h->cl);
  free(h->bll);
  free(h->eta);
  free(h->tau);
  free(h->src_route);
  free(h->src_pos);
  free(h->gb_route);
  free(h->routes);
  free(h->lens);
  free(h->cnt);
  free(h);
}

void orc_run(orc_instance *h, int32_t iterations) {
  const int32_t n = h->n;
  for (int32_t it = 0; it < iterations; ++it) {
    uint64_t t = (uint64_t)(h->iter + 1);
    memset(h->cnt, 0, sizeof(int64_t) * (size_t)h->A * ORC_NCNT);
#pragma omp parallel num_threads(h->n_threads)
    {
      scratch_t S;
      scratch_alloc(&S, n);
#pragma omp for schedule(dynamic, 1)
      for (int32_t a = 0; a < h->A; ++a) {
        int32_t *route = h->routes + (size_t)a * n;
        int64_t *cnt = h->cnt + (size_t)a * ORC_NCNT;
        int32_t nchk = 0;
        int64_t len = construct(h, t, (uint64_t)a, route, S.visited, S.chk,
                                &nchk, cnt);
        if (h->p.ls_flags & (ORC_LS_2OPT | ORC_LS_OROPT))
          len -= local_search(h, route, S.chk, nchk, h->p.ls_flags & ~ORC_LS_INIT_3OPT,
                              &S, cnt);
        h->lens[a] = len;
      }
      scratch_free(&S);
    }
    colony_update(h, t);
    h->iter += 1;
  }
}

/* ------------------------------------------------------------------------ */

int64_t orc_best(const orc_instance *h, int32_t *tour) {
  if (tour) memcpy(tour, h->gb_route, sizeof(int32_t) * (size_t)h->n);
  return h->gb_len;
}
int64_t orc_source(const orc_instance *h, int32_t *tour) {
  if (tour) memcpy(tour, h->src_route, sizeof(int32_t) * (size_t)h->n);
  return h->src_len;
}
void orc_ant_routes(const orc_instance *h, int32_t *out) {
  memcpy(out, h->routes, sizeof(int32_t) * (size_t)h->n * h->A);
}
void orc_ant_lengths(const orc_instance *h, int64_t *out) {
  memcpy(out, h->lens, sizeof(int64_t) * (size_t)h->A);
}
void orc_ant_counters(const orc_instance *h, int64_t *out) {
  memcpy(out, h->cnt, sizeof(int64_t) * (size_t)h->A * ORC_NCNT);
}
void orc_init_counters(const orc_instance *h, int64_t *out) {
  memcpy(out, h->init_cnt, sizeof(int64_t) * ORC_NCNT);
}
void orc_pheromone(const orc_instance *h, float *out) {
  memcpy(out, h->tau, sizeof(float) * (size_t)h->n * h->k);
}
void orc_heuristic(const orc_instance *h, float *out) {
  memcpy(out, h->eta, sizeof(float) * (size_t)h->n * h->k);
}
void orc_lists(const orc_instance *h, int32_t *cl, int32_t *bl) {
  if (cl) memcpy(cl, h->cl, sizeof(int32_t) * (size_t)h->n * h->k);
  if (bl) memcpy(bl, h->bll, sizeof(int32_t) * (size_t)h->n * h->bl);
}
void orc_limits(const orc_instance *h, float *lim) {
  lim[0] = h->tau_min;
  lim[1] = h->tau_max;
  lim[2] = h->delta;
}
void orc_info(const orc_instance *h, int64_t *info) {
  info[0] = h->iter;
  info[1] = h->k;
  info[2] = h->bl;
  info[3] = h->last_ib;
  info[4] = h->last_src_gb;
  info[5] = h->init_len;
  info[6] = h->gb_len;
  info[7] = h->src_len;
}
void orc_set_source(orc_instance *h, const int32_t *tour) {
  set_source(h, tour, orc_tour_length(h->xy, h->n, tour));
}
void orc_set_pheromone(orc_instance *h, const float *tau) {
  memcpy(h->tau, tau, sizeof(float) * (size_t)h->n * h->k);
}

int64_t orc_construct(const orc_instance *h, uint64_t t, uint64_t ant,
                      int32_t *route, int32_t *checklist, int32_t *n_check,
                      int64_t *counters) {
  uint8_t *vis = (uint8_t *)malloc((size_t)h->n);
  int64_t len = construct(h, t, ant, route, vis, checklist, n_check, counters);
  free(vis);
  return len;
}

int64_t orc_local_search(const orc_instance *h, int32_t *route,
                         const int32_t *checklist, int32_t n_check,
                         uint32_t flags, int64_t *counters) {
  scratch_t S;
  scratch_alloc(&S, h->n);
  int64_t g = local_search(h, route, checklist, n_check, flags, &S, counters);
  scratch_free(&S);
  return g;
}

int64_t orc_nearest_neighbour(const orc_instance *h, int32_t *route) {
  uint8_t *vis = (uint8_t *)malloc((size_t)h->n);
  int64_t len = nearest_neighbour_tour(h, route, vis);
  free(vis);
  return len;
}

int64_t orc_best_move_gain(const orc_instance *h, const int32_t *route,
                           int32_t a, uint32_t flags) {
  int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)h->n);
  for (int32_t i = 0; i < h->n; ++i) pos[route[i]] = i;
  tour_t T = {(int32_t *)route, pos, h->n};
  move_t mv;
  best_move(h, &T, a, flags, &mv);
  free(pos);
  return mv.gain;
}
