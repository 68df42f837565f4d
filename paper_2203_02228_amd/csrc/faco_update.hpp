// faco_update.hpp -- the per-instance update after the ants (colony: iteration
// best, global best + limits, source choice; source materialisation; Eq. (2)
// pheromone update) as device functions, shared by the per-phase kernels and
// the persistent batched kernel.
#pragma once
#include "device_common.hpp"
#include "faco_device.hpp"

namespace faco {

// ===================================================================== //
// Colony update (after the ants): iteration best, global best + limits
// (Sec. 4.5), source choice.  One wave.
// ===================================================================== //
FACO_DEV void limits(const Inst &I, int64_t gb_len, float &tmin_f, float &tmax_f) {
  const double tmax = 1.0 / ((double)gb_len * (1.0 - (double)I.rho));
  const double num = 1.0 - I.p_root;
  const double den = (double)(I.k - 1) * I.p_root;
  double tmin = tmax * num / den;
  if (tmin > tmax) tmin = tmax;
  tmax_f = (float)tmax;
  tmin_f = (float)tmin;
}

FACO_DEV void run_colony(const Inst &I) {
  const int lane = lane_id();
  DevState *st = I.st;
  const uint64_t t = (uint64_t)st->iter + 1;
  int64_t bl = INT64_MAX;
  int ba = 0x7fffffff;
  for (int a = lane; a < I.A; a += kWave) {
    const int64_t L = I.lens[a];
    if (L < bl) {
      bl = L;
      ba = a;
    }
  }
  const int64_t minL = wave_min_i64(bl);
  const int ib = wave_min_i32(bl == minL ? ba : 0x7fffffff);
  int64_t gb = st->gb_len;
  const bool improved = minL < gb;
  float tmin = st->tau_min, tmax = st->tau_max;
  if (improved) {
    gb = minL;
    limits(I, gb, tmin, tmax);
  }
  const uint64_t x = philox_word0(I.seed, t, ~0ull, 0, kPurposeSource);
  const bool use_gb = (double)(uint32_t)(x >> 40) < I.p_gb * 16777216.0;
  const int64_t src_len = use_gb ? gb : minL;
  const float delta = (float)(1.0 / (double)src_len);
  if (lane == 0) {
    st->gb_len = gb;
    st->tau_min = tmin;
    st->tau_max = tmax;
    st->ib = ib;
    st->improved = improved ? 1 : 0;
    st->src_gb = use_gb ? 1 : 0;
    st->src_len = src_len;
    st->delta = delta;
    st->iter = (int64_t)t;
  }
}

// Source materialisation: the chosen tour becomes source_solution (route and
// its inverse), the iteration best becomes the global best when it improved.
// init: source := global best (before the first iteration).
FACO_DEV void run_source(const Inst &I, int i, int init) {
  const int n = I.n;
  if (i >= n) return;
  const DevState *st = I.st;
  const int i1 = i + 1 == n ? 0 : i + 1, i0 = i == 0 ? n - 1 : i - 1;
  const int32_t *from;
  if (init) {
    from = I.gb_route;
  } else {
    const int32_t *ibr = ant_route(I, st->ib);
    from = (st->src_gb && !st->improved) ? I.gb_route : ibr;
  }
  const int node = from[i], next = from[i1], prev = from[i0];
  if (!init && st->improved) I.gb_route[i] = node;
  I.src_route[i] = node;
  I.src_pos[node] = i;
  I.src_adj[node] = make_int2(next, prev);
  const int2 xn = I.xy[node];
  I.src_xy[i] = xn;
  I.src_d[i] = cost(xn, I.xy[next]);
}

// Eq. (2) with the deposit on the source edges: tau' = clamp(rho tau + delta
// [edge in source]).  init: tau = tau_max everywhere.
FACO_DEV void run_pheromone(const Inst &I, size_t idx, int init) {
  const int n = I.n, K = I.k;
  if (idx >= (size_t)n * (size_t)K) return;
  const DevState *st = I.st;
  const float tmin = st->tau_min, tmax = st->tau_max;
  const int j = I.cl[idx];
  float tnew;
  if (init) {
    tnew = tmax;
  } else {
    const int i = (int)(idx / (size_t)K);
    const int2 adj = I.src_adj[i];
    const float t1 = I.rho * I.tau[idx];
    float t2 = (j == adj.x || j == adj.y) ? t1 + st->delta : t1;
    if (t2 > tmax) t2 = tmax;
    if (t2 < tmin) t2 = tmin;
    tnew = t2;
  }
  I.tau[idx] = tnew;
  // candidate row of city i moved to row src_pos(i), read by the next
  // construction: the city, its Eq. (1) weight, source position and cost
  const int i = (int)(idx / (size_t)K), s = (int)(idx - (size_t)i * K);
  const size_t o = srow(I.src_pos[i], s, K);
  I.scl[o] = j;
  I.sw[o] = tnew * I.eta[idx];
  I.ssp[o] = I.src_pos[j];
  I.sd[o] = I.cl_d[idx];
}

}  // namespace faco
