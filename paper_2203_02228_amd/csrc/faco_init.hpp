// faco_init.hpp -- the initial solution's local search with 3-opt (gfx950).
//
// Alg. 2 starts from a nearest-neighbour tour improved with 2-opt and 3-opt
// (Sec. 4.3).  With FACO_LS_INIT_3OPT the ant kernel leaves the plain
// nearest-neighbour tour in ant slot 0 (route, pos, tour coordinates) and this
// kernel runs the whole initial search on it: every city listed in ascending
// original number, best improvement per listed city trying 2-opt, then
// Or-opt, then the pure 3-opt reconnection (two adjacent blocks exchange
// places, both keep their orientation), and the sweep over every touched
// city until none improves or n changes were made.  Setup only: one wave,
// written for clarity rather than speed.  Compound moves are realised as
// sequences of range reversals that leave exactly the array the move
// defines.
#pragma once
#include "device_common.hpp"
#include "faco_device.hpp"

namespace faco {

struct InitMove {
  int kind;      // 0 none, 1 2-opt, 2 Or-opt, 3 3-opt
  int64_t gain;
  int c;         // the winning combination (per kind)
};

struct InitTour {
  int n;
  int32_t *route, *pos;
  int2 *rxy;
  const int2 *xy;
  FACO_DEV int at(int p) const { return route[p]; }
  FACO_DEV int succ(int x) const {
    const int q = pos[x] + 1;
    return route[q == n ? 0 : q];
  }
  FACO_DEV int pred(int x) const {
    const int q = pos[x] - 1;
    return route[q < 0 ? n - 1 : q];
  }
  FACO_DEV int step(int x, int dir) const { return dir == 0 ? succ(x) : pred(x); }
  FACO_DEV int d(int u, int v) const { return cost(xy[u], xy[v]); }
};

FACO_DEV int cyc(int q, int n) {
  q %= n;
  return q < 0 ? q + n : q;
}

// The best improving move from city a, as the sequential search orders it:
// among equal gains the first in evaluation order.  Each kind's variants are
// numbered in that order; lanes take 64 at a time; the key packs the gain
// above the complement of the variant number.
FACO_DEV InitMove init_best_move(const Inst &I, const InitTour &T, int a, uint32_t flags) {
  const int n = I.n, K = I.k, lane = lane_id();
  InitMove mv = {0, 0, 0};
  if (flags & LS_2OPT) {
    // variant s < K: loop 1 over the candidates (succ), K + s: loop 2 (pred)
    const int as = T.succ(a), ap = T.pred(a);
    const int d_as = T.d(a, as), d_ap = T.d(ap, a);
    int64_t key = 0;
    for (int c = lane; c < 2 * K; c += kWave) {
      const int s = c < K ? c : c - K;
      const int b = I.cl[(size_t)a * K + s];
      const int d_ab = I.cl_d[(size_t)a * K + s];
      int64_t g = 0;
      if (c < K) {
        if (d_as > d_ab) {
          const int bs = T.succ(b);
          g = (int64_t)d_as + T.d(b, bs) - d_ab - T.d(as, bs);
        }
      } else if (d_ap > d_ab) {
        const int bp = T.pred(b);
        g = (int64_t)d_ap + T.d(bp, b) - d_ab - T.d(ap, bp);
      }
      const int64_t k = g > 0 ? ((g << 20) | (int64_t)(0xFFFFF - c)) : 0;
      key = k > key ? k : key;
    }
    key = wave_max_i64(key);
    if (key > 0) return {1, key >> 20, 0xFFFFF - (int)(key & 0xFFFFF)};
  }
  if (flags & LS_OROPT) {
    // variant ((slot * K) + s) * 2 + side; slots: forward L = 1..Lmax, then
    // backward L = 2..Lmax
    const int Lmax = I.oropt_max < n - 3 ? I.oropt_max : n - 3;
    const int nslot = Lmax + (Lmax - 1);
    const int pa = T.pos[a];
    int64_t key = 0;
    for (int c = lane; c < nslot * K * 2; c += kWave) {
      const int side = c & 1, s = (c >> 1) % K, slot = (c >> 1) / K;
      const int dir = slot < Lmax ? 0 : 1;
      const int L = dir == 0 ? slot + 1 : slot - Lmax + 2;
      const int fpos = dir == 0 ? pa : cyc(pa - (L - 1), n);
      const int lpos = cyc(fpos + L - 1, n);
      const int f = T.at(fpos), l = T.at(lpos);
      const int p = T.at(cyc(fpos - 1, n)), q = T.at(cyc(lpos + 1, n));
      const int o = dir == 0 ? l : f;
      const int d_rem_a = dir == 0 ? T.d(p, a) : T.d(a, q);
      const int b = I.cl[(size_t)a * K + s];
      if (cyc(T.pos[b] - fpos, n) < L) continue;
      const int d_ab = I.cl_d[(size_t)a * K + s];
      if (!(d_ab < d_rem_a)) continue;
      const int e = side == 0 ? T.succ(b) : T.pred(b);
      if (cyc(T.pos[e] - fpos, n) < L) continue;
      const int64_t g = (int64_t)T.d(p, f) + T.d(l, q) - T.d(p, q) + T.d(b, e) - d_ab - T.d(o, e);
      const int64_t k = g > 0 ? ((g << 20) | (int64_t)(0xFFFFF - c)) : 0;
      key = k > key ? k : key;
    }
    key = wave_max_i64(key);
    if (key > 0) return {2, key >> 20, 0xFFFFF - (int)(key & 0xFFFFF)};
  }
  if (flags & LS_INIT_3OPT) {
    // variant (dir * K + s) * K + r: orientation, t3 = slot s of cl(t2),
    // t5 = slot r of cl(t4)
    int64_t key = 0;
    for (int c = lane; c < 2 * K * K; c += kWave) {
      const int r = c % K, s = (c / K) % K, dir = c / (K * K);
      const int t1 = a, t2 = T.step(t1, dir);
      const int t3 = I.cl[(size_t)t2 * K + s];
      const int64_t g1 = (int64_t)T.d(t1, t2) - I.cl_d[(size_t)t2 * K + s];
      if (g1 <= 0 || t3 == t1) continue;
      const int t4 = T.step(t3, dir);
      if (t4 == t1) continue;
      const int t5 = I.cl[(size_t)t4 * K + r];
      const int64_t g2 = g1 + T.d(t3, t4) - I.cl_d[(size_t)t4 * K + r];
      if (g2 <= 0) continue;
      const int p2 = T.pos[t2];
      const int off3 = dir == 0 ? cyc(T.pos[t3] - p2, n) : cyc(p2 - T.pos[t3], n);
      const int off5 = dir == 0 ? cyc(T.pos[t5] - p2, n) : cyc(p2 - T.pos[t5], n);
      if (off5 >= off3) continue;
      const int t6 = T.step(t5, dir);
      const int64_t g = g2 + T.d(t5, t6) - T.d(t6, t1);
      const int64_t k = g > 0 ? ((g << 20) | (int64_t)(0xFFFFF - c)) : 0;
      key = k > key ? k : key;
    }
    key = wave_max_i64(key);
    if (key > 0) return {3, key >> 20, 0xFFFFF - (int)(key & 0xFFFFF)};
  }
  return mv;
}

// Reverse the cyclic range [s, s + L) of route/pos/rxy (one wave; pairs are
// disjoint, so each lane reads its pair and writes it back swapped).
FACO_DEV void init_reverse(const InitTour &T, int s, int L) {
  const int n = T.n;
  for (int i = lane_id(); i < L / 2; i += kWave) {
    const int p1 = cyc(s + i, n), p2 = cyc(s + L - 1 - i, n);
    const int v1 = T.route[p1], v2 = T.route[p2];
    const int2 c1 = T.rxy[p1], c2 = T.rxy[p2];
    T.route[p1] = v2;
    T.route[p2] = v1;
    T.rxy[p1] = c2;
    T.rxy[p2] = c1;
    T.pos[v2] = p1;
    T.pos[v1] = p2;
  }
  wave_fence();
}

// Apply move mv found at city a; ends[] gets the cities to list, in order.
// Returns the elements the move rewrites (the array move's own count).
FACO_DEV int64_t init_apply(const Inst &I, const InitTour &T, int a, const InitMove &mv,
                            int *ends, int &nends) {
  const int n = I.n, K = I.k;
  if (mv.kind == 1) {
    const int c = mv.c, s = c < K ? c : c - K;
    const int b = I.cl[(size_t)a * K + s];
    int w, x, y, z;
    if (c < K) {
      w = a; x = T.succ(a); y = b; z = T.succ(b);
    } else {
      w = T.pred(a); x = a; y = T.pred(b); z = b;
    }
    const int L1 = cyc(T.pos[y] - T.pos[x], n) + 1;
    int64_t moved;
    if (2 * L1 <= n) {
      init_reverse(T, T.pos[x], L1);
      moved = L1;
    } else {
      init_reverse(T, T.pos[z], n - L1);
      moved = n - L1;
    }
    ends[0] = w; ends[1] = x; ends[2] = y; ends[3] = z;
    nends = 4;
    return moved;
  }
  if (mv.kind == 2) {
    const int Lmax = I.oropt_max < n - 3 ? I.oropt_max : n - 3;
    const int c = mv.c, side = c & 1, s = (c >> 1) % K, slot = (c >> 1) / K;
    const int dir = slot < Lmax ? 0 : 1;
    const int L = dir == 0 ? slot + 1 : slot - Lmax + 2;
    const int pa = T.pos[a];
    const int fpos = dir == 0 ? pa : cyc(pa - (L - 1), n);
    const int lpos = cyc(fpos + L - 1, n);
    const int f = T.at(fpos), l = T.at(lpos);
    const int p = T.at(cyc(fpos - 1, n)), q = T.at(cyc(lpos + 1, n));
    const int b = I.cl[(size_t)a * K + s];
    const int e = side == 0 ? T.succ(b) : T.pred(b);
    const bool b_first = T.succ(b) == e;          // edge (b, e) in array order
    const int x1 = b_first ? b : e, x2 = b_first ? e : b;
    // inserted in array order: a..o when x1 == b, else o..a; the segment is
    // f..l in array order, so it is reversed when a is not where it must be
    const bool rev = b_first ? (a != f) : (a == f);
    const int D1 = cyc(T.pos[x1] - T.pos[q], n) + 1;
    const int D2 = cyc(T.pos[p] - T.pos[x2], n) + 1;
    int64_t moved;
    if (D1 <= D2) {
      // [segment][block q..x1] -> [block][inserted]
      init_reverse(T, fpos, L + D1);
      init_reverse(T, fpos, D1);
      if (!rev) init_reverse(T, cyc(fpos + D1, n), L);
      moved = D1 + L;
    } else {
      // [block x2..p][segment] -> [inserted][block]
      const int s0 = T.pos[x2];
      init_reverse(T, s0, D2 + L);
      init_reverse(T, cyc(s0 + L, n), D2);
      if (!rev) init_reverse(T, s0, L);
      moved = D2 + L;
    }
    ends[0] = p; ends[1] = q; ends[2] = b; ends[3] = e; ends[4] = f; ends[5] = l;
    nends = 6;
    return moved;
  }
  // 3-opt: [first block][second block] -> [second][first] in array order
  const int c = mv.c, r = c % K, s = (c / K) % K, dir = c / (K * K);
  const int t1 = a, t2 = T.step(t1, dir);
  const int t3 = I.cl[(size_t)t2 * K + s];
  const int t4 = T.step(t3, dir);
  const int t5 = I.cl[(size_t)t4 * K + r];
  const int t6 = T.step(t5, dir);
  int s0, L1, L2;
  if (dir == 0) {
    s0 = T.pos[t2];
    L1 = cyc(T.pos[t5] - s0, n) + 1;
    L2 = cyc(T.pos[t3] - T.pos[t6], n) + 1;
  } else {
    s0 = T.pos[t3];
    L1 = cyc(T.pos[t6] - s0, n) + 1;
    L2 = cyc(T.pos[t2] - T.pos[t5], n) + 1;
  }
  init_reverse(T, s0, L1 + L2);
  init_reverse(T, s0, L2);
  init_reverse(T, cyc(s0 + L2, n), L1);
  ends[0] = t1; ends[1] = t2; ends[2] = t3; ends[3] = t4; ends[4] = t5; ends[5] = t6;
  nends = 6;
  return (int64_t)L1 + L2;
}

// One wave.  LDS: "listed" and "touched" bitmaps (2 * ceil(n / 32) words).
// The queue ring is ant slot 0's ring (n entries).
__global__ void __launch_bounds__(64) init_search_kernel(Inst I) {
  extern __shared__ uint32_t init_lds[];
  const int n = I.n, W = (n + 31) >> 5, lane = lane_id();
  uint32_t *inq = init_lds, *touched = init_lds + W;
  InitTour T{n, I.routes, I.pos, I.rxy, I.xy};
  int32_t *ring = I.ring;
  const uint32_t flags =
      LS_2OPT | LS_SWEEP | (I.ls_flags & (LS_OROPT | LS_INIT_3OPT));
  // every city listed, in ascending original number
  for (int i = lane; i < n; i += kWave) ring[i] = I.int_of[i];
  for (int w = lane; w < W; w += kWave) {
    const int rem = n - w * 32;
    const uint32_t full = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
    inq[w] = full;
    touched[w] = full;
  }
  wave_fence();
  int head = 0, tail = 0, count = n;
  int64_t changes = 0, gain = 0;
  int64_t c_pops = 0, c_m2 = 0, c_mo = 0, c_m3 = 0, c_moved = 0, c_sweeps = 0;
  auto push = [&](int x) {
    if (!bit_get(inq, x)) {
      if (lane == 0) {
        bit_set(inq, x);
        bit_set(touched, x);
        ring[tail] = x;
      }
      tail = tail + 1 == n ? 0 : tail + 1;
      ++count;
      wave_fence();
    }
  };
  for (;;) {
    while (count > 0 && changes < n) {
      const int a = uniform_i(ring[head]);
      head = head + 1 == n ? 0 : head + 1;
      --count;
      if (lane == 0) bit_clear(inq, a);
      wave_fence();
      ++c_pops;
      const InitMove mv = init_best_move(I, T, a, flags);
      if (mv.kind == 0) continue;
      int ends[6], nends = 0;
      c_moved += init_apply(I, T, a, mv, ends, nends);
      for (int i = 0; i < nends; ++i) push(uniform_i(ends[i]));
      c_m2 += mv.kind == 1;
      c_mo += mv.kind == 2;
      c_m3 += mv.kind == 3;
      ++changes;
      gain += mv.gain;
    }
    if (changes >= n) break;
    ++c_sweeps;
    int pushed = 0;
    for (int o = 0; o < n; ++o) {
      const int x = uniform_i(I.int_of[o]);
      if (!bit_get(touched, x)) continue;
      if (init_best_move(I, T, x, flags).kind != 0) {
        push(x);
        ++pushed;
      }
    }
    if (pushed == 0) break;
  }
  for (int i = lane; i < n; i += kWave) I.gb_route[i] = T.route[i];
  if (lane == 0) {
    DevState *st = I.st;
    st->gb_len -= gain;
    st->init_len = st->gb_len;
    for (int c = 0; c < NCNT; ++c) st->init_cnt[c] = 0;
    st->init_cnt[CNT_LS_POPS] = c_pops;
    st->init_cnt[CNT_MOVES_2OPT] = c_m2;
    st->init_cnt[CNT_MOVES_OROPT] = c_mo;
    st->init_cnt[CNT_MOVES_3OPT] = c_m3;
    st->init_cnt[CNT_MOVED_ELEMS] = c_moved;
    st->init_cnt[CNT_SWEEPS] = c_sweeps;
    st->init_cnt[CNT_CHECKLIST0] = n;
    st->init_cnt[CNT_LS_GAIN] = gain;
  }
}

}  // namespace faco
