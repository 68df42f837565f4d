// faco_kernels.hpp -- HIP kernels of the FACO hot path for gfx950.
//
// One wavefront (64 lanes) owns one ant: the candidate row of the current city
// is spread over the lanes, the Eq. (1) cumulative sums are formed lane-wise in
// slot order, the choice is a ballot, the copy-from-source step and the
// 2-opt/Or-opt array rewrites move 64 elements per instruction.  Visited and
// "on the checklist" sets are bitmaps in LDS; tours live in HBM.
#pragma once
#include "device_common.hpp"
#include "faco_device.hpp"

namespace faco {

FACO_DEV int wrapn(int q, int n) {
  q %= n;
  return q < 0 ? q + n : q;
}
// for 0 <= q < 2n
FACO_DEV int wrap1(int q, int n) { return q >= n ? q - n : q; }

// ===================================================================== //
// Next-city choice (Eq. (1), then the backup list, then the nearest
// unvisited city).  Uniform result across the wave.
// ===================================================================== //
FACO_DEV int select_next(const Inst &I, int u, int2 xu, const uint32_t *vis,
                         bool greedy, uint64_t t, uint64_t ant, uint64_t step,
                         int64_t *cnt) {
  const int K = I.k, lane = lane_id();
  const size_t row = (size_t)u * (size_t)K;
  int cand = -1;
  bool unv = false;
  float w = 0.0f;
  if (lane < K) {
    cand = I.cl[row + lane];
    unv = !bit_get(vis, cand);
    if (!greedy && unv) w = I.tau[row + lane] * I.eta[row + lane];
  }
  const uint64_t um = ballot(unv);
  if (um) {
    if (greedy) return readlane_i(cand, ctz64(um));
    // cumulative sum in slot order: lane s holds fl(...fl(w_0 + w_1)... + w_s)
    float P = 0.0f;
    for (int j = 0; j < K; ++j) {
      float wj = readlane_f(w, j);
      if (j <= lane) P = P + wj;
    }
    const float total = readlane_f(P, K - 1);
    const float U = unit24(philox_word0(I.seed, t, ant, step, kPurposeRoulette));
    const float r = U * total;
    const uint64_t sm = ballot(lane < K && P > r);
    const int s = sm ? ctz64(sm) : msb64(um);
    return readlane_i(cand, s);
  }
  // backup list: first unvisited
  int b = -1;
  bool bu = false;
  if (lane < I.bl) {
    b = I.bll[(size_t)u * (size_t)I.bl + lane];
    bu = !bit_get(vis, b);
  }
  const uint64_t bm = ballot(bu);
  if (bm) {
    cnt[CNT_BACKUP]++;
    return readlane_i(b, ctz64(bm));
  }
  // best heuristic value = nearest unvisited city, ties by smaller id
  cnt[CNT_FALLBACK]++;
  int64_t bd = INT64_MAX;
  int bj = 0x7fffffff;
  for (int j = lane; j < I.n; j += kWave) {
    if (!bit_get(vis, j)) {
      int64_t d = (int64_t)sqd(xu, I.xy[j]);
      if (d < bd) {
        bd = d;
        bj = j;
      }
    }
  }
  const int64_t md = wave_min_i64(bd);
  return wave_min_i32(bd == md ? bj : 0x7fffffff);
}

// ===================================================================== //
// Copy-from-source: append source cities in direction `dir` starting after
// source position pv while they are unvisited.  Returns the count.
// ===================================================================== //
FACO_DEV int copy_run(const Inst &I, int dir, int pv, int &k, int &u, int2 &xu,
                      int64_t &len, int32_t *route, int32_t *pos,
                      uint32_t *vis) {
  const int n = I.n, lane = lane_id();
  int app = 0, pcur = pv;
  for (;;) {
    const int q = wrapn(pcur + dir * (lane + 1), n);
    const int c = I.src_route[q];
    const bool vc = bit_get(vis, c);
    const uint64_t stop = ballot(vc);
    const int j = stop ? ctz64(stop) : kWave;
    const int2 xc = I.xy[c];
    const int px = __shfl_up(xc.x, 1), py = __shfl_up(xc.y, 1);
    const int2 xp = lane == 0 ? xu : make_int2(px, py);
    const int d = lane < j ? cost(xp, xc) : 0;
    if (lane < j) {
      route[k + lane] = c;
      pos[c] = k + lane;
      bit_set(vis, c);
    }
    len += wave_sum_i32(d);
    if (j > 0) {
      u = readlane_i(c, j - 1);
      xu = readlane_i2(xc, j - 1);
    }
    k += j;
    app += j;
    pcur = wrapn(pcur + dir * j, n);
    wave_fence();
    if (j < kWave) break;
  }
  return app;
}

// ===================================================================== //
// Focused construction (Alg. 2 inner loop).  greedy: nearest-neighbour tour
// from city 0 (initial solution), no source, no copy.
// The checklist is written into ring[0..nchk) with its LDS bits set in inq.
// ===================================================================== //
FACO_DEV int64_t construct(const Inst &I, uint64_t t, int ant, bool greedy,
                           int32_t *route, int32_t *pos, int32_t *ring,
                           uint32_t *vis, uint32_t *inq, int W, int &nchk,
                           int64_t *cnt) {
  const int n = I.n, lane = lane_id();
  for (int w = lane; w < W; w += kWave) {
    vis[w] = 0u;
    inq[w] = 0u;
  }
  wave_fence();
  const int r0 = greedy ? 0
                        : uniform_node(philox_word0(I.seed, t, (uint64_t)ant, 0,
                                                    kPurposeStart),
                                       n);
  int u = r0;
  int2 xu = I.xy[u];
  const int2 x0 = xu;
  if (lane == 0) {
    route[0] = u;
    pos[u] = 0;
    bit_set(vis, u);
  }
  wave_fence();
  int k = 1, new_edges = 0;
  nchk = 0;
  int64_t len = 0;
  uint64_t step = 0;
  while (k < n) {
    const int v = select_next(I, u, xu, vis, greedy, t, (uint64_t)ant, step, cnt);
    ++step;
    const int2 xv = I.xy[v];
    len += cost(xu, xv);
    if (lane == 0) {
      route[k] = v;
      pos[v] = k;
      bit_set(vis, v);
    }
    ++k;
    if (!greedy) {
      const int ps = I.src_pos[u];
      const int sn = I.src_route[ps + 1 == n ? 0 : ps + 1];
      const int pn = I.src_route[ps == 0 ? n - 1 : ps - 1];
      if (v != sn && v != pn) {
        ++new_edges;
        if (lane == 0) {
          ring[nchk] = v;
          bit_set(inq, v);
        }
        ++nchk;
      }
    }
    u = v;
    xu = xv;
    wave_fence();
    if (!greedy && new_edges >= I.m && k < n) {
      const int pv = I.src_pos[v];
      int app = copy_run(I, +1, pv, k, u, xu, len, route, pos, vis);
      if (app == 0) app = copy_run(I, -1, pv, k, u, xu, len, route, pos, vis);
      cnt[CNT_COPIED] += app;
    }
  }
  len += cost(xu, x0);
  cnt[CNT_ACO_STEPS] += (int64_t)step;
  cnt[CNT_NEW_EDGES] += new_edges;
  return len;
}

// ===================================================================== //
// Local search (Alg. 3 + Or-opt + sweep)
// ===================================================================== //
struct Move {
  int kind;  // 0 none, 1 2-opt, 2 Or-opt
  int gain;
  int w, x, y, z;
  int f, l, p, q, a, o, b, e, L;
};

// Or-opt variants in evaluation order, one fixed slot each:
// slot 0..2 = forward L = 1..3, slot 3..4 = backward L = 2..3.
constexpr int kOrSlots = 5;
struct OrVariant {
  int f, l, p, q, o, fpos, L, rem_a, g_rem;
  int2 xo;
  bool valid;
};

FACO_DEV void or_variants(const Inst &I, int a, int pa, int2 xa, int nb,
                          OrVariant (&vs)[kOrSlots]) {
  // nb on lane j holds route[pa + j - 3]
  const int n = I.n;
  int Lmax = I.oropt_max;
  if (Lmax > n - 3) Lmax = n - 3;
#pragma unroll
  for (int slot = 0; slot < kOrSlots; ++slot) {
    const int dir = slot < 3 ? 0 : 1;
    const int L = slot < 3 ? slot + 1 : slot - 1;
    OrVariant &v = vs[slot];
    v.L = L;
    v.valid = L <= Lmax;
    if (dir == 0) {
      v.f = a;
      v.l = readlane_i(nb, 3 + L - 1);
      v.p = readlane_i(nb, 2);
      v.q = readlane_i(nb, 3 + L);
      v.o = v.l;
      v.fpos = pa;
    } else {
      v.l = a;
      v.f = readlane_i(nb, 3 - L + 1);
      v.p = readlane_i(nb, 3 - L);
      v.q = readlane_i(nb, 4);
      v.o = v.f;
      v.fpos = wrapn(pa - L + 1, n);
    }
    const int2 xf = I.xy[v.f], xl = I.xy[v.l], xp = I.xy[v.p], xq = I.xy[v.q];
    v.xo = dir == 0 ? xl : xf;
    v.rem_a = dir == 0 ? cost(xp, xa) : cost(xa, xq);
    v.g_rem = cost(xp, xf) + cost(xl, xq) - cost(xp, xq);
  }
}

// Best move from city a, evaluated across the wave.  Ties resolve to the
// first candidate in the sequential evaluation order of Alg. 3.
FACO_DEV void eval_best_move(const Inst &I, uint32_t flags, int a,
                             const int32_t *route, const int32_t *pos,
                             Move &mv) {
  const int n = I.n, K = I.k, lane = lane_id();
  mv.kind = 0;
  mv.gain = 0;
  const int pa = pos[a];
  const int nb = lane < 7 ? route[wrapn(pa + lane - 3, n)] : 0;
  const int a_s = readlane_i(nb, 4), a_p = readlane_i(nb, 2);
  const int2 xa = I.xy[a], xas = I.xy[a_s], xap = I.xy[a_p];
  const size_t row = (size_t)a * (size_t)K;
  if (flags & LS_2OPT) {
    const int d_as = cost(xa, xas), d_ap = cost(xap, xa);
    const int s = lane & 31;
    const bool loop2 = lane >= 32;
    const bool act = s < K;
    int b = 0, other = 0, g = 0;
    if (act) {
      b = I.cl[row + s];
      const int2 xb = I.xy[b];
      const int d_ab = cost(xa, xb);
      if (loop2 ? (d_ap > d_ab) : (d_as > d_ab)) {
        const int pb = pos[b];
        other = route[loop2 ? (pb == 0 ? n - 1 : pb - 1) : (pb + 1 == n ? 0 : pb + 1)];
        const int2 xo = I.xy[other];
        g = loop2 ? (d_ap + cost(xo, xb) - d_ab - cost(xap, xo))
                  : (d_as + cost(xb, xo) - d_ab - cost(xas, xo));
      }
    }
    const int64_t key = g > 0 ? (((int64_t)g << 8) | (int64_t)(255 - lane)) : 0;
    const int64_t best = wave_max_i64(key);
    if (best > 0) {
      const int bl = 255 - (int)(best & 255);
      const int bb = readlane_i(b, bl), oo = readlane_i(other, bl);
      mv.kind = 1;
      mv.gain = (int)(best >> 8);
      if (bl < 32) {
        mv.w = a; mv.x = a_s; mv.y = bb; mv.z = oo;
      } else {
        mv.w = a_p; mv.x = a; mv.y = oo; mv.z = bb;
      }
      return;
    }
  }
  if (!(flags & LS_OROPT)) return;
  OrVariant vs[kOrSlots];
  or_variants(I, a, pa, xa, nb, vs);
  int lbest = 0, lidx = 0;
  int b = 0, bs = 0, bp = 0;
  if (lane < K) {
    b = I.cl[row + lane];
    const int pb = pos[b];
    const int pbs = pb + 1 == n ? 0 : pb + 1, pbp = pb == 0 ? n - 1 : pb - 1;
    bs = route[pbs];
    bp = route[pbp];
    const int2 xb = I.xy[b], xbs = I.xy[bs], xbp = I.xy[bp];
    const int d_ab = cost(xa, xb), d_bs = cost(xb, xbs), d_bp = cost(xb, xbp);
#pragma unroll
    for (int vi = 0; vi < kOrSlots; ++vi) {
      const OrVariant &v = vs[vi];
      if (!v.valid) continue;
      if (wrapn(pb - v.fpos, n) < v.L) continue;
      if (!(d_ab < v.rem_a)) continue;
      if (wrapn(pbs - v.fpos, n) >= v.L) {
        const int g = v.g_rem + d_bs - d_ab - cost(v.xo, xbs);
        if (g > lbest) {
          lbest = g;
          lidx = (vi * K + lane) * 2 + 0;
        }
      }
      if (wrapn(pbp - v.fpos, n) >= v.L) {
        const int g = v.g_rem + d_bp - d_ab - cost(v.xo, xbp);
        if (g > lbest) {
          lbest = g;
          lidx = (vi * K + lane) * 2 + 1;
        }
      }
    }
  }
  const int64_t key = lbest > 0 ? (((int64_t)lbest << 16) | (int64_t)(0xFFFF - lidx)) : 0;
  const int64_t best = wave_max_i64(key);
  if (best > 0) {
    const int idx = 0xFFFF - (int)(best & 0xFFFF);
    const int side = idx & 1;
    const int s = (idx >> 1) % K;
    const int vi = (idx >> 1) / K;
    OrVariant v = vs[0];
#pragma unroll
    for (int j = 1; j < kOrSlots; ++j)
      if (j == vi) v = vs[j];
    mv.kind = 2;
    mv.gain = (int)(best >> 16);
    mv.f = v.f; mv.l = v.l; mv.p = v.p; mv.q = v.q; mv.o = v.o; mv.L = v.L;
    mv.a = a;
    mv.b = readlane_i(b, s);
    mv.e = side ? readlane_i(bp, s) : readlane_i(bs, s);
  }
}

// Lane-serial test: does city x have an improving move?  (used by the sweep,
// one city per lane)
FACO_DEV bool has_improving(const Inst &I, uint32_t flags, int x,
                            const int32_t *route, const int32_t *pos) {
  const int n = I.n, K = I.k;
  const int px = pos[x];
  const int xs = route[px + 1 == n ? 0 : px + 1];
  const int xp = route[px == 0 ? n - 1 : px - 1];
  const int2 cx = I.xy[x], cxs = I.xy[xs], cxp = I.xy[xp];
  const size_t row = (size_t)x * (size_t)K;
  if (flags & LS_2OPT) {
    const int d_s = cost(cx, cxs), d_p = cost(cxp, cx);
    for (int s = 0; s < K; ++s) {
      const int b = I.cl[row + s];
      const int2 cb = I.xy[b];
      const int d_xb = cost(cx, cb);
      if (d_s <= d_xb && d_p <= d_xb) break;  // list sorted by distance
      const int pb = pos[b];
      if (d_s > d_xb) {
        const int bs = route[pb + 1 == n ? 0 : pb + 1];
        const int2 cbs = I.xy[bs];
        if (d_s + cost(cb, cbs) - d_xb - cost(cxs, cbs) > 0) return true;
      }
      if (d_p > d_xb) {
        const int bp = route[pb == 0 ? n - 1 : pb - 1];
        const int2 cbp = I.xy[bp];
        if (d_p + cost(cbp, cb) - d_xb - cost(cxp, cbp) > 0) return true;
      }
    }
  }
  if (flags & LS_OROPT) {
    int Lmax = I.oropt_max;
    if (Lmax > n - 3) Lmax = n - 3;
    for (int dir = 0; dir < 2; ++dir) {
      for (int L = (dir == 0 ? 1 : 2); L <= Lmax; ++L) {
        int f, l, p, q, fpos;
        if (dir == 0) {
          fpos = px;
          f = x;
          l = route[wrapn(px + L - 1, n)];
          p = xp;
          q = route[wrapn(px + L, n)];
        } else {
          fpos = wrapn(px - L + 1, n);
          l = x;
          f = route[fpos];
          p = route[wrapn(px - L, n)];
          q = xs;
        }
        const int2 cf = I.xy[f], cl_ = I.xy[l], cp = I.xy[p], cq = I.xy[q];
        const int2 co = dir == 0 ? cl_ : cf;
        const int rem = dir == 0 ? cost(cp, cx) : cost(cx, cq);
        const int g_rem = cost(cp, cf) + cost(cl_, cq) - cost(cp, cq);
        for (int s = 0; s < K; ++s) {
          const int b = I.cl[row + s];
          const int2 cb = I.xy[b];
          const int d_xb = cost(cx, cb);
          if (!(d_xb < rem)) break;  // list sorted by distance
          const int pb = pos[b];
          if (wrapn(pb - fpos, n) < L) continue;
          const int pbs = pb + 1 == n ? 0 : pb + 1, pbp = pb == 0 ? n - 1 : pb - 1;
          if (wrapn(pbs - fpos, n) >= L) {
            const int e = route[pbs];
            const int2 ce = I.xy[e];
            if (g_rem + cost(cb, ce) - d_xb - cost(co, ce) > 0) return true;
          }
          if (wrapn(pbp - fpos, n) >= L) {
            const int e = route[pbp];
            const int2 ce = I.xy[e];
            if (g_rem + cost(cb, ce) - d_xb - cost(co, ce) > 0) return true;
          }
        }
      }
    }
  }
  return false;
}

// Reverse the cyclic array range of length L starting at s (wave-wide).
FACO_DEV void reverse_range(int n, int s, int L, int32_t *route, int32_t *pos) {
  const int lane = lane_id();
  const int half = L >> 1;
  for (int base = 0; base < half; base += 4 * kWave) {
    int p1[4], p2[4], v1[4], v2[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = base + c * kWave + lane;
      if (i < half) {
        p1[c] = wrap1(s + i, n);
        p2[c] = wrap1(s + L - 1 - i, n);
        v1[c] = route[p1[c]];
        v2[c] = route[p2[c]];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = base + c * kWave + lane;
      if (i < half) {
        route[p1[c]] = v2[c];
        route[p2[c]] = v1[c];
        pos[v2[c]] = p1[c];
        pos[v1[c]] = p2[c];
      }
    }
  }
  wave_fence();
}

// "Flip a section between x and y": the shorter of the paths x..y and z..w.
FACO_DEV int apply_2opt(const Inst &I, const Move &mv, int32_t *route,
                        int32_t *pos) {
  const int n = I.n;
  const int px = pos[mv.x], py = pos[mv.y];
  const int L1 = wrapn(py - px, n) + 1;
  if (2 * L1 <= n) {
    reverse_range(n, px, L1, route, pos);
    return L1;
  }
  const int pz = pos[mv.z];
  reverse_range(n, pz, n - L1, route, pos);
  return n - L1;
}

// Or-opt: the segment and the shorter block between its old place and the
// insertion edge exchange places (block keeps its orientation).
FACO_DEV int apply_oropt(const Inst &I, const Move &mv, int32_t *route,
                         int32_t *pos) {
  const int n = I.n, L = mv.L, lane = lane_id();
  const int pb = pos[mv.b];
  const int sb = route[pb + 1 == n ? 0 : pb + 1];
  int x1, x2;
  if (sb == mv.e) {
    x1 = mv.b;
    x2 = mv.e;
  } else {
    x1 = mv.e;
    x2 = mv.b;
  }
  const int fpos = pos[mv.f];
  // segment in forward order, reordered into the inserted orientation
  const int segv = lane < L ? route[wrap1(fpos + lane, n)] : 0;
  const bool rev = (mv.a != mv.f) != (x1 != mv.b);
  const int src_lane = rev ? (L - 1 - lane) : lane;
  const int ins = __shfl(segv, src_lane < 0 ? 0 : src_lane);
  const int pq = pos[mv.q], px1 = pos[x1], pp = pos[mv.p], px2 = pos[x2];
  const int D1 = wrapn(px1 - pq, n) + 1;
  const int D2 = wrapn(pp - px2, n) + 1;
  if (D1 <= D2) {
    // block q..x1 moves back by L to start at fpos; segment follows it
    for (int base = 0; base < D1; base += 4 * kWave) {
      int v[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = base + c * kWave + lane;
        if (i < D1) v[c] = route[wrap1(pq + i, n)];
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = base + c * kWave + lane;
        if (i < D1) {
          const int d = wrap1(fpos + i, n);
          route[d] = v[c];
          pos[v[c]] = d;
        }
      }
    }
    wave_fence();
    if (lane < L) {
      const int d = wrapn(fpos + D1 + lane, n);
      route[d] = ins;
      pos[ins] = d;
    }
    wave_fence();
    return D1 + L;
  }
  // block x2..p moves forward by L; segment goes in front of it
  const int top = ((D2 - 1) / (4 * kWave)) * (4 * kWave);
  for (int base = top; base >= 0; base -= 4 * kWave) {
    int v[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = base + c * kWave + lane;
      if (i < D2) v[c] = route[wrap1(px2 + i, n)];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = base + c * kWave + lane;
      if (i < D2) {
        const int d = wrapn(px2 + L + i, n);
        route[d] = v[c];
        pos[v[c]] = d;
      }
    }
  }
  wave_fence();
  if (lane < L) {
    const int d = wrap1(px2 + lane, n);
    route[d] = ins;
    pos[ins] = d;
  }
  wave_fence();
  return D2 + L;
}

struct Queue {
  int head, tail, count;
};

FACO_DEV void push(int n, int x, Queue &Q, int32_t *ring, uint32_t *inq,
                   uint32_t *touched) {
  if (!bit_get(inq, x)) {
    if (lane_id() == 0) {
      bit_set(inq, x);
      bit_set(touched, x);
      ring[Q.tail] = x;
    }
    Q.tail = Q.tail + 1 == n ? 0 : Q.tail + 1;
    Q.count++;
    wave_fence();
  }
}

// Sweep: test every touched city (ascending id) and list the improvable ones.
FACO_DEV int sweep(const Inst &I, uint32_t flags, int W, Queue &Q,
                   const int32_t *route, const int32_t *pos, int32_t *ring,
                   uint32_t *inq, uint32_t *touched) {
  const int lane = lane_id();
  int pushed = 0;
  int bx = -1, bcount = 0;
  auto flush = [&](int cnt) {
    bool f = false;
    if (lane < cnt) f = has_improving(I, flags, bx, route, pos);
    uint64_t m = ballot(f);
    while (m) {
      const int l = ctz64(m);
      m &= m - 1;
      push(I.n, readlane_i(bx, l), Q, ring, inq, touched);
      ++pushed;
    }
  };
  for (int w0 = 0; w0 < W; w0 += kWave) {
    const uint32_t word = (w0 + lane < W) ? touched[w0 + lane] : 0u;
    uint64_t nz = ballot(word != 0u);
    while (nz) {
      const int l = ctz64(nz);
      nz &= nz - 1;
      uint32_t bits = (uint32_t)readlane_i((int)word, l);
      while (bits) {
        const int bpos = __builtin_ctz(bits);
        bits &= bits - 1;
        const int x = (w0 + l) * 32 + bpos;
        if (lane == bcount) bx = x;
        if (++bcount == kWave) {
          flush(kWave);
          bcount = 0;
        }
      }
    }
  }
  if (bcount) flush(bcount);
  return pushed;
}

FACO_DEV int64_t local_search(const Inst &I, uint32_t flags, int32_t *route,
                              int32_t *pos, int32_t *ring, uint32_t *inq,
                              uint32_t *touched, int W, Queue Q, int64_t *cnt) {
  const int n = I.n;
  int64_t changes = 0, gain = 0, changes_at_sweep = -1;
  Move mv;
  for (;;) {
    while (Q.count > 0 && changes < n) {
      const int a = ring[Q.head];
      Q.head = Q.head + 1 == n ? 0 : Q.head + 1;
      Q.count--;
      if (lane_id() == 0) bit_clear(inq, a);
      wave_fence();
      cnt[CNT_LS_POPS]++;
      eval_best_move(I, flags, a, route, pos, mv);
      if (mv.kind == 1) {
        cnt[CNT_MOVED_ELEMS] += apply_2opt(I, mv, route, pos);
        push(n, mv.w, Q, ring, inq, touched);
        push(n, mv.x, Q, ring, inq, touched);
        push(n, mv.y, Q, ring, inq, touched);
        push(n, mv.z, Q, ring, inq, touched);
        cnt[CNT_MOVES_2OPT]++;
      } else if (mv.kind == 2) {
        cnt[CNT_MOVED_ELEMS] += apply_oropt(I, mv, route, pos);
        push(n, mv.p, Q, ring, inq, touched);
        push(n, mv.q, Q, ring, inq, touched);
        push(n, mv.b, Q, ring, inq, touched);
        push(n, mv.e, Q, ring, inq, touched);
        push(n, mv.f, Q, ring, inq, touched);
        push(n, mv.l, Q, ring, inq, touched);
        cnt[CNT_MOVES_OROPT]++;
      } else {
        continue;
      }
      ++changes;
      gain += mv.gain;
    }
    if (!(flags & LS_SWEEP) || changes >= n) break;
    // Every city a sweep lists has an improving move, so a sweep that was
    // followed by no change can only come from the two evaluators disagreeing;
    // stop instead of spinning.
    if (changes == changes_at_sweep) break;
    changes_at_sweep = changes;
    cnt[CNT_SWEEPS]++;
    if (sweep(I, flags, W, Q, route, pos, ring, inq, touched) == 0) break;
  }
  cnt[CNT_LS_GAIN] += gain;
  return gain;
}

// ===================================================================== //
// One ant: construction + local search.  mode 0: ant `ant` of iteration
// st->iter + 1.  mode 1: initial solution (nearest neighbour + LS over all
// cities) written to the global best.
// ===================================================================== //
FACO_DEV void run_ant(const Inst &I, int ant, int mode, uint32_t *lds) {
  const int n = I.n, lane = lane_id();
  const int W = (n + 31) >> 5;
  uint32_t *vis = lds;
  uint32_t *inq = lds + W;
  int32_t *route = I.routes + (size_t)ant * (size_t)n;
  int32_t *pos = I.pos + (size_t)ant * (size_t)n;
  int32_t *ring = I.ring + (size_t)ant * (size_t)n;
  int64_t cnt[NCNT];
#pragma unroll
  for (int c = 0; c < NCNT; ++c) cnt[c] = 0;
  const bool init = mode == 1;
  const uint64_t t = (uint64_t)I.st->iter + 1;
  int nchk = 0;
  int64_t len = construct(I, t, ant, init, route, pos, ring, vis, inq, W, nchk, cnt);
  uint32_t flags = I.ls_flags;
  Queue Q;
  if (init) {
    // the initial solution reports only its local-search counters
    for (int c = 0; c < CNT_LS_POPS; ++c) cnt[c] = 0;
    flags = LS_2OPT | LS_SWEEP | (I.ls_flags & LS_OROPT);
    for (int i = lane; i < n; i += kWave) ring[i] = i;
    for (int w = lane; w < W; w += kWave) {
      const int rem = n - w * 32;
      const uint32_t full = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
      inq[w] = full;
      vis[w] = full;  // touched
    }
    Q.head = 0;
    Q.tail = 0;
    Q.count = n;
    cnt[CNT_CHECKLIST0] = n;
  } else {
    for (int w = lane; w < W; w += kWave) vis[w] = 0u;
    wave_fence();
    for (int i = lane; i < nchk; i += kWave) bit_set(vis, ring[i]);
    Q.head = 0;
    Q.tail = nchk;
    Q.count = nchk;
    if (flags & (LS_2OPT | LS_OROPT)) cnt[CNT_CHECKLIST0] = nchk;
  }
  wave_fence();
  if (flags & (LS_2OPT | LS_OROPT))
    len -= local_search(I, flags, route, pos, ring, inq, vis, W, Q, cnt);
  if (init) {
    for (int i = lane; i < n; i += kWave) I.gb_route[i] = route[i];
    if (lane == 0) {
      I.st->gb_len = len;
      I.st->init_len = len;
      for (int c = 0; c < NCNT; ++c) I.st->init_cnt[c] = cnt[c];
    }
  } else if (lane == 0) {
    I.lens[ant] = len;
    for (int c = 0; c < NCNT; ++c) I.cnt[(size_t)ant * NCNT + c] = cnt[c];
  }
}

__global__ void __launch_bounds__(64) ant_kernel(Inst I, int mode) {
  extern __shared__ uint32_t lds[];
  run_ant(I, (int)blockIdx.x, mode, lds);
}

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

__global__ void __launch_bounds__(64) colony_kernel(Inst I) { run_colony(I); }

// Source materialisation: the chosen tour becomes source_solution (route and
// its inverse), the iteration best becomes the global best when it improved.
// init: source := global best (before the first iteration).
FACO_DEV void run_source(const Inst &I, int i, int init) {
  const int n = I.n;
  if (i >= n) return;
  const DevState *st = I.st;
  int node;
  if (init) {
    node = I.gb_route[i];
  } else {
    const int32_t *ibr = I.routes + (size_t)st->ib * (size_t)n;
    const int v = ibr[i];
    node = (st->src_gb && !st->improved) ? I.gb_route[i] : v;
    if (st->improved) I.gb_route[i] = v;
  }
  I.src_route[i] = node;
  I.src_pos[node] = i;
}

__global__ void __launch_bounds__(256) source_kernel(Inst I, int init) {
  run_source(I, (int)(blockIdx.x * blockDim.x + threadIdx.x), init);
}

// Eq. (2) with the deposit on the source edges: tau' = clamp(rho tau + delta
// [edge in source]).  init: tau = tau_max everywhere.
FACO_DEV void run_pheromone(const Inst &I, size_t idx, int init) {
  const int n = I.n, K = I.k;
  if (idx >= (size_t)n * (size_t)K) return;
  const DevState *st = I.st;
  const float tmin = st->tau_min, tmax = st->tau_max;
  if (init) {
    I.tau[idx] = tmax;
    return;
  }
  const int i = (int)(idx / (size_t)K);
  const int p = I.src_pos[i];
  const int sn = I.src_route[p + 1 == n ? 0 : p + 1];
  const int pn = I.src_route[p == 0 ? n - 1 : p - 1];
  const int j = I.cl[idx];
  const float t1 = I.rho * I.tau[idx];
  float t2 = (j == sn || j == pn) ? t1 + st->delta : t1;
  if (t2 > tmax) t2 = tmax;
  if (t2 < tmin) t2 = tmin;
  I.tau[idx] = t2;
}

__global__ void __launch_bounds__(256) pheromone_kernel(Inst I, int init) {
  run_pheromone(I, (size_t)blockIdx.x * blockDim.x + threadIdx.x, init);
}

// Limits of the initial solution; state before the first iteration.
__global__ void init_state_kernel(Inst I) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  DevState *st = I.st;
  float tmin, tmax;
  limits(I, st->gb_len, tmin, tmax);
  st->tau_min = tmin;
  st->tau_max = tmax;
  st->src_len = st->gb_len;
  st->delta = 0.0f;
  st->ib = -1;
  st->src_gb = 0;
  st->improved = 0;
  st->iter = 0;
}

// ===================================================================== //
// Candidate + backup lists (Sec. 4.1): the K + BL nearest cities by
// (squared distance, id); eta = 1/d.  One query city per lane; candidate
// cities stream through LDS in tiles; each lane keeps its sorted list in LDS.
// ===================================================================== //
constexpr int kKnnTile = 256;

__global__ void __launch_bounds__(64) knn_kernel(const int2 *xy, int n, int K, int BL,
                                                 int32_t *cl, int32_t *bll, float *eta,
                                                 DevState *st) {
  extern __shared__ unsigned char knn_lds[];
  const int KK = K + BL;
  const int tid = threadIdx.x;
  int2 *tile = reinterpret_cast<int2 *>(knn_lds);
  double *kd = reinterpret_cast<double *>(knn_lds + sizeof(int2) * kKnnTile);
  int32_t *kj = reinterpret_cast<int32_t *>(knn_lds + sizeof(int2) * kKnnTile +
                                            sizeof(double) * (size_t)KK * 64);
  const int i = blockIdx.x * 64 + tid;
  const bool valid = i < n;
  const int2 xi = valid ? xy[i] : make_int2(0, 0);
  int cnt = 0;
  double worst = 0.0;
  for (int t0 = 0; t0 < n; t0 += kKnnTile) {
    __syncthreads();
    for (int j = tid; j < kKnnTile; j += 64)
      if (t0 + j < n) tile[j] = xy[t0 + j];
    __syncthreads();
    const int tn = min(kKnnTile, n - t0);
    if (!valid) continue;
    for (int jj = 0; jj < tn; ++jj) {
      const int j = t0 + jj;
      if (j == i) continue;
      const double d = sqd(xi, tile[jj]);
      if (cnt == KK && !(d < worst)) continue;
      int q = cnt < KK ? cnt++ : KK - 1;
      while (q > 0 && kd[(q - 1) * 64 + tid] > d) {
        kd[q * 64 + tid] = kd[(q - 1) * 64 + tid];
        kj[q * 64 + tid] = kj[(q - 1) * 64 + tid];
        --q;
      }
      kd[q * 64 + tid] = d;
      kj[q * 64 + tid] = j;
      if (cnt == KK) worst = kd[(KK - 1) * 64 + tid];
    }
  }
  if (!valid) return;
  for (int s = 0; s < K; ++s) {
    const double d2 = kd[s * 64 + tid];
    cl[(size_t)i * K + s] = kj[s * 64 + tid];
    const int d = (int)floor(sqrt(d2) + 0.5);
    eta[(size_t)i * K + s] = (float)(1.0 / (double)d);
  }
  for (int s = 0; s < BL; ++s) bll[(size_t)i * BL + s] = kj[(K + s) * 64 + tid];
  if (kd[tid] == 0.0) atomicOr(&st->dup, 1);
}

}  // namespace faco
