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

// q mod n; the common cases (q within one period of [0, n)) avoid a division
FACO_DEV int64_t ticks() { return (int64_t)wall_clock64(); }

FACO_DEV int wrapn(int q, int n) {
  if (q >= n) {
    q -= n;
    if (q >= n) q %= n;
  } else if (q < 0) {
    q += n;
    if (q < 0) {
      q %= n;
      q = q < 0 ? q + n : q;
    }
  }
  return q;
}
// for 0 <= q < 2n
FACO_DEV int wrap1(int q, int n) { return q >= n ? q - n : q; }

// Offset a source position by |off| <= 256 (cheap form when n > 256).
FACO_DEV int wrap_off(int q, int off, int n) {
  if (n > 256) {
    q += off;
    return q >= n ? q - n : (q < 0 ? q + n : q);
  }
  return wrapn(q + off, n);
}

// ===================================================================== //
// Backup list, then the nearest unvisited city (when no candidate of u is
// unvisited).  Uniform result.
// ===================================================================== //
FACO_DEV int select_fallback(const Inst &I, int u, const uint32_t *vis, int64_t *cnt) {
  const int lane = lane_id();
  int b = 0;
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
  // best heuristic value = nearest unvisited city, ties by smaller id.
  // Lane l scans bitmap words l, l + 64, ...; fully visited words are skipped.
  cnt[CNT_FALLBACK]++;
  const int2 xu = I.xy[u];
  const int W = (I.n + 31) >> 5;
  int64_t bd = INT64_MAX;
  int bj = 0x7fffffff;
  for (int w = lane; w < W; w += kWave) {
    uint32_t free_bits = ~vis[w];
    const int rem = I.n - w * 32;
    if (rem < 32) free_bits &= (1u << rem) - 1u;
    while (free_bits) {
      const int j = w * 32 + __builtin_ctz(free_bits);
      free_bits &= free_bits - 1;
      const int64_t d = (int64_t)sqd_u64(xu, I.xy[j]);
      if (d < bd) {
        bd = d;
        bj = j;
      }
    }
  }
  const int64_t md = wave_min_i64(bd);
  return wave_min_i32(bd == md ? bj : 0x7fffffff);
}

// Greedy step of the nearest-neighbour tour: first unvisited candidate
// (lists are sorted by distance), else the fallback chain.  dv = its cost.
FACO_DEV int select_greedy(const Inst &I, int u, const uint32_t *vis, int &dv,
                           int64_t *cnt) {
  const int K = I.k, lane = lane_id();
  const size_t row = (size_t)u * (size_t)K;
  const bool act = lane < K;
  const int cand = act ? I.cl[row + lane] : 0;
  const int cd = act ? I.cl_d[row + lane] : 0;
  const uint64_t um = ballot(act && !bit_get(vis, cand));
  if (um) {
    const int s = ctz64(um);
    dv = readlane_i(cd, s);
    return readlane_i(cand, s);
  }
  const int v = select_fallback(I, u, vis, cnt);
  dv = cost(I.xy[u], I.xy[v]);
  return v;
}

// ===================================================================== //
// Copy-from-source (Alg. 2, reading: forward from v while unvisited, else
// backward).  The first round probes 64 positions in both directions at
// once; later rounds take 256 positions.  Edge costs come from the
// per-iteration source edge table.  Returns the count; u/pu become the last
// appended city and its source position.
// ===================================================================== //
FACO_DEV int copy_from(const Inst &I, int pv, int &k, int &u, int &pu, int64_t &len,
                       int32_t *route, int32_t *pos, int2 *rxy, uint32_t *vis) {
  const int n = I.n, lane = lane_id();
  const int qf = wrap_off(pv, lane + 1, n), qb = wrap_off(pv, -lane - 1, n);
  const int cf = I.src_route[qf], cb = I.src_route[qb];
  const int df = I.src_d[qf == 0 ? n - 1 : qf - 1], db = I.src_d[qb];
  const uint64_t mf = ballot(bit_get(vis, cf));
  const int jf = mf ? ctz64(mf) : kWave;
  int dir, j, c, d;
  if (jf > 0) {
    dir = 1; j = jf; c = cf; d = df;
  } else {
    const uint64_t mb = ballot(bit_get(vis, cb));
    dir = -1; j = mb ? ctz64(mb) : kWave; c = cb; d = db;
  }
  if (j == 0) return 0;
  if (lane < j) {
    route[k + lane] = c;
    pos[c] = k + lane;
    rxy[k + lane] = I.xy[c];
    bit_set(vis, c);
  }
  len += wave_sum_i64(lane < j ? (int64_t)d : 0);
  u = readlane_i(c, j - 1);
  k += j;
  int app = j, pcur = wrap_off(pv, dir * j, n);
  if (j < kWave) {
    pu = pcur;
    return app;
  }
  for (;;) {
    int cc[4], dd[4];
    bool vc[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int q = wrap_off(pcur, dir * (h * kWave + lane + 1), n);
      cc[h] = I.src_route[q];
      dd[h] = I.src_d[dir > 0 ? (q == 0 ? n - 1 : q - 1) : q];
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) vc[h] = bit_get(vis, cc[h]);
    int jj = 4 * kWave;
#pragma unroll
    for (int h = 3; h >= 0; --h) {
      const uint64_t m = ballot(vc[h]);
      if (m) jj = h * kWave + ctz64(m);
    }
    int64_t dsum = 0;
    int last = 0;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int idx = h * kWave + lane;
      if (idx < jj) {
        route[k + idx] = cc[h];
        pos[cc[h]] = k + idx;
        rxy[k + idx] = I.xy[cc[h]];
        bit_set(vis, cc[h]);
        dsum += dd[h];
      }
      if (idx == jj - 1) last = cc[h];
    }
    len += wave_sum_i64(dsum);
    if (jj > 0) u = readlane_i(last, (jj - 1) & (kWave - 1));
    k += jj;
    app += jj;
    pcur = wrapn(pcur + dir * jj, n);
    if (jj < 4 * kWave) break;
  }
  pu = pcur;
  return app;
}

// ===================================================================== //
// Speculative source-following window.  Lane i evaluates ACO step `step + i`
// as if the ant had followed the source in direction dir for the previous i
// steps: its current city is q_i (q_0 = u at source position pu), its
// visited set V + {q_1..q_i} (V in LDS, the q's recognised by their source
// positions).  The first lane whose choice is not q_{i+1} ends the window;
// its choice is exact because every earlier lane confirmed the assumption.
// Same draws, same weights, same order as the one-step-at-a-time rule.
// Output: acc = steps that followed the source; then, unless the window ran
// out (v = -2), the decision of step `step + acc`: v with its cost dv and
// source position pv, or v = -1 when no candidate is unvisited.
// ===================================================================== //
struct Draws {
  uint64_t base;  // lane j holds the roulette draw of step base + j
  float u;
  bool valid;
};

template <int KT>
FACO_DEV int spec_block(const Inst &I, uint64_t t, uint64_t ant, uint64_t step,
                        int u, int pu, int dir, int k, int maxw, const uint32_t *vis,
                        Draws &D, int &v, int &dv, int &pv, int &lastq,
                        int64_t &src_len_sum) {
  const int n = I.n, K = I.k, lane = lane_id();
  // every load below is addressed by source position: one round trip
  const int rpos = wrap_off(pu, dir * lane, n);      // position of q_lane
  const int qpos = wrap_off(pu, dir * (lane + 1), n);
  const int qn = I.src_route[qpos];                   // q_{lane+1}
  const int ed = I.src_d[dir > 0 ? rpos : qpos];      // cost q_lane -> q_{lane+1}
  const size_t row = (size_t)rpos * (size_t)K;
  int c[KT], sp[KT], cd[KT];
  float wt[KT];
#pragma unroll
  for (int s = 0; s < KT; ++s) {
    if (s < K) {
      c[s] = I.scl[row + s];
      wt[s] = I.sw[row + s];
      sp[s] = I.ssp[row + s];
      cd[s] = I.sd[row + s];
    }
  }
  // draws: a one-step window reuses the 64 draws computed for earlier steps
  float U;
  if (maxw == 1 && D.valid && step >= D.base && step < D.base + kWave) {
    U = readlane_f(D.u, (int)(step - D.base));
  } else {
    D.u = unit24(philox_word0(I.seed, t, ant, step + (uint64_t)lane, kPurposeRoulette));
    D.base = step;
    D.valid = true;
    U = D.u;
  }
  float P[KT];
  float total = 0.0f;
  int last = -1;
#pragma unroll
  for (int s = 0; s < KT; ++s) {
    if (s < K) {
      const int off = dir > 0 ? sp[s] - pu : pu - sp[s];
      const int offw = off < 0 ? off + n : off;
      const bool visited = bit_get(vis, c[s]) || (offw >= 1 && offw <= lane);
      if (!visited) {
        total = total + wt[s];
        last = s;
      }
      P[s] = total;
    }
  }
  const bool special = last < 0;
  int choice = 0, choice_d = 0, choice_p = 0;
  if (!special) {
    const float r = U * total;
    int sel = -1;
#pragma unroll
    for (int s = KT - 1; s >= 0; --s)
      if (s < K && P[s] > r) sel = s;
    if (sel < 0) sel = last;
#pragma unroll
    for (int s = 0; s < KT; ++s)
      if (s == sel) {
        choice = c[s];
        choice_d = cd[s];
        choice_p = sp[s];
      }
  }
  int valid = n - k < kWave ? n - k : kWave;  // steps left
  valid = valid < maxw ? valid : maxw;
  const bool match = !special && choice == qn && lane < valid;
  const uint64_t mm = ballot(!match);
  const int f = mm ? ctz64(mm) : kWave;
  const int acc = f < valid ? f : valid;  // accepted source-following steps
  src_len_sum = wave_sum_i64(lane < acc ? (int64_t)ed : 0);
  lastq = acc > 0 ? readlane_i(qn, acc - 1) : u;
  if (acc < valid) {
    if (readlane_i(special ? 1 : 0, acc)) {
      v = -1;
    } else {
      v = readlane_i(choice, acc);
      dv = readlane_i(choice_d, acc);
      pv = readlane_i(choice_p, acc);
    }
  } else {
    v = -2;  // every step of the window followed the source
  }
  return acc;
}

// One ACO step from the city at source position pu, lane s = candidate slot
// s (used once new_edges >= m, when every step is followed by a copy).
// v = -1 when no candidate is unvisited.
FACO_DEV int one_step(const Inst &I, uint64_t t, uint64_t ant, uint64_t step, int pu,
                      const uint32_t *vis, Draws &D, int &dv, int &pv) {
  const int n = I.n, K = I.k, lane = lane_id();
  (void)n;
  const bool act = lane < K;
  const size_t row = (size_t)pu * (size_t)K;
  const int c = act ? I.scl[row + lane] : 0;
  const float w = act ? I.sw[row + lane] : 0.0f;
  const int sp = act ? I.ssp[row + lane] : 0;
  const int d = act ? I.sd[row + lane] : 0;
  const bool unv = act && !bit_get(vis, c);
  const uint64_t um = ballot(unv);
  if (!um) return -1;
  if (!(D.valid && step >= D.base && step < D.base + kWave)) {
    D.u = unit24(philox_word0(I.seed, t, ant, step + (uint64_t)lane, kPurposeRoulette));
    D.base = step;
    D.valid = true;
  }
  const float U = readlane_f(D.u, (int)(step - D.base));
  const float wv = unv ? w : 0.0f;
  // cumulative sum in slot order: lane s holds fl(...fl(w_0 + w_1)... + w_s)
  float P = 0.0f;
  for (int j = 0; j < K; ++j) {
    const float wj = readlane_f(wv, j);
    if (j <= lane) P = P + wj;
  }
  const float r = U * readlane_f(P, K - 1);
  const uint64_t sm = ballot(act && P > r);
  const int s = sm ? ctz64(sm) : msb64(um);
  dv = readlane_i(d, s);
  pv = readlane_i(sp, s);
  return readlane_i(c, s);
}

// ===================================================================== //
// Focused construction (Alg. 2 inner loop).  greedy: nearest-neighbour tour
// from city 0 (initial solution), no source, no copy.
// The checklist is written into ring[0..nchk) with its LDS bits set in inq.
// ===================================================================== //
FACO_DEV void append_city(const Inst &I, int v, int k, int32_t *route, int32_t *pos,
                          int2 *rxy, uint32_t *vis) {
  if (lane_id() == 0) {
    route[k] = v;
    pos[v] = k;
    rxy[k] = I.xy[v];
    bit_set(vis, v);
  }
}

// tk: [5] speculative windows, [6] one-step calls, [7] copies, [8..10] their
// ticks, [11] ticks in backup/nearest-city choices
template <int KT>
FACO_DEV int64_t construct(const Inst &I, uint64_t t, int ant, bool greedy,
                           int32_t *route, int32_t *pos, int2 *rxy, int32_t *ring,
                           uint32_t *vis, uint32_t *inq, int W, int &nchk,
                           int64_t *cnt, int64_t *tk) {
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
  append_city(I, u, 0, route, pos, rxy, vis);
  int k = 1, new_edges = 0;
  nchk = 0;
  int64_t len = 0;
  uint64_t step = 0;
  if (greedy) {
    while (k < n) {
      int dv;
      const int v = select_greedy(I, u, vis, dv, cnt);
      ++step;
      len += dv;
      append_city(I, v, k, route, pos, rxy, vis);
      ++k;
      u = v;
    }
  } else {
    int pu = I.src_pos[u];
    int dir = 1;
    Draws D;
    D.base = 0;
    D.u = 0.0f;
    D.valid = false;
    while (k < n) {
      // Once new_edges >= m every ACO step is followed by a copy, so the
      // window is one step wide.
      const int maxw = new_edges >= I.m ? 1 : kWave;
      int v, dv = 0, pv = 0, lastq = u;
      int64_t srcsum = 0;
      int acc = 0;
      const int64_t c0 = ticks();
      if (maxw == 1) {
        v = one_step(I, t, (uint64_t)ant, step, pu, vis, D, dv, pv);
        tk[6]++;
        tk[9] += ticks() - c0;
      } else {
        acc = spec_block<KT>(I, t, (uint64_t)ant, step, u, pu, dir, k, maxw, vis, D, v, dv,
                             pv, lastq, srcsum);
        tk[5]++;
        tk[8] += ticks() - c0;
      }
      if (acc > 0) {
        // accepted steps follow the source: q_1..q_acc at k..k+acc-1
        if (lane < acc) {
          const int q = I.src_route[wrap_off(pu, dir * (lane + 1), n)];
          route[k + lane] = q;
          pos[q] = k + lane;
          rxy[k + lane] = I.xy[q];
          bit_set(vis, q);
        }
        k += acc;
        step += acc;
        len += srcsum;
        pu = wrap_off(pu, dir * acc, n);
        u = lastq;
      }
      if (v == -2) {
        // the whole window followed the source; no step off the path
        v = u;
        pv = pu;
      } else {
        if (v == -1) {
          const int64_t c1 = ticks();
          v = select_fallback(I, u, vis, cnt);
          dv = cost(I.xy[u], I.xy[v]);
          pv = I.src_pos[v];
          tk[11] += ticks() - c1;
        }
        ++step;
        len += dv;
        append_city(I, v, k, route, pos, rxy, vis);
        ++k;
        const int fwd = pu + 1 == n ? 0 : pu + 1, bwd = pu == 0 ? n - 1 : pu - 1;
        if (pv != fwd && pv != bwd) {
          ++new_edges;
          if (lane == 0) {
            ring[nchk] = v;
            bit_set(inq, v);
          }
          ++nchk;
        }
        dir = pv == bwd ? -1 : 1;
      }
      u = v;
      pu = pv;
      if (new_edges >= I.m && k < n) {
        const int64_t c2 = ticks();
        const int app = copy_from(I, pv, k, u, pu, len, route, pos, rxy, vis);
        cnt[CNT_COPIED] += app;
        tk[7]++;
        tk[10] += ticks() - c2;
      }
    }
  }
  len += cost(I.xy[u], I.xy[r0]);
  cnt[CNT_ACO_STEPS] += (int64_t)step;
  cnt[CNT_NEW_EDGES] += new_edges;
  wave_fence();
  return len;
}

// ===================================================================== //
// Local search (Alg. 3 + Or-opt + sweep)
// ===================================================================== //
struct Move {
  int kind;  // 0 none, 1 2-opt, 2 Or-opt
  int gain;
  int w, x, y, z;     // 2-opt: remove (w,x), (y,z)
  int px, py, pz;     // positions of x, y, z
  int f, l, p, q, a, o, b, e, L;  // Or-opt
  int fpos, pq, pp, pb, side;     // positions of f, q, p, b; e = succ(b) if side 0
  int s0, s1, s2;     // segment in array order
  int2 xs0, xs1, xs2; // and its coordinates
};

// Or-opt variants in evaluation order, one fixed slot each:
// slot 0..2 = forward L = 1..3, slot 3..4 = backward L = 2..3.
// For slot (dir, L) and nb[j] = route[pa + j - 3]: lanes of f, l, p, q.
constexpr int kOrSlots = 5;
FACO_DEV void or_slot_lanes(int slot, int &dir, int &L, int &lf, int &ll, int &lp, int &lq) {
  dir = slot < 3 ? 0 : 1;
  L = slot < 3 ? slot + 1 : slot - 1;
  if (dir == 0) {
    lf = 3; ll = 3 + L - 1; lp = 2; lq = 3 + L;
  } else {
    lf = 3 - L + 1; ll = 3; lp = 3 - L; lq = 4;
  }
}
FACO_DEV int or_lmax(const Inst &I) {
  return I.oropt_max < I.n - 3 ? I.oropt_max : I.n - 3;
}

FACO_DEV int2 shfl_i2(int2 v, int l) { return make_int2(__shfl(v.x, l), __shfl(v.y, l)); }

template <int GS>
FACO_DEV int64_t group_max(int64_t v) {
#pragma unroll
  for (int m = GS / 2; m >= 1; m >>= 1) {
    const int64_t o = shfl_xor_i64(v, m);
    v = o > v ? o : v;
  }
  return v;
}

// Per-lane state of a grouped evaluation: GS lanes evaluate one city a
// (slot s = lane % GS handles candidate s), 64 / GS cities per wave.
struct GroupEval {
  int a, pa, b, pb, pbs, pbp, bs, bp, nb, d_ab;
  int2 xa, xnb, xb, xbs, xbp;
  int64_t key2, keyo;  // group maxima: 2-opt, Or-opt (0 = none)
};

// All loads for both move kinds of every city of the wave are issued
// together (4 dependent levels).  Keys order candidates as the sequential
// evaluation does: 2-opt loop 1 over the list, loop 2 over the list; Or-opt
// variants, list slots, succ before pred.
template <int GS>
FACO_DEV GroupEval eval_group(const Inst &I, uint32_t flags, int a, bool gvalid,
                              const int32_t *route, const int32_t *pos, const int2 *rxy) {
  const int n = I.n, K = I.k, lane = lane_id();
  const int gb = lane & ~(GS - 1);
  const int s = lane & (GS - 1);
  const bool act = gvalid && s < K;
  const size_t row = (size_t)a * (size_t)K;
  GroupEval R;
  R.a = a;
  // level 1: indexed by a
  const int pa = pos[a];
  const int b = act ? I.cl[row + s] : a;
  const int d_ab = act ? I.cl_d[row + s] : 0;
  const int2 xa = I.xy[a];
  // level 2
  const int pn = wrapn(pa + s - 3, n);
  const int nb = s < 7 ? route[pn] : a;
  const int2 xnb = s < 7 ? rxy[pn] : xa;
  const int pb = pos[b];
  const int2 xb = I.xy[b];
  // level 3
  const int pbs = pb + 1 == n ? 0 : pb + 1, pbp = pb == 0 ? n - 1 : pb - 1;
  const int bs = route[pbs], bp = route[pbp];
  const int2 xbs = rxy[pbs], xbp = rxy[pbp];
  R.pa = pa; R.b = b; R.pb = pb; R.pbs = pbs; R.pbp = pbp; R.bs = bs; R.bp = bp;
  R.nb = nb; R.xa = xa; R.xnb = xnb; R.xb = xb; R.xbs = xbs; R.xbp = xbp; R.d_ab = d_ab;
  const int2 xas = shfl_i2(xnb, gb + 4), xap = shfl_i2(xnb, gb + 2);
  R.key2 = 0;
  if (flags & LS_2OPT) {
    const int d_as = cost(xa, xas), d_ap = cost(xap, xa);
    int g1 = 0, g2 = 0;
    if (act && d_as > d_ab) g1 = d_as + cost(xb, xbs) - d_ab - cost(xas, xbs);
    if (act && d_ap > d_ab) g2 = d_ap + cost(xbp, xb) - d_ab - cost(xap, xbp);
    const int64_t k1 = g1 > 0 ? (((int64_t)g1 << 8) | (int64_t)(255 - s)) : 0;
    const int64_t k2 = g2 > 0 ? (((int64_t)g2 << 8) | (int64_t)(255 - 32 - s)) : 0;
    R.key2 = group_max<GS>(k1 > k2 ? k1 : k2);
  }
  R.keyo = 0;
  return R;
}

// Or-opt keys for the cities of the groups with `want` set (the others get 0).
template <int GS>
FACO_DEV void eval_group_oropt(const Inst &I, bool want, GroupEval &R) {
  const int n = I.n, K = I.k, lane = lane_id();
  const int gb = lane & ~(GS - 1);
  const int s = lane & (GS - 1);
  const bool act = want && s < K;
  const int pa = R.pa, pb = R.pb, pbs = R.pbs, pbp = R.pbp, d_ab = R.d_ab;
  const int2 xa = R.xa, xnb = R.xnb, xb = R.xb, xbs = R.xbs, xbp = R.xbp;
  const int Lmax = or_lmax(I);
  int lbest = 0, lidx = 0;
  const int d_bs = cost(xb, xbs), d_bp = cost(xb, xbp);
#pragma unroll
  for (int vi = 0; vi < kOrSlots; ++vi) {
    int dir, L, lf, ll, lp, lq;
    or_slot_lanes(vi, dir, L, lf, ll, lp, lq);
    if (L > Lmax) continue;
    const int2 xf = shfl_i2(xnb, gb + lf), xl = shfl_i2(xnb, gb + ll);
    const int2 xp = shfl_i2(xnb, gb + lp), xq = shfl_i2(xnb, gb + lq);
    const int2 xo = dir == 0 ? xl : xf;
    const int fpos = dir == 0 ? pa : wrapn(pa - L + 1, n);
    const int rem_a = dir == 0 ? cost(xp, xa) : cost(xa, xq);
    if (!act) continue;
    if (!(d_ab < rem_a)) continue;
    if (wrapn(pb - fpos, n) < L) continue;
    const int g_rem = cost(xp, xf) + cost(xl, xq) - cost(xp, xq);
    if (wrapn(pbs - fpos, n) >= L) {
      const int g = g_rem + d_bs - d_ab - cost(xo, xbs);
      if (g > lbest) {
        lbest = g;
        lidx = (vi * K + s) * 2 + 0;
      }
    }
    if (wrapn(pbp - fpos, n) >= L) {
      const int g = g_rem + d_bp - d_ab - cost(xo, xbp);
      if (g > lbest) {
        lbest = g;
        lidx = (vi * K + s) * 2 + 1;
      }
    }
  }
  const int64_t key = lbest > 0 ? (((int64_t)lbest << 16) | (int64_t)(0xFFFF - lidx)) : 0;
  R.keyo = group_max<GS>(key);
}

// The move found for the city of group j (uniform j), from the group's lanes.
template <int GS>
FACO_DEV Move extract_move(const Inst &I, const GroupEval &R, int j) {
  const int n = I.n, K = I.k, base = j * GS;
  Move mv = {};
  const int64_t key2 = readlane_i64(R.key2, base);
  const int a = readlane_i(R.a, base);
  const int pa = readlane_i(R.pa, base);
  if (key2 > 0) {
    const int idx = 255 - (int)(key2 & 255);
    mv.kind = 1;
    mv.gain = (int)(key2 >> 8);
    if (idx < 32) {  // loop 1: (a, succ a, b, succ b), flip succ a .. b
      const int l = base + idx;
      mv.w = a; mv.x = readlane_i(R.nb, base + 4);
      mv.y = readlane_i(R.b, l); mv.z = readlane_i(R.bs, l);
      mv.px = pa + 1 == n ? 0 : pa + 1;
      mv.py = readlane_i(R.pb, l);
      mv.pz = readlane_i(R.pbs, l);
    } else {         // loop 2: (pred a, a, pred b, b), flip a .. pred b
      const int l = base + idx - 32;
      mv.w = readlane_i(R.nb, base + 2); mv.x = a;
      mv.y = readlane_i(R.bp, l); mv.z = readlane_i(R.b, l);
      mv.px = pa;
      mv.py = readlane_i(R.pbp, l);
      mv.pz = readlane_i(R.pb, l);
    }
    return mv;
  }
  const int64_t keyo = readlane_i64(R.keyo, base);
  if (keyo <= 0) return mv;
  const int idx = 0xFFFF - (int)(keyo & 0xFFFF);
  const int side = idx & 1;
  const int s = (idx >> 1) % K;
  const int vi = (idx >> 1) / K;
  int dir, L, lf, ll, lp, lq;
  or_slot_lanes(vi, dir, L, lf, ll, lp, lq);
  const int l = base + s;
  mv.kind = 2;
  mv.gain = (int)(keyo >> 16);
  mv.L = L;
  mv.a = a;
  mv.f = readlane_i(R.nb, base + lf);
  mv.l = readlane_i(R.nb, base + ll);
  mv.p = readlane_i(R.nb, base + lp);
  mv.q = readlane_i(R.nb, base + lq);
  mv.o = dir == 0 ? mv.l : mv.f;
  mv.b = readlane_i(R.b, l);
  mv.e = side ? readlane_i(R.bp, l) : readlane_i(R.bs, l);
  mv.side = side;
  mv.pb = readlane_i(R.pb, l);
  mv.fpos = dir == 0 ? pa : wrapn(pa - L + 1, n);
  mv.pq = wrapn(mv.fpos + L, n);
  mv.pp = mv.fpos == 0 ? n - 1 : mv.fpos - 1;
  mv.s0 = readlane_i(R.nb, base + lf);
  mv.s1 = readlane_i(R.nb, base + lf + (L > 1 ? 1 : 0));
  mv.s2 = readlane_i(R.nb, base + lf + (L > 2 ? 2 : 0));
  mv.xs0 = readlane_i2(R.xnb, base + lf);
  mv.xs1 = readlane_i2(R.xnb, base + lf + (L > 1 ? 1 : 0));
  mv.xs2 = readlane_i2(R.xnb, base + lf + (L > 2 ? 2 : 0));
  return mv;
}

// Lane-serial test used by the sweep (one city per lane): does x have an
// improving move?  Loads are issued before gains are formed; candidate lists
// are sorted by distance, so a slot that fails the pruning test ends the scan.
template <int KT>
FACO_DEV bool has_improving(const Inst &I, uint32_t flags, int x,
                            const int32_t *route, const int32_t *pos, const int2 *rxy) {
  const int n = I.n, K = I.k;
  const size_t row = (size_t)x * (size_t)K;
  const int px = pos[x];
  int b[KT], dxb[KT];
#pragma unroll
  for (int s = 0; s < KT; ++s) {
    b[s] = s < K ? I.cl[row + s] : x;
    dxb[s] = s < K ? I.cl_d[row + s] : 0;
  }
  const int2 cx = I.xy[x];
  int xnx[7], xny[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int2 q = rxy[wrapn(px + j - 3, n)];
    xnx[j] = q.x; xny[j] = q.y;
  }
  int pb[KT], xbx[KT], xby[KT];
#pragma unroll
  for (int s = 0; s < KT; ++s) {
    pb[s] = pos[b[s]];
    const int2 q = I.xy[b[s]];
    xbx[s] = q.x; xby[s] = q.y;
  }
  int xbsx[KT], xbsy[KT], xbpx[KT], xbpy[KT];
#pragma unroll
  for (int s = 0; s < KT; ++s) {
    const int2 q1 = rxy[pb[s] + 1 == n ? 0 : pb[s] + 1];
    const int2 q2 = rxy[pb[s] == 0 ? n - 1 : pb[s] - 1];
    xbsx[s] = q1.x; xbsy[s] = q1.y;
    xbpx[s] = q2.x; xbpy[s] = q2.y;
  }
#define XN(j) make_int2(xnx[j], xny[j])
#define XB(s) make_int2(xbx[s], xby[s])
#define XBS(s) make_int2(xbsx[s], xbsy[s])
#define XBP(s) make_int2(xbpx[s], xbpy[s])
  if (flags & LS_2OPT) {
    const int d_s = cost(cx, XN(4)), d_p = cost(XN(2), cx);
#pragma unroll
    for (int s = 0; s < KT; ++s) {
      if (s >= K) break;
      const int d_xb = dxb[s];
      if (d_s <= d_xb && d_p <= d_xb) break;
      if (d_s > d_xb && d_s + cost(XB(s), XBS(s)) - d_xb - cost(XN(4), XBS(s)) > 0) return true;
      if (d_p > d_xb && d_p + cost(XBP(s), XB(s)) - d_xb - cost(XN(2), XBP(s)) > 0) return true;
    }
  }
  if (flags & LS_OROPT) {
    const int Lmax = or_lmax(I);
#pragma unroll
    for (int vi = 0; vi < kOrSlots; ++vi) {
      int dir, L, lf, ll, lp, lq;
      or_slot_lanes(vi, dir, L, lf, ll, lp, lq);
      if (L > Lmax) continue;
      const int fpos = dir == 0 ? px : wrapn(px - L + 1, n);
      const int2 xo = dir == 0 ? XN(ll) : XN(lf);
      const int rem = dir == 0 ? cost(XN(lp), cx) : cost(cx, XN(lq));
      if (!(dxb[0] < rem)) continue;
      const int g_rem = cost(XN(lp), XN(lf)) + cost(XN(ll), XN(lq)) - cost(XN(lp), XN(lq));
#pragma unroll
      for (int s = 0; s < KT; ++s) {
        if (s >= K) break;
        const int d_xb = dxb[s];
        if (!(d_xb < rem)) break;
        if (wrapn(pb[s] - fpos, n) < L) continue;
        const int pbs = pb[s] + 1 == n ? 0 : pb[s] + 1, pbp = pb[s] == 0 ? n - 1 : pb[s] - 1;
        if (wrapn(pbs - fpos, n) >= L &&
            g_rem + cost(XB(s), XBS(s)) - d_xb - cost(xo, XBS(s)) > 0)
          return true;
        if (wrapn(pbp - fpos, n) >= L &&
            g_rem + cost(XB(s), XBP(s)) - d_xb - cost(xo, XBP(s)) > 0)
          return true;
      }
    }
  }
#undef XN
#undef XB
#undef XBS
#undef XBP
  return false;
}

constexpr int kChunks = 16;  // 64-element chunks in flight per round

// Reverse the cyclic array range of length L starting at s (wave-wide).
FACO_DEV void reverse_range(int n, int s, int L, int32_t *route, int32_t *pos, int2 *rxy) {
  const int lane = lane_id();
  const int half = L >> 1;
  for (int base = 0; base < half; base += kChunks * kWave) {
    int p1[kChunks], p2[kChunks], v1[kChunks], v2[kChunks];
    int c1x[kChunks], c1y[kChunks], c2x[kChunks], c2y[kChunks];
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const int i = base + c * kWave + lane;
      if (i < half) {
        p1[c] = wrap1(s + i, n);
        p2[c] = wrap1(s + L - 1 - i, n);
        v1[c] = route[p1[c]];
        v2[c] = route[p2[c]];
        const int2 a1 = rxy[p1[c]], a2 = rxy[p2[c]];
        c1x[c] = a1.x; c1y[c] = a1.y;
        c2x[c] = a2.x; c2y[c] = a2.y;
      }
    }
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const int i = base + c * kWave + lane;
      if (i < half) {
        route[p1[c]] = v2[c];
        route[p2[c]] = v1[c];
        rxy[p1[c]] = make_int2(c2x[c], c2y[c]);
        rxy[p2[c]] = make_int2(c1x[c], c1y[c]);
        pos[v2[c]] = p1[c];
        pos[v1[c]] = p2[c];
      }
    }
  }
}

// "Flip a section between x and y": the shorter of the paths x..y and z..w.
// px, py, pz: array positions of x, y, z.
FACO_DEV int apply_2opt(int n, int px, int py, int pz, int32_t *route,
                        int32_t *pos, int2 *rxy) {
  const int L1 = wrapn(py - px, n) + 1;
  int moved;
  if (2 * L1 <= n) {
    reverse_range(n, px, L1, route, pos, rxy);
    moved = L1;
  } else {
    reverse_range(n, pz, n - L1, route, pos, rxy);
    moved = n - L1;
  }
  wave_fence();
  return moved;
}

// Or-opt: the segment and the shorter block between its old place and the
// insertion edge exchange places (block keeps its orientation).
FACO_DEV int apply_oropt(int n, int L, int a, int f, int b, int e, int side,
                         int pb, int fpos, int pq, int pp, int s0, int s1, int s2,
                         int2 xs0, int2 xs1, int2 xs2, int32_t *route, int32_t *pos,
                         int2 *rxy) {
  const int lane = lane_id();
  int x1, px1, px2;
  if (side == 0) {  // e = succ(b): edge (b, e)
    x1 = b;
    px1 = pb;
    px2 = pb + 1 == n ? 0 : pb + 1;
  } else {          // e = pred(b): edge (e, b)
    x1 = e;
    px1 = pb == 0 ? n - 1 : pb - 1;
    px2 = pb;
  }
  // segment in array order, then in the inserted orientation
  int segv = s0;
  segv = lane == 1 ? s1 : segv;
  segv = lane == 2 ? s2 : segv;
  int2 segx = xs0;
  segx = lane == 1 ? xs1 : segx;
  segx = lane == 2 ? xs2 : segx;
  const bool rev = (a != f) != (x1 != b);
  int src_lane = rev ? (L - 1 - lane) : lane;
  src_lane = src_lane < 0 ? 0 : (src_lane > 2 ? 2 : src_lane);
  const int ins = __shfl(segv, src_lane);
  const int2 insx = shfl_i2(segx, src_lane);
  const int D1 = wrapn(px1 - pq, n) + 1;
  const int D2 = wrapn(pp - px2, n) + 1;
  int moved;
  if (D1 <= D2) {
    // block q..x1 moves back by L to start at fpos; segment follows it
    for (int base = 0; base < D1; base += kChunks * kWave) {
      int v[kChunks], cvx[kChunks], cvy[kChunks];
#pragma unroll
      for (int c = 0; c < kChunks; ++c) {
        const int i = base + c * kWave + lane;
        if (i < D1) {
          const int sp = wrap1(pq + i, n);
          v[c] = route[sp];
          const int2 q = rxy[sp];
          cvx[c] = q.x; cvy[c] = q.y;
        }
      }
#pragma unroll
      for (int c = 0; c < kChunks; ++c) {
        const int i = base + c * kWave + lane;
        if (i < D1) {
          const int d = wrap1(fpos + i, n);
          route[d] = v[c];
          rxy[d] = make_int2(cvx[c], cvy[c]);
          pos[v[c]] = d;
        }
      }
    }
    if (lane < L) {
      const int d = wrapn(fpos + D1 + lane, n);
      route[d] = ins;
      rxy[d] = insx;
      pos[ins] = d;
    }
    moved = D1 + L;
  } else {
    // block x2..p moves forward by L; segment goes in front of it
    const int top = ((D2 - 1) / (kChunks * kWave)) * (kChunks * kWave);
    for (int base = top; base >= 0; base -= kChunks * kWave) {
      int v[kChunks], cvx[kChunks], cvy[kChunks];
#pragma unroll
      for (int c = 0; c < kChunks; ++c) {
        const int i = base + c * kWave + lane;
        if (i < D2) {
          const int sp = wrap1(px2 + i, n);
          v[c] = route[sp];
          const int2 q = rxy[sp];
          cvx[c] = q.x; cvy[c] = q.y;
        }
      }
#pragma unroll
      for (int c = 0; c < kChunks; ++c) {
        const int i = base + c * kWave + lane;
        if (i < D2) {
          const int d = wrapn(px2 + L + i, n);
          route[d] = v[c];
          rxy[d] = make_int2(cvx[c], cvy[c]);
          pos[v[c]] = d;
        }
      }
    }
    if (lane < L) {
      const int d = wrap1(px2 + lane, n);
      route[d] = ins;
      rxy[d] = insx;
      pos[ins] = d;
    }
    moved = D2 + L;
  }
  wave_fence();
  return moved;
}

struct Queue {
  int head, tail, count;
};

// The ring is written and read by lane 0 only (program order makes its own
// stores visible to it); the LDS bits are read by every lane, and LDS
// operations of one wave complete in order.
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
  }
}

// Sweep: test every touched city (ascending id) and list the improvable ones.
template <int KT>
FACO_DEV int sweep(const Inst &I, uint32_t flags, int W, Queue &Q,
                   const int32_t *route, const int32_t *pos, const int2 *rxy, int32_t *ring,
                   uint32_t *inq, uint32_t *touched) {
  const int lane = lane_id();
  int pushed = 0;
  int bx = -1, bcount = 0;
  auto flush = [&](int cnt) {
    bool f = false;
    if (lane < cnt) f = has_improving<KT>(I, flags, bx, route, pos, rxy);
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


template <int KT>
FACO_DEV int64_t local_search(const Inst &I, uint32_t flags, int32_t *route,
                              int32_t *pos, int2 *rxy, int32_t *ring, uint32_t *inq,
                              uint32_t *touched, int W, Queue Q, int64_t *cnt,
                              int64_t *tk) {
  constexpr int GS = KT <= 16 ? 16 : 32;  // lanes per evaluated city
  constexpr int G = kWave / GS;           // cities evaluated together
  const int n = I.n, lane = lane_id();
  const int grp = lane / GS;
  int64_t changes = 0, gain = 0, changes_at_sweep = -1;
  for (;;) {
    while (Q.count > 0 && changes < n) {
      // Evaluate the next G listed cities on the current tour.  The first one
      // with a move is applied; the ones before it are popped with no move;
      // the ones after it stay listed (their evaluation is discarded).
      const int gcount = Q.count < G ? Q.count : G;
      int e[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        int h = Q.head + g;
        h = h >= n ? h - n : h;
        e[g] = readlane_i(lane == 0 && g < gcount ? ring[h] : 0, 0);
      }
      int a = e[0];
#pragma unroll
      for (int g = 1; g < G; ++g) a = grp == g ? e[g] : a;
      const int64_t t0 = ticks();
      GroupEval R = eval_group<GS>(I, flags, a, grp < gcount, route, pos, rxy);
      // Or-opt is only tried where no 2-opt move exists, and only cities
      // before the first one with a 2-opt move can be the chosen one
      const uint64_t h2 = ballot((lane & (GS - 1)) == 0 && grp < gcount && R.key2 > 0);
      const int j2 = h2 ? ctz64(h2) / GS : gcount;
      if ((flags & LS_OROPT) && j2 > 0) eval_group_oropt<GS>(I, grp < j2, R);
      const int64_t t1 = ticks();
      tk[1] += t1 - t0;
      tk[12]++;
      const uint64_t hm = ballot((lane & (GS - 1)) == 0 && grp < gcount &&
                                 (R.key2 > 0 || R.keyo > 0));
      const int j = hm ? ctz64(hm) / GS : gcount;
      const int npop = j < gcount ? j + 1 : gcount;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g < npop) {
          if (lane == 0) bit_clear(inq, e[g]);
          Q.head = Q.head + 1 == n ? 0 : Q.head + 1;
          Q.count--;
          cnt[CNT_LS_POPS]++;
        }
      }
      if (j >= gcount) continue;
      const Move mv = extract_move<GS>(I, R, j);
      if (mv.kind == 1) {
        cnt[CNT_MOVED_ELEMS] += apply_2opt(n, mv.px, mv.py, mv.pz, route, pos, rxy);
        push(n, mv.w, Q, ring, inq, touched);
        push(n, mv.x, Q, ring, inq, touched);
        push(n, mv.y, Q, ring, inq, touched);
        push(n, mv.z, Q, ring, inq, touched);
        cnt[CNT_MOVES_2OPT]++;
      } else {
        cnt[CNT_MOVED_ELEMS] +=
            apply_oropt(n, mv.L, mv.a, mv.f, mv.b, mv.e, mv.side, mv.pb, mv.fpos, mv.pq,
                        mv.pp, mv.s0, mv.s1, mv.s2, mv.xs0, mv.xs1, mv.xs2, route, pos, rxy);
        push(n, mv.p, Q, ring, inq, touched);
        push(n, mv.q, Q, ring, inq, touched);
        push(n, mv.b, Q, ring, inq, touched);
        push(n, mv.e, Q, ring, inq, touched);
        push(n, mv.f, Q, ring, inq, touched);
        push(n, mv.l, Q, ring, inq, touched);
        cnt[CNT_MOVES_OROPT]++;
      }
      tk[2] += ticks() - t1;
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
    const int64_t t2 = ticks();
    const int pushed = sweep<KT>(I, flags, W, Q, route, pos, rxy, ring, inq, touched);
    tk[3] += ticks() - t2;
    if (pushed == 0) break;
  }
  cnt[CNT_LS_GAIN] += gain;
  return gain;
}

// ===================================================================== //
// One ant: construction + local search.  mode 0: ant `ant` of iteration
// st->iter + 1.  mode 1: initial solution (nearest neighbour + LS over all
// cities) written to the global best.
// ===================================================================== //
template <int KT>
FACO_DEV void run_ant(const Inst &I, int ant, int mode, uint32_t *lds) {
  const int n = I.n, lane = lane_id();
  const int W = (n + 31) >> 5;
  uint32_t *vis = lds;
  uint32_t *inq = lds + W;
  int32_t *route = I.routes + (size_t)ant * (size_t)n;
  int32_t *pos = I.pos + (size_t)ant * (size_t)n;
  int32_t *ring = I.ring + (size_t)ant * (size_t)n;
  int2 *rxy = I.rxy + (size_t)ant * (size_t)n;
  int64_t cnt[NCNT];
#pragma unroll
  for (int c = 0; c < NCNT; ++c) cnt[c] = 0;
  int64_t tk[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) tk[c] = 0;
  const bool init = mode == 1;
  const uint64_t t = (uint64_t)I.st->iter + 1;
  int nchk = 0;
  const int64_t t0 = ticks();
  int64_t len = construct<KT>(I, t, ant, init, route, pos, rxy, ring, vis, inq, W, nchk, cnt, tk);
  tk[0] = ticks() - t0;
  uint32_t flags = I.ls_flags;
  Queue Q;
  if (init) {
    // the initial solution reports only its local-search counters
#pragma unroll
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
    len -= local_search<KT>(I, flags, route, pos, rxy, ring, inq, vis, W, Q, cnt, tk);
  if (init) {
    for (int i = lane; i < n; i += kWave) I.gb_route[i] = route[i];
    if (lane == 0) {
      I.st->gb_len = len;
      I.st->init_len = len;
#pragma unroll
      for (int c = 0; c < NCNT; ++c) I.st->init_cnt[c] = cnt[c];
    }
  } else if (lane == 0) {
    I.lens[ant] = len;
#pragma unroll
    for (int c = 0; c < NCNT; ++c) {
      I.cnt[(size_t)ant * NCNT + c] = cnt[c];
      I.cnt_acc[(size_t)ant * NCNT + c] += cnt[c];
    }
    int64_t *tr = I.ticks + (size_t)ant * 16;
    tk[4] = ticks() - t0;
#pragma unroll
    for (int c = 0; c < 16; ++c) tr[c] += tk[c];
  }
}

template <int KT>
__global__ void __launch_bounds__(64) ant_kernel(Inst I, int mode) {
  extern __shared__ uint32_t lds[];
  run_ant<KT>(I, (int)blockIdx.x, mode, lds);
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
  const int i1 = i + 1 == n ? 0 : i + 1, i0 = i == 0 ? n - 1 : i - 1;
  const int32_t *from;
  if (init) {
    from = I.gb_route;
  } else {
    const int32_t *ibr = I.routes + (size_t)st->ib * (size_t)n;
    from = (st->src_gb && !st->improved) ? I.gb_route : ibr;
  }
  const int node = from[i], next = from[i1], prev = from[i0];
  if (!init && st->improved) I.gb_route[i] = node;
  I.src_route[i] = node;
  I.src_pos[node] = i;
  I.src_adj[node] = make_int2(next, prev);
  I.src_d[i] = cost(I.xy[node], I.xy[next]);
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
  const size_t o = (size_t)I.src_pos[i] * (size_t)K + s;
  I.scl[o] = j;
  I.sw[o] = tnew * I.eta[idx];
  I.ssp[o] = I.src_pos[j];
  I.sd[o] = I.cl_d[idx];
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
// Batched execution: one launch per phase covers every ant of every instance
// of a batch.  Each instance reads only its own Inst, so it evolves exactly as
// it would alone.
//   insts  Inst [count]
//   amap   int2 [total ants]: (instance, ant) of wave w = block * apb + wave
// ===================================================================== //
template <int KT>
__global__ void __launch_bounds__(256) ant_batch_kernel(const Inst *insts, const int2 *amap,
                                                       int total, int apb, int lds_words) {
  extern __shared__ uint32_t lds[];
  const int wave = (int)(threadIdx.x / kWave);
  const int w = (int)blockIdx.x * apb + wave;
  if (w >= total) return;
  const int2 m = amap[w];
  run_ant<KT>(insts[m.x], m.y, 0, lds + (size_t)wave * (size_t)lds_words);
}

__global__ void __launch_bounds__(64) colony_batch_kernel(const Inst *insts) {
  run_colony(insts[blockIdx.x]);
}

// blockIdx.y = instance; blocks past an instance's size return
__global__ void __launch_bounds__(256) source_batch_kernel(const Inst *insts) {
  run_source(insts[blockIdx.y], (int)(blockIdx.x * blockDim.x + threadIdx.x), 0);
}

__global__ void __launch_bounds__(256) pheromone_batch_kernel(const Inst *insts) {
  run_pheromone(insts[blockIdx.y], (size_t)blockIdx.x * blockDim.x + threadIdx.x, 0);
}

// ===================================================================== //
// Candidate + backup lists (Sec. 4.1): the K + BL nearest cities by
// (squared distance, id); eta = 1/d.  One query city per lane; candidate
// cities stream through LDS in tiles; each lane keeps its sorted list in LDS.
// ===================================================================== //
constexpr int kKnnTile = 256;

__global__ void __launch_bounds__(64) knn_kernel(const int2 *xy, int n, int K, int BL,
                                                 int32_t *cl, int32_t *bll, float *eta,
                                                 int32_t *cl_d, DevState *st) {
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
    cl_d[(size_t)i * K + s] = d;
    eta[(size_t)i * K + s] = (float)(1.0 / (double)d);
  }
  for (int s = 0; s < BL; ++s) bll[(size_t)i * BL + s] = kj[(K + s) * 64 + tid];
  if (kd[tid] == 0.0) atomicOr(&st->dup, 1);
}

}  // namespace faco
