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
#include "faco_update.hpp"

namespace faco {

// q mod n; the common cases (q within one period of [0, n)) avoid a division
FACO_DEV int64_t ticks() { return (int64_t)wall_clock64(); }

// Clock reads inside the local-search rounds and the construction steps (the
// per-phase breakdown); each one waits for the wave's outstanding LDS and
// scalar operations.  Building with FACO_FINE_TICKS=0 leaves only the
// per-ant totals.
#ifndef FACO_FINE_TICKS
#define FACO_FINE_TICKS 1
#endif
FACO_DEV int64_t fine_ticks() { return FACO_FINE_TICKS ? ticks() : 0; }

// Per-ant event counters and tick sums, one per lane (lane c holds entry c)
// instead of one scalar register pair each: the local search needs the
// scalar registers for its own state.  Updates take the first active lane's
// increment, which is the wave's (every update sits in uniform control flow).
struct LaneCounters {
  int64_t v = 0;
  struct Ref {
    int64_t &v;
    int c;
    FACO_DEV void operator+=(int64_t d) {
      d = (int64_t)uniform_u64((uint64_t)d);
      v += lane_id() == c ? d : 0;
    }
    FACO_DEV void operator++(int) { v += lane_id() == c ? 1 : 0; }
    FACO_DEV void operator=(int64_t x) {
      x = (int64_t)uniform_u64((uint64_t)x);
      v = lane_id() == c ? x : v;
    }
  };
  FACO_DEV Ref operator[](int c) { return Ref{v, c}; }
};

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

// Offset a source position by |off| <= 4096 (cheap form when n >= 4096).
FACO_DEV int wrap_off(int q, int off, int n) {
  if (n >= 4096) {
    q += off;
    return q >= n ? q - n : (q < 0 ? q + n : q);
  }
  return wrapn(q + off, n);
}

// ===================================================================== //
// Ant teams.  An ant may own TW waves of one workgroup.  Wave 0 (the leader)
// runs every decision of the ant; the other waves wait at a workgroup
// barrier for a command posted in LDS and take a share of the wide steps:
// the speculative source-following window (64 TW steps at once), the array
// rewrites of 2-opt and Or-opt moves, and the move tests of a sweep.  Who
// computes a step never changes its result.
//   protocol: leader writes op + arguments, barrier; every wave does its
//   share (a step with a read/write hazard has barriers of its own, taken by
//   every wave alike); barrier; the leader reads what the op left in LDS.
// ===================================================================== //
constexpr int kMaxTeam = 8;
enum TeamOp {
  OP_EXIT = 0, OP_REVERSE = 1, OP_SHIFT = 2, OP_WINDOW = 3, OP_SWEEP = 4, OP_COPY = 5,
  OP_NEAREST = 6, OP_OROPT = 7, OP_SEGPERM = 8, OP_SEGMAT = 9
};
struct TeamLds {
  int op;
  int arg[11];
  uint64_t arg64[2];
  int f[2 * kMaxTeam];           // per-wave first stop (window, copy: by round parity)
  int res[4];                    // window: last followed city; decision v, dv, pv
  int64_t part[kMaxTeam];        // window: per-wave sums of source edge costs
  int64_t ub[kMaxTeam];          // nearest: per-wave bounds
  int cities[kMaxTeam * kWave];  // sweep: the batch of cities to test
  int disp[4];                   // persistent batches: the next task
  int64_t okey[kMaxTeam][4];     // Or-opt: per-wave maxima of each listed city
  int orx[14][kWave];            // Or-opt: the leader's loaded neighbourhoods
  int sgs[4];                    // segment-list tour: live buffer, epoch, last move's records
  int sov[9];                    // segment-list move: link overrides
};
template <int TW>
constexpr int team_words() {
  return TW > 1 ? (int)((sizeof(TeamLds) + 15) / 16) * 4 : 0;
}

FACO_DEV void team_post(TeamLds *tl, int op, int a0 = 0, int a1 = 0, int a2 = 0, int a3 = 0,
                        int a4 = 0) {
  if (lane_id() == 0) {
    tl->op = op;
    tl->arg[0] = a0;
    tl->arg[1] = a1;
    tl->arg[2] = a2;
    tl->arg[3] = a3;
    tl->arg[4] = a4;
  }
  team_sync();
}
FACO_DEV int team_arg(const TeamLds *tl, int i) { return uniform_i(tl->arg[i]); }

// ===================================================================== //
// Backup list, then the nearest unvisited city (when no candidate of u is
// unvisited).  Uniform result.
// ===================================================================== //
// Nearest unvisited city to u by (squared distance, original number): lane l
// of wave w scans bitmap words w * 64 + l, + 64 TW, ...; fully visited words
// and words whose bounding box lies beyond a bound are skipped.  Each wave
// leaves its (distance, city) minimum in LDS (TW > 1).
template <int TW>
FACO_DEV void nearest_part(const Inst &I, int u, int w, const uint32_t *vis, TeamLds *tl,
                           int64_t &md, int &mj) {
  const int lane = lane_id();
  const int2 xu = I.xy[u];
  const int W = (I.n + 31) >> 5;
  auto free_word = [&](int wi) -> uint32_t {
    if (wi >= W) return 0u;
    uint32_t f = ~vis[wi];
    const int rem = I.n - wi * 32;
    if (rem < 32) f &= (1u << rem) - 1u;
    return f;
  };
  // A bound first: the nearest of the first unvisited cities of the TW 64
  // bitmap words around u's (labels follow a space-filling curve, so these
  // are close).  A word whose cities' bounding box lies farther than the
  // bound cannot hold the nearest city (nor one tied with it) and is skipped.
  int64_t ub = INT64_MAX;
  {
    constexpr int span = TW * kWave;
    int lo = (u >> 5) - span / 2;
    lo = lo > W - span ? W - span : lo;
    lo = lo < 0 ? 0 : lo;
    const int wi = lo + w * kWave + lane;
    const uint32_t f = free_word(wi);
    if (f) ub = (int64_t)sqd_u64(xu, I.xy[wi * 32 + __builtin_ctz(f)]);
  }
  ub = wave_min_i64(ub);
  if (TW > 1) {
    if (lane == 0) tl->ub[w] = ub;
    team_sync();
    ub = wave_min_i64(lane < TW ? tl->ub[lane] : INT64_MAX);
  }
  // distances only; equal distances are settled by original number below.
  // Lane l of wave w takes words w 64 + l + i TW 64, i = 0, 1, ..., 32 at a
  // time: their boxes are tested with the loads in flight together, then the
  // unvisited cities of the kept words are taken kNearBatch at a time, so that
  // their coordinate loads are in flight together too.
  constexpr int kNearBatch = 8;
  constexpr int stride = TW * kWave;
  int64_t bd = INT64_MAX;
  int bj = 0x7fffffff;
  bool tie = false;
  for (int g0 = w * kWave + lane; g0 < W; g0 += 32 * stride) {
    uint32_t keep = 0u;
    for (int k0 = 0; k0 < 32; k0 += 8) {
      int4 bx[8];
      bool has[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int wk = g0 + (k0 + k) * stride;
        has[k] = free_word(wk) != 0u;
        bx[k] = has[k] ? I.wbox[wk] : make_int4(0, 0, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (has[k]) {
          const int64_t dx = xu.x < bx[k].x ? (int64_t)bx[k].x - xu.x
                                            : (xu.x > bx[k].z ? (int64_t)xu.x - bx[k].z : 0);
          const int64_t dy = xu.y < bx[k].y ? (int64_t)bx[k].y - xu.y
                                            : (xu.y > bx[k].w ? (int64_t)xu.y - bx[k].w : 0);
          if (dx * dx + dy * dy <= ub) keep |= 1u << (k0 + k);
        }
      }
      if (g0 + (k0 + 8) * stride >= W) break;
    }
    int wi = 0;
    uint32_t fb = 0u;
    for (;;) {
      int jb[kNearBatch];
      bool vb[kNearBatch];
#pragma unroll
      for (int k = 0; k < kNearBatch; ++k) {
        while (fb == 0u && keep != 0u) {
          wi = g0 + __builtin_ctz(keep) * stride;
          keep &= keep - 1u;
          fb = free_word(wi);
        }
        vb[k] = fb != 0u;
        jb[k] = vb[k] ? wi * 32 + __builtin_ctz(fb) : u;
        fb &= fb - 1u;
      }
      if (!vb[0]) break;
      int2 xb[kNearBatch];
#pragma unroll
      for (int k = 0; k < kNearBatch; ++k) xb[k] = I.xy[jb[k]];
#pragma unroll
      for (int k = 0; k < kNearBatch; ++k) {
        if (vb[k]) {
          const int64_t d = (int64_t)sqd_u64(xu, xb[k]);
          if (d < bd) {
            bd = d;
            bj = jb[k];
            tie = false;
          } else if (d == bd) {
            tie = true;
          }
        }
      }
    }
  }
  md = wave_min_i64(bd);
  int mo = 0x7fffffff;
  mj = 0x7fffffff;
  if (md != INT64_MAX) {
    const uint64_t at = ballot(bd == md);
    if (__builtin_popcountll(at) == 1 && !ballot(bd == md && tie)) {
      mj = readlane_i(bj, ctz64(at));
      mo = uniform_i(I.orig_of[mj]);
    } else {
      // several cities at distance md: the smallest original number
      int bo = 0x7fffffff, bj2 = 0x7fffffff;
      for (int wi = w * kWave + lane; wi < W; wi += TW * kWave) {
        uint32_t free_bits = ~vis[wi];
        const int rem = I.n - wi * 32;
        if (rem < 32) free_bits &= (1u << rem) - 1u;
        while (free_bits) {
          const int j = wi * 32 + __builtin_ctz(free_bits);
          free_bits &= free_bits - 1;
          if ((int64_t)sqd_u64(xu, I.xy[j]) == md) {
            const int o = I.orig_of[j];
            if (o < bo) {
              bo = o;
              bj2 = j;
            }
          }
        }
      }
      mo = wave_min_i32(bo);
      mj = wave_min_i32(bo == mo ? bj2 : 0x7fffffff);
    }
  }
  if (TW > 1 && lane == 0) {
    tl->part[w] = md;
    tl->f[w] = mo;
    tl->f[kMaxTeam + w] = mj;
  }
}

template <int TW>
FACO_DEV int select_fallback(const Inst &I, int u, const uint32_t *vis, TeamLds *tl,
                             LaneCounters &cnt) {
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
  // best heuristic value = nearest unvisited city, ties by smaller original number
  cnt[CNT_FALLBACK]++;
  int64_t md;
  int mj;
  if (TW == 1) {
    nearest_part<1>(I, u, 0, vis, tl, md, mj);
    return mj;
  }
  team_post(tl, OP_NEAREST, u);
  nearest_part<TW>(I, u, 0, vis, tl, md, mj);
  team_sync();
  const int64_t d = lane < TW ? tl->part[lane] : INT64_MAX;
  const int o = lane < TW ? tl->f[lane] : 0x7fffffff;
  const int j = lane < TW ? tl->f[kMaxTeam + lane] : 0x7fffffff;
  const int64_t dmin = wave_min_i64(d);
  const int omin = wave_min_i32(d == dmin ? o : 0x7fffffff);
  return uniform_i(wave_min_i32(d == dmin && o == omin ? j : 0x7fffffff));
}

// Greedy step of the nearest-neighbour tour: first unvisited candidate
// (lists are sorted by distance), else the fallback chain.  dv = its cost.
template <int TW>
FACO_DEV int select_greedy(const Inst &I, int u, const uint32_t *vis, TeamLds *tl, int &dv,
                           LaneCounters &cnt) {
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
  const int v = select_fallback<TW>(I, u, vis, tl, cnt);
  dv = cost(I.xy[u], I.xy[v]);
  return v;
}

// ===================================================================== //
// Copy-from-source (Alg. 2, reading: forward from v while unvisited, else
// backward).  The first probe looks 64 positions both ways at once; later
// rounds take 256 positions per wave (64 TW * 4 per round for a team).
// Edge costs come from the per-iteration source edge table.  Returns the
// count; u/pu become the last appended city and its source position.
// ===================================================================== //
struct CopyOut {
  int app;      // cities appended
  int last;     // the last of them (-1: none)
  int64_t sum;  // their edge costs
};

// Rounds from source position pcur in direction dir, appending at k.  A
// round's cities lie past every earlier round's (the walk stops before it
// could wrap onto them), so a round reads no visited bit another wave of the
// same round sets.  The per-wave stops of consecutive rounds use alternate
// LDS slots, so one barrier per round suffices.
template <int TW>
FACO_DEV void copy_rounds(const Inst &I, int pcur, int dir, int k, int w, TeamLds *tl,
                          uint32_t *vis, int32_t *route, int32_t *pos, int2 *rxy,
                          CopyOut &o) {
  const int n = I.n, lane = lane_id();
  constexpr int RW = 4 * kWave;  // positions per wave and round
  int64_t dsum = 0;
  int app = 0, last = -1;
  for (int r = 0;; ++r) {
    int cc[4], dd[4];
    int2 cx[4];
    bool vc[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int q = wrap_off(pcur, dir * (w * RW + h * kWave + lane + 1), n);
      cc[h] = I.src_route[q];
      cx[h] = I.src_xy[q];
      dd[h] = I.src_d[dir > 0 ? (q == 0 ? n - 1 : q - 1) : q];
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) vc[h] = bit_get(vis, cc[h]);
    int jj = RW;
#pragma unroll
    for (int h = 3; h >= 0; --h) {
      const uint64_t m = ballot(vc[h]);
      if (m) jj = h * kWave + ctz64(m);
    }
    int J;
    if (TW > 1) {
      int *f = tl->f + (r & 1) * kMaxTeam;
      if (lane == 0) f[w] = jj < RW ? w * RW + jj : TW * RW;
      team_sync();
      J = uniform_i(wave_min_i32(lane < TW ? f[lane] : 0x7fffffff));
    } else {
      J = jj;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int idx = w * RW + h * kWave + lane;
      if (idx < J) {
        route[k + idx] = cc[h];
        pos[cc[h]] = k + idx;
        rxy[k + idx] = cx[h];
        bit_set(vis, cc[h]);
        dsum += dd[h];
      }
      if (idx == J - 1) {
        if (TW > 1)
          tl->res[0] = cc[h];
        else
          last = cc[h];
      }
    }
    if (TW == 1 && J > 0) last = readlane_i(last, (J - 1) & (kWave - 1));
    app += J;
    k += J;
    pcur = wrapn(pcur + dir * J, n);
    if (J < TW * RW) break;
  }
  o.app = app;
  o.last = last;
  o.sum = wave_sum_i64(dsum);
  if (TW > 1 && lane == 0) tl->part[w] = o.sum;
}

template <int TW>
FACO_DEV int copy_from(const Inst &I, int pv, int &k, int &u, int &pu, int64_t &len,
                       TeamLds *tl, int32_t *route, int32_t *pos, int2 *rxy, uint32_t *vis) {
  const int n = I.n, lane = lane_id();
  const int qf = wrap_off(pv, lane + 1, n), qb = wrap_off(pv, -lane - 1, n);
  const int cf = I.src_route[qf], cb = I.src_route[qb];
  const int2 xf = I.src_xy[qf], xb = I.src_xy[qb];
  const int df = I.src_d[qf == 0 ? n - 1 : qf - 1], db = I.src_d[qb];
  const uint64_t mf = ballot(bit_get(vis, cf));
  const int jf = mf ? ctz64(mf) : kWave;
  int dir, j, c, d;
  int2 cxy;
  if (jf > 0) {
    dir = 1; j = jf; c = cf; d = df; cxy = xf;
  } else {
    const uint64_t mb = ballot(bit_get(vis, cb));
    dir = -1; j = mb ? ctz64(mb) : kWave; c = cb; d = db; cxy = xb;
  }
  if (j == 0) return 0;
  if (lane < j) {
    route[k + lane] = c;
    pos[c] = k + lane;
    rxy[k + lane] = cxy;
    bit_set(vis, c);
  }
  len += wave_sum_i64(lane < j ? (int64_t)d : 0);
  u = readlane_i(c, j - 1);
  k += j;
  const int pcur = wrap_off(pv, dir * j, n);
  if (j < kWave) {
    pu = pcur;
    return j;
  }
  CopyOut o;
  if (TW > 1) {
    team_post(tl, OP_COPY, pcur, dir, k);
    copy_rounds<TW>(I, pcur, dir, k, 0, tl, vis, route, pos, rxy, o);
    team_sync();
    o.app = uniform_i(o.app);
    o.sum = wave_sum_i64(lane < TW ? tl->part[lane] : 0);
    o.last = o.app > 0 ? uniform_i(tl->res[0]) : -1;
  } else {
    wave_fence();
    copy_rounds<1>(I, pcur, dir, k, 0, tl, vis, route, pos, rxy, o);
  }
  len += o.sum;
  if (o.app > 0) u = o.last;
  k += o.app;
  pu = wrapn(pcur + dir * o.app, n);
  return j + o.app;
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

struct WinOut {
  int acc;        // steps that followed the source
  int v, dv, pv;  // decision of step `step + acc` (v = -2: window ran out)
  int lastq;      // city reached after the accepted steps
  int64_t srcsum; // their edge costs
};

// Wave w of a team evaluates steps step + 64 w + lane (TW = 1: lanes only).
// The accepted steps are appended to the tour here (route, pos, rxy and the
// visited bits), by the wave that evaluated them.
template <int KT, int TW>
FACO_DEV void window_part(const Inst &I, uint64_t t, uint64_t ant, uint64_t step, int u,
                          int pu, int dir, int k, int maxw, int w, TeamLds *tl,
                          uint32_t *vis, int32_t *route, int32_t *pos, int2 *rxy, Draws &D,
                          WinOut &o, int round = 0) {
  const int n = I.n, K = I.k, lane = lane_id();
  const int g = w * kWave + lane;
  o.v = -2;
  o.dv = 0;
  o.pv = 0;
  o.lastq = u;
  o.srcsum = 0;
  // every load below is addressed by source position: one round trip
  const int rpos = wrap_off(pu, dir * g, n);      // position of q_g
  const int qpos = wrap_off(pu, dir * (g + 1), n);
  const int qn = I.src_route[qpos];                // q_{g+1}
  const int2 qxy = I.src_xy[qpos];
  const int ed = I.src_d[dir > 0 ? rpos : qpos];   // cost q_g -> q_{g+1}
  const size_t row = srow(rpos, 0, K);
  int c[KT], sp[KT], cd[KT];
  float wt[KT];
#pragma unroll
  for (int s = 0; s < KT; ++s) {
    if (s < K) {
      c[s] = I.scl[row + 64 * s];
      wt[s] = I.sw[row + 64 * s];
      sp[s] = I.ssp[row + 64 * s];
      cd[s] = I.sd[row + 64 * s];
    }
  }
  D.u = unit24(philox_word0(I.seed, t, ant, step + (uint64_t)g, kPurposeRoulette));
  D.base = step + (uint64_t)(w * kWave);
  D.valid = true;
  const float U = D.u;
  float P[KT];
  float total = 0.0f;
  int last = -1;
#pragma unroll
  for (int s = 0; s < KT; ++s) {
    if (s < K) {
      const int off = dir > 0 ? sp[s] - pu : pu - sp[s];
      const int offw = off < 0 ? off + n : off;
      const bool visited = bit_get(vis, c[s]) || (offw >= 1 && offw <= g);
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
  int valid = n - k < TW * kWave ? n - k : TW * kWave;  // steps left
  valid = valid < maxw ? valid : maxw;
  const bool match = !special && choice == qn && g < valid;
  const uint64_t mm = ballot(!match);
  int F = mm ? w * kWave + ctz64(mm) : TW * kWave;
  if (TW > 1) {
    int *f = tl->f + (round & 1) * kMaxTeam;
    if (lane == 0) f[w] = F;
    team_sync();  // every wave's evaluation is done before any append
    F = uniform_i(wave_min_i32(lane < TW ? f[lane] : 0x7fffffff));
  }
  const int acc = F < valid ? F : valid;
  if (g < acc) {
    route[k + g] = qn;
    pos[qn] = k + g;
    rxy[k + g] = qxy;
    bit_set(vis, qn);
  }
  const int64_t ssum = wave_sum_i64(g < acc ? (int64_t)ed : 0);
  o.acc = acc;
  if (TW == 1) {
    o.srcsum = ssum;
    o.lastq = acc > 0 ? readlane_i(qn, acc - 1) : u;
    if (acc < valid) {
      if (readlane_i(special ? 1 : 0, acc)) {
        o.v = -1;
      } else {
        o.v = readlane_i(choice, acc);
        o.dv = readlane_i(choice_d, acc);
        o.pv = readlane_i(choice_p, acc);
      }
    } else {
      o.v = -2;
    }
  } else {
    // results for the leader, read after the closing barrier
    o.srcsum = ssum;
    if (acc > 0 && g == acc - 1) tl->res[0] = qn;
    if (acc < valid && g == acc) {
      tl->res[1] = special ? -1 : choice;
      tl->res[2] = choice_d;
      tl->res[3] = choice_p;
    }
    o.v = acc < valid ? 0 : -2;
  }
}

// A team runs up to kWinRounds windows in one command: while a window is
// followed to its end, the next one starts from where it stopped (every wave
// derives the new start alike; the last followed city comes through LDS).
// Per-wave partial sums of the followed edges end in tl->part.
constexpr int kWinRounds = 16;
template <int KT, int TW>
FACO_DEV void window_rounds(const Inst &I, uint64_t t, uint64_t ant, uint64_t step, int u,
                            int pu, int dir, int k, int maxw, int w, TeamLds *tl,
                            uint32_t *vis, int32_t *route, int32_t *pos, int2 *rxy, Draws &D,
                            WinOut &o) {
  const int n = I.n;
  int total = 0;
  int64_t sum = 0;
  for (int r = 0;; ++r) {
    WinOut q;
    window_part<KT, TW>(I, t, ant, step, u, pu, dir, k, maxw, w, tl, vis, route, pos, rxy, D,
                        q, r);
    const int acc = uniform_i(q.acc);
    total += acc;
    sum += q.srcsum;
    int valid = n - k < TW * kWave ? n - k : TW * kWave;
    valid = valid < maxw ? valid : maxw;
    team_sync();  // this window's appends and results are visible
    if (acc < valid || r + 1 >= kWinRounds || k + acc >= n) {
      o = q;
      break;
    }
    u = uniform_i(tl->res[0]);
    pu = wrap_off(pu, dir * acc, n);
    k += acc;
    step += (uint64_t)acc;
  }
  o.acc = total;
  if (lane_id() == 0) tl->part[w] = sum;
}

// Leader side of a window (TW > 1: posts it, takes wave 0's share, collects).
template <int KT, int TW>
FACO_DEV WinOut team_window(const Inst &I, uint64_t t, uint64_t ant, uint64_t step, int u,
                            int pu, int dir, int k, int maxw, TeamLds *tl, uint32_t *vis,
                            int32_t *route, int32_t *pos, int2 *rxy, Draws &D) {
  WinOut o;
  if (TW > 1) {
    if (lane_id() == 0) {
      tl->arg64[0] = t;
      tl->arg64[1] = step;
    }
    team_post(tl, OP_WINDOW, u, pu, dir, k, maxw);
  }
  if (TW > 1)
    window_rounds<KT, TW>(I, t, ant, step, u, pu, dir, k, maxw, 0, tl, vis, route, pos, rxy, D,
                          o);
  else
    window_part<KT, TW>(I, t, ant, step, u, pu, dir, k, maxw, 0, tl, vis, route, pos, rxy, D,
                        o);
  if (TW > 1) {
    team_sync();
    o.acc = uniform_i(o.acc);
    o.srcsum = wave_sum_i64(lane_id() < TW ? tl->part[lane_id()] : 0);
    o.lastq = o.acc > 0 ? uniform_i(tl->res[0]) : u;
    if (uniform_i(o.v) == 0) {
      o.v = uniform_i(tl->res[1]);
      o.dv = uniform_i(tl->res[2]);
      o.pv = uniform_i(tl->res[3]);
    } else {
      o.v = -2;
    }
  }
  return o;
}

// One ACO step from the city at source position pu, lane s = candidate slot
// s (used once new_edges >= m, when every step is followed by a copy).
// v = -1 when no candidate is unvisited.
FACO_DEV int one_step(const Inst &I, uint64_t t, uint64_t ant, uint64_t step, int pu,
                      const uint32_t *vis, Draws &D, int &dv, int &pv) {
  const int n = I.n, K = I.k, lane = lane_id();
  (void)n;
  const bool act = lane < K;
  const size_t row = srow(pu, act ? lane : 0, K);
  const int c = act ? I.scl[row] : 0;
  const float w = act ? I.sw[row] : 0.0f;
  const int sp = act ? I.ssp[row] : 0;
  const int d = act ? I.sd[row] : 0;
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
template <int KT, int TW>
FACO_DEV int64_t construct(const Inst &I, uint64_t t, int ant, bool greedy,
                           int32_t *route, int32_t *pos, int2 *rxy, int32_t *ring,
                           uint32_t *vis, uint32_t *inq, TeamLds *tl, int W, int &nchk,
                           LaneCounters &cnt, LaneCounters &tk) {
  const int n = I.n, lane = lane_id();
  for (int w = lane; w < W; w += kWave) {
    vis[w] = 0u;
    inq[w] = 0u;
  }
  wave_fence();
  // start: city 0 for the greedy tour, else a uniform draw (original numbers)
  const int r0 = uniform_i(
      I.int_of[greedy ? 0
                      : uniform_node(philox_word0(I.seed, t, (uint64_t)ant, 0, kPurposeStart),
                                     n)]);
  int u = r0;
  append_city(I, u, 0, route, pos, rxy, vis);
  // calc_num_new_edges() (Alg. 2): the constant min_new_edges, or this ant's
  // uniform draw from [min_new_edges, min_new_edges_max]
  int m = I.m;
  if (!greedy && I.m_hi > I.m)
    m += (int)__umul64hi(philox_word0(I.seed, t, (uint64_t)ant, 0, kPurposeNewEdges),
                         (uint64_t)(I.m_hi - I.m) + 1u);
  m = uniform_i(m);
  int k = 1, new_edges = 0;
  nchk = 0;
  int64_t len = 0;
  uint64_t step = 0;
  if (greedy) {
    while (k < n) {
      int dv;
      const int v = uniform_i(select_greedy<TW>(I, u, vis, tl, dv, cnt));
      ++step;
      len += dv;
      append_city(I, v, k, route, pos, rxy, vis);
      k = uniform_i(k + 1);
      u = v;
    }
  } else {
    int pu = uniform_i(I.src_pos[u]);
    int dir = 1;
    Draws D;
    D.base = 0;
    D.u = 0.0f;
    D.valid = false;
    while (k < n) {
      // Once new_edges >= m every ACO step is followed by a copy, so the
      // window is one step wide.
      // loop state is wave-uniform; keep it in scalar registers so that the
      // team barriers below sit in scalar control flow
      k = uniform_i(k);
      new_edges = uniform_i(new_edges);
      u = uniform_i(u);
      pu = uniform_i(pu);
      dir = uniform_i(dir);
      step = uniform_u64(step);
      const int maxw = new_edges >= m ? 1 : TW * kWave;
      int v, dv = 0, pv = 0;
      const int64_t c0 = fine_ticks();
      if (maxw == 1) {
        v = one_step(I, t, (uint64_t)ant, step, pu, vis, D, dv, pv);
        tk[6]++;
        tk[9] += fine_ticks() - c0;
      } else {
        // accepted steps follow the source: q_1..q_acc appended at k..k+acc-1
        const WinOut o = team_window<KT, TW>(I, t, (uint64_t)ant, step, u, pu, dir, k, maxw,
                                             tl, vis, route, pos, rxy, D);
        tk[5]++;
        tk[8] += fine_ticks() - c0;
        const int acc = uniform_i(o.acc);
        v = uniform_i(o.v);
        dv = uniform_i(o.dv);
        pv = uniform_i(o.pv);
        if (acc > 0) {
          k += acc;
          step += acc;
          len += o.srcsum;
          pu = wrap_off(pu, dir * acc, n);
          u = uniform_i(o.lastq);
        }
        wave_fence();
      }
      if (v == -2) {
        // the whole window followed the source; no step off the path
        v = u;
        pv = pu;
      } else {
        if (v == -1) {
          const int64_t c1 = fine_ticks();
          v = uniform_i(select_fallback<TW>(I, u, vis, tl, cnt));
          dv = uniform_i(cost(I.xy[u], I.xy[v]));
          pv = uniform_i(I.src_pos[v]);
          tk[11] += fine_ticks() - c1;
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
      u = uniform_i(v);
      pu = uniform_i(pv);
      new_edges = uniform_i(new_edges);
      k = uniform_i(k);
      dir = uniform_i(dir);
      if (new_edges >= m && k < n) {
        const int64_t c2 = fine_ticks();
        const int app = copy_from<TW>(I, pv, k, u, pu, len, tl, route, pos, rxy, vis);
        cnt[CNT_COPIED] += app;
        tk[7]++;
        tk[10] += fine_ticks() - c2;
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
// Loads of a segment-list evaluation a split city may come from: the city a
// itself, a neighbour of it, a candidate b, b's successor.
enum { SL_A = 0, SL_NB = 1, SL_B = 2, SL_BS = 3 };
struct Move {
  int kind;  // 0 none, 1 2-opt, 2 Or-opt
  int gain;
  int w, x, y, z;     // 2-opt: remove (w,x), (y,z)
  int px, py, pz;     // positions of x, y, z
  int f, l, p, q, a, o, b, e, L;  // Or-opt
  int fpos, pq, pp, pb, side;     // positions of f, q, p, b; e = succ(b) if side 0
  int s0, s1, s2;     // segment in array order
  int2 xs0, xs1, xs2; // and its coordinates
  // where a segment-list tour finds the cities a move splits at (2-opt: x, z;
  // Or-opt: the segment's first city, q, the insertion edge's second city):
  // the lane holding it and which of its loads (SegEval)
  int ln[3], lk[3];
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

// Lane j (constant after unrolling) of the lane's group of GS lanes.
template <int GS>
FACO_DEV int grp_lane(int v, int j) {
  if (GS == 16) return row_bcast(v, j);
  return __shfl(v, (lane_id() & ~(GS - 1)) + j);
}
template <int GS>
FACO_DEV int2 grp_lane2(int2 v, int j) {
  return make_int2(grp_lane<GS>(v.x, j), grp_lane<GS>(v.y, j));
}

// Maximum over the GS lanes of a group (GS = 16: one DPP row; 32: two).
template <int GS>
FACO_DEV int64_t group_max(int64_t v) {
  v = row_reduce_i64(v, OpMax());
  if (GS == 32) {
    const int64_t o = shfl_xor_i64(v, 16);
    v = o > v ? o : v;
  }
  return v;
}

// Per-lane state of a grouped evaluation: GS lanes evaluate one city a
// (slot s = lane % GS handles candidate s), 64 / GS cities per wave.
struct GroupEval {
  int a, pa, b, pb, pbs, pbp, bs, bp, nb, d_ab;
  int uc;          // lane s < 11: neighbourhood cost s of the group's city
  int d_bs, d_bp;  // costs of b's tour edges
  int2 xa, xnb, xb, xbs, xbp;
  int64_t key2, keyo;  // group maxima: 2-opt, Or-opt (0 = none)
};

template <int GS>
FACO_DEV void group_keys(uint32_t flags, bool act, GroupEval &R);

// All loads for both move kinds of every city of the wave are issued
// together (4 dependent levels).  Keys order candidates as the sequential
// evaluation does: 2-opt loop 1 over the list, loop 2 over the list; Or-opt
// variants, list slots, succ before pred.
template <int GS>
FACO_DEV GroupEval eval_group(const Inst &I, uint32_t flags, int a, bool gvalid,
                              const int32_t *route, const int32_t *pos, const int2 *rxy) {
  const int n = I.n, K = I.k, lane = lane_id();
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
  group_keys<GS>(flags, act, R);
  return R;
}

// The loads of a group that never change along a local search: the city's
// candidate row (candidate and cost) and its coordinates.  Loaded for the
// next group while the current move is applied.
struct GroupStatic {
  int a;       // the group's city (-1: none)
  int b, d_ab;
  int2 xa;
};
template <int GS>
FACO_DEV GroupStatic group_static(const Inst &I, int a, bool gvalid) {
  const int K = I.k, s = lane_id() & (GS - 1);
  const bool act = gvalid && s < K;
  const size_t row = (size_t)a * (size_t)K;
  GroupStatic P;
  P.a = gvalid ? a : -1;
  P.b = act ? I.cl[row + s] : a;
  P.d_ab = act ? I.cl_d[row + s] : 0;
  P.xa = I.xy[a];
  return P;
}

// eval_group with the static loads in registers: the positions of a and of
// its candidates are then the first level of loads, and the tour neighbours
// of both the second.
template <int GS>
FACO_DEV GroupEval eval_group_pre(const Inst &I, uint32_t flags, int a, bool gvalid,
                                  const GroupStatic &P, const int32_t *route,
                                  const int32_t *pos, const int2 *rxy) {
  const int n = I.n, K = I.k, lane = lane_id();
  const int s = lane & (GS - 1);
  const bool act = gvalid && s < K;
  GroupEval R;
  R.a = a;
  const int b = P.b, d_ab = P.d_ab;
  const int2 xa = P.xa;
  // level 1
  const int pa = pos[a];
  const int pb = pos[b];
  const int2 xb = I.xy[b];
  // level 2
  const int pn = wrapn(pa + s - 3, n);
  const int nb = s < 7 ? route[pn] : a;
  const int2 xnb = s < 7 ? rxy[pn] : xa;
  const int pbs = pb + 1 == n ? 0 : pb + 1, pbp = pb == 0 ? n - 1 : pb - 1;
  const int bs = route[pbs], bp = route[pbp];
  const int2 xbs = rxy[pbs], xbp = rxy[pbp];
  R.pa = pa; R.b = b; R.pb = pb; R.pbs = pbs; R.pbp = pbp; R.bs = bs; R.bp = bp;
  R.nb = nb; R.xa = xa; R.xnb = xnb; R.xb = xb; R.xbs = xbs; R.xbp = xbp; R.d_ab = d_ab;
  group_keys<GS>(flags, act, R);
  return R;
}

// The part of a group evaluation after the loads: neighbourhood costs and
// the 2-opt keys.
template <int GS>
FACO_DEV void group_keys(uint32_t flags, bool act, GroupEval &R) {
  const int lane = lane_id();
  const int gb = lane & ~(GS - 1);
  const int s = lane & (GS - 1);
  const int2 xnb = R.xnb, xb = R.xb, xbs = R.xbs, xbp = R.xbp;
  const int d_ab = R.d_ab;
  const int2 xas = grp_lane2<GS>(xnb, 4), xap = grp_lane2<GS>(xnb, 2);
  // Costs that depend only on the city's neighbourhood nb_0..nb_6 (tour
  // positions pa-3..pa+3), one per lane of the group: the tour edges
  // (nb_j, nb_j+1), j = 0..5, and the shortcuts (nb_2, nb_4), (nb_2, nb_5),
  // (nb_2, nb_6), (nb_1, nb_4), (nb_0, nb_4) that close the gap a removed
  // Or-opt segment leaves.  Consumers read them from the group's lanes.
  {
    const int su = s <= 5 ? s : (s <= 8 ? 2 : (s == 9 ? 1 : 0));
    const int sv = s <= 5 ? s + 1 : (s <= 8 ? s - 2 : 4);
    R.uc = cost(shfl_i2(xnb, gb + su), shfl_i2(xnb, gb + sv));
  }
  R.d_bs = cost(xb, xbs);
  R.d_bp = cost(xbp, xb);
  R.key2 = 0;
  if (flags & LS_2OPT) {
    const int d_as = grp_lane<GS>(R.uc, 3), d_ap = grp_lane<GS>(R.uc, 2);
    int g1 = 0, g2 = 0;
    if (act && d_as > d_ab) g1 = d_as + R.d_bs - d_ab - cost(xas, xbs);
    if (act && d_ap > d_ab) g2 = d_ap + R.d_bp - d_ab - cost(xap, xbp);
    const int64_t k1 = g1 > 0 ? (((int64_t)g1 << 8) | (int64_t)(255 - s)) : 0;
    const int64_t k2 = g2 > 0 ? (((int64_t)g2 << 8) | (int64_t)(255 - 32 - s)) : 0;
    R.key2 = group_max<GS>(k1 > k2 ? k1 : k2);
  }
  R.keyo = 0;
}

// Or-opt keys for the cities of the groups with `want` set (the others get 0).
// slot_mask selects the segment variants (slots) to evaluate.
template <int GS>
FACO_DEV void eval_group_oropt(const Inst &I, bool want, GroupEval &R,
                               uint32_t slot_mask = (1u << kOrSlots) - 1u) {
  const int n = I.n, K = I.k, lane = lane_id();
  const int s = lane & (GS - 1);
  const bool act = want && s < K;
  const int pa = R.pa, pb = R.pb, pbs = R.pbs, pbp = R.pbp, d_ab = R.d_ab;
  const int2 xnb = R.xnb, xbs = R.xbs, xbp = R.xbp;
  const int Lmax = or_lmax(I);
  int lbest = 0, lidx = 0;
  const int d_bs = R.d_bs, d_bp = R.d_bp;
  int u[11];
#pragma unroll
  for (int j = 0; j < 11; ++j) u[j] = grp_lane<GS>(R.uc, j);
#pragma unroll
  for (int vi = 0; vi < kOrSlots; ++vi) {
    int dir, L, lf, ll, lp, lq;
    or_slot_lanes(vi, dir, L, lf, ll, lp, lq);
    if (L > Lmax || !((slot_mask >> vi) & 1u)) continue;
    const int2 xf = grp_lane2<GS>(xnb, lf), xl = grp_lane2<GS>(xnb, ll);
    const int2 xo = dir == 0 ? xl : xf;
    const int fpos = dir == 0 ? pa : wrapn(pa - L + 1, n);
    // removal: (p, f) + (l, q) - (p, q); rem_a: the edge at a it removes
    const int rem_a = dir == 0 ? u[2] : u[3];
    const int g_rem = dir == 0 ? u[2] + u[2 + L] - u[5 + L]
                               : u[3 - L] + u[3] - (L == 2 ? u[9] : u[10]);
    if (!act) continue;
    if (!(d_ab < rem_a)) continue;
    if (wrapn(pb - fpos, n) < L) continue;
    // costs are >= 0: a variant whose gain without the new edge's cost
    // cannot beat lbest needs no cost
    if (wrapn(pbs - fpos, n) >= L && g_rem + d_bs - d_ab > lbest) {
      const int g = g_rem + d_bs - d_ab - cost(xo, xbs);
      if (g > lbest) {
        lbest = g;
        lidx = (vi * K + s) * 2 + 0;
      }
    }
    if (wrapn(pbp - fpos, n) >= L && g_rem + d_bp - d_ab > lbest) {
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
      mv.ln[0] = base + 4; mv.lk[0] = SL_NB;
      mv.ln[1] = l; mv.lk[1] = SL_BS;
    } else {         // loop 2: (pred a, a, pred b, b), flip a .. pred b
      const int l = base + idx - 32;
      mv.w = readlane_i(R.nb, base + 2); mv.x = a;
      mv.y = readlane_i(R.bp, l); mv.z = readlane_i(R.b, l);
      mv.px = pa;
      mv.py = readlane_i(R.pbp, l);
      mv.pz = readlane_i(R.pb, l);
      mv.ln[0] = base; mv.lk[0] = SL_A;
      mv.ln[1] = l; mv.lk[1] = SL_B;
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
  mv.ln[0] = base + lf; mv.lk[0] = SL_NB;
  mv.ln[1] = base + lq; mv.lk[1] = SL_NB;
  mv.ln[2] = l; mv.lk[2] = side ? SL_B : SL_BS;
  return mv;
}

// Lane-serial test used by the sweep (one city per lane): does x have an
// improving move?  Candidate lists are sorted by distance and every move
// through candidate b needs d(x, b) below the longer tour edge at x, so only
// a prefix of the list matters.  The candidates are taken CK at a time (a
// chunk is loaded, then tested), while a lane of the wave still needs them;
// inside a chunk every array index is a compile-time constant, so nothing
// is indexed at run time.
// candidates per chunk of the sweep's test (4: the test stops sooner than
// with 8, measured on the sweeps of the 100k workload; 16 at once spills)
#ifndef FACO_SWEEP_CK
#define FACO_SWEEP_CK 4
#endif
template <int KT>
FACO_DEV bool has_improving(const Inst &I, uint32_t flags, int x,
                            const int32_t *route, const int32_t *pos, const int2 *rxy) {
  constexpr int CK = KT < FACO_SWEEP_CK ? KT : FACO_SWEEP_CK;
  const int n = I.n, K = I.k;
  const size_t row = (size_t)x * (size_t)K;
  // first chunk of the list with the city's own data
  int cb[CK], cd[CK];
#pragma unroll
  for (int j = 0; j < CK; ++j) {
    cb[j] = j < K ? I.cl[row + j] : x;
    cd[j] = j < K ? I.cl_d[row + j] : 0x7fffffff;
  }
  const int px = pos[x];
  const int2 cx = I.xy[x];
  int xnx[7], xny[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int2 q = rxy[wrapn(px + j - 3, n)];
    xnx[j] = q.x; xny[j] = q.y;
  }
#define XN(j) make_int2(xnx[j], xny[j])
  const bool two = (flags & LS_2OPT) != 0, orr = (flags & LS_OROPT) != 0;
  const int d_s = cost(cx, XN(4)), d_p = cost(XN(2), cx);
  // Or-opt, per segment slot: where the segment starts, its length, the
  // endpoint that meets the insertion edge, the removed edge at x (0 when
  // the slot cannot apply: no candidate cost is below it) and the removal
  // gain
  int sf[kOrSlots], sl[kOrSlots], srem[kOrSlots], sg[kOrSlots], sox[kOrSlots], soy[kOrSlots];
  int lim = two ? (d_s > d_p ? d_s : d_p) : 0;
  const int Lmax = or_lmax(I);
#pragma unroll
  for (int vi = 0; vi < kOrSlots; ++vi) {
    int dir, L, lf, ll, lp, lq;
    or_slot_lanes(vi, dir, L, lf, ll, lp, lq);
    sl[vi] = L;
    sf[vi] = dir == 0 ? px : wrapn(px - L + 1, n);
    const int2 xo = dir == 0 ? XN(ll) : XN(lf);
    sox[vi] = xo.x;
    soy[vi] = xo.y;
    const int rem = dir == 0 ? d_p : d_s;
    srem[vi] = (orr && L <= Lmax && cd[0] < rem) ? rem : 0;
    sg[vi] = cost(XN(lp), XN(lf)) + cost(XN(ll), XN(lq)) - cost(XN(lp), XN(lq));
    lim = srem[vi] > lim ? srem[vi] : lim;
  }
  bool found = false;
  for (int c0 = 0;;) {
    int pb[CK], xbx[CK], xby[CK];
#pragma unroll
    for (int j = 0; j < CK; ++j) {
      pb[j] = pos[cb[j]];
      const int2 q = I.xy[cb[j]];
      xbx[j] = q.x; xby[j] = q.y;
    }
    int sx[CK], sy[CK], qx[CK], qy[CK];  // succ and pred of b
#pragma unroll
    for (int j = 0; j < CK; ++j) {
      const int2 q1 = rxy[pb[j] + 1 == n ? 0 : pb[j] + 1];
      const int2 q2 = rxy[pb[j] == 0 ? n - 1 : pb[j] - 1];
      sx[j] = q1.x; sy[j] = q1.y;
      qx[j] = q2.x; qy[j] = q2.y;
    }
#pragma unroll
    for (int j = 0; j < CK; ++j) {
      const int d_xb = cd[j];
      if (!found && c0 + j < K && d_xb < lim) {
        const int2 xb = make_int2(xbx[j], xby[j]);
        const int2 xbs = make_int2(sx[j], sy[j]), xbp = make_int2(qx[j], qy[j]);
        const int es = cost(xb, xbs) - d_xb, ep = cost(xbp, xb) - d_xb;
        if (two && d_s > d_xb && d_s + es - cost(XN(4), xbs) > 0) found = true;
        if (two && d_p > d_xb && d_p + ep - cost(XN(2), xbp) > 0) found = true;
        const int pbs = pb[j] + 1 == n ? 0 : pb[j] + 1, pbp = pb[j] == 0 ? n - 1 : pb[j] - 1;
#pragma unroll
        for (int vi = 0; vi < kOrSlots; ++vi) {
          const int L = sl[vi], fpos = sf[vi];
          if (!found && d_xb < srem[vi] && wrapn(pb[j] - fpos, n) >= L) {
            const int2 xo = make_int2(sox[vi], soy[vi]);
            // costs are >= 0: no cost of the new edge is needed unless the
            // rest of the gain is positive
            if (wrapn(pbs - fpos, n) >= L) {
              const int rest = sg[vi] + es;
              if (rest > 0 && rest - cost(xo, xbs) > 0) found = true;
            }
            if (wrapn(pbp - fpos, n) >= L) {
              const int rest = sg[vi] + ep;
              if (rest > 0 && rest - cost(xo, xbp) > 0) found = true;
            }
          }
        }
      }
    }
    c0 += CK;
    if (c0 >= K) break;
    // the next chunk, if a lane of the wave still needs it
    const int dn = I.cl_d[row + c0];
    if (!ballot(!found && dn < lim)) break;
#pragma unroll
    for (int j = 0; j < CK; ++j) {
      cb[j] = c0 + j < K ? I.cl[row + c0 + j] : x;
      cd[j] = c0 + j < K ? I.cl_d[row + c0 + j] : 0x7fffffff;
    }
  }
#undef XN
  return found;
}

// The flat tour (arrays in array order) as the sweep's test reads it.
struct FlatT {
  const int32_t *route, *pos;
  const int2 *rxy;
};
template <int KT>
FACO_DEV bool has_improving(const Inst &I, uint32_t flags, int x, const FlatT &T) {
  return has_improving<KT>(I, flags, x, T.route, T.pos, T.rxy);
}

#include "faco_seg.hpp"

constexpr int kChunks = 16;  // 64-element chunks in flight per wave and round
// Rewrites of more pairs than this (elements, for block moves: twice this)
// are shared by the team; shorter ones are the leader's alone.
constexpr int kTeamMinPairs = 256;
// Chunks in flight per wave of a team rewrite (one round covers
// TW * kTeamChunks * 64 pairs).
constexpr int kTeamChunks = 16;

// Reverse the cyclic array range of length L starting at s: pairs (i,
// L-1-i) are disjoint, so the 64-pair chunks are dealt to the waves of a
// team of TW in turn (chunk c to wave c mod TW), CH per wave in flight.
template <int TW, int CH = kChunks>
FACO_DEV void reverse_part(int n, int s, int L, int w, int32_t *route, int32_t *pos,
                           int2 *rxy) {
  const int lane = lane_id();
  const int half = L >> 1;
  const int nch = (half + kWave - 1) / kWave;
  for (int c0 = w; c0 < nch; c0 += TW * CH) {
    int p1[CH], p2[CH], v1[CH], v2[CH];
    int c1x[CH], c1y[CH], c2x[CH], c2y[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int i = (c0 + c * TW) * kWave + lane;
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
    for (int c = 0; c < CH; ++c) {
      const int i = (c0 + c * TW) * kWave + lane;
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

// Move the cyclic block of D elements at src to dst = src -+ L (L <= 3,
// D + L < n), keeping its order.  down: dst below src, rounds ascend; else
// rounds descend.  A round reads TW * CH * 64 elements, then (after a
// barrier when TW > 1) writes them: no round reads what a later-starting
// write of another wave could clobber.
template <int TW, int CH = kChunks>
FACO_DEV void shift_part(int n, int src, int dst, int D, bool down, int w, int32_t *route,
                         int32_t *pos, int2 *rxy) {
  const int lane = lane_id();
  constexpr int R = TW * CH * kWave;
  const int nr = (D + R - 1) / R;
  for (int r = 0; r < nr; ++r) {
    // round r covers elements [rb, rb + R); its chunks go to the waves in turn
    const int rb = (down ? r : nr - 1 - r) * R;
    int v[CH], cvx[CH], cvy[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int i = rb + (w + c * TW) * kWave + lane;
      if (i < D) {
        const int sp = wrap1(src + i, n);
        v[c] = route[sp];
        const int2 q = rxy[sp];
        cvx[c] = q.x; cvy[c] = q.y;
      }
    }
    if (TW > 1) team_sync();
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int i = rb + (w + c * TW) * kWave + lane;
      if (i < D) {
        const int d = wrap1(dst + i, n);
        route[d] = v[c];
        rxy[d] = make_int2(cvx[c], cvy[c]);
        pos[v[c]] = d;
      }
    }
  }
}

// Rewrites run by the leader alone when one round of its own covers them.
template <int TW>
FACO_DEV void team_reverse(int n, int s, int L, TeamLds *tl, int32_t *route, int32_t *pos,
                           int2 *rxy) {
  if (TW > 1 && (L >> 1) > kTeamMinPairs) {
    team_post(tl, OP_REVERSE, s, L);
    reverse_part<TW, kTeamChunks>(n, s, L, 0, route, pos, rxy);
    team_sync();
  } else if (TW > 1) {
    reverse_part<1, kTeamMinPairs / kWave>(n, s, L, 0, route, pos, rxy);
    wave_fence();
  } else {
    reverse_part<1>(n, s, L, 0, route, pos, rxy);
    wave_fence();
  }
}
template <int TW>
FACO_DEV void team_shift(int n, int src, int dst, int D, bool down, TeamLds *tl,
                         int32_t *route, int32_t *pos, int2 *rxy) {
  if (TW > 1 && D > 2 * kTeamMinPairs) {
    team_post(tl, OP_SHIFT, src, dst, D, down ? 1 : 0);
    shift_part<TW, kTeamChunks>(n, src, dst, D, down, 0, route, pos, rxy);
    team_sync();
  } else if (TW > 1) {
    shift_part<1, 2 * kTeamMinPairs / kWave>(n, src, dst, D, down, 0, route, pos, rxy);
    wave_fence();
  } else {
    shift_part<1>(n, src, dst, D, down, 0, route, pos, rxy);
    wave_fence();
  }
}

// "Flip a section between x and y": the shorter of the paths x..y and z..w.
// px, py, pz: array positions of x, y, z.
template <int TW>
FACO_DEV int apply_2opt(int n, int px, int py, int pz, TeamLds *tl, int32_t *route,
                        int32_t *pos, int2 *rxy) {
  const int L1 = wrapn(py - px, n) + 1;
  if (2 * L1 <= n) {
    team_reverse<TW>(n, px, L1, tl, route, pos, rxy);
    return L1;
  }
  team_reverse<TW>(n, pz, n - L1, tl, route, pos, rxy);
  return n - L1;
}

// Or-opt: the segment and the shorter block between its old place and the
// insertion edge exchange places (block keeps its orientation).
template <int TW>
FACO_DEV int apply_oropt(int n, int L, int a, int f, int b, int e, int side,
                         int pb, int fpos, int pq, int pp, int s0, int s1, int s2,
                         int2 xs0, int2 xs1, int2 xs2, TeamLds *tl, int32_t *route,
                         int32_t *pos, int2 *rxy) {
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
    team_shift<TW>(n, pq, fpos, D1, true, tl, route, pos, rxy);
    if (lane < L) {
      const int d = wrapn(fpos + D1 + lane, n);
      route[d] = ins;
      rxy[d] = insx;
      pos[ins] = d;
    }
    moved = D1 + L;
  } else {
    // block x2..p moves forward by L; segment goes in front of it
    team_shift<TW>(n, px2, wrap1(px2 + L, n), D2, false, tl, route, pos, rxy);
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

// Work queue of listed cities (FIFO).  Entries sit in an LDS ring while they
// fit (capacity I.lcap <= n), else in the ant's global ring (capacity n);
// a full LDS ring moves its entries to the global ring, oldest first, and
// the queue stays there.  Entries are written by lane 0; LDS operations of
// one wave complete in order, and the global ring is read by lane 0 only.
struct Queue {
  int head, tail, count;
  int cap;      // capacity of the ring in use
  int in_lds;   // 1: the LDS ring
  int32_t *lr;  // LDS ring
  int32_t *gr;  // global ring
};

FACO_DEV void q_spill(Queue &Q, int n) {
  const int lane = lane_id();
  for (int i = lane; i < Q.count; i += kWave) {
    int h = Q.head + i;
    h = h >= Q.cap ? h - Q.cap : h;
    Q.gr[i] = Q.lr[h];
  }
  wave_fence();
  Q.head = 0;
  Q.tail = Q.count == n ? 0 : Q.count;
  Q.cap = n;
  Q.in_lds = 0;
}

// push() of the cities x of the lanes with `take`, in lane order, all at once
// (the cities are distinct).
FACO_DEV int push_lanes(int n, int x, bool take, Queue &Q, uint32_t *inq, uint32_t *touched) {
  const int lane = lane_id();
  take = take && !bit_get(inq, x);
  const uint64_t pm = ballot(take);
  const int np = __builtin_popcountll(pm);
  if (np == 0) return 0;
  if (Q.in_lds && Q.count + np > Q.cap) q_spill(Q, n);
  if (take) {
    int t = Q.tail + __builtin_popcountll(pm & ((1ull << lane) - 1ull));
    t = t >= Q.cap ? t - Q.cap : t;
    bit_set(inq, x);
    bit_set(touched, x);
    (Q.in_lds ? Q.lr : Q.gr)[t] = x;
  }
  if (!Q.in_lds) wave_fence();  // the global ring is read back by lane 0
  Q.tail = Q.tail + np >= Q.cap ? Q.tail + np - Q.cap : Q.tail + np;
  Q.count += np;
  return np;
}

// push() of c[0], c[1], ... in that order, all at once: lane i takes c[i];
// it is listed unless it already is or an earlier lane holds the same city,
// and goes to the tail plus the number of listed lanes before it.
template <int NP>
FACO_DEV void push_all(int n, const int *c, Queue &Q, uint32_t *inq, uint32_t *touched) {
  const int lane = lane_id();
  int x = 0;
#pragma unroll
  for (int i = 0; i < NP; ++i) x = lane == i ? c[i] : x;
  bool take = lane < NP && !bit_get(inq, x);
#pragma unroll
  for (int i = 0; i < NP; ++i)
    if (i < lane && c[i] == x) take = false;
  const uint64_t pm = ballot(take);
  const int np = __builtin_popcountll(pm);
  if (np == 0) return;
  if (Q.in_lds && Q.count + np > Q.cap) q_spill(Q, n);
  if (take) {
    int t = Q.tail + __builtin_popcountll(pm & ((1ull << lane) - 1ull));
    t = t >= Q.cap ? t - Q.cap : t;
    bit_set(inq, x);
    bit_set(touched, x);
    (Q.in_lds ? Q.lr : Q.gr)[t] = x;
  }
  if (!Q.in_lds) wave_fence();  // the global ring is read back by lane 0
  Q.tail = Q.tail + np >= Q.cap ? Q.tail + np - Q.cap : Q.tail + np;
  Q.count += np;
}

// Sweep: test every touched city and list the improvable ones in ascending
// original number.  The touched cities are tested in label order, 64 TW at a
// time (wave w takes the w-th 64): labels follow a space-filling curve, so the
// cities of a batch have nearby candidate rows and tour neighbourhoods.  Each
// improvable city's original number is marked in the `ord` bitmap; `ord` is
// then read in ascending order and the marked cities are listed in that
// order (and `ord` is left clear).  The tour does not change during a sweep,
// so the order of the tests does not matter.
template <int KT, int TW, class TT>
FACO_DEV void sweep_part(const Inst &I, uint32_t flags, int count, int w, TeamLds *tl,
                         uint32_t *ord, const TT &T) {
  const int i = w * kWave + lane_id();
  if (i < count) {
    const int x = tl->cities[i];
    const int ox = I.orig_of[x];
    if (has_improving<KT>(I, flags, x, T)) bit_set(ord, ox);
  }
}

// Sweep tick slots (per ant): ticks in the move tests, ticks in listing the
// improvable cities, cities tested.
enum { TK_SWEEP_TESTS = 24, TK_SWEEP_LIST = 25, TK_SWEEP_CITIES = 26 };

template <int KT, int TW, class TT>
FACO_DEV int sweep(const Inst &I, uint32_t flags, int W, Queue &Q, const TT &T,
                   uint32_t *inq, uint32_t *touched, uint32_t *ord, TeamLds *tl,
                   LaneCounters &tk) {
  const int lane = lane_id();
  int bx = -1, bcount = 0;
  auto test = [&](int cnt) {
    const int64_t t0 = fine_ticks();
    tk[TK_SWEEP_CITIES] += cnt;
    if (TW == 1) {
      if (lane < cnt) {
        const int ox = I.orig_of[bx];
        if (has_improving<KT>(I, flags, bx, T)) bit_set(ord, ox);
      }
      tk[TK_SWEEP_TESTS] += fine_ticks() - t0;
      return;
    }
    // cnt cities sit in tl->cities[0..cnt)
    team_post(tl, OP_SWEEP, cnt, (int)flags);
    sweep_part<KT, TW>(I, flags, cnt, 0, tl, ord, T);
    team_sync();
    tk[TK_SWEEP_TESTS] += fine_ticks() - t0;
  };
  if (TW == 1) {
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
          if (lane == bcount) bx = (w0 + l) * 32 + bpos;
          if (++bcount == kWave) {
            test(kWave);
            bcount = 0;
          }
        }
      }
    }
    if (bcount) test(bcount);
  } else {
    // every lane with touched bits in its word places its lowest one per
    // pass (the order of the tests does not matter), slots by rank
    constexpr int cap = TW * kWave;
    int fill = 0;
    for (int w0 = 0; w0 < W; w0 += kWave) {
      uint32_t word = (w0 + lane < W) ? touched[w0 + lane] : 0u;
      for (;;) {
        const uint64_t m = ballot(word != 0u);
        if (!m) break;
        const int room = cap - fill;
        const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (word != 0u && r < room) {
          tl->cities[fill + r] = (w0 + lane) * 32 + __builtin_ctz(word);
          word &= word - 1u;
        }
        const int np = __builtin_popcountll(m);
        fill += np < room ? np : room;
        if (fill == cap) {
          test(cap);
          fill = 0;
        }
      }
    }
    if (fill) test(fill);
  }
  wave_fence();
  const int64_t tl0 = fine_ticks();
  // list the marked cities, ascending original number, 64 at a time
  int pushed = 0, bo = -1;
  bcount = 0;
  auto list = [&](int cnt) {
    const int x = lane < cnt ? I.int_of[bo] : 0;
    pushed += cnt;
    push_lanes(I.n, x, lane < cnt, Q, inq, touched);
  };
  for (int w0 = 0; w0 < W; w0 += kWave) {
    const uint32_t word = (w0 + lane < W) ? ord[w0 + lane] : 0u;
    if (w0 + lane < W) ord[w0 + lane] = 0u;
    uint64_t nz = ballot(word != 0u);
    while (nz) {
      const int l = ctz64(nz);
      nz &= nz - 1;
      uint32_t bits = (uint32_t)readlane_i((int)word, l);
      while (bits) {
        const int bpos = __builtin_ctz(bits);
        bits &= bits - 1;
        if (lane == bcount) bo = (w0 + l) * 32 + bpos;
        if (++bcount == kWave) {
          list(kWave);
          bcount = 0;
        }
      }
    }
  }
  if (bcount) list(bcount);
  tk[TK_SWEEP_LIST] += fine_ticks() - tl0;
  return pushed;
}

// The Or-opt evaluation of an LS round, shared by the helper waves of a team.
// The leader has loaded the listed cities' neighbourhoods and evaluated the
// 2-opt moves; when a city before the first one with a 2-opt move needs
// Or-opt, it leaves what the evaluation needs in tl->orx (lane by lane) and
// helper wave w (1 <= w < TW) takes segment variants w - 1, w - 1 + (TW - 1),
// ... for the cities before arg[0], leaving each city's maximum key in
// tl->okey[w].  Keys order variants as the sequential evaluation does, so the
// maximum over the waves is the sequential evaluation's result.
template <int TW>
FACO_DEV uint32_t or_slot_mask(int w) {
  uint32_t m = 0;
  for (int vi = w - 1; vi >= 0 && vi < kOrSlots; vi += TW - 1) m |= 1u << vi;
  return m;
}

FACO_DEV void or_share(TeamLds *tl, const GroupEval &R) {
  const int l = lane_id();
  tl->orx[0][l] = R.pa;
  tl->orx[1][l] = R.pb;
  tl->orx[2][l] = R.pbs;
  tl->orx[3][l] = R.pbp;
  tl->orx[4][l] = R.d_ab;
  tl->orx[5][l] = R.d_bs;
  tl->orx[6][l] = R.d_bp;
  tl->orx[7][l] = R.uc;
  tl->orx[8][l] = R.xnb.x;
  tl->orx[9][l] = R.xnb.y;
  tl->orx[10][l] = R.xbs.x;
  tl->orx[11][l] = R.xbs.y;
  tl->orx[12][l] = R.xbp.x;
  tl->orx[13][l] = R.xbp.y;
}

template <int KT, int TW>
FACO_DEV void oropt_part(const Inst &I, int w, TeamLds *tl) {
  constexpr int GS = KT <= 16 ? 16 : 32;
  const uint32_t mask = or_slot_mask<TW>(w);
  if (!mask) return;
  const int l = lane_id(), grp = l / GS;
  const int j2 = team_arg(tl, 0);
  GroupEval R;
  R.pa = tl->orx[0][l];
  R.pb = tl->orx[1][l];
  R.pbs = tl->orx[2][l];
  R.pbp = tl->orx[3][l];
  R.d_ab = tl->orx[4][l];
  R.d_bs = tl->orx[5][l];
  R.d_bp = tl->orx[6][l];
  R.uc = tl->orx[7][l];
  R.xnb = make_int2(tl->orx[8][l], tl->orx[9][l]);
  R.xbs = make_int2(tl->orx[10][l], tl->orx[11][l]);
  R.xbp = make_int2(tl->orx[12][l], tl->orx[13][l]);
  eval_group_oropt<GS>(I, grp < j2, R, mask);
  if ((l & (GS - 1)) == 0) tl->okey[w][grp] = R.keyo;
}

// The first fault of the instance keeps its ant (-1: the initial solution)
// and the iteration being built.
FACO_DEV void record_fault(const Inst &I, int32_t bit, int ant) {
  if (lane_id() == 0) {
    if (atomicOr(&I.st->fault, bit) == 0) {
      I.st->fault_ant = ant;
      I.st->fault_iter = I.st->iter + 1;
    }
  }
}

// SEG: the tour is a segment list (SQ); else the flat arrays route, pos, rxy.
template <int KT, int TW, bool SEG>
FACO_DEV int64_t local_search(const Inst &I, uint32_t flags, int32_t *route,
                              int32_t *pos, int2 *rxy, uint32_t *inq, uint32_t *touched,
                              uint32_t *ord, TeamLds *tl, int W, Queue Q, LaneCounters &cnt,
                              LaneCounters &tk, int ant, SegState &SQ) {
  constexpr int GS = KT <= 16 ? 16 : 32;  // lanes per evaluated city
  constexpr int G = kWave / GS;           // cities evaluated together
  const int n = I.n, lane = lane_id();
  const int grp = lane / GS;
  flags = (uint32_t)uniform_i((int)flags);
  int changes = 0, changes_at_sweep = -1;
  int64_t gain = 0;
  // The next round's static loads (its groups' candidate rows and
  // coordinates), issued during this round for the groups it will most
  // likely hold; used if it holds them.
  GroupStatic pre;
  pre.a = -1;
  pre.b = pre.d_ab = 0;
  pre.xa = make_int2(0, 0);
  for (;;) {
    for (;;) {
      Q.count = uniform_i(Q.count);
      Q.head = uniform_i(Q.head);
      Q.tail = uniform_i(Q.tail);
      Q.cap = uniform_i(Q.cap);
      Q.in_lds = uniform_i(Q.in_lds);
      changes = uniform_i(changes);
      if (!(Q.count > 0 && changes < n)) break;
      // Evaluate the next G listed cities on the current tour.  The first one
      // with a move is applied; the ones before it are popped with no move;
      // the ones after it stay listed (their evaluation is discarded).
      const int gcount = Q.count < G ? Q.count : G;
      int e[G];
      if (Q.in_lds) {
        int h = Q.head + lane;
        h = h >= Q.cap ? h - Q.cap : h;
        const int hv = lane < gcount ? Q.lr[h] : 0;
#pragma unroll
        for (int g = 0; g < G; ++g) e[g] = readlane_i(hv, g);
      } else {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          int h = Q.head + g;
          h = h >= Q.cap ? h - Q.cap : h;
          e[g] = readlane_i(lane == 0 && g < gcount ? Q.gr[h] : 0, 0);
        }
      }
      int a = e[0];
#pragma unroll
      for (int g = 1; g < G; ++g) a = grp == g ? e[g] : a;
      const int64_t t0 = fine_ticks();
      SegEval Z;
      GroupEval R;
      if constexpr (SEG) {
        R = eval_group_seg<GS>(I, flags, a, grp < gcount, SQ.T, Z);
      } else {
        // the prefetched loads serve if every group is full and holds the
        // city they were loaded for
        const bool hit = ballot(!(grp < gcount && pre.a == a)) == 0ull;
        if (hit)
          R = eval_group_pre<GS>(I, flags, a, true, pre, route, pos, rxy);
        else
          R = eval_group<GS>(I, flags, a, grp < gcount, route, pos, rxy);
        pre.a = -1;
      }
      // Or-opt is only tried where no 2-opt move exists, and only cities
      // before the first one with a 2-opt move can be the chosen one
      const uint64_t h2 = ballot((lane & (GS - 1)) == 0 && grp < gcount && R.key2 > 0);
      const int j2 = uniform_i(h2 ? ctz64(h2) / GS : gcount);
      // Most likely the move is the first 2-opt one (j2) and the next round
      // holds the G listed cities after it: load their static data now,
      // beside the rest of this round (a wrong guess only costs the loads).
      if constexpr (!SEG) {
        const int np_guess = j2 < gcount ? j2 + 1 : gcount;
        if (Q.in_lds && j2 < gcount && Q.count - np_guess >= G) {
          int h = Q.head + np_guess + grp;
          h = h >= Q.cap ? h - Q.cap : h;
          pre = group_static<GS>(I, Q.lr[h], true);
        }
      }
      if (TW > 1 && (flags & LS_OROPT) && j2 > 0) {
        // the team's helpers evaluate the Or-opt variants from the leader's loads
        const int64_t to = fine_ticks();
        or_share(tl, R);
        team_post(tl, OP_OROPT, j2);
        team_sync();
        int64_t k = 0;
#pragma unroll
        for (int w = 1; w < TW; ++w)
          if (or_slot_mask<TW>(w)) {
            const int64_t kw = tl->okey[w][grp];
            k = kw > k ? kw : k;
          }
        R.keyo = grp < j2 ? k : 0;
        tk[14]++;
        tk[13] += fine_ticks() - to;
      } else if ((flags & LS_OROPT) && j2 > 0) {
        const int64_t to = fine_ticks();
        eval_group_oropt<GS>(I, grp < j2, R);
        tk[13] += fine_ticks() - to;
        tk[14]++;
      }
      const int64_t t1 = fine_ticks();
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
          Q.head = Q.head + 1 == Q.cap ? 0 : Q.head + 1;
          Q.count--;
        }
      }
      cnt[CNT_LS_POPS] += npop;
      if (j >= gcount) continue;
      const Move mv = extract_move<GS>(I, R, j);
      const int64_t ta = fine_ticks();
      if (uniform_i(mv.kind) == 1) {
        if constexpr (SEG)
          cnt[CNT_MOVED_ELEMS] += seg_apply_2opt<TW>(I, SQ, tl, mv, Z, tk);
        else
          cnt[CNT_MOVED_ELEMS] += apply_2opt<TW>(n, uniform_i(mv.px), uniform_i(mv.py),
                                                 uniform_i(mv.pz), tl, route, pos, rxy);
        tk[15] += fine_ticks() - ta;
        const int pc[4] = {mv.w, mv.x, mv.y, mv.z};
        push_all<4>(n, pc, Q, inq, touched);
        cnt[CNT_MOVES_2OPT]++;
      } else {
        if constexpr (SEG)
          cnt[CNT_MOVED_ELEMS] += seg_apply_oropt<TW>(I, SQ, tl, mv, Z, tk);
        else
          cnt[CNT_MOVED_ELEMS] +=
              apply_oropt<TW>(n, uniform_i(mv.L), mv.a, mv.f, mv.b, mv.e, uniform_i(mv.side),
                              uniform_i(mv.pb), uniform_i(mv.fpos), uniform_i(mv.pq),
                              uniform_i(mv.pp), mv.s0, mv.s1, mv.s2, mv.xs0, mv.xs1, mv.xs2,
                              tl, route, pos, rxy);
        tk[15] += fine_ticks() - ta;
        const int pc[6] = {mv.p, mv.q, mv.b, mv.e, mv.f, mv.l};
        push_all<6>(n, pc, Q, inq, touched);
        cnt[CNT_MOVES_OROPT]++;
      }
      if constexpr (SEG) {
        // room for the next move's splits
        if (uniform_i(SQ.S) + 3 > I.seg_max) seg_materialize<TW>(I, ant < 0 ? 0 : ant, SQ, tl, tk);
      }
      tk[2] += fine_ticks() - t1;
      ++changes;
      gain += mv.gain;
    }
    changes = uniform_i(changes);
    if (!(flags & LS_SWEEP) || changes >= n) break;
    // Every city a sweep lists has an improving move, so a sweep that was
    // followed by no change can only come from the two move tests
    // disagreeing: stop instead of spinning, and report it.
    if (changes == changes_at_sweep) {
      record_fault(I, FAULT_LS_STALL, ant);
      break;
    }
    changes_at_sweep = changes;
    cnt[CNT_SWEEPS]++;
    const int64_t t2 = ticks();
    int pushed;
    if constexpr (SEG)
      pushed = uniform_i(sweep<KT, TW>(I, flags, W, Q, SQ.T, inq, touched, ord, tl, tk));
    else
      pushed = uniform_i(sweep<KT, TW>(I, flags, W, Q, FlatT{route, pos, rxy}, inq, touched,
                                       ord, tl, tk));
    tk[3] += ticks() - t2;
    if (pushed == 0) break;
  }
  cnt[CNT_LS_GAIN] += gain;
  return gain;
}

// ===================================================================== //
// Helper waves of a team: wait for a command, take this wave's share, repeat
// until the leader posts OP_EXIT.
// ===================================================================== //
template <int KT, int TW, bool SEG>
FACO_DEV void team_helper(const Inst &I, int ant, int w, TeamLds *tl, uint32_t *vis,
                          uint32_t *ord, int32_t *route, int32_t *pos, int2 *rxy, int4 *rec) {
  Draws D;
  // a segment-list move's record whose cities this wave labels after the move
  int rl_h = -1, rl_lo = 0, rl_hi = -1;
  SegT rl_T;
  for (;;) {
    if (SEG && rl_h >= 0) {
      seg_relabel(rl_T, rl_lo, rl_hi, rl_h);
      rl_h = -1;
    }
    team_sync();
    const int op = uniform_i(tl->op);
    if (op == OP_EXIT) break;
    if (op == OP_REVERSE) {
      reverse_part<TW, kTeamChunks>(I.n, team_arg(tl, 0), team_arg(tl, 1), w, route, pos, rxy);
    } else if (op == OP_SHIFT) {
      shift_part<TW, kTeamChunks>(I.n, team_arg(tl, 0), team_arg(tl, 1), team_arg(tl, 2),
                                  team_arg(tl, 3) != 0, w, route, pos, rxy);
    } else if (op == OP_WINDOW) {
      WinOut o;
      window_rounds<KT, TW>(I, uniform_u64(tl->arg64[0]), (uint64_t)ant,
                            uniform_u64(tl->arg64[1]), team_arg(tl, 0), team_arg(tl, 1),
                            team_arg(tl, 2), team_arg(tl, 3), team_arg(tl, 4), w, tl, vis,
                            route, pos, rxy, D, o);
    } else if (op == OP_COPY) {
      CopyOut o;
      copy_rounds<TW>(I, team_arg(tl, 0), team_arg(tl, 1), team_arg(tl, 2), w, tl, vis, route,
                      pos, rxy, o);
    } else if (op == OP_NEAREST) {
      int64_t md;
      int mj;
      nearest_part<TW>(I, team_arg(tl, 0), w, vis, tl, md, mj);
    } else if (op == OP_SWEEP) {
      if constexpr (SEG)
        sweep_part<KT, TW>(I, (uint32_t)team_arg(tl, 1), team_arg(tl, 0), w, tl, ord,
                           seg_view(I, ant, rec, uniform_i(tl->sgs[0]), uniform_i(tl->sgs[1]),
                                    uniform_i(tl->sgs[2]), uniform_i(tl->sgs[3])));
      else
        sweep_part<KT, TW>(I, (uint32_t)team_arg(tl, 1), team_arg(tl, 0), w, tl, ord,
                           FlatT{route, pos, rxy});
    } else if (SEG && op == OP_SEGPERM) {
      const SegT T = seg_view(I, ant, rec, uniform_i(tl->sgs[0]), uniform_i(tl->sgs[1]));
      const int rv = team_arg(tl, 5);
      const int S0 = team_arg(tl, 0), S = team_arg(tl, 1);
      // the new record this wave labels: read before the pass's barrier (the
      // leader may change records again once the move is over)
      if (S0 + w - 1 < S) {
        const int4 r = rec[S0 + w - 1];
        rl_h = S0 + w - 1;
        rl_lo = uniform_i(r.x);
        rl_hi = uniform_i(r.y);
        rl_T = T;
      }
      SegOv O;
#pragma unroll
      for (int j = 0; j < kSovPre + kSovPost; ++j) O.v[j] = uniform_i(tl->sov[j]);
      seg_perm_part(T, w * kWave + lane_id(), kWave * TW, S, team_arg(tl, 2), team_arg(tl, 3),
                    team_arg(tl, 4), rv & 1, (rv >> 1) & 1, O, team_arg(tl, 6),
                    team_arg(tl, 7));
      if (!FACO_SEG_DEFER && rl_h >= 0) {
        seg_relabel(rl_T, rl_lo, rl_hi, rl_h);
        rl_h = -1;
      }
    } else if (SEG && op == OP_SEGMAT) {
      const int live = uniform_i(tl->sgs[0]);
      const SegT T = seg_view(I, ant, rec, live, uniform_i(tl->sgs[1]), uniform_i(tl->sgs[2]),
                              uniform_i(tl->sgs[3]));
      const size_t o = (size_t)ant * (size_t)I.n;
      const int tid = w * kWave + lane_id();
      seg_mat_part(T, tid, kWave * TW, (live ? I.routes : I.r2) + o, (live ? I.rxy : I.x2) + o,
                   (live ? I.pos : I.p2) + o);
      team_sync();
      seg_reset_part(rec, tid, kWave * TW, (I.n + (1 << I.seg_shift) - 1) >> I.seg_shift, I.n,
                     I.seg_shift);
    } else if (op == OP_OROPT) {
      oropt_part<KT, TW>(I, w, tl);
    }
    team_sync();
  }
}

// ===================================================================== //
// One ant: construction + local search.  mode 0: ant `ant` of iteration
// st->iter + 1.  mode 1: initial solution (nearest neighbour + LS over all
// cities) written to the global best.
//   lds: [team area][visited W][listed W][sweep order W]
//        [SEG: segment records, I.seg_max int4 at a 16-byte boundary]
//        [queue ring I.lcap].
// ===================================================================== //
__host__ __device__ inline int seg_lds_words(int tw_words, int W) { return (tw_words + 3 * W + 3) & ~3; }

template <int KT, int TW, bool SEG = false>
FACO_DEV void run_ant(const Inst &I, int ant, int mode, uint32_t *lds) {
  const int n = I.n, lane = lane_id();
  const int W = (n + 31) >> 5;
  TeamLds *tl = (TeamLds *)lds;
  uint32_t *vis = lds + team_words<TW>();
  uint32_t *inq = vis + W;
  uint32_t *ord = inq + W;
  int4 *rec = (int4 *)(lds + seg_lds_words(team_words<TW>(), W));
  int32_t *route = I.routes + (size_t)ant * (size_t)n;
  int32_t *pos = I.pos + (size_t)ant * (size_t)n;
  int32_t *ring = I.ring + (size_t)ant * (size_t)n;
  int2 *rxy = I.rxy + (size_t)ant * (size_t)n;
  if (TW > 1) {
    const int w = uniform_i((int)(threadIdx.x >> 6));
    if (w > 0) {
      team_helper<KT, TW, SEG>(I, ant, w, tl, vis, ord, route, pos, rxy, rec);
      return;
    }
  }
  LaneCounters cnt, tk;
  const bool init = mode == 1;
  const uint64_t t = (uint64_t)I.st->iter + 1;
  int nchk = 0;
  const int64_t t0 = ticks();
  int64_t len = construct<KT, TW>(I, t, ant, init, route, pos, rxy, ring, vis, inq, tl, W, nchk,
                                  cnt, tk);
  tk[0] = ticks() - t0;
  uint32_t flags = I.ls_flags;
  const int lcap = I.lcap;
  Queue Q;
  Q.lr = SEG ? (int32_t *)(rec + I.seg_max) : (int32_t *)(ord + W);
  Q.gr = ring;
  if (init) {
    // the initial solution reports only its local-search counters
#pragma unroll
    for (int c = 0; c < CNT_LS_POPS; ++c) cnt[c] = 0;
    // with 3-opt, the initial search runs in init_search_kernel afterwards
    flags = (I.ls_flags & LS_INIT_3OPT) ? 0u : (LS_2OPT | LS_SWEEP | (I.ls_flags & LS_OROPT));
    Q.in_lds = n <= lcap ? 1 : 0;
    Q.cap = Q.in_lds ? lcap : n;
    // every city listed, in ascending original number
    for (int i = lane; i < n; i += kWave) (Q.in_lds ? Q.lr : ring)[i] = I.int_of[i];
    for (int w = lane; w < W; w += kWave) {
      const int rem = n - w * 32;
      const uint32_t full = rem >= 32 ? 0xFFFFFFFFu : ((1u << rem) - 1u);
      inq[w] = full;
      vis[w] = full;  // touched
    }
    Q.count = n;
    cnt[CNT_CHECKLIST0] = n;
  } else {
    for (int w = lane; w < W; w += kWave) vis[w] = 0u;
    wave_fence();
    Q.in_lds = nchk <= lcap ? 1 : 0;
    Q.cap = Q.in_lds ? lcap : n;
    for (int i = lane; i < nchk; i += kWave) {
      const int c = ring[i];
      bit_set(vis, c);
      if (Q.in_lds) Q.lr[i] = c;
    }
    Q.count = nchk;
    if (flags & (LS_2OPT | LS_OROPT)) cnt[CNT_CHECKLIST0] = nchk;
  }
  Q.head = 0;
  Q.tail = Q.count == Q.cap ? 0 : Q.count;
  for (int w = lane; w < W; w += kWave) ord[w] = 0u;  // sweeps leave it clear
  wave_fence();
  flags = (uint32_t)uniform_i((int)flags);
  Q.head = uniform_i(Q.head);
  Q.tail = uniform_i(Q.tail);
  Q.count = uniform_i(Q.count);
  Q.cap = uniform_i(Q.cap);
  Q.in_lds = uniform_i(Q.in_lds);
  SegState SQ;
  if constexpr (SEG) seg_begin(I, ant, rec, tl, TW > 1, SQ);
  if (flags & (LS_2OPT | LS_OROPT))
    len -= local_search<KT, TW, SEG>(I, flags, route, pos, rxy, inq, vis, ord, tl, W, Q, cnt,
                                     tk, init ? -1 : ant, SQ);
  int live = 0;
  if constexpr (SEG) {
    if (uniform_i(SQ.dirty)) seg_materialize<TW>(I, ant, SQ, tl, tk);
    live = uniform_i(SQ.live);
    if (lane == 0) I.sepoch[ant] = SQ.T.epoch;
  }
  if (TW > 1) {
    if (lane == 0) tl->op = OP_EXIT;
    team_sync();
  }
  if (init) {
    const int32_t *fr = (live ? I.r2 : I.routes) + (size_t)ant * (size_t)n;
    for (int i = lane; i < n; i += kWave) I.gb_route[i] = fr[i];
    if (lane == 0) {
      I.st->gb_len = len;
      I.st->init_len = len;
    }
    if (lane < NCNT) I.st->init_cnt[lane] = cnt.v;
    tk[4] = ticks() - t0;
    if (lane < kTicks) I.st->init_ticks[lane] = tk.v;
  } else {
    if (lane == 0) {
      I.lens[ant] = len;
      I.rsel[ant] = live;
    }
    if (lane < NCNT) {
      I.cnt[(size_t)ant * NCNT + lane] = cnt.v;
      I.cnt_acc[(size_t)ant * NCNT + lane] += cnt.v;
    }
    tk[4] = ticks() - t0;
    if (lane < kTicks) I.ticks[(size_t)ant * kTicks + lane] += tk.v;
  }
}

// One workgroup of TW waves per ant.
template <int KT, int TW, bool SEG = false>
__global__ void __launch_bounds__(64 * TW) ant_kernel(Inst I, int mode) {
  extern __shared__ uint32_t lds[];
  run_ant<KT, TW, SEG>(I, (int)blockIdx.x, mode, lds);
}

// ===================================================================== //
// Batched execution: one launch per phase covers every ant of every instance
// of a batch.  Each instance reads only its own Inst, so it evolves exactly as
// it would alone.
//   insts  Inst [count]
//   amap   int2 [total ants]: (instance, ant) of wave w = block * apb + wave
//          (TW > 1: of block w, whose TW waves form the ant's team)
// ===================================================================== //
template <int KT, int TW>
__global__ void __launch_bounds__(TW > 1 ? 64 * TW : 256)
    ant_batch_kernel(const Inst *insts, const int2 *amap, int total, int apb, int lds_words) {
  extern __shared__ uint32_t lds[];
  if (TW > 1) {
    // one workgroup of TW waves per ant
    const int2 m = amap[blockIdx.x];
    run_ant<KT, TW>(insts[m.x], m.y, 0, lds);
    return;
  }
  const int wave = (int)(threadIdx.x / kWave);
  const int w = (int)blockIdx.x * apb + wave;
  if (w >= total) return;
  const int2 m = amap[w];
  run_ant<KT, 1>(insts[m.x], m.y, 0, lds + (size_t)wave * (size_t)lds_words);
}

// ===================================================================== //
// Persistent batched execution.  One launch runs `iterations` iterations of
// every instance of a batch, and each instance advances on its own: the ants
// of its next iteration become available as soon as its own update is done,
// whatever the other instances are doing.  Per instance (BatchCtl):
//   ticket  ant tasks handed out in this launch (iteration e + 1 of the
//           launch owns tickets e A .. e A + A - 1)
//   done    ants of the current iteration that have finished
//   epoch   iterations completed (update included) in this launch
// Workers (a workgroup of TW waves when TW > 1, else each wave) take an ant
// task by compare-and-swap on a ticket of the current iteration, so no ant
// of iteration e + 2 can start before the update of iteration e + 1 is
// published.  The worker that finishes an instance's last ant runs the
// instance's update (colony, source, pheromone: the same functions as the
// per-phase kernels) and publishes the next epoch.  Workers leave once every
// instance has completed; a worker that sees no ant finish anywhere for
// kStallPolls polls records a stall fault in every unfinished instance and
// leaves, so no wait is unbounded.
// ===================================================================== //
constexpr int kStallPolls = 1 << 21;  // ~7 s of polls without any ant finishing

// An ant task of the current iteration of some instance, largest instances
// first (the host orders the table by tour length, descending).  The whole
// wave scans 64 instances at a time; the lanes of instances with tickets
// left try them in order, one at a time.  Uniform result.
FACO_DEV bool grab_task(BatchCtl *ctl, int count, int iters, int &inst, int &ant) {
  const int lane = lane_id();
  for (int base = 0; base < count; base += kWave) {
    const int i = base + lane;
    int e = 0;
    int64_t A = 0, t = 0;
    bool avail = false;
    if (i < count) {
      e = ld_agent(&ctl[i].epoch);
      if (e < iters) {
        A = ctl[i].ants;
        t = ld_agent64(&ctl[i].ticket);
        avail = t < ((int64_t)e + 1) * A;
      }
    }
    uint64_t m = ballot(avail);
    while (m) {
      const int l = ctz64(m);
      m &= m - 1;
      int won = 0, a = 0;
      if (lane == l) {
        const int64_t lim = ((int64_t)e + 1) * A;
        while (t < lim) {
          const int64_t seen = cas_agent64(&ctl[i].ticket, t, t + 1);
          if (seen == t) {
            won = 1;
            a = (int)(t - (int64_t)e * A);
            break;
          }
          t = seen;
        }
      }
      if (readlane_i(won, l)) {
        inst = base + l;
        ant = readlane_i(a, l);
        return true;
      }
    }
  }
  return false;
}

// After an ant: count it; true for the instance's last ant of the iteration.
// One lane.
FACO_DEV bool finish_ant(BatchCtl *ctl, BatchRun *run, int inst) {
  fence_release_agent();
  const int d = add_agent(&ctl[inst].done, 1) + 1;
  add_agent(&run->progress, 1);
  return d == ctl[inst].ants;
}

// After the update: publish the next epoch.  One lane.
FACO_DEV void publish_epoch(BatchCtl *ctl, BatchRun *run, int inst, int iters) {
  st_agent(&ctl[inst].done, 0);
  fence_release_agent();
  const int e = ld_agent(&ctl[inst].epoch) + 1;
  st_agent(&ctl[inst].epoch, e);
  if (e == iters) add_agent(&run->finished, 1);
}

// The update of one instance by the worker's NT threads (thread tid).
template <int TW>
FACO_DEV void worker_update(const Inst &I, int tid, int nt) {
  if (tid < kWave) run_colony(I);
  if (TW > 1) team_sync(); else wave_fence();
  for (int i = tid; i < I.n; i += nt) run_source(I, i, 0);
  if (TW > 1) team_sync(); else wave_fence();
  const size_t slots = (size_t)I.n * (size_t)I.k;
  for (size_t s = (size_t)tid; s < slots; s += (size_t)nt) run_pheromone(I, s, 0);
  if (TW > 1) team_sync(); else wave_fence();
}

FACO_DEV void mark_stall(const Inst *insts, BatchCtl *ctl, int count, int iters) {
  for (int i = 0; i < count; ++i)
    if (ld_agent(&ctl[i].epoch) < iters) atomicOr(&insts[i].st->fault, FAULT_BATCH_STALL);
}

template <int KT, int TW>
__global__ void __launch_bounds__(TW > 1 ? 64 * TW : 256)
    ant_persist_kernel(const Inst *insts, BatchCtl *ctl, BatchRun *run, int lds_words) {
  extern __shared__ uint32_t lds[];
  const int count = run->count, iters = run->iterations;
  const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
  int polls = 0, seen = -1;
  if (TW > 1) {
    // the workgroup is one worker; wave 0 takes the tasks
    TeamLds *tl = (TeamLds *)lds;
    for (;;) {
      if (w == 0) {
        int cmd = 2, inst = 0, ant = 0;  // 0 ant, 1 idle, 2 leave, 3 stalled
        if (uniform_i(ld_agent(&run->finished)) < count) {
          if (grab_task(ctl, count, iters, inst, ant)) {
            cmd = 0;
          } else {
            const int pr = uniform_i(ld_agent(&run->progress));
            if (pr != seen) {
              seen = pr;
              polls = 0;
            }
            cmd = ++polls > kStallPolls ? 3 : 1;
          }
        }
        if (lane == 0) {
          tl->disp[0] = cmd;
          tl->disp[1] = inst;
          tl->disp[2] = ant;
        }
      }
      team_sync();
      const int cmd = uniform_i(tl->disp[0]);
      const int inst = uniform_i(tl->disp[1]), ant = uniform_i(tl->disp[2]);
      team_sync();  // every wave has read the task before it is replaced
      if (cmd == 2) break;
      if (cmd == 3) {
        if (w == 0 && lane == 0) mark_stall(insts, ctl, count, iters);
        break;
      }
      if (cmd == 1) {
        __builtin_amdgcn_s_sleep(127);
        continue;
      }
      fence_acquire_agent();
      run_ant<KT, TW>(insts[inst], ant, 0, lds);
      team_sync();
      if (w == 0 && lane == 0) tl->disp[3] = finish_ant(ctl, run, inst) ? 1 : 0;
      team_sync();
      if (uniform_i(tl->disp[3])) {
        fence_acquire_agent();
        worker_update<TW>(insts[inst], (int)threadIdx.x, 64 * TW);
        if (w == 0 && lane == 0) publish_epoch(ctl, run, inst, iters);
      }
    }
  } else {
    // every wave is a worker with its own slice of LDS
    uint32_t *mine = lds + (size_t)w * (size_t)lds_words;
    for (;;) {
      int cmd = 2, inst = 0, ant = 0;  // 0 ant, 1 idle, 2 leave, 3 stalled
      if (uniform_i(ld_agent(&run->finished)) < count) {
        if (grab_task(ctl, count, iters, inst, ant)) {
          cmd = 0;
        } else {
          const int pr = uniform_i(ld_agent(&run->progress));
          if (pr != seen) {
            seen = pr;
            polls = 0;
          }
          cmd = ++polls > kStallPolls ? 3 : 1;
        }
      }
      cmd = uniform_i(cmd);
      inst = uniform_i(inst);
      ant = uniform_i(ant);
      if (cmd == 2) break;
      if (cmd == 3) {
        if (lane == 0) mark_stall(insts, ctl, count, iters);
        break;
      }
      if (cmd == 1) {
        __builtin_amdgcn_s_sleep(127);
        continue;
      }
      fence_acquire_agent();
      run_ant<KT, 1>(insts[inst], ant, 0, mine);
      int last = 0;
      if (lane == 0) last = finish_ant(ctl, run, inst) ? 1 : 0;
      if (readlane_i(last, 0)) {
        fence_acquire_agent();
        worker_update<1>(insts[inst], lane, kWave);
        if (lane == 0) publish_epoch(ctl, run, inst, iters);
      }
    }
  }
}

}  // namespace faco
