// faco_seg.hpp -- segment-list ant tours for the local search (included by
// faco_kernels.hpp after the move evaluation).
//
// Sec. 4.4 notes that a 2-opt flip on an array costs O(n) and the local
// search up to O(n^2) per ant.  Here, between materialisations, an ant's tour
// is its storage arrays (route, pos and tour-order coordinates of the last
// materialisation, read only) seen through segment records held in LDS.  A
// record is a storage range, its orientation and the array position of its
// first element; the records form a cyclic list in array order.  A move
// splits at most three records at its boundaries and rewrites the records
// inside its range (their positions, orientation and links); no element
// moves.  The array semantics stay exactly those of the flat tour: a city's
// position is its record's position plus its offset, so every position-
// dependent rule (which side a flip reverses, where an Or-opt block goes, the
// order of a tour's neighbours) is unchanged.  When the records run short the
// tour is written out in array order to the other storage buffer
// (materialised) and the records start again as fixed-length chunks.
//
// Record (int4): x = first storage index, y = last storage index, z = array
// position of the first element in array order, w = links and orientation
// (bits 0..14 previous record, 15..29 next record, bit 30 reversed: array
// order runs from y down to x).
//
// A city's record: its storage index s = P[c]; after a materialisation every
// city is in the chunk record s >> shift; a split gives part of a record a
// new record id, and the cities of that part carry it in G[c] = (epoch, id),
// valid only in the epoch it was written in (each materialisation and each
// local search starts a new epoch).  The helper waves write a move's labels
// after the move, while the leader evaluates the next one, so a label may
// still be missing: a lookup checks that the record's storage range holds
// s, and otherwise takes the record of the last move that does (ranges are
// disjoint, so the check is exact).
#pragma once

FACO_DEV int sg_prv(int w) { return w & (kSegCap - 1); }
FACO_DEV int sg_nxt(int w) { return (w >> 15) & (kSegCap - 1); }
FACO_DEV int sg_rev(int w) { return (w >> 30) & 1; }
FACO_DEV int sg_meta(int prv, int nxt, int rev) { return prv | (nxt << 15) | (rev << 30); }
FACO_DEV int sg_len(int4 r) { return r.y - r.x + 1; }
FACO_DEV int sg_off(int4 r, int s) { return sg_rev(r.w) ? r.y - s : s - r.x; }
FACO_DEV int sg_at(int4 r, int o) { return sg_rev(r.w) ? r.y - o : r.x + o; }
FACO_DEV int sg_pos(int4 r, int s, int n) {
  const int p = r.z + sg_off(r, s);
  return p >= n ? p - n : p;
}

// The live view of a segment-list tour.
struct SegT {
  int4 *rec;          // LDS records
  int32_t *R, *P;     // storage: city by storage index, storage index by city
  int2 *X;            // storage: coordinates by storage index
  int2 *G;            // (epoch, record) by city
  int epoch, shift, n;
  int lS0, lS;        // records made by the last move (labels maybe unwritten)
};

FACO_DEV SegT seg_view(const Inst &I, int ant, int4 *rec, int live, int epoch, int lS0 = 0,
                       int lS = 0) {
  const size_t o = (size_t)ant * (size_t)I.n;
  SegT T;
  T.rec = rec;
  T.R = (live ? I.r2 : I.routes) + o;
  T.P = (live ? I.p2 : I.pos) + o;
  T.X = (live ? I.x2 : I.rxy) + o;
  T.G = I.sgid + o;
  T.epoch = epoch;
  T.shift = I.seg_shift;
  T.n = I.n;
  T.lS0 = lS0;
  T.lS = lS;
  return T;
}

// The record holding storage index s, from the city's label gv; r its value.
FACO_DEV int sg_lookup(const SegT &T, int2 gv, int s, int4 &r) {
  int g = (gv.x == T.epoch ? gv.y : (s >> T.shift)) & (kSegCap - 1);
  r = T.rec[g];
  if (s < r.x || s > r.y) {
    for (int h = T.lS0; h < T.lS; ++h) {
      const int4 t = T.rec[h];
      if (t.x <= s && s <= t.y) {
        g = h;
        r = t;
      }
    }
  }
  return g;
}

// Storage index of the element d (|d| <= 3) places after the element at
// offset o of record g in array order; g and r follow to its record.  The
// bounds only matter for records that were corrupted.
constexpr int kWalkCap = 8;
FACO_DEV int sg_walk(const int4 *rec, int &g, int4 &r, int o, int d, int n) {
  o += d;
  if (o < 0 || o >= sg_len(r)) {
    for (int i = 0; i < kWalkCap && o < 0; ++i) {
      g = sg_prv(r.w);
      r = rec[g];
      o += sg_len(r);
    }
    for (int i = 0; i < kWalkCap && o >= sg_len(r); ++i) {
      o -= sg_len(r);
      g = sg_nxt(r.w);
      r = rec[g];
    }
    o = o < 0 ? 0 : (o >= sg_len(r) ? sg_len(r) - 1 : o);
  }
  const int s = sg_at(r, o);
  return s < 0 ? 0 : (s >= n ? n - 1 : s);
}

// Per-lane record data of a segment-list group evaluation: the group's city
// a, its neighbour nb (lanes 0..6 of the group), the candidate b, b's
// successor and predecessor.
struct SegEval {
  int ga, sa, gn, sn, gb, sb, gbs, sbs, gbp, sbp;
};

// eval_group on a segment-list tour: the same loads by position, resolved
// through the records (one LDS level after each city's storage index).
template <int GS>
FACO_DEV GroupEval eval_group_seg(const Inst &I, uint32_t flags, int a, bool gvalid,
                                  const SegT &T, SegEval &Z) {
  const int n = I.n, K = I.k, lane = lane_id();
  const int s = lane & (GS - 1);
  const bool act = gvalid && s < K;
  const size_t row = (size_t)a * (size_t)K;
  GroupEval R;
  R.a = a;
  // level 1: indexed by a
  const int sa = T.P[a];
  const int2 gva = T.G[a];
  const int b = act ? I.cl[row + s] : a;
  const int d_ab = act ? I.cl_d[row + s] : 0;
  const int2 xa = I.xy[a];
  int4 ra;
  const int ga = sg_lookup(T, gva, sa, ra);
  const int pa = sg_pos(ra, sa, n);
  const int oa = sg_off(ra, sa);
  // level 2: a's neighbourhood, b's storage index
  int gn = ga, sn = sa;
  int nb = a;
  int2 xnb = xa;
  if (s < 7) {
    int4 rn = ra;
    sn = sg_walk(T.rec, gn, rn, oa, s - 3, n);
    nb = T.R[sn];
    xnb = T.X[sn];
  }
  const int sb = T.P[b];
  const int2 gvb = T.G[b];
  const int2 xb = I.xy[b];
  int4 rb;
  const int gb = sg_lookup(T, gvb, sb, rb);
  const int pb = sg_pos(rb, sb, n);
  const int ob = sg_off(rb, sb);
  // level 3: b's tour neighbours
  int gbs = gb, gbp = gb;
  int4 rbs = rb, rbp = rb;
  const int sbs = sg_walk(T.rec, gbs, rbs, ob, 1, n);
  const int sbp = sg_walk(T.rec, gbp, rbp, ob, -1, n);
  const int bs = T.R[sbs], bp = T.R[sbp];
  const int2 xbs = T.X[sbs], xbp = T.X[sbp];
  const int pbs = pb + 1 == n ? 0 : pb + 1, pbp = pb == 0 ? n - 1 : pb - 1;
  R.pa = pa; R.b = b; R.pb = pb; R.pbs = pbs; R.pbp = pbp; R.bs = bs; R.bp = bp;
  R.nb = nb; R.xa = xa; R.xnb = xnb; R.xb = xb; R.xbs = xbs; R.xbp = xbp; R.d_ab = d_ab;
  Z.ga = ga; Z.sa = sa; Z.gn = gn; Z.sn = sn; Z.gb = gb; Z.sb = sb;
  Z.gbs = gbs; Z.sbs = sbs; Z.gbp = gbp; Z.sbp = sbp;
  group_keys<GS>(flags, act, R);
  return R;
}

// Record and storage index of split city i of a move (uniform).
// (Values, not references, are selected: a conditional between two fields
// would select their addresses and keep the struct out of registers.)
FACO_DEV void seg_split_city(const SegEval &Z, const Move &mv, int i, int &g, int &s) {
  const int k = mv.lk[i];
  const int ga = Z.ga, sa = Z.sa, gn = Z.gn, sn = Z.sn;
  const int gb = Z.gb, sb = Z.sb, gbs = Z.gbs, sbs = Z.sbs;
  const int gl = k == SL_A ? ga : (k == SL_NB ? gn : (k == SL_B ? gb : gbs));
  const int sl = k == SL_A ? sa : (k == SL_NB ? sn : (k == SL_B ? sb : sbs));
  g = readlane_i(gl, mv.ln[i]);
  s = readlane_i(sl, mv.ln[i]);
}

// The storage indices of positions p-3 .. p+3 around the element at offset o
// of record g (p its position), for one lane.
FACO_DEV void sg_nbhd7(const int4 *rec, int g, int4 r, int o, int n, int *sx) {
  sx[3] = sg_at(r, o);
  int gl = g, ol = o;
  int4 rl = r;
#pragma unroll
  for (int k = 1; k <= 3; ++k) {
    if (--ol < 0) {
      gl = sg_prv(rl.w);
      rl = rec[gl];
      ol = sg_len(rl) - 1;
    }
    sx[3 - k] = sg_at(rl, ol);
  }
  int gr = g, orr = o;
  int4 rr = r;
#pragma unroll
  for (int k = 1; k <= 3; ++k) {
    if (++orr >= sg_len(rr)) {
      gr = sg_nxt(rr.w);
      rr = rec[gr];
      orr = 0;
    }
    sx[3 + k] = sg_at(rr, orr);
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) sx[k] = sx[k] < 0 ? 0 : (sx[k] >= n ? n - 1 : sx[k]);
}

// has_improving on a segment-list tour (the sweep's test, one city per lane).
template <int KT>
FACO_DEV bool has_improving(const Inst &I, uint32_t flags, int x, const SegT &T) {
  constexpr int CK = KT < FACO_SWEEP_CK ? KT : FACO_SWEEP_CK;
  const int n = I.n, K = I.k;
  const size_t row = (size_t)x * (size_t)K;
  int cb[CK], cd[CK];
#pragma unroll
  for (int j = 0; j < CK; ++j) {
    cb[j] = j < K ? I.cl[row + j] : x;
    cd[j] = j < K ? I.cl_d[row + j] : 0x7fffffff;
  }
  const int sx0 = T.P[x];
  const int2 gvx = T.G[x];
  const int2 cx = I.xy[x];
  int4 rx;
  const int gx = sg_lookup(T, gvx, sx0, rx);
  const int px = sg_pos(rx, sx0, n);
  int sxn[7];
  sg_nbhd7(T.rec, gx, rx, sg_off(rx, sx0), n, sxn);
  int xnx[7], xny[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) {
    const int2 q = T.X[sxn[j]];
    xnx[j] = q.x; xny[j] = q.y;
  }
#define XN(j) make_int2(xnx[j], xny[j])
  const bool two = (flags & LS_2OPT) != 0, orr = (flags & LS_OROPT) != 0;
  const int d_s = cost(cx, XN(4)), d_p = cost(XN(2), cx);
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
    int pb[CK], xbx[CK], xby[CK], sx[CK], sy[CK], qx[CK], qy[CK];
    int bsb[CK];
    int2 gvb[CK];
#pragma unroll
    for (int j = 0; j < CK; ++j) {
      bsb[j] = T.P[cb[j]];
      gvb[j] = T.G[cb[j]];
      const int2 q = I.xy[cb[j]];
      xbx[j] = q.x; xby[j] = q.y;
    }
#pragma unroll
    for (int j = 0; j < CK; ++j) {
      int4 r;
      const int g = sg_lookup(T, gvb[j], bsb[j], r);
      pb[j] = sg_pos(r, bsb[j], n);
      const int o = sg_off(r, bsb[j]);
      int g1 = g, g2 = g;
      int4 r1 = r, r2 = r;
      const int2 q1 = T.X[sg_walk(T.rec, g1, r1, o, 1, n)];
      const int2 q2 = T.X[sg_walk(T.rec, g2, r2, o, -1, n)];
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

// ----------------------------------------------------------- records ---

// Records of a fresh epoch: chunk g = storage [g << shift, ...) at array
// position g << shift (storage = array order).  Wave w of TW, lanes in turn.
FACO_DEV void seg_reset_part(int4 *rec, int tid, int nt, int S, int n, int shift) {
  for (int g = tid; g < S; g += nt) {
    const int lo = g << shift;
    const int hi = ((g + 1) << shift) < n ? ((g + 1) << shift) - 1 : n - 1;
    rec[g] = make_int4(lo, hi, lo, sg_meta(g == 0 ? S - 1 : g - 1, g + 1 == S ? 0 : g + 1, 0));
  }
}

// 1: helper waves label a move's cities after the move (lookups check the
// label against the record's storage range); 0: before the move ends.
#ifndef FACO_SEG_DEFER
#define FACO_SEG_DEFER 1
#endif

// Link overrides (record, field, value) packed in one int: record bits
// 0..10, field bit 11 (0 previous, 1 next), value bits 12..22.
constexpr int kSovPre = 3, kSovPost = 6;
static_assert(sizeof(((TeamLds *)nullptr)->sov) == sizeof(int) * (kSovPre + kSovPost),
              "override table size");
FACO_DEV int sov_pack(int g, int f, int v) { return g | (f << 11) | (v << 12); }
FACO_DEV int sg_set_link(int w, int f, int v) {
  return f ? (w & ~((kSegCap - 1) << 15)) | (v << 15) : (w & ~(kSegCap - 1)) | v;
}

// A move's share of thread tid of nt: every record of 0 .. S-1 takes the
// link overrides made by the move's splits, then, if it lies inside the
// cyclic range [ps, ps + len), its new place: the range's first block (la
// elements) and its second block exchange places, revA / revB reversing the
// first / second block (a reversal alone: la = len with revA); then the
// overrides that relink the range's ends.
struct SegOv {
  int v[kSovPre + kSovPost];  // kSovPre before the transform, then kSovPost after
};
FACO_DEV void seg_perm_part(const SegT &T, int tid, int nt, int S, int ps, int la, int len,
                            int revA, int revB, const SegOv &O, int npre, int npost) {
  const int n = T.n;
  const int *ov = O.v;
  for (int g = tid; g < S; g += nt) {
    int4 r = T.rec[g];
#pragma unroll
    for (int j = 0; j < kSovPre; ++j)
      if (j < npre && (ov[j] & (kSegCap - 1)) == g)
        r.w = sg_set_link(r.w, (ov[j] >> 11) & 1, ov[j] >> 12);
    int u = r.z - ps;
    u = u < 0 ? u + n : u;
    if (u < len) {
      const int sl = sg_len(r);
      int u2;
      bool flip;
      if (u < la) {
        flip = revA != 0;
        u2 = (len - la) + (flip ? la - u - sl : u);
      } else {
        flip = revB != 0;
        const int v = u - la;
        u2 = flip ? (len - la) - v - sl : v;
      }
      if (flip) r.w = sg_meta(sg_nxt(r.w), sg_prv(r.w), sg_rev(r.w) ^ 1);
      const int p = ps + u2;
      r.z = p >= n ? p - n : p;
    }
#pragma unroll
    for (int j = 0; j < kSovPost; ++j) {
      const int o = ov[kSovPre + j];
      if (j < npost && (o & (kSegCap - 1)) == g) r.w = sg_set_link(r.w, (o >> 11) & 1, o >> 12);
    }
    T.rec[g] = r;
  }
}

// Label the cities of storage range [lo, hi] with record h (one wave).
FACO_DEV void seg_relabel(const SegT &T, int lo, int hi, int h) {
  const int n = T.n;
  lo = lo < 0 ? 0 : lo;
  hi = hi >= n ? n - 1 : hi;
  for (int s = lo + lane_id(); s <= hi; s += kWave) {
    const int c = T.R[s];
    if ((unsigned)c < (unsigned)n) T.G[c] = make_int2(T.epoch, h);
  }
}

// The records a move reads (its boundary cities' records) or makes, one per
// lane of the leader wave (lane j < cnt holds entry j: record id and value),
// and the links it changes in other records (lane j < npre holds override
// j).  Finding an entry is a ballot; changing one is a select in its lane.
constexpr int kMvTab = 6;
struct SegMv {
  int id, x, y, z, w;  // this lane's entry
  int cnt;             // entries (uniform)
  int pre;             // this lane's override
  int npre;            // overrides (uniform)
};
FACO_DEV void mv_init(SegMv &M) {
  M.id = -1;
  M.x = 0;
  M.y = -1;
  M.z = M.w = 0;
  M.cnt = 0;
  M.pre = 0;
  M.npre = 0;
}
FACO_DEV int mv_index(const SegMv &M, int g) {
  const uint64_t b = ballot(lane_id() < M.cnt && M.id == g);
  return b ? ctz64(b) : -1;
}
// the entry whose storage range holds s
FACO_DEV int mv_find(const SegMv &M, int s) {
  const uint64_t b = ballot(lane_id() < M.cnt && M.x <= s && s <= M.y);
  return b ? ctz64(b) : 0;
}
FACO_DEV int mv_id(const SegMv &M, int k) { return readlane_i(M.id, k); }
FACO_DEV int4 mv_val(const SegMv &M, int k) {
  return make_int4(readlane_i(M.x, k), readlane_i(M.y, k), readlane_i(M.z, k),
                   readlane_i(M.w, k));
}
// entry k := r
FACO_DEV void mv_put(SegMv &M, int k, int4 r) {
  const bool me = lane_id() == k;
  M.x = me ? r.x : M.x;
  M.y = me ? r.y : M.y;
  M.z = me ? r.z : M.z;
  M.w = me ? r.w : M.w;
}
// a new entry (g, r)
FACO_DEV void mv_add(SegMv &M, int g, int4 r) {
  const bool me = lane_id() == M.cnt;
  M.id = me ? g : M.id;
  M.x = me ? r.x : M.x;
  M.y = me ? r.y : M.y;
  M.z = me ? r.z : M.z;
  M.w = me ? r.w : M.w;
  M.cnt++;
}
// set link f of record g to v: in its entry, else as an override
FACO_DEV void mv_link(SegMv &M, int g, int f, int v) {
  const int k = mv_index(M, g);
  if (k >= 0) {
    const int w = sg_set_link(readlane_i(M.w, k), f, v);
    M.w = lane_id() == k ? w : M.w;
  } else {
    M.pre = lane_id() == M.npre ? sov_pack(g, f, v) : M.pre;
    M.npre++;
  }
}

// Make the element at storage index s the first of its record in array
// order (nothing to do if it is): the smaller part becomes record S (S grows
// by one).  Uniform control flow.
FACO_DEV void mv_split(SegMv &M, int &S, int s, int n) {
  const int k = mv_find(M, s);
  const int g = mv_id(M, k);
  const int4 r = mv_val(M, k);
  const int rv = sg_rev(r.w);
  const int o = rv ? r.y - s : s - r.x;
  if (o <= 0) return;
  const int len = sg_len(r);
  const int q = r.z + o >= n ? r.z + o - n : r.z + o;
  // part 1: the first o elements in array order, part 2: the rest
  const int p1lo = rv ? s + 1 : r.x, p1hi = rv ? r.y : s - 1;
  const int p2lo = rv ? r.x : s, p2hi = rv ? s : r.y;
  const int h = S++;
  const int nx = sg_nxt(r.w), pv = sg_prv(r.w);
  if (len - o <= o) {
    // h = part 2, after g
    mv_put(M, k, make_int4(p1lo, p1hi, r.z, sg_meta(pv, h, rv)));
    mv_add(M, h, make_int4(p2lo, p2hi, q, sg_meta(g, nx, rv)));
    mv_link(M, nx, 0, h);
  } else {
    // h = part 1, before g
    mv_put(M, k, make_int4(p2lo, p2hi, q, sg_meta(h, nx, rv)));
    mv_add(M, h, make_int4(p1lo, p1hi, r.z, sg_meta(pv, g, rv)));
    mv_link(M, pv, 1, h);
  }
}

// Write the tour out in array order to the other storage buffer: element at
// storage index s goes to its array position.  Thread tid of nt.
FACO_DEV void seg_mat_part(const SegT &T, int tid, int nt, int32_t *Rd, int2 *Xd, int32_t *Pd) {
  constexpr int U = 8;
  const int n = T.n;
  for (int b0 = tid; b0 < n; b0 += U * nt) {
    int c[U];
    int2 x[U], gv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = b0 + u * nt;
      if (s < n) {
        c[u] = T.R[s];
        x[u] = T.X[s];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = b0 + u * nt;
      if (s < n) gv[u] = T.G[c[u] < 0 ? 0 : (c[u] >= n ? n - 1 : c[u])];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int s = b0 + u * nt;
      if (s < n) {
        int4 r;
        sg_lookup(T, gv[u], s, r);
        int p = sg_pos(r, s, n);
        p = p < 0 ? 0 : (p >= n ? n - 1 : p);
        const int cc = c[u] < 0 ? 0 : (c[u] >= n ? n - 1 : c[u]);
        Rd[p] = cc;
        Xd[p] = x[u];
        Pd[cc] = p;
      }
    }
  }
}

// ------------------------------------------------------------ leader ---

// Leader-side state of an ant's segment-list tour.
struct SegState {
  SegT T;
  int S;        // records in use
  int S_init;   // records of a fresh epoch
  int live;     // storage buffer in use (0: routes/pos/rxy, 1: r2/p2/x2)
  int dirty;    // a move since the last materialisation
};

// Tick and count slots of the segment-list tour (per ant).
enum { TK_SEG_MATS = 16, TK_SEG_MAT_TICKS = 17, TK_SEG_RELABELLED = 18, TK_SEG_SPLITS = 19,
       TK_SEG_RECORDS = 20, TK_SEG_LEADER = 21, TK_SEG_TEAM = 22 };

FACO_DEV void seg_begin(const Inst &I, int ant, int4 *rec, TeamLds *tl, int team,
                        SegState &Q) {
  const int n = I.n, lane = lane_id();
  Q.S_init = (n + (1 << I.seg_shift) - 1) >> I.seg_shift;
  Q.S = Q.S_init;
  Q.live = 0;
  Q.dirty = 0;
  const int ep = uniform_i(I.sepoch[ant]) + 1;
  Q.T = seg_view(I, ant, rec, 0, ep);
  seg_reset_part(rec, lane, kWave, Q.S_init, n, I.seg_shift);
  if (team && lane == 0) {
    tl->sgs[0] = 0;
    tl->sgs[1] = ep;
    tl->sgs[2] = 0;
    tl->sgs[3] = 0;
  }
  wave_fence();
}

// Materialise: the tour in array order goes to the other storage buffer,
// which becomes the live one; records restart as chunks in a new epoch.
template <int TW>
FACO_DEV void seg_materialize(const Inst &I, int ant, SegState &Q, TeamLds *tl,
                              LaneCounters &tk) {
  const int64_t t0 = fine_ticks();
  const int n = I.n, lane = lane_id();
  const size_t o = (size_t)ant * (size_t)n;
  const int dl = Q.live ^ 1;
  int32_t *Rd = (dl ? I.r2 : I.routes) + o;
  int2 *Xd = (dl ? I.x2 : I.rxy) + o;
  int32_t *Pd = (dl ? I.p2 : I.pos) + o;
  if (TW > 1) {
    team_post(tl, OP_SEGMAT, Q.S);
    seg_mat_part(Q.T, lane, kWave * TW, Rd, Xd, Pd);
    team_sync();
    seg_reset_part(Q.T.rec, lane, kWave * TW, Q.S_init, n, I.seg_shift);
    team_sync();
  } else {
    seg_mat_part(Q.T, lane, kWave, Rd, Xd, Pd);
    wave_fence();
    seg_reset_part(Q.T.rec, lane, kWave, Q.S_init, n, I.seg_shift);
    wave_fence();
  }
  Q.live = dl;
  Q.T = seg_view(I, ant, Q.T.rec, dl, Q.T.epoch + 1);
  if (TW > 1 && lane == 0) {
    tl->sgs[0] = Q.live;
    tl->sgs[1] = Q.T.epoch;
    tl->sgs[2] = 0;
    tl->sgs[3] = 0;
  }
  Q.S = Q.S_init;
  Q.dirty = 0;
  tk[TK_SEG_MATS]++;
  tk[TK_SEG_MAT_TICKS] += fine_ticks() - t0;
}

// A move on the segment list.  NP (2 or 3) boundary cities, record pg[i] and
// storage index psx[i], in order: the range's first element, the second
// block's first element (NP = 3), the element after the range.  The leader
// reads their records once, splits at the cities in registers, writes the
// changed and new records, and the team places every record (the blocks of
// [ps, ps + len) exchange places, revA / revB reversing them) and relinks
// the range's ends; the helpers label the cities of the new records after.
template <int TW, int NP>
FACO_DEV void seg_permute(const Inst &I, SegState &Q, TeamLds *tl, const int *pg,
                          const int *psx, int ps, int la, int len, int revA, int revB,
                          LaneCounters &tk) {
  const int64_t t0 = fine_ticks();
  int4 *rec = Q.T.rec;
  const int n = I.n, lane = lane_id();
  SegMv M;
  mv_init(M);
  int4 r0[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) r0[i] = rec[pg[i]];
#pragma unroll
  for (int i = 0; i < NP; ++i)
    if (mv_index(M, pg[i]) < 0) mv_add(M, pg[i], r0[i]);
  const int S0 = Q.S;
  int S = S0;
#pragma unroll
  for (int i = 0; i < NP; ++i) mv_split(M, S, psx[i], n);
  const int kA = mv_find(M, psx[0]);
  const int kB = mv_find(M, psx[NP == 3 ? 1 : 0]);
  const int kE = mv_find(M, psx[NP - 1]);
  const int Af = mv_id(M, kA), Bf = mv_id(M, kB), E = mv_id(M, kE);
  const int P0 = sg_prv(mv_val(M, kA).w);
  const int Al = sg_prv(mv_val(M, NP == 3 ? kB : kE).w);
  const int Bl = sg_prv(mv_val(M, kE).w);
  const int Xf = revA ? Al : Af, Xl = revA ? Af : Al;
  int post[kSovPost];
  int npost;
  if (NP == 3) {
    const int Yf = revB ? Bl : Bf, Yl = revB ? Bf : Bl;
    post[0] = sov_pack(P0, 1, Yf);
    post[1] = sov_pack(Yf, 0, P0);
    post[2] = sov_pack(Yl, 1, Xf);
    post[3] = sov_pack(Xf, 0, Yl);
    post[4] = sov_pack(Xl, 1, E);
    post[5] = sov_pack(E, 0, Xl);
    npost = 6;
  } else {
    post[0] = sov_pack(P0, 1, Xf);
    post[1] = sov_pack(Xf, 0, P0);
    post[2] = sov_pack(Xl, 1, E);
    post[3] = sov_pack(E, 0, Xl);
    post[4] = post[5] = 0;
    npost = 4;
  }
  const bool mine = lane < M.cnt;
  const int relab = wave_sum_i32((mine && M.id >= S0) ? M.y - M.x + 1 : 0);
  SegOv O;
#pragma unroll
  for (int j = 0; j < kSovPre; ++j) O.v[j] = readlane_i(M.pre, j);
#pragma unroll
  for (int j = 0; j < kSovPost; ++j) O.v[kSovPre + j] = post[j];
  // each lane writes its entry
  if (mine) rec[M.id] = make_int4(M.x, M.y, M.z, M.w);
  if (TW > 1) {
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < kSovPre + kSovPost; ++j) tl->sov[j] = O.v[j];
      tl->arg[5] = revA | (revB << 1);
      tl->arg[6] = M.npre;
      tl->arg[7] = npost;
    }
    const int64_t t1 = fine_ticks();
    tk[TK_SEG_LEADER] += t1 - t0;
    team_post(tl, OP_SEGPERM, S0, S, ps, la, len);
    seg_perm_part(Q.T, lane, kWave * TW, S, ps, la, len, revA, revB, O, M.npre, npost);
    team_sync();
    tk[TK_SEG_TEAM] += fine_ticks() - t1;
  } else {
    wave_lds_sync();
    seg_perm_part(Q.T, lane, kWave, S, ps, la, len, revA, revB, O, M.npre, npost);
    wave_lds_sync();
    for (int h = S0; h < S; ++h) {
      const int4 r = rec[h];
      seg_relabel(Q.T, r.x, r.y, h);
    }
  }
  tk[TK_SEG_SPLITS] += S - S0;
  tk[TK_SEG_RELABELLED] += relab;
  tk[TK_SEG_RECORDS] += S;
  Q.S = S;
  Q.T.lS0 = S0;
  Q.T.lS = S;
  if (TW > 1 && lane == 0) {
    tl->sgs[2] = S0;
    tl->sgs[3] = S;
  }
  Q.dirty = 1;
}

// The flips of apply_2opt on the segment list (same side choice).
template <int TW>
FACO_DEV int seg_apply_2opt(const Inst &I, SegState &Q, TeamLds *tl, const Move &mv,
                            const SegEval &Z, LaneCounters &tk) {
  const int n = I.n;
  const int px = uniform_i(mv.px), py = uniform_i(mv.py), pz = uniform_i(mv.pz);
  int gx, sx, gz, sz;
  seg_split_city(Z, mv, 0, gx, sx);
  seg_split_city(Z, mv, 1, gz, sz);
  const int L1 = wrapn(py - px, n) + 1;
  if (2 * L1 <= n) {
    const int pg[2] = {gx, gz}, ps[2] = {sx, sz};
    seg_permute<TW, 2>(I, Q, tl, pg, ps, px, L1, L1, 1, 0, tk);
    return L1;
  }
  const int pg[2] = {gz, gx}, ps[2] = {sz, sx};
  seg_permute<TW, 2>(I, Q, tl, pg, ps, pz, n - L1, n - L1, 1, 0, tk);
  return n - L1;
}

// The block exchange of apply_oropt on the segment list (same block choice).
template <int TW>
FACO_DEV int seg_apply_oropt(const Inst &I, SegState &Q, TeamLds *tl, const Move &mv,
                             const SegEval &Z, LaneCounters &tk) {
  const int n = I.n;
  const int L = uniform_i(mv.L), side = uniform_i(mv.side), pb = uniform_i(mv.pb);
  const int fpos = uniform_i(mv.fpos), pq = uniform_i(mv.pq), pp = uniform_i(mv.pp);
  const int a = uniform_i(mv.a), f = uniform_i(mv.f), b = uniform_i(mv.b);
  const int e = uniform_i(mv.e);
  int g0, s0, gq, sq, g2, s2;
  seg_split_city(Z, mv, 0, g0, s0);
  seg_split_city(Z, mv, 1, gq, sq);
  seg_split_city(Z, mv, 2, g2, s2);
  const int x1 = side == 0 ? b : e;
  const int px1 = side == 0 ? pb : (pb == 0 ? n - 1 : pb - 1);
  const int px2 = side == 0 ? (pb + 1 == n ? 0 : pb + 1) : pb;
  const int rev = ((a != f) != (x1 != b)) ? 1 : 0;
  const int D1 = wrapn(px1 - pq, n) + 1;
  const int D2 = wrapn(pp - px2, n) + 1;
  if (D1 <= D2) {
    const int pg[3] = {g0, gq, g2}, ps[3] = {s0, sq, s2};
    seg_permute<TW, 3>(I, Q, tl, pg, ps, fpos, L, L + D1, rev, 0, tk);
    return D1 + L;
  }
  const int pg[3] = {g2, g0, gq}, ps[3] = {s2, s0, sq};
  seg_permute<TW, 3>(I, Q, tl, pg, ps, px2, D2, D2 + L, 0, rev, tk);
  return D2 + L;
}
