// faco_api.hip -- host side of the C ABI declared in include/faco.h.
//
// Owns the device state of each instance, validates arguments, launches the
// kernels on the instance's stream.  No step of the
// method runs on the host: the host only derives p_best^(1/n) once per build
// (a parameter of the trail-limit formula, Sec. 4.5) and marshals pointers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/faco.h"
#include "ant_kernels.hpp"
#include "faco_aux.hpp"
#include "faco_init.hpp"

using faco::DevState;
using faco::Inst;

struct TimedLaunch {
  int phase;
  hipEvent_t a, b;
};

struct faco_instance {
  faco_params p{};
  int32_t n = 0, k = 0, bl = 0;
  hipStream_t stream = nullptr;
  Inst dv{};
  std::vector<std::pair<void *, size_t>> allocs;  // device blocks and their sizes
  std::string err;
  size_t lds_ant = 0;   // LDS of the per-iteration ant kernel
  size_t lds_init = 0;  // LDS of the initial solution's ant kernel (flat tour)
  int tw = 1;  // waves per ant in the per-instance ant kernel
  int device = 0;  // the device current at build
  std::vector<int32_t> orig_of, int_of;  // internal label <-> original city number
  std::vector<int32_t> xy_host;          // the build's coordinates (autotuner twins)
  bool timing = false;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> ev_pool;  // timing events, created once and reused
  double phase_ms[4] = {0, 0, 0, 0};
  int64_t phase_n[4] = {0, 0, 0, 0};
};

static thread_local std::string g_err;

static int set_err(faco_instance *h, int code, const std::string &msg) {
  if (h)
    h->err = msg;
  else
    g_err = msg;
  return code;
}

#define HIP_TRY(h, expr)                                                        \
  do {                                                                          \
    hipError_t _e = (expr);                                                     \
    if (_e != hipSuccess)                                                       \
      return set_err(h, FACO_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
  } while (0)

static const char *validate(const faco_params *p, int32_t n) {
  if (!p) return "params is NULL";
  if (n < 4) return "n must be at least 4";
  if (n > (1 << 18)) return "n must be at most 262144";
  if (p->cl_size < 2 || p->cl_size > faco::kMaxCl) return "cl_size must be in [2, 32]";
  if (p->bl_size < 0 || p->bl_size > faco::kMaxBl) return "bl_size must be in [0, 64]";
  if (p->n_ants < 1 || p->n_ants > 4096) return "n_ants must be in [1, 4096]";
  if (p->min_new_edges < 0) return "min_new_edges must be >= 0";
  if (p->min_new_edges_max < 0 ||
      (p->min_new_edges_max > 0 && p->min_new_edges_max < p->min_new_edges))
    return "min_new_edges_max must be 0 or >= min_new_edges";
  if (p->reserved1 != 0) return "reserved1 must be 0";
  if (!(p->rho >= 0.0f) || !(p->rho < 1.0f)) return "rho must be in [0, 1)";
  if (p->reserved0 != 0.0f) return "reserved0 must be 0";
  if (!(p->p_best > 0.0) || !(p->p_best < 1.0)) return "p_best must be in (0, 1)";
  if (!(p->p_source_gbest >= 0.0) || !(p->p_source_gbest <= 1.0))
    return "p_source_gbest must be in [0, 1]";
  if (p->ls_flags & ~15u) return "unknown ls_flags bits";
  if (p->oropt_max_seg < 1 || p->oropt_max_seg > faco::kMaxOrSeg)
    return "oropt_max_seg must be in [1, 3]";
  return nullptr;
}

static void effective_sizes(int32_t n, const faco_params *p, int32_t *k, int32_t *bl) {
  *k = p->cl_size < n - 1 ? p->cl_size : n - 1;
  *bl = p->bl_size < n - 1 - *k ? p->bl_size : n - 1 - *k;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }


// Held while a batch graph is being captured, and around device allocation
// and release, which may synchronise implicitly and must not meet a capture
// in progress on another thread.
static std::mutex g_capture_mu;

// Device blocks released by destroyed instances and outgrown batch tables,
// kept per device for later allocations.  hipFree waits for all work queued
// on the device: in a serving loop every retirement would stall the other
// streams' solves and leave the GPU idle while it drained.  A block enters
// the cache only once no queued work can still touch it; sizes are rounded
// to eighths of their leading power of two so that blocks fit later requests
// of similar size.
static std::mutex g_blk_mu;
static std::map<int, std::multimap<size_t, void *>> g_blk_free;
static size_t g_blk_cached = 0;
static const size_t kBlkCacheLimit = (size_t)32 << 30;

static size_t blk_round(size_t b) {
  if (b <= 256) return 256;
  const int e = 63 - __builtin_clzll((unsigned long long)b);
  const size_t step = (size_t)1 << (e - 3);
  return (b + step - 1) / step * step;
}

// Free every cached block of `dev` (waits for the device's queued work).
static void blk_trim(int dev) {
  std::vector<void *> out;
  {
    std::lock_guard<std::mutex> lk(g_blk_mu);
    auto &m = g_blk_free[dev];
    for (auto &kv : m) {
      out.push_back(kv.second);
      g_blk_cached -= kv.first;
    }
    m.clear();
  }
  std::lock_guard<std::mutex> lk(g_capture_mu);
  for (void *q : out) (void)hipFree(q);
}

// A block of at least `bytes` on the current device `dev`: a cached one of
// at most 5/4 the rounded size, else a new allocation (after one trim of the
// cache if the device is out of memory).  *got receives the block's size.
static hipError_t blk_get(int dev, size_t bytes, void **ptr, size_t *got) {
  const size_t want = blk_round(bytes);
  {
    std::lock_guard<std::mutex> lk(g_blk_mu);
    auto &m = g_blk_free[dev];
    auto it = m.lower_bound(want);
    if (it != m.end() && it->first <= want + want / 4) {
      *ptr = it->second;
      *got = it->first;
      g_blk_cached -= it->first;
      m.erase(it);
      return hipSuccess;
    }
  }
  hipError_t e;
  {
    std::lock_guard<std::mutex> lk(g_capture_mu);
    e = hipMalloc(ptr, want);
  }
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    blk_trim(dev);
    std::lock_guard<std::mutex> lk(g_capture_mu);
    e = hipMalloc(ptr, want);
  }
  if (e != hipSuccess) {
    *ptr = nullptr;
    return e;
  }
  *got = want;
  return hipSuccess;
}

// Return a block that no queued work uses any more; beyond the cache's limit
// it is freed instead.
static void blk_put(int dev, void *p, size_t bytes) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_blk_mu);
    if (g_blk_cached + bytes <= kBlkCacheLimit) {
      g_blk_free[dev].emplace(bytes, p);
      g_blk_cached += bytes;
      return;
    }
  }
  std::lock_guard<std::mutex> lk(g_capture_mu);
  (void)hipFree(p);
}

static int dalloc(faco_instance *h, void **ptr, size_t bytes) {
  size_t got = 0;
  const hipError_t e = blk_get(h->device, bytes ? bytes : 4, ptr, &got);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return set_err(h, FACO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  h->allocs.emplace_back(*ptr, got);
  return FACO_OK;
}

static size_t knn_lds_bytes(int K, int BL) {
  return (sizeof(double) + sizeof(int32_t)) * (size_t)(K + BL) * 64;
}

static hipEvent_t take_event(faco_instance *h) {
  hipEvent_t e = nullptr;
  if (!h->ev_pool.empty()) {
    e = h->ev_pool.back();
    h->ev_pool.pop_back();
  } else {
    (void)hipEventCreate(&e);
  }
  return e;
}
static void begin_timed(faco_instance *h, int phase, TimedLaunch &tl) {
  tl.phase = phase;
  tl.a = take_event(h);
  tl.b = take_event(h);
  (void)hipEventRecord(tl.a, h->stream);
}
static void end_timed(faco_instance *h, TimedLaunch &tl) {
  (void)hipEventRecord(tl.b, h->stream);
  h->pending.push_back(tl);
}

// Waves per ant for instances built from now on (0 = by size: large tours
// with few enough ants to leave the chip's wave slots to the teams).
static std::mutex g_team_mu;
static int g_team_waves = 0;

extern "C" int faco_set_team_waves(int32_t tw) {
  if (tw != 0 && tw != 1 && tw != 4 && tw != 8)
    return set_err(nullptr, FACO_EINVAL, "team waves must be 0, 1, 4 or 8");
  std::lock_guard<std::mutex> lk(g_team_mu);
  g_team_waves = tw;
  return FACO_OK;
}

// LDS capacity of an ant's work queue for instances built from now on.
static int g_queue_lds_cap = faco::kLdsRingMax;

extern "C" int faco_set_queue_lds_capacity(int32_t cap) {
  if (cap != 0 && (cap < 64 || cap > faco::kLdsRingMax))
    return set_err(nullptr, FACO_EINVAL, "queue LDS capacity must be 0 or in [64, 16384]");
  std::lock_guard<std::mutex> lk(g_team_mu);
  g_queue_lds_cap = cap ? cap : faco::kLdsRingMax;
  return FACO_OK;
}

// The queue ring takes what LDS is left next to the team area and three
// n-bit bitmaps (160 KB per CU).
static int queue_lds_cap_for(int32_t n, int extra_words = 0) {
  int cap;
  {
    std::lock_guard<std::mutex> lk(g_team_mu);
    cap = n < g_queue_lds_cap ? n : g_queue_lds_cap;
  }
  const int room = 160 * 1024 / 4 - faco_team_lds_words(8) - 3 * ((n + 31) / 32) - 4 -
                   extra_words;
  return cap < room ? cap : room;
}

static int team_waves_for(int32_t n, int32_t ants) {
  int tw;
  {
    std::lock_guard<std::mutex> lk(g_team_mu);
    tw = g_team_waves;
  }
  if (tw) return tw;
  if (n < 2048) return 1;
  if (ants <= 256) return 8;
  if (ants <= 512) return 4;
  return 1;
}

// Segment-list ant tours: 0 and 1 flat arrays (the default: on this GPU a
// segment-list move costs as much as a flat rewrite of a typical move, and
// every evaluation pays the record lookups), 2 segment lists; segment length
// 2^g_seg_log2 (0: by size); records in use that trigger a materialisation
// (0: the table's capacity).
static int g_seg_mode = 0, g_seg_log2 = 0, g_seg_max = 0;

extern "C" int faco_set_tour_segments(int32_t mode, int32_t length_log2,
                                      int32_t max_records) {
  if (mode < 0 || mode > 2)
    return set_err(nullptr, FACO_EINVAL, "tour segment mode must be 0, 1 or 2");
  if (length_log2 < 0 || length_log2 > 24)
    return set_err(nullptr, FACO_EINVAL, "segment length log2 must be in [0, 24]");
  if (max_records != 0 && (max_records < 8 || max_records > faco::kSegCap))
    return set_err(nullptr, FACO_EINVAL, "segment records must be 0 or in [8, 2048]");
  std::lock_guard<std::mutex> lk(g_team_mu);
  g_seg_mode = mode;
  g_seg_log2 = length_log2;
  g_seg_max = max_records;
  return FACO_OK;
}

struct SegPlan {
  int on = 0, shift = 0, max = 0;
};

// Whether an instance of n cities whose ants have tw waves runs its local
// search on segment lists, and with which segment length and record limit.
// Auto length: the smallest power of two >= 64 that cuts the tour into at
// most a quarter of the record table.
static int seg_plan(int32_t n, int tw, SegPlan *sp) {
  int mode, lg, mx;
  {
    std::lock_guard<std::mutex> lk(g_team_mu);
    mode = g_seg_mode;
    lg = g_seg_log2;
    mx = g_seg_max;
  }
  *sp = SegPlan{};
  (void)tw;
  if (mode != 2) return FACO_OK;
  sp->on = 1;
  sp->max = mx ? mx : faco::kSegCap;
  if (lg) {
    sp->shift = lg;
  } else {
    sp->shift = 6;
    while (((int64_t)n + (1 << sp->shift) - 1) >> sp->shift > faco::kSegCap / 4) ++sp->shift;
  }
  const int64_t chunks = ((int64_t)n + (1 << sp->shift) - 1) >> sp->shift;
  if (chunks + 4 > sp->max)
    return set_err(nullptr, FACO_EINVAL,
                   "segment records must exceed the tour's chunks by 4 (raise the record "
                   "limit or the segment length)");
  return FACO_OK;
}

extern "C" uint64_t faco_footprint_bytes(int32_t n, const faco_params *p) {
  if (validate(p, n)) return 0;
  int32_t k, bl;
  effective_sizes(n, p, &k, &bl);
  const uint64_t N = (uint64_t)n, A = (uint64_t)p->n_ants;
  uint64_t b = 0;
  b += align_up(8 * N);                    // xy
  b += align_up(16 * ((N + 31) / 32));     // bounding boxes of 32-label words
  const uint64_t NB = (N + 63) / 64 * 64;   // source-ordered tables: whole 64-position blocks
  b += 4 * align_up(4 * N * (uint64_t)k);   // cl, cost, eta, tau
  b += 4 * align_up(4 * NB * (uint64_t)k);  // source-ordered city, weight, position, cost
  b += align_up(4 * N * (uint64_t)bl + 4); // backup lists
  b += 4 * align_up(4 * N) + 2 * align_up(8 * N); // source route/pos/edge costs/coordinates, adjacency, global best
  b += 2 * align_up(4 * N);                   // label maps
  b += 3 * align_up(4 * N * A) + align_up(8 * N * A);  // ant routes, pos, rings, tour coordinates
  b += align_up(8 * A) + 2 * align_up(8 * A * faco::NCNT) + align_up(8 * faco::kTicks * A);
  b += align_up(4 * A);  // final tour buffer of each ant
  SegPlan sp;
  if (seg_plan(n, team_waves_for(n, p->n_ants), &sp) == FACO_OK && sp.on)
    b += 2 * align_up(4 * N * A) + 2 * align_up(8 * N * A) + align_up(4 * A);  // segment lists
  b += 2 * align_up(8 * (A + 1)) + align_up(4 * (A + 1));  // verification
  b += align_up(sizeof(DevState));
  return b;
}

// tour-length verification of the ants (ants != 0) and the global best
static void enqueue_verify(faco_instance *h, int ants, int iter_ahead) {
  const Inst &I = h->dv;
  hipLaunchKernelGGL(faco::verify_kernel, dim3(faco::verify_chunks(I.n), (unsigned)I.A + 1),
                     dim3(faco::kVerifyBlock), 0, h->stream, I, ants);
  hipLaunchKernelGGL(faco::verify_finish_kernel, dim3(1), dim3(faco::kVerifyBlock), 0,
                     h->stream, I, ants, iter_ahead);
}

// enqueue the four phases of one iteration
static int enqueue_iteration(faco_instance *h) {
  const Inst &I = h->dv;
  const int n = h->n;
  const unsigned nb_src = (unsigned)((n + 255) / 256);
  const size_t slots = (size_t)n * (size_t)h->k;
  const unsigned nb_tau = (unsigned)((slots + 255) / 256);
  TimedLaunch tl;
  if (h->timing) begin_timed(h, 0, tl);
  hipLaunchKernelGGL(I.seg_on ? faco_ant_seg_kernel(h->k, h->tw) : faco_ant_kernel(h->k, h->tw),
                     dim3(h->p.n_ants), dim3(64 * h->tw), h->lds_ant, h->stream, I, 0);
  if (h->timing) {
    end_timed(h, tl);
    begin_timed(h, 1, tl);
  }
  if (I.verify) enqueue_verify(h, 1, 1);
  hipLaunchKernelGGL(faco::colony_kernel, dim3(1), dim3(64), 0, h->stream, I);
  if (h->timing) {
    end_timed(h, tl);
    begin_timed(h, 2, tl);
  }
  hipLaunchKernelGGL(faco::source_kernel, dim3(nb_src), dim3(256), 0, h->stream, I, 0);
  if (h->timing) {
    end_timed(h, tl);
    begin_timed(h, 3, tl);
  }
  hipLaunchKernelGGL(faco::pheromone_kernel, dim3(nb_tau), dim3(256), 0, h->stream, I, 0);
  if (h->timing) end_timed(h, tl);
  HIP_TRY(h, hipGetLastError());
  return FACO_OK;
}

// Internal labels: the cities in the order of a Hilbert curve over the
// coordinates (16-bit cells over the bounding box; ties by original number).
// A relabelling only: every rule that depends on city numbers uses the
// original ones, so results do not change.
static uint64_t hilbert_d(uint32_t x, uint32_t y) {
  const uint32_t side = 1u << 16;
  uint64_t d = 0;
  for (uint32_t s = side >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += (uint64_t)s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = side - 1 - x;
        y = side - 1 - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

static void hilbert_labels(const int32_t *xy, int32_t n, std::vector<int32_t> &orig_of,
                           std::vector<int32_t> &int_of) {
  int64_t x0 = xy[0], x1 = xy[0], y0 = xy[1], y1 = xy[1];
  for (int32_t i = 1; i < n; ++i) {
    x0 = std::min<int64_t>(x0, xy[2 * i]);
    x1 = std::max<int64_t>(x1, xy[2 * i]);
    y0 = std::min<int64_t>(y0, xy[2 * i + 1]);
    y1 = std::max<int64_t>(y1, xy[2 * i + 1]);
  }
  const int64_t span = std::max<int64_t>(1, std::max(x1 - x0, y1 - y0));
  std::vector<std::pair<uint64_t, int32_t>> key((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    const uint32_t gx = (uint32_t)((xy[2 * i] - x0) * 65535 / span);
    const uint32_t gy = (uint32_t)((xy[2 * i + 1] - y0) * 65535 / span);
    key[(size_t)i] = {hilbert_d(gx, gy), i};
  }
  std::sort(key.begin(), key.end());
  orig_of.resize((size_t)n);
  int_of.resize((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    orig_of[(size_t)i] = key[(size_t)i].second;
    int_of[(size_t)key[(size_t)i].second] = i;
  }
}

extern "C" int faco_build_instance(const int32_t *xy, int32_t n, const faco_params *p,
                                   void *hip_stream, faco_instance **out) {
  if (!out) return set_err(nullptr, FACO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!xy) return set_err(nullptr, FACO_EINVAL, "xy is NULL");
  if (const char *m = validate(p, n)) return set_err(nullptr, FACO_EINVAL, m);
  for (int64_t i = 0; i < 2 * (int64_t)n; ++i)
    if (xy[i] < 0 || xy[i] >= (1 << 26))
      return set_err(nullptr, FACO_EINVAL, "coordinates must be in [0, 2^26)");
  const int tw = team_waves_for(n, p->n_ants);
  SegPlan sp;
  if (int rc = seg_plan(n, tw, &sp)) return rc;

  faco_instance *h = new faco_instance();
  h->tw = tw;
  h->p = *p;
  h->n = n;
  h->xy_host.assign(xy, xy + 2 * (size_t)n);
  effective_sizes(n, p, &h->k, &h->bl);
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return set_err(nullptr, FACO_EDEVICE, "hipGetDevice failed");
  }
  const size_t N = (size_t)n, A = (size_t)p->n_ants, K = (size_t)h->k, BL = (size_t)h->bl;
  const size_t NB = (N + 63) / 64 * 64;

  Inst &I = h->dv;
  I.n = n;
  I.k = h->k;
  I.bl = h->bl;
  I.A = p->n_ants;
  I.m = p->min_new_edges;
  I.m_hi = p->min_new_edges_max;
  I.verify = 0;
  I.seg_on = sp.on;
  I.seg_shift = sp.shift;
  I.seg_max = sp.max;
  I.lcap = queue_lds_cap_for(n, sp.on ? 4 * sp.max : 0);
  I.rho = p->rho;
  I.ls_flags = p->ls_flags;
  I.oropt_max = p->oropt_max_seg;
  I.seed = p->seed;
  I.p_gb = p->p_source_gbest;
  I.p_root = std::pow(p->p_best, 1.0 / (double)n);

  void *ptr;
  int rc = FACO_OK;
#define ALLOC(field, type, count)                      \
  if ((rc = dalloc(h, &ptr, sizeof(type) * (count)))) { \
    faco_destroy_instance(h);                          \
    g_err = "device allocation failed";                \
    return rc;                                         \
  }                                                    \
  I.field = (type *)ptr;
  ALLOC(xy, int2, N);
  ALLOC(wbox, int4, (N + 31) / 32);
  ALLOC(orig_of, int32_t, N);
  ALLOC(int_of, int32_t, N);
  ALLOC(cl, int32_t, N * K);
  ALLOC(bll, int32_t, N * BL + 1);
  ALLOC(eta, float, N * K);
  ALLOC(cl_d, int32_t, N * K);
  ALLOC(tau, float, N * K);
  ALLOC(scl, int32_t, NB * K);
  ALLOC(sw, float, NB * K);
  ALLOC(ssp, int32_t, NB * K);
  ALLOC(sd, int32_t, NB * K);
  ALLOC(src_route, int32_t, N);
  ALLOC(src_pos, int32_t, N);
  ALLOC(gb_route, int32_t, N);
  ALLOC(src_adj, int2, N);
  ALLOC(src_d, int32_t, N);
  ALLOC(src_xy, int2, N);
  ALLOC(routes, int32_t, N * A);
  ALLOC(pos, int32_t, N * A);
  ALLOC(ring, int32_t, N * A);
  ALLOC(rxy, int2, N * A);
  ALLOC(lens, int64_t, A);
  ALLOC(cnt, int64_t, A * faco::NCNT);
  ALLOC(cnt_acc, int64_t, A * faco::NCNT);
  ALLOC(ticks, int64_t, A * faco::kTicks);
  ALLOC(rsel, int32_t, A);
  if (sp.on) {
    ALLOC(r2, int32_t, N * A);
    ALLOC(p2, int32_t, N * A);
    ALLOC(x2, int2, N * A);
    ALLOC(sgid, int2, N * A);
    ALLOC(sepoch, int32_t, A);
  }
  ALLOC(vsum, int64_t, A + 1);
  ALLOC(vbad, int32_t, A + 1);
  ALLOC(vout, int64_t, A + 1);
  ALLOC(st, DevState, 1);
#undef ALLOC

  auto fail = [&](int code) {
    std::string m = h->err;
    faco_destroy_instance(h);
    g_err = m;
    return code;
  };
  hipError_t e;
#define BTRY(expr)                                                           \
  if ((e = (expr)) != hipSuccess) {                                          \
    h->err = std::string(#expr ": ") + hipGetErrorString(e);                 \
    return fail(FACO_EDEVICE);                                               \
  }
  BTRY(hipMemsetAsync(I.st, 0, sizeof(DevState), h->stream));
  BTRY(hipMemsetAsync(I.cnt_acc, 0, sizeof(int64_t) * A * faco::NCNT, h->stream));
  // ant state before the first iteration: no tours (-1), lengths and counters 0
  BTRY(hipMemsetAsync(I.routes, 0xFF, sizeof(int32_t) * N * A, h->stream));
  BTRY(hipMemsetAsync(I.lens, 0, sizeof(int64_t) * A, h->stream));
  BTRY(hipMemsetAsync(I.cnt, 0, sizeof(int64_t) * A * faco::NCNT, h->stream));
  BTRY(hipMemsetAsync(I.ticks, 0, sizeof(int64_t) * A * faco::kTicks, h->stream));
  BTRY(hipMemsetAsync(I.rsel, 0, sizeof(int32_t) * A, h->stream));
  if (sp.on) {
    // epochs start at 1: no record label matches before it is written
    BTRY(hipMemsetAsync(I.sgid, 0, sizeof(int2) * N * A, h->stream));
    BTRY(hipMemsetAsync(I.sepoch, 0, sizeof(int32_t) * A, h->stream));
  }
  BTRY(hipMemsetAsync(I.vsum, 0, sizeof(int64_t) * (A + 1), h->stream));
  BTRY(hipMemsetAsync(I.vbad, 0, sizeof(int32_t) * (A + 1), h->stream));
  BTRY(hipMemsetAsync(I.vout, 0, sizeof(int64_t) * (A + 1), h->stream));
  hilbert_labels(xy, n, h->orig_of, h->int_of);
  std::vector<int32_t> xy_int(2 * N);
  for (size_t i = 0; i < N; ++i) {
    xy_int[2 * i] = xy[2 * (size_t)h->orig_of[i]];
    xy_int[2 * i + 1] = xy[2 * (size_t)h->orig_of[i] + 1];
  }
  BTRY(hipMemcpyAsync((void *)I.xy, xy_int.data(), sizeof(int2) * N, hipMemcpyHostToDevice,
                      h->stream));
  // bounding box of each bitmap word's 32 labels (the nearest-unvisited scan
  // skips words whose box lies beyond its bound)
  std::vector<int32_t> wbox(4 * ((N + 31) / 32));
  for (size_t wi = 0; wi < (N + 31) / 32; ++wi) {
    int32_t x0 = INT32_MAX, y0 = INT32_MAX, x1 = INT32_MIN, y1 = INT32_MIN;
    for (size_t i = 32 * wi; i < std::min(N, 32 * wi + 32); ++i) {
      x0 = std::min(x0, xy_int[2 * i]);
      y0 = std::min(y0, xy_int[2 * i + 1]);
      x1 = std::max(x1, xy_int[2 * i]);
      y1 = std::max(y1, xy_int[2 * i + 1]);
    }
    wbox[4 * wi] = x0;
    wbox[4 * wi + 1] = y0;
    wbox[4 * wi + 2] = x1;
    wbox[4 * wi + 3] = y1;
  }
  BTRY(hipMemcpyAsync((void *)I.wbox, wbox.data(), sizeof(int32_t) * wbox.size(),
                      hipMemcpyHostToDevice, h->stream));
  BTRY(hipMemcpyAsync((void *)I.orig_of, h->orig_of.data(), sizeof(int32_t) * N,
                      hipMemcpyHostToDevice, h->stream));
  BTRY(hipMemcpyAsync((void *)I.int_of, h->int_of.data(), sizeof(int32_t) * N,
                      hipMemcpyHostToDevice, h->stream));

  const size_t klds = knn_lds_bytes(h->k, h->bl);
  BTRY(hipFuncSetAttribute((const void *)faco::knn_kernel,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)klds));
  hipLaunchKernelGGL(faco::knn_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), klds,
                     h->stream, I.xy, I.orig_of, I.int_of, I.wbox, n, h->k, h->bl,
                     (int32_t *)I.cl,
                     (int32_t *)I.bll,
                     (float *)I.eta, (int32_t *)I.cl_d, I.st);
  BTRY(hipGetLastError());
  DevState hs;
  BTRY(hipMemcpyAsync(&hs, I.st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  BTRY(hipStreamSynchronize(h->stream));
  if (hs.dup) {
    h->err = "two cities share coordinates";
    return fail(FACO_EDUP);
  }

  h->lds_init = sizeof(uint32_t) * ((size_t)faco_team_lds_words(h->tw) +
                                    3 * (size_t)((n + 31) / 32) + (size_t)I.lcap);
  BTRY(hipFuncSetAttribute((const void *)faco_ant_kernel(h->k, h->tw),
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds_init));
  h->lds_ant = h->lds_init;
  if (I.seg_on) {
    h->lds_ant = sizeof(uint32_t) * ((size_t)faco_seg_lds_words(h->tw, n) +
                                     4 * (size_t)I.seg_max + (size_t)I.lcap);
    BTRY(hipFuncSetAttribute((const void *)faco_ant_seg_kernel(h->k, h->tw),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds_ant));
  }
  // initial solution (ant slot 0, flat tour), limits, tau = tau_max, source =
  // global best
  hipLaunchKernelGGL(faco_ant_kernel(h->k, h->tw), dim3(1), dim3(64 * h->tw), h->lds_init,
                     h->stream, I, 1);
  if (p->ls_flags & FACO_LS_INIT_3OPT) {
    // the initial search with 3-opt, on the nearest-neighbour tour
    const size_t ilds = sizeof(uint32_t) * 2 * ((N + 31) / 32);
    BTRY(hipFuncSetAttribute((const void *)faco::init_search_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)ilds));
    hipLaunchKernelGGL(faco::init_search_kernel, dim3(1), dim3(64), ilds, h->stream, I);
  }
  hipLaunchKernelGGL(faco::init_state_kernel, dim3(1), dim3(1), 0, h->stream, I);
  hipLaunchKernelGGL(faco::source_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     h->stream, I, 1);
  const size_t slots = N * K;
  hipLaunchKernelGGL(faco::pheromone_kernel, dim3((unsigned)((slots + 255) / 256)), dim3(256),
                     0, h->stream, I, 1);
  BTRY(hipGetLastError());
  BTRY(hipStreamSynchronize(h->stream));
#undef BTRY
  *out = h;
  return FACO_OK;
}

extern "C" int faco_run_iterations(faco_instance *h, int32_t iterations) {
  if (!h) return set_err(nullptr, FACO_EINVAL, "handle is NULL");
  if (iterations < 0) return set_err(h, FACO_EINVAL, "iterations must be >= 0");
  for (int32_t i = 0; i < iterations; ++i) {
    int rc = enqueue_iteration(h);
    if (rc) return rc;
  }
  return FACO_OK;
}

// Device-to-host copy on the handle's stream, then wait for it.  (The
// legacy stream is avoided: another thread may be capturing a batch graph.)
static hipError_t d2h(faco_instance *h, void *dst, const void *src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(h->stream);
}

static int fault_error(faco_instance *h, const DevState &hs) {
  std::string what;
  if (hs.fault & faco::FAULT_LS_STALL)
    what += " local search stopped: a sweep listed cities that the move evaluation found no"
            " move for;";
  if (hs.fault & faco::FAULT_LENGTH)
    what += " a recomputed tour length differs from the tracked one;";
  if (hs.fault & faco::FAULT_PERMUTATION) what += " an ant's route is not a permutation;";
  if (hs.fault & faco::FAULT_BATCH_STALL) what += " a persistent batch stalled;";
  return set_err(h, FACO_EDEVICE,
                 "device fault" + what + " first at ant " + std::to_string(hs.fault_ant) +
                     " (-1: initial solution or global best), iteration " +
                     std::to_string(hs.fault_iter));
}

extern "C" int faco_set_verify(faco_instance *h, int32_t enable) {
  if (!h) return set_err(nullptr, FACO_EINVAL, "handle is NULL");
  h->dv.verify = enable ? 1 : 0;
  return FACO_OK;
}

extern "C" int faco_get_best_tour(faco_instance *h, int32_t *tour_out, int64_t *length_out) {
  if (!h) return set_err(nullptr, FACO_EINVAL, "handle is NULL");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (tour_out) {
    HIP_TRY(h, d2h(h, tour_out, h->dv.gb_route, sizeof(int32_t) * (size_t)h->n));
    for (int32_t i = 0; i < h->n; ++i) tour_out[i] = h->orig_of[(size_t)tour_out[i]];
  }
  DevState hs;
  HIP_TRY(h, d2h(h, &hs, h->dv.st, sizeof(DevState)));
  if (length_out) *length_out = hs.gb_len;
  if (hs.fault) return fault_error(h, hs);
  return FACO_OK;
}

extern "C" void faco_destroy_instance(faco_instance *h) {
  if (!h) return;
  // every batch that used the instance is ordered before its stream's later
  // work, so after this wait no queued work touches its blocks
  const bool idle = hipStreamSynchronize(h->stream) == hipSuccess;
  for (auto &tl : h->pending) {
    (void)hipEventDestroy(tl.a);
    (void)hipEventDestroy(tl.b);
  }
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (idle) {
    for (auto &a : h->allocs) blk_put(h->device, a.first, a.second);
  } else {
    std::lock_guard<std::mutex> lk(g_capture_mu);
    for (auto &a : h->allocs) (void)hipFree(a.first);
  }
  delete h;
}

extern "C" int faco_set_stream(faco_instance *h, void *hip_stream) {
  if (!h) return set_err(nullptr, FACO_EINVAL, "handle is NULL");
  const hipStream_t ns = (hipStream_t)hip_stream;
  if (ns == h->stream) return FACO_OK;
  hipEvent_t ev;
  HIP_TRY(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  hipError_t e = hipEventRecord(ev, h->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(ns, ev, 0);
  (void)hipEventDestroy(ev);
  HIP_TRY(h, e);
  h->stream = ns;
  return FACO_OK;
}

extern "C" const char *faco_last_error(const faco_instance *h) {
  return h ? h->err.c_str() : g_err.c_str();
}

extern "C" int faco_debug_get(faco_instance *h, int32_t what, void *out, size_t bytes) {
  if (!h) return set_err(nullptr, FACO_EINVAL, "handle is NULL");
  if (!out) return set_err(h, FACO_EINVAL, "out is NULL");
  const size_t N = (size_t)h->n, A = (size_t)h->p.n_ants, K = (size_t)h->k, BL = (size_t)h->bl;
  const void *src = nullptr;
  size_t need = 0;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  DevState hs;
  HIP_TRY(h, d2h(h, &hs, h->dv.st, sizeof(DevState)));
  switch (what) {
    case FACO_DBG_ANT_ROUTES: {
      // each ant's tour sits in the storage buffer its local search left it in
      if (bytes != 4 * N * A) return set_err(h, FACO_EINVAL, "size mismatch");
      std::vector<int32_t> sel(A);
      HIP_TRY(h, d2h(h, sel.data(), h->dv.rsel, 4 * A));
      for (size_t a = 0; a < A; ++a) {
        const int32_t *base = sel[a] && h->dv.r2 ? h->dv.r2 : h->dv.routes;
        HIP_TRY(h, d2h(h, (int32_t *)out + a * N, base + a * N, 4 * N));
      }
      break;
    }
    case FACO_DBG_ANT_LENGTHS: src = h->dv.lens; need = 8 * A; break;
    case FACO_DBG_PHEROMONE: src = h->dv.tau; need = 4 * N * K; break;
    case FACO_DBG_SOURCE: src = h->dv.src_route; need = 4 * N; break;
    case FACO_DBG_COUNTERS: src = h->dv.cnt; need = 8 * A * faco::NCNT; break;
    case FACO_DBG_COUNTER_TOTALS: src = h->dv.cnt_acc; need = 8 * A * faco::NCNT; break;
    case FACO_DBG_PHASE_TICKS: src = h->dv.ticks; need = 8 * A * faco::kTicks; break;
    case FACO_DBG_CAND_LISTS: src = h->dv.cl; need = 4 * N * K; break;
    case FACO_DBG_BACKUP_LISTS: src = h->dv.bll; need = 4 * N * BL; break;
    case FACO_DBG_HEURISTIC: src = h->dv.eta; need = 4 * N * K; break;
    case FACO_DBG_LIMITS: {
      if (bytes != 12) return set_err(h, FACO_EINVAL, "size mismatch");
      float f[3] = {hs.tau_min, hs.tau_max, hs.delta};
      std::memcpy(out, f, 12);
      return FACO_OK;
    }
    case FACO_DBG_INFO: {
      if (bytes != 64) return set_err(h, FACO_EINVAL, "size mismatch");
      int64_t v[8] = {hs.iter, h->k, h->bl, hs.ib, hs.src_gb, hs.init_len, hs.gb_len, hs.src_len};
      std::memcpy(out, v, 64);
      return FACO_OK;
    }
    case FACO_DBG_FAULT: {
      if (bytes != 32) return set_err(h, FACO_EINVAL, "size mismatch");
      int64_t v[4] = {hs.fault, hs.fault_ant, hs.fault_iter, hs.verified};
      std::memcpy(out, v, 32);
      return FACO_OK;
    }
    case FACO_DBG_RECOMPUTED_LENGTHS: {
      if (bytes != 8 * (A + 1)) return set_err(h, FACO_EINVAL, "size mismatch");
      // ant tours exist once an iteration has run
      enqueue_verify(h, hs.iter > 0 ? 1 : 0, 0);
      HIP_TRY(h, hipGetLastError());
      HIP_TRY(h, d2h(h, out, h->dv.vout, 8 * (A + 1)));
      if (hs.iter == 0)
        for (size_t a = 0; a < A; ++a) ((int64_t *)out)[a] = 0;
      return FACO_OK;
    }
    case FACO_DBG_TEAM_WAVES: {
      if (bytes != 4) return set_err(h, FACO_EINVAL, "size mismatch");
      const int32_t tw = h->tw;
      std::memcpy(out, &tw, 4);
      return FACO_OK;
    }
    case FACO_DBG_TOUR: {
      if (bytes != 24) return set_err(h, FACO_EINVAL, "size mismatch");
      const Inst &I = h->dv;
      int64_t v[3] = {I.seg_on, I.seg_on ? (int64_t)1 << I.seg_shift : 0, I.seg_max};
      std::memcpy(out, v, 24);
      return FACO_OK;
    }
    case FACO_DBG_INIT_TICKS: {
      if (bytes != 8 * (size_t)faco::kTicks) return set_err(h, FACO_EINVAL, "size mismatch");
      std::memcpy(out, hs.init_ticks, 8 * (size_t)faco::kTicks);
      return FACO_OK;
    }
    case FACO_DBG_INIT_COUNTERS: {
      if (bytes != 8 * faco::NCNT) return set_err(h, FACO_EINVAL, "size mismatch");
      std::memcpy(out, hs.init_cnt, 8 * faco::NCNT);
      return FACO_OK;
    }
    default: return set_err(h, FACO_EINVAL, "unknown dump");
  }
  if (what != FACO_DBG_ANT_ROUTES) {
    if (bytes != need) return set_err(h, FACO_EINVAL, "size mismatch");
    if (need) HIP_TRY(h, d2h(h, out, src, need));
  }
  // back to original city numbers: city values, and rows indexed by city
  const auto &orig = h->orig_of;
  auto map_values = [&](int32_t *v, size_t cnt) {
    for (size_t i = 0; i < cnt; ++i) v[i] = (uint32_t)v[i] < (uint32_t)N ? orig[(size_t)v[i]] : -1;
  };
  auto permute_rows = [&](void *base, size_t row_bytes) {
    std::vector<unsigned char> tmp((unsigned char *)base, (unsigned char *)base + N * row_bytes);
    for (size_t i = 0; i < N; ++i)
      std::memcpy((unsigned char *)base + (size_t)orig[i] * row_bytes, tmp.data() + i * row_bytes,
                  row_bytes);
  };
  switch (what) {
    case FACO_DBG_ANT_ROUTES: map_values((int32_t *)out, N * A); break;
    case FACO_DBG_SOURCE: map_values((int32_t *)out, N); break;
    case FACO_DBG_PHEROMONE:
    case FACO_DBG_HEURISTIC: permute_rows(out, 4 * K); break;
    case FACO_DBG_CAND_LISTS:
      map_values((int32_t *)out, N * K);
      permute_rows(out, 4 * K);
      break;
    case FACO_DBG_BACKUP_LISTS:
      map_values((int32_t *)out, N * BL);
      if (BL) permute_rows(out, 4 * BL);
      break;
    default: break;
  }
  return FACO_OK;
}

extern "C" int faco_set_timing(faco_instance *h, int32_t enable) {
  if (!h) return set_err(nullptr, FACO_EINVAL, "handle is NULL");
  if (enable < 0) return set_err(h, FACO_EINVAL, "enable must be >= 0");
  h->timing = enable != 0;
  // events for `enable` iterations (two per phase) made ahead of the launches
  const size_t want = enable > 1 ? (size_t)enable * 8 : 0;
  while (h->ev_pool.size() < want) {
    hipEvent_t e;
    HIP_TRY(h, hipEventCreate(&e));
    h->ev_pool.push_back(e);
  }
  return FACO_OK;
}

extern "C" int faco_phase_times(faco_instance *h, double *ms_out, int64_t *launches) {
  if (!h) return set_err(nullptr, FACO_EINVAL, "handle is NULL");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (auto &tl : h->pending) {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, tl.a, tl.b);
    h->phase_ms[tl.phase] += ms;
    h->phase_n[tl.phase] += 1;
    h->ev_pool.push_back(tl.a);
    h->ev_pool.push_back(tl.b);
  }
  h->pending.clear();
  for (int i = 0; i < 4; ++i) {
    if (ms_out) ms_out[i] = h->phase_ms[i];
    if (launches) launches[i] = h->phase_n[i];
    h->phase_ms[i] = 0;
    h->phase_n[i] = 0;
  }
  return FACO_OK;
}

// ------------------------------------------------------------------------
// Batched execution (faco_run_batch).  The launch tables live in a workspace
// per stream that grows on demand; calls are serialised.  How a batch is
// launched (one persistent launch or launches per phase, waves per ant, ants
// per workgroup, LDS queue capacity) is a faco_batch_config: the one
// faco_autotune_batch stored for the batch's size class, else the
// process-wide default.  None of it changes a result.

static const size_t kLdsBytes = 160 * 1024;  // LDS of one CU (gfx950)
static std::mutex g_batch_mu;
static faco_batch_config g_batch_cfg = {0, 0, 1, 0, 0, 0};
// tuned configurations by size class (log2 of the longest tour)
static std::map<int, faco_batch_config> g_tuned;

struct BatchWs {
  Inst *insts = nullptr;
  int2 *amap = nullptr;
  faco::BatchCtl *ctl = nullptr;
  faco::BatchRun *run = nullptr;
  size_t cap_insts = 0, cap_amap = 0, cap_ctl = 0;
  hipEvent_t last_done = nullptr;  // completion of the previous batch
  hipStream_t cap = nullptr;       // the stream the batch iteration is captured on
};
// one workspace per stream, so batches on different streams run concurrently
static std::map<hipStream_t, BatchWs> g_ws_map;

static const char *check_config(const faco_batch_config *c) {
  if (!c) return "config is NULL";
  if (c->persistent != 0 && c->persistent != 1) return "persistent must be 0 or 1";
  if (c->team_waves != 0 && c->team_waves != 1 && c->team_waves != 4 && c->team_waves != 8)
    return "team_waves must be 0, 1, 4 or 8";
  if (c->ants_per_block != 1 && c->ants_per_block != 2 && c->ants_per_block != 4)
    return "ants_per_block must be 1, 2 or 4";
  if (c->queue_lds_capacity != 0 &&
      (c->queue_lds_capacity < 64 || c->queue_lds_capacity > faco::kLdsRingMax))
    return "queue_lds_capacity must be 0 or in [64, 16384]";
  if (c->big_percent < 0 || c->big_percent > 100) return "big_percent must be in [0, 100]";
  if (c->big_percent > 0 && c->big_team_waves != 1 && c->big_team_waves != 4 &&
      c->big_team_waves != 8)
    return "big_team_waves must be 1, 4 or 8";
  return nullptr;
}

extern "C" int faco_set_batch_config(const faco_batch_config *c) {
  if (const char *m = check_config(c)) return set_err(nullptr, FACO_EINVAL, m);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_batch_cfg = *c;
  g_tuned.clear();
  return FACO_OK;
}

extern "C" int faco_get_batch_config(faco_batch_config *c) {
  if (!c) return set_err(nullptr, FACO_EINVAL, "config is NULL");
  std::lock_guard<std::mutex> lk(g_batch_mu);
  *c = g_batch_cfg;
  return FACO_OK;
}

extern "C" int faco_set_batch_ants_per_block(int32_t apb) {
  if (apb != 1 && apb != 2 && apb != 4) return set_err(nullptr, FACO_EINVAL, "ants per block must be 1, 2 or 4");
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_batch_cfg.ants_per_block = apb;
  return FACO_OK;
}

static int ilog2(int64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
}

static int size_class(faco_instance *const *hs, int32_t count) {
  int maxn = 0;
  for (int32_t i = 0; i < count; ++i) maxn = hs[i]->n > maxn ? hs[i]->n : maxn;
  return ilog2(maxn);
}

// Argument checks shared by the batched entry points.
static const char *check_batch_args(faco_instance *const *hs, int32_t count,
                                    int32_t iterations) {
  if (!hs || count < 0) return "bad handle array";
  if (iterations < 0) return "iterations must be >= 0";
  for (int32_t i = 0; i < count; ++i) {
    if (!hs[i]) return "NULL handle in batch";
    for (int32_t j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return "handles must be distinct";
  }
  return nullptr;
}

static int batch_ant_count(faco_instance *const *hs, int32_t count) {
  int total = 0;
  for (int32_t i = 0; i < count; ++i) total += hs[i]->p.n_ants;
  return total;
}

// Launch shape of one batch.
struct BatchShape {
  int count = 0, total = 0, kmax = 2, maxn = 0, max_ants = 0, tw = 1, apb = 1;
  bool any_verify = false, persistent = false;
  size_t lds_words = 0, max_slots = 0, lds_bytes = 0;
  AntBatchFn antk = nullptr;
  AntPersistFn persk = nullptr;
};

// Fill the host tables (insts[count], amap[total ants]) and derive the
// launch shape from the configuration.  Caller holds g_batch_mu.
static void batch_shape(faco_instance *const *hs, int32_t count, Inst *insts, int2 *amap,
                        const faco_batch_config &cfg, BatchShape &B) {
  B.count = count;
  for (int32_t i = 0; i < count; ++i) {
    faco_instance *h = hs[i];
    B.kmax = h->k > B.kmax ? h->k : B.kmax;
    B.maxn = h->n > B.maxn ? h->n : B.maxn;
    B.max_ants = h->p.n_ants > B.max_ants ? h->p.n_ants : B.max_ants;
    B.any_verify = B.any_verify || h->dv.verify;
    B.total += h->p.n_ants;
  }
  // waves per ant: the configuration's, else as for a lone instance (from
  // the longest tour and the ant count)
  B.tw = cfg.team_waves ? cfg.team_waves : team_waves_for(B.maxn, B.total);
  int w = 0;
  for (int32_t i = 0; i < count; ++i) {
    faco_instance *h = hs[i];
    insts[i] = h->dv;
    if (cfg.queue_lds_capacity) {
      // the queue's LDS part: the configured capacity, within what LDS has
      // left beside the team area and the three bitmaps
      const int room = 160 * 1024 / 4 - faco_team_lds_words(8) - 3 * ((h->n + 31) / 32);
      int cap = h->n < cfg.queue_lds_capacity ? h->n : cfg.queue_lds_capacity;
      insts[i].lcap = cap < room ? cap : room;
    }
    const size_t words = 3 * (size_t)((h->n + 31) / 32) + (size_t)insts[i].lcap;
    B.lds_words = words > B.lds_words ? words : B.lds_words;
    const size_t slots = (size_t)h->n * (size_t)h->k;
    B.max_slots = slots > B.max_slots ? slots : B.max_slots;
    if (amap)
      for (int a = 0; a < h->p.n_ants; ++a) amap[w++] = make_int2(i, a);
  }
  // with one wave per ant, ants per workgroup: the configured number,
  // lowered until their LDS fits a CU
  B.apb = B.tw > 1 ? 1 : cfg.ants_per_block;
  while (B.apb > 1 && sizeof(uint32_t) * B.lds_words * (size_t)B.apb > kLdsBytes) B.apb >>= 1;
  B.lds_bytes =
      sizeof(uint32_t) * ((size_t)faco_team_lds_words(B.tw) + B.lds_words * (size_t)B.apb);
  B.antk = faco_ant_batch_kernel(B.kmax, B.tw);
  B.persk = faco_ant_persist_kernel(B.kmax, B.tw);
  // the per-iteration verification runs in the per-phase launches
  B.persistent = cfg.persistent == 1 && !B.any_verify;
}

// The launches of one batched iteration over the device tables.
static void enqueue_batch_iteration(const BatchShape &B, const Inst *d_insts,
                                    const int2 *d_amap, hipStream_t s) {
  const unsigned nb_ant = (unsigned)((B.total + B.apb - 1) / B.apb);
  const dim3 g_src((unsigned)((B.maxn + 255) / 256), (unsigned)B.count);
  const dim3 g_tau((unsigned)((B.max_slots + 255) / 256), (unsigned)B.count);
  hipLaunchKernelGGL(B.antk, dim3(nb_ant), dim3(64 * (B.tw > 1 ? B.tw : B.apb)), B.lds_bytes,
                     s, d_insts, d_amap, B.total, B.apb, (int)B.lds_words);
  if (B.any_verify) {
    hipLaunchKernelGGL(faco::verify_batch_kernel,
                       dim3(faco::verify_chunks(B.maxn), (unsigned)B.max_ants + 1,
                            (unsigned)B.count),
                       dim3(faco::kVerifyBlock), 0, s, d_insts);
    hipLaunchKernelGGL(faco::verify_finish_batch_kernel, dim3((unsigned)B.count),
                       dim3(faco::kVerifyBlock), 0, s, d_insts);
  }
  hipLaunchKernelGGL(faco::colony_batch_kernel, dim3((unsigned)B.count), dim3(64), 0, s,
                     d_insts);
  hipLaunchKernelGGL(faco::source_batch_kernel, g_src, dim3(256), 0, s, d_insts);
  hipLaunchKernelGGL(faco::pheromone_batch_kernel, g_tau, dim3(256), 0, s, d_insts);
}

// Grow a workspace array (the previous batch on the stream has finished, so
// the old block goes back to the cache) to at least twice its size.
template <class T>
static hipError_t ws_grow(int dev, T *&ptr, size_t &cap, size_t want) {
  if (cap >= want) return hipSuccess;
  if (want < 2 * cap) want = 2 * cap;
  blk_put(dev, ptr, sizeof(T) * cap);  // at most the block's true size
  ptr = nullptr;
  cap = 0;
  void *q = nullptr;
  size_t got = 0;
  const hipError_t e = blk_get(dev, sizeof(T) * want, &q, &got);
  if (e == hipSuccess) {
    ptr = (T *)q;
    cap = got / sizeof(T);
  }
  return e;
}

// One batch call with an explicit configuration.
// One (sub-)batch with an explicit configuration.  Caller holds g_batch_mu.
// handles: order the batch after the work already on the handles' own
// streams, and their later work after the batch (a split does that once for
// both of its parts).
static int run_batch_one(faco_instance *const *hs, int32_t count, int32_t iterations,
                         hipStream_t st, const faco_batch_config &cfg, bool handles = true) {
  BatchWs &g_ws = g_ws_map[st];
  hipError_t e;
#define BT(expr)                                                                      \
  if ((e = (expr)) != hipSuccess)                                                     \
    return set_err(nullptr, FACO_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e));
  // host tables
  std::vector<Inst> insts((size_t)count);
  std::vector<int2> amap((size_t)batch_ant_count(hs, count));
  BatchShape B;
  batch_shape(hs, count, insts.data(), amap.data(), cfg, B);
  const int total = B.total;
  // the tables are shared: the previous batch must be done with them
  if (!g_ws.last_done) BT(hipEventCreateWithFlags(&g_ws.last_done, hipEventDisableTiming));
  const bool grow = g_ws.cap_insts < (size_t)count || g_ws.cap_amap < (size_t)total ||
                    g_ws.cap_ctl < (size_t)count || !g_ws.run;
  if (grow) BT(hipEventSynchronize(g_ws.last_done));
  BT(hipStreamWaitEvent(st, g_ws.last_done, 0));
  // device tables
  if (grow) {
    int dev = 0;
    BT(hipGetDevice(&dev));
    BT(ws_grow(dev, g_ws.insts, g_ws.cap_insts, (size_t)count));
    BT(ws_grow(dev, g_ws.amap, g_ws.cap_amap, (size_t)total));
    BT(ws_grow(dev, g_ws.ctl, g_ws.cap_ctl, (size_t)count));
    size_t cap_run = 0;
    if (!g_ws.run) BT(ws_grow(dev, g_ws.run, cap_run, 1));
  }
  // order after the handles' own streams
  for (int32_t i = 0; i < count && handles; ++i) {
    if (hs[i]->stream == st) continue;
    hipEvent_t ev;
    BT(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    BT(hipEventRecord(ev, hs[i]->stream));
    BT(hipStreamWaitEvent(st, ev, 0));
    BT(hipEventDestroy(ev));
  }
  if (B.persistent) {
    // largest tours first: their ants are the longest chains
    std::vector<int> order((size_t)count);
    for (int32_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return hs[a]->n > hs[b]->n; });
    std::vector<Inst> sorted((size_t)count);
    std::vector<faco::BatchCtl> ctl((size_t)count);
    for (int32_t j = 0; j < count; ++j) {
      sorted[(size_t)j] = insts[(size_t)order[(size_t)j]];
      ctl[(size_t)j] = faco::BatchCtl{0, 0, 0, hs[order[(size_t)j]]->p.n_ants, 0};
    }
    const faco::BatchRun run = {count, iterations, 0, 0};
    BT(hipMemcpyAsync(g_ws.insts, sorted.data(), sizeof(Inst) * (size_t)count,
                      hipMemcpyHostToDevice, st));
    BT(hipMemcpyAsync(g_ws.ctl, ctl.data(), sizeof(faco::BatchCtl) * (size_t)count,
                      hipMemcpyHostToDevice, st));
    BT(hipMemcpyAsync(g_ws.run, &run, sizeof(run), hipMemcpyHostToDevice, st));
    BT(hipFuncSetAttribute((const void *)B.persk, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)B.lds_bytes));
    // as many workers as can be resident, at most one per ant
    const int threads = 64 * (B.tw > 1 ? B.tw : B.apb);
    int per_cu = 0, dev = 0, ncu = 0;
    BT(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)B.persk, threads,
                                                    B.lds_bytes));
    BT(hipGetDevice(&dev));
    BT(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int want = B.tw > 1 ? total : (total + B.apb - 1) / B.apb;
    int grid = (per_cu > 0 ? per_cu : 1) * (ncu > 0 ? ncu : 1);
    grid = grid < want ? grid : want;
    hipLaunchKernelGGL(B.persk, dim3((unsigned)grid), dim3((unsigned)threads), B.lds_bytes, st,
                       (const Inst *)g_ws.insts, g_ws.ctl, g_ws.run, (int)B.lds_words);
    BT(hipGetLastError());
  } else {
    BT(hipMemcpyAsync(g_ws.insts, insts.data(), sizeof(Inst) * (size_t)count,
                      hipMemcpyHostToDevice, st));
    BT(hipMemcpyAsync(g_ws.amap, amap.data(), sizeof(int2) * (size_t)total,
                      hipMemcpyHostToDevice, st));
    BT(hipFuncSetAttribute((const void *)B.antk, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)B.lds_bytes));
    if (iterations == 1) {
      enqueue_batch_iteration(B, g_ws.insts, g_ws.amap, st);
      BT(hipGetLastError());
    } else {
      // one iteration captured as a graph, replayed
      if (!g_ws.cap) BT(hipStreamCreateWithFlags(&g_ws.cap, hipStreamNonBlocking));
      hipStream_t cap = g_ws.cap;
      hipGraph_t graph;
      hipGraphExec_t exec;
      {
        std::lock_guard<std::mutex> clk(g_capture_mu);
        BT(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        enqueue_batch_iteration(B, g_ws.insts, g_ws.amap, cap);
        BT(hipStreamEndCapture(cap, &graph));
      }
      BT(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      for (int32_t it = 0; it < iterations; ++it) BT(hipGraphLaunch(exec, st));
      BT(hipGraphExecDestroy(exec));
      BT(hipGraphDestroy(graph));
    }
  }
  // later calls on each handle's stream, and the next batch, come after this one
  BT(hipEventRecord(g_ws.last_done, st));
  for (int32_t i = 0; i < count && handles; ++i)
    if (hs[i]->stream != st) BT(hipStreamWaitEvent(hs[i]->stream, g_ws.last_done, 0));
#undef BT
  return FACO_OK;
}

// A second stream per batch stream, for the large instances of a split batch.
struct SplitStream {
  hipStream_t s = nullptr, s2 = nullptr;  // the big and the small part
  hipEvent_t start = nullptr, done = nullptr, done2 = nullptr;
};
static std::map<hipStream_t, SplitStream> g_split_map;

// One batch call with an explicit configuration: the whole batch at once, or
// (big_percent > 0) the largest instances as a sub-batch of their own (waves
// per ant big_team_waves) beside the rest, each part on a non-blocking stream
// of the library (the caller's stream may be the legacy default stream, which
// would serialise with the other part), the call still ordered on st.
static int run_batch_cfg(faco_instance *const *hs, int32_t count, int32_t iterations,
                         hipStream_t st, const faco_batch_config &cfg) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  const int nbig = cfg.big_percent > 0 ? (count * cfg.big_percent + 99) / 100 : 0;
  if (nbig == 0 || nbig >= count) return run_batch_one(hs, count, iterations, st, cfg);
  hipError_t e;
#define BT(expr)                                                                      \
  if ((e = (expr)) != hipSuccess)                                                     \
    return set_err(nullptr, FACO_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e));
  std::vector<faco_instance *> order(hs, hs + count);
  std::stable_sort(order.begin(), order.end(),
                   [](const faco_instance *a, const faco_instance *b) { return a->n > b->n; });
  SplitStream &sp = g_split_map[st];
  if (!sp.s) {
    BT(hipStreamCreateWithFlags(&sp.s, hipStreamNonBlocking));
    BT(hipStreamCreateWithFlags(&sp.s2, hipStreamNonBlocking));
    BT(hipEventCreateWithFlags(&sp.start, hipEventDisableTiming));
    BT(hipEventCreateWithFlags(&sp.done, hipEventDisableTiming));
    BT(hipEventCreateWithFlags(&sp.done2, hipEventDisableTiming));
  }
  // both streams start after the work already on st and on the handles' own
  // streams, and end before anything enqueued on them later (once for both
  // parts: a part that waited for the handles' streams after the other part
  // had been ordered before them would wait for that whole part)
  std::vector<hipStream_t> hstreams;
  for (int32_t i = 0; i < count; ++i)
    if (hs[i]->stream != st &&
        std::find(hstreams.begin(), hstreams.end(), hs[i]->stream) == hstreams.end())
      hstreams.push_back(hs[i]->stream);
  BT(hipEventRecord(sp.start, st));
  BT(hipStreamWaitEvent(sp.s, sp.start, 0));
  BT(hipStreamWaitEvent(sp.s2, sp.start, 0));
  for (hipStream_t hx : hstreams) {
    hipEvent_t ev;
    BT(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    BT(hipEventRecord(ev, hx));
    BT(hipStreamWaitEvent(sp.s, ev, 0));
    BT(hipStreamWaitEvent(sp.s2, ev, 0));
    BT(hipEventDestroy(ev));
  }
  faco_batch_config big = cfg;
  big.persistent = 0;
  big.team_waves = cfg.big_team_waves;
  big.big_percent = 0;
  faco_batch_config small = cfg;
  small.big_percent = 0;
  int rc = run_batch_one(order.data(), nbig, iterations, sp.s, big, false);
  if (rc) return rc;
  rc = run_batch_one(order.data() + nbig, count - nbig, iterations, sp.s2, small, false);
  if (rc) return rc;
  BT(hipEventRecord(sp.done, sp.s));
  BT(hipEventRecord(sp.done2, sp.s2));
  BT(hipStreamWaitEvent(st, sp.done, 0));
  BT(hipStreamWaitEvent(st, sp.done2, 0));
  for (hipStream_t hx : hstreams) {
    BT(hipStreamWaitEvent(hx, sp.done, 0));
    BT(hipStreamWaitEvent(hx, sp.done2, 0));
  }
#undef BT
  return FACO_OK;
}

// The tuned configuration of the batch's size class, else of the nearest
// tuned class (the smaller one on a tie), else the default.
static faco_batch_config config_for(faco_instance *const *hs, int32_t count) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (g_tuned.empty()) return g_batch_cfg;
  const int c = size_class(hs, count);
  int best = -1;
  for (const auto &kv : g_tuned)
    if (best < 0 || std::abs(kv.first - c) < std::abs(best - c)) best = kv.first;
  return g_tuned[best];
}

extern "C" int faco_run_batch(faco_instance *const *hs, int32_t count, int32_t iterations,
                              void *hip_stream) {
  if (const char *m = check_batch_args(hs, count, iterations))
    return set_err(nullptr, FACO_EINVAL, m);
  if (count == 0 || iterations == 0) return FACO_OK;
  return run_batch_cfg(hs, count, iterations, (hipStream_t)hip_stream, config_for(hs, count));
}

extern "C" int faco_autotune_batch(faco_instance *const *hs, int32_t count,
                                   int32_t trial_iterations, void *hip_stream,
                                   faco_batch_config *best_out) {
  if (const char *m = check_batch_args(hs, count, trial_iterations))
    return set_err(nullptr, FACO_EINVAL, m);
  if (count == 0 || trial_iterations < 1)
    return set_err(nullptr, FACO_EINVAL, "need at least one handle and one trial iteration");
  hipStream_t st = (hipStream_t)hip_stream;
  // twins of the handles from their stored inputs: the handles themselves
  // do not move
  std::vector<faco_instance *> twins;
  auto drop = [&]() {
    for (faco_instance *t : twins) faco_destroy_instance(t);
  };
  for (int32_t i = 0; i < count; ++i) {
    faco_instance *t = nullptr;
    const int rc = faco_build_instance(hs[i]->xy_host.data(), hs[i]->n, &hs[i]->p, hip_stream, &t);
    if (rc) {
      drop();
      return rc;
    }
    twins.push_back(t);
  }
  // per phase: waves per ant, ants per workgroup, queue capacity; persistent
  // teams; the largest 10% .. 30% split off with 4- or 8-wave teams
  std::vector<faco_batch_config> cand;
  for (int tw : {1, 4, 8})
    for (int apb : {1, 2})
      for (int cap : {0, 2048}) {
        if (tw > 1 && apb > 1) continue;
        cand.push_back({0, tw, apb, cap, 0, 0});
      }
  for (int tw : {4, 8}) cand.push_back({1, tw, 1, 2048, 0, 0});
  if (count >= 4)
    for (int pct : {10, 15, 20, 30})
      for (int btw : {4, 8}) cand.push_back({0, 1, 1, 2048, pct, btw});
  // Every device block of the twins is copied aside at the start of a round
  // and copied back before each candidate's trial, so that all candidates of
  // a round run the same iterations from the same state.  Rounds lie apart
  // along the run (the work per iteration changes as it goes), and a
  // first, untimed pass runs each candidate once (first launches of its
  // kernels, its streams and tables).
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    drop();
    return set_err(nullptr, FACO_EDEVICE, "hipGetDevice failed");
  }
  std::vector<faco::CopySeg> segs;  // [save..., load...]
  size_t snap_bytes = 0;
  for (faco_instance *t : twins)
    for (auto &a : t->allocs) snap_bytes += (a.second + 255) & ~(size_t)255;
  void *snap = nullptr, *dsegs = nullptr;
  size_t snap_got = 0, segs_got = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    blk_put(dev, snap, snap_got);
    blk_put(dev, dsegs, segs_got);
    drop();
  };
  if (blk_get(dev, snap_bytes, &snap, &snap_got) != hipSuccess) {
    snap = nullptr;
    release();
    return set_err(nullptr, FACO_ENOMEM, "no device memory for the trial snapshot");
  }
  {
    size_t off = 0;
    for (faco_instance *t : twins)
      for (auto &a : t->allocs) {
        segs.push_back({(const unsigned char *)a.first, (unsigned char *)snap + off, a.second});
        off += (a.second + 255) & ~(size_t)255;
      }
    const size_t nseg = segs.size();
    for (size_t k = 0; k < nseg; ++k)
      segs.push_back({segs[k].dst, const_cast<unsigned char *>(segs[k].src), segs[k].bytes});
  }
  const int nseg = (int)(segs.size() / 2);
  if (blk_get(dev, sizeof(faco::CopySeg) * segs.size(), &dsegs, &segs_got) != hipSuccess) {
    dsegs = nullptr;
    release();
    return set_err(nullptr, FACO_ENOMEM, "no device memory for the trial snapshot");
  }
  const faco::CopySeg *d_save = (const faco::CopySeg *)dsegs, *d_load = d_save + nseg;
  auto copy = [&](const faco::CopySeg *list) {
    hipLaunchKernelGGL(faco::copy_segments_kernel, dim3((unsigned)std::min(nseg, 2048)),
                       dim3(256), 0, st, list, nseg);
    return hipGetLastError() == hipSuccess ? FACO_OK
                                           : set_err(nullptr, FACO_EDEVICE, "snapshot copy failed");
  };
  if (hipMemcpyAsync(dsegs, segs.data(), sizeof(faco::CopySeg) * segs.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    return set_err(nullptr, FACO_EDEVICE, "setting up the trials failed");
  }
  const int rounds = trial_iterations >= 3 ? 3 : 1;
  std::vector<float> total(cand.size(), 0.0f);
  int rc = copy(d_save);
  for (size_t ci = 0; ci < cand.size() && rc == FACO_OK; ++ci) {
    rc = copy(d_load);
    if (rc == FACO_OK) rc = run_batch_cfg(twins.data(), count, 1, st, cand[ci]);
  }
  if (rc == FACO_OK) rc = copy(d_load);
  for (int r = 0; r < rounds && rc == FACO_OK; ++r) {
    const int its = trial_iterations / rounds + (r < trial_iterations % rounds ? 1 : 0);
    if (r > 0) {
      faco_batch_config plain;
      {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        plain = g_batch_cfg;
      }
      rc = run_batch_cfg(twins.data(), count, 5 * its, st, plain);
    }
    if (rc == FACO_OK) rc = copy(d_save);
    for (size_t ci = 0; ci < cand.size() && rc == FACO_OK; ++ci) {
      rc = copy(d_load);
      if (rc) break;
      if (hipEventRecord(e0, st) != hipSuccess) {
        rc = set_err(nullptr, FACO_EDEVICE, "timing a trial failed");
        break;
      }
      rc = run_batch_cfg(twins.data(), count, its, st, cand[ci]);
      if (rc) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = set_err(nullptr, FACO_EDEVICE, "timing a trial failed");
        break;
      }
      total[ci] += ms;
    }
  }
  faco_batch_config best = g_batch_cfg;
  for (size_t ci = 0, bi = 0; ci < cand.size() && rc == FACO_OK; ++ci)
    if (ci == 0 || total[ci] < total[bi]) {
      bi = ci;
      best = cand[ci];
    }
  release();
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    g_tuned[size_class(hs, count)] = best;
  }
  if (best_out) *best_out = best;
  return FACO_OK;
}

// ------------------------------------------------------------------------
// faco_run_batch_noalloc: the launches of faco_run_batch with the instance
// and ant tables in a fixed device array instead of an allocated workspace,
// and without graph capture or events.

constexpr int kNoAllocMaxInstances = 256;
constexpr int kNoAllocMaxAnts = 16384;
constexpr size_t kScratchInstBytes = (size_t)kNoAllocMaxInstances * sizeof(Inst);
constexpr size_t kScratchBytes = 256 * 1024;
static_assert(kScratchInstBytes % 256 == 0, "ant table must stay aligned");
static_assert(kScratchInstBytes + (size_t)kNoAllocMaxAnts * sizeof(int2) <= kScratchBytes,
              "tables exceed the fixed array");

// Each device holds its own copy until the process ends.  In host code the
// name is a stand-in for the symbol only: the device address of each copy
// comes from hipGetSymbolAddress and is the only thing passed to copies and
// kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_dev[kMaxDevices];  // looked up once per device

// Device address of `scratch` on device dev (which must be current).
static int scratch_address(int dev, unsigned char **out) {
  if (dev < 0 || dev >= kMaxDevices) return set_err(nullptr, FACO_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_err(nullptr, FACO_EDEVICE,
                     std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (unsigned char *)ptr;
  }
  *out = g_scratch_dev[dev];
  return FACO_OK;
}

// host staging of the tables (guarded by g_batch_mu)
static Inst g_na_insts[kNoAllocMaxInstances];
static int2 g_na_amap[kNoAllocMaxAnts];

extern "C" int faco_run_batch_noalloc(faco_instance *const *hs, int32_t count,
                                      int32_t iterations, void *hip_stream) {
  if (const char *m = check_batch_args(hs, count, iterations))
    return set_err(nullptr, FACO_EINVAL, m);
  if (count == 0 || iterations == 0) return FACO_OK;
  if (count > kNoAllocMaxInstances)
    return set_err(nullptr, FACO_EINVAL,
                   "faco_run_batch_noalloc: at most 256 instances per call");
  if (batch_ant_count(hs, count) > kNoAllocMaxAnts)
    return set_err(nullptr, FACO_EINVAL,
                   "faco_run_batch_noalloc: at most 16384 ants per call (all instances)");
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0;
  hipError_t e;
#define BT(expr)                                                                      \
  if ((e = (expr)) != hipSuccess)                                                     \
    return set_err(nullptr, FACO_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e));
  BT(hipGetDevice(&dev));
  for (int32_t i = 0; i < count; ++i) {
    if (hs[i]->stream != st)
      return set_err(nullptr, FACO_EINVAL,
                     "faco_run_batch_noalloc: every handle must run on hip_stream");
    if (hs[i]->device != dev)
      return set_err(nullptr, FACO_EINVAL,
                     "faco_run_batch_noalloc: every handle must live on the current device");
  }
  unsigned char *base = nullptr;
  if (int rc = scratch_address(dev, &base)) return rc;
  Inst *d_insts = reinterpret_cast<Inst *>(base);
  int2 *d_amap = reinterpret_cast<int2 *>(base + kScratchInstBytes);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  BatchShape B;
  batch_shape(hs, count, g_na_insts, g_na_amap, g_batch_cfg, B);
  BT(hipMemcpyAsync(d_insts, g_na_insts, sizeof(Inst) * (size_t)count, hipMemcpyHostToDevice,
                    st));
  BT(hipMemcpyAsync(d_amap, g_na_amap, sizeof(int2) * (size_t)B.total, hipMemcpyHostToDevice,
                    st));
  BT(hipFuncSetAttribute((const void *)B.antk, hipFuncAttributeMaxDynamicSharedMemorySize,
                         (int)B.lds_bytes));
  for (int32_t it = 0; it < iterations; ++it) enqueue_batch_iteration(B, d_insts, d_amap, st);
  BT(hipGetLastError());
#undef BT
  return FACO_OK;
}
