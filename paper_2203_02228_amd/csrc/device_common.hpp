// device_common.hpp -- wave64 helpers, EUC_2D cost and Philox4x64-10 for the
// FACO kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FACO_DEV __device__ __forceinline__

namespace faco {

constexpr int kWave = 64;

// ---------------------------------------------------------------- wave ---

FACO_DEV int lane_id() { return (int)__lane_id(); }

FACO_DEV uint64_t ballot(bool p) { return (uint64_t)__ballot((int)p); }

FACO_DEV int ctz64(uint64_t m) { return __builtin_ctzll(m); }
FACO_DEV int msb64(uint64_t m) { return 63 - __builtin_clzll(m); }

FACO_DEV int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
FACO_DEV float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
FACO_DEV int64_t readlane_i64(int64_t v, int l) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
FACO_DEV int2 readlane_i2(int2 v, int l) {
  return make_int2(readlane_i(v.x, l), readlane_i(v.y, l));
}

FACO_DEV int64_t shfl_xor_i64(int64_t v, int m) {
  int lo = __shfl_xor((int)(uint32_t)v, m);
  int hi = __shfl_xor((int)(uint32_t)(v >> 32), m);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// Data-parallel-primitive (DPP) moves within rows of 16 lanes: the quad
// permutations [1,0,3,2] and [2,3,0,1], the half-row mirror (lane i <-> 7-i)
// and the row mirror (i <-> 15-i).  Applied in that order with a combining
// operation they leave every lane of a row holding the row's combination.
constexpr int kDppQuad1032 = 0xB1;
constexpr int kDppQuad2301 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
FACO_DEV int dpp_i(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
FACO_DEV int64_t dpp_i64(int64_t v) {
  const uint32_t lo = (uint32_t)dpp_i<CTRL>((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)dpp_i<CTRL>((int)(uint32_t)(v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane j of each 16-lane row to the whole row (DPP row broadcast, CDNA3+).
FACO_DEV int row_bcast(int v, int j) {
  switch (j) {
#define FACO_BC(J) \
  case J:          \
    return dpp_i<0x150 + J>(v);
    FACO_BC(0) FACO_BC(1) FACO_BC(2) FACO_BC(3) FACO_BC(4) FACO_BC(5) FACO_BC(6) FACO_BC(7)
    FACO_BC(8) FACO_BC(9) FACO_BC(10) FACO_BC(11) FACO_BC(12) FACO_BC(13) FACO_BC(14)
    FACO_BC(15)
#undef FACO_BC
  }
  return v;
}

struct OpMax { template <class T> FACO_DEV T operator()(T a, T b) const { return a > b ? a : b; } };
struct OpMin { template <class T> FACO_DEV T operator()(T a, T b) const { return a < b ? a : b; } };
struct OpAdd { template <class T> FACO_DEV T operator()(T a, T b) const { return a + b; } };

template <class Op>
FACO_DEV int64_t row_reduce_i64(int64_t v, Op op) {
  v = op(v, dpp_i64<kDppQuad1032>(v));
  v = op(v, dpp_i64<kDppQuad2301>(v));
  v = op(v, dpp_i64<kDppRowHalfMirror>(v));
  v = op(v, dpp_i64<kDppRowMirror>(v));
  return v;
}
template <class Op>
FACO_DEV int row_reduce_i32(int v, Op op) {
  v = op(v, dpp_i<kDppQuad1032>(v));
  v = op(v, dpp_i<kDppQuad2301>(v));
  v = op(v, dpp_i<kDppRowHalfMirror>(v));
  v = op(v, dpp_i<kDppRowMirror>(v));
  return v;
}
// Whole-wave reductions: rows by DPP, then the four row results.  Every
// lane must be active; the result is uniform.
template <class Op>
FACO_DEV int64_t wave_reduce_i64(int64_t v, Op op) {
  v = row_reduce_i64(v, op);
  const int64_t r0 = readlane_i64(v, 0), r1 = readlane_i64(v, 16);
  const int64_t r2 = readlane_i64(v, 32), r3 = readlane_i64(v, 48);
  return op(op(r0, r1), op(r2, r3));
}
template <class Op>
FACO_DEV int wave_reduce_i32(int v, Op op) {
  v = row_reduce_i32(v, op);
  const int r0 = readlane_i(v, 0), r1 = readlane_i(v, 16);
  const int r2 = readlane_i(v, 32), r3 = readlane_i(v, 48);
  return op(op(r0, r1), op(r2, r3));
}
FACO_DEV int64_t wave_max_i64(int64_t v) { return wave_reduce_i64(v, OpMax()); }
FACO_DEV int64_t wave_min_i64(int64_t v) { return wave_reduce_i64(v, OpMin()); }
FACO_DEV int64_t wave_sum_i64(int64_t v) { return wave_reduce_i64(v, OpAdd()); }
FACO_DEV int wave_sum_i32(int v) { return wave_reduce_i32(v, OpAdd()); }
FACO_DEV int wave_min_i32(int v) { return wave_reduce_i32(v, OpMin()); }

// A value every lane holds alike, moved to a scalar register: control flow
// on it is a scalar branch (needed where a workgroup barrier follows).
FACO_DEV int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
FACO_DEV uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Workgroup barrier; global and LDS writes before it are visible to every
// wave of the workgroup after it.
FACO_DEV void team_sync() { __syncthreads(); }

// Order this wave's LDS writes before its later LDS reads (a write by one
// lane read back by all).
FACO_DEV void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Make this wave's global and LDS writes visible to its other lanes.
FACO_DEV void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// -------------------------------------------- device-wide coordination ---
// Relaxed atomics at agent (device) scope, and the fences that order plain
// memory accesses around them (a release fence before publishing, an acquire
// fence after observing).

FACO_DEV int ld_agent(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
FACO_DEV void st_agent(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
FACO_DEV int add_agent(int *p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
FACO_DEV int64_t ld_agent64(const int64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// compare-and-swap; returns the value found
FACO_DEV int64_t cas_agent64(int64_t *p, int64_t expected, int64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;
}
FACO_DEV void fence_acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
FACO_DEV void fence_release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// --------------------------------------------------------------- bitmap ---

FACO_DEV bool bit_get(const uint32_t *bm, int x) {
  return (bm[x >> 5] >> (x & 31)) & 1u;
}
FACO_DEV void bit_set(uint32_t *bm, int x) { atomicOr(&bm[x >> 5], 1u << (x & 31)); }
FACO_DEV void bit_clear(uint32_t *bm, int x) {
  atomicAnd(&bm[x >> 5], ~(1u << (x & 31)));
}

// ---------------------------------------------------------------- cost ---
// TSPLIB EUC_2D: nint(sqrt(dx^2 + dy^2)).  With |dx|,|dy| < 2^26 the squared
// length is an exact integer below 2^53 in binary64.

FACO_DEV double sqd(int2 a, int2 b) {
  double dx = (double)(a.x - b.x);
  double dy = (double)(a.y - b.y);
  return dx * dx + dy * dy;
}
FACO_DEV uint64_t sqd_u64(int2 a, int2 b) {
  const int dx = a.x - b.x, dy = a.y - b.y;
  const uint32_t ax = (uint32_t)(dx < 0 ? -dx : dx), ay = (uint32_t)(dy < 0 ? -dy : dy);
  return (uint64_t)ax * ax + (uint64_t)ay * ay;
}
// nint(sqrt(d2)) for an integer d2 < 2^53 (held exactly).  It is the unique
// C >= 0 with C^2 - C < d2 <= C^2 + C (d2 = 0: C = 0), because sqrt(d2) is
// never a half-integer.  The hardware square root estimates sqrt(d2) to far
// better than +-0.5, so its nearest integer r is C or a neighbour.  The fused
// multiply-add gives e = r^2 - d2 exactly (a small integer; the product is
// not rounded), and C = r unless e < -r (C = r + 1) or e >= r > 0 (C = r - 1).
FACO_DEV int nint_sqrt(double d2) {
  const double r = __builtin_rint(__builtin_amdgcn_sqrt(d2));
  const double e = __builtin_fma(r, r, -d2);
  return (int)r + (e < -r ? 1 : 0) - (e >= r && r > 0.0 ? 1 : 0);
}

FACO_DEV int cost(int2 a, int2 b) {
  // dy^2 < 2^52 and dx^2 + dy^2 < 2^53 are exact; the fused form rounds once
  const double dx = (double)(a.x - b.x), dy = (double)(a.y - b.y);
  return nint_sqrt(__builtin_fma(dx, dx, dy * dy));
}

// ----------------------------------------------------------- Philox4x64 ---
// Salmon et al., SC'11: 10 rounds, multipliers M0, M1, Weyl key increments.

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

enum : uint64_t {
  kPurposeRoulette = 0,
  kPurposeStart = 1,
  kPurposeSource = 2,
  kPurposeNewEdges = 3
};

// Full 128-bit product m * x from four 32 x 32 -> 64 partial products, each
// with the carry-in folded into its addend (no partial sum overflows 64 bits:
// (2^32 - 1)^2 + 2 (2^32 - 1) = 2^64 - 1), so each is one multiply-add.
FACO_DEV void mulhilo64(uint64_t m, uint64_t x, uint64_t &hi, uint64_t &lo) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t m0 = (uint32_t)m, m1 = (uint32_t)(m >> 32);
  const uint64_t p00 = (uint64_t)x0 * m0;
  const uint64_t t = (uint64_t)x1 * m0 + (p00 >> 32);
  const uint64_t u = (uint64_t)x0 * m1 + (uint32_t)t;
  hi = (uint64_t)x1 * m1 + ((t >> 32) + (u >> 32));
  lo = (u << 32) | (uint32_t)p00;
}

FACO_DEV uint64_t philox_word0(uint64_t key0, uint64_t c0, uint64_t c1,
                               uint64_t c2, uint64_t c3) {
  uint64_t k0 = key0, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(kM0, c0, hi0, lo0);
    mulhilo64(kM1, c2, hi1, lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// top 24 bits as an exact binary32 in [0, 1)
FACO_DEV float unit24(uint64_t x) {
  return (float)(uint32_t)(x >> 40) * 0x1p-24f;
}
// floor(x * n / 2^64)
FACO_DEV int uniform_node(uint64_t x, int n) {
  return (int)__umul64hi(x, (uint64_t)n);
}

}  // namespace faco
