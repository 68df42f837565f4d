// faco_aux.hpp -- per-iteration colony, source and pheromone kernels, the
// batched forms of those, and the candidate/backup list builder (gfx950).
#pragma once
#include "device_common.hpp"
#include "faco_device.hpp"
#include "faco_update.hpp"

namespace faco {

__global__ void __launch_bounds__(64) colony_kernel(Inst I) { run_colony(I); }

__global__ void __launch_bounds__(256) source_kernel(Inst I, int init) {
  run_source(I, (int)(blockIdx.x * blockDim.x + threadIdx.x), init);
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
// Tour-length verification: every ant's tour (when `ants` is set) and the
// global best are summed again from the stored tours and the coordinates
// (int64, exact), and each ant's route is checked against its inverse
// (route[pos[c]] = c for every position: a permutation).  The sums are
// compared with the lengths the construction and local search tracked; a
// mismatch sets a fault.  Partial sums accumulate in vsum/vbad (zero
// between verifications; the finishing kernel reads and clears them).
//   verify: grid (chunks, A + 1 tours), block kVerifyBlock
// ===================================================================== //
constexpr int kVerifyBlock = 256;

FACO_DEV void verify_part(const Inst &I, int tour, int ants, int chunk, int nchunks) {
  const int n = I.n;
  const bool gb = tour == I.A;
  if (!gb && !ants) return;
  const int32_t *r = gb ? I.gb_route : ant_route(I, tour);
  const int32_t *pos = gb ? nullptr : ant_pos(I, tour);
  int64_t s = 0;
  bool bad = false;
  for (int i = chunk * kVerifyBlock + (int)threadIdx.x; i < n; i += nchunks * kVerifyBlock) {
    const int c = r[i], d = r[i + 1 == n ? 0 : i + 1];
    if ((unsigned)c >= (unsigned)n || (unsigned)d >= (unsigned)n) {
      bad = true;
      continue;
    }
    if (pos && pos[c] != i) bad = true;
    s += cost(I.xy[c], I.xy[d]);
  }
  s = wave_sum_i64(s);
  const bool wbad = ballot(bad) != 0;
  if (lane_id() == 0) {
    if (s) atomicAdd((unsigned long long *)&I.vsum[tour], (unsigned long long)s);
    if (wbad) atomicOr(&I.vbad[tour], 1);
  }
}

// Compare, publish the recomputed lengths in vout, clear the partial sums.
// iter_ahead: 1 when the ants being checked belong to the iteration in
// progress (before the colony update counts it), else 0.
FACO_DEV void verify_finish(const Inst &I, int ants, int iter_ahead) {
  DevState *st = I.st;
  for (int t = (int)threadIdx.x; t <= I.A; t += (int)blockDim.x) {
    if (t < I.A && !ants) continue;
    const int64_t L = I.vsum[t];
    const bool bad = I.vbad[t] != 0;
    const int64_t want = t < I.A ? I.lens[t] : st->gb_len;
    I.vout[t] = bad ? -1 : L;
    if (bad || L != want) {
      const int32_t bit = bad ? FAULT_PERMUTATION : FAULT_LENGTH;
      if (atomicOr(&st->fault, bit) == 0) {
        st->fault_ant = t < I.A ? t : -1;
        st->fault_iter = st->iter + iter_ahead;
      }
    }
    I.vsum[t] = 0;
    I.vbad[t] = 0;
  }
  if (threadIdx.x == 0) st->verified += (ants ? I.A : 0) + 1;
}

__global__ void __launch_bounds__(kVerifyBlock) verify_kernel(Inst I, int ants) {
  verify_part(I, (int)blockIdx.y, ants, (int)blockIdx.x, (int)gridDim.x);
}
__global__ void __launch_bounds__(kVerifyBlock) verify_finish_kernel(Inst I, int ants,
                                                                     int iter_ahead) {
  verify_finish(I, ants, iter_ahead);
}

// chunks per tour of a verification launch
__host__ __device__ inline unsigned verify_chunks(int n) {
  const int c = (n + 4 * kVerifyBlock - 1) / (4 * kVerifyBlock);
  return (unsigned)(c < 1 ? 1 : (c > 128 ? 128 : c));
}

// ===================================================================== //
// Batched forms: blockIdx selects the instance; each instance reads only
// its own Inst.
// ===================================================================== //
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

// blockIdx.z = instance; instances without verification, and tours or
// chunks past an instance's own, return
__global__ void __launch_bounds__(kVerifyBlock) verify_batch_kernel(const Inst *insts) {
  const Inst &I = insts[blockIdx.z];
  if (!I.verify || (int)blockIdx.y > I.A) return;
  const unsigned nc = verify_chunks(I.n);
  if (blockIdx.x >= nc) return;
  verify_part(I, (int)blockIdx.y, 1, (int)blockIdx.x, (int)nc);
}
__global__ void __launch_bounds__(kVerifyBlock) verify_finish_batch_kernel(const Inst *insts) {
  const Inst &I = insts[blockIdx.x];
  if (I.verify) verify_finish(I, 1, 1);
}

// ===================================================================== //
// Candidate + backup lists (Sec. 4.1): the K + BL nearest cities by
// (squared distance, original number); eta = 1/d.  One query city per lane
// (64 consecutive labels per workgroup); each lane keeps its list sorted in
// LDS.  Labels follow the Hilbert curve, so each run of 32 labels is a
// compact box (wbox).  The wave visits the runs outward from its own in label
// order (near cities first, so the lists fill with close cities early) and
// skips a run when every lane's list is full and the run's box lies strictly
// farther than the lane's last kept entry.  A skipped run holds no city that
// could enter a list (a tie at the last entry's distance is still examined),
// and the kept set does not depend on the visiting order: the lists are
// exactly those of a scan over all cities.
// ===================================================================== //
constexpr int kKnnRun = 32;

__global__ void __launch_bounds__(64) knn_kernel(const int2 *xy, const int32_t *orig_of,
                                                 const int32_t *int_of, const int4 *wbox,
                                                 int n, int K, int BL, int32_t *cl,
                                                 int32_t *bll, float *eta, int32_t *cl_d,
                                                 DevState *st) {
  extern __shared__ unsigned char knn_lds[];
  const int KK = K + BL;
  const int tid = threadIdx.x;
  double *kd = reinterpret_cast<double *>(knn_lds);
  int32_t *ko = reinterpret_cast<int32_t *>(knn_lds + sizeof(double) * (size_t)KK * 64);
  const int i = blockIdx.x * 64 + tid;
  const bool valid = i < n;
  const int2 xi = valid ? xy[i] : make_int2(0, 0);
  const int oi = valid ? orig_of[i] : -1;
  const int nrun = (n + kKnnRun - 1) / kKnnRun;
  const int c0 = (blockIdx.x * 64) / kKnnRun;
  const int reach = c0 > nrun - 1 - c0 ? c0 : nrun - 1 - c0;
  int cnt = 0;
  double worst = 0.0;
  int worst_o = 0;
  for (int d = 0; d <= reach; ++d) {
    for (int side = 0; side < 2; ++side) {
      if (d == 0 && side == 1) break;
      const int c = side == 0 ? c0 + d : c0 - d;
      if (c < 0 || c >= nrun) continue;
      // does any lane still need this run?
      bool need = valid;
      if (valid && cnt == KK) {
        const int4 b = wbox[c];
        const int dx = max(max(b.x - xi.x, xi.x - b.z), 0);
        const int dy = max(max(b.y - xi.y, xi.y - b.w), 0);
        const double bd = (double)dx * (double)dx + (double)dy * (double)dy;
        need = !(bd > worst);
      }
      if (!__any(need)) continue;
      const int base = c * kKnnRun;
      const int tn = min(kKnnRun, n - base);
      if (!need) continue;
      for (int jj = 0; jj < tn; ++jj) {
        const int oj = orig_of[base + jj];
        if (oj == oi) continue;
        const double dd = sqd(xi, xy[base + jj]);
        // the list is sorted by (squared distance, original number)
        if (cnt == KK && !(dd < worst || (dd == worst && oj < worst_o))) continue;
        int q = cnt < KK ? cnt++ : KK - 1;
        while (q > 0 && (kd[(q - 1) * 64 + tid] > dd ||
                         (kd[(q - 1) * 64 + tid] == dd && ko[(q - 1) * 64 + tid] > oj))) {
          kd[q * 64 + tid] = kd[(q - 1) * 64 + tid];
          ko[q * 64 + tid] = ko[(q - 1) * 64 + tid];
          --q;
        }
        kd[q * 64 + tid] = dd;
        ko[q * 64 + tid] = oj;
        if (cnt == KK) {
          worst = kd[(KK - 1) * 64 + tid];
          worst_o = ko[(KK - 1) * 64 + tid];
        }
      }
    }
  }
  if (!valid) return;
  for (int s = 0; s < K; ++s) {
    const double d2 = kd[s * 64 + tid];
    cl[(size_t)i * K + s] = int_of[ko[s * 64 + tid]];
    const int d = nint_sqrt(d2);
    cl_d[(size_t)i * K + s] = d;
    eta[(size_t)i * K + s] = (float)(1.0 / (double)d);
  }
  for (int s = 0; s < BL; ++s) bll[(size_t)i * BL + s] = int_of[ko[(K + s) * 64 + tid]];
  if (kd[tid] == 0.0) atomicOr(&st->dup, 1);
}

// ===================================================================== //
// Device-to-device copies of a list of blocks (the autotuner's snapshot and
// restore of its trial instances): one workgroup per block at a time, 16-byte
// words while both addresses are 16-byte aligned, single bytes for the rest.
// ===================================================================== //
struct CopySeg {
  const unsigned char *src;
  unsigned char *dst;
  uint64_t bytes;
};

__global__ void __launch_bounds__(256) copy_segments_kernel(const CopySeg *segs, int nseg) {
  for (int s = blockIdx.x; s < nseg; s += gridDim.x) {
    const CopySeg g = segs[s];
    const bool vec = (((uintptr_t)g.src | (uintptr_t)g.dst) & 15u) == 0;
    const uint64_t nv = vec ? g.bytes / 16 : 0;
    const uint4 *sv = reinterpret_cast<const uint4 *>(g.src);
    uint4 *dv = reinterpret_cast<uint4 *>(g.dst);
    for (uint64_t k = threadIdx.x; k < nv; k += blockDim.x) dv[k] = sv[k];
    for (uint64_t k = nv * 16 + threadIdx.x; k < g.bytes; k += blockDim.x) g.dst[k] = g.src[k];
  }
}

}  // namespace faco
