// Per-map finisher of the batched PCG: reduces one map's FP64 tile partials
// and advances its state machine (Algorithm 1's scalar steps: alpha, beta,
// the stop tests).  Runs either as its own kernel (one block per map) or at
// the end of the tile kernel whose partials it reduces, in the block whose
// tile of the map finished last.
#pragma once

#include "lpu_internal.h"
#include "lpu_device.h"

namespace lpu {

enum FinOp : int {
  kFinInit = 0,     // slots 0,1,2 over stencil tiles: r.r, r.s, b.b
  kFinAlpha = 1,    // slot 0: d^T q
  kFinUpdate = 2,   // slots 0,1: r.r, r.s
  kFinConfirm = 3,  // slots 0,1: r.r, r.s
  kFinTail = 4,     // slot 1 over DCT tiles (or one sweep partial): r.s
  kFinSum2 = 5,     // slots 0,1 over stencil tiles -> rr, bb (no state change)
  kFinTailS = 6     // slot 1 over stencil tiles (two-colour preconditioners): r.s
};

__device__ inline void map_finish(MapState& s, int mode, double rs) {
  if (mode == kFinishIter) {
    s.delta_old = s.delta_new;
    s.delta_new = rs;
    s.beta = rs / s.delta_old;
    s.l += 1;
  } else if (mode == kFinishConfirm) {
    s.delta_new = rs;
    s.beta = rs / s.delta_old;
  } else {
    s.delta_new = rs;
    s.delta0 = rs;
    s.beta = 0.0;
    s.thr_delta = s.eps2 * rs;
  }
  s.nfinish += 1;
  int st = kRun;
  if (s.rule == LPU_STOP_PAPER) {
    if (!(s.delta_new > s.thr_delta)) st = kDone;
  } else if (s.rr <= s.thr_rr && (s.replaced || mode != kFinishIter)) {
    st = kDone;
  }
  if (st == kRun) {
    if (!isfinite(s.delta_new) || s.delta_new < 0.0 || !isfinite(s.beta)) st = kBreakdown;
    else if (s.l >= s.l_max) st = kCap;
  }
  s.state = st;
}

// Stagnation of a mixed-precision inner solve.  Checkpoints are the true
// residuals the iteration forms anyway (periodic replacements and failed
// confirmations).  Two checkpoints at least chk_gap iterations apart are
// compared (chk_gap = min(MN, max(period, 256)): in exact arithmetic CG ends
// within MN iterations, and over shorter spans the residual norm of CG need
// not decrease); if the later one is still above the bound and not at least
// 10 % (in norm) below the earlier one, the FP32 iterate has reached what its
// precision can resolve and the solve stops; the FP64 refinement around it
// continues from its iterate.
__device__ inline bool stagnated(MapState& s, double rr_true) {
  if (!s.stall || s.rule != LPU_STOP_RELRES || rr_true <= s.thr_rr) return false;
  if (s.rr_chk <= 0.0) {
    s.rr_chk = rr_true;
    s.l_chk = s.l;
    return false;
  }
  if (s.l - s.l_chk < s.chk_gap) return false;
  const bool stuck = rr_true >= 0.81 * s.rr_chk;
  s.rr_chk = rr_true;
  s.l_chk = s.l;
  return stuck;
}

// Tile partials are exchanged through agent-coherent accesses (see last_arrival).
__device__ __forceinline__ void store_partial(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_partial(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where a finisher reads a map's sums: the tile partials (P, one row of
// pstride doubles per slot), or the group sums a fused kernel published
// (gsum, one row of gstride doubles per entry of the op's slot list).
struct FinSrc {
  const double* P;
  long long pstride;
  const double* gsum;
  long long gstride;
};

// Association of the sums over a map's tiles.  They are fixed functions of
// the map and the kernel (so runs are bit-reproducible and a map's result
// does not depend on its batch-mates or on the launch shape):
//  * flat (standalone finishers, and fused ones whose block reads every
//    partial in one round of at most kFlatLoads loads per thread): thread t
//    adds partials t, t + blockDim, ... in order, then a fixed tree adds the
//    threads;
//  * grouped (fused finishers of larger maps): the tiles in groups of
//    kArriveGroup consecutive tiles, a group's sum a pairwise tree over its
//    32 partials (absent tiles count as 0), formed by the block that
//    completes the group (last_arrival); the map's sum then formed by one
//    wave, lane k adding the sums of groups k, k + 64, ... in order, then a
//    pairwise tree over the 64 lanes.  The map's last block reads one value
//    per group instead of every tile's partial.
constexpr int kFlatLoads = 8;
static_assert(kArriveGroup == 32, "a group's sum is a tree over half a wave");

__device__ __forceinline__ double tree32(double v) {  // lanes 0 and 32: the sum of their half
#pragma unroll
  for (int off = 16; off > 0; off >>= 1) v += __shfl_down(v, off, 32);
  return v;
}
__device__ __forceinline__ double tree64(double v) {  // lane 0: the sum of the wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Flat sums of `count` tile partials from `first`, one per entry of `slots`;
// every thread of the block takes part; the result is valid in thread 0.
// smem: 3 * blockDim.x / 64 doubles.
template <int NS>
__device__ __forceinline__ void fin_sums_flat(const double* __restrict__ P, long long pstride,
                                              int first, int count, const int (&slots)[NS],
                                              double (&out)[NS], double* smem) {
  // The loads of kFlatLoads consecutive terms are issued together, since
  // they go to the level the XCDs share and a chain of single loads would put
  // their full latency on the map's finisher, often the last work of a launch.
  constexpr int kU = kFlatLoads;
  const int nb = blockDim.x;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double* base = P + slots[k] * pstride + first;
    double v = 0.0;
    for (int t0 = threadIdx.x; t0 < count; t0 += kU * nb) {
      double x[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int t = t0 + u * nb;
        x[u] = t < count ? load_partial(base + t) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (t0 + u * nb < count) v += x[u];
    }
    out[k] = v;
  }
  block_sum<NS>(out, smem);
}

// Grouped sums from the group sums of `ngrp` groups from `gbase`; wave 0
// only (the other waves' results are zeros); the result is valid in thread 0.
template <int NS>
__device__ __forceinline__ void fin_sums_groups(const double* __restrict__ gsum, long long gstride,
                                                int gbase, int ngrp, double (&out)[NS]) {
  constexpr int kU = 4;  // few registers: the finisher is fused into tile kernels
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double* base = gsum + k * gstride + gbase;
    double acc = 0.0;
    if (threadIdx.x < 64) {
      for (int j0 = 0; j0 < ngrp; j0 += 64 * kU) {
        double x[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int j = j0 + 64 * u + lane;
          x[u] = j < ngrp ? load_partial(base + j) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (j0 + 64 * u + lane < ngrp) acc += x[u];
      }
    }
    out[k] = tree64(acc);
  }
}

// GROUPS: from the group sums (a fused finisher of a large map), else flat
template <bool GROUPS, int NS>
__device__ __forceinline__ void fin_sums(const FinSrc& src, int first, int count, int gbase,
                                         const int (&slots)[NS], double (&out)[NS], double* smem) {
  if constexpr (GROUPS)
    fin_sums_groups<NS>(src.gsum, src.gstride, gbase, (count + kArriveGroup - 1) / kArriveGroup,
                        out);
  else
    fin_sums_flat<NS>(src.P, src.pstride, first, count, slots, out, smem);
}

// One map's finisher, executed by every thread of the calling block (any
// multiple of 64 threads); GROUPS: the sums from the group sums (smem
// unused), else flat (smem: 3 * blockDim.x / 64 doubles).
template <bool GROUPS>
__device__ inline void finish_map(const MapDesc* __restrict__ desc, MapState* ms, const FinSrc& src,
                                  int m, int op, int mode, int pointwise, double* smem) {
  MapState& s = ms[m];
  const MapDesc& d = desc[m];
  double v[3] = {0.0, 0.0, 0.0};
  if (op == kFinInit) {
    // three slots: standalone finishers only (fused_finish rejects the op)
    if constexpr (!GROUPS) {
      const int sl[3] = {0, 1, 2};
      fin_sums<GROUPS, 3>(src, d.tile0, d.ntiles, d.gb, sl, v, smem);
    }
  } else if (op == kFinAlpha) {
    const int sl[1] = {0};
    double w[1];
    fin_sums<GROUPS, 1>(src, d.tile0, d.ntiles, d.gb, sl, w, smem);
    v[0] = w[0];
  } else if (op == kFinTail) {
    const int sl[1] = {1};
    double w[1];
    fin_sums<GROUPS, 1>(src, d.dtile0, d.ndt, d.gbd, sl, w, smem);
    v[0] = w[0];
  } else if (op == kFinTailS) {
    const int sl[1] = {1};
    double w[1];
    fin_sums<GROUPS, 1>(src, d.tile0, d.ntiles, d.gb, sl, w, smem);
    v[0] = w[0];
  } else {
    const int sl[2] = {0, 1};
    double w[2];
    fin_sums<GROUPS, 2>(src, d.tile0, d.ntiles, d.gb, sl, w, smem);
    v[0] = w[0];
    v[1] = w[1];
  }
  if (threadIdx.x != 0) return;
  switch (op) {
    case kFinInit:
      s.rr = v[0];
      s.bb = v[2];
      s.thr_rr = s.tol2 * v[2];
      s.l = 0;
      s.replaced = 1;
      s.alpha_p = 0.0;
      s.xi = 0;
      if (v[2] == 0.0) s.state = kDone;
      else if (pointwise) map_finish(s, kFinishInit, v[1]);
      else s.state = kInitPc;
      break;
    case kFinAlpha:
      s.alpha_p = 0.0;  // every tile of the SpMV has added the pending term
      s.dq = v[0];
      if (!(v[0] > 0.0) || !isfinite(v[0]) || (s.brk_at > 0 && s.l + 1 >= s.brk_at))
        s.state = kBreakdown;
      else s.alpha = s.delta_new / v[0];
      break;
    case kFinUpdate: {
      const bool replace = (s.l % s.period) == 0;
      s.rr = v[0];
      s.replaced = replace ? 1 : 0;
      // a replacement wrote x + alpha d to the other buffer; otherwise the
      // step alpha d is left to the next SpMV (x is not needed before it)
      if (replace) s.xi ^= 1;
      s.alpha_p = replace ? 0.0 : s.alpha;
      if (replace && stagnated(s, v[0])) {
        s.delta_old = s.delta_new;
        s.l += 1;  // the iterate of this update is the one returned
        s.state = kStall;
      } else if (s.rule == LPU_STOP_RELRES && !replace && v[0] <= s.thr_rr) {
        s.delta_old = s.delta_new;
        s.l += 1;
        s.state = kConfirm;
      } else if (pointwise) {
        map_finish(s, kFinishIter, v[1]);
      }
    } break;
    case kFinConfirm:
      s.rr = v[0];
      s.replaced = 1;
      if (v[0] <= s.thr_rr) s.state = kDone;
      else if (stagnated(s, v[0])) s.state = kStall;
      else if (pointwise) map_finish(s, kFinishConfirm, v[1]);
      else s.state = kConfirmPc;
      break;
    case kFinTail:
    case kFinTailS:
      s.rs = v[0];
      s.amax[1] = s.amax[2] = s.amax[3] = 0.0f;  // scaled-fp16 maxima of this application
      map_finish(s, mode, v[0]);
      break;
    case kFinSum2:
      s.rr = v[0];
      s.bb = v[1];
      break;
  }
}

// Arrival of tile `local` (of `total`, from tile `first`) of map m, after
// its thread 0 stored the tile's partials of the op's slots with
// store_partial.  Tiles first count in their group of kArriveGroup (counter
// gcnt[gbase + local / kArriveGroup]); the block that completes a group
// counts once in the map's counter, so no counter takes more than a few
// dozen atomics (one address takes them one at a time).  For a map whose
// partials the finishing block cannot read in one round (more than
// kFlatLoads per thread), the block that completes a group first forms the
// group's sums and publishes them in gsum (row k for slots[k], column
// gbase + group).  Partials and group sums are agent-coherent stores
// (written through to the level the XCDs share) whose completion the storing
// wave waits for before its agent-scope atomic; each later arrival follows a
// returned atomic, and the blocks that read them use agent-coherent loads.
// That orders exactly the data exchanged, without an L2 write-back.
struct Arrival {
  int* fcnt;
  int* gcnt;
  double* gsum;
  long long gstride;
  const double* P;
  long long pstride;
};

__device__ __forceinline__ void wait_stores() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

enum ArrivalKind : int {
  kArrNotLast = 0,  // not the map's last block
  kArrFlat = 1,     // the map's last block: flat sums of the tile partials
  kArrGroups = 2    // the map's last block: sums of the published group sums
};

// flag is shared memory.
template <int NS>
__device__ inline int last_arrival(const Arrival& a, const int (&slots)[NS], int first, int m,
                                   int local, int total, int gbase, int* flag) {
  static_assert(NS <= 2, "one slot per half-wave");
  const int grp = local / kArriveGroup;
  const int ngrp = (total + kArriveGroup - 1) / kArriveGroup;
  const bool publish = total > kFlatLoads * (int)blockDim.x;
  if (threadIdx.x == 0) {
    wait_stores();
    const int in_grp = min(kArriveGroup, total - grp * kArriveGroup);
    int kind = kArrNotLast;
    if (__hip_atomic_fetch_add(a.gcnt + gbase + grp, 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) == in_grp - 1) {
      __hip_atomic_store(a.gcnt + gbase + grp, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      kind = kArrGroups;  // this block completed the group
      if (!publish)
        kind = __hip_atomic_fetch_add(a.fcnt + m, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                       ngrp - 1
                   ? kArrFlat
                   : kArrNotLast;
    }
    *flag = kind;
  }
  __syncthreads();
  if (!publish || *flag == kArrNotLast) return *flag;  // uniform over the block
  __syncthreads();  // every thread has read the flag
  if (threadIdx.x < 64) {
    // the group's sums: lanes 0-31 the first slot, lanes 32-63 the second
    const int lane = threadIdx.x, k = lane >> 5;
    const int t = grp * kArriveGroup + (lane & 31);
    const double x = (k < NS && t < total)
                         ? load_partial(a.P + slots[k < NS ? k : 0] * a.pstride + first + t)
                         : 0.0;
    const double v = tree32(x);
    if ((lane & 31) == 0 && k < NS) store_partial(a.gsum + k * a.gstride + gbase + grp, v);
    if (lane == 0) {
      wait_stores();
      *flag = __hip_atomic_fetch_add(a.fcnt + m, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                      ngrp - 1
                  ? kArrGroups
                  : kArrNotLast;
    }
  }
  __syncthreads();
  return *flag;
}

// The finisher fused into a tile kernel: the arrival of tile `local` (of
// `total`, from tile `first`) of map m after its partials of `slots` were
// stored, and in the block that completes the map, the map's finisher (then
// the map counter is rearmed).  flag and smem (3 * blockDim.x / 64 doubles)
// are shared memory.
template <int OP, int NS>
__device__ inline void fused_finish(const Arrival& a, const int (&slots)[NS], int first, int local,
                                    int total, int gbase, const MapDesc* desc, MapState* ms, int m,
                                    int mode, int pointwise, int* flag, double* smem) {
  static_assert(OP != kFinInit, "group sums hold two slots; the set-up sums are not fused");
  const int kind = last_arrival<NS>(a, slots, first, m, local, total, gbase, flag);
  if (kind == kArrNotLast) return;
  const FinSrc src{a.P, a.pstride, a.gsum, a.gstride};
  if (kind == kArrFlat) finish_map<false>(desc, ms, src, m, OP, mode, pointwise, smem);
  else finish_map<true>(desc, ms, src, m, OP, mode, pointwise, smem);
  if (threadIdx.x == 0) __hip_atomic_store(a.fcnt + m, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace lpu
