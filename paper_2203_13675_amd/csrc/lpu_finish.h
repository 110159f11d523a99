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

template <int NS>
__device__ __forceinline__ void fin_sums(const double* __restrict__ P, long long pstride, int first,
                                         int count, const int* slots, double (&out)[NS],
                                         double* smem) {
  // Each thread adds the partials t = tid, tid + blockDim, ... in that order;
  // the loads of eight consecutive terms are issued together, since they go
  // to the level the XCDs share and a chain of single loads would put their
  // full latency on the map's finisher, often the last work of a launch.
  constexpr int kU = 8;
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

// One map's finisher, executed by every thread of the calling block (any
// multiple of 64 threads); smem holds 3 * blockDim.x / 64 doubles.
__device__ inline void finish_map(const MapDesc* __restrict__ desc, MapState* ms,
                                  const double* __restrict__ P, long long pstride, int m, int op,
                                  int mode, int pointwise, int tail_single, double* smem) {
  MapState& s = ms[m];
  const MapDesc& d = desc[m];
  double v[3] = {0.0, 0.0, 0.0};
  if (op == kFinInit) {
    const int sl[3] = {0, 1, 2};
    fin_sums<3>(P, pstride, d.tile0, d.ntiles, sl, v, smem);
  } else if (op == kFinAlpha) {
    const int sl[1] = {0};
    double w[1];
    fin_sums<1>(P, pstride, d.tile0, d.ntiles, sl, w, smem);
    v[0] = w[0];
  } else if (op == kFinTail) {
    const int sl[1] = {1};
    double w[1];
    fin_sums<1>(P, pstride, d.dtile0, tail_single ? 1 : d.ndt, sl, w, smem);
    v[0] = w[0];
  } else if (op == kFinTailS) {
    const int sl[1] = {1};
    double w[1];
    fin_sums<1>(P, pstride, d.tile0, d.ntiles, sl, w, smem);
    v[0] = w[0];
  } else {
    const int sl[2] = {0, 1};
    double w[2];
    fin_sums<2>(P, pstride, d.tile0, d.ntiles, sl, w, smem);
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

// Arrival of tile `local` (of `total`) of map m, by thread 0 after it stored
// the tile's partials with store_partial: true in the block whose tile is the
// map's last of this launch, which then finishes the map and rearms the map
// counter.  Tiles first count in their group of kArriveGroup (counter
// gcnt[gbase + local / kArriveGroup]); the last of a group counts once in the
// map's counter, so no counter takes more than a few dozen atomics (one
// address takes them one at a time).  The partials are agent-coherent
// stores (written through to the level the XCDs share) and thread 0 waits
// for their completion before its agent-scope atomics; each later arrival
// follows a returned atomic, and the finishing block reads the partials with
// agent-coherent loads.  That orders exactly the data exchanged, without an
// L2 write-back.
__device__ inline bool last_arrival(int* fcnt, int* gcnt, int m, int local, int total, int gbase,
                                    int* flag) {
  if (threadIdx.x == 0) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    const int grp = local / kArriveGroup;
    const int in_grp = min(kArriveGroup, total - grp * kArriveGroup);
    const int ngrp = (total + kArriveGroup - 1) / kArriveGroup;
    int* gc = gcnt + gbase + grp;
    int last = 0;
    if (__hip_atomic_fetch_add(gc, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == in_grp - 1) {
      __hip_atomic_store(gc, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // rearm the group
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      last = __hip_atomic_fetch_add(fcnt + m, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
             ngrp - 1;
    }
    *flag = last;
  }
  __syncthreads();
  return *flag != 0;
}

__device__ inline void rearm(int* cnt, int m) {
  if (threadIdx.x == 0) __hip_atomic_store(cnt + m, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace lpu
