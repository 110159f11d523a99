// Natural-order ILU(0) = IC(0) and SSOR preconditioners (Section 2.1's list,
// items 3-5) across the whole device.
//
// With P the pivots and L the strict lower part of A (entries -U west, -V
// north), M = (P + L) P^{-1} (P + L^T) (times 1/(2 - omega) for SSOR, where
// P = D/omega), so s = M^{-1} r is
//   forward : y_ij = (r_ij + V_{i-1,j} y_{i-1,j} + U_{i,j-1} y_{i,j-1}) / p_ij
//   backward: z_ij = y_ij + (U_ij z_{i,j+1} + V_ij z_{i+1,j}) / p_ij,  s = c z
// (the solves multiply by 1 / p_ij, formed once per tile before its wavefront)
// (c = 2 - omega for SSOR, 1 otherwise), and the ILU(0) pivots are
//   p_ij = a_ij - U_{i,j-1}^2 / p_{i,j-1} - V_{i-1,j}^2 / p_{i-1,j}
// (a_ij the diagonal of A; below 1e-4 a_ij the pivot falls back to a_ij; an
// isolated pixel, a_ij = 0, gets 1).  Each value depends on its west and north
// neighbours (east and south for the backward solve), so the maps are cut into
// 64 x 64 tiles, the tiles with I + J = d form anti-diagonal d, and the tiles
// of one anti-diagonal are independent: one launch per anti-diagonal (tiles
// of every active map with that many diagonals), in increasing d for the
// forward solve and the pivots and from the bottom-right corner for the
// backward solve.  Inside a tile one wave runs a skewed wavefront: lane t owns
// row t and at step k handles column k - t, so the north neighbour is lane
// t - 1's value of the previous step (a DPP lane shift) and the west one its
// own; the tile's operands are staged in LDS first with coalesced row loads,
// and its results leave the same way.  Boundary values come from the tiles of
// the previous anti-diagonal.  Every kernel completes on its own (no waits
// across blocks).

#include "lpu_internal.h"
#include "lpu_device.h"
#include "lpu_finish.h"

namespace lpu {

constexpr int kWWaves = 4;               // waves per tile: all stage and store, wave 0 sweeps
constexpr int kWThreads = 64 * kWWaves;
constexpr int kWT = 64;  // tile side (rows = columns = lanes of a wave); LDS rows are kWT
                         // elements apart, so the wavefront's reads (row t, column k - t)
                         // fall in distinct banks

struct WArgs {
  const MapDesc* desc;
  MapState* ms;
  const int* mact;
  int mact_cap;  // entries of mact (its capacity)
  const int* counts;
  double* P;
  long long pstride;
  const void *U, *V, *piv, *r;
  void *s, *y;
  int expect;  // state of the maps to work on (-1: every active map)
  int diag;    // anti-diagonal index (backward solve: counted from the bottom-right)
  double omega;
  int ssor;
};

// Tile of anti-diagonal a.diag of the map in slot blockIdx.y, position
// blockIdx.x along the diagonal; false when there is none.
struct WTile {
  int m, M, N, i0, j0, local, tx;
  long long off;
};

// The lookups form a chain of memory round trips ahead of the operands: the
// active-map count, the block's map, the map's state and its descriptor.
// The map is requested with the count (through an index clamped to the
// list's capacity, used only when the slot is active) and the descriptor
// with the state, so the chain is two round trips instead of four; the
// empty asm statements keep the compiler from sinking the second load of
// each pair below the branch that follows.
template <bool REV>
__device__ __forceinline__ bool wf_tile(const WArgs& a, WTile& w) {
  const int nm = a.counts[2];
  const int m = a.mact[min((int)blockIdx.y, max(a.mact_cap - 1, 0))];
  __asm__ volatile("" ::"s"(nm), "s"(m));
  if ((int)blockIdx.y >= nm) return false;
  w.m = m;
  const MapDesc& d = a.desc[m];
  w.M = d.M;
  w.N = d.N;
  w.off = d.off;
  const int st = a.ms[m].state;
  __asm__ volatile("" ::"s"(w.M), "s"(w.N), "s"(w.off), "s"(st));
  if (a.expect >= 0 && st != a.expect) return false;
  const int ty = (d.M + kWT - 1) / kWT;
  w.tx = (d.N + kWT - 1) / kWT;
  if (a.diag >= ty + w.tx - 1) return false;
  const int imin = max(0, a.diag - w.tx + 1), imax = min(a.diag, ty - 1);
  const int I = imin + (int)blockIdx.x;
  if (I > imax) return false;
  int ti = I, tj = a.diag - I;
  if (REV) {
    ti = ty - 1 - ti;
    tj = w.tx - 1 - tj;
  }
  w.i0 = ti * kWT;
  w.j0 = tj * kWT;
  w.local = ti * w.tx + tj;
  return true;
}

// DPP whole-wave shift: lane l receives lane l-1's value (lane 0 receives 0).
__device__ __forceinline__ int wshr(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ float from_prev_lane(float v) {
  return __builtin_bit_cast(float, wshr(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double from_prev_lane(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = wshr((int)(b & 0xffffffffLL)), hi = wshr((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// DPP whole-wave shift with a fill: lane l receives lane l-1's v, lane 0 keeps
// its own value of fill.
__device__ __forceinline__ int wshr_fill(int fill, int v) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ float from_prev_lane(float fill, float v) {
  return __builtin_bit_cast(float, wshr_fill(__builtin_bit_cast(int, fill), __builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double from_prev_lane(double fill, double v) {
  const long long f = __builtin_bit_cast(long long, fill), b = __builtin_bit_cast(long long, v);
  const int lo = wshr_fill((int)(f & 0xffffffffLL), (int)(b & 0xffffffffLL));
  const int hi = wshr_fill((int)(f >> 32), (int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Lane `src` (wave-uniform) of v, in every lane.
__device__ __forceinline__ float lane_value(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double lane_value(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wf_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
using lptr = __attribute__((address_space(3))) void*;

// In-grid element (i, j) of a map, clamped into it, and whether it is inside.
__device__ __forceinline__ size_t wf_at(int i, int j, int M, int N, bool& ok) {
  ok = (unsigned)i < (unsigned)M && (unsigned)j < (unsigned)N;
  return (size_t)min(max(i, 0), M - 1) * N + min(max(j, 0), N - 1);
}

template <typename T>
__device__ __forceinline__ T wf_ld(gptr<T> a, int i, int j, int M, int N, T outside) {
  bool ok;
  const T v = a[wf_at(i, j, M, N, ok)];
  return ok ? v : outside;
}

// One 64-element vector of array a along the tile's edge, staged like the
// tile: element t at (i0 + t * di + oi, j0 + t * dj + oj), `outside` off the
// map.
template <typename T>
struct WEdge {
  T* dst;
  gptr<T> src;
  int di, dj, oi, oj;
  T outside;
};

// Stage NA arrays of the tile (dst[q][t][c] = src[q](i0 + t, j0 + c); the
// rows of each dst contiguous) and NE edge vectors straight from memory into
// LDS with LDS-direct loads, every load issued before one wait, no registers
// held.  Lanes whose element lies off the map read a clamped in-map element
// instead, and those entries are then overwritten with 0 (1 for array
// q == one) or the edge's `outside`.
template <typename T, int NA, int NE>
__device__ __forceinline__ void wf_stage(T (*const (&dst)[NA])[kWT], const gptr<T> (&src)[NA],
                                         int one, const WEdge<T> (&edge)[NE], const WTile& w) {
  constexpr int kParts = sizeof(T) / 4;  // instructions per row
  // one wave can keep at most 63 loads in flight, so every wave of the block
  // takes its share of the rows (wave wv: rows wv, wv + kWWaves, ...)
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  using gbyte = const __attribute__((address_space(1))) unsigned char*;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e % kWWaves != wv) continue;
#pragma unroll
    for (int h = 0; h < kParts; ++h) {
      const int dw = h * 64 + l, t = dw / kParts, part = dw % kParts;
      bool ok;
      const size_t at = wf_at(w.i0 + t * edge[e].di + edge[e].oi, w.j0 + t * edge[e].dj + edge[e].oj,
                              w.M, w.N, ok);
      __builtin_amdgcn_global_load_lds((gbyte)edge[e].src + at * sizeof(T) + part * 4,
                                       (lptr)((unsigned char*)edge[e].dst + h * 256), 4, 0, 0);
    }
  }
  // A tile wholly inside the map whose rows start 16-byte aligned goes in
  // 16-byte pieces, kVR rows per instruction (lane l: row l / (64 / kVR) of
  // the group, piece l % (64 / kVR)); the rest dword by dword, clamped.
  bool vec = w.i0 + kWT <= w.M && w.j0 + kWT <= w.N && (w.N * sizeof(T)) % 16 == 0;
#pragma unroll
  for (int q = 0; q < NA; ++q) vec = vec && ((size_t)src[q] & 15) == 0;
  if (vec) {
    constexpr int kVR = 64 * 16 / (kWT * (int)sizeof(T));  // rows per instruction
    const int sub = l / (64 / kVR), piece = l % (64 / kVR);
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      for (int g = wv; g < kWT / kVR; g += kWWaves) {
        const int t = g * kVR + sub;
        const size_t at = (size_t)(w.i0 + t) * w.N + w.j0;
        __builtin_amdgcn_global_load_lds((gbyte)src[q] + at * sizeof(T) + piece * 16,
                                         (lptr)&dst[q][g * kVR][0], 16, 0, 0);
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      for (int t = wv; t < kWT; t += kWWaves) {
#pragma unroll
        for (int h = 0; h < kParts; ++h) {
          // dword h * 64 + l of row t's kWT elements
          const int dw = h * 64 + l, c = dw / kParts, part = dw % kParts;
          bool ok;
          const size_t at = wf_at(w.i0 + t, w.j0 + c, w.M, w.N, ok);
          __builtin_amdgcn_global_load_lds((gbyte)src[q] + at * sizeof(T) + part * 4,
                                           (lptr)((unsigned char*)&dst[q][t][0] + h * 256), 4, 0,
                                           0);
        }
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    if (e % kWWaves != wv) continue;
    bool ok;
    (void)wf_at(w.i0 + l * edge[e].di + edge[e].oi, w.j0 + l * edge[e].dj + edge[e].oj, w.M, w.N, ok);
    if (!ok) edge[e].dst[l] = edge[e].outside;
  }
  if (w.i0 + kWT > w.M || w.j0 + kWT > w.N) {
    const int j = w.j0 + l;
    for (int t = wv; t < kWT; t += kWWaves) {
      if (w.i0 + t < w.M && j < w.N) continue;
#pragma unroll
      for (int q = 0; q < NA; ++q) dst[q][t][l] = q == one ? T(1) : T(0);
    }
  }
  __syncthreads();
}

constexpr int kWR = 8;  // steps between reading a column's operands and using them
                        // (4: 16.0 us per 1280 x 960 FP64 launch, 6: 15.1, 8: 14.9, 10: 15.0)
constexpr int kWSteps = (2 * kWT - 1 + kWR - 1) / kWR * kWR;  // wavefront steps, rounded up

// The staged pivots and U of the tile (two 64 x 64 arrays, pivots first, in
// pu's space) rewritten in place as {1 / p, U} pairs, so the solves multiply
// (no division on the wavefront's chain) and read both with one instruction.
// Every thread reads its elements before any is written.
template <typename T>
__device__ __forceinline__ void wf_pivot_pairs(T (*pu)[kWT][2]) {
  constexpr int kPer = kWT / kWWaves;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const T* staged = &pu[0][0][0];
  T pv[kPer], uv[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int t = wv + kWWaves * i;
    pv[i] = staged[t * kWT + l];
    uv[i] = staged[kWT * kWT + t * kWT + l];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int t = wv + kWWaves * i;
    pu[t][l][0] = T(1) / pv[i];
    pu[t][l][1] = uv[i];
  }
  __syncthreads();
}

// Rows of the tile back to memory, every wave taking its share.
template <typename T>
__device__ __forceinline__ void wf_store(T* out, const T (*src)[kWT], const WTile& w) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, j = w.j0 + l;
  for (int t = wv; t < kWT; t += kWWaves) {
    const int i = w.i0 + t;
    if (i < w.M && j < w.N) out[(size_t)i * w.N + j] = src[t][l];
  }
}

// ---------------------------------------------------------------------------
// ILU(0) pivots, one anti-diagonal of tiles.  Lane l walks row l; the west
// coupling U(i, j-1) is the U it read one step earlier, the north coupling
// V(i-1, j) and pivot come from lane l-1's previous step.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kWThreads) k_wf_pivots(WArgs a) {
  __shared__ __attribute__((aligned(16))) T Us[kWT][kWT], Vs[kWT][kWT];
  __shared__ T left[kWT], top[kWT], ul[kWT], vt[kWT];
  WTile w;
  if (!wf_tile<false>(a, w)) return;
  const gptr<T> U = (gptr<T>)(reinterpret_cast<const T*>(a.U) + w.off);
  const gptr<T> V = (gptr<T>)(reinterpret_cast<const T*>(a.V) + w.off);
  T* piv = reinterpret_cast<T*>(const_cast<void*>(a.piv)) + w.off;
  const int l = threadIdx.x & 63;
  {
    T (*const dst[2])[kWT] = {Us, Vs};
    const gptr<T> src[2] = {U, V};
    const WEdge<T> edge[4] = {{left, (gptr<T>)piv, 1, 0, 0, -1, T(1)},
                              {top, (gptr<T>)piv, 0, 1, -1, 0, T(1)},
                              {ul, U, 1, 0, 0, -1, T(0)},
                              {vt, V, 0, 1, -1, 0, T(0)}};
    wf_stage<T, 2, 4>(dst, src, -1, edge, w);
  }
  // wave 0, lane l owns tile row l; at step k it computes column k - l (the
  // pivot overwrites Us there, whose value it has read)
  // Row 0's north neighbours (the tile above) are held one per lane and
  // broadcast by lane index, so no LDS read sits on the chain.
  if (threadIdx.x < 64) {
  const T top_l = top[l], vt_l = vt[l];
  T pw = left[l], pn = T(1), vn_own = T(0), uwest = ul[l];
  T nu = T(0), nv = T(0);
  if (l == 0) nu = Us[0][0], nv = Vs[0][0];
  for (int k = 0; k < 2 * kWT - 1; ++k) {
    const int c = k - l;
    const T ue = nu, vs = nv;
    const int cn = (c + 1) & (kWT - 1);  // wrapped for idle steps, as in the forward solve
    nu = Us[l][cn], nv = Vs[l][cn];
    const T p_above = from_prev_lane(pn);
    const T v_above = from_prev_lane(vn_own);
    const int k0 = min(k, kWT - 1);
    const T top_k = lane_value(top_l, k0), vt_k = lane_value(vt_l, k0);
    if (c >= 0 && c < kWT) {
      const T uw = uwest, vn = l == 0 ? vt_k : v_above;
      const T pup = l == 0 ? top_k : p_above;
      const T av = uw + ue + vn + vs;
      T pv;
      if (av == T(0)) {
        pv = T(1);
      } else {
        T v = av;
        if (uw != T(0)) v -= uw * uw / pw;
        if (vn != T(0)) v -= vn * vn / pup;
        if (v < (T)kPivotFloor * av) v = av;
        pv = v;
      }
      Us[l][c] = pv;
      pw = pv;
      pn = pv;
      vn_own = vs;
      uwest = ue;
    }
  }
  }
  __syncthreads();
  wf_store<T>(piv, Us, w);
}

// SSOR "pivots" D / omega are pointwise: every active map, grid-stride.
template <typename T>
__global__ void __launch_bounds__(256) k_wf_ssor_diag(WArgs a) {
  if ((int)blockIdx.y >= a.counts[2]) return;
  const int m = a.mact[blockIdx.y];
  const MapDesc& d = a.desc[m];
  const T* U = reinterpret_cast<const T*>(a.U) + d.off;
  const T* V = reinterpret_cast<const T*>(a.V) + d.off;
  T* piv = reinterpret_cast<T*>(const_cast<void*>(a.piv)) + d.off;
  const int M = d.M, N = d.N;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < (long long)M * N;
       p += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(p / N), j = (int)(p % N);
    const T dg = (j > 0 ? U[p - 1] : T(0)) + U[p] + (i > 0 ? V[p - N] : T(0)) + V[p];
    piv[p] = dg == T(0) ? T(1) : dg / (T)a.omega;
  }
}

// ---------------------------------------------------------------------------
// Forward solve (P + L) y = r, one anti-diagonal of tiles
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kWThreads) k_wf_forward(WArgs a) {
  // sm[0]: r, overwritten by y; sm[1]: V.  Row 0 of each holds the row
  // above the tile (its y and V), rows 1..64 the tile, so one instruction
  // reads a lane's operand and the value above it, and both arrays are read
  // from one address.  pu: {1 / p, U} pairs of the tile.
  __shared__ __attribute__((aligned(16))) T sm[2][kWT + 1][kWT];
  __shared__ __attribute__((aligned(16))) T pu[kWT][kWT][2];
  __shared__ T left[kWT], ul[kWT];
  WTile w;
  if (!wf_tile<false>(a, w)) return;
  const gptr<T> U = (gptr<T>)(reinterpret_cast<const T*>(a.U) + w.off);
  const gptr<T> V = (gptr<T>)(reinterpret_cast<const T*>(a.V) + w.off);
  const gptr<T> piv = (gptr<T>)(reinterpret_cast<const T*>(a.piv) + w.off);
  const gptr<T> r = (gptr<T>)(reinterpret_cast<const T*>(a.r) + w.off);
  T* y = reinterpret_cast<T*>(a.y) + w.off;
  const int l = threadIdx.x & 63;
  {
    T* const stg = &pu[0][0][0];
    T (*const dst[4])[kWT] = {&sm[0][1], reinterpret_cast<T (*)[kWT]>(stg),
                              reinterpret_cast<T (*)[kWT]>(stg + kWT * kWT), &sm[1][1]};
    const gptr<T> src[4] = {r, piv, U, V};
    const WEdge<T> e[4] = {{left, (gptr<T>)y, 1, 0, 0, -1, T(0)},
                           {&sm[0][0][0], (gptr<T>)y, 0, 1, -1, 0, T(0)},
                           {ul, U, 1, 0, 0, -1, T(0)},
                           {&sm[1][0][0], V, 0, 1, -1, 0, T(0)}};
    wf_stage<T, 4, 4>(dst, src, 1, e, w);
  }
  wf_pivot_pairs<T>(pu);
  // Wave 0 runs the wavefront, lane l on tile row l.  The operands of
  // column c + kWR are read kWR steps ahead into a ring of registers (each
  // slot refilled after its step used it), so the recurrence never waits for
  // LDS.  A lane with no column at a step reads column c mod 64 of its row
  // and ignores the value: a wrapped column keeps the wave's reads in
  // distinct banks (lane l reads word 63 l + const of the tile), where a
  // clamped one would put every such lane on one column, a single bank.  The
  // north neighbours come from lane l - 1's previous step by a DPP shift;
  // lane 0 keeps the values above the tile, which its reads of the row above
  // its own fetched.
  if (threadIdx.x < 64) {
  T y_own = left[l], uwest = ul[l];
  T ra[kWR], rr[kWR], va[kWR], vv[kWR], pp[kWR], uu[kWR];
  auto fetch = [&](int u, int col) {
    ra[u] = sm[0][l][col], rr[u] = sm[0][l + 1][col];
    va[u] = sm[1][l][col], vv[u] = sm[1][l + 1][col];
    pp[u] = pu[l][col][0], uu[u] = pu[l][col][1];
  };
#pragma unroll
  for (int u = 0; u < kWR; ++u) fetch(u, (u - l) & (kWT - 1));
  // The north coupling V(l - 1, c) a lane uses at a step is lane l - 1's
  // own operand of the previous step, shifted at the end of that step before
  // its slot is refilled (lane 0: the row above's, from the next slot).
  T vn = va[0];
  for (int k0 = 0; k0 < kWSteps; k0 += kWR) {
#pragma unroll
    for (int u = 0; u < kWR; ++u) {
      const int c = k0 + u - l;
      const T yup = from_prev_lane(ra[u], y_own);  // lane 0: y of the row above, column k
      if (c >= 0 && c < kWT) {
        const T v = (rr[u] + vn * yup + uwest * y_own) * pp[u];  // pp = 1 / p
        sm[0][l + 1][c] = v;
        y_own = v;
        uwest = uu[u];
      }
      vn = from_prev_lane(va[(u + 1) % kWR], vv[u]);
      fetch(u, (c + kWR) & (kWT - 1));
    }
  }
  }
  __syncthreads();
  wf_store<T>(y, &sm[0][1], w);
}

// ---------------------------------------------------------------------------
// Backward solve (P + L^T) z = P y (z overwrites y), s = c z, and the tile's
// FP64 partial of r^T s; one anti-diagonal of tiles from the bottom-right
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kWThreads) k_wf_backward(WArgs a) {
  // sm rows 0..63: y of the tile, overwritten by z; row 64: z of the row
  // below the tile; rows 65..128: V of the tile (so a lane's operand, the
  // value below it and its V are read from one address).  pu: {1 / p, U}.
  __shared__ __attribute__((aligned(16))) T sm[2 * kWT + 1][kWT];
  __shared__ __attribute__((aligned(16))) T pu[kWT][kWT][2];
  __shared__ T right[kWT];
  __shared__ double red[kWWaves];
  T (*const Yz)[kWT] = sm;
  WTile w;
  if (!wf_tile<true>(a, w)) return;
  const gptr<T> U = (gptr<T>)(reinterpret_cast<const T*>(a.U) + w.off);
  const gptr<T> V = (gptr<T>)(reinterpret_cast<const T*>(a.V) + w.off);
  const gptr<T> piv = (gptr<T>)(reinterpret_cast<const T*>(a.piv) + w.off);
  const gptr<T> r = (gptr<T>)(reinterpret_cast<const T*>(a.r) + w.off);
  T* s = reinterpret_cast<T*>(a.s) + w.off;
  T* y = reinterpret_cast<T*>(a.y) + w.off;
  const int M = w.M, N = w.N, l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  {
    T* const stg = &pu[0][0][0];
    T (*const dst[4])[kWT] = {&sm[0], reinterpret_cast<T (*)[kWT]>(stg),
                              reinterpret_cast<T (*)[kWT]>(stg + kWT * kWT), &sm[kWT + 1]};
    const gptr<T> src[4] = {(gptr<T>)y, piv, U, V};
    const WEdge<T> edge[2] = {{right, (gptr<T>)y, 1, 0, 0, kWT, T(0)},
                              {&sm[kWT][0], (gptr<T>)y, 0, 1, kWT, 0, T(0)}};
    wf_stage<T, 4, 2>(dst, src, 1, edge, w);
  }
  wf_pivot_pairs<T>(pu);
  // r for the closing r^T s (wave wv: rows wv, wv + kWWaves, ...), requested
  // before the wavefront so its latency hides behind the chain
  constexpr int kRows = kWT / kWWaves;
  const int j = w.j0 + l;
  const int dt0 = a.desc[w.m].dtile0;
  T rv[kRows];
#pragma unroll
  for (int u = 0; u < kRows; ++u) rv[u] = wf_ld<T>(r, w.i0 + wv + u * kWWaves, j, M, N, T(0));
  // wave 0, lane l owns tile row 63 - l; at step k it computes column
  // 63 - (k - l); operands read kWR steps ahead, and lane 0's south
  // neighbours (the row below the tile) carried as in the forward solve
  if (threadIdx.x < 64) {
  const int row = kWT - 1 - l;
  T z_own = right[row];
  T yy[kWR], yb[kWR], vv[kWR], pp[kWR], uu[kWR];
  auto fetch = [&](int u, int col) {
    yy[u] = sm[row][col], yb[u] = sm[row + 1][col], vv[u] = sm[kWT + 1 + row][col];
    pp[u] = pu[row][col][0], uu[u] = pu[row][col][1];
  };
#pragma unroll
  for (int u = 0; u < kWR; ++u) fetch(u, (kWT - 1 - (u - l)) & (kWT - 1));  // wrapped as forward
  for (int k0 = 0; k0 < kWSteps; k0 += kWR) {
#pragma unroll
    for (int u = 0; u < kWR; ++u) {
      const int c = kWT - 1 - (k0 + u - l);
      const T zdown = from_prev_lane(yb[u], z_own);  // lane 0: z of the row below, column 63 - k
      if (c >= 0 && c < kWT) {
        const T v = yy[u] + (uu[u] * z_own + vv[u] * zdown) * pp[u];  // pp = 1 / p
        Yz[row][c] = v;
        z_own = v;
      }
      fetch(u, (c - kWR) & (kWT - 1));
    }
  }
  }
  __syncthreads();
  // z back to y, s = c z, and the tile's partial of r^T s (wave wv: rows wv,
  // wv + kWWaves, ...; the waves' sums added in a fixed order)
  const T scale = a.ssor ? (T)(2.0 - a.omega) : T(1);
  double part = 0.0;
  T z[kRows];
#pragma unroll
  for (int u = 0; u < kRows; ++u) z[u] = Yz[wv + u * kWWaves][l];
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int i = w.i0 + wv + u * kWWaves;
    if (i < M && j < N) {
      const size_t p = (size_t)i * N + j;
      const T sv = scale * z[u];
      y[p] = z[u];
      s[p] = sv;
      part += (double)rv[u] * (double)sv;
    }
  }
  part = wf_wave_sum(part);
  if (l == 0) red[wv] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
#pragma unroll
    for (int k = 0; k < kWWaves; ++k) tot += red[k];
    store_partial(a.P + 1 * a.pstride + dt0 + w.local, tot);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static WArgs make_wargs(const Engine& e, int expect, bool ssor, double omega, const void* r,
                        void* s, void* y) {
  WArgs a;
  a.desc = e.desc;
  a.ms = e.ms;
  a.mact = e.mact;
  a.mact_cap = e.cap_maps;
  a.counts = e.counts;
  a.P = e.P;
  a.pstride = e.pstride;
  a.U = e.U;
  a.V = e.V;
  a.piv = e.aux;
  a.r = r;
  a.s = s;
  a.y = y;
  a.expect = expect;
  a.diag = 0;
  a.omega = omega;
  a.ssor = ssor ? 1 : 0;
  return a;
}

// Launches per solve: e.wf_diags anti-diagonals (the most any map has), each a
// grid of (longest diagonal, active maps) one-wave blocks.
template <typename T>
void e_pivots(hipStream_t st, const Engine& e, int nmaps, bool ssor, double omega) {
  WArgs a = make_wargs(e, -1, ssor, omega, nullptr, nullptr, nullptr);
  const int nm = std::max(1, nmaps);
  if (ssor) {
    hipLaunchKernelGGL(k_wf_ssor_diag<T>, dim3(64, nm), dim3(256), 0, st, a);
    return;
  }
  for (int d = 0; d < e.wf_diags; ++d) {
    a.diag = d;
    hipLaunchKernelGGL(k_wf_pivots<T>, dim3(std::max(1, e.wf_len), nm), dim3(kWThreads), 0, st, a);
  }
}

template <typename T>
void e_sweep(hipStream_t st, const Engine& e, int nmaps, int expect, bool ssor, double omega,
             const void* r, void* s, void* y) {
  WArgs a = make_wargs(e, expect, ssor, omega, r, s, y);
  const dim3 g(std::max(1, e.wf_len), std::max(1, nmaps));
  for (int d = 0; d < e.wf_diags; ++d) {
    a.diag = d;
    hipLaunchKernelGGL(k_wf_forward<T>, g, dim3(kWThreads), 0, st, a);
  }
  for (int d = 0; d < e.wf_diags; ++d) {
    a.diag = d;
    hipLaunchKernelGGL(k_wf_backward<T>, g, dim3(kWThreads), 0, st, a);
  }
}

void wf_shape(int M, int N, int* diags, int* len) {
  const int ty = (M + kWT - 1) / kWT, tx = (N + kWT - 1) / kWT;
  *diags = ty + tx - 1;
  *len = std::min(ty, tx);
}

template void e_pivots<float>(hipStream_t, const Engine&, int, bool, double);
template void e_pivots<double>(hipStream_t, const Engine&, int, bool, double);
template void e_sweep<float>(hipStream_t, const Engine&, int, int, bool, double, const void*, void*,
                             void*);
template void e_sweep<double>(hipStream_t, const Engine&, int, int, bool, double, const void*, void*,
                              void*);

}  // namespace lpu
