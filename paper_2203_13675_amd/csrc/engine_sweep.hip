// Natural-order ILU(0) = IC(0) and SSOR preconditioners (Section 2.1's list,
// items 3-5) across the whole device.
//
// With P the pivots and L the strict lower part of A (entries -U west, -V
// north), M = (P + L) P^{-1} (P + L^T) (times 1/(2 - omega) for SSOR, where
// P = D/omega), so s = M^{-1} r is
//   forward : y_ij = (r_ij + V_{i-1,j} y_{i-1,j} + U_{i,j-1} y_{i,j-1}) / p_ij
//   backward: z_ij = y_ij + (U_ij z_{i,j+1} + V_ij z_{i+1,j}) / p_ij,  s = c z
// (the solves multiply by 1 / p_ij, formed while a tile's operands are staged)
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

constexpr int kWT = 64;       // tile side (rows = columns = lanes of a wave)
constexpr int kWLD = kWT + 2;  // LDS row pitch: the wavefront's column-skewed reads hit
                               // distinct banks

struct WArgs {
  const MapDesc* desc;
  MapState* ms;
  const int* mact;
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

template <bool REV>
__device__ __forceinline__ bool wf_tile(const WArgs& a, WTile& w) {
  if ((int)blockIdx.y >= a.counts[2]) return false;
  w.m = a.mact[blockIdx.y];
  if (a.expect >= 0 && a.ms[w.m].state != a.expect) return false;
  const MapDesc& d = a.desc[w.m];
  w.M = d.M;
  w.N = d.N;
  w.off = d.off;
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

__device__ __forceinline__ double wf_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Row loads of the tile's operands: lane l reads column j0 + l of the rows, at
// an index clamped into the map (the load always executes, so a batch of rows
// is in flight at once) and replaced by `outside` off the map.  Reads go
// through global-address-space pointers, so the compiler may keep them ahead
// of the LDS stores.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ T wf_ld(gptr<T> a, int i, int j, int M, int N, T outside) {
  const bool ok = (unsigned)i < (unsigned)M && (unsigned)j < (unsigned)N;
  const int ic = min(max(i, 0), M - 1), jc = min(max(j, 0), N - 1);
  const T v = a[(size_t)ic * N + jc];
  return ok ? v : outside;
}

constexpr int kWB = 16;  // rows per batch of loads

// Stage NA arrays: dst[q][t][c] = src[q](i0 + t + di[q], j0 + c + dj[q]), 0
// (1 for q == one) off the map, batches of kWB rows with every load of a
// batch issued before its LDS stores.  Array q == one is stored as its
// reciprocal (the solves multiply by 1 / p, so no division sits on the
// wavefront's dependency chain).
template <typename T, int NA>
__device__ __forceinline__ void wf_stage(T (*const (&dst)[NA])[kWLD], const gptr<T> (&src)[NA],
                                         const int (&di)[NA], const int (&dj)[NA], int one,
                                         const WTile& w) {
  const int l = threadIdx.x, j = w.j0 + l;
  for (int t0 = 0; t0 < kWT; t0 += kWB) {
    T v[NA][kWB];
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
      for (int u = 0; u < kWB; ++u) {
        const int i = w.i0 + t0 + u;
        // off the map for the tile's own pixel, or a neighbour outside it
        const bool own = i < w.M && j < w.N;
        const T x = wf_ld<T>(src[q], i + di[q], j + dj[q], w.M, w.N, T(0));
        v[q][u] = own ? x : (q == one ? T(1) : T(0));
      }
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
      for (int u = 0; u < kWB; ++u) dst[q][t0 + u][l] = q == one ? T(1) / v[q][u] : v[q][u];
  }
}

// ---------------------------------------------------------------------------
// ILU(0) pivots, one anti-diagonal of tiles
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kWT) k_wf_pivots(WArgs a) {
  __shared__ T Ue[kWT][kWLD], Uw[kWT][kWLD], Vn[kWT][kWLD], Vs[kWT][kWLD];
  __shared__ T left[kWT], top[kWT];
  WTile w;
  if (!wf_tile<false>(a, w)) return;
  const gptr<T> U = (gptr<T>)(reinterpret_cast<const T*>(a.U) + w.off);
  const gptr<T> V = (gptr<T>)(reinterpret_cast<const T*>(a.V) + w.off);
  T* piv = reinterpret_cast<T*>(const_cast<void*>(a.piv)) + w.off;
  const int N = w.N, l = threadIdx.x;
  {
    T (*const dst[4])[kWLD] = {Ue, Uw, Vn, Vs};
    const gptr<T> src[4] = {U, U, V, V};
    const int di[4] = {0, 0, -1, 0}, dj[4] = {0, -1, 0, 0};
    wf_stage<T, 4>(dst, src, di, dj, -1, w);
  }
  {
    const int i = w.i0 + l, j = w.j0 + l;
    left[l] = (w.j0 > 0 && i < w.M) ? piv[(size_t)i * N + w.j0 - 1] : T(1);
    top[l] = (w.i0 > 0 && j < N) ? piv[(size_t)(w.i0 - 1) * N + j] : T(1);
  }
  __syncthreads();
  // lane l owns tile row l; at step k it computes column k - l (the pivot
  // overwrites Ue there, whose value it has read)
  T pw = left[l], pn = T(1);
  T nu = T(0), nw = T(0), nn = T(0), ns = T(0);
  if (l == 0) nu = Ue[0][0], nw = Uw[0][0], nn = Vn[0][0], ns = Vs[0][0];
  for (int k = 0; k < 2 * kWT - 1; ++k) {
    const int c = k - l;
    const T ue = nu, uw = nw, vn = nn, vs = ns;
    const int cn = c + 1;
    if (cn >= 0 && cn < kWT) nu = Ue[l][cn], nw = Uw[l][cn], nn = Vn[l][cn], ns = Vs[l][cn];
    const T from_above = from_prev_lane(pn);
    if (c >= 0 && c < kWT) {
      const T av = uw + ue + vn + vs;
      const T pup = l == 0 ? top[c] : from_above;
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
      Ue[l][c] = pv;
      pw = pv;
      pn = pv;
    }
  }
  __syncthreads();
  const int j = w.j0 + l;
  for (int t0 = 0; t0 < kWT; t0 += kWB) {
    T v[kWB];
#pragma unroll
    for (int u = 0; u < kWB; ++u) v[u] = Ue[t0 + u][l];
#pragma unroll
    for (int u = 0; u < kWB; ++u) {
      const int i = w.i0 + t0 + u;
      if (i < w.M && j < N) piv[(size_t)i * N + j] = v[u];
    }
  }
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
__global__ void __launch_bounds__(kWT) k_wf_forward(WArgs a) {
  __shared__ T Ry[kWT][kWLD], Pv[kWT][kWLD], Uw[kWT][kWLD], Vn[kWT][kWLD];
  __shared__ T left[kWT], top[kWT];
  WTile w;
  if (!wf_tile<false>(a, w)) return;
  const gptr<T> U = (gptr<T>)(reinterpret_cast<const T*>(a.U) + w.off);
  const gptr<T> V = (gptr<T>)(reinterpret_cast<const T*>(a.V) + w.off);
  const gptr<T> piv = (gptr<T>)(reinterpret_cast<const T*>(a.piv) + w.off);
  const gptr<T> r = (gptr<T>)(reinterpret_cast<const T*>(a.r) + w.off);
  T* y = reinterpret_cast<T*>(a.y) + w.off;
  const int N = w.N, l = threadIdx.x;
  {
    const int i = w.i0 + l, j = w.j0 + l;
    left[l] = (w.j0 > 0 && i < w.M) ? y[(size_t)i * N + w.j0 - 1] : T(0);
    top[l] = (w.i0 > 0 && j < N) ? y[(size_t)(w.i0 - 1) * N + j] : T(0);
  }
  {
    T (*const dst[4])[kWLD] = {Ry, Pv, Uw, Vn};
    const gptr<T> src[4] = {r, piv, U, V};
    const int di[4] = {0, 0, 0, -1}, dj[4] = {0, 0, -1, 0};
    wf_stage<T, 4>(dst, src, di, dj, 1, w);
  }
  __syncthreads();
  T yw = left[l], yn = T(0);
  T nr = T(0), np = T(1), nu = T(0), nv = T(0);
  if (l == 0) nr = Ry[0][0], np = Pv[0][0], nu = Uw[0][0], nv = Vn[0][0];
  for (int k = 0; k < 2 * kWT - 1; ++k) {
    const int c = k - l;
    const T cr = nr, cp = np, cu = nu, cv = nv;
    const int cn = c + 1;
    if (cn >= 0 && cn < kWT) nr = Ry[l][cn], np = Pv[l][cn], nu = Uw[l][cn], nv = Vn[l][cn];
    const T from_above = from_prev_lane(yn);
    if (c >= 0 && c < kWT) {
      const T yup = l == 0 ? top[c] : from_above;
      const T v = (cr + cv * yup + cu * yw) * cp;  // cp = 1 / p
      Ry[l][c] = v;
      yw = v;
      yn = v;
    }
  }
  __syncthreads();
  const int j = w.j0 + l;
  for (int t0 = 0; t0 < kWT; t0 += kWB) {
    T v[kWB];
#pragma unroll
    for (int u = 0; u < kWB; ++u) v[u] = Ry[t0 + u][l];
#pragma unroll
    for (int u = 0; u < kWB; ++u) {
      const int i = w.i0 + t0 + u;
      if (i < w.M && j < N) y[(size_t)i * N + j] = v[u];
    }
  }
}

// ---------------------------------------------------------------------------
// Backward solve (P + L^T) z = P y (z overwrites y), s = c z, and the tile's
// FP64 partial of r^T s; one anti-diagonal of tiles from the bottom-right
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kWT) k_wf_backward(WArgs a) {
  __shared__ T Yz[kWT][kWLD], Pv[kWT][kWLD], Ue[kWT][kWLD], Vs[kWT][kWLD];
  __shared__ T right[kWT], below[kWT];
  WTile w;
  if (!wf_tile<true>(a, w)) return;
  const gptr<T> U = (gptr<T>)(reinterpret_cast<const T*>(a.U) + w.off);
  const gptr<T> V = (gptr<T>)(reinterpret_cast<const T*>(a.V) + w.off);
  const gptr<T> piv = (gptr<T>)(reinterpret_cast<const T*>(a.piv) + w.off);
  const gptr<T> r = (gptr<T>)(reinterpret_cast<const T*>(a.r) + w.off);
  T* s = reinterpret_cast<T*>(a.s) + w.off;
  T* y = reinterpret_cast<T*>(a.y) + w.off;
  const int M = w.M, N = w.N, l = threadIdx.x;
  {
    const int i = w.i0 + l, j = w.j0 + l, jr = w.j0 + kWT, ib = w.i0 + kWT;
    right[l] = (jr < N && i < M) ? y[(size_t)i * N + jr] : T(0);
    below[l] = (ib < M && j < N) ? y[(size_t)ib * N + j] : T(0);
  }
  {
    T (*const dst[4])[kWLD] = {Yz, Pv, Ue, Vs};
    const gptr<T> src[4] = {(gptr<T>)y, piv, U, V};
    const int di[4] = {0, 0, 0, 0}, dj[4] = {0, 0, 0, 0};
    wf_stage<T, 4>(dst, src, di, dj, 1, w);
  }
  __syncthreads();
  // lane l owns tile row 63 - l; at step k it computes column 63 - (k - l)
  const int row = kWT - 1 - l;
  T ze = right[row], zs = T(0);
  T ny = T(0), np = T(1), nu = T(0), nv = T(0);
  if (l == 0) ny = Yz[row][kWT - 1], np = Pv[row][kWT - 1], nu = Ue[row][kWT - 1],
              nv = Vs[row][kWT - 1];
  for (int k = 0; k < 2 * kWT - 1; ++k) {
    const int c = kWT - 1 - (k - l);
    const T cy = ny, cp = np, cu = nu, cv = nv;
    const int cn = c - 1;
    if (k + 1 - l >= 0 && cn >= 0 && cn < kWT)
      ny = Yz[row][cn], np = Pv[row][cn], nu = Ue[row][cn], nv = Vs[row][cn];
    const T from_below = from_prev_lane(zs);
    if (k - l >= 0 && c >= 0) {
      const T zdown = l == 0 ? below[c] : from_below;
      const T v = cy + (cu * ze + cv * zdown) * cp;  // cp = 1 / p
      Yz[row][c] = v;
      ze = v;
      zs = v;
    }
  }
  __syncthreads();
  const T scale = a.ssor ? (T)(2.0 - a.omega) : T(1);
  const int j = w.j0 + l;
  double part = 0.0;
  for (int t0 = 0; t0 < kWT; t0 += kWB) {
    T z[kWB], rv[kWB];
#pragma unroll
    for (int u = 0; u < kWB; ++u) {
      z[u] = Yz[t0 + u][l];
      rv[u] = wf_ld<T>(r, w.i0 + t0 + u, j, M, N, T(0));
    }
#pragma unroll
    for (int u = 0; u < kWB; ++u) {
      const int i = w.i0 + t0 + u;
      if (i < M && j < N) {
        const size_t p = (size_t)i * N + j;
        const T sv = scale * z[u];
        y[p] = z[u];
        s[p] = sv;
        part += (double)rv[u] * (double)sv;
      }
    }
  }
  part = wf_wave_sum(part);
  if (l == 0) store_partial(a.P + 1 * a.pstride + a.desc[w.m].dtile0 + w.local, part);
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
    hipLaunchKernelGGL(k_wf_pivots<T>, dim3(std::max(1, e.wf_len), nm), dim3(kWT), 0, st, a);
  }
}

template <typename T>
void e_sweep(hipStream_t st, const Engine& e, int nmaps, int expect, bool ssor, double omega,
             const void* r, void* s, void* y) {
  WArgs a = make_wargs(e, expect, ssor, omega, r, s, y);
  const dim3 g(std::max(1, e.wf_len), std::max(1, nmaps));
  for (int d = 0; d < e.wf_diags; ++d) {
    a.diag = d;
    hipLaunchKernelGGL(k_wf_forward<T>, g, dim3(kWT), 0, st, a);
  }
  for (int d = 0; d < e.wf_diags; ++d) {
    a.diag = d;
    hipLaunchKernelGGL(k_wf_backward<T>, g, dim3(kWT), 0, st, a);
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
