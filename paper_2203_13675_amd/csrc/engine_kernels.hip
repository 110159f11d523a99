// Batched kernels of the phase-unwrapping PCG (gfx950).
//
// Stencil tiles are 128 columns x 16 rows, one 64-lane wave each: lane l owns
// columns j0 + l and j0 + 64 + l (two coalesced 64-wide rows per load), the
// wave marches down the 16 rows keeping rows i-1, i, i+1 of the operand in
// registers, and horizontal neighbours come from lane shuffles (plus one halo
// column at each side, loaded by lanes 0 and 63).  Each tile writes its FP64
// partial sums to its own slot; finisher kernels reduce per map.
//
// The operator is Eq. (7):
//   (A x)_{i,j} = (U_{i,j-1} + U_{i,j} + V_{i-1,j} + V_{i,j}) x_{i,j}
//               - U_{i,j} x_{i,j+1} - U_{i,j-1} x_{i,j-1}
//               - V_{i,j} x_{i+1,j} - V_{i-1,j} x_{i-1,j},
// out-of-grid terms zero (U is 0 on the last column, V on the last row).

#include <type_traits>

#include "lpu_internal.h"
#include "lpu_device.h"
#include "lpu_finish.h"

namespace lpu {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
template <typename T>
struct R2 {
  T a, b;  // columns j0 + lane, j0 + 64 + lane
};

template <typename T>
struct R3 {
  T s, w, d;  // raw loads of one operand element (see the field loaders)
};
template <typename T>
struct R4 {
  T s, w, d, x;  // R3 and the iterate (SpMV)
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Lane moves on the VALU instead of the LDS crossbar: DPP whole-wave shifts
// by one lane (wave_shr:1 = 0x138: lane l receives lane l-1; wave_shl:1 =
// 0x130: lane l receives lane l+1; the lane with no source receives 0 and is
// overwritten by the caller) and readlane broadcasts.
template <int CTRL>
__device__ __forceinline__ int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, dpp32<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp32<CTRL>((int)(b & 0xffffffffLL)), hi = dpp32<CTRL>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float bcast(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double bcast(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T shup(T v) { return dpp_move<0x138>(v); }
template <typename T>
__device__ __forceinline__ T shdn(T v) { return dpp_move<0x130>(v); }
template <typename T>
__device__ __forceinline__ T shfrom(T v, int src) { return bcast(v, src); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

struct TilePos {
  int m, i0, j0, M, N, rows;
  long long off;
};

__device__ __forceinline__ TilePos tile_pos(const MapDesc* __restrict__ desc,
                                            const int* __restrict__ tile_map, int g) {
  TilePos t;
  t.m = tile_map[g];
  const MapDesc& d = desc[t.m];
  const int lt = g - d.tile0;
  const int ty = lt / d.tiles_x;
  t.rows = d.th;
  t.i0 = ty * d.th;
  t.j0 = (lt - ty * d.tiles_x) * kTW;
  t.M = d.M;
  t.N = d.N;
  t.off = d.off;
  return t;
}

// left/right neighbours of a row pair (lane shuffles + halo values)
template <typename T>
__device__ __forceinline__ void neighbours(const R2<T>& v, T halo, R2<T>& w, R2<T>& e) {
  const int l = lane_id();
  const T up_a = shup(v.a), up_b = shup(v.b);
  const T dn_a = shdn(v.a), dn_b = shdn(v.b);
  const T a63 = shfrom(v.a, 63), b0 = shfrom(v.b, 0);
  const T h0 = shfrom(halo, 0), h63 = shfrom(halo, 63);
  w.a = l > 0 ? up_a : h0;     // column j0 - 1 for lane 0
  w.b = l > 0 ? up_b : a63;    // column j0 + 63 for lane 0
  e.a = l < 63 ? dn_a : b0;    // column j0 + 64 for lane 63
  e.b = l < 63 ? dn_b : h63;   // column j0 + 128 for lane 63
}

// In-grid index of (i, j) clamped to the grid, and whether (i, j) is inside.
// Loads through a clamped index always execute (no lane-divergent branch
// around them), so the compiler can issue the loads of several rows at once;
// the value is then replaced by zero where (i, j) is outside.
__device__ __forceinline__ size_t clamp_at(int i, int j, int M, int N, bool& ok) {
  ok = (unsigned)i < (unsigned)M && (unsigned)j < (unsigned)N;
  const int ic = min(max(i, 0), M - 1), jc = min(max(j, 0), N - 1);
  return (size_t)ic * N + jc;
}

template <typename T>
__device__ __forceinline__ T ldz(const T* __restrict__ a, int i, int j, int M, int N) {
  bool ok;
  const T v = a[clamp_at(i, j, M, N, ok)];
  return ok ? v : T(0);
}

template <typename T>
__device__ __forceinline__ R2<T> ldrow(const T* __restrict__ a, int i, int j0, int M, int N) {
  const int l = lane_id();
  R2<T> v;
  v.a = ldz(a, i, j0 + l, M, N);
  v.b = ldz(a, i, j0 + 64 + l, M, N);
  return v;
}

// Halo column of this lane's halo load: lane 0 uses column j0 - 1, lane 63
// column j0 + 128.  The other lanes' values are never used, but the load is
// one instruction for the whole wave: they read the same two columns, so the
// instruction touches only the two halo lines (a lane clamped to column 0
// would fetch one more line of every row).
__device__ __forceinline__ int halo_col(int j0) {
  return lane_id() < 32 ? j0 - 1 : j0 + kTW;
}

template <typename T>
__device__ __forceinline__ T stencil5(T uw, T uc, T vn, T vc, T xc, T xw, T xe, T xn, T xs) {
  return (uw + uc + vn + vc) * xc - uc * xe - uw * xw - vc * xs - vn * xn;
}

// March the tile: for every interior pixel call epi(i, j, x_ij, (A x)_ij),
// or epi(i, j, x_ij, (A x)_ij, raw_ij) when epi takes the element's raw loads
// as well.  The operand x is formed as make(load(i, j)): load issues the raw
// loads of one element (zero outside the grid, through a clamped index), make
// combines them.  Loads run two rows ahead of the arithmetic (operand row i + 2, U and
// V row i + 1 while row i is computed) and their values are first combined in
// the next step, so a row's loads are in flight while the previous row is
// computed and stored (vector loads and stores share one counter on this
// architecture; a value used in the step that loads it would make the wave
// wait for everything issued before).
template <int TH, bool FULL, typename T, typename Ld, typename Mk, typename E>
__device__ __forceinline__ void march_stencil(const TilePos& tp, const T* __restrict__ U,
                                              const T* __restrict__ V, Ld load, Mk make, E epi) {
  const int M = tp.M, N = tp.N, i0 = tp.i0, j0 = tp.j0, l = lane_id();
  const int hj = halo_col(j0), uj = j0 - 1;  // U's halo: column j0 - 1 (lane 0's), every lane
  const int ca = j0 + l, cb = j0 + 64 + l;
  using Raw = decltype(load(0, 0));
  struct Row {
    Raw a, b, h;  // columns ca, cb and this lane's halo column
  };
  auto lrow = [&](int i) {
    Row r;
    r.a = load(i, ca);
    r.b = load(i, cb);
    r.h = load(i, hj);
    return r;
  };
  constexpr bool kRaw = std::is_invocable_v<E, int, int, T, T, const Raw&>;
  auto call = [&](int i, int j, T xv, T ax, const Raw& raw) {
    if constexpr (kRaw) epi(i, j, xv, ax, raw);
    else epi(i, j, xv, ax);
  };
  R2<T> xm, xc;
  Row rcur;  // raw loads of the row being computed (kept only when epi reads them)
  {
    const Row rm = lrow(i0 - 1), rc = lrow(i0);
    xm.a = make(rm.a);
    xm.b = make(rm.b);
    xc.a = make(rc.a);
    xc.b = make(rc.b);
    rcur = rc;
  }
  T xh = make(lrow(i0).h);
  Row rp = lrow(i0 + 1);
  R2<T> vn = ldrow(V, i0 - 1, j0, M, N), vc = ldrow(V, i0, j0, M, N);
  R2<T> uc = ldrow(U, i0, j0, M, N);
  T uh = ldz(U, i0, uj, M, N);
  auto step = [&](int k) {
    const int i = i0 + k;
    // next rows' loads first
    const Row rpp = lrow(i + 2);
    const R2<T> un = ldrow(U, i + 1, j0, M, N);
    const T unh = ldz(U, i + 1, uj, M, N);
    const R2<T> vnx = ldrow(V, i + 1, j0, M, N);
    R2<T> xp;
    xp.a = make(rp.a);
    xp.b = make(rp.b);
    const T xph = make(rp.h);
    R2<T> xw, xe, uw, ue;
    neighbours(xc, xh, xw, xe);
    neighbours(uc, uh, uw, ue);
    if (FULL || ca < N)
      call(i, ca, xc.a, stencil5<T>(uw.a, uc.a, vn.a, vc.a, xc.a, xw.a, xe.a, xm.a, xp.a), rcur.a);
    if (FULL || cb < N)
      call(i, cb, xc.b, stencil5<T>(uw.b, uc.b, vn.b, vc.b, xc.b, xw.b, xe.b, xm.b, xp.b), rcur.b);
    xm = xc;
    xc = xp;
    xh = xph;
    if constexpr (kRaw) rcur = rp;
    rp = rpp;
    vn = vc;
    vc = vnx;
    uc = un;
    uh = unh;
  };
  // TH > 0: compile-time tile height, unrolled (the lane shuffles inside keep
  // the compiler from unrolling a loop of run-time length); TH == 0: tp.rows
  if constexpr (TH > 0) {
#pragma unroll 4
    for (int k = 0; k < TH; ++k) {
      if (i0 + k >= M) break;
      step(k);
    }
  } else {
    const int kend = min(tp.rows, M - i0);
    for (int k = 0; k < kend; ++k) step(k);
  }
}

// Tiles that lie wholly inside the map's columns (every map side a multiple
// of 128 gives only such tiles) take a copy of the march without per-lane
// column guards, so no store or load sits behind a lane-divergent branch.
template <int TH, typename T, typename Ld, typename Mk, typename E>
__device__ __forceinline__ void march_tile(const TilePos& tp, const T* __restrict__ U,
                                           const T* __restrict__ V, Ld load, Mk make, E epi) {
  if (tp.j0 + kTW <= tp.N) march_stencil<TH, true, T>(tp, U, V, load, make, epi);
  else march_stencil<TH, false, T>(tp, U, V, load, make, epi);
}

// Elementwise walk over the tile's pixels.
template <typename E>
__device__ __forceinline__ void march_points(const TilePos& tp, E epi) {
  const int l = lane_id();
  const int kend = min(tp.rows, tp.M - tp.i0);
  for (int k = 0; k < kend; ++k) {
    const int i = tp.i0 + k;
    const int ca = tp.j0 + l, cb = tp.j0 + 64 + l;
    if (ca < tp.N) epi(i, ca);
    if (cb < tp.N) epi(i, cb);
  }
}

// Elementwise walk in groups of G rows: load(i, j) issues every load of one
// pixel (the walk passes in-grid coordinates, clamped for lanes and rows past
// the map, whose results are dropped), store(i, j, v) computes and stores.
// All loads of a group are issued before its first store: loads and stores
// share one wait counter, so a load issued after a store would also wait for
// the store, a memory round trip per pixel row.
template <int G, typename L, typename S>
__device__ __forceinline__ void march_points_grouped(const TilePos& tp, L load, S store) {
  const int l = lane_id();
  const int kend = min(tp.rows, tp.M - tp.i0);
  const int ca = tp.j0 + l, cb = tp.j0 + 64 + l;
  const int ja = min(ca, tp.N - 1), jb = min(cb, tp.N - 1);
  using Val = decltype(load(0, 0));
  for (int k0 = 0; k0 < kend; k0 += G) {
    Val v[G][2];
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int i = min(tp.i0 + k0 + c, tp.M - 1);
      v[c][0] = load(i, ja);
      v[c][1] = load(i, jb);
    }
#pragma unroll
    for (int c = 0; c < G; ++c) {
      if (k0 + c >= kend) break;  // uniform over the wave
      const int i = tp.i0 + k0 + c;
      if (ca < tp.N) store(i, ca, v[c][0]);
      if (cb < tp.N) store(i, cb, v[c][1]);
    }
  }
}

template <typename T>
__device__ __forceinline__ T* vec(void* base, long long off) {
  return reinterpret_cast<T*>(base) + off;
}
template <typename T>
__device__ __forceinline__ const T* cvec(const void* base, long long off) {
  return reinterpret_cast<const T*>(base) + off;
}

// Kernel arguments shared by the tile kernels.
struct EArgs {
  const MapDesc* desc;
  MapState* ms;
  const int* tile_map;
  const int* act;
  int act_cap;  // entries of act (its capacity)
  const int* counts;
  double* P;
  long long pstride;
  void *U, *V, *aux, *x0, *x1, *d0, *d1, *r, *s, *q, *b;
  double *dx, *dy, *phi_prev, *r64;
  const unsigned char* iso;
  int *fcnt, *gcnt;  // arrival counters of the finisher fused into the tile kernel
  double* gsum;      // its group sums (rows of gstride)
  long long gstride;
  int fuse_pw;  // -1: no fused finisher; else its pointwise-preconditioner flag
  int expect;   // two-colour preconditioner: state of the maps it applies to
  int fin_mode;  // two-colour preconditioner: FinishMode of its fused finisher (0: none)
};

__device__ __forceinline__ Arrival arrival(const EArgs& A) {
  return Arrival{A.fcnt, A.gcnt, A.gsum, A.gstride, A.P, A.pstride};
}

// Grid-stride walk over the active tiles.  The block's first list entry is
// requested together with the list's length (through an index clamped to
// the list's capacity; it is used only when the block has a tile), so the
// walk starts one memory round trip earlier.
#define TILE_LOOP(A)                                                          \
  const int n_act_ = (A).counts[0];                                           \
  const int g_first_ = (A).act[min((int)blockIdx.x, max((A).act_cap - 1, 0))]; \
  __asm__ volatile("" ::"s"(n_act_), "s"(g_first_)); /* both loads issued here */ \
  for (int t_ = blockIdx.x; t_ < n_act_; t_ += gridDim.x)
#define TILE_G(A) (t_ == (int)blockIdx.x ? g_first_ : (A).act[t_])

// ---------------------------------------------------------------------------
// Set-up kernels: wrapped differences, weights, Jacobi diagonal, isolation
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wrap_w(double x) {
#pragma clang fp contract(off)
  const double k = ceil((x - kPi) / kTwoPi);
  return x - kTwoPi * k;
}

// zero_phi: also set the caller's phi to 0 (the start value when the caller
// does not supply one)
__global__ void __launch_bounds__(64) k_e_wrapdiff(EArgs A, int zero_phi) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const double* psi = A.desc[tp.m].psi;
    double* phi = A.desc[tp.m].phi;
    double* dx = A.dx + tp.off;
    double* dy = A.dy + tp.off;
    struct Px {
      double c, e, s;
    };
    march_points_grouped<4>(
        tp,
        [&](int i, int j) {
          // neighbours outside the grid read the pixel itself (never used)
          const size_t p = (size_t)i * tp.N + j;
          Px x;
          x.c = psi[p];
          x.e = psi[j < tp.N - 1 ? p + 1 : p];
          x.s = psi[i < tp.M - 1 ? p + tp.N : p];
          return x;
        },
        [&](int i, int j, const Px& x) {
          const size_t p = (size_t)i * tp.N + j;
          dx[p] = (j < tp.N - 1) ? wrap_w(x.e - x.c) : 0.0;
          dy[p] = (i < tp.M - 1) ? wrap_w(x.s - x.c) : 0.0;
          if (zero_phi) phi[p] = 0.0;
        });
  }
}

// Input check of every map in one launch: *bad |= 1 when psi holds a
// non-finite value or the mask one outside [0, 1].
__global__ void __launch_bounds__(64) k_e_check(EArgs A, unsigned int* bad) {
  unsigned int b = 0;
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const double* psi = A.desc[tp.m].psi;
    const float* mask = A.desc[tp.m].mask;
    march_points(tp, [&](int i, int j) {
      const size_t p = (size_t)i * tp.N + j;
      if (!isfinite(psi[p])) b = 1;
      if (mask && !(isfinite(mask[p]) && mask[p] >= 0.0f && mask[p] <= 1.0f)) b = 1;
    });
  }
  if (b) atomicOr(bad, 1u);
}

__device__ __forceinline__ double abs_pow(double r, double e) {
  if (e == 2.0) return r * r;
  if (e == 1.0) return fabs(r);
  if (e == 0.0) return 1.0;
  return pow(fabs(r), e);
}

// U, V of Eq. (6) from phi (FP64), stored as T; also the Jacobi inverse
// diagonal needs U, V of neighbours, so it is a separate pass.
template <typename T>
__global__ void __launch_bounds__(64) k_e_weights(EArgs A, double e, double tau) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const MapDesc& d = A.desc[tp.m];
    const double* phi = d.phi;
    const float* mask = d.mask;
    const double* dx = A.dx + tp.off;
    const double* dy = A.dy + tp.off;
    T* U = vec<T>(A.U, tp.off);
    T* V = vec<T>(A.V, tp.off);
    struct Px {
      double c, e, s, dx, dy;
      float mc, me, ms;
    };
    march_points_grouped<2>(
        tp,
        [&](int i, int j) {
          // neighbours outside the grid read the pixel itself (never used)
          const size_t p = (size_t)i * tp.N + j;
          const size_t pe = j < tp.N - 1 ? p + 1 : p, ps = i < tp.M - 1 ? p + tp.N : p;
          Px x;
          x.c = phi[p];
          x.e = phi[pe];
          x.s = phi[ps];
          x.dx = dx[p];
          x.dy = dy[p];
          x.mc = mask ? mask[p] : 1.0f;
          x.me = mask ? mask[pe] : 1.0f;
          x.ms = mask ? mask[ps] : 1.0f;
          return x;
        },
        [&](int i, int j, const Px& x) {
          const size_t p = (size_t)i * tp.N + j;
          double u = 0.0, v = 0.0;
          if (j < tp.N - 1) {
            const double r = x.e - x.c - x.dx;
            const double w = mask ? (double)fminf(x.mc, x.me) : 1.0;
            u = w * (tau / (abs_pow(r, e) + tau));
          }
          if (i < tp.M - 1) {
            const double r = x.s - x.c - x.dy;
            const double w = mask ? (double)fminf(x.mc, x.ms) : 1.0;
            v = w * (tau / (abs_pow(r, e) + tau));
          }
          U[p] = (T)u;
          V[p] = (T)v;
        });
  }
}

// Jacobi inverse diagonal (0 on isolated pixels) and isolation flags.
template <typename T>
__global__ void __launch_bounds__(64) k_e_diag(EArgs A, int want_inv) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    T* inv = vec<T>(A.aux, tp.off);
    unsigned char* iso = const_cast<unsigned char*>(A.iso) + tp.off;
    march_points(tp, [&](int i, int j) {
      const size_t p = (size_t)i * tp.N + j;
      const T dg = ldz(U, i, j - 1, tp.M, tp.N) + U[p] + ldz(V, i - 1, j, tp.M, tp.N) + V[p];
      if (want_inv) inv[p] = dg > T(0) ? T(1) / dg : T(0);
      iso[p] = dg == T(0) ? 1 : 0;
    });
  }
}

// ---------------------------------------------------------------------------
// b = D^T W Delta and r64 = b - A phi (FP64; r formed as D^T W (Delta - D phi)).
// mode 0: b as T and as FP64 in r64 (phi unused); mode 1: r64 and (T) r64 into b;
// mode 2: r64 only.  Partials: slot 0 = r.r (mode 0: b.b), slot 1 = b.b.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) k_e_rhs(EArgs A, int mode) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const MapDesc& d = A.desc[tp.m];
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    const double* dx = A.dx + tp.off;
    const double* dy = A.dy + tp.off;
    const double* phi = d.phi;
    T* bT = vec<T>(A.b, tp.off);
    double* r64 = A.r64 + tp.off;
    const int M = tp.M, N = tp.N;
    const bool usephi = mode != 0;
    double srr = 0.0, sbb = 0.0;
    struct Px {
      double pc, pe, pw, pn, ps, dxc, dxw, dyc, dyn;
      T uc, uw, vc, vn;
    };
    march_points_grouped<2>(
        tp,
        [&](int i, int j) {
          // neighbours outside the grid read the pixel itself (never used)
          const size_t p = (size_t)i * N + j;
          const size_t pe = j < N - 1 ? p + 1 : p, pw = j > 0 ? p - 1 : p;
          const size_t pn = i > 0 ? p - N : p, ps = i < M - 1 ? p + N : p;
          Px x;
          x.pc = usephi ? phi[p] : 0.0;
          x.pe = usephi ? phi[pe] : 0.0;
          x.pw = usephi ? phi[pw] : 0.0;
          x.pn = usephi ? phi[pn] : 0.0;
          x.ps = usephi ? phi[ps] : 0.0;
          x.dxc = dx[p];
          x.dxw = dx[pw];
          x.dyc = dy[p];
          x.dyn = dy[pn];
          x.uc = U[p];
          x.uw = U[pw];
          x.vc = V[p];
          x.vn = V[pn];
          return x;
        },
        [&](int i, int j, const Px& x) {
          const size_t p = (size_t)i * N + j;
          double hx = 0.0, hy = 0.0, bx = 0.0, by = 0.0, hxw = 0.0, hyn = 0.0, bxw = 0.0, byn = 0.0;
          if (j < N - 1) {
            const double u = (double)x.uc;
            bx = u * x.dxc;
            hx = usephi ? u * (x.dxc - (x.pe - x.pc)) : bx;
          }
          if (i < M - 1) {
            const double v = (double)x.vc;
            by = v * x.dyc;
            hy = usephi ? v * (x.dyc - (x.ps - x.pc)) : by;
          }
          if (j > 0) {
            const double u = (double)x.uw;
            bxw = u * x.dxw;
            hxw = usephi ? u * (x.dxw - (x.pc - x.pw)) : bxw;
          }
          if (i > 0) {
            const double v = (double)x.vn;
            byn = v * x.dyn;
            hyn = usephi ? v * (x.dyn - (x.pc - x.pn)) : byn;
          }
          const double b = bxw + byn - bx - by;
          const double r = hxw + hyn - hx - hy;
          if (mode == 0) bT[p] = (T)b;
          if (mode == 1) bT[p] = (T)r;
          r64[p] = mode == 0 ? b : r;
          srr += r * r;
          sbb += b * b;
        });
    srr = wave_sum(srr);
    sbb = wave_sum(sbb);
    if (lane_id() == 0) {
      A.P[0 * A.pstride + g] = srr;
      A.P[1 * A.pstride + g] = sbb;
    }
  }
}

// ---------------------------------------------------------------------------
// Small per-tile passes used by the outer loop
// ---------------------------------------------------------------------------
// op 0: phi_prev = phi; op 1: x0 = phi (T); op 2: x0 = 0;
// op 3: phi += x_final (x[xi] plus a pending step); op 4: partials of
// ||phi - phi_prev||^2 (slot 0) and ||phi_prev||^2 (slot 1);
// op 5: phi = x_final (FP64 path).
template <typename T>
__global__ void __launch_bounds__(64) k_e_pass(EArgs A, int op) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    double* phi = A.desc[tp.m].phi;
    double* pp = A.phi_prev + tp.off;
    const MapState& ms = A.ms[tp.m];
    const long long l = ms.l;
    T* x0 = vec<T>(A.x0, tp.off);
    // the final iterate: x[xi] plus the pending step alpha_p d[l & 1]
    const T* xf = cvec<T>(ms.xi ? A.x1 : A.x0, tp.off);
    const T* dp = cvec<T>((l & 1) ? A.d1 : A.d0, tp.off);
    const T ap = (T)ms.alpha_p;
    const bool pend = ms.alpha_p != 0.0;
    double s0 = 0.0, s1 = 0.0;
    struct Px {
      double a, b;  // phi (ops 0, 1, 3, 4), phi_prev (op 4)
      T x, dd;      // final iterate and pending direction (ops 3, 5)
    };
    march_points_grouped<4>(
        tp,
        [&](int i, int j) {
          const size_t p = (size_t)i * tp.N + j;
          Px v{0.0, 0.0, T(0), T(0)};
          if (op == 0 || op == 1 || op == 3 || op == 4) v.a = phi[p];
          if (op == 4) v.b = pp[p];
          if (op == 3 || op == 5) {
            v.x = xf[p];
            if (pend) v.dd = dp[p];
          }
          return v;
        },
        [&](int i, int j, const Px& v) {
          const size_t p = (size_t)i * tp.N + j;
          switch (op) {
            case 0: pp[p] = v.a; break;
            case 1: x0[p] = (T)v.a; break;
            case 2: x0[p] = T(0); break;
            case 3: phi[p] = v.a + (double)(pend ? v.x + ap * v.dd : v.x); break;
            case 4: {
              const double dd = v.a - v.b;
              s0 += dd * dd;
              s1 += v.b * v.b;
            } break;
            case 5: phi[p] = (double)(pend ? v.x + ap * v.dd : v.x); break;
          }
        });
    if (op == 4) {
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      if (lane_id() == 0) {
        A.P[0 * A.pstride + g] = s0;
        A.P[1 * A.pstride + g] = s1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// PCG tile kernels
// ---------------------------------------------------------------------------
// init: r = b - A x0, d_old(parity 0) = 0, pointwise s; partials r.r, r.s, b.b
// confirm (CONF = 1): r = b - A x (current parity), pointwise s; partials r.r, r.s
template <typename T, int PC, int CONF>
__global__ void __launch_bounds__(64) k_e_resid(EArgs A) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const MapState& st = A.ms[tp.m];
    if (st.state != (CONF ? kConfirm : kRun)) continue;
    const long long l = st.l;
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    const T* aux = cvec<T>(A.aux, tp.off);
    const T* b = cvec<T>(A.b, tp.off);
    // the iterate: x0 (init), or x[xi] plus the pending step alpha_p d[l & 1]
    const T* x = cvec<T>(CONF && st.xi ? A.x1 : A.x0, tp.off);
    const T* dp = cvec<T>((l & 1) ? A.d1 : A.d0, tp.off);
    const T ap = CONF ? (T)st.alpha_p : T(0);
    const bool pend = CONF && st.alpha_p != 0.0;
    T* r = vec<T>(A.r, tp.off);
    T* d0 = vec<T>(A.d0, tp.off);
    const int M = tp.M, N = tp.N;
    double srr = 0.0, srs = 0.0, sbb = 0.0;
    march_tile<0, T>(tp, U, V,
                     [&](int i, int j) {
                       R3<T> v;  // x, unused, d (zero when no step is pending)
                       v.s = ldz(x, i, j, M, N);
                       v.w = T(1);
                       v.d = pend ? ldz(dp, i, j, M, N) : T(0);
                       return v;
                     },
                     [&](const R3<T>& v) { return pend ? v.s + ap * v.d : v.s; },
                     [&](int i, int j, T, T ax) {
                       const size_t p = (size_t)i * N + j;
                       const T bv = b[p];
                       const T rv = bv - ax;
                       r[p] = rv;
                       if (!CONF) d0[p] = T(0);
                       const T sv = PC == kPcJacobi ? rv * aux[p] : rv;
                       srr += (double)rv * (double)rv;
                       srs += (double)rv * (double)sv;
                       sbb += (double)bv * (double)bv;
                     });
    srr = wave_sum(srr);
    srs = wave_sum(srs);
    sbb = wave_sum(sbb);
    if (lane_id() == 0) {
      A.P[0 * A.pstride + g] = srr;
      A.P[1 * A.pstride + g] = srs;
      A.P[2 * A.pstride + g] = sbb;
    }
  }
}

// Non-temporal accesses for data whose next use is a later iteration (the
// iterate, the new direction) or that is dead after this read (q in the
// update): they leave the caches to what the next kernel reads.
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) { __builtin_nontemporal_store(v, p); }

// spmv: d_new = s + beta d_old; q = A d_new; partial d^T q.  Also adds the
// previous iteration's step to the iterate, x += alpha_p d_old (the update
// leaves it here: x is first needed again by a replacement or at the end, and
// this kernel reads d_old anyway, so the step costs one read and one write of
// x instead of two reads, a write and a second read of d in the update).
template <typename T, int PC, int TH>
__global__ void __launch_bounds__(64) k_e_spmv(EArgs A) {
  __shared__ double fred[3];
  __shared__ int fflag;
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const MapState& st = A.ms[tp.m];
    if (st.state != kRun) continue;
    const long long l = st.l;
    const T beta = (T)st.beta;
    const T ap = (T)st.alpha_p;
    const bool pend = st.alpha_p != 0.0;
    T* x = vec<T>(st.xi ? A.x1 : A.x0, tp.off);
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    const T* aux = cvec<T>(A.aux, tp.off);
    const T* src = cvec<T>(PC == kPcNone || PC == kPcJacobi ? A.r : A.s, tp.off);
    const T* dold = cvec<T>((l & 1) ? A.d1 : A.d0, tp.off);
    T* dnew = vec<T>((l & 1) ? A.d0 : A.d1, tp.off);
    T* q = vec<T>(A.q, tp.off);
    const int M = tp.M, N = tp.N;
    double sdq = 0.0;
    // rows of the tile: x is loaded (with the operand's loads, two rows ahead)
    // only for the tile's own elements, never for its halo
    const int i_end = tp.i0 + (TH > 0 ? TH : tp.rows);
    march_tile<TH, T>(
        tp, U, V,
        [&](int i, int j) {
          bool ok;
          const size_t p = clamp_at(i, j, M, N, ok);
          // unconditional loads through the clamped index, zeroed outside the grid
          const T s0 = src[p], d0 = dold[p];
          R4<T> v;  // s (or r), inverse diagonal, d_old, x
          v.s = ok ? s0 : T(0);
          v.w = PC == kPcJacobi ? aux[p] : T(1);
          v.d = ok ? d0 : T(0);
          v.x = T(0);
          if (pend && i >= tp.i0 && i < i_end && j >= tp.j0 && j < tp.j0 + kTW) v.x = ld_stream(x + p);
          return v;
        },
        [&](const R4<T>& v) { return (PC == kPcJacobi ? v.s * v.w : v.s) + beta * v.d; },
        [&](int i, int j, T dv, T qv, const R4<T>& raw) {
          const size_t p = (size_t)i * N + j;
          st_stream(dnew + p, dv);
          q[p] = qv;
          if (pend) st_stream(x + p, raw.x + ap * raw.d);
          sdq += (double)dv * (double)qv;
        });
    sdq = wave_sum(sdq);
    if (lane_id() == 0) store_partial(A.P + 0 * A.pstride + g, sdq);
    if (A.fuse_pw >= 0) {
      const MapDesc& dm = A.desc[tp.m];
      const int sl[1] = {0};
      fused_finish<kFinAlpha, 1>(arrival(A), sl, dm.tile0, g - dm.tile0, dm.ntiles, dm.gb, A.desc,
                                 A.ms, tp.m, kFinishNone, A.fuse_pw, &fflag, fred);
    }
  }
}

// update: r -= alpha q (the step alpha d is added to x by the next SpMV), or,
// when l is a multiple of the replacement period, x_new = x + alpha d into
// the other x buffer and r = b - A x_new; pointwise s; partials r.r, r.s
// Five waves per SIMD fit without spills (96 VGPRs); the update is a short
// stream, so the extra wave in flight helps a little (about 1 %).
template <typename T, int PC, int TH>
__global__ void __launch_bounds__(64, 5) k_e_update(EArgs A) {
  __shared__ double fred[3];
  __shared__ int fflag;
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const MapState& st = A.ms[tp.m];
    if (st.state != kRun) continue;
    const long long l = st.l;
    const T alpha = (T)st.alpha;
    const bool replace = (l % st.period) == 0;
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    const T* aux = cvec<T>(A.aux, tp.off);
    const T* b = cvec<T>(A.b, tp.off);
    const T* q = cvec<T>(A.q, tp.off);
    T* r = vec<T>(A.r, tp.off);
    const int M = tp.M, N = tp.N;
    double srr = 0.0, srs = 0.0;
    if (replace) {
      const T* xold = cvec<T>(st.xi ? A.x1 : A.x0, tp.off);
      T* xnew = vec<T>(st.xi ? A.x0 : A.x1, tp.off);
      const T* d = cvec<T>((l & 1) ? A.d0 : A.d1, tp.off);
      march_tile<TH, T>(
          tp, U, V,
          [&](int i, int j) {
            bool ok;
            const size_t p = clamp_at(i, j, M, N, ok);
            const T x0 = xold[p], d0 = d[p];
            R3<T> v;  // x_old, unused, d; zeroed outside the grid
            v.s = ok ? x0 : T(0);
            v.w = T(1);
            v.d = ok ? d0 : T(0);
            return v;
          },
          [&](const R3<T>& v) { return v.s + alpha * v.d; },
          [&](int i, int j, T xv, T ax) {
            const size_t p = (size_t)i * N + j;
            const T rv = b[p] - ax;
            xnew[p] = xv;
            r[p] = rv;
            const T sv = PC == kPcJacobi ? rv * aux[p] : rv;
            srr += (double)rv * (double)rv;
            srs += (double)rv * (double)sv;
          });
    } else {
      // elementwise; loads through a clamped column (always executed, so the
      // loads of several rows can be in flight), stores only on the map
      const int l = lane_id();
      const int ja = min(tp.j0 + l, N - 1), jb = min(tp.j0 + 64 + l, N - 1);
      const bool oka = tp.j0 + l < N, okb = tp.j0 + 64 + l < N;
      const int kend = min(TH > 0 ? TH : tp.rows, M - tp.i0);
      // eight rows at a time: all loads of the group (through a clamped row)
      // are issued before its first store, so 32 loads per wave are in flight
      auto walk = [&](auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        constexpr int G = 8;
        for (int k0 = 0; k0 < kend; k0 += G) {
          T rv[G][2], qv[G][2], wv[G][2];
#pragma unroll
          for (int c = 0; c < G; ++c) {
            const size_t row = (size_t)min(tp.i0 + k0 + c, M - 1) * N;
            const size_t pa = row + ja, pb = row + jb;
            rv[c][0] = r[pa], rv[c][1] = r[pb];
            qv[c][0] = ld_stream(q + pa), qv[c][1] = ld_stream(q + pb);
            wv[c][0] = PC == kPcJacobi ? aux[pa] : T(1);
            wv[c][1] = PC == kPcJacobi ? aux[pb] : T(1);
          }
#pragma unroll
          for (int c = 0; c < G; ++c) {
            if (k0 + c >= kend) break;  // uniform over the wave
            const size_t row = (size_t)(tp.i0 + k0 + c) * N;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              if (!FULL && !(h ? okb : oka)) continue;
              const size_t p = row + (h ? jb : ja);
              const T rn = rv[c][h] - alpha * qv[c][h];
              r[p] = rn;
              const T sv = PC == kPcJacobi ? rn * wv[c][h] : rn;
              srr += (double)rn * (double)rn;
              srs += (double)rn * (double)sv;
            }
          }
        }
      };
      if (tp.j0 + kTW <= N) walk(std::true_type());
      else walk(std::false_type());
    }
    srr = wave_sum(srr);
    srs = wave_sum(srs);
    if (lane_id() == 0) {
      store_partial(A.P + 0 * A.pstride + g, srr);
      store_partial(A.P + 1 * A.pstride + g, srs);
    }
    if (A.fuse_pw >= 0) {
      const MapDesc& dm = A.desc[tp.m];
      const int sl[2] = {0, 1};
      fused_finish<kFinUpdate, 2>(arrival(A), sl, dm.tile0, g - dm.tile0, dm.ntiles, dm.gb, A.desc,
                                  A.ms, tp.m, kFinishNone, A.fuse_pw, &fflag, fred);
    }
  }
}

// ---------------------------------------------------------------------------
// Two-colour ILU(0) = IC(0) and SSOR of Eq. (7)'s matrix (a GPU-parallel
// change of M; the paper's sweeps use the natural order).  Pixel (i, j) is
// "even" when i + j is even.  With the even pixels ordered first the matrix is
// [[D_e, -B], [-B^T, D_o]]: no two pixels of one colour are coupled, so the
// no-fill factorisation keeps the even diagonal as pivots and gives the odd
// pivots p_o = a_oo - sum over even neighbours e of a_oe^2 / a_ee (SSOR: every
// pivot a / omega).  M = (P + L) P^-1 (P + L^T) (over 2 - omega for SSOR) is
// applied in two passes, c = 2 - omega for SSOR and 1 otherwise:
//   odd pixels:  s_o = c (r_o + sum_e w_oe r_e / p_e) / p_o   (forward solve)
//   even pixels: s_e = (c r_e + sum_o w_eo s_o) / p_e         (backward solve)
// Each pass is a stencil march of Eq. (7) with an operand that is zero on the
// pixels it writes, so the neighbour sum is -(A x) there; the first pass only
// writes odd pixels and the second only even ones, and each reads s only on
// the colour it does not write.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) k_e_tc_pivots(EArgs A, int ssor, double omega) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    T* piv = vec<T>(A.aux, tp.off);
    unsigned char* iso = const_cast<unsigned char*>(A.iso) + tp.off;
    const int M = tp.M, N = tp.N;
    auto diag = [&](int i, int j) {
      return ldz(U, i, j - 1, M, N) + ldz(U, i, j, M, N) + ldz(V, i - 1, j, M, N) + ldz(V, i, j, M, N);
    };
    march_points(tp, [&](int i, int j) {
      const size_t p = (size_t)i * N + j;
      const T d = diag(i, j);
      iso[p] = d == T(0) ? 1 : 0;
      T q = d;
      if (d == T(0)) {
        q = T(1);  // isolated pixel: identity row, output forced to zero
      } else if (ssor) {
        q = d / (T)omega;
      } else if ((i + j) & 1) {
        // couplings to the four (even) neighbours and their diagonals
        const T w[4] = {ldz(U, i, j - 1, M, N), ldz(U, i, j, M, N), ldz(V, i - 1, j, M, N),
                        ldz(V, i, j, M, N)};
        const int ni[4] = {i, i, i - 1, i + 1}, nj[4] = {j - 1, j + 1, j, j};
        T sub = T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (w[k] != T(0)) sub += w[k] * w[k] / diag(ni[k], nj[k]);
        q = d - sub;
        if (q < T(1e-4) * d) q = d;  // the pivot floor of the natural-order factorisation
      }
      piv[p] = q;
    });
  }
}

template <typename T, int PASS, int TH>
__global__ void __launch_bounds__(64) k_e_twocolor(EArgs A, T c) {
  __shared__ double fred[3];
  __shared__ int fflag;
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    if (A.ms[tp.m].state != A.expect) continue;
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    const T* piv = cvec<T>(A.aux, tp.off);
    const T* r = cvec<T>(A.r, tp.off);
    T* s = vec<T>(A.s, tp.off);
    const unsigned char* iso = A.iso + tp.off;
    const int M = tp.M, N = tp.N;
    double part = 0.0;
    march_tile<TH, T>(
        tp, U, V,
        [&](int i, int j) {
          bool ok;
          const size_t p = clamp_at(i, j, M, N, ok);
          const bool even = ((i + j) & 1) == 0;
          R3<T> v;  // pass 0: r and the pivot on even pixels; pass 1: s on odd pixels
          if (PASS == 0) {
            const T r0 = r[p], p0 = piv[p];
            v.s = ok && even ? r0 : T(0);
            v.w = p0;
          } else {
            const T s0 = s[p];
            v.s = ok && !even ? s0 : T(0);
            v.w = T(1);
          }
          v.d = T(0);
          return v;
        },
        [&](const R3<T>& v) { return PASS == 0 ? v.s / v.w : v.s; },
        [&](int i, int j, T xv, T ax) {
          const size_t p = (size_t)i * N + j;
          const bool even = ((i + j) & 1) == 0;
          if (PASS == 0) {
            if (!even) s[p] = iso[p] ? T(0) : c * (r[p] - ax) / piv[p];
          } else {
            const T rv = r[p];
            T sv = xv;
            if (even) {
              sv = iso[p] ? T(0) : (c * rv - ax) / piv[p];
              s[p] = sv;
            }
            part += (double)rv * (double)sv;
          }
        });
    if (PASS == 1) {
      part = wave_sum(part);
      if (lane_id() == 0) store_partial(A.P + 1 * A.pstride + g, part);
      if (A.fin_mode) {
        const MapDesc& dm = A.desc[tp.m];
        const int sl[1] = {1};
        fused_finish<kFinTailS, 1>(arrival(A), sl, dm.tile0, g - dm.tile0, dm.ntiles, dm.gb, A.desc,
                                   A.ms, tp.m, A.fin_mode, 0, &fflag, fred);
      }
    }
  }
}

// y = A x for the step entry point (x in A.s, y in A.q)
template <typename T>
__global__ void __launch_bounds__(64) k_e_apply(EArgs A) {
  TILE_LOOP(A) {
    const int g = TILE_G(A);
    const TilePos tp = tile_pos(A.desc, A.tile_map, g);
    const T* U = cvec<T>(A.U, tp.off);
    const T* V = cvec<T>(A.V, tp.off);
    const T* x = cvec<T>(A.s, tp.off);
    T* y = vec<T>(A.q, tp.off);
    const int M = tp.M, N = tp.N;
    march_tile<0, T>(tp, U, V, [&](int i, int j) { return ldz(x, i, j, M, N); },
                     [](T v) { return v; },
                     [&](int i, int j, T, T ax) { y[(size_t)i * N + j] = ax; });
  }
}

// ---------------------------------------------------------------------------
// Finisher: one block per map, fixed-order sums of the map's partials, then
// the map's PCG state advances.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_e_finish(const MapDesc* __restrict__ desc, MapState* ms,
                                                  const double* __restrict__ P, long long pstride,
                                                  int op, int expect, int mode, int pointwise) {
  __shared__ double red[3 * 4];
  const int m = blockIdx.x;
  if (expect >= 0 && ms[m].state != expect) return;
  const FinSrc src{P, pstride, nullptr, 0};
  finish_map<false>(desc, ms, src, m, op, mode, pointwise, red);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// Grid of the tile kernels: the next power of two >= the active tiles, capped
// (blocks stride over the list, so any grid is correct; few distinct shapes
// keep captured graphs reusable as the active set shrinks).
int egrid(const Engine& e, int ntiles) {
  int g = 1;
  while (g < ntiles && g < e.grid) g <<= 1;
  return std::max(1, std::min(g, e.grid));
}

EArgs make_args(const Engine& e) {
  EArgs a;
  a.desc = e.desc;
  a.ms = e.ms;
  a.tile_map = e.tile_map;
  a.act = e.act;
  a.act_cap = (int)e.cap_tiles;
  a.counts = e.counts;
  a.P = e.P;
  a.pstride = e.pstride;
  a.U = e.U;
  a.V = e.V;
  a.aux = e.aux;
  a.x0 = e.x[0];
  a.x1 = e.x[1];
  a.d0 = e.d[0];
  a.d1 = e.d[1];
  a.r = e.r;
  a.s = e.s;
  a.q = e.q;
  a.b = e.b;
  a.dx = e.dx;
  a.dy = e.dy;
  a.phi_prev = e.phi_prev;
  a.r64 = e.r64;
  a.iso = e.iso;
  a.fcnt = e.fcnt;
  a.gcnt = e.gcnt;
  a.gsum = e.gsum;
  a.gstride = e.gstride;
  a.fuse_pw = -1;
  a.expect = kRun;
  a.fin_mode = 0;
  return a;
}

void e_wrapdiff(hipStream_t st, const Engine& e, int ntiles, bool zero_phi) {
  hipLaunchKernelGGL(k_e_wrapdiff, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e),
                     zero_phi ? 1 : 0);
}

void e_check(hipStream_t st, const Engine& e, int ntiles, unsigned int* bad) {
  hipLaunchKernelGGL(k_e_check, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e), bad);
}

template <typename T>
void e_weights(hipStream_t st, const Engine& e, int ntiles, double p, double tau) {
  hipLaunchKernelGGL(k_e_weights<T>, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e),
                     2.0 - p, tau);
}

template <typename T>
void e_diag(hipStream_t st, const Engine& e, int ntiles, bool inv) {
  hipLaunchKernelGGL(k_e_diag<T>, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e),
                     inv ? 1 : 0);
}

template <typename T>
void e_rhs(hipStream_t st, const Engine& e, int ntiles, int mode) {
  hipLaunchKernelGGL(k_e_rhs<T>, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e), mode);
}

template <typename T>
void e_pass(hipStream_t st, const Engine& e, int ntiles, int op) {
  hipLaunchKernelGGL(k_e_pass<T>, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e), op);
}

template <typename T, int PC>
static void e_resid_pc(hipStream_t st, const Engine& e, int ntiles, bool confirm) {
  if (confirm)
    hipLaunchKernelGGL((k_e_resid<T, PC, 1>), dim3(egrid(e, ntiles)), dim3(64), 0, st,
                       make_args(e));
  else
    hipLaunchKernelGGL((k_e_resid<T, PC, 0>), dim3(egrid(e, ntiles)), dim3(64), 0, st,
                       make_args(e));
}

template <typename T>
void e_resid(hipStream_t st, const Engine& e, int ntiles, int pc, bool confirm) {
  if (pc == kPcJacobi) e_resid_pc<T, kPcJacobi>(st, e, ntiles, confirm);
  else e_resid_pc<T, kPcNone>(st, e, ntiles, confirm);
}

template <typename T, int PC>
static void e_spmv_pc(hipStream_t st, const Engine& e, int gr, int fuse_pw) {
  EArgs a = make_args(e);
  a.fuse_pw = fuse_pw;
  switch (e.th) {
    case 4: hipLaunchKernelGGL((k_e_spmv<T, PC, 4>), dim3(gr), dim3(64), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_e_spmv<T, PC, 8>), dim3(gr), dim3(64), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_e_spmv<T, PC, 16>), dim3(gr), dim3(64), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_e_spmv<T, PC, 32>), dim3(gr), dim3(64), 0, st, a); break;
    default: hipLaunchKernelGGL((k_e_spmv<T, PC, 0>), dim3(gr), dim3(64), 0, st, a); break;
  }
}

// fused: the launch also runs the per-map finisher of its partials (alpha
// after the SpMV, the update's stop tests and pointwise beta after the update)
template <typename T>
void e_spmv(hipStream_t st, const Engine& e, int ntiles, int pc, bool fused) {
  const int gr = egrid(e, ntiles);
  const int pw = pc == kPcNone || pc == kPcJacobi ? 1 : 0;
  const int f = fused ? pw : -1;
  if (pc == kPcNone) e_spmv_pc<T, kPcNone>(st, e, gr, f);
  else if (pc == kPcJacobi) e_spmv_pc<T, kPcJacobi>(st, e, gr, f);
  else e_spmv_pc<T, kPcDct>(st, e, gr, f);
}

template <typename T, int PC>
static void e_update_pc(hipStream_t st, const Engine& e, int gr, int fuse_pw) {
  EArgs a = make_args(e);
  a.fuse_pw = fuse_pw;
  switch (e.th) {
    case 4: hipLaunchKernelGGL((k_e_update<T, PC, 4>), dim3(gr), dim3(64), 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_e_update<T, PC, 8>), dim3(gr), dim3(64), 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_e_update<T, PC, 16>), dim3(gr), dim3(64), 0, st, a); break;
    case 32: hipLaunchKernelGGL((k_e_update<T, PC, 32>), dim3(gr), dim3(64), 0, st, a); break;
    default: hipLaunchKernelGGL((k_e_update<T, PC, 0>), dim3(gr), dim3(64), 0, st, a); break;
  }
}

template <typename T>
void e_update(hipStream_t st, const Engine& e, int ntiles, int pc, bool fused) {
  const int gr = egrid(e, ntiles);
  const int pw = pc == kPcNone || pc == kPcJacobi ? 1 : 0;
  const int f = fused ? pw : -1;
  if (pc == kPcJacobi) e_update_pc<T, kPcJacobi>(st, e, gr, f);
  else e_update_pc<T, kPcNone>(st, e, gr, f);
}

template <typename T>
void e_tc_pivots(hipStream_t st, const Engine& e, int ntiles, bool ssor, double omega) {
  hipLaunchKernelGGL(k_e_tc_pivots<T>, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e),
                     ssor ? 1 : 0, omega);
}

template <typename T, int PASS>
static void e_twocolor_pass(hipStream_t st, const Engine& e, int gr, const EArgs& a, T c) {
  switch (e.th) {
    case 4: hipLaunchKernelGGL((k_e_twocolor<T, PASS, 4>), dim3(gr), dim3(64), 0, st, a, c); break;
    case 8: hipLaunchKernelGGL((k_e_twocolor<T, PASS, 8>), dim3(gr), dim3(64), 0, st, a, c); break;
    case 16: hipLaunchKernelGGL((k_e_twocolor<T, PASS, 16>), dim3(gr), dim3(64), 0, st, a, c); break;
    case 32: hipLaunchKernelGGL((k_e_twocolor<T, PASS, 32>), dim3(gr), dim3(64), 0, st, a, c); break;
    default: hipLaunchKernelGGL((k_e_twocolor<T, PASS, 0>), dim3(gr), dim3(64), 0, st, a, c); break;
  }
}

// s = M^-1 r of the two-colour preconditioner for the maps in state `expect`;
// fin_mode != 0 runs the per-map finisher of r^T s at the end of the second pass
template <typename T>
void e_twocolor(hipStream_t st, const Engine& e, int ntiles, int expect, bool ssor, double omega,
                int fin_mode) {
  const int gr = egrid(e, ntiles);
  EArgs a = make_args(e);
  a.expect = expect;
  const T c = ssor ? (T)(2.0 - omega) : T(1);
  e_twocolor_pass<T, 0>(st, e, gr, a, c);
  a.fin_mode = fin_mode;
  e_twocolor_pass<T, 1>(st, e, gr, a, c);
}

template <typename T>
void e_apply(hipStream_t st, const Engine& e, int ntiles) {
  hipLaunchKernelGGL(k_e_apply<T>, dim3(egrid(e, ntiles)), dim3(64), 0, st, make_args(e));
}

void e_finish(hipStream_t st, const Engine& e, int op, int expect, int mode, bool pointwise) {
  hipLaunchKernelGGL(k_e_finish, dim3(e.n_maps), dim3(256), 0, st, e.desc, e.ms, e.P, e.pstride,
                     op, expect, mode, pointwise ? 1 : 0);
}

#define LPU_INST_E(T)                                                                   \
  template void e_weights<T>(hipStream_t, const Engine&, int, double, double);         \
  template void e_diag<T>(hipStream_t, const Engine&, int, bool);                      \
  template void e_rhs<T>(hipStream_t, const Engine&, int, int);                        \
  template void e_pass<T>(hipStream_t, const Engine&, int, int);                       \
  template void e_resid<T>(hipStream_t, const Engine&, int, int, bool);                \
  template void e_spmv<T>(hipStream_t, const Engine&, int, int, bool);                       \
  template void e_update<T>(hipStream_t, const Engine&, int, int, bool);                     \
  template void e_apply<T>(hipStream_t, const Engine&, int);                            \
  template void e_tc_pivots<T>(hipStream_t, const Engine&, int, bool, double);         \
  template void e_twocolor<T>(hipStream_t, const Engine&, int, int, bool, double, int);
LPU_INST_E(float)
LPU_INST_E(double)

}  // namespace lpu
