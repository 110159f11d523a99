// Batched DCT Poisson preconditioner: grouped contractions over all active maps.
//
// DCT (s = L0^+ r, L0 the unit-weight Neumann Laplacian):
//   s = C_M^T [ (C_M r C_N^T) ./ Lambda ] C_N,
//   C_n[k][j] = s_k cos(pi k (2j+1) / (2n)), Lambda_kl = (2 - 2cos(pi k/M)) + (2 - 2cos(pi l/N)),
//   zero mode dropped.  Four stages of Out^T = X B^T (rows of X transformed by
//   the basis in B, result stored transposed):
//     stage 0: X = r  (M x N), B = C_N   -> t1 (N x M)
//     stage 1: X = t1 (N x M), B = C_M   -> t2 (M x N), t2 ./= Lambda
//     stage 2: X = t2 (M x N), B = C_N^T -> t1 (N x M)
//     stage 3: X = t1 (N x M), B = C_M^T -> s  (M x N), zero on isolated pixels,
//              FP64 partial of r^T s per 64 x 64 tile.
// Every map contributes ceil(M/64) ceil(N/64) output tiles to every stage.

#include "lpu_internal.h"
#include "lpu_device.h"
#include "lpu_finish.h"

namespace lpu {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

struct DArgs {
  const MapDesc* desc;
  MapState* ms;
  const int* dtile_map;
  const int* dact;
  const int* counts;
  double* P;
  long long pstride;
  const void* X;
  void* Out;
  const void* rvec;
  const unsigned char* iso;
  int stage, expect;
  int trows;  // output tile rows: 64 (dense kernels) or 128 (even/odd kernels)
  int cidx;   // counts[] slot holding the length of `dact`
  int dact_cap;  // entries of `dact` (its capacity)
  int *fcnt, *gcnt;  // arrival counters of the fused finisher
  double* gsum;      // its group sums (rows of gstride)
  long long gstride;
  const EoTile* eot;  // even/odd tile records: [stage parity][global DCT tile]
  long long eot_cap;
  int fin_mode;  // last stage of the even/odd kernels: 0, or the FinishMode of
                 // the fused finisher (the map's r^T s, beta and stop tests)
};

struct DTile {
  int m, R, K, r0, c0;
  long long off;
  const DctTabDev* tab;
  bool ok;
};

__device__ __forceinline__ DTile dtile(const DArgs& a, int g) {
  DTile t;
  t.m = a.dtile_map[g];
  const MapDesc& d = a.desc[t.m];
  t.ok = a.ms[t.m].state == a.expect;
  const bool rows_m = (a.stage & 1) == 0;
  t.R = rows_m ? d.M : d.N;
  t.K = rows_m ? d.N : d.M;
  const int tiles_r = (t.R + a.trows - 1) / a.trows;
  const int local = g - d.dtile0;
  t.r0 = (local % tiles_r) * a.trows;
  t.c0 = (local / tiles_r) * kDT;
  t.off = d.off;
  t.tab = rows_m ? d.tabN : d.tabM;
  return t;
}

// ---------------------------------------------------------------------------
// MFMA stage (mixed path): 4 waves, 32 x 32 outputs each, K step 32; lane l
// supplies row (l mod 16) and K values 8*(l/16) .. +7 of the 16x16x32 ops.
// ---------------------------------------------------------------------------
__device__ __forceinline__ f32x8 load_x8(const float* __restrict__ X, int R, int K, int row, int k,
                                         bool vec_ok) {
  f32x8 v;
  if (row < R && vec_ok && k + 7 < K) {
    const float4* p = reinterpret_cast<const float4*>(X + (size_t)row * K + k);
    const float4 a = p[0], b = p[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (row < R && k + e < K) ? X[(size_t)row * K + k + e] : 0.0f;
  }
  return v;
}

__device__ __forceinline__ u16x8 load_t8(const uint16_t* __restrict__ B, int K, int row, int k,
                                         bool vec_ok) {
  u16x8 v;
  if (row < K && vec_ok && k + 7 < K) {
    v = *as_global(reinterpret_cast<const u16x8*>(B + (size_t)row * K + k));
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (row < K && k + e < K) ? as_global(B)[(size_t)row * K + k + e] : 0;
  }
  return v;
}

__device__ __forceinline__ float fp16_scale(float amax) {
  if (!(amax > 0.0f) || !isfinite(amax)) return 1.0f;
  int e;
  frexpf(amax, &e);
  return ldexpf(1.0f, 14 - e);
}

template <int SPLIT>
__global__ void __launch_bounds__(256) k_e_dct_mfma(DArgs a) {
  __shared__ double red[4];
  const int nact = a.counts[a.cidx];
  // the block's first list entry is requested with the list's length
  const int g_first = a.dact[min((int)blockIdx.x, max(a.dact_cap - 1, 0))];
  __asm__ volatile("" ::"s"(nact), "s"(g_first));  // both loads issued before the loop test
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t_ = blockIdx.x; t_ < nact; t_ += gridDim.x) {
    const int g = t_ == (int)blockIdx.x ? g_first : a.dact[t_];
    if (g < 0) continue;  // padding slot of the XCD-ordered list
    const DTile t = dtile(a, g);
    if (!t.ok) continue;  // uniform over the block
    const int R = t.R, K = t.K;
    const float* X = reinterpret_cast<const float*>(a.X) + t.off;
    float* Out = reinterpret_cast<float*>(a.Out) + t.off;
    const uint16_t* Bh;
    const uint16_t* Bl;
    if (a.stage < 2) {
      Bh = SPLIT ? t.tab->chi : t.tab->ch;
      Bl = t.tab->clo;
    } else {
      Bh = SPLIT ? t.tab->cthi : t.tab->cth;
      Bl = t.tab->ctlo;
    }
    const int r0 = t.r0 + (w & 1) * 32, c0 = t.c0 + (w >> 1) * 32;
    const int lr = lane & 15, kg = (lane >> 4) * 8;
    const bool vec_ok = (K % 8) == 0;
    float xs = 1.0f, inv_xs = 1.0f;
    MapState& st = a.ms[t.m];
    if (!SPLIT) {
      const float amax = a.stage == 0 ? (float)sqrt(st.rr) * 1.0000001f : st.amax[a.stage];
      xs = fp16_scale(amax);
      inv_xs = 1.0f / xs;
    }
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      u16x8 bh[2], bl[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bh[j] = load_t8(Bh, K, c0 + j * 16 + lr, k0 + kg, vec_ok);
        if (SPLIT) bl[j] = load_t8(Bl, K, c0 + j * 16 + lr, k0 + kg, vec_ok);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const f32x8 xv = load_x8(X, R, K, r0 + i * 16 + lr, k0 + kg, vec_ok);
        if (SPLIT) {
          bf16x8 xh, xl;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const __bf16 h = (__bf16)xv[e];
            xh[e] = h;
            xl[e] = (__bf16)(xv[e] - (float)h);
          }
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const bf16x8 ch = __builtin_bit_cast(bf16x8, bh[j]);
            const bf16x8 cl = __builtin_bit_cast(bf16x8, bl[j]);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ch, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, cl, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, ch, acc[i][j], 0, 0, 0);
          }
        } else {
          f16x8 xh;
#pragma unroll
          for (int e = 0; e < 8; ++e) xh[e] = (_Float16)(xv[e] * xs);
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(xh, __builtin_bit_cast(f16x8, bh[j]),
                                                               acc[i][j], 0, 0, 0);
        }
      }
    }
    // epilogue: lane holds D[row 4*(lane/16) + e][col lane mod 16] of each 16x16 tile
    const MapDesc& d = a.desc[t.m];
    const float* rv = reinterpret_cast<const float*>(a.rvec) + t.off;
    const unsigned char* iso = (a.iso && d.use_iso) ? a.iso + t.off : nullptr;
    double part = 0.0;
    float vmax = 0.0f;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = c0 + j * 16 + lr;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int rb = r0 + i * 16 + (lane >> 4) * 4;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = rb + e;
          float y = acc[i][j][e] * inv_xs;
          const bool in = c < K && r < R;
          if (a.stage == 1 && in)
            y = (c == 0 && r == 0) ? 0.0f
                                   : (float)((double)y / (as_global(d.tabM->lam)[c] + as_global(d.tabN->lam)[r]));
          if (a.stage == 3 && in) {
            const size_t o = (size_t)c * R + r;
            if (iso && iso[o]) y = 0.0f;
            part += (double)rv[o] * (double)y;
          }
          v[e] = y;
          if (in) vmax = fmaxf(vmax, fabsf(y));
        }
        if (c < K) {
          if (rb + 3 < R && (R % 4) == 0) {
            *reinterpret_cast<float4*>(Out + (size_t)c * R + rb) = make_float4(v[0], v[1], v[2], v[3]);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (rb + e < R) Out[(size_t)c * R + rb + e] = v[e];
          }
        }
      }
    }
    if (!SPLIT && a.stage < 3) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) vmax = fmaxf(vmax, __shfl_down(vmax, off, 64));
      if (lane == 0)
        atomicMax(reinterpret_cast<unsigned int*>(&st.amax[a.stage + 1]), __float_as_uint(vmax));
    }
    if (a.stage == 3) {
      double vv[1] = {part};
      block_sum<1>(vv, red);
      if (threadIdx.x == 0) a.P[1 * a.pstride + g] = vv[0];
    }
  }
}

// ---------------------------------------------------------------------------
// Even/odd MFMA stage (mixed path, both sides multiples of 128).
//
// The basis satisfies C[k][n-1-j] = (-1)^k C[k][j].  With h = n/2 and the
// spectrum kept in split order (even k first):
//   forward  X_even = E (x_a + x_b),  X_odd = O (x_a - x_b),
//            x_a = x[0..h), x_b = x[n-1 .. h] (mirrored), E, O the h x h
//            even/odd rows of C restricted to j < h;
//   inverse  u = E^T X_even, v = O^T X_odd;  x[j] = u_j + v_j,
//            x[n-1-j] = u_j - v_j  (j < h).
// Both halve the multiply-adds of the dense transform.
//
// A block owns 128 rows of X and 64 output columns c0 .. c0+63 of the half
// range [0, h), in two halves computed side by side from the same loads:
//   forward: half 0 = even outputs c (A = x_a + x_b), half 1 = odd outputs
//            h + c (A = x_a - x_b);
//   inverse: half 0 = u (spectrum columns [0, h)), half 1 = v (columns
//            [h, n)), combined at the end into outputs c and n-1-c.
// Wave w computes rows 64 (w & 1) .. +63 of half w >> 1 as 4 x 4 MFMA tiles
// of 16 x 16 (64 accumulator registers).  Each K step of KS (32 for the bf16
// split, 64 for fp16, whose operands take half the registers) stages both
// halves of A (128 x KS) and of the table slice (64 x KS) in LDS, converted
// once to bf16 hi/lo (or scaled fp16); the next step's global loads are in
// flight while the MFMAs of the current one run, so a longer step keeps more
// bytes in flight per block.  LDS rows are KS 16-bit values without padding;
// the 16-byte chunk q of row r sits at q ^ swz(r), which keeps both the
// staging writes and the fragment reads free of bank conflicts (rows of 4
// chunks: 8 rows read in one LDS cycle land in 8 distinct bank quads; rows of
// 8 chunks: likewise for 8 or 16 rows).
// ---------------------------------------------------------------------------
template <int NC>
__device__ __forceinline__ int swz(int r) {
  return NC == 4 ? (((r >> 1) ^ (r >> 2)) & 3) : ((r ^ (r >> 3)) & 7);
}
// offset (16-bit elements) of element 8q + e of LDS row r (rows of NC chunks)
template <int NC>
__device__ __forceinline__ int lds_at(int r, int q) { return r * (8 * NC) + ((q ^ swz<NC>(r)) << 3); }

typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

// NW: 16-column groups per wave.  NW = 4 is the tile described above
// (64 output pairs).  NW = 8 (scaled fp16 only, 32-wide K steps) covers two
// such tiles side by side, 128 output pairs, from the same staged rows of X:
// half the re-reads of X and less LDS traffic per output.  It pays on
// launches of many tiles only (half as many tiles to spread over the CUs):
// the first three stages of the batch's launches of at least 1024 list
// positions take 6-9 % less time, those of a 4096 x 4096 map 15 % less.  A
// wide tile is named by its left narrow tile; where the map has no right
// partner (h an odd multiple of 64) it stages its own table rows twice and
// stores the left half only.  Per output the MFMAs run over the same K
// chunks in the same order in both shapes, so the outputs are identical.
template <int SPLIT, int INV, int IN16, int OUT16, int NW>
__global__ void __launch_bounds__(256, 2) k_e_dct_eo(DArgs a) {
  static_assert(NW == 4 || (NW == 8 && !SPLIT && OUT16), "wide tiles: scaled fp16, stages 0-2");
  constexpr int NP = SPLIT ? 2 : 1;                // hi (+ lo) planes
  constexpr int KS = (SPLIT || NW == 8) ? 32 : 64;  // K step
  constexpr int NC = KS / 8;                       // 16-byte chunks per LDS row
  constexpr int kBW = 16 * NW;                     // table rows per half (output pairs)
  constexpr int kA = 128 * KS, kB = kBW * KS;      // elements of one A / B half-plane
  constexpr int kStage = NP * 2 * (kA + kB) * 2;   // bytes of staged operands
  constexpr int kXchg = 2 * 2 * 16 * 64 * 16;      // bytes of the inverse's u/v exchange (4 column groups)
  constexpr int kSmem = kStage > kXchg ? kStage : kXchg;
  constexpr int VPT = IN16 ? 8 : 4;                // X staging: values per thread and load
  constexpr int TPR = KS / VPT;                    // X staging: threads per row
  constexpr int XP = 128 * TPR / 256;              // X staging passes (rows xr + XP-stride)
  constexpr int SEGS = 256 / NC;                   // table staging: segments per pass
  constexpr int TP = NP * 2 * kBW / SEGS;          // table staging passes
  static_assert(NW == 4 || SEGS == 64, "wide tiles: a pass stages 64 rows of one half");
  __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
  __shared__ double red[4];
  __shared__ double fred[3 * 4];
  __shared__ int fflag;
  uint16_t* As = reinterpret_cast<uint16_t*>(smem);  // [plane][half][128 x KS]
  uint16_t* Bs = As + NP * 2 * kA;                   // [plane][half][kBW x KS]
  const int nact = a.counts[a.cidx];
  // the block's first list entry is requested with the list's length
  const int g_first = a.dact[min((int)blockIdx.x, max(a.dact_cap - 1, 0))];
  __asm__ volatile("" ::"s"(nact), "s"(g_first));  // both loads issued before the loop test
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int wr = (w & 1) * 64, hf = w >> 1;
  const int lr = lane & 15, kq = lane >> 4;        // MFMA operand map: row lr, k chunk kq
  const int xr = tid / TPR, xk = (tid % TPR) * VPT;  // X staging: rows xr + (256/TPR) p, k xk ..
  static_assert(!(SPLIT && (IN16 || OUT16)), "the bf16 split keeps FP32 intermediates");
  const int bseg = tid / NC, bq = tid % NC;         // table staging: segment, 16-byte chunk
  for (int t_ = blockIdx.x; t_ < nact; t_ += gridDim.x) {
    const int g = t_ == (int)blockIdx.x ? g_first : a.dact[t_];
    if (g < 0) continue;  // padding slot of the XCD-ordered list
    // the tile's record (one load); its first K step is fetched before the
    // map's state is read, so the two round trips overlap
    const EoTile& tt = a.eot[(size_t)(a.stage & 1) * a.eot_cap + g];
    const int R = tt.R, n = tt.K, h = n >> 1, c0 = tt.c0, r0 = tt.r0, tm = tt.m;
    const long long toff = tt.off;
    const int t_local = tt.local, t_ndt = tt.ndt, t_gbd = tt.gbd;
    const float t_lmin = tt.lmin;
    // wide tiles: does the right partner exist (uniform over the block)?
    const bool full = NW == 4 || c0 + 128 <= h;
    const double* t_lam_m = tt.lam_m;
    const double* t_lam_n = tt.lam_n;
    const float* X = reinterpret_cast<const float*>(a.X) + toff;
    const uint16_t* X16 = reinterpret_cast<const uint16_t*>(a.X) + toff;
    float* Out = reinterpret_cast<float*>(a.Out) + toff;
    uint16_t* Out16 = reinterpret_cast<uint16_t*>(a.Out) + toff;
    const uint16_t* T0 = INV ? (SPLIT ? tt.ti[1] : tt.ti[0]) : (SPLIT ? tt.tf[1] : tt.tf[0]);
    const uint16_t* T1 = INV ? tt.ti[2] : tt.tf[2];
    float xs = 1.0f, inv_xs = 1.0f, os = 1.0f;
    // register staging of one K step
    float4 sa[IN16 ? 1 : XP], sb[IN16 ? 1 : XP];
    u16x8 ha[IN16 ? XP : 1], hb[IN16 ? XP : 1];
    u16x8 sT[TP];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int p = 0; p < XP; ++p) {
        const size_t ro = (size_t)(r0 + xr + (256 / TPR) * p) * n;
        const int ka = k0 + xk, kb = INV ? h + k0 + xk : n - VPT - k0 - xk;
        if (IN16) {
          ha[p] = *reinterpret_cast<const u16x8*>(X16 + ro + ka);
          hb[p] = *reinterpret_cast<const u16x8*>(X16 + ro + kb);
        } else {
          sa[p] = *reinterpret_cast<const float4*>(X + ro + ka);
          sb[p] = *reinterpret_cast<const float4*>(X + ro + kb);
        }
      }
#pragma unroll
      for (int p = 0; p < TP; ++p) {
        const int s = p * SEGS + bseg;                // segment: ((half * NP) + plane) * kBW + row
        const int half = s / (kBW * NP), plane = (s / kBW) % NP;
        // a wide tile without its partner stages its own rows twice (the
        // extra outputs are computed but never stored)
        const int row = full ? s % kBW : s % 64;
        const uint16_t* T = plane ? T1 : T0;
        const uint16_t* src = INV ? T + (size_t)(c0 + row) * n + (half ? h : 0) + k0 + 8 * bq
                                  : T + (size_t)((half ? h : 0) + c0 + row) * h + k0 + 8 * bq;
        sT[p] = *as_global(reinterpret_cast<const u16x8*>(src));
      }
    };
    auto stash = [&]() {
      if constexpr (IN16) {
        // fp16 input already carries the stage's scale: the inverse copies
        // it, the forward folds x_a +- x_b in FP32 and rounds once more
#pragma unroll
        for (int p = 0; p < XP; ++p) {
          const int r = xr + (256 / TPR) * p;
          u16x8 v0 = ha[p], v1 = hb[p];
          if (!INV) {
            // whole-vector form: x_b reversed (it holds x[n-1-k] from the top),
            // sum and difference in FP32, one rounding back to fp16
            const f16x8 fa = __builtin_bit_cast(f16x8, ha[p]);
            const f16x8 fbr = __builtin_bit_cast(f16x8, hb[p]);
            const f16x8 fb = __builtin_shufflevector(fbr, fbr, 7, 6, 5, 4, 3, 2, 1, 0);
            const f32x8 a32 = __builtin_convertvector(fa, f32x8);
            const f32x8 b32 = __builtin_convertvector(fb, f32x8);
            v0 = __builtin_bit_cast(u16x8, __builtin_convertvector(a32 + b32, f16x8));
            v1 = __builtin_bit_cast(u16x8, __builtin_convertvector(a32 - b32, f16x8));
          }
          const int o = lds_at<NC>(r, xk >> 3);
          *reinterpret_cast<u16x8*>(As + 0 * kA + o) = v0;
          *reinterpret_cast<u16x8*>(As + 1 * kA + o) = v1;
        }
      } else {
#pragma unroll
      for (int p = 0; p < XP; ++p) {
        const int r = xr + (256 / TPR) * p;
        const float av[4] = {sa[p].x, sa[p].y, sa[p].z, sa[p].w};
        // forward: the b part is x mirrored, x[n-1-k] for k = k0 + xk .. +3
        const float bv[4] = {INV ? sb[p].x : sb[p].w, INV ? sb[p].y : sb[p].z,
                             INV ? sb[p].z : sb[p].y, INV ? sb[p].w : sb[p].x};
        u16x4 hv[2], lv[2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float v0 = INV ? av[e] : av[e] + bv[e];
          const float v1 = INV ? bv[e] : av[e] - bv[e];
          if (SPLIT) {
            const __bf16 h0 = (__bf16)v0, h1 = (__bf16)v1;
            hv[0][e] = __builtin_bit_cast(uint16_t, h0);
            hv[1][e] = __builtin_bit_cast(uint16_t, h1);
            lv[0][e] = __builtin_bit_cast(uint16_t, (__bf16)(v0 - (float)h0));
            lv[1][e] = __builtin_bit_cast(uint16_t, (__bf16)(v1 - (float)h1));
          } else {
            hv[0][e] = __builtin_bit_cast(uint16_t, (_Float16)(v0 * xs));
            hv[1][e] = __builtin_bit_cast(uint16_t, (_Float16)(v1 * xs));
          }
        }
        const int o = lds_at<NC>(r, xk >> 3) + (xk & 4);
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          *reinterpret_cast<u16x4*>(As + (0 * 2 + half) * kA + o) = hv[half];
          if (SPLIT) *reinterpret_cast<u16x4*>(As + (1 * 2 + half) * kA + o) = lv[half];
        }
      }
      }
#pragma unroll
      for (int p = 0; p < TP; ++p) {
        const int s = p * SEGS + bseg;
        const int half = s / (kBW * NP), plane = (s / kBW) % NP, row = s % kBW;
        *reinterpret_cast<u16x8*>(Bs + (plane * 2 + half) * kB + lds_at<NC>(row, bq)) = sT[p];
      }
    };
    f32x4 acc[4][NW];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NW; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nsteps = h / KS;
    // the map's state and the first step's operands are requested together;
    // the compiler barriers keep that order (it would otherwise sink the
    // operand loads behind the state test's branch)
    const int m_state = a.ms[tm].state;
    const double m_rr = a.ms[tm].rr;
    const int t_iso = a.desc[tm].use_iso;
    __asm__ volatile("" ::: "memory");
    fetch(0);
    __asm__ volatile("" ::: "memory");
    if (m_state != a.expect) continue;  // uniform over the block
    const auto* lamMs = as_global(t_lam_m);
    const auto* lamNs = as_global(t_lam_n);
    // output index of column group j and first output row of row group i
    auto out_c = [&](int j) {
      const int c = c0 + 16 * j + lr;
      return INV ? (hf ? n - 1 - c : c) : (hf ? h : 0) + c;
    };
    auto out_rb = [&](int i) { return r0 + wr + 16 * i + 4 * kq; };
    // Everything the epilogue reads is loaded before its first store: loads
    // and stores share one counter, so a load issued after a store would wait
    // for that store too, one memory round trip per output tile.  The
    // eigenvalues are requested here, ahead of the K loop; r and the
    // isolated-pixel flags (stage 3) one column group ahead in the epilogue.
    // Which stages an instance can run: the forward instances with fp16 input
    // (or the split's, which serve both forward stages) run stage 1, the
    // inverse instances with an FP32 output run stage 3.
    constexpr bool kS1 = !INV && (SPLIT || IN16);
    constexpr bool kS3 = INV && !OUT16;
    const bool st1 = kS1 && a.stage == 1, st3 = kS3 && a.stage == 3;
    float lam_c[NW], lam_r[4][4];  // stage 1: eigenvalues along M and N (FP32)
    if (st1) {
#pragma unroll
      for (int j = 0; j < NW; ++j) lam_c[j] = (j < 4 || full) ? (float)lamMs[out_c(j)] : 0.0f;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) lam_r[i][e] = (float)lamNs[out_rb(i) + e];
    }
    if (!SPLIT) {
      // Scaled fp16: power-of-two scales from bounds that hold before any
      // value exists.  The transforms are orthonormal, so every stage output
      // is bounded by the Frobenius norm of r (first forward stage; twice
      // that after the even/odd fold) or of S ./ Lambda <= ||r|| / lambda_min
      // (second forward stage and the first inverse stage).
      const float nr = (float)sqrt(m_rr) * 1.0000001f;
      const float b01 = 2.0f * nr, b23 = nr / t_lmin * 1.0000001f;
      xs = fp16_scale(a.stage <= 1 ? b01 : b23);
      inv_xs = 1.0f / xs;
      os = fp16_scale(a.stage == 0 ? b01 : b23);
    }
    for (int s = 0; s < nsteps; ++s) {
      __syncthreads();  // readers of the previous step (or tile) are done
      stash();
      __syncthreads();
      if (s + 1 < nsteps) fetch((s + 1) * KS);
      const uint16_t* Ah = As + (0 * 2 + hf) * kA;
      const uint16_t* Al = As + (1 * 2 + hf) * kA;
      const uint16_t* Bh = Bs + (0 * 2 + hf) * kB;
      const uint16_t* Bl = Bs + (1 * 2 + hf) * kB;
#pragma unroll
      for (int ks = 0; ks < KS / 32; ++ks) {
      const int q = 4 * ks + kq;
      u16x8 bh[NW], bl[NW];
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        bh[j] = *reinterpret_cast<const u16x8*>(Bh + lds_at<NC>(16 * j + lr, q));
        if (SPLIT) bl[j] = *reinterpret_cast<const u16x8*>(Bl + lds_at<NC>(16 * j + lr, q));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const u16x8 ah = *reinterpret_cast<const u16x8*>(Ah + lds_at<NC>(wr + 16 * i + lr, q));
        u16x8 al;
        if (SPLIT) al = *reinterpret_cast<const u16x8*>(Al + lds_at<NC>(wr + 16 * i + lr, q));
#pragma unroll
        for (int j = 0; j < NW; ++j) {
          if (SPLIT) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bl[j]), acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, al), __builtin_bit_cast(bf16x8, bh[j]), acc[i][j], 0, 0, 0);
          } else {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                __builtin_bit_cast(f16x8, ah), __builtin_bit_cast(f16x8, bh[j]), acc[i][j], 0, 0, 0);
          }
        }
      }
      }  // ks
    }
    // epilogue: lane holds D[row 4*(lane/16) + e][col lane mod 16] of each 16x16 tile,
    // i.e. outputs (c, rb .. rb+3) with rb a multiple of 4
    const float* rv = reinterpret_cast<const float*>(a.rvec) + toff;
    const unsigned char* iso = (a.iso && t_iso) ? a.iso + toff : nullptr;
    // stage 3: r and the isolated-pixel flags at the outputs of one column
    // group, loaded one group ahead of the group being stored
    f32x4 r_cur[4], r_nxt[4];
    unsigned int z_cur[4], z_nxt[4];
    auto load_rz = [&](int j, f32x4 (&rr)[4], unsigned int (&zz)[4]) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const size_t o = (size_t)out_c(j) * R + out_rb(i);
        rr[i] = *as_global(reinterpret_cast<const f32x4*>(rv + o));
        zz[i] = iso ? *as_global(reinterpret_cast<const unsigned int*>(iso + o)) : 0u;
      }
    };
    if (st3) load_rz(0, r_cur, z_cur);
    double part = 0.0;
    auto emit = [&](int i, int j, const float (&y)[4]) {
      const int c = out_c(j), rb = out_rb(i);
      float v[4] = {y[0], y[1], y[2], y[3]};
      if (st1) {
        // spectrum ./ Lambda with the zero mode dropped; an FP32 reciprocal
        // (the preconditioner stays one fixed linear map)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float l = lam_c[j] + lam_r[i][e];
          v[e] = (c == 0 && rb + e == 0) ? 0.0f : v[e] * __builtin_amdgcn_rcpf(l);
        }
      }
      if (st3) {
        // zero on isolated pixels; FP64 partial of r^T s (four outputs at once)
        const unsigned int z = z_cur[i];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if ((z >> (8 * e)) & 0xffu) v[e] = 0.0f;
          part += (double)r_cur[i][e] * (double)v[e];
        }
      }
      if (OUT16) {
        u16x4 hv;
#pragma unroll
        for (int e = 0; e < 4; ++e) hv[e] = __builtin_bit_cast(uint16_t, (_Float16)(v[e] * os));
        *reinterpret_cast<u16x4*>(Out16 + (size_t)c * R + rb) = hv;
      } else {
        *reinterpret_cast<float4*>(Out + (size_t)c * R + rb) = make_float4(v[0], v[1], v[2], v[3]);
      }
    };
    if (!INV) {
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        if (j >= 4 && !full) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float y[4] = {acc[i][j][0] * inv_xs, acc[i][j][1] * inv_xs, acc[i][j][2] * inv_xs,
                              acc[i][j][3] * inv_xs};
          emit(i, j, y);
        }
      }
    } else {
      // u (half 0) and v (half 1) of the same rows meet through LDS: the
      // waves of half 0 write u + v to output c, those of half 1 write
      // u - v to output n-1-c
      f32x4* xg = reinterpret_cast<f32x4*>(smem);  // [half][row group][16 tiles][64 lanes]
      const int oh = hf ^ 1;
      // one round per four column groups (wide tiles: two rounds, the
      // second only when the partner exists; uniform over the block)
#pragma unroll
      for (int jr = 0; jr < NW / 4; ++jr) {
        if (jr > 0 && !full) break;
        __syncthreads();  // every wave is done reading the staged operands (or the last round)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            xg[((hf * 2 + (w & 1)) * 16 + i * 4 + jj) * 64 + lane] = acc[i][4 * jr + jj];
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int j = 4 * jr + jj;
          if (st3 && j < 3) load_rz(j + 1, r_nxt, z_nxt);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const f32x4 o = xg[((oh * 2 + (w & 1)) * 16 + i * 4 + jj) * 64 + lane];  // the other half
            const float y[4] = {(hf ? o[0] - acc[i][j][0] : acc[i][j][0] + o[0]) * inv_xs,
                                (hf ? o[1] - acc[i][j][1] : acc[i][j][1] + o[1]) * inv_xs,
                                (hf ? o[2] - acc[i][j][2] : acc[i][j][2] + o[2]) * inv_xs,
                                (hf ? o[3] - acc[i][j][3] : acc[i][j][3] + o[3]) * inv_xs};
            emit(i, j, y);
          }
          if (st3 && j < 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) r_cur[i] = r_nxt[i], z_cur[i] = z_nxt[i];
          }
        }
      }
    }
    if (st3) {
      double vv[1] = {part};
      block_sum<1>(vv, red);
      if (tid == 0) store_partial(a.P + 1 * a.pstride + g, vv[0]);
      if (a.fin_mode) {
        const int sl[1] = {1};
        fused_finish<kFinTail, 1>(Arrival{a.fcnt, a.gcnt, a.gsum, a.gstride, a.P, a.pstride}, sl,
                                  g - t_local, t_local, t_ndt, t_gbd, a.desc, a.ms, tm,
                                  a.fin_mode, 0, &fflag, fred);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FMA stage (FP64 path, FP32 option): 64 x 64 tile, 16 x 16 threads x 4 x 4.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_e_dct_fma(DArgs a) {
  __shared__ T Xs[16][64 + 4];
  __shared__ T Bs[16][64 + 4];
  __shared__ double red[4];
  const int nact = a.counts[a.cidx];
  // the block's first list entry is requested with the list's length
  const int g_first = a.dact[min((int)blockIdx.x, max(a.dact_cap - 1, 0))];
  __asm__ volatile("" ::"s"(nact), "s"(g_first));  // both loads issued before the loop test
  const int tid = threadIdx.x, tr = tid % 16, tc = tid / 16;
  const int lrow = tid / 4, lk = (tid % 4) * 4;
  for (int t_ = blockIdx.x; t_ < nact; t_ += gridDim.x) {
    const int g = t_ == (int)blockIdx.x ? g_first : a.dact[t_];
    if (g < 0) continue;  // padding slot of the XCD-ordered list
    const DTile t = dtile(a, g);
    if (!t.ok) continue;
    const int R = t.R, K = t.K, r0 = t.r0, c0 = t.c0;
    const T* X = reinterpret_cast<const T*>(a.X) + t.off;
    T* Out = reinterpret_cast<T*>(a.Out) + t.off;
    const T* B;
    if (sizeof(T) == 8)
      B = reinterpret_cast<const T*>(a.stage < 2 ? (const void*)t.tab->c64 : (const void*)t.tab->ct64);
    else
      B = reinterpret_cast<const T*>(a.stage < 2 ? (const void*)t.tab->c32 : (const void*)t.tab->ct32);
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
    for (int k0 = 0; k0 < K; k0 += 16) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + lk + e, rr = r0 + lrow, cc = c0 + lrow;
        Xs[lk + e][lrow] = (rr < R && k < K) ? X[(size_t)rr * K + k] : T(0);
        Bs[lk + e][lrow] = (cc < K && k < K) ? as_global(B)[(size_t)cc * K + k] : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        T xa[4], bb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) xa[i] = Xs[kk][4 * tr + i];
#pragma unroll
        for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][4 * tc + j];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += xa[i] * bb[j];
      }
    }
    const MapDesc& d = a.desc[t.m];
    const T* rv = reinterpret_cast<const T*>(a.rvec) + t.off;
    const unsigned char* iso = (a.iso && d.use_iso) ? a.iso + t.off : nullptr;
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + 4 * tc + j;
      if (c >= K) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + 4 * tr + i;
        if (r >= R) continue;
        const size_t o = (size_t)c * R + r;
        T v = acc[i][j];
        if (a.stage == 1) v = (c == 0 && r == 0) ? T(0) : (T)((double)v / (as_global(d.tabM->lam)[c] + as_global(d.tabN->lam)[r]));
        if (a.stage == 3) {
          if (iso && iso[o]) v = T(0);
          part += (double)rv[o] * (double)v;
        }
        Out[o] = v;
      }
    }
    if (a.stage == 3) {
      double vv[1] = {part};
      block_sum<1>(vv, red);
      if (tid == 0) a.P[1 * a.pstride + g] = vv[0];
    }
    __syncthreads();
  }
}

// Grid of a DCT stage: the next power of two >= the list length, capped; a
// multiple of 8, so list position q always runs on XCD q mod 8.
int dct_grid_for(const Engine& e, int ndtiles) {
  const int cap = std::max(8, e.dct_grid / 8 * 8);
  int g = 8;
  while (g < ndtiles && g < cap) g <<= 1;
  return std::min(g, cap);
}

// Launches over at least kWideMin list positions of narrow tiles run the
// first three stages of the scaled-fp16 even/odd path on wide tiles (on
// fewer tiles, half as many wide ones leave CUs idle).  The choice changes no
// output: the last stage, whose per-tile partial sums fix the association of
// r^T s, always runs on narrow tiles.  It is part of the captured graphs' key.
constexpr int kWideMin = 1024;

bool dct_wide_for(const Engine& e, int ndtiles, int kind) {
  return kind == 5 && e.dct_trows == 128 && ndtiles >= kWideMin;
}

void e_dct_stage(hipStream_t st, const Engine& e, int ndtiles, int stage, int expect, int kind,
                 const void* X, void* Out, const void* rvec, int fin_mode) {
  const int grid = dct_grid_for(e, ndtiles);
  const bool wide = stage < 3 && dct_wide_for(e, ndtiles, kind);
  DArgs a;
  a.fcnt = e.fcnt;
  a.gcnt = e.gcnt;
  a.gsum = e.gsum;
  a.gstride = e.gstride;
  a.eot = e.eot;
  a.eot_cap = e.cap_dtiles;
  // the finisher rides on the last stage of the even/odd kernels only
  a.fin_mode = (stage == 3 && kind >= 4) ? fin_mode : 0;
  a.desc = e.desc;
  a.ms = e.ms;
  a.dtile_map = e.dtile_map;
  // lists: narrow tiles of the two stage parities, then wide tiles
  a.dact = e.dact + ((wide ? 2 : 0) + (stage & 1)) * e.dlist_cap;
  a.dact_cap = (int)e.dlist_cap;
  a.cidx = (wide ? 4 : 0) + ((stage & 1) ? 3 : 1);
  a.counts = e.counts;
  a.P = e.P;
  a.pstride = e.pstride;
  a.X = X;
  a.Out = Out;
  a.rvec = rvec;
  a.iso = e.iso;
  a.stage = stage;
  a.expect = expect;
  a.trows = kind >= 4 ? 128 : 64;
  // kind: 0 FP64 FMA, 1 FP32 FMA, 2 split-bf16 MFMA, 3 scaled-fp16 MFMA;
  // +2 (kinds 4, 5): the even/odd MFMA kernels (every side a multiple of 128)
  if (kind == 0) hipLaunchKernelGGL(k_e_dct_fma<double>, dim3(grid), dim3(256), 0, st, a);
  else if (kind == 1) hipLaunchKernelGGL(k_e_dct_fma<float>, dim3(grid), dim3(256), 0, st, a);
  else if (kind == 2) hipLaunchKernelGGL(k_e_dct_mfma<1>, dim3(grid), dim3(256), 0, st, a);
  else if (kind == 3) hipLaunchKernelGGL(k_e_dct_mfma<0>, dim3(grid), dim3(256), 0, st, a);
  // scaled fp16 even/odd: intermediates between the stages are stored as
  // scaled fp16 (first stage reads FP32 r, last stage writes FP32 s)
  else if (kind == 4 && stage < 2) hipLaunchKernelGGL((k_e_dct_eo<1, 0, 0, 0, 4>), dim3(grid), dim3(256), 0, st, a);
  else if (kind == 4) hipLaunchKernelGGL((k_e_dct_eo<1, 1, 0, 0, 4>), dim3(grid), dim3(256), 0, st, a);
  else if (stage == 0 && wide) hipLaunchKernelGGL((k_e_dct_eo<0, 0, 0, 1, 8>), dim3(grid), dim3(256), 0, st, a);
  else if (stage == 0) hipLaunchKernelGGL((k_e_dct_eo<0, 0, 0, 1, 4>), dim3(grid), dim3(256), 0, st, a);
  else if (stage == 1 && wide) hipLaunchKernelGGL((k_e_dct_eo<0, 0, 1, 1, 8>), dim3(grid), dim3(256), 0, st, a);
  else if (stage == 1) hipLaunchKernelGGL((k_e_dct_eo<0, 0, 1, 1, 4>), dim3(grid), dim3(256), 0, st, a);
  else if (stage == 2 && wide) hipLaunchKernelGGL((k_e_dct_eo<0, 1, 1, 1, 8>), dim3(grid), dim3(256), 0, st, a);
  else if (stage == 2) hipLaunchKernelGGL((k_e_dct_eo<0, 1, 1, 1, 4>), dim3(grid), dim3(256), 0, st, a);
  else hipLaunchKernelGGL((k_e_dct_eo<0, 1, 1, 0, 4>), dim3(grid), dim3(256), 0, st, a);
}

}  // namespace lpu
