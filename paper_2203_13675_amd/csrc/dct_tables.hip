// DCT tables for the fast-Poisson preconditioner (host side).
//
// C_n[k][j] = s_k cos(pi k (2j + 1) / (2n)), s_0 = sqrt(1/n), s_k = sqrt(2/n)
// (orthonormal DCT-II), its transpose, and the eigenvalues 2 - 2 cos(pi k / n)
// of the unit-weight 1-D Neumann Laplacian, evaluated in long double and
// stored in every arithmetic the contraction kernels use: FP64, FP32, a bf16
// hi/lo split (hi = bf16(c), lo = bf16(c - hi)) and fp16.

#include <cmath>
#include <cstring>
#include <vector>

#include "lpu_internal.h"

namespace lpu {

static uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

static float bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

static void free_tables(DctTables& t) {
  void* tp[] = {t.c64,   t.ct64,   t.c32,  t.ct32,   t.c_hi,   t.c_lo, t.ct_hi,    t.ct_lo, t.c_h,
                t.ct_h,  t.lam,    t.eo_hi, t.eo_lo, t.eo_h, t.eot_hi, t.eot_lo, t.eot_h, t.lam_split};
  for (void* p : tp)
    if (p) (void)hipFree(p);
}

const DctTables* get_dct_tables(lp_unwrap_ctx* ctx, int n, int* status) {
  for (auto& t : ctx->dct)
    if (t.n == n) {
      *status = LPU_OK;
      return &t;
    }
  const long double pi = 3.141592653589793238462643383279502884L;
  DctTables t;
  t.n = n;
  const size_t nn = (size_t)n * n;
  std::vector<double> c(nn), ct(nn), lam(n);
  for (int k = 0; k < n; ++k) {
    const long double s = (k == 0) ? std::sqrt(1.0L / n) : std::sqrt(2.0L / n);
    for (int j = 0; j < n; ++j) {
      const long double v = s * std::cos(pi * k * (2.0L * j + 1.0L) / (2.0L * n));
      c[(size_t)k * n + j] = (double)v;
      ct[(size_t)j * n + k] = (double)v;
    }
    lam[k] = (double)(2.0L - 2.0L * std::cos(pi * k / n));
  }
  std::vector<float> c32(nn), ct32(nn);
  std::vector<uint16_t> chi(nn), clo(nn), cthi(nn), ctlo(nn), ch(nn), cth(nn);
  for (size_t q = 0; q < nn; ++q) {
    c32[q] = (float)c[q];
    ct32[q] = (float)ct[q];
    chi[q] = f32_to_bf16_rne(c32[q]);
    clo[q] = f32_to_bf16_rne(c32[q] - bf16_to_f32(chi[q]));
    cthi[q] = f32_to_bf16_rne(ct32[q]);
    ctlo[q] = f32_to_bf16_rne(ct32[q] - bf16_to_f32(cthi[q]));
    const _Float16 h = (_Float16)c32[q];
    const _Float16 ht = (_Float16)ct32[q];
    std::memcpy(&ch[q], &h, 2);
    std::memcpy(&cth[q], &ht, 2);
  }
  bool ok = true;
  auto up = [&](void** dst, const void* src, size_t bytes) {
    if (!ok) return;
    ok = hipMalloc(dst, bytes) == hipSuccess &&
         hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  up((void**)&t.c64, c.data(), nn * 8);
  up((void**)&t.ct64, ct.data(), nn * 8);
  up((void**)&t.c32, c32.data(), nn * 4);
  up((void**)&t.ct32, ct32.data(), nn * 4);
  up((void**)&t.c_hi, chi.data(), nn * 2);
  up((void**)&t.c_lo, clo.data(), nn * 2);
  up((void**)&t.ct_hi, cthi.data(), nn * 2);
  up((void**)&t.ct_lo, ctlo.data(), nn * 2);
  up((void**)&t.c_h, ch.data(), nn * 2);
  up((void**)&t.ct_h, cth.data(), nn * 2);
  up((void**)&t.lam, lam.data(), (size_t)n * 8);
  if (n % 128 == 0) {
    // even/odd split: C[k][n-1-j] = (-1)^k C[k][j]
    const int h = n / 2;
    const size_t nh = (size_t)n * h;
    std::vector<uint16_t> eh(nh), el(nh), e16(nh), th(nh), tl(nh), t16(nh);
    std::vector<double> ls(n);
    for (int c = 0; c < n; ++c) {
      const int k = c < h ? 2 * c : 2 * (c - h) + 1;
      ls[c] = lam[k];
      for (int j = 0; j < h; ++j) {
        const float v = c32[(size_t)k * n + j];
        const uint16_t hi = f32_to_bf16_rne(v);
        const uint16_t lo = f32_to_bf16_rne(v - bf16_to_f32(hi));
        const _Float16 hv = (_Float16)v;
        uint16_t hb;
        std::memcpy(&hb, &hv, 2);
        // EO[c][j] and EOt[j][c]
        eh[(size_t)c * h + j] = hi;
        el[(size_t)c * h + j] = lo;
        e16[(size_t)c * h + j] = hb;
        th[(size_t)j * n + c] = hi;
        tl[(size_t)j * n + c] = lo;
        t16[(size_t)j * n + c] = hb;
      }
    }
    up((void**)&t.eo_hi, eh.data(), nh * 2);
    up((void**)&t.eo_lo, el.data(), nh * 2);
    up((void**)&t.eo_h, e16.data(), nh * 2);
    up((void**)&t.eot_hi, th.data(), nh * 2);
    up((void**)&t.eot_lo, tl.data(), nh * 2);
    up((void**)&t.eot_h, t16.data(), nh * 2);
    up((void**)&t.lam_split, ls.data(), (size_t)n * 8);
  }
  if (!ok) {
    free_tables(t);
    *status = set_error(ctx, LPU_ERR_OOM, "DCT table allocation failed");
    return nullptr;
  }
  ctx->dct.push_back(t);
  *status = LPU_OK;
  return &ctx->dct.back();
}

void free_dct_tables(lp_unwrap_ctx* ctx) {
  for (auto& t : ctx->dct) free_tables(t);
  ctx->dct.clear();
  for (auto& p : ctx->dct_dev) (void)hipFree(p.second);
  ctx->dct_dev.clear();
}

}  // namespace lpu
