// The C ABI of liblp_unwrap (include/lp_unwrap.h): contexts, argument checks,
// dispatch to the batched engine, single-step entry points, instrumentation.

#include <cmath>
#include <cstring>

#include "lpu_internal.h"

namespace lpu {

int set_error(lp_unwrap_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

// ----------------------------------------------------------------------------
// Instrumentation
// ----------------------------------------------------------------------------
constexpr int kTimerPairs = 4096;

int KTimer::begin(int cls, hipStream_t st) {
  if (!on(cls)) return -1;
  if (events.empty()) {
    events.resize(2 * kTimerPairs);
    for (auto& e : events)
      if (hipEventCreate(&e) != hipSuccess) e = nullptr;
  }
  if (next_event + 2 > (int)events.size()) flush();
  const int a = next_event;
  next_event += 2;
  if (events[a]) (void)hipEventRecord(events[a], st);
  return a;
}

void KTimer::end(int idx, int cls, hipStream_t st) {
  if (idx < 0) return;
  if (events[idx + 1]) (void)hipEventRecord(events[idx + 1], st);
  pending.push_back({idx, idx + 1, cls});
  n[cls] += 1;
}

void KTimer::flush() {
  if (!pending.empty() && events[pending.back().b]) (void)hipEventSynchronize(events[pending.back().b]);
  for (const Rec& r : pending) {
    float t = 0.0f;
    if (events[r.a] && events[r.b] && hipEventElapsedTime(&t, events[r.a], events[r.b]) == hipSuccess)
      ms[r.cls] += t;
  }
  pending.clear();
  next_event = 0;
}

void KTimer::reset() {
  flush();
  for (int c = 0; c < LPU_KC_COUNT; ++c) ms[c] = 0.0, n[c] = 0, bytes[c] = 0.0, flops[c] = 0.0;
}

void KTimer::destroy() {
  for (auto& e : events)
    if (e) (void)hipEventDestroy(e);
  events.clear();
  pending.clear();
}

}  // namespace lpu

using namespace lpu;

namespace {

int check_common(lp_unwrap_ctx* ctx, int M, int N) {
  if (!ctx) return LPU_ERR_INVALID_ARG;
  ctx->last_error.clear();
  if (M < 1 || N < 1) return set_error(ctx, LPU_ERR_INVALID_ARG, "empty map");
  if ((long long)M * N > (1LL << 31)) return set_error(ctx, LPU_ERR_INVALID_ARG, "map too large");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, LPU_ERR_HIP, "hipSetDevice");
  return LPU_OK;
}

int check_options(lp_unwrap_ctx* ctx, int M, int N, int pc, const lpu_options& o) {
  if (o.k_max < 0) return set_error(ctx, LPU_ERR_INVALID_ARG, "k_max < 0");
  if (o.stop_rule != LPU_STOP_RELRES && o.stop_rule != LPU_STOP_PAPER)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown stop rule");
  if (!(o.eps_cg > 0.0)) return set_error(ctx, LPU_ERR_INVALID_ARG, "eps_cg <= 0");
  if (!(o.ssor_omega > 0.0 && o.ssor_omega < 2.0))
    return set_error(ctx, LPU_ERR_INVALID_ARG, "ssor_omega outside (0, 2)");
  if (o.precision != LPU_FP64 && o.precision != LPU_MIXED)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown precision");
  if (o.dct_mode < LPU_DCT_FP32 || o.dct_mode > LPU_DCT_FP16_SCALED)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown dct_mode");
  if (!(o.refine_eta > 0.0 && o.refine_eta < 1.0))
    return set_error(ctx, LPU_ERR_INVALID_ARG, "refine_eta outside (0, 1)");
  if (o.max_refine < 1) return set_error(ctx, LPU_ERR_INVALID_ARG, "max_refine < 1");
  if (pc < LPU_PC_NONE || pc > LPU_PC_SSOR_RB)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown preconditioner");
  if ((pc == LPU_PC_ILU0 || pc == LPU_PC_IC0 || pc == LPU_PC_SSOR) && N > 4096)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "sweep preconditioners support N <= 4096");
  if (pc == LPU_PC_DCT && (M > 8192 || N > 8192))
    return set_error(ctx, LPU_ERR_INVALID_ARG, "DCT preconditioner supports M, N <= 8192");
  return LPU_OK;
}

int check_scalars(lp_unwrap_ctx* ctx, double p, double eps, double tol) {
  if (!(p >= 0.0 && p <= 2.0)) return set_error(ctx, LPU_ERR_INVALID_ARG, "p outside [0, 2]");
  if (!(eps > 0.0) || !std::isfinite(eps)) return set_error(ctx, LPU_ERR_INVALID_ARG, "eps <= 0");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return set_error(ctx, LPU_ERR_INVALID_ARG, "tol < 0");
  return LPU_OK;
}

int finish_call(lp_unwrap_ctx* ctx, int rc) {
  if (rc < 0 && rc != LPU_ERR_BREAKDOWN && rc != LPU_ERR_NONFINITE && rc != LPU_ERR_INVALID_ARG) {
    // a HIP error may leave the engine's buffers in an unknown state
    (void)hipStreamSynchronize(ctx->stream);
  }
  return rc;
}

}  // namespace

extern "C" {

void lpu_default_options(lpu_options* o) {
  if (!o) return;
  o->k_max = 500;
  o->outer_tol = 1e-6;
  o->l_max = 0;
  o->stop_rule = LPU_STOP_RELRES;
  o->eps_cg = 0.005;
  o->residual_period = 0;
  o->ssor_omega = 1.0;
  o->precision = LPU_MIXED;
  o->dct_mode = LPU_DCT_SPLIT_BF16;
  o->use_phi0 = 0;
  o->refine_eta = 1e-3;
  o->max_refine = 30;
}

void lpu_default_tuning(lpu_tuning* t) {
  if (!t) return;
  t->tile_rows = kTH;
  t->grid = kEngineGrid;
  t->dct_grid = kDctGrid;
  t->use_graph = 1;
  t->max_batch_iters = 64;
}

int lp_unwrap_create(lp_unwrap_ctx** out, int device, void* stream, int max_rows, int max_cols) {
  if (!out || max_rows < 0 || max_cols < 0) return LPU_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return LPU_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return LPU_ERR_HIP;
  lp_unwrap_ctx* ctx = new lp_unwrap_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  lpu_default_tuning(&ctx->tune);
  if (hipEventCreateWithFlags(&ctx->list_event, hipEventDisableTiming) != hipSuccess) {
    delete ctx;
    return LPU_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipEventDestroy(ctx->list_event);
    delete ctx;
    return LPU_ERR_HIP;
  }
  // the no-allocation entry point's scratch array, once per device
  if (noalloc_bind(device) != LPU_OK) {
    lp_unwrap_destroy(ctx);
    return LPU_ERR_HIP;
  }
  if (max_rows > 0 && max_cols > 0) {
    if ((long long)max_rows * max_cols > (1LL << 31)) {
      lp_unwrap_destroy(ctx);
      return LPU_ERR_INVALID_ARG;
    }
    const int rc = engine_reserve(ctx, max_rows, max_cols);
    if (rc != LPU_OK) {
      lp_unwrap_destroy(ctx);
      return rc;
    }
  }
  *out = ctx;
  return LPU_OK;
}

int lpu_debug_force_breakdown(lp_unwrap_ctx* ctx, long long iteration) {
  if (!ctx) return LPU_ERR_INVALID_ARG;
  ctx->debug_breakdown_at = iteration > 0 ? iteration : 0;
  return LPU_OK;
}

void lp_unwrap_destroy(lp_unwrap_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  engine_release(ctx);
  free_dct_tables(ctx);
  ctx->kt.destroy();
  if (ctx->list_event) (void)hipEventDestroy(ctx->list_event);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

int lp_unwrap_set_tuning(lp_unwrap_ctx* ctx, const lpu_tuning* t) {
  if (!ctx || !t) return LPU_ERR_INVALID_ARG;
  ctx->last_error.clear();
  const int tr = t->tile_rows;
  if (tr != 4 && tr != 8 && tr != 16 && tr != 32 && tr != 64)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "tile_rows must be 4, 8, 16, 32 or 64");
  if (t->grid < 64 || t->grid > 65536) return set_error(ctx, LPU_ERR_INVALID_ARG, "grid outside [64, 65536]");
  if (t->dct_grid < 64 || t->dct_grid > 65536)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "dct_grid outside [64, 65536]");
  if (t->use_graph != 0 && t->use_graph != 1) return set_error(ctx, LPU_ERR_INVALID_ARG, "use_graph not 0/1");
  if (t->max_batch_iters < 2 || t->max_batch_iters > 1024)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "max_batch_iters outside [2, 1024]");
  ctx->tune = *t;
  return LPU_OK;
}

int lp_unwrap_get_tuning(lp_unwrap_ctx* ctx, lpu_tuning* t) {
  if (!ctx || !t) return LPU_ERR_INVALID_ARG;
  *t = ctx->tune;
  return LPU_OK;
}

const char* lp_unwrap_status_string(int s) {
  switch (s) {
    case LPU_OK: return "ok";
    case LPU_NOT_CONVERGED: return "not converged (an iteration cap was hit)";
    case LPU_ERR_INVALID_ARG: return "invalid argument";
    case LPU_ERR_OOM: return "out of device memory";
    case LPU_ERR_HIP: return "HIP runtime error";
    case LPU_ERR_NONFINITE: return "non-finite input";
    case LPU_ERR_BREAKDOWN: return "PCG breakdown";
    default: return "unknown status";
  }
}

const char* lp_unwrap_last_error(const lp_unwrap_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : "";
}

int lp_unwrap_solve(lp_unwrap_ctx* ctx, int M, int N, const double* psi, const float* mask,
                    double p, double eps, int preconditioner, double tol, const lpu_options* opts,
                    double* phi, lpu_stats* stats) {
  int rc = check_common(ctx, M, N);
  if (rc) return rc;
  if (!psi || !phi) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  if ((rc = check_scalars(ctx, p, eps, tol))) return rc;
  lpu_options o;
  if (opts) o = *opts;
  else lpu_default_options(&o);
  if ((rc = check_options(ctx, M, N, preconditioner, o))) return rc;
  lpu_stats st;
  std::memset(&st, 0, sizeof(st));
  lpu_map mp;
  mp.rows = M;
  mp.cols = N;
  mp.psi = psi;
  mp.mask = mask;
  mp.phi = phi;
  rc = finish_call(ctx, engine_solve(ctx, 1, &mp, p, eps, preconditioner, tol, o, &st));
  st.status = rc;
  if (stats) *stats = st;
  return rc;
}

int lp_unwrap_batch(lp_unwrap_ctx* ctx, int n_maps, const lpu_map* maps, double p, double eps,
                    int preconditioner, double tol, const lpu_options* opts, lpu_stats* per_map) {
  if (!ctx || n_maps < 0 || (n_maps > 0 && !maps)) return LPU_ERR_INVALID_ARG;
  ctx->last_error.clear();
  if (n_maps == 0) return LPU_OK;
  int rc = check_scalars(ctx, p, eps, tol);
  if (rc) return rc;
  lpu_options o;
  if (opts) o = *opts;
  else lpu_default_options(&o);
  for (int m = 0; m < n_maps; ++m) {
    const lpu_map& mp = maps[m];
    if ((rc = check_common(ctx, mp.rows, mp.cols))) return rc;
    if (!mp.psi || !mp.phi) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer in map");
    if ((rc = check_options(ctx, mp.rows, mp.cols, preconditioner, o))) return rc;
  }
  std::vector<lpu_stats> st(n_maps);
  std::memset(st.data(), 0, sizeof(lpu_stats) * n_maps);
  rc = finish_call(ctx, engine_solve(ctx, n_maps, maps, p, eps, preconditioner, tol, o, st.data()));
  if (per_map)
    for (int m = 0; m < n_maps; ++m) per_map[m] = st[m];
  return rc;
}

// ----------------------------------------------------------------------------
// Single steps
// ----------------------------------------------------------------------------
int lpu_wrapped_differences(lp_unwrap_ctx* ctx, int M, int N, const double* psi, double* dx,
                            double* dy) {
  int rc = check_common(ctx, M, N);
  if (rc) return rc;
  if (!psi || !dx || !dy) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  return step_wrapdiff(ctx, M, N, psi, dx, dy);
}

int lpu_weights(lp_unwrap_ctx* ctx, int M, int N, int precision, const double* phi,
                const double* dx, const double* dy, const float* mask, double p, double tau,
                void* U, void* V) {
  int rc = check_common(ctx, M, N);
  if (rc) return rc;
  if (!phi || !dx || !dy || !U || !V) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  if (!(p >= 0.0 && p <= 2.0) || !(tau > 0.0)) return set_error(ctx, LPU_ERR_INVALID_ARG, "p/tau");
  if (precision == LPU_FP64)
    return step_weights<double>(ctx, M, N, phi, dx, dy, mask, p, tau, (double*)U, (double*)V);
  if (precision == LPU_MIXED)
    return step_weights<float>(ctx, M, N, phi, dx, dy, mask, p, tau, (float*)U, (float*)V);
  return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown precision");
}

int lpu_apply_A(lp_unwrap_ctx* ctx, int M, int N, int precision, const void* U, const void* V,
                const void* x, void* y) {
  int rc = check_common(ctx, M, N);
  if (rc) return rc;
  if (!U || !V || !x || !y) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  if (precision == LPU_FP64)
    return step_apply<double>(ctx, M, N, (const double*)U, (const double*)V, (const double*)x,
                              (double*)y);
  if (precision == LPU_MIXED)
    return step_apply<float>(ctx, M, N, (const float*)U, (const float*)V, (const float*)x,
                             (float*)y);
  return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown precision");
}

int lpu_rhs(lp_unwrap_ctx* ctx, int M, int N, int precision, const void* U, const void* V,
            const double* dx, const double* dy, double* b) {
  int rc = check_common(ctx, M, N);
  if (rc) return rc;
  if (!U || !V || !dx || !dy || !b) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  if (precision == LPU_FP64)
    return step_rhs<double>(ctx, M, N, (const double*)U, (const double*)V, dx, dy, b);
  if (precision == LPU_MIXED)
    return step_rhs<float>(ctx, M, N, (const float*)U, (const float*)V, dx, dy, b);
  return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown precision");
}

int lpu_precond_apply(lp_unwrap_ctx* ctx, int M, int N, int precision, int preconditioner,
                      int dct_mode, double omega, const void* U, const void* V, const void* r,
                      void* s) {
  int rc = check_common(ctx, M, N);
  if (rc) return rc;
  if (!U || !V || !r || !s) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  lpu_options o;
  lpu_default_options(&o);
  o.dct_mode = dct_mode;
  o.ssor_omega = omega;
  if ((rc = check_options(ctx, M, N, preconditioner, o))) return rc;
  if (precision == LPU_FP64)
    return step_precond<double>(ctx, M, N, preconditioner, dct_mode, omega, (const double*)U,
                                (const double*)V, (const double*)r, (double*)s);
  if (precision == LPU_MIXED)
    return step_precond<float>(ctx, M, N, preconditioner, dct_mode, omega, (const float*)U,
                               (const float*)V, (const float*)r, (float*)s);
  return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown precision");
}

int lpu_ilu_pivots(lp_unwrap_ctx* ctx, int M, int N, int precision, const void* U, const void* V,
                   void* piv) {
  int rc = check_common(ctx, M, N);
  if (rc) return rc;
  if (!U || !V || !piv) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  if (N > 4096) return set_error(ctx, LPU_ERR_INVALID_ARG, "N > 4096");
  if (precision == LPU_FP64)
    return step_pivots<double>(ctx, M, N, (const double*)U, (const double*)V, (double*)piv, false, 1.0);
  if (precision == LPU_MIXED)
    return step_pivots<float>(ctx, M, N, (const float*)U, (const float*)V, (float*)piv, false, 1.0);
  return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown precision");
}

int lpu_kernel_timing(lp_unwrap_ctx* ctx, unsigned int class_mask) {
  if (!ctx) return LPU_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  ctx->kt.reset();
  ctx->kt.mask = class_mask;
  return LPU_OK;
}

int lpu_kernel_timing_get(lp_unwrap_ctx* ctx, int kernel_class, double* total_ms,
                          long long* launches, double* alg_bytes, double* alg_flops) {
  if (!ctx || kernel_class < 0 || kernel_class >= LPU_KC_COUNT) return LPU_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  ctx->kt.flush();
  if (total_ms) *total_ms = ctx->kt.ms[kernel_class];
  if (launches) *launches = ctx->kt.n[kernel_class];
  if (alg_bytes) *alg_bytes = ctx->kt.bytes[kernel_class];
  if (alg_flops) *alg_flops = ctx->kt.flops[kernel_class];
  return LPU_OK;
}

}  // extern "C"
