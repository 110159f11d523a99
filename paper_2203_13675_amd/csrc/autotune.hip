// Launch autotuner: picks the stencil tile height, the grid caps and the
// graph/eager issue mode for a batch by timing short fixed-work probes of the
// real solve, with an optional text cache keyed by device and batch shape.

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lpu_internal.h"

namespace {

std::string tune_key(lp_unwrap_ctx* ctx, int n, const lpu_map* maps, int pc, const lpu_options& o) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ') c = '_';
  std::vector<std::pair<int, int>> shapes(n);
  for (int m = 0; m < n; ++m) shapes[m] = {maps[m].rows, maps[m].cols};
  std::sort(shapes.begin(), shapes.end());
  unsigned long long h = 1469598103934665603ULL;  // FNV-1a, 64 bit
  auto mix = [&](unsigned int v) {
    for (int b = 0; b < 4; ++b) {
      h ^= (v >> (8 * b)) & 0xffu;
      h *= 1099511628211ULL;
    }
  };
  for (auto& s : shapes) mix((unsigned)s.first), mix((unsigned)s.second);
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|pc=%d|prec=%d|dct=%d|n=%d|shapes=%016llx", arch.c_str(), pc,
                o.precision, o.dct_mode, n, h);
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, lpu_tuning* t) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512], k[400];
  bool hit = false;
  lpu_tuning v;
  while (std::fgets(line, sizeof(line), f)) {
    if (std::sscanf(line, "%399s %d %d %d %d %d", k, &v.tile_rows, &v.grid, &v.dct_grid,
                    &v.use_graph, &v.max_batch_iters) == 6 &&
        key == k) {
      *t = v;  // the last entry for a key wins
      hit = true;
    }
  }
  std::fclose(f);
  return hit;
}

void cache_store(const char* path, const std::string& key, const lpu_tuning& t) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), t.tile_rows, t.grid, t.dct_grid, t.use_graph,
               t.max_batch_iters);
  std::fclose(f);
}

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" int lp_unwrap_autotune(lp_unwrap_ctx* ctx, int n_maps, const lpu_map* maps, double p,
                                  double eps, int preconditioner, double tol,
                                  const lpu_options* opts, int probe_iters, const char* cache_path,
                                  lpu_tuning* best, double* tune_ms) {
  if (!ctx) return LPU_ERR_INVALID_ARG;
  if (n_maps < 1 || !maps || probe_iters < 1)
    return lpu::set_error(ctx, LPU_ERR_INVALID_ARG, "autotune needs maps and probe_iters >= 1");
  if (tune_ms) *tune_ms = 0.0;
  lpu_options o;
  if (opts) o = *opts;
  else lpu_default_options(&o);
  const std::string key = tune_key(ctx, n_maps, maps, preconditioner, o);
  const lpu_tuning saved = ctx->tune;
  if (cache_path) {
    lpu_tuning t;
    if (cache_lookup(cache_path, key, &t)) {
      const int rc = lp_unwrap_set_tuning(ctx, &t);
      if (rc) return rc;
      if (best) *best = ctx->tune;
      return LPU_OK;
    }
  }
  // fixed work per candidate: one outer iteration, at most probe_iters PCG
  // iterations per map and one refinement step
  lpu_options po = o;
  po.k_max = 1;
  po.outer_tol = 0.0;
  po.l_max = probe_iters;
  po.max_refine = 1;
  po.use_phi0 = 0;
  const double t0 = wall_ms();
  int err = LPU_OK;
  auto measure = [&](const lpu_tuning& t) -> double {
    if (lp_unwrap_set_tuning(ctx, &t)) return 1e300;
    double bestt = 1e300;
    for (int rep = 0; rep < 3; ++rep) {  // first run also captures graphs / grows buffers
      const double a = wall_ms();
      const int rc = lp_unwrap_batch(ctx, n_maps, maps, p, eps, preconditioner, tol, &po, nullptr);
      const double b = wall_ms();
      if (rc < 0) {
        err = rc;
        return 1e300;
      }
      if (rep > 0) bestt = std::min(bestt, b - a);
    }
    return bestt;
  };
  lpu_tuning cur = saved;
  double cur_t = measure(cur);
  if (err) {
    ctx->tune = saved;
    return err;
  }
  auto sweep = [&](int lpu_tuning::*field, std::initializer_list<int> vals) {
    for (int v : vals) {
      if (cur.*field == v) continue;
      lpu_tuning t = cur;
      t.*field = v;
      const double tt = measure(t);
      if (err) return;
      // a candidate must be 1 % faster to replace the current choice: the
      // probe's run-to-run spread is about that, and the current tuning is
      // the default or an earlier winner
      if (tt < 0.99 * cur_t) cur = t, cur_t = tt;
    }
  };
  sweep(&lpu_tuning::tile_rows, {4, 8, 16, 32});
  if (!err) sweep(&lpu_tuning::grid, {1024, 2048, 4096, 8192, 16384});
  if (!err && preconditioner == LPU_PC_DCT) sweep(&lpu_tuning::dct_grid, {512, 1024, 2048, 4096});
  if (!err) sweep(&lpu_tuning::use_graph, {0, 1});
  if (err) {
    ctx->tune = saved;
    return err;
  }
  ctx->tune = cur;
  if (tune_ms) *tune_ms = wall_ms() - t0;
  if (best) *best = cur;
  if (cache_path) cache_store(cache_path, key, cur);
  return LPU_OK;
}
