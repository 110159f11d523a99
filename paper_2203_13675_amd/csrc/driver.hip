// Host driver of the batched engine: Algorithm 1 for a set of maps.
//
// Outer loop (all maps in lock-step, each map stops on its own):
//   phi_prev = phi; U, V from phi (Eq. (6)); preconditioner set-up;
//   FP64 path : b (Eq. (7)); PCG from phi^k; phi = x.
//   mixed path: r64 = b - A phi (FP64, float weights promoted); while
//               ||r64|| > tol ||b||: PCG (FP32, FP64 dots) on A e = r64 to a
//               relative reduction eta; phi += e; recompute r64.
//   outer error ||phi - phi_prev|| / ||phi_prev||.
// The PCG loop enqueues K iterations for every running map, reads the map
// states back once, drops finished maps from the tile lists and adapts K to
// the predicted iterations left.

#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstring>

#include "lpu_internal.h"

namespace lpu {

// engine_kernels.hip / engine_dct.hip
void e_wrapdiff(hipStream_t st, const Engine& e, int ntiles, bool zero_phi);
void e_check(hipStream_t st, const Engine& e, int ntiles, unsigned int* bad);
template <typename T> void e_weights(hipStream_t, const Engine&, int, double, double);
template <typename T> void e_diag(hipStream_t, const Engine&, int, bool);
template <typename T> void e_rhs(hipStream_t, const Engine&, int, int);
template <typename T> void e_pass(hipStream_t, const Engine&, int, int);
template <typename T> void e_resid(hipStream_t, const Engine&, int, int, bool);
template <typename T> void e_spmv(hipStream_t, const Engine&, int, int, bool);
template <typename T> void e_update(hipStream_t, const Engine&, int, int, bool);
template <typename T> void e_apply(hipStream_t, const Engine&, int);
void e_finish(hipStream_t st, const Engine& e, int op, int expect, int mode, bool pointwise);
void e_dct_stage(hipStream_t st, const Engine& e, int ndtiles, int stage, int expect, int kind,
                 const void* X, void* Out, const void* rvec, int fin_mode);
int egrid(const Engine& e, int ntiles);
int dct_grid_for(const Engine& e, int ndtiles);
bool dct_wide_for(const Engine& e, int ndtiles, int kind);
template <typename T> void e_pivots(hipStream_t, const Engine&, int, bool, double);
void wf_shape(int M, int N, int* diags, int* len);
template <typename T> void e_tc_pivots(hipStream_t, const Engine&, int, bool, double);
template <typename T>
void e_twocolor(hipStream_t, const Engine&, int, int, bool, double, int);
template <typename T>
void e_sweep(hipStream_t, const Engine&, int, int, bool, double, const void*, void*, void*);

enum { kIdle = 99 };
enum FinOpH { kFinInitH = 0, kFinAlphaH = 1, kFinUpdateH = 2, kFinConfirmH = 3, kFinTailH = 4,
              kFinSum2H = 5 };
enum PassOp { kPassSavePhi = 0, kPassX0Phi = 1, kPassX0Zero = 2, kPassPhiAdd = 3,
              kPassDiffNorms = 4, kPassPhiSet = 5 };

// Contraction kernel of the DCT stages: 0 FP64 FMA, 1 FP32 FMA, 2 split-bf16
// MFMA, 3 scaled-fp16 MFMA, 4/5 the even/odd MFMA versions of 2/3 (every map
// side a multiple of 128).
static int dct_kind_for(const Engine& e, bool mixed, int dct_mode) {
  if (!mixed) return 0;
  if (dct_mode == LPU_DCT_FP32) return 1;
  bool sym = true;
  for (const MapDesc& d : e.hdesc) sym = sym && (d.M % 128 == 0) && (d.N % 128 == 0);
  const int k = dct_mode == LPU_DCT_SPLIT_BF16 ? 2 : 3;
  return sym ? k + 2 : k;
}

static double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// engine set-up
// ---------------------------------------------------------------------------
static void engine_free(Engine& e) {
  // counts, mact, act and dact live in one allocation that starts at counts
  void* ptrs[] = {e.desc, e.ms, e.tile_map, e.dtile_map, e.fcnt, e.gcnt, e.gsum, e.eot, e.counts,
                  e.dx, e.dy, e.phi_prev, e.r64, e.U, e.V, e.aux, e.x[0], e.x[1], e.d[0],
                  e.d[1], e.r, e.s, e.q, e.b, e.t1, e.t2, e.iso, e.P};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (e.hms) (void)hipHostFree(e.hms);
  if (e.hlist) (void)hipHostFree(e.hlist);
  e = Engine();
}

void release_graphs(lp_unwrap_ctx* ctx) {
  for (GraphEntry& g : ctx->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  ctx->graphs.clear();
}

void engine_release(lp_unwrap_ctx* ctx) {
  release_graphs(ctx);
  engine_free(ctx->eng);
}

static const DctTabDev* dct_dev(lp_unwrap_ctx* ctx, int n, int* status) {
  const DctTables* t = get_dct_tables(ctx, n, status);
  if (!t) return nullptr;
  for (auto& p : ctx->dct_dev)
    if (p.first == n) return p.second;
  DctTabDev h;
  h.n = n;
  h.pad = 0;
  h.c64 = t->c64;
  h.ct64 = t->ct64;
  h.c32 = t->c32;
  h.ct32 = t->ct32;
  h.chi = t->c_hi;
  h.clo = t->c_lo;
  h.cthi = t->ct_hi;
  h.ctlo = t->ct_lo;
  h.ch = t->c_h;
  h.cth = t->ct_h;
  h.lam = t->lam;
  h.eo_hi = t->eo_hi;
  h.eo_lo = t->eo_lo;
  h.eo_h = t->eo_h;
  h.eot_hi = t->eot_hi;
  h.eot_lo = t->eot_lo;
  h.eot_h = t->eot_h;
  h.lam_split = t->lam_split;
  DctTabDev* d = nullptr;
  if (hipMalloc((void**)&d, sizeof(DctTabDev)) != hipSuccess ||
      hipMemcpy(d, &h, sizeof(DctTabDev), hipMemcpyHostToDevice) != hipSuccess) {
    *status = set_error(ctx, LPU_ERR_OOM, "DCT table allocation failed");
    return nullptr;
  }
  ctx->dct_dev.push_back({n, d});
  return d;
}

// Lay out n maps; (re)allocate grow-only; upload descriptors and tile maps.
// DCT output tiles are 64 x 64 for the dense kernels; the even/odd kernels
// (used when every side is a multiple of 128 in the mixed path with MFMA
// transforms) take 128 rows x 64 output pairs.  The count per map is the same
// in all stages.
static bool even_odd_ok(const lpu_map* maps, int n, bool mixed, int dct_mode) {
  if (!mixed || dct_mode == LPU_DCT_FP32) return false;
  for (int m = 0; m < n; ++m)
    if (maps[m].rows % 128 != 0 || maps[m].cols % 128 != 0) return false;
  return true;
}

static int engine_setup(lp_unwrap_ctx* ctx, int n, const lpu_map* maps, int elem, bool need_dct,
                        int dct_trows = kDT) {
  Engine& e = ctx->eng;
  std::vector<MapDesc> hd(n);
  long long px = 0;
  int tiles = 0, dtiles = 0, maxN = 1, groups = 0, wfd = 1, wfl = 1;
  for (int m = 0; m < n; ++m) {
    MapDesc& d = hd[m];
    std::memset(&d, 0, sizeof(d));
    d.M = maps[m].rows;
    d.N = maps[m].cols;
    d.th = ctx->tune.tile_rows;
    d.tiles_x = (d.N + kTW - 1) / kTW;
    d.ntiles = d.tiles_x * ((d.M + d.th - 1) / d.th);
    d.tile0 = tiles;
    tiles += d.ntiles;
    // even/odd tiles (128 rows) cover 64 output pairs, i.e. 128 columns of n
    const int ccols = dct_trows == 128 ? 128 : kDT;
    d.ndt = ((d.M + dct_trows - 1) / dct_trows) * ((d.N + ccols - 1) / ccols);
    d.dtile0 = dtiles;
    dtiles += d.ndt;
    d.gb = groups;
    groups += (d.ntiles + kArriveGroup - 1) / kArriveGroup;
    d.gbd = groups;
    groups += (d.ndt + kArriveGroup - 1) / kArriveGroup;
    d.off = px;
    px += ((long long)d.M * d.N + 63) / 64 * 64;
    d.psi = maps[m].psi;
    d.mask = maps[m].mask;
    d.phi = maps[m].phi;
    d.use_iso = maps[m].mask != nullptr ? 1 : 0;
    maxN = std::max(maxN, d.N);
    int dg = 1, ln = 1;
    wf_shape(d.M, d.N, &dg, &ln);
    wfd = std::max(wfd, dg);
    wfl = std::max(wfl, ln);
    if (need_dct) {
      int stt = 0;
      d.tabM = dct_dev(ctx, d.M, &stt);
      d.tabN = dct_dev(ctx, d.N, &stt);
      if (!d.tabM || !d.tabN) return stt ? stt : LPU_ERR_OOM;
    }
  }
  const bool grow = px > e.cap_px || tiles > e.cap_tiles || dtiles > e.cap_dtiles ||
                    n > e.cap_maps || elem > e.elem;
  if (grow) {
    // captured graphs hold the buffers' addresses; every other argument they
    // capture is part of their key, and the layout itself is device data
    release_graphs(ctx);
    engine_free(e);
    const long long cpx = std::max(px, 1LL);
    const size_t eb = (size_t)cpx * elem;
    const long long pst = std::max(tiles, dtiles) + 64;
    bool ok = true;
    auto A = [&](void** p, size_t bytes) {
      if (ok && hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) ok = false;
    };
    A((void**)&e.desc, sizeof(MapDesc) * n);
    A((void**)&e.ms, sizeof(MapState) * n);
    A((void**)&e.tile_map, 4 * (size_t)tiles);
    A((void**)&e.dtile_map, 4 * (size_t)dtiles);
    A((void**)&e.eot, sizeof(EoTile) * 2 * (size_t)std::max(dtiles, 1));
    // the lists of one activation, in one allocation laid out like the
    // pinned staging (counts, active maps, stencil tiles, the two DCT
    // lists), so the first three go up in one copy
    const long long dcap = (long long)dtiles + 8LL * (n + 1) * 256 + 64;
    const size_t list_ints = kListHead + (size_t)n + (size_t)tiles + 4 * (size_t)dcap;
    A((void**)&e.counts, 4 * list_ints);
    if (ok) {
      e.mact = e.counts + kListHead;
      e.act = e.mact + n;
      e.dact = e.act + tiles;
    }
    A((void**)&e.fcnt, 4 * (size_t)n);
    // groups <= tiles / G + dtiles / G + 2 n for any layout within these capacities
    const long long gcap = (long long)(tiles + dtiles) / kArriveGroup + 2LL * n + 8;
    A((void**)&e.gcnt, 4 * (size_t)gcap);
    A((void**)&e.gsum, 8 * 2 * (size_t)gcap);
    A((void**)&e.dx, 8 * (size_t)cpx);
    A((void**)&e.dy, 8 * (size_t)cpx);
    A((void**)&e.phi_prev, 8 * (size_t)cpx);
    A((void**)&e.r64, 8 * (size_t)cpx);
    void** tv[] = {&e.U, &e.V, &e.aux, &e.x[0], &e.x[1], &e.d[0], &e.d[1],
                   &e.r, &e.s, &e.q, &e.b, &e.t1, &e.t2};
    for (void** p : tv) A(p, eb);
    A((void**)&e.iso, (size_t)cpx);
    A((void**)&e.P, 8 * (size_t)kNumSlots * pst);
    if (ok && hipHostMalloc((void**)&e.hms, sizeof(MapState) * n) != hipSuccess) ok = false;
    if (ok && hipHostMalloc((void**)&e.hlist, 4 * list_ints) != hipSuccess) ok = false;
    e.dlist_cap = dcap;
    if (!ok) {
      engine_free(e);
      return set_error(ctx, LPU_ERR_OOM, "engine allocation failed");
    }
    e.cap_px = px;
    e.cap_tiles = tiles;
    e.cap_dtiles = dtiles;
    e.cap_maps = n;
    e.elem = elem;
    e.pstride = pst;
    e.gstride = gcap;
    if (hipMemset(e.iso, 0, (size_t)cpx) != hipSuccess)
      return set_error(ctx, LPU_ERR_HIP, "hipMemset");
  }
  // arrival counters start at zero (every launch leaves them so; cleared
  // here as well, outside any graph capture)
  if (hipMemsetAsync(e.fcnt, 0, 4 * (size_t)n, ctx->stream) != hipSuccess ||
      hipMemsetAsync(e.gcnt, 0, 4 * (size_t)std::max(groups, 1), ctx->stream) != hipSuccess)
    return set_error(ctx, LPU_ERR_HIP, "hipMemsetAsync");
  e.n_maps = n;
  e.total_px = px;
  e.total_tiles = tiles;
  e.total_dtiles = dtiles;
  e.max_n = maxN;
  e.wf_diags = wfd;
  e.wf_len = wfl;
  e.th = ctx->tune.tile_rows;
  e.grid = ctx->tune.grid;
  e.dct_grid = ctx->tune.dct_grid;
  e.dct_trows = dct_trows;
  e.hdesc = hd;
  hipStream_t st = ctx->stream;
  // descriptors and tile -> map tables (staged through the pinned list buffer)
  std::vector<int> tm(tiles), dm(dtiles);
  for (int m = 0; m < n; ++m) {
    for (int t = 0; t < hd[m].ntiles; ++t) tm[hd[m].tile0 + t] = m;
    for (int t = 0; t < hd[m].ndt; ++t) dm[hd[m].dtile0 + t] = m;
  }
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.desc, hd.data(), sizeof(MapDesc) * n, hipMemcpyHostToDevice, st));
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.tile_map, tm.data(), 4 * (size_t)tiles, hipMemcpyHostToDevice, st));
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.dtile_map, dm.data(), 4 * (size_t)dtiles, hipMemcpyHostToDevice, st));
  std::vector<EoTile> eo;
  if (need_dct && dct_trows == 128 && dtiles > 0) {
    // even/odd tile records for both stage parities
    eo.resize(2 * (size_t)dtiles);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int m = 0; m < n; ++m) {
      const MapDesc& d = hd[m];
      int stt = 0;
      const DctTables* tM = get_dct_tables(ctx, d.M, &stt);
      const DctTables* tN = tM ? get_dct_tables(ctx, d.N, &stt) : nullptr;
      if (!tM || !tN) return stt ? stt : LPU_ERR_OOM;
      const double l1M = (double)(2.0L - 2.0L * std::cos(pi / d.M));
      const double l1N = (double)(2.0L - 2.0L * std::cos(pi / d.N));
      for (int par = 0; par < 2; ++par) {
        const DctTables* tk = par ? tM : tN;  // the contracted side's tables
        const int R = par ? d.N : d.M, K = par ? d.M : d.N;
        const int tiles_r = (R + 127) / 128;
        for (int local = 0; local < d.ndt; ++local) {
          EoTile& r = eo[(size_t)par * dtiles + d.dtile0 + local];
          r.off = d.off;
          r.tf[0] = tk->eo_h;
          r.tf[1] = tk->eo_hi;
          r.tf[2] = tk->eo_lo;
          r.ti[0] = tk->eot_h;
          r.ti[1] = tk->eot_hi;
          r.ti[2] = tk->eot_lo;
          r.lam_m = tM->lam_split;
          r.lam_n = tN->lam_split;
          r.m = m;
          r.R = R;
          r.K = K;
          r.r0 = (local % tiles_r) * 128;
          r.c0 = (local / tiles_r) * kDT;
          r.local = local;
          r.ndt = d.ndt;
          r.gbd = d.gbd;
          r.pad = 0;
          r.lmin = (float)std::fmin(l1M, l1N);
        }
      }
    }
    LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.eot, eo.data(), sizeof(EoTile) * dtiles, hipMemcpyHostToDevice, st));
    LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.eot + e.cap_dtiles, eo.data() + dtiles, sizeof(EoTile) * dtiles,
                                      hipMemcpyHostToDevice, st));
  }
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(st));  // pageable sources
  return LPU_OK;
}

// Size the work buffers for one map of M x N in FP64 (enough for any one map
// of at most that size in either precision, under the current tile height);
// called by lp_unwrap_create so a first solve allocates nothing.
int engine_reserve(lp_unwrap_ctx* ctx, int M, int N) {
  lpu_map mp;
  mp.rows = M;
  mp.cols = N;
  mp.psi = nullptr;
  mp.mask = nullptr;
  mp.phi = nullptr;
  return engine_setup(ctx, 1, &mp, 8, false, kDT);
}

// Make the tile lists cover exactly the maps in `set`.
static int engine_activate(lp_unwrap_ctx* ctx, const std::vector<int>& set, int* ntiles,
                           int* ndtiles) {
  Engine& e = ctx->eng;
  hipStream_t st = ctx->stream;
  // the staging buffer may still feed a previous upload
  if (ctx->list_event_live) {
    LPU_HIP_CHECK(ctx, hipEventSynchronize(ctx->list_event));
    ctx->list_event_live = false;
  }
  // staging with the device layout: counts, maps, stencil tiles, DCT lists
  int* hc = e.hlist;
  int* hm = hc + kListHead;
  int* h = hm + e.cap_maps;
  int* hd = h + e.cap_tiles;
  int nt = 0;
  for (int m : set)
    for (int t = 0; t < e.hdesc[m].ntiles; ++t) h[nt++] = e.hdesc[m].tile0 + t;
  // DCT tiles, one list per stage parity (rows of X are the map's rows for
  // stages 0 and 2, its columns for stages 1 and 3).  Blocks are dispatched
  // round-robin over the 8 XCDs, so list position q runs on XCD q mod 8 (the
  // grid is a multiple of 8).  All column tiles of one row block go to one
  // XCD, consecutively, so the block's rows of X are re-read from that XCD's
  // L2; row blocks are balanced over the XCDs largest first.  (Grouping the
  // row blocks of one contraction length on few XCDs, so that each XCD
  // fetches fewer basis tables, cut the counted traffic by 10 % but made the
  // stages 27 % slower: short and long tiles no longer mix on an XCD.)
  // Unused slots hold -1.
  // The even/odd kernels also take wide tiles (two neighbouring column
  // tiles of a row block, named by the left one; the last one of a row
  // block alone when it has no partner): lists 2 and 3, built the same way.
  int ndl[4] = {0, 0, 0, 0};
  const int nlists = e.dct_trows == 128 ? 4 : 2;
  for (int li = 0; li < nlists; ++li) {
    const int par = li & 1, step = li < 2 ? 1 : 2;
    int* out = hd + li * e.dlist_cap;
    struct Unit {
      int tile0, tr, tc;
      long long w;
    };
    std::vector<Unit> units;
    for (int m : set) {
      const MapDesc& d = e.hdesc[m];
      const int R = par ? d.N : d.M, K = par ? d.M : d.N;
      const int ccols = e.dct_trows == 128 ? 128 : kDT;
      const int tr = (R + e.dct_trows - 1) / e.dct_trows, tc = (K + ccols - 1) / ccols;
      for (int rt = 0; rt < tr; ++rt) units.push_back({d.dtile0 + rt, tr, tc, (long long)tc * K});
    }
    std::stable_sort(units.begin(), units.end(),
                     [](const Unit& a, const Unit& b) { return a.w > b.w; });
    std::vector<std::vector<int>> q(8);
    long long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (const Unit& u : units) {
      int x = 0;
      for (int k = 1; k < 8; ++k)
        if (load[k] < load[x]) x = k;
      for (int ct = 0; ct < u.tc; ct += step) q[x].push_back(u.tile0 + ct * u.tr);
      load[x] += u.w;
    }
    size_t L = 0;
    for (int x = 0; x < 8; ++x) L = std::max(L, q[x].size());
    int len = 0;
    if (8 * (long long)L <= e.dlist_cap) {
      for (size_t j = 0; j < L; ++j)
        for (int x = 0; x < 8; ++x) out[len++] = j < q[x].size() ? q[x][j] : -1;
    } else {
      // the padded form would not fit: every tile once, in XCD order
      for (int x = 0; x < 8; ++x)
        for (int t : q[x]) out[len++] = t;
    }
    ndl[li] = len;
  }
  const int nd = std::max(ndl[0], ndl[1]);
  int nm = 0;
  for (int m : set) hm[nm++] = m;
  std::fill(hc, hc + kListHead, 0);
  hc[0] = nt;
  hc[1] = ndl[0];
  hc[2] = nm;
  hc[3] = ndl[1];
  hc[5] = ndl[2];
  hc[7] = ndl[3];
  // counts, maps and stencil tiles in one copy, then each DCT list
  const size_t head = (size_t)kListHead + (size_t)e.cap_maps + (size_t)nt;
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.counts, hc, 4 * head, hipMemcpyHostToDevice, st));
  for (int li = 0; li < nlists; ++li)
    if (ndl[li])
      LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.dact + li * e.dlist_cap, hd + li * e.dlist_cap,
                                        4 * (size_t)ndl[li], hipMemcpyHostToDevice, st));
  LPU_HIP_CHECK(ctx, hipEventRecord(ctx->list_event, st));
  ctx->list_event_live = true;
  *ntiles = nt;
  *ndtiles = nd;
  return LPU_OK;
}

static int read_states(lp_unwrap_ctx* ctx) {
  Engine& e = ctx->eng;
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.hms, e.ms, sizeof(MapState) * e.n_maps,
                                    hipMemcpyDeviceToHost, ctx->stream));
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  return LPU_OK;
}

static int write_states(lp_unwrap_ctx* ctx) {
  Engine& e = ctx->eng;
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.ms, e.hms, sizeof(MapState) * e.n_maps,
                                    hipMemcpyHostToDevice, ctx->stream));
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  return LPU_OK;
}

// ---------------------------------------------------------------------------
// PCG over a set of maps
// ---------------------------------------------------------------------------
template <typename T>
struct Pcg {
  lp_unwrap_ctx* ctx;
  int pc, dct_kind;
  double omega;

  bool pointwise() const { return pc == kPcNone || pc == kPcJacobi; }

  // Preconditioner apply s = M^-1 r for the maps in state `expect`, then the
  // per-map finisher of r^T s with FinishMode `mode` (inside the last DCT
  // stage for the even/odd kernels and the second two-colour pass, as a
  // launch of its own otherwise).
  void tail(hipStream_t st, int nt, int ndt, int nmaps, int expect, int mode) {
    Engine& e = ctx->eng;
    KTimer& kt = ctx->kt;
    bool fused = false;
    if (two_colour(pc)) {
      const int ev = kt.begin(LPU_KC_TWOCOLOR, st);
      e_twocolor<T>(st, e, nt, expect, pc == kPcSsorRb, omega, mode);
      kt.end(ev, LPU_KC_TWOCOLOR, st);
      fused = true;
    } else if (pc == kPcDct) {
      const void* in[4] = {e.r, e.t1, e.t2, e.t1};
      void* out[4] = {e.t1, e.t2, e.t1, e.s};
      fused = dct_kind >= 4;
      for (int s = 0; s < 4; ++s) {
        const int ev = kt.begin(LPU_KC_DCT, st);
        e_dct_stage(st, e, ndt, s, expect, dct_kind, in[s], out[s], e.r, mode);
        kt.end(ev, LPU_KC_DCT, st);
      }
    } else {
      const int ev = kt.begin(LPU_KC_SWEEP, st);
      e_sweep<T>(st, e, nmaps, expect, pc == kPcSsor, omega, e.r, e.s, e.t1);
      kt.end(ev, LPU_KC_SWEEP, st);
    }
    if (!fused) fin(st, kFinTailH, expect, mode);
  }

  void fin(hipStream_t st, int op, int expect, int mode = kFinishNone) {
    // the preconditioner partials of r^T s: one per DCT or sweep tile
    e_finish(st, ctx->eng, op, expect, mode, pointwise());
  }

  // One PCG iteration for every running map of the active set (Algorithm 1's
  // inner loop body): direction update + SpMV, alpha, x/r update, beta or
  // stop test, preconditioner.
  void body(hipStream_t st, int nt, int nd, int nm) {
    Engine& e = ctx->eng;
    KTimer& kt = ctx->kt;
    // the finishers of alpha and of the update run inside the two launches
    int ev = kt.begin(LPU_KC_SPMV, st);
    e_spmv<T>(st, e, nt, pc, true);
    kt.end(ev, LPU_KC_SPMV, st);
    ev = kt.begin(LPU_KC_UPDATE, st);
    e_update<T>(st, e, nt, pc, true);
    kt.end(ev, LPU_KC_UPDATE, st);
    if (!pointwise()) tail(st, nt, nd, nm, kRun, kFinishIter);
  }

  // Issue K iterations: as launches of captured graphs of 8, 4, 2 and 1
  // iterations of the body (one graph per chunk and launch shape, cached for
  // this engine layout; consecutive kernels of one graph start back to back,
  // while each graph launch costs a few microseconds), or launch by launch
  // while kernel timing is on.
  int iterate(int nt, int nd, int nm, long long K) {
    hipStream_t st = ctx->stream;
    if (!ctx->tune.use_graph || ctx->kt.mask != 0) {
      for (long long k = 0; k < K; ++k) body(st, nt, nd, nm);
      return LPU_OK;
    }
    const Engine& e = ctx->eng;
    // the natural-order sweeps launch one grid per tile anti-diagonal over the
    // active maps; every other kernel's shape depends on the tile counts only
    const bool sweep = !pointwise() && !two_colour(pc) && pc != kPcDct;
    // every launch argument that is not a fixed buffer address
    int om[2] = {0, 0};
    if (!pointwise() && pc != kPcDct) std::memcpy(om, &omega, sizeof(om));
    for (int chunk = 8; chunk >= 1; chunk >>= 1) {
      if (K < chunk) continue;
      const int key[kGraphKey] = {egrid(e, nt), pointwise() ? 0 : dct_grid_for(e, nd),
                                  pc == kPcDct && dct_wide_for(e, nd, dct_kind) ? 1 : 0,
                                  sweep ? nm : 0, sweep ? (e.wf_diags << 16) | e.wf_len : 0,
                                  pc, dct_kind,
                                  (int)sizeof(T), e.th, om[0], om[1], chunk};
      hipGraphExec_t ex = nullptr;
      for (const GraphEntry& g : ctx->graphs)
        if (std::equal(key, key + kGraphKey, g.key)) ex = g.exec;
      if (!ex) {
        hipStream_t cs = ctx->cap_stream;
        LPU_HIP_CHECK(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < chunk; ++k) body(cs, nt, nd, nm);
        hipGraph_t g = nullptr;
        LPU_HIP_CHECK(ctx, hipStreamEndCapture(cs, &g));
        const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess)
          return set_error(ctx, LPU_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        if (ctx->graphs.size() >= 64) {
          (void)hipGraphExecDestroy(ctx->graphs.front().exec);
          ctx->graphs.erase(ctx->graphs.begin());
        }
        GraphEntry ge;
        std::copy(key, key + kGraphKey, ge.key);
        ge.exec = ex;
        ctx->graphs.push_back(ge);
      }
      for (; K >= chunk; K -= chunk) LPU_HIP_CHECK(ctx, hipGraphLaunch(ex, st));
    }
    return LPU_OK;
  }

  // Run PCG for the maps in `set` from x0; per-map tol2 already in hms.
  // Returns LPU_OK or an error; per-map final states/iterations are in hms.
  int run(std::vector<int> set, int rule, double eps, const std::vector<double>& tol,
          const std::vector<long long>& lmax, const std::vector<long long>& period) {
    Engine& e = ctx->eng;
    hipStream_t st = ctx->stream;
    KTimer& kt = ctx->kt;
    int rc;
    for (int m = 0; m < e.n_maps; ++m) e.hms[m].state = kIdle;
    for (size_t k = 0; k < set.size(); ++k) {
      MapState& s = e.hms[set[k]];
      std::memset(&s, 0, sizeof(s));
      s.tol2 = tol[k] * tol[k];
      s.eps2 = eps * eps;
      s.l_max = lmax[k];
      s.period = period[k];
      s.rule = rule;
      s.stall = sizeof(T) == 4 ? 1 : 0;  // refinement follows every mixed inner solve
      const long long px = (long long)e.hdesc[set[k]].M * e.hdesc[set[k]].N;
      s.chk_gap = std::min(px, std::max(period[k], 256LL));
      s.brk_at = ctx->debug_breakdown_at;
      s.state = kRun;
    }
    if ((rc = write_states(ctx))) return rc;
    int nt = 0, nd = 0;
    if ((rc = engine_activate(ctx, set, &nt, &nd))) return rc;
    const bool pw = pointwise();
    int ev = kt.begin(LPU_KC_INIT, st);
    e_resid<T>(st, e, nt, pc, false);
    kt.end(ev, LPU_KC_INIT, st);
    fin(st, kFinInitH, kRun);
    if (!pw) {
      tail(st, nt, nd, (int)set.size(), kInitPc, kFinishInit);
    }
    long long K = 4;
    const long long Kcap = std::max(2, ctx->tune.max_batch_iters);
    std::vector<double> prev_metric(e.n_maps, -1.0);
    std::vector<long long> prev_l(e.n_maps, 0);
    for (;;) {
      if ((rc = iterate(nt, nd, (int)set.size(), K))) return rc;
      ev = kt.begin(LPU_KC_CONFIRM, st);
      e_resid<T>(st, e, nt, pc, true);
      kt.end(ev, LPU_KC_CONFIRM, st);
      fin(st, kFinConfirmH, kConfirm);
      if (!pw) {
        tail(st, nt, nd, (int)set.size(), kConfirmPc, kFinishConfirm);
      }
      if ((rc = read_states(ctx))) return rc;
      std::vector<int> still;
      std::vector<long long> guesses;
      for (int m : set) {
        const MapState& s = e.hms[m];
        if (s.state == kDone || s.state == kCap || s.state == kBreakdown || s.state == kStall)
          continue;
        still.push_back(m);
        const double metric = rule == LPU_STOP_PAPER ? s.delta_new : s.rr;
        const double target = rule == LPU_STOP_PAPER ? s.thr_delta : s.thr_rr;
        long long guess = 2 * K;
        if (prev_metric[m] > 0.0 && metric > 0.0 && s.l > prev_l[m] && metric < prev_metric[m]) {
          const double rate = std::log(metric / prev_metric[m]) / (double)(s.l - prev_l[m]);
          const double left = std::log(target / metric) / rate;
          if (std::isfinite(left)) guess = (long long)std::ceil(left * 0.9) + 1;
        }
        prev_metric[m] = metric;
        prev_l[m] = s.l;
        guesses.push_back(guess);
      }
      if (still.empty()) break;
      if (still.size() != set.size()) {
        // Finished maps' tiles skip all work, so the lists are rebuilt (a
        // host round trip of several uploads) only once they hold at least
        // 10 % dead stencil tiles.
        long long live = 0;
        for (int m : still) live += e.hdesc[m].ntiles;
        if (live * 10 <= (long long)nt * 9) {
          set = still;
          if ((rc = engine_activate(ctx, set, &nt, &nd))) return rc;
        }
      }
      // Round length: the median of the maps' predicted remaining iterations.
      // A map that meets its bound inside a round stops iterating and waits
      // for the round's confirmation, so a longer round wastes no work on it,
      // while every round costs a confirmation pass and a host round trip
      // (the earliest map's prediction made rounds 3x more frequent and the
      // batch 3 % slower).
      long long nextK = Kcap;
      if (!guesses.empty()) {
        std::nth_element(guesses.begin(), guesses.begin() + guesses.size() / 2, guesses.end());
        nextK = guesses[guesses.size() / 2];
      }
      K = std::max(2LL, std::min(nextK, Kcap));
    }
    return LPU_OK;
  }
};

// ---------------------------------------------------------------------------
// Algorithm 1 for a set of maps
// ---------------------------------------------------------------------------
template <typename T>
static int run_maps(lp_unwrap_ctx* ctx, int n, const lpu_map* maps, double p, double tau, int pc,
                    double tol, const lpu_options& o, lpu_stats* stats) {
  const double t_start = now_ms();
  hipStream_t st = ctx->stream;
  const bool mixed = sizeof(T) == 4;
  // 64 x 64 DCT tiles double as the sweeps' tiles (one partial of r^T s each)
  int rc = engine_setup(ctx, n, maps, (int)sizeof(T), pc == kPcDct,
                        pc == kPcDct && even_odd_ok(maps, n, mixed, o.dct_mode) ? 128 : kDT);
  if (rc) return rc;
  Engine& e = ctx->eng;
  KTimer& kt = ctx->kt;

  std::vector<int> all(n);
  for (int m = 0; m < n; ++m) all[m] = m;
  int nt = 0, nd = 0;
  if ((rc = engine_activate(ctx, all, &nt, &nd))) return rc;

  // inputs must be finite (mask in [0, 1]); one launch over every map's tiles
  LPU_HIP_CHECK(ctx, hipMemsetAsync(e.counts + 8, 0, 4, st));
  e_check(st, e, nt, (unsigned int*)(e.counts + 8));
  unsigned int bad = 0;
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(&bad, e.counts + 8, 4, hipMemcpyDeviceToHost, st));
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(st));
  if (bad) return set_error(ctx, LPU_ERR_NONFINITE, "psi or mask holds NaN/Inf (or mask outside [0,1])");

  // wrapped differences; phi = 0 unless the caller supplies the start value
  e_wrapdiff(st, e, nt, !o.use_phi0);

  const bool need_diag = pc == kPcJacobi;
  bool any_mask = false;
  for (int m = 0; m < n; ++m) any_mask |= maps[m].mask != nullptr;

  std::vector<long long> lmax(n), period(n);
  for (int m = 0; m < n; ++m) {
    const long long px = (long long)maps[m].rows * maps[m].cols;
    lmax[m] = o.l_max > 0 ? o.l_max : 2 * px;
    period[m] = o.residual_period > 0 ? o.residual_period
                                      : std::max(1LL, (long long)std::floor(std::sqrt((double)px)));
  }
  std::vector<int> outer(n, 0), refinements(n, 0), status(n, LPU_OK);
  std::vector<long long> inner(n, 0);
  std::vector<double> err(n, INFINITY), relres(n, 0.0);
  std::vector<bool> finished(n, false), outer_conv(n, false), inner_ok(n, true);
  double setup_ms = 0.0;
  Pcg<T> pcg{ctx, pc, dct_kind_for(e, mixed, o.dct_mode), o.ssor_omega};

  auto credit = [&](const std::vector<int>& set) {
    // algorithmic figures of the PCG launches that did work
    // the DCT tables of one side length serve every map of that side in a
    // launch, so they count once per launch in which any such map is active:
    // a map is active in a prefix of the run's applications, so that is the
    // largest application count among the maps of that side
    std::map<int, long long> side_apps;
    for (int m : set) {
      const MapState& s = e.hms[m];
      const double px = (double)maps[m].rows * maps[m].cols, el = (double)sizeof(T);
      const double jac = pc == kPcJacobi ? 1.0 : 0.0;
      // SpMV: read s (or r), d_old, U, V (+ inverse diagonal), write d, q,
      // and x += alpha_p d_old (read and write x) after every update that was
      // not a replacement; update: read r, q (+ inverse diagonal), write r,
      // or at a replacement read x, d, U, V, b (+ inverse diagonal) and write
      // x, r
      const double l = (double)s.l;
      const double rep = s.period > 0 ? std::min(l, std::floor((l - 1.0) / s.period) + 1.0) : 0.0;
      kt.credit(LPU_KC_SPMV, s.l, px * el * (l * (6.0 + jac) + 2.0 * std::max(0.0, l - 1.0 - rep)),
                l * px * 13.0 + std::max(0.0, l - 1.0 - rep) * px * 2.0);
      kt.credit(LPU_KC_UPDATE, s.l, px * el * ((l - rep) * (3.0 + jac) + rep * (7.0 + jac)),
                (l - rep) * px * 6.0 + rep * px * 15.0);
      const double Mm = maps[m].rows, Nn = maps[m].cols;
      if (pc == kPcDct) {
        // per application: 4 contractions; MFMA products per multiply-add
        // (3 for the bf16 split); the even/odd kernels do half the work
        const int kd = pcg.dct_kind;
        const double prod = (kd == 2 || kd == 4) ? 3.0 : 1.0;
        const double half = kd >= 4 ? 0.5 : 1.0;
        // X in, Out out per stage (the scaled-fp16 even/odd path keeps the
        // three intermediates in 2 bytes), and r again in the last stage
        const double io = (kd == 5 ? px * (4.0 + 2.0 + 2.0 + 2.0 + 2.0 + 2.0 + 2.0 + 4.0)
                                   : 8.0 * px * el) + px * el;
        kt.credit(LPU_KC_DCT, 4 * s.nfinish, s.nfinish * io,
                  s.nfinish * 4.0 * px * (Mm + Nn) * prod * half);
        for (int side : {maps[m].rows, maps[m].cols}) {
          long long& a = side_apps[side];
          a = std::max(a, s.nfinish);
        }
      } else if (two_colour(pc)) {
        // per application, two passes: read r, pivots, U, V (+ s on half the
        // pixels in the second) and write s on half the pixels each
        kt.credit(LPU_KC_TWOCOLOR, 2 * s.nfinish, s.nfinish * px * el * 10.0, s.nfinish * px * 30.0);
      } else if (!pcg.pointwise()) {
        kt.credit(LPU_KC_SWEEP, s.nfinish, s.nfinish * px * el * 10.0, s.nfinish * px * 14.0);
      }
    }
    if (pc == kPcDct) {
      // per application and side n: a forward and an inverse table of n x n
      // entries (n x n/2 for the even/odd split), 2, 4 (the bf16 hi and lo
      // planes, or FP32) or 8 bytes each
      const int kd = pcg.dct_kind;
      const double half = kd >= 4 ? 0.5 : 1.0;
      const double tab = kd == 0 ? 8.0 : (kd == 1 ? 4.0 : ((kd == 2 || kd == 4) ? 4.0 : 2.0));
      for (const auto& sa : side_apps)
        kt.credit(LPU_KC_DCT, 0, (double)sa.second * 2.0 * half * sa.first * sa.first * tab, 0.0);
    }
  };

  for (int k = 0; k < o.k_max; ++k) {
    std::vector<int> act;
    for (int m = 0; m < n; ++m)
      if (!finished[m]) act.push_back(m);
    if (act.empty()) break;
    const double ts = now_ms();
    if ((rc = engine_activate(ctx, act, &nt, &nd))) return rc;
    const int ev = kt.begin(LPU_KC_SETUP, st);
    e_pass<T>(st, e, nt, kPassSavePhi);
    e_weights<T>(st, e, nt, p, tau);
    if (need_diag || any_mask) e_diag<T>(st, e, nt, need_diag);
    if (pc == kPcIlu || pc == kPcIc || pc == kPcSsor)
      e_pivots<T>(st, e, (int)act.size(), pc == kPcSsor, o.ssor_omega);
    else if (two_colour(pc))
      e_tc_pivots<T>(st, e, nt, pc == kPcSsorRb, o.ssor_omega);
    kt.end(ev, LPU_KC_SETUP, st);
    if (!mixed) {
      e_rhs<T>(st, e, nt, 0);
      e_pass<T>(st, e, nt, kPassX0Phi);
      // the set-up kernels' own time (the PCG below starts with a synchronising
      // state upload anyway)
      LPU_HIP_CHECK(ctx, hipStreamSynchronize(st));
      setup_ms += now_ms() - ts;
      std::vector<double> tl(act.size(), tol);
      std::vector<long long> lm, pr;
      for (int m : act) lm.push_back(lmax[m]), pr.push_back(period[m]);
      if ((rc = pcg.run(act, o.stop_rule, o.eps_cg, tl, lm, pr))) return rc;
      credit(act);
      for (int m : act) {
        const MapState& s = e.hms[m];
        inner[m] += s.l;
        refinements[m] += 1;
        inner_ok[m] = s.state == kDone;
        if (s.state == kBreakdown) status[m] = LPU_ERR_BREAKDOWN, finished[m] = true;
      }
      if ((rc = engine_activate(ctx, act, &nt, &nd))) return rc;
      e_pass<T>(st, e, nt, kPassPhiSet);
    } else {
      e_rhs<T>(st, e, nt, 1);
      e_finish(st, e, kFinSum2H, -1, kFinishNone, true);
      if ((rc = read_states(ctx))) return rc;
      setup_ms += now_ms() - ts;
      std::vector<double> rr(n, 0.0), bb(n, 0.0);
      for (int m : act) rr[m] = e.hms[m].rr, bb[m] = e.hms[m].bb;
      std::vector<int> ref;
      for (int m : act)
        if (bb[m] > 0.0 && rr[m] > tol * tol * bb[m]) ref.push_back(m);
      for (int j = 0; !ref.empty() && j < o.max_refine; ++j) {
        std::vector<double> tl;
        std::vector<long long> lm, pr;
        for (int m : ref) {
          double eta = o.refine_eta;
          if (o.stop_rule == LPU_STOP_RELRES) eta = std::max(eta, 0.5 * tol / std::sqrt(rr[m] / bb[m]));
          tl.push_back(std::min(eta, 0.5));
          lm.push_back(lmax[m]);
          pr.push_back(period[m]);
        }
        if ((rc = engine_activate(ctx, ref, &nt, &nd))) return rc;
        e_pass<T>(st, e, nt, kPassX0Zero);
        if ((rc = pcg.run(ref, o.stop_rule, o.eps_cg, tl, lm, pr))) return rc;
        credit(ref);
        std::vector<int> cont, okm;
        for (int m : ref) {
          const MapState& s = e.hms[m];
          inner[m] += s.l;
          refinements[m] += 1;
          if (s.state == kBreakdown) status[m] = LPU_ERR_BREAKDOWN, finished[m] = true;
          else okm.push_back(m);
        }
        if (okm.empty()) break;
        ref = okm;
        if ((rc = engine_activate(ctx, ref, &nt, &nd))) return rc;
        e_pass<T>(st, e, nt, kPassPhiAdd);
        e_rhs<T>(st, e, nt, 1);
        e_finish(st, e, kFinSum2H, -1, kFinishNone, true);
        if ((rc = read_states(ctx))) return rc;
        for (int m : ref) {
          if (finished[m]) continue;
          rr[m] = e.hms[m].rr;
          if (o.stop_rule != LPU_STOP_PAPER && rr[m] > tol * tol * bb[m]) cont.push_back(m);
        }
        ref = cont;
      }
      for (int m : act)
        inner_ok[m] = o.stop_rule == LPU_STOP_PAPER || bb[m] == 0.0 || rr[m] <= tol * tol * bb[m];
    }
    // outer error
    std::vector<int> act2;
    for (int m : act)
      if (!finished[m]) act2.push_back(m);
    if (act2.empty()) break;
    if ((rc = engine_activate(ctx, act2, &nt, &nd))) return rc;
    e_pass<T>(st, e, nt, kPassDiffNorms);
    e_finish(st, e, kFinSum2H, -1, kFinishNone, true);
    if ((rc = read_states(ctx))) return rc;
    for (int m : act2) {
      outer[m] = k + 1;
      const double dn = e.hms[m].rr, pn = e.hms[m].bb;
      err[m] = pn > 0.0 ? std::sqrt(dn / pn) : INFINITY;
      if (o.outer_tol > 0.0 && err[m] <= o.outer_tol) outer_conv[m] = true, finished[m] = true;
    }
  }
  // FP64 relative residual of each map's last system
  std::vector<int> done_any;
  for (int m = 0; m < n; ++m)
    if (outer[m] > 0 && status[m] >= 0) done_any.push_back(m);
  if (!done_any.empty()) {
    if ((rc = engine_activate(ctx, done_any, &nt, &nd))) return rc;
    e_rhs<T>(st, e, nt, 2);
    e_finish(st, e, kFinSum2H, -1, kFinishNone, true);
    if ((rc = read_states(ctx))) return rc;
    for (int m : done_any)
      relres[m] = e.hms[m].bb > 0 ? std::sqrt(e.hms[m].rr / e.hms[m].bb) : 0.0;
  }
  int worst = LPU_OK;
  const double total_ms = now_ms() - t_start;
  for (int m = 0; m < n; ++m) {
    if (status[m] >= 0) {
      if (o.outer_tol > 0.0) status[m] = outer_conv[m] ? LPU_OK : LPU_NOT_CONVERGED;
      else status[m] = inner_ok[m] ? LPU_OK : LPU_NOT_CONVERGED;
      if (o.k_max == 0) status[m] = LPU_OK;
    }
    if (status[m] < 0 && (worst >= 0 || status[m] < worst)) worst = status[m];
    else if (worst >= 0 && status[m] > worst) worst = status[m];
    if (stats) {
      lpu_stats& s = stats[m];
      s.outer_iters = outer[m];
      s.inner_iters_total = inner[m];
      s.refinements = refinements[m];
      s.final_relres = relres[m];
      s.outer_err = err[m];
      s.setup_ms = setup_ms;
      s.solve_ms = total_ms;
      s.converged = status[m] == LPU_OK;
      s.status = status[m];
    }
  }
  if (worst == LPU_ERR_BREAKDOWN) set_error(ctx, worst, "PCG breakdown");
  return worst;
}

int engine_solve(lp_unwrap_ctx* ctx, int n, const lpu_map* maps, double p, double tau, int pc,
                 double tol, const lpu_options& o, lpu_stats* stats) {
  if (o.precision == LPU_FP64) return run_maps<double>(ctx, n, maps, p, tau, pc, tol, o, stats);
  return run_maps<float>(ctx, n, maps, p, tau, pc, tol, o, stats);
}

// ---------------------------------------------------------------------------
// Step entry points: one map through the engine's kernels
// ---------------------------------------------------------------------------
static int step_setup(lp_unwrap_ctx* ctx, int M, int N, int elem, bool dct, const double* psi,
                      const float* mask, double* phi, int dct_mode = LPU_DCT_FP32) {
  lpu_map mp;
  mp.rows = M;
  mp.cols = N;
  mp.psi = psi;
  mp.mask = mask;
  mp.phi = phi;
  const bool eo = dct && even_odd_ok(&mp, 1, elem == 4, dct_mode);
  int rc = engine_setup(ctx, 1, &mp, elem, dct, eo ? 128 : kDT);
  if (rc) return rc;
  std::vector<int> one(1, 0);
  int nt, nd;
  return engine_activate(ctx, one, &nt, &nd);
}

static int copy_in(lp_unwrap_ctx* ctx, void* dst, const void* src, size_t bytes) {
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  return LPU_OK;
}

int step_wrapdiff(lp_unwrap_ctx* ctx, int M, int N, const double* psi, double* dx, double* dy) {
  int rc = step_setup(ctx, M, N, 8, false, psi, nullptr, nullptr);
  if (rc) return rc;
  Engine& e = ctx->eng;
  e_wrapdiff(ctx->stream, e, e.total_tiles, false);
  const size_t b = (size_t)M * N * 8;
  if ((rc = copy_in(ctx, dx, e.dx, b)) || (rc = copy_in(ctx, dy, e.dy, b))) return rc;
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  return LPU_OK;
}

template <typename T>
int step_weights(lp_unwrap_ctx* ctx, int M, int N, const double* phi, const double* dx,
                 const double* dy, const float* mask, double p, double tau, T* U, T* V) {
  int rc = step_setup(ctx, M, N, sizeof(T), false, nullptr, mask, const_cast<double*>(phi));
  if (rc) return rc;
  Engine& e = ctx->eng;
  const size_t n = (size_t)M * N;
  if ((rc = copy_in(ctx, e.dx, dx, n * 8)) || (rc = copy_in(ctx, e.dy, dy, n * 8))) return rc;
  e_weights<T>(ctx->stream, e, e.total_tiles, p, tau);
  if ((rc = copy_in(ctx, U, e.U, n * sizeof(T))) || (rc = copy_in(ctx, V, e.V, n * sizeof(T))))
    return rc;
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  return LPU_OK;
}

template <typename T>
int step_apply(lp_unwrap_ctx* ctx, int M, int N, const T* U, const T* V, const T* x, T* y) {
  int rc = step_setup(ctx, M, N, sizeof(T), false, nullptr, nullptr, nullptr);
  if (rc) return rc;
  Engine& e = ctx->eng;
  const size_t b = (size_t)M * N * sizeof(T);
  if ((rc = copy_in(ctx, e.U, U, b)) || (rc = copy_in(ctx, e.V, V, b)) || (rc = copy_in(ctx, e.s, x, b)))
    return rc;
  e_apply<T>(ctx->stream, e, e.total_tiles);
  if ((rc = copy_in(ctx, y, e.q, b))) return rc;
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  return LPU_OK;
}

template <typename T>
int step_rhs(lp_unwrap_ctx* ctx, int M, int N, const T* U, const T* V, const double* dx,
             const double* dy, double* b) {
  int rc = step_setup(ctx, M, N, sizeof(T), false, nullptr, nullptr, nullptr);
  if (rc) return rc;
  Engine& e = ctx->eng;
  const size_t n = (size_t)M * N;
  if ((rc = copy_in(ctx, e.U, U, n * sizeof(T))) || (rc = copy_in(ctx, e.V, V, n * sizeof(T))) ||
      (rc = copy_in(ctx, e.dx, dx, n * 8)) || (rc = copy_in(ctx, e.dy, dy, n * 8)))
    return rc;
  e_rhs<T>(ctx->stream, e, e.total_tiles, 0);
  if ((rc = copy_in(ctx, b, e.r64, n * 8))) return rc;
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  return LPU_OK;
}

template <typename T>
int step_pivots(lp_unwrap_ctx* ctx, int M, int N, const T* U, const T* V, T* piv, bool ssor,
                double omega) {
  int rc = step_setup(ctx, M, N, sizeof(T), false, nullptr, nullptr, nullptr);
  if (rc) return rc;
  Engine& e = ctx->eng;
  const size_t b = (size_t)M * N * sizeof(T);
  if ((rc = copy_in(ctx, e.U, U, b)) || (rc = copy_in(ctx, e.V, V, b))) return rc;
  e_pivots<T>(ctx->stream, e, 1, ssor, omega);
  if ((rc = copy_in(ctx, piv, e.aux, b))) return rc;
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
  return LPU_OK;
}

template <typename T>
int step_precond(lp_unwrap_ctx* ctx, int M, int N, int pc, int dct_mode, double omega, const T* U,
                 const T* V, const T* r, T* s) {
  int rc = step_setup(ctx, M, N, sizeof(T), pc == kPcDct, nullptr, nullptr, nullptr, dct_mode);
  if (rc) return rc;
  Engine& e = ctx->eng;
  hipStream_t st = ctx->stream;
  const size_t n = (size_t)M * N, b = n * sizeof(T);
  if ((rc = copy_in(ctx, e.U, U, b)) || (rc = copy_in(ctx, e.V, V, b)) || (rc = copy_in(ctx, e.r, r, b)))
    return rc;
  // preconditioner output is zeroed on isolated pixels
  e.hdesc[0].use_iso = 1;
  LPU_HIP_CHECK(ctx, hipMemcpyAsync(e.desc, e.hdesc.data(), sizeof(MapDesc), hipMemcpyHostToDevice, st));
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(st));
  e_diag<T>(st, e, e.total_tiles, pc == kPcJacobi);
  MapState& h = e.hms[0];
  std::memset(&h, 0, sizeof(h));
  h.state = kRun;
  if (pc == kPcDct && sizeof(T) == 4 && dct_mode == LPU_DCT_FP16_SCALED) {
    // the scaled-fp16 stage 0 needs ||r||^2
    std::vector<T> hr(n);
    LPU_HIP_CHECK(ctx, hipMemcpy(hr.data(), r, b, hipMemcpyDeviceToHost));
    double rr = 0.0;
    for (T v : hr) rr += (double)v * (double)v;
    h.rr = rr;
  }
  if ((rc = write_states(ctx))) return rc;
  if (pc == kPcNone) {
    if ((rc = copy_in(ctx, s, r, b))) return rc;
  } else if (pc == kPcJacobi) {
    launch_scale_by<T>(st, n, r, (const T*)e.aux, s);
  } else if (pc == kPcDct) {
    const int kind = dct_kind_for(e, sizeof(T) == 4, dct_mode);
    const void* in[4] = {e.r, e.t1, e.t2, e.t1};
    void* out[4] = {e.t1, e.t2, e.t1, e.s};
    for (int k = 0; k < 4; ++k) {
      const int ev = ctx->kt.begin(LPU_KC_DCT, st);
      e_dct_stage(st, e, e.total_dtiles, k, kRun, kind, in[k], out[k], e.r, 0);
      ctx->kt.end(ev, LPU_KC_DCT, st);
    }
    if ((rc = copy_in(ctx, s, e.s, b))) return rc;
  } else if (two_colour(pc)) {
    e_tc_pivots<T>(st, e, e.total_tiles, pc == kPcSsorRb, omega);
    const int ev = ctx->kt.begin(LPU_KC_TWOCOLOR, st);
    e_twocolor<T>(st, e, e.total_tiles, kRun, pc == kPcSsorRb, omega, 0);
    ctx->kt.end(ev, LPU_KC_TWOCOLOR, st);
    if ((rc = copy_in(ctx, s, e.s, b))) return rc;
  } else {
    e_pivots<T>(st, e, 1, pc == kPcSsor, omega);
    e_sweep<T>(st, e, 1, kRun, pc == kPcSsor, omega, e.r, e.s, e.t1);
    if ((rc = copy_in(ctx, s, e.s, b))) return rc;
  }
  LPU_HIP_CHECK(ctx, hipStreamSynchronize(st));
  return LPU_OK;
}

#define LPU_INST_STEP(T)                                                                          \
  template int step_weights<T>(lp_unwrap_ctx*, int, int, const double*, const double*,            \
                               const double*, const float*, double, double, T*, T*);               \
  template int step_apply<T>(lp_unwrap_ctx*, int, int, const T*, const T*, const T*, T*);          \
  template int step_rhs<T>(lp_unwrap_ctx*, int, int, const T*, const T*, const double*,            \
                           const double*, double*);                                                \
  template int step_pivots<T>(lp_unwrap_ctx*, int, int, const T*, const T*, T*, bool, double);     \
  template int step_precond<T>(lp_unwrap_ctx*, int, int, int, int, double, const T*, const T*,     \
                               const T*, T*);
LPU_INST_STEP(float)
LPU_INST_STEP(double)

}  // namespace lpu
