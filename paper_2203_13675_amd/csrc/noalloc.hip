// lpu_precond_apply_noalloc: the preconditioner apply of lpu_precond_apply
// for callers that cannot allocate device memory (graph capture, serving
// loops).  It launches the same kernels on the caller's U, V, r and s; every
// buffer beyond those (map descriptor and state, tile lists, arrival
// counters, partial sums, pivots or inverse diagonal, the sweep's
// intermediate, isolation flags) is carved out of one file-scope device
// array, `scratch`, whose address is looked up once per device when a
// context is created there.
//
// Sizes: at most kNoAllocMaxPixels pixels and kNoAllocMaxTiles stencil tiles
// per call.  Every call on a device shares that device's array: calls that
// overlap on one device (two streams, two contexts) race.  Each call
// rewrites what it reads before reading it (the layout kernel zeroes the
// arrival counters and writes the lists; the set-up kernels write flags,
// pivots and diagonals for every pixel).

#include <mutex>

#include "lpu_internal.h"

namespace lpu {

// kernels shared with the rest of the library
template <typename T> void e_diag(hipStream_t, const Engine&, int, bool);
template <typename T> void e_pivots(hipStream_t, const Engine&, int, bool, double);
template <typename T>
void e_sweep(hipStream_t, const Engine&, int, int, bool, double, const void*, void*, void*);
void wf_shape(int M, int N, int* diags, int* len);
template <typename T> void e_tc_pivots(hipStream_t, const Engine&, int, bool, double);
template <typename T> void e_twocolor(hipStream_t, const Engine&, int, int, bool, double, int);

constexpr long long kNoAllocMaxPixels = 1LL << 20;  // one 1024 x 1024 map
constexpr int kNoAllocMaxTiles = 1 << 16;

// byte offsets of the regions (each 256-byte aligned)
constexpr size_t al256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kOffDesc = 0;
constexpr size_t kOffState = kOffDesc + al256(sizeof(MapDesc));
constexpr size_t kListInts = kListHead + 1 + kNoAllocMaxTiles;  // counts, one active map, tiles
constexpr size_t kOffCounts = kOffState + al256(sizeof(MapState));
constexpr size_t kOffTileMap = kOffCounts + al256(4 * kListInts);
constexpr size_t kGroups = kNoAllocMaxTiles / kArriveGroup + 8;
constexpr size_t kOffFcnt = kOffTileMap + al256(4 * (size_t)kNoAllocMaxTiles);
constexpr size_t kOffGcnt = kOffFcnt + 256;
constexpr long long kPstride = kNoAllocMaxTiles + 64;
constexpr size_t kOffP = kOffGcnt + al256(4 * kGroups);
constexpr size_t kOffAux = kOffP + al256(8 * (size_t)kNumSlots * kPstride);
constexpr size_t kOffT1 = kOffAux + al256(8 * (size_t)kNoAllocMaxPixels);
constexpr size_t kOffIso = kOffT1 + al256(8 * (size_t)kNoAllocMaxPixels);
constexpr size_t kScratchBytes = kOffIso + al256((size_t)kNoAllocMaxPixels);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// device address of `scratch` per device (the host-side name is not one)
constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// Looks up the scratch array's address on the current device `device`; called
// by lp_unwrap_create with that device current.  Returns LPU_OK or LPU_ERR_HIP.
int noalloc_bind(int device) {
  if (device < 0 || device >= kMaxDevices) return LPU_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return LPU_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LPU_ERR_HIP;
  g_scratch[device] = p;
  return LPU_OK;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

// Descriptor, state and tile lists of one M x N map at element offset 0 with
// `th`-row stencil tiles; clears the arrival counters.
__global__ void k_na_layout(MapDesc* desc, MapState* ms, int* counts, int* tile_map, int* fcnt,
                            int* gcnt, int M, int N, int th, int ntiles, int ngroups) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  int* mact = counts + kListHead;
  int* act = mact + 1;
  for (int t = tid; t < ntiles; t += nth) {
    tile_map[t] = 0;
    act[t] = t;
  }
  for (int g = tid; g < ngroups; g += nth) gcnt[g] = 0;
  if (tid == 0) {
    MapDesc d;
    d.M = M;
    d.N = N;
    d.th = th;
    d.tiles_x = (N + kTW - 1) / kTW;
    d.ntiles = ntiles;
    d.tile0 = 0;
    d.ndt = ((M + 63) / 64) * ((N + 63) / 64);  // 64 x 64 sweep tiles, one partial each
    d.dtile0 = 0;
    d.gb = 0;
    d.gbd = ngroups;
    d.use_iso = 1;
    d.off = 0;
    d.psi = nullptr;
    d.mask = nullptr;
    d.phi = nullptr;
    d.tabM = nullptr;
    d.tabN = nullptr;
    *desc = d;
    MapState s;
    unsigned char* b = reinterpret_cast<unsigned char*>(&s);
    for (size_t k = 0; k < sizeof(MapState); ++k) b[k] = 0;
    s.state = kRun;
    *ms = s;
    for (int k = 0; k < kListHead; ++k) counts[k] = 0;
    counts[0] = ntiles;
    counts[2] = 1;
    mact[0] = 0;
    fcnt[0] = 0;
  }
}

template <typename T>
static int apply(lp_unwrap_ctx* ctx, int M, int N, int pc, double omega, const T* U, const T* V,
                 const T* r, T* s) {
  unsigned char* base = static_cast<unsigned char*>(scratch_of(ctx->device));
  if (!base)
    return set_error(ctx, LPU_ERR_HIP, "scratch array of the no-allocation entry point not bound "
                                       "on this device");
  hipStream_t st = ctx->stream;
  const int th = ctx->tune.tile_rows;
  const long long ntl = (long long)((N + kTW - 1) / kTW) * ((M + th - 1) / th);
  if (ntl > kNoAllocMaxTiles)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "map needs more than 65536 stencil tiles "
                                               "(no-allocation entry point)");
  const int ntiles = (int)ntl;
  const int ngroups = (ntiles + kArriveGroup - 1) / kArriveGroup + 1;
  Engine e;
  e.elem = sizeof(T);
  e.n_maps = e.cap_maps = 1;
  e.total_px = e.cap_px = (long long)M * N;
  e.total_tiles = e.cap_tiles = ntiles;
  e.max_n = N;
  wf_shape(M, N, &e.wf_diags, &e.wf_len);
  e.th = th;
  e.grid = ctx->tune.grid;
  e.dct_grid = ctx->tune.dct_grid;
  e.desc = reinterpret_cast<MapDesc*>(base + kOffDesc);
  e.ms = reinterpret_cast<MapState*>(base + kOffState);
  e.counts = reinterpret_cast<int*>(base + kOffCounts);
  e.mact = e.counts + kListHead;
  e.act = e.mact + 1;
  e.tile_map = reinterpret_cast<int*>(base + kOffTileMap);
  e.fcnt = reinterpret_cast<int*>(base + kOffFcnt);
  e.gcnt = reinterpret_cast<int*>(base + kOffGcnt);
  e.P = reinterpret_cast<double*>(base + kOffP);
  e.pstride = kPstride;
  e.aux = base + kOffAux;
  e.t1 = base + kOffT1;
  e.iso = base + kOffIso;
  e.U = const_cast<T*>(U);
  e.V = const_cast<T*>(V);
  e.r = const_cast<T*>(r);
  e.s = s;
  const int lg = std::max(1, std::min(1024, (ntiles + 255) / 256));
  hipLaunchKernelGGL(k_na_layout, dim3(lg), dim3(256), 0, st, e.desc, e.ms, e.counts, e.tile_map,
                     e.fcnt, e.gcnt, M, N, th, ntiles, ngroups);
  // as lpu_precond_apply: isolation flags (and the inverse diagonal for Jacobi)
  e_diag<T>(st, e, ntiles, pc == kPcJacobi);
  const size_t n = (size_t)M * N;
  if (pc == kPcNone) {
    LPU_HIP_CHECK(ctx, hipMemcpyAsync(s, r, n * sizeof(T), hipMemcpyDeviceToDevice, st));
  } else if (pc == kPcJacobi) {
    launch_scale_by<T>(st, n, r, (const T*)e.aux, s);
  } else if (two_colour(pc)) {
    e_tc_pivots<T>(st, e, ntiles, pc == kPcSsorRb, omega);
    e_twocolor<T>(st, e, ntiles, kRun, pc == kPcSsorRb, omega, 0);
  } else {
    e_pivots<T>(st, e, 1, pc == kPcSsor, omega);
    e_sweep<T>(st, e, 1, kRun, pc == kPcSsor, omega, e.r, e.s, e.t1);
  }
  const hipError_t le = hipGetLastError();
  if (le != hipSuccess)
    return set_error(ctx, LPU_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(le));
  return LPU_OK;
}

}  // namespace lpu

using namespace lpu;

extern "C" int lpu_precond_apply_noalloc(lp_unwrap_ctx* ctx, int M, int N, int precision,
                                         int preconditioner, double omega, const void* U,
                                         const void* V, const void* r, void* s) {
  if (!ctx) return LPU_ERR_INVALID_ARG;
  ctx->last_error.clear();
  if (M < 1 || N < 1) return set_error(ctx, LPU_ERR_INVALID_ARG, "empty map");
  if ((long long)M * N > kNoAllocMaxPixels)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "map above 1048576 pixels (no-allocation entry point)");
  if (!U || !V || !r || !s) return set_error(ctx, LPU_ERR_INVALID_ARG, "null pointer");
  if (preconditioner < LPU_PC_NONE || preconditioner > LPU_PC_SSOR_RB)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown preconditioner");
  if (preconditioner == LPU_PC_DCT)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "the DCT preconditioner needs its tables allocated "
                                               "(use lpu_precond_apply)");
  if ((preconditioner == LPU_PC_ILU0 || preconditioner == LPU_PC_IC0 ||
       preconditioner == LPU_PC_SSOR) && N > 4096)
    return set_error(ctx, LPU_ERR_INVALID_ARG, "sweep preconditioners support N <= 4096");
  if (!(omega > 0.0 && omega < 2.0))
    return set_error(ctx, LPU_ERR_INVALID_ARG, "omega outside (0, 2)");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_error(ctx, LPU_ERR_HIP, "hipSetDevice");
  if (precision == LPU_FP64)
    return apply<double>(ctx, M, N, preconditioner, omega, (const double*)U, (const double*)V,
                         (const double*)r, (double*)s);
  if (precision == LPU_MIXED)
    return apply<float>(ctx, M, N, preconditioner, omega, (const float*)U, (const float*)V,
                        (const float*)r, (float*)s);
  return set_error(ctx, LPU_ERR_INVALID_ARG, "unknown precision");
}
