// Batched PCG engine: data layout shared by the kernels and the host driver.
//
// Every solve -- one map or many -- runs on an Engine: the maps' work vectors
// are concatenated (each map contiguous, row-major, at a 64-element aligned
// offset), and every kernel walks a device-resident list of active tiles
// (grid-stride, fixed grid), so one launch serves all maps of a phase and maps
// that have stopped cost nothing once the host compacts the list.
//
// Reductions: each tile writes its FP64 partial sums to its own slot; a
// finisher (a kernel of one block per map, or fused into the tile kernel,
// in the block that completes the map) sums the map's slots in a fixed
// order and advances that map's PCG state.  No grid-wide fences, so results
// are deterministic and nothing serialises across the chip's L2s.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace lpu {

constexpr int kTW = 128;  // stencil tile width (columns): two per lane of one wave
constexpr int kTH = 16;   // default stencil tile height (rows), marched by the wave
constexpr int kDT = 64;   // DCT output tile (64 x 64)
constexpr int kEngineGrid = 16384;  // default cap on the blocks of the grid-stride tile kernels
constexpr int kDctGrid = 2048;     // default cap on the blocks of a DCT stage
constexpr int kArriveGroup = 32;   // tiles per first-level arrival counter of the fused finishers
constexpr int kNumSlots = 4;       // partial-sum slots
constexpr int kListHead = 16;      // ints of counts[] ahead of the active-map list

// DCT tables of one size n as seen by the kernels.
struct DctTabDev {
  int n;
  int pad;
  const double* c64;
  const double* ct64;
  const float* c32;
  const float* ct32;
  const uint16_t* chi;
  const uint16_t* clo;
  const uint16_t* cthi;
  const uint16_t* ctlo;
  const uint16_t* ch;
  const uint16_t* cth;
  const double* lam;
  const uint16_t* eo_hi;   // even/odd split tables (null unless n % 128 == 0)
  const uint16_t* eo_lo;
  const uint16_t* eo_h;
  const uint16_t* eot_hi;
  const uint16_t* eot_lo;
  const uint16_t* eot_h;
  const double* lam_split;
};

// One tile of the even/odd DCT stages for one stage parity (rows of X are the
// map's rows for parity 0, its columns for parity 1), with everything a block
// reads to start the tile, so a tile costs one record load instead of a chain
// of descriptor loads.
struct EoTile {
  long long off;          // element offset of the map
  const uint16_t* tf[3];  // forward tables EO of the contracted side: fp16, bf16 hi, bf16 lo
  const uint16_t* ti[3];  // inverse tables EOt: fp16, bf16 hi, bf16 lo
  const double* lam_m;    // eigenvalues along M and along N, in split order
  const double* lam_n;
  int m, R, K, r0, c0;    // map, rows and contraction length at this parity, tile origin
  int local, ndt, gbd;    // tile index within the map, the map's tile count, arrival group base
  float lmin;             // smallest nonzero eigenvalue of the map's Laplacian
  int pad;
};

struct MapDesc {
  int M, N;
  int th;                     // stencil tile height (rows)
  int tiles_x, ntiles, tile0;  // stencil tiles
  int ndt, dtile0;             // DCT tiles (same count in every stage)
  int gb, gbd;                 // first arrival-group counter of the stencil / DCT tiles
  int use_iso;                 // zero the preconditioner output on isolated pixels
  long long off;               // element offset of this map in the work vectors
  const double* psi;           // caller's wrapped phase
  const float* mask;           // caller's quality mask or null
  double* phi;                 // caller's solution (FP64)
  const DctTabDev* tabM;
  const DctTabDev* tabN;
};

// PCG state of one map (written only by finisher kernels and by the host).
struct MapState {
  double delta_new, delta_old, delta0;
  double alpha, beta;
  double alpha_p;              // x[xi] lacks alpha_p d[l & 1] (added by the next SpMV)
  double dq, rr, bb, rs;
  double thr_rr, thr_delta, tol2, eps2;
  double rr_chk;               // true residual at the last stagnation checkpoint
  long long l_chk, chk_gap;    // its iteration; least iterations between compared checkpoints
  long long l, l_max, period, nfinish;
  long long brk_at;            // > 0: report iteration brk_at's d^T A d as a breakdown (testing hook)
  int state, rule, replaced, stall;  // stall: 1 = stop when the true residual stagnates
  int xi, pad_;                // x[xi] holds the iterate (up to the pending term)
  float amax[4];
};

struct Engine {
  int elem = 0;              // sizeof(T) of the vectors this engine was sized for
  int n_maps = 0, cap_maps = 0;
  long long total_px = 0, cap_px = 0;
  int total_tiles = 0, total_dtiles = 0, cap_tiles = 0, cap_dtiles = 0;
  int max_n = 1;             // widest map
  int wf_diags = 1, wf_len = 1;  // natural-order sweeps: most 64 x 64 tile anti-diagonals of a
                                 // map, and most tiles on one anti-diagonal
  int th = kTH;              // stencil tile height (rows)
  int grid = kEngineGrid;    // cap on the blocks of the stencil tile kernels
  int dct_grid = kDctGrid;   // cap on the blocks of a DCT stage (multiple of 8)
  std::vector<MapDesc> hdesc;
  MapDesc* desc = nullptr;
  MapState* ms = nullptr;
  MapState* hms = nullptr;   // pinned mirror
  int* tile_map = nullptr;   // global stencil tile -> map
  int* dtile_map = nullptr;  // global DCT tile -> map
  int* act = nullptr;        // active stencil tiles
  int* dact = nullptr;       // active DCT tiles: XCD-ordered lists of narrow tiles for the
                             // two stage parities, then of wide tiles (see driver)
  long long dlist_cap = 0;   // capacity of each of the four DCT lists
  int dct_trows = kDT;       // DCT output tile rows (64 dense, 128 even/odd)
  int* mact = nullptr;       // active maps (sweep kernels)
  int* fcnt = nullptr;       // per-map arrival counters of the fused finishers (zero between launches)
  int* gcnt = nullptr;       // per-group arrival counters (groups of kArriveGroup tiles of one map)
  double* gsum = nullptr;    // group sums of the fused finishers: 2 rows of gstride
  long long gstride = 0;
  EoTile* eot = nullptr;     // even/odd DCT tile records, [parity][global DCT tile]
  int* counts = nullptr;     // [0] active tiles, [1] DCT list (even stages), [2] active
                             // maps, [3] DCT list (odd stages), [5] and [7] the wide-tile
                             // lists; kListHead ints, followed in the same allocation by
                             // mact, act and dact
  int* hlist = nullptr;      // pinned staging for counts and the lists, same layout
  // FP64 arrays
  double* dx = nullptr;
  double* dy = nullptr;
  double* phi_prev = nullptr;
  double* r64 = nullptr;
  // T arrays (elem bytes per pixel)
  void* U = nullptr;
  void* V = nullptr;
  void* aux = nullptr;
  void* x[2] = {nullptr, nullptr};
  void* d[2] = {nullptr, nullptr};
  void* r = nullptr;
  void* s = nullptr;
  void* q = nullptr;
  void* b = nullptr;
  void* t1 = nullptr;
  void* t2 = nullptr;
  unsigned char* iso = nullptr;  // isolated-pixel flags
  double* P = nullptr;           // partials: kNumSlots x pstride
  long long pstride = 0;
};

}  // namespace lpu
