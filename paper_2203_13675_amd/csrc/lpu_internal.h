// Internal declarations shared by the HIP translation units of liblp_unwrap.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lp_unwrap.h"

namespace lpu {

constexpr double kPi = 3.141592653589793115997963468544185161590576171875;  // FP64 pi
constexpr double kTwoPi = 2.0 * kPi;
constexpr double kPivotFloor = 1e-4;  // ILU/IC pivot below this x diagonal -> diagonal

// PCG state machine of one map, kept in device memory and advanced by the
// finisher kernels, so the host can enqueue many iterations without reading
// anything back.
enum CgState : int {
  kRun = 0,        // iterate
  kConfirm = 1,    // the recursive residual met the bound: replace it by b - A x
  kConfirmPc = 2,  // true residual formed, waiting for the preconditioner
  kInitPc = 3,     // initial residual formed, waiting for the preconditioner
  kDone = 4,       // stop rule met
  kCap = 5,        // l_max reached
  kBreakdown = 6,  // d^T A d <= 0 or non-finite scalars
  kStall = 7       // true residual stopped improving (mixed inner solves only)
};

// How a finisher completes a PCG step.
enum FinishMode : int { kFinishNone = 0, kFinishInit = 1, kFinishIter = 2, kFinishConfirm = 3 };

enum PcKind : int { kPcNone = 0, kPcJacobi = 1, kPcIlu = 2, kPcIc = 3, kPcSsor = 4, kPcDct = 5,
                    kPcIluRb = 6, kPcIcRb = 7, kPcSsorRb = 8 };
// two-colour (red-black) ordered factorisations
inline bool two_colour(int pc) { return pc == kPcIluRb || pc == kPcIcRb || pc == kPcSsorRb; }

// DCT tables for one size n, in every arithmetic the kernels use.
struct DctTables {
  int n = 0;
  double* c64 = nullptr;    // C[k][j], n*n
  double* ct64 = nullptr;   // C^T
  float* c32 = nullptr;
  float* ct32 = nullptr;
  uint16_t* c_hi = nullptr;   // bf16 split of C
  uint16_t* c_lo = nullptr;
  uint16_t* ct_hi = nullptr;  // bf16 split of C^T
  uint16_t* ct_lo = nullptr;
  uint16_t* c_h = nullptr;    // fp16 C
  uint16_t* ct_h = nullptr;   // fp16 C^T
  double* lam = nullptr;      // 2 - 2 cos(pi k / n)
  // Even/odd factorisation (n a multiple of 128, h = n/2): spectra are kept
  // in split order (even k first, then odd k).
  //   EO  (n x h): row c < h is C[2c][0..h), row h + c is C[2c+1][0..h)
  //   EOt (h x n): row j is [C[0][j], C[2][j], ..., C[1][j], C[3][j], ...]
  uint16_t* eo_hi = nullptr;
  uint16_t* eo_lo = nullptr;
  uint16_t* eo_h = nullptr;
  uint16_t* eot_hi = nullptr;
  uint16_t* eot_lo = nullptr;
  uint16_t* eot_h = nullptr;
  double* lam_split = nullptr;  // eigenvalues in split order
};

// HIP-event timing of selected kernel classes (instrumentation).
struct KTimer {
  unsigned int mask = 0;
  struct Rec {
    int a, b, cls;
  };
  std::vector<hipEvent_t> events;  // pool
  std::vector<Rec> pending;
  int next_event = 0;
  double ms[LPU_KC_COUNT] = {};
  long long n[LPU_KC_COUNT] = {};
  double bytes[LPU_KC_COUNT] = {};
  double flops[LPU_KC_COUNT] = {};
  bool on(int cls) const { return (mask >> cls) & 1u; }
  int begin(int cls, hipStream_t st);  // start event index or -1
  void end(int idx, int cls, hipStream_t st);
  // credit the algorithmic figures of work done by timed launches (launches
  // themselves are counted as they are recorded)
  void credit(int cls, long long launches, double b, double f) {
    (void)launches;
    if (!on(cls)) return;
    bytes[cls] += b;
    flops[cls] += f;
  }
  void flush();
  void reset();
  void destroy();
};

}  // namespace lpu

#include "engine.h"

namespace lpu {

// Executable graph of one PCG iteration for one launch shape; valid until the
// engine is laid out again (the cache is emptied by every engine set-up).
constexpr int kGraphKey = 12;
struct GraphEntry {
  int key[kGraphKey];  // launch shapes, DCT tile width, preconditioner and its parameters, precision,
                       // tile height, iterations per graph
  hipGraphExec_t exec;
};

}  // namespace lpu

struct lp_unwrap_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  std::string last_error;
  lpu_tuning tune;
  lpu::Engine eng;
  std::vector<lpu::GraphEntry> graphs;  // small cache, emptied by every engine set-up
  std::deque<lpu::DctTables> dct;  // cached per size (deque: stable references)
  std::vector<std::pair<int, lpu::DctTabDev*>> dct_dev;
  hipEvent_t list_event = nullptr;  // last upload from the pinned list staging
  bool list_event_live = false;
  lpu::KTimer kt;
  long long debug_breakdown_at = 0;  // lpu_debug_force_breakdown (0: off)
};

namespace lpu {

int set_error(lp_unwrap_ctx* ctx, int code, const std::string& msg);
#define LPU_HIP_CHECK(ctx, call)                                                       \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::lpu::set_error((ctx), LPU_ERR_HIP,                                      \
                              std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

const DctTables* get_dct_tables(lp_unwrap_ctx* ctx, int n, int* status);
void free_dct_tables(lp_unwrap_ctx* ctx);

// engine (driver.hip)
void release_graphs(lp_unwrap_ctx* ctx);
int engine_solve(lp_unwrap_ctx* ctx, int n, const lpu_map* maps, double p, double tau, int pc,
                 double tol, const lpu_options& o, lpu_stats* stats);
void engine_release(lp_unwrap_ctx* ctx);
int engine_reserve(lp_unwrap_ctx* ctx, int M, int N);
// noalloc.hip: look up the no-allocation entry point's scratch array on `device`
// (current); LPU_OK or LPU_ERR_HIP
int noalloc_bind(int device);
int step_wrapdiff(lp_unwrap_ctx* ctx, int M, int N, const double* psi, double* dx, double* dy);
template <typename T>
int step_weights(lp_unwrap_ctx* ctx, int M, int N, const double* phi, const double* dx,
                 const double* dy, const float* mask, double p, double tau, T* U, T* V);
template <typename T>
int step_apply(lp_unwrap_ctx* ctx, int M, int N, const T* U, const T* V, const T* x, T* y);
template <typename T>
int step_rhs(lp_unwrap_ctx* ctx, int M, int N, const T* U, const T* V, const double* dx,
             const double* dy, double* b);
template <typename T>
int step_pivots(lp_unwrap_ctx* ctx, int M, int N, const T* U, const T* V, T* piv, bool ssor,
                double omega);
template <typename T>
int step_precond(lp_unwrap_ctx* ctx, int M, int N, int pc, int dct_mode, double omega, const T* U,
                 const T* V, const T* r, T* s);

// small utilities (util.hip)
template <typename T>
void launch_scale_by(hipStream_t st, size_t n, const T* a, const T* b, T* out);

}  // namespace lpu
