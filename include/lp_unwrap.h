/*
 * lp_unwrap -- L^p-norm phase unwrapping on one AMD Instinct MI355X (gfx950).
 *
 * The method (Legarda-Saenz, Brito-Loeza, Espinosa-Romero, "On the
 * performance of preconditioned methods to solve L^p-norm phase unwrapping",
 * arXiv 2203.13675):
 *
 *   Section 2, Eq. (2): minimise sum |grad phi - W(grad psi)|^p over the
 *   unwrapped phase phi, given the wrapped phase psi (Eq. (1)).
 *   Section 2.1, Eqs. (4)-(7): finite differences turn the Euler-Lagrange
 *   equation into A(U,V) phi = b, a weighted five-point Neumann Laplacian with
 *   weights U, V (Eq. (6)) that depend on phi.
 *   Algorithm 1: fixed-point loop -- recompute U, V from phi^k, solve the
 *   linear system with preconditioned CG (warm start phi^k), repeat.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Maps are M rows x N columns, row-major, contiguous (element (i, j) at
 *    i*N + j).  "x" differences run along j (contiguous), "y" along i.
 *  * Every array argument is a DEVICE pointer on the context's device, owned
 *    by the caller, that must stay valid until the call returns.  Calls are
 *    ordered on the context's stream and return only after the work they
 *    enqueue has completed (they read device status words).
 *  * A context is not thread-safe: use one context per host thread / stream.
 *  * Functions return an lpu_status; a negative value is an error and the
 *    outputs are unspecified.  lp_unwrap_last_error() describes the most
 *    recent error on a context.
 *  * Precision LPU_FP64: every vector, weight and reduction in double.
 *    Precision LPU_MIXED: weights and CG vectors in float, inner products
 *    accumulated in double, the outer residual b - A phi and the solution phi
 *    in double (iterative refinement).
 */
#ifndef LP_UNWRAP_H
#define LP_UNWRAP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lp_unwrap_ctx lp_unwrap_ctx;

/* Status codes. */
enum lpu_status {
    LPU_OK = 0,                /* converged (stop rule met)                       */
    LPU_NOT_CONVERGED = 1,     /* a cap (k_max, l_max, max_refine) was hit; the
                                  output phi is valid                              */
    LPU_ERR_INVALID_ARG = -1,  /* null pointer, empty map, p outside [0,2],
                                  tau <= 0, tol < 0, unknown preconditioner ...    */
    LPU_ERR_OOM = -2,          /* device allocation failed                        */
    LPU_ERR_HIP = -3,          /* HIP runtime error (message in last_error)       */
    LPU_ERR_NONFINITE = -4,    /* psi or the mask holds NaN/Inf                   */
    LPU_ERR_BREAKDOWN = -5     /* PCG breakdown: d^T A d <= 0 or a non-finite
                                  alpha/beta/delta                                 */
};

/* The preconditioners M of Section 2.1's list (I, D, ILU(0), IC(0), SOR) and
 * the DCT fast-Poisson preconditioner (M = unit-weight Neumann Laplacian). */
enum lpu_preconditioner {
    LPU_PC_NONE = 0,    /* M = I: plain CG                                      */
    LPU_PC_JACOBI = 1,  /* M = diag(A)                                          */
    LPU_PC_ILU0 = 2,    /* incomplete LU, no fill-in, natural row-major order    */
    LPU_PC_IC0 = 3,     /* incomplete Cholesky, no fill-in; for this symmetric
                           five-point matrix it equals ILU(0)                    */
    LPU_PC_SSOR = 4,    /* symmetric SOR with relaxation ssor_omega              */
    LPU_PC_DCT = 5,     /* DCT-II/III Poisson solve, zero mode dropped           */
    /* The same three factorisations of the matrix taken in two-colour (red-black)
       order: pixels with i + j even first, then odd, row-major within a colour.
       A different M from the natural-order ones (not in the paper); both of its
       triangular solves are one parallel pass each.                            */
    LPU_PC_ILU0_RB = 6, /* ILU(0) in two-colour order                            */
    LPU_PC_IC0_RB = 7,  /* IC(0) in two-colour order (equals LPU_PC_ILU0_RB)      */
    LPU_PC_SSOR_RB = 8  /* SSOR(ssor_omega) in two-colour order                  */
};

enum lpu_stop_rule {
    LPU_STOP_RELRES = 0, /* ||b - A phi|| <= tol ||b||, confirmed on the true residual */
    LPU_STOP_PAPER = 1   /* delta_new <= eps_cg^2 delta_0 (Algorithm 1's inner test)   */
};

enum lpu_precision { LPU_FP64 = 0, LPU_MIXED = 1 };

/* Arithmetic of the DCT transforms in the MIXED path (FP64 path: always FP64). */
enum lpu_dct_mode {
    LPU_DCT_FP32 = 0,        /* FP32 FMA GEMMs                                   */
    LPU_DCT_SPLIT_BF16 = 1,  /* bf16 hi/lo split, 3 MFMA products, FP32 accumulate */
    LPU_DCT_FP16_SCALED = 2  /* power-of-two scaled fp16, 1 MFMA product, FP32 acc */
};

typedef struct lpu_options {
    int k_max;             /* outer iterations cap (default 500, Section 3)            */
    double outer_tol;      /* outer relative-change tolerance (default 1e-6, Section 3);
                              <= 0: run exactly k_max outer iterations                  */
    long long l_max;       /* inner iterations cap per solve; <= 0: 2*M*N (Section 3)   */
    int stop_rule;         /* lpu_stop_rule (default LPU_STOP_RELRES)                   */
    double eps_cg;         /* epsilon of LPU_STOP_PAPER (default 0.005, Section 3)      */
    int residual_period;   /* true-residual replacement period; <= 0: floor(sqrt(MN))  */
    double ssor_omega;     /* SSOR relaxation in (0, 2) (default 1)                     */
    int precision;         /* lpu_precision (default LPU_MIXED)                         */
    int dct_mode;          /* lpu_dct_mode (default LPU_DCT_SPLIT_BF16)                 */
    int use_phi0;          /* 1: phi holds the start value on entry; 0: start at 0      */
    double refine_eta;     /* MIXED: relative residual reduction asked of each FP32
                              inner solve (default 1e-3)                               */
    int max_refine;        /* MIXED: refinement steps cap per outer iteration (default 30) */
} lpu_options;

typedef struct lpu_stats {
    int outer_iters;             /* outer iterations run                              */
    long long inner_iters_total; /* PCG iterations summed over all inner solves       */
    int refinements;             /* MIXED: FP32 inner solves run (FP64: = outer_iters) */
    double final_relres;         /* ||b - A phi|| / ||b|| of the last system, in FP64  */
    double outer_err;            /* last ||phi^{k+1} - phi^k|| / ||phi^k|| (inf at 0)   */
    double setup_ms;             /* time building U, V, b and M                        */
    double solve_ms;             /* wall time of the whole call                        */
    int converged;               /* 1 when the call returns LPU_OK                     */
    int status;                  /* status of this map                                 */
} lpu_stats;

/* One map of a batch (all pointers device pointers, see conventions). */
typedef struct lpu_map {
    int rows, cols;        /* M, N                                                 */
    const double* psi;     /* wrapped phase, M*N doubles in (-pi, pi]               */
    const float* mask;     /* quality in [0,1], M*N floats, or NULL (all ones)      */
    double* phi;           /* output unwrapped phase, M*N doubles (input: phi0)     */
} lpu_map;

/* Fill *opt with the defaults listed above. */
void lpu_default_options(lpu_options* opt);

/* Create a context bound to HIP device `device` and stream `stream` (a
 * hipStream_t; NULL = the null stream).  With max_rows, max_cols > 0 the work
 * buffers for one map of up to max_rows x max_cols (either precision, the
 * default tile height) are allocated now, so a first lp_unwrap_solve of such
 * a map allocates only its DCT tables; 0, 0 allocates on first use.  A batch,
 * a larger map or a smaller tile height grows the buffers (reallocation drops
 * the context's cached graphs).  The context owns its workspace; free it
 * with lp_unwrap_destroy.  Errors: LPU_ERR_INVALID_ARG (also for
 * max_rows * max_cols > 2^31), LPU_ERR_OOM, LPU_ERR_HIP. */
int lp_unwrap_create(lp_unwrap_ctx** out, int device, void* stream, int max_rows, int max_cols);

/* Destroy a context and free its device memory.  NULL is ignored. */
void lp_unwrap_destroy(lp_unwrap_ctx* ctx);

/* Unwrap one map: Algorithm 1 with the chosen preconditioner.
 *   psi      [in]  M*N doubles, the wrapped phase of Eq. (1).
 *   mask     [in]  M*N floats in [0,1] or NULL.  Edge quality is
 *                  min(mask_a, mask_b) and multiplies the weights U, V of
 *                  Eq. (6).  Pixels with no weighted edge keep phi0.
 *   p        L^p exponent of Eq. (2), 0 <= p <= 2.
 *   eps      tau of Eq. (6) (> 0; the paper uses 0.01).
 *   preconditioner  lpu_preconditioner.
 *   tol      inner stop tolerance: relative residual of each linear system
 *            (LPU_STOP_RELRES) -- the target the outer loop also uses for the
 *            FP64 residual in the MIXED path.
 *   opts     NULL for lpu_default_options.
 *   phi      [in/out] M*N doubles.
 *   stats    [out] may be NULL.
 * Returns LPU_OK, LPU_NOT_CONVERGED or an error (see lpu_status). */
int lp_unwrap_solve(lp_unwrap_ctx* ctx, int M, int N, const double* psi, const float* mask,
                    double p, double eps, int preconditioner, double tol,
                    const lpu_options* opts, double* phi, lpu_stats* stats);

/* Unwrap n_maps independent maps of possibly different sizes together.
 * `maps` is a HOST array of n_maps descriptors whose pointers are device
 * pointers.  Every map runs Algorithm 1 with the same p, eps, preconditioner,
 * tol and options; each map stops on its own (per-map convergence flags), and
 * every step of every iteration is one launch for all active maps.
 * Every preconditioner of lpu_preconditioner is supported.  The natural-order
 * ILU(0) / IC(0) / SSOR sweeps are sequential along each map, so each map's
 * sweep is walked by one workgroup; the other preconditioners are tiled over
 * the whole device.
 * per_map: HOST array of n_maps lpu_stats, or NULL.
 * Returns the worst status over the maps (an error if any map failed). */
int lp_unwrap_batch(lp_unwrap_ctx* ctx, int n_maps, const lpu_map* maps, double p, double eps,
                    int preconditioner, double tol, const lpu_options* opts, lpu_stats* per_map);

/* Text for a status code; never NULL. */
const char* lp_unwrap_status_string(int status);

/* Description of the last error on ctx (empty string if none); never NULL. */
const char* lp_unwrap_last_error(const lp_unwrap_ctx* ctx);

/* ----------------------------------------------------------------------------
 * Single steps of the path, exposed so each step can be checked on its own.
 * The wrapped differences, weights, right-hand side, pivots and the DCT, sweep
 * and two-colour preconditioner applies run the kernels the solver runs.  Two
 * steps run a plain kernel of their own instead of the solver's fused one:
 * lpu_apply_A (the solver forms A d inside its fused direction-update + SpMV
 * kernel) and the Jacobi apply of lpu_precond_apply (the solver scales r inside
 * its fused update kernel); the fused kernels are checked through whole solves.
 * All step calls use the context's work buffers and synchronise the stream
 * before returning.  `precision` selects the element type of the
 * weight/vector arguments typed void*: float for LPU_MIXED, double for
 * LPU_FP64.
 * ------------------------------------------------------------------------- */

/* Section 2.1: Delta^x_{i,j} = W(psi_{i,j+1} - psi_{i,j}) for j < N-1 and
 * Delta^y_{i,j} = W(psi_{i+1,j} - psi_{i,j}) for i < M-1, with
 * W(x) = x - 2 pi ceil((x - pi) / (2 pi)) in (-pi, pi] (Eq. (1) range),
 * evaluated in FP64.  dx's last column and dy's last row are written as 0.
 * psi, dx, dy: M*N doubles. */
int lpu_wrapped_differences(lp_unwrap_ctx* ctx, int M, int N, const double* psi,
                            double* dx, double* dy);

/* Eq. (6): U_{i,j} = w^x_{i,j} tau / (|phi_{i,j+1} - phi_{i,j} - Delta^x_{i,j}|^(2-p) + tau)
 * for j < N-1 and 0 on the last column; V likewise along i with 0 on the last
 * row.  w is the edge quality min(mask_a, mask_b) (1 without a mask).
 * phi, dx, dy: M*N doubles; mask: M*N floats or NULL; U, V: M*N elements of
 * the precision's type. */
int lpu_weights(lp_unwrap_ctx* ctx, int M, int N, int precision, const double* phi,
                const double* dx, const double* dy, const float* mask, double p, double tau,
                void* U, void* V);

/* Eq. (7), left side: y = A(U,V) x for every pixel.  U, V, x, y: M*N elements. */
int lpu_apply_A(lp_unwrap_ctx* ctx, int M, int N, int precision, const void* U, const void* V,
                const void* x, void* y);

/* Eq. (7), right side: b = Delta^x_{i,j-1}U_{i,j-1} - Delta^x_{i,j}U_{i,j}
 * + Delta^y_{i-1,j}V_{i-1,j} - Delta^y_{i,j}V_{i,j}, computed in FP64 from
 * the stored weights.  b: M*N doubles. */
int lpu_rhs(lp_unwrap_ctx* ctx, int M, int N, int precision, const void* U, const void* V,
            const double* dx, const double* dy, double* b);

/* s = M^{-1} r for the preconditioner built from U, V (Section 2.1's list
 * and the DCT Poisson solve); zero on pixels with no weighted edge.
 * dct_mode applies to LPU_MIXED only.  U, V, r, s: M*N elements. */
int lpu_precond_apply(lp_unwrap_ctx* ctx, int M, int N, int precision, int preconditioner,
                      int dct_mode, double omega, const void* U, const void* V,
                      const void* r, void* s);

/* ILU(0) = IC(0) pivots of A(U,V) in natural order: the diagonal of the
 * no-fill factor, d_{i,j} = a_{i,j} - U_{i,j-1}^2/d_{i,j-1} - V_{i-1,j}^2/d_{i-1,j},
 * a pivot below 1e-4 a_{i,j} replaced by a_{i,j}; 1 on isolated pixels.
 * U, V, piv: M*N elements. */
int lpu_ilu_pivots(lp_unwrap_ctx* ctx, int M, int N, int precision, const void* U,
                   const void* V, void* piv);

/* ----------------------------------------------------------------------------
 * Instrumentation (tracing).  Kernel classes of the path: */
enum lpu_kernel_class {
    LPU_KC_SPMV = 0,     /* direction update + q = A d + d^T q           */
    LPU_KC_UPDATE = 1,   /* x, r updates, pointwise preconditioner, dots  */
    LPU_KC_CONFIRM = 2,  /* true-residual confirmation                     */
    LPU_KC_INIT = 3,     /* r0 = b - A x0                                  */
    LPU_KC_DCT = 4,      /* one DCT contraction stage                      */
    LPU_KC_SWEEP = 5,    /* ILU/IC/SSOR forward+backward sweeps            */
    LPU_KC_SETUP = 6,    /* weights, b, preconditioner set-up, refinement  */
    LPU_KC_TWOCOLOR = 7, /* the two passes of a two-colour preconditioner  */
    LPU_KC_COUNT = 8
};

/* Time every launch of the kernel classes whose bit (1 << class) is set in
 * class_mask with HIP events recorded on the context's stream (0: off; the
 * events add a little host work per launch).  Resets the accumulators. */
int lpu_kernel_timing(lp_unwrap_ctx* ctx, unsigned int class_mask);

/* Accumulated figures of one class since the last lpu_kernel_timing call:
 * summed event durations (ms), number of launches, and the algorithmic bytes
 * moved and flops executed by those launches (from the launch shapes: the
 * bytes each kernel must read and write once, the contraction's multiply-adds
 * x 2 x products per element for MFMA stages).  Any output may be NULL. */
int lpu_kernel_timing_get(lp_unwrap_ctx* ctx, int kernel_class, double* total_ms,
                          long long* launches, double* alg_bytes, double* alg_flops);

/* ----------------------------------------------------------------------------
 * Launch tuning.  None of these settings changes what is computed (Algorithm
 * 1 and its arithmetic are the same); they change tile shapes, grid sizes and
 * how the PCG iterations are issued.  Tile shape and grid size change the
 * order in which FP64 partial sums of the dot products are added, so results
 * may differ in the last bits between settings (bit-identical for repeated
 * calls with one setting).
 * ------------------------------------------------------------------------- */
typedef struct lpu_tuning {
    int tile_rows;        /* rows per stencil tile (one wave, 128 columns): 4, 8, 16, 32 or 64 */
    int grid;             /* blocks of the grid-stride stencil kernels: 64 .. 65536            */
    int dct_grid;         /* cap on the blocks of a DCT stage: 64 .. 65536                     */
    int use_graph;        /* 1: issue PCG iterations as captured HIP graphs of 8, 4, 2 and 1
                             iterations.  The context keeps up to 64 of them across calls
                             (keyed on launch shapes and preconditioner parameters) and
                             drops them when its work buffers are reallocated or it is
                             destroyed                                                      */
    int max_batch_iters;  /* iterations issued between host reads of the map states: 2 .. 1024 */
} lpu_tuning;

/* Defaults: tile_rows 16, grid 16384, dct_grid 2048, use_graph 1,
 * max_batch_iters 64. */
void lpu_default_tuning(lpu_tuning* t);

/* Replace / read the context's tuning.  Out-of-range fields give
 * LPU_ERR_INVALID_ARG and leave the tuning unchanged. */
int lp_unwrap_set_tuning(lp_unwrap_ctx* ctx, const lpu_tuning* t);
int lp_unwrap_get_tuning(lp_unwrap_ctx* ctx, lpu_tuning* t);

/* Autotuner: time candidate tunings on the given batch (same arguments as
 * lp_unwrap_batch) and install the fastest on ctx.  Each candidate runs one
 * outer iteration capped at `probe_iters` PCG iterations per map (a fixed
 * amount of work for every candidate); the maps' phi arrays are overwritten
 * (with use_phi0 = 0 semantics).  Coordinate search: tile_rows, then grid,
 * then dct_grid, then use_graph; a candidate replaces the current choice only
 * when it is at least 1 % faster.
 *   cache_path  text file of "key tile_rows grid dct_grid use_graph
 *               max_batch_iters" lines, or NULL.  The key covers the device
 *               name, preconditioner, precision, DCT mode and the multiset of
 *               map shapes.  A hit installs the stored tuning without timing;
 *               a miss appends the winner.
 *   best        [out] the installed tuning, may be NULL.
 *   tune_ms     [out] wall time spent timing candidates (0 on a cache hit),
 *               may be NULL.
 * Returns LPU_OK or an error; the context keeps its previous tuning on error. */
int lp_unwrap_autotune(lp_unwrap_ctx* ctx, int n_maps, const lpu_map* maps, double p, double eps,
                       int preconditioner, double tol, const lpu_options* opts, int probe_iters,
                       const char* cache_path, lpu_tuning* best, double* tune_ms);

/* ----------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * preconditioner apply of lpu_precond_apply without any allocation.
 *   s = M^{-1} r for every preconditioner except LPU_PC_DCT (whose tables
 *   must be allocated; use lpu_precond_apply), same kernels and results as
 *   lpu_precond_apply with the context's tile height.  U, V, r, s: M*N device
 *   elements of the precision's type (caller-owned, as there).
 *   Limits: M*N <= 1048576 pixels (1024 x 1024), at most 65536 stencil tiles,
 *   N <= 4096 for the natural-order sweeps; larger inputs give
 *   LPU_ERR_INVALID_ARG with a message.  omega: SSOR relaxation in (0, 2).
 * Working memory is one static device array of about 20 MB per device, held
 * until the process ends and shared by every call on that device: calls that
 * overlap on one device (several streams or contexts) race and must be
 * serialised by the caller.  The call only enqueues work on the context's
 * stream (no allocation, no synchronisation, no host read-back) and returns
 * LPU_OK; s is ready when the stream reaches that point.  Errors:
 * LPU_ERR_INVALID_ARG, LPU_ERR_HIP (launch failure, or the array's address
 * could not be looked up when the context was created).
 * ------------------------------------------------------------------------- */
int lpu_precond_apply_noalloc(lp_unwrap_ctx* ctx, int M, int N, int precision, int preconditioner,
                              double omega, const void* U, const void* V, const void* r, void* s);

/* ----------------------------------------------------------------------------
 * Testing hook for the failure path of Algorithm 1's inner loop: from the
 * next solve on, the step length of PCG iteration `iteration` (1-based) of
 * every inner solve is treated as a breakdown (as if d^T A d <= 0), so the
 * solve returns LPU_ERR_BREAKDOWN through the same per-map state and exit as
 * a real breakdown; every kernel still runs to completion.  iteration <= 0
 * switches it off.  Errors: LPU_ERR_INVALID_ARG for a null context.
 * ------------------------------------------------------------------------- */
int lpu_debug_force_breakdown(lp_unwrap_ctx* ctx, long long iteration);

#ifdef __cplusplus
}
#endif

#endif /* LP_UNWRAP_H */
