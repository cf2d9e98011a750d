/*
 * qbw.h - C ABI of libqbw: quantization-based bounds on the Wasserstein
 * metric for discrete measures on regular grids, on AMD MI355X (gfx950).
 *
 * The method (Bobrutsky & Moscovich, "Quantization-based Bounds on the
 * Wasserstein Metric"): measures a (= mu) and b (= nu) on X = [N]^d with
 * ground cost |x - y|^p are sum-pooled by a factor k onto an n^d coarse grid
 * (n = N / k, Section 2.2); one exact coarse Kantorovich problem on the
 * centre cost is solved; then
 *   - lower bound (Section 3.5, Algorithm 5): the coarse potential is
 *     upscaled by multilinear interpolation and improved by two c-transforms
 *     over all fine pixel pairs; bound = (<f, a> + <g, b>)^(1/p);
 *   - upper bound (Section 3.4, Algorithm 4): the coarse coupling is upscaled
 *     with the uniform kernel, its marginals corrected by iterative
 *     proportional fitting (IPF), its fine cost evaluated on its support, and
 *     weighted total-variation corrections (eq. of the weighted total
 *     variation) added.
 * The marginally weighted coarse cost C-bar of Section 3.2 (Algorithm 3) is
 * exported as well.
 *
 * Conventions shared by every call:
 *   - A measure is float64, C-contiguous with shape (N,)*d, nonnegative; a
 *     and b must have equal mass (they are normally probability vectors).
 *     Pixel (x_0, ..., x_{d-1}) has integer coordinates in 0..N-1 and flat
 *     index ((x_0 N + x_1) N + ...) (C order).  Coarse block K has flat index
 *     over [n]^d in the same order; its centre is k K + (k - 1) / 2.
 *   - d in {2, 3}, p in {1, 2}, N % k == 0, 1 <= k <= N.  Violations return
 *     QBW_E_GRID.
 *   - "device" pointers are HIP device memory of the context's device;
 *     "host" pointers are ordinary host memory.  The caller owns every buffer
 *     it passes; the library owns its context workspaces.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *     enqueued on it; calls that return host values synchronise it.
 *   - Every call returns a qbw_status; nothing is thrown across the ABI.  On
 *     failure qbw_last_error() returns a message for the calling thread.
 *   - Contexts are not thread safe: use one context per host thread.
 */
#ifndef QBW_H
#define QBW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum qbw_status {
  QBW_OK = 0,
  QBW_E_INVAL = 1,  /* null pointer, bad option, bad size */
  QBW_E_GRID = 2,   /* d not in {2,3}, p not in {1,2}, N % k != 0, ... */
  QBW_E_MASS = 3,   /* negative or NaN mass, unequal or zero total mass */
  QBW_E_LP = 4,     /* the coarse network simplex failed */
  QBW_E_HIP = 5,    /* a HIP runtime call failed */
  QBW_E_NOMEM = 6,  /* device or host allocation failed */
  QBW_E_STATE = 7   /* object used in the wrong state */
} qbw_status;

typedef struct qbw_grid {
  int32_t d;  /* dimension, 2 or 3 */
  int32_t N;  /* fine grid side */
  int32_t k;  /* pooling factor kappa; coarse side n = N / k */
  int32_t p;  /* ground cost |x - y|^p, p in {1, 2} */
} qbw_grid;

/* qbw_opts.flags */
#define QBW_WANT_ARGMIN 1u   /* also compute c-transform arg-mins (needed for d/d f^) */
#define QBW_SAVE_FOR_BWD 2u  /* keep what qbw_bounds_backward needs */
#define QBW_SEPARABLE 4u     /* p = 2: evaluate each c-transform as d nested 1-D transforms
                                (O(N^(d+1)) instead of O(N^(2d)); float32 rounding once per
                                axis, larger derived shift); ignored for p = 1 */
#define QBW_SEPARABLE_EXACT 32u /* p = 2: the same values and arg-mins as the all-pairs
                                   c-transform (Section 4), from exact per-axis minima in
                                   float64, certified per target against float32 rounding,
                                   brute force where a target cannot be certified (near or
                                   exact ties); not with QBW_SEPARABLE; ignored for p = 1 */
/* Interpolation R of the coarse potential (Section 3.5 admits any; the
 * default is multilinear, as in the paper's experiments).  At most one. */
#define QBW_INTERP_NEAREST 8u  /* f^ = f~ of the pixel's own block (its nearest centre) */
#define QBW_INTERP_CUBIC 16u   /* separable Catmull-Rom cubic convolution through the
                                  block centres, edge taps replicated */

/* qbw_result.warn bits */
#define QBW_WARN_IPF_NOT_CONVERGED 1u /* stopped at max_ipf_iter; the upper bound stays valid */
#define QBW_WARN_LB_CLIPPED 2u        /* <f,a>+<g,b>-shift <= 0; lower bound clipped to 0 */

typedef struct qbw_opts {
  double xi;            /* IPF stop: ||a^ - a||_1 + ||b - b^||_1 < xi (default 1e-12) */
  int32_t max_ipf_iter; /* IPF iteration cap (default 50, >= 1) */
  uint32_t flags;       /* QBW_WANT_ARGMIN | QBW_SAVE_FOR_BWD | QBW_SEPARABLE or
                           QBW_SEPARABLE_EXACT | QBW_INTERP_NEAREST or QBW_INTERP_CUBIC */
} qbw_opts;

typedef struct qbw_result {
  double lower;            /* emitted lower bound on W_p (<= the float64 value of Algorithm 5) */
  double upper;            /* emitted upper bound on W_p (>= the float64 value of Algorithm 4) */
  double lower_S;          /* <f,a> + <g,b> - feas_shift, in units of W_p^p */
  double feas_shift;       /* float32 rounding shift subtracted from <f,a> + <g,b> */
  double upper_cost;       /* emitted <pi^_xi, C> (units of W_p^p), rounded outwards */
  double tv_mu, tv_nu;     /* emitted weighted-TV corrections Delta_mu^, Delta_nu^ */
  double ipf_residual;     /* ||a^ - a||_1 + ||b - b^||_1 at the last IPF iteration */
  double coarse_objective; /* <pi~, C~> of the coarse coupling used */
  int32_t ipf_iters;       /* IPF iterations taken */
  uint32_t warn;           /* QBW_WARN_* bits */
} qbw_result;

/* A coarse solution (pi~, f~) in host memory, owned by the caller.
 * rows/cols/vals: the coupling of the coarse measures as COO with block
 * indices in [0, Q); f: the coarse potential on the a side (length Q).
 * Any coupling of the coarse measures gives a valid upper bound and any f
 * gives a valid lower bound (the lemma of the triangle-inequality upper bound
 * and the proposition of Section 3.5); optimal ones give the tight bounds. */
typedef struct qbw_coarse {
  int32_t Q;   /* n^d */
  int32_t nnz; /* entries of the coupling (<= 2Q - 1 for a basic solution) */
  const int32_t* rows;
  const int32_t* cols;
  const double* vals;
  const double* f;
} qbw_coarse;

typedef struct qbw_ctx qbw_ctx;
typedef struct qbw_saved qbw_saved;
typedef struct qbw_batch qbw_batch;
typedef void* qbw_stream; /* hipStream_t */

/* ---- context ----------------------------------------------------------- */

/* Create a context bound to HIP device `device` (workspaces grow on demand).
 * A context is used by one thread at a time; saved records (below) may be
 * freed from any thread.  Errors: QBW_E_HIP if the device cannot be set,
 * QBW_E_NOMEM. */
qbw_status qbw_create(qbw_ctx** ctx, int32_t device);
/* Free a context and its workspaces (NULL is a no-op).  Saved records still
 * alive are detached and stay valid until qbw_saved_free. */
void qbw_destroy(qbw_ctx* ctx);
/* Thread-local message of the last failure (never NULL). */
const char* qbw_last_error(void);
/* xi = 1e-12, max_ipf_iter = 50, flags = 0. */
qbw_opts qbw_default_opts(void);
/* Library version string. */
const char* qbw_version(void);

/* ---- whole method ------------------------------------------------------ */

/* Lower and upper bound of W_p(a, b) (Algorithms 4 and 5).  a, b: device.
 * Pools a and b on the device, copies the coarse measures to the host, solves
 * the coarse problem with the project's network simplex (host, serial),
 * uploads the solution and runs the fine stages on the device.  out: host.
 * saved: if opts.flags has QBW_SAVE_FOR_BWD and saved != NULL, receives a
 * handle for qbw_bounds_backward (free with qbw_saved_free); a and b must stay
 * valid until then.  Errors: QBW_E_GRID, QBW_E_MASS (checked on the pooled
 * masses), QBW_E_LP, QBW_E_HIP. */
qbw_status qbw_bounds(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                      const qbw_opts* opts, qbw_result* out, qbw_saved** saved, qbw_stream stream);

/* Same as qbw_bounds with the coarse solution supplied by the caller (host
 * memory, see qbw_coarse); no coarse solve.  Validates coarse->Q == n^d and
 * every index.  Errors: QBW_E_GRID, QBW_E_INVAL, QBW_E_HIP. */
qbw_status qbw_bounds_with_coarse(qbw_ctx* ctx, const qbw_grid* grid, const double* a,
                                  const double* b, const qbw_coarse* coarse, const qbw_opts* opts,
                                  qbw_result* out, qbw_saved** saved, qbw_stream stream);

/* Gradients of dlower * lower + dupper * upper with respect to a and b, with
 * the coarse solution frozen, accumulated (+=) into grad_a, grad_b (device,
 * float64, shape of a).  Lower bound: through the potentials (d S / d a = f,
 * d S / d b = g).  Upper bound: through the plan cost and the exact number of
 * IPF iterations of the forward pass (checkpointed iterates); the TV
 * corrections are treated as constants.  grad_fhat (device float64 of length
 * N^d, may be NULL) receives d lower / d f^ through the c-transform arg-mins
 * (requires QBW_WANT_ARGMIN in the forward).  Errors: QBW_E_STATE. */
qbw_status qbw_bounds_backward(qbw_ctx* ctx, const qbw_saved* saved, double dlower, double dupper,
                               double* grad_a, double* grad_b, double* grad_fhat,
                               qbw_stream stream);
/* Free a saved record (NULL is a no-op).  Its device memory goes back to the
 * context that made it, if that context still exists, for the next record. */
void qbw_saved_free(qbw_saved* saved);

/* ---- stages (each follows one step of the method) ---------------------- */

/* SumPool with size and stride k (Section 2.2): out[K] = sum of m over block
 * K.  m: device (N^d), out: device (n^d float64). */
qbw_status qbw_sumpool(qbw_ctx* ctx, const qbw_grid* grid, const double* m, double* out,
                       qbw_stream stream);

/* Centre cost C~_KL = |x~_K - x~_L|^p (Algorithms 4-5): out host, n^d x n^d,
 * row-major. */
qbw_status qbw_coarse_cost(const qbw_grid* grid, double* out);

/* Marginally weighted cost (Section 3.2, Algorithm 3):
 * C-bar_KL = sum_{x in X_K, y in Y_L} |x - y|^p a(x) b(y) / (a~_K b~_L), with
 * C-bar_KL = C~_KL where a~_K b~_L = 0.  a, b: device; out: device, n^d x n^d
 * float64 row-major. */
qbw_status qbw_cbar(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                    double* out, qbw_stream stream);

/* Exact coarse Kantorovich solve on C~ (network simplex, host).  a_t, b_t:
 * host coarse measures (n^d).  Outputs (host, caller-allocated): rows, cols,
 * vals with capacity 2 n^d - 1, *nnz; f, g (n^d) optimal potentials with
 * f_K + g_L <= C~_KL, shifted so that sum_K a_t[K] f[K] = 0 (within 1/2 for
 * p = 2, where the shift is rounded to keep the potentials integers);
 * *objective = <pi~, C~>.  Errors: QBW_E_MASS, QBW_E_LP. */
qbw_status qbw_coarse_solve_host(const qbw_grid* grid, const double* a_t, const double* b_t,
                                 int32_t* rows, int32_t* cols, double* vals, int32_t* nnz,
                                 double* f, double* g, double* objective);

/* Multilinear upscaling of a coarse potential (Section 3.5, interpolation
 * R): ftil device float64 (n^d) -> fhat device float32 (N^d).  Pixels
 * outside the hull of the block centres take the nearest edge value. */
qbw_status qbw_upscale_potential(qbw_ctx* ctx, const qbw_grid* grid, const double* ftil,
                                 float* fhat, qbw_stream stream);

/* The same with another interpolation R (Section 3.5): interp is 0
 * (multilinear), QBW_INTERP_NEAREST or QBW_INTERP_CUBIC.  Cubic: along each
 * axis, at coarse position t = (2x - (k-1)) / (2k) clamped to [0, n-1],
 * i = floor(t), s = t - i, the taps F[i-1..i+2] (indices clamped to the
 * grid) weighted (2s^2-s^3-s)/2, (3s^3-5s^2+2)/2, (4s^2-3s^3+s)/2,
 * (s^3-s^2)/2, in float64; axes nested, last axis innermost; rounded once
 * to float32.  Errors: QBW_E_INVAL for another interp value. */
qbw_status qbw_upscale_potential_interp(qbw_ctx* ctx, const qbw_grid* grid, uint32_t interp,
                                        const double* ftil, float* fhat, qbw_stream stream);

/* Tiling of the single-pair calls (qbw_bounds*, qbw_ctransform): targets per
 * lane R come from the environment variable QBW_TILE_R if it is set to one of
 * 32, 16, 8, 4, 2, 1 dividing N, else from qbw_autotune_ctransform's result for
 * the grid, else the largest of 32, 16, 8, 4, 2 dividing N (1 otherwise).
 * Results do not depend on R. */

/* Lazy c-transform (Section 4, eq. of the lazy c-transform):
 * dst[j] = min_i RN32(RN32(|x_i - x_j|^p) - src[i]) over all N^d pixels,
 * float32, exact min; argmin (device int32, may be NULL) = the lowest flat
 * index attaining it.  src, dst: device float32, each exactly N^d elements in
 * C order (the library cannot see a buffer's size: a shorter one is read or
 * written past its end); argmin likewise N^d int32.  grid->k is ignored. */
qbw_status qbw_ctransform(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst,
                          int32_t* argmin, qbw_stream stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it): the
 * c-transform of qbw_ctransform, the same values and arg-mins bit for bit,
 * with every intermediate buffer (job record, work-item table, counters,
 * winning splits, partial minima) in a static device array of 64 MiB that
 * each GPU the library runs on holds until the process ends.  The call
 * allocates nothing: no hipMalloc, hipHostMalloc or hipFree, and the context's
 * own workspaces are not touched.  The caller still passes src, dst and
 * argmin (N^d elements each, as in qbw_ctransform).  The source splits are
 * reduced until the buffers fit; a grid that does not fit at one split (about
 * 8.3 million pixels and up) is rejected with QBW_E_INVAL and a message.
 * All calls on one GPU share its array and leave their contents in it: calls
 * that overlap on one GPU (other streams or threads) race; calls on one
 * stream are ordered.  Synchronises `stream` before returning. */
qbw_status qbw_ctransform_noalloc(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst,
                                  int32_t* argmin, qbw_stream stream);

/* The same c-transform for p = 2 evaluated separably: d nested 1-D
 * c-transforms, last axis first (pass 1 subtracts src, later passes add the
 * previous result), each candidate rounded to float32 once per axis; argmin
 * (may be NULL) = the passes' lowest indices composed.  grid->p must be 2
 * (QBW_E_GRID otherwise); src, dst, argmin hold N^d elements each, as in
 * qbw_ctransform. */
qbw_status qbw_ctransform_separable(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst,
                                    int32_t* argmin, qbw_stream stream);

/* The lazy c-transform of qbw_ctransform (Section 4, eq. of the lazy
 * c-transform) for p = 2, bit for bit (values and arg-mins), evaluated
 * separably: the exact minimum of |x - y|^2 - src
 * over the sources is a sum of per-axis minima, taken in float64 (d passes,
 * last axis first); rounding to float32 is monotone, so dst = RN32 of that
 * minimum wherever the float64 error bound cannot straddle a rounding
 * boundary, and the arg-min is the best source wherever every other source
 * rounds higher.  The other targets are evaluated by brute force.
 * n_fallback (host int32, may be NULL) receives their number.  grid->p
 * must be 2 (QBW_E_GRID otherwise); src, dst, argmin as in qbw_ctransform
 * (N^d elements each). */
/* (Each stage gives a lane 16, 8, 4 or 2 targets along its axis, the most
 * that still leave a launch about four waves per SIMD; 16 only without
 * arg-mins and for N <= 2048.  The environment variable QBW_XS_T = 2, 4, 8
 * or 16 overrides the choice within those limits, for tests.) */
qbw_status qbw_ctransform_exact(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst,
                                int32_t* argmin, int32_t* n_fallback, qbw_stream stream);

/* IPF of Algorithm 4 on the uniformly upscaled coupling: from b_s = 1,
 * repeat a_s = a / (pi^ b_s), b_s = b / (pi^T a_s) until the L1 marginal
 * error < opts->xi or opts->max_ipf_iter iterations (0/0 := 0).  a_s, b_s:
 * device float64 (N^d) outputs.  *iters, *residual: host. */
qbw_status qbw_ipf(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                   const qbw_coarse* coarse, const qbw_opts* opts, double* a_s, double* b_s,
                   int32_t* iters, double* residual, qbw_stream stream);

/* <diag(a_s) pi^ diag(b_s), C> summed over the support of pi^ (Section 4):
 * *cost host. */
qbw_status qbw_plan_cost(qbw_ctx* ctx, const qbw_grid* grid, const qbw_coarse* coarse,
                         const double* a_s, const double* b_s, double* cost, qbw_stream stream);

/* Weighted-TV corrections of Algorithm 4 for scalings a_s, b_s:
 * Delta_mu = 2^(1-1/p) <w, |a_s * (pi^ b_s) - a|>^(1/p), Delta_nu likewise,
 * w_i = |x-bar - x_i|^p, x-bar the grid mean.  Values as the paper defines
 * them (no rounding allowance).  *tv_mu, *tv_nu host. */
qbw_status qbw_tv(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                  const qbw_coarse* coarse, const double* a_s, const double* b_s,
                  double* tv_mu, double* tv_nu, qbw_stream stream);

/* Upper bound of Algorithm 4 with a caller-chosen kernel for upscaling the
 * coarse coupling (Section 3.4, eq. of the upscaled coupling tensor and the
 * lemma on normalised kernels; the paper's algorithm takes the uniform one).
 * The upscaled coupling is pi^_ij = pi~_KL kernel[s(i) * m + t(j)] for pixel
 * i in block K and j in block L, m = k^d, where s(i) and t(j) are the
 * C-order flat indices of the pixels' positions inside their blocks
 * (0 .. m-1).  kernel: host, m x m float64, row-major, nonnegative and
 * finite, summing to 1 within 1e-12 (QBW_E_INVAL otherwise); m <= 4096
 * (QBW_E_GRID otherwise).  With a non-uniform kernel the fitting no longer
 * stops after one iteration: it runs on fine vectors, from b_s = 1, until
 * ||a^ - a||_1 + ||b - b^||_1 < opts->xi or opts->max_ipf_iter iterations
 * (0/0 := 0; opts->flags are ignored), then the plan cost over the support
 * and the weighted-TV corrections follow as in qbw_bounds.  out (host): the
 * upper-bound fields, rounded outwards (relative 2^-40 + (m^2 + nnz) 2^-52
 * on the plan cost, absolute 2^-40 <w, a> and <w, b> on the TV sums), the
 * fitting's iterations, residual and warning; lower, lower_S and feas_shift
 * are 0.  a_s, b_s: device float64 (N^d), may be NULL; receive the final
 * scalings.  grad_a, grad_b: device float64 (N^d), may be NULL; if either is
 * given, dupper * d upper / d a and dupper * d upper / d b are added (+=) into
 * the non-NULL ones, through the plan cost and the fitting's iterations with the coarse
 * coupling, the kernel and the iteration count frozen, the TV corrections
 * taken as constants (as qbw_bounds_backward); every iterate is kept, which
 * needs 8 N^d (2 max_ipf_iter + 8) bytes of device memory (QBW_E_NOMEM above
 * 32 GiB).  a, b: device.  Synchronises `stream`.  Errors: QBW_E_GRID,
 * QBW_E_INVAL, QBW_E_HIP, QBW_E_NOMEM. */
qbw_status qbw_upper_kernel(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                            const qbw_coarse* coarse, const double* kernel, const qbw_opts* opts,
                            qbw_result* out, double* a_s, double* b_s, double dupper,
                            double* grad_a, double* grad_b, qbw_stream stream);

/* A kernel for qbw_upper_kernel: weight exp(-|s - t|^2 / (2 sigma^2))
 * between in-block offsets s, t (integer vectors in [k]^d), normalised to
 * total 1; it keeps a pixel's relative position inside its block when the
 * coarse coupling moves the block.  sigma = +inf gives the uniform kernel.
 * out: host, k^d x k^d float64.  Errors: QBW_E_INVAL, QBW_E_GRID
 * (k^d > 4096).  No device work. */
qbw_status qbw_plan_kernel_gaussian(int32_t k, int32_t d, double sigma, double* out);

/* Weighted-cost upper bound (Section 3.2, Algorithm 3; theorem of the
 * weighted-cost upper bound): L_{C-bar}(a~, b~)^(1/p) >= W_p(a, b).  Pools and
 * builds C-bar on the device, copies it to the host (n^d x n^d float64) and
 * solves the coarse problem on it with the host network simplex.  *upper is
 * the bound, rounded outwards by a relative 2^-40 for the float64 sums;
 * *objective (may be NULL) = <pi~, C-bar> of the optimal coupling.  Host
 * outputs.  Errors: as qbw_bounds. */
qbw_status qbw_weighted_cost_upper(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                                   double* upper, double* objective, qbw_stream stream);

/* Min-cost lower bound (Section 3.3): L_{C^min}(a~, b~)^(1/p) <= W_p(a, b),
 * C^min_KL = min over x in X_K, y in Y_L of |x - y|^p (closed form on the grid).
 * The bound is the dual objective of the host simplex's potentials, lowered by
 * their largest violation of f_K + g_L <= C^min_KL (so any rounding keeps it
 * valid) and by a relative 2^-40; clipped at 0.  Host outputs. */
qbw_status qbw_min_cost_lower(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                              double* lower, double* objective, qbw_stream stream);

/* ---- batched path: many pairs of uneven sizes in one persistent launch --- */

typedef struct qbw_job {
  qbw_grid grid;
  const double* a; /* device */
  const double* b; /* device */
  double* grad_a;  /* device, may be NULL (no backward for this job) */
  double* grad_b;  /* device, may be NULL */
} qbw_job;

#define QBW_BATCH_BACKWARD 1u /* qbw_batch_run also runs the backward pass */
#define QBW_BATCH_GRAPH 2u    /* capture the device work in a hipGraph, replay it */
#define QBW_BATCH_AUTOTUNE 4u /* time c-transform tilings at creation, keep the fastest */

/* Build a batch: validates every job, pools the measures, solves the coarse
 * problems (host threads) unless `coarse` (array of njobs, host) is given,
 * uploads the coarse solutions, plans the persistent work queues and (flag)
 * autotunes and captures a graph.  The job buffers must stay valid for the
 * batch's life.  Errors as qbw_bounds. */
qbw_status qbw_batch_create(qbw_ctx* ctx, const qbw_job* jobs, int32_t njobs,
                            const qbw_coarse* coarse, const qbw_opts* opts, uint32_t batch_flags,
                            qbw_batch** out, qbw_stream stream);
/* One forward (+ backward with QBW_BATCH_BACKWARD) pass over every job.
 * dlower, dupper: host arrays of njobs upstream gradients (used only with
 * QBW_BATCH_BACKWARD; NULL means 1).  Asynchronous. */
qbw_status qbw_batch_run(qbw_batch* batch, const double* dlower, const double* dupper,
                         qbw_stream stream);
/* Copy the last run's results (host, njobs entries); synchronises. */
qbw_status qbw_batch_results(qbw_batch* batch, qbw_result* out, qbw_stream stream);
/* Tile shape chosen for a job: targets per lane and source splits. */
qbw_status qbw_batch_tiling(const qbw_batch* batch, int32_t job, int32_t* targets_per_lane,
                            int32_t* splits);
void qbw_batch_destroy(qbw_batch* batch);

/* Kernel timing for measurement: while enabled, eager (non-graph) runs record
 * a pair of hipEvents on the run's stream around every c-transform launch
 * (the all-pairs kernel, and each stage of the exact separable one).
 * qbw_batch_ctransform_time synchronises on them and returns the mean launch
 * duration (ms) and the number of launches recorded since the last call,
 * then forgets them.  Graph runs record nothing.  Outputs host. */
qbw_status qbw_batch_set_timing(qbw_batch* batch, int32_t enable);
qbw_status qbw_batch_ctransform_time(qbw_batch* batch, double* mean_ms, int32_t* launches);
/* Candidate evaluations (source, target) per timed c-transform launch, over
 * one phase's launches: an all-pairs launch evaluates (N^d)^2 per job, an
 * exact separable stage N^d x N per job (d stages per job).  Divided by the
 * mean launch time it gives evaluations per second. */
qbw_status qbw_batch_ctransform_pairs(const qbw_batch* batch, double* pairs);

/* Convenience: create, run the forward pass once, fetch results, destroy. */
qbw_status qbw_bounds_batched(qbw_ctx* ctx, const qbw_job* jobs, int32_t njobs,
                              const qbw_opts* opts, qbw_result* out, qbw_stream stream);

/* ---- autotuner --------------------------------------------------------- */

/* Time the c-transform tilings for `grid` (targets per lane x source splits)
 * on the device and remember the fastest in the context and in the on-disk
 * cache (path from env QBW_TUNE_CACHE, default ~/.cache/qbw_tune.txt).
 * Outputs host. */
qbw_status qbw_autotune_ctransform(qbw_ctx* ctx, const qbw_grid* grid, int32_t* targets_per_lane,
                                   int32_t* splits, double* best_ms, qbw_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* QBW_H */
