// Internal declarations shared by the host orchestration and the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qbw.h"

namespace qbw {

// ---------------------------------------------------------------- host side

struct CoarseProblem {
  int Q;
  const double* mu;    // host, Q
  const double* nu;    // host, Q
  const double* cost;  // host, Q x Q row-major
  bool integer_cost;   // p = 2: C~ is an integer matrix
};

struct CoarseSolution {
  std::vector<int> rows, cols;
  std::vector<double> vals, f, g;
  double objective = 0;
  int64_t pivots = 0;
  int rounds = 0;          // pricing rounds of a multiscale solve (candidates, then checks of every pair)
};

int coarse_solve(const CoarseProblem& P, CoarseSolution* out);
// The same optimum from a multiscale start: P's blocks form an n^d grid (C
// order); its half-resolution problem is solved first and its support's
// children are priced first.  Below kMultiscaleMinQ blocks, or for odd n,
// the plain solve.
constexpr int kMultiscaleMinQ = 256;
int coarse_solve_multiscale(const CoarseProblem& P, int n, int d, int p, CoarseSolution* out);
void centre_cost(const qbw_grid& g, double* out);  // C~, host
void set_error(const char* fmt, ...);

// ---------------------------------------------------------------- device job

// Layout of the per-job result block (doubles) written by the finalize kernel.
enum ResultSlot {
  RS_LOWER = 0, RS_UPPER, RS_LOWER_S, RS_SHIFT, RS_UPPER_COST, RS_TV_MU, RS_TV_NU,
  RS_IPF_RESID, RS_COARSE_OBJ, RS_IPF_ITERS, RS_WARN,
  RS_S32, RS_PCOST_RAW, RS_MAX_FHAT, RS_MAX_G, RS_MAX_F, RS_TVSUM_MU, RS_TVSUM_NU,
  RS_MW_MU, RS_MW_NU, RS_TV_RAW_MU, RS_TV_RAW_NU,
  RS_COUNT = 24
};

// Lanes that reduce one coarse block in the pooling and moment kernels: the
// smallest power of two >= min(m, 64), m = pixels per block.
constexpr int reduce_group(int m) {
  int g = 1;
  while (g < m && g < 64) g <<= 1;
  return g;
}
constexpr int kChunk = 1024;       // pixels per work-group in the O(P) kernels
constexpr int kRedSlotsLB = 5;     // per chunk: sum f*mu, sum g*nu, max|fhat|, max|g|, max|f|
constexpr int kRedSlotsTV = 4;     // per chunk: sum w|mu^-mu|, sum w|nu-nu^|, sum w mu, sum w nu

// Everything a kernel needs to know about one job.  Plain data; pointers are
// device memory.  The host builds an array of these and uploads it.
struct DevJob {
  int d, N, k, p;
  int n, P, Q, rows;        // n = N/k, P = N^d, Q = n^d, rows = N^(d-1)
  int R, S;                 // c-transform: targets per lane, source splits
  int chunks;               // ceil(P / kChunk)
  int nnz;                  // coarse coupling entries
  int max_iter;             // IPF cap
  int want_argmin;
  int interp;               // 0 multilinear, 1 nearest, 2 cubic
  double xi;
  double coarse_obj;
  const double* mu;         // fine measures
  const double* nu;
  double* mu_t;             // pooled measures (Q)
  double* nu_t;
  const double* ftil;       // coarse potential (Q)
  float* fhat;              // upscaled potential (P)
  float* g;                 // first c-transform (P)
  float* f;                 // second c-transform (P)
  float* part;              // partial minima (S x P)
  int* win;                 // winning split per target (P)
  int* arg_g;               // arg-mins (P) or null
  int* arg_f;
  // coarse coupling: entry list (sorted by row) and CSR / CSC views
  const int* e_row;
  const int* e_col;
  const double* e_val;
  const int* csr_ptr;       // Q+1, entries of row K are [csr_ptr[K], csr_ptr[K+1]) of the list
  const int* csc_ptr;       // Q+1
  const int* csc_idx;       // nnz: entry ids sorted by column
  double* ipf_u;            // (max_iter + 2) x Q: u^t (t = 1..T+1)
  double* ipf_v;            // (max_iter + 1) x Q: v^t (t = 1..T)
  double* a_s;              // fine IPF scalings (P)
  double* b_s;
  double* red_lb;           // chunks x kRedSlotsLB
  double* red_tv;           // chunks x kRedSlotsTV
  double* red_pc;           // nnz: per-entry sum of a_s b_s c
  double* red_pm;           // nnz (p = 2): per-entry bound on the absolute values of the moment form's terms
  int row_max, col_max;     // longest row and column of the coarse coupling (entries)
  double* result;           // RS_COUNT doubles
  int* flags;               // bit 0: negative entry, bit 1: NaN (pool kernel)
  // backward
  double* grad_a;
  double* grad_b;
  double* gbar_mu;          // Q: d P / d mu~ (coarse adjoint)
  double* gbar_nu;
  double* coef;             // nnz: d P / d S_e coefficient
  double* gquad;            // Q x 2 x 5: per block and side, h(x) = A |z|^2 + B.z + C, z = x - centre
  double* part1;            // p = 1 partial sums: nnz x ceil(k^d / 64) (plan cost), then
                            // nnz x ceil(k^d / 64) x 64 (upper-bound gradient, one side at a time)
  // per-block moments about the block centre, 5 doubles per block:
  // (sum m, sum m delta_0, sum m delta_1, sum m delta_2, sum m |delta|^2)
  double* mom_mu;           // of mu
  double* mom_nu;           // of nu
  double* mom_as;           // of the IPF scalings a_s
  double* mom_bs;           // of b_s
  // separable c-transform (p = 2): two float32 ping-pong buffers and d arg-min planes
  int sep;
  int sep_R;                // 0: k_ct1d (one wave per line chunk, arg-mins); 4, 8, 16: k_ct1d_fast<R>
  int p1_nt;                // p = 1 plan cost / gradient: 0 direct kernels, 64 or 256 distance-table kernels
  float* sep_tmp;           // 2 x P
  const float* sqrt_tab;    // p = 1 c-transform table fill: RN32(sqrt(n)) for n < kSqrtTab, or null
  int xs;                   // p = 2 c-transforms by exact separable minima (certified, re-evaluated where not)
  int xs_T;                 // targets per lane of its stages (8, 4 or 2)
  int xs_xt;                // 2D, no arg-mins, 8 or 16 targets per lane: axis 0 first (1: xs_item_xt,
                            // every source; 2: xs_item_win, argmin windows)
  double* xs_v;             // 2 x (2 P): per stage buffer, best value then runner-up value
  int* xs_i;                // 2 x P: per stage buffer, flat source index of the best value
  int* sep_arg;             // d x P or null
};

struct CtItem { int job, tile, split, pad; };

// One pair's upper bound with a caller-chosen kernel for upscaling the coarse
// coupling (Section 3.4): pi^_ij = pi~_KL Kst[s(i) m + t(j)], s and t the
// in-block offsets (C order), m = k^d.  The fitting no longer stays on coarse
// vectors: a, b, mu^, nu^ are fine.  Passed to the kernels by value.
struct KubJob {
  int d, N, k, p, n, P, Q, m, nnz, max_iter;
  int nt;                   // offsets per work-group (64 or 256)
  int cpb;                  // work-groups per block: ceil(m / nt)
  int chunks;               // ceil(P / kChunk)
  double xi;
  double coarse_obj;
  const double* mu;         // fine measures
  const double* nu;
  const int* e_row;         // coarse coupling, entries sorted by row
  const int* e_col;
  const double* e_val;
  const int* csr_ptr;       // Q+1
  const int* csc_ptr;       // Q+1
  const int* csc_idx;       // nnz: entry ids by column
  const double* Kst;        // m x m, [s][t]
  const double* Kts;        // m x m, [t][s] (the transpose, for coalesced reads)
  double* a0;               // a^t for even t
  double* a1;               // a^t for odd t
  double* b;                // b^t
  double* muh;              // mu^ = a^t (pi^ b^t)
  double* nuh;              // nu^ = b^t (pi^T a^t)
  double* part_mu;          // Q x cpb: sums of |mu^ - mu|
  double* part_nu;          // Q x cpb: sums of |nu - nu^|
  double* pc_part;          // nnz x cpb: plan-cost partials
  double* red_tv;           // chunks x kRedSlotsTV
  int* state;               // [0]: fitting stopped
  double* result;           // RS_COUNT
  // gradient (null without): checkpointed iterates and adjoints
  double* hist_u;           // (max_iter + 2) x P: row t holds u^t = pi^ b^(t-1)
  double* hist_v;           // (max_iter + 1) x P: row t holds v^t = pi^T a^t
  double* g_mu;             // d P / d mu (P = plan cost), accumulated over the iterations
  double* g_nu;
  double* g_abar;           // d P / d a^T through the plan cost
  double* g_ubar;           // adjoint of u^t
  double* g_vbar;           // adjoint of v^t
};

int launch_kub_row(const KubJob& J, int t, void* stream);
int launch_kub_col(const KubJob& J, int t, void* stream);
int launch_kub_check(const KubJob& J, int t, void* stream);
int launch_kub_plancost(const KubJob& J, void* stream);
int launch_kub_tv(const KubJob& J, void* stream);
int launch_kub_finalize(const KubJob& J, void* stream);
int launch_kub_backward(const KubJob& J, int T, double dupper, double* grad_a, double* grad_b, void* stream);

// Kernel launchers (kernels.hip).  All enqueue on `stream`.
struct Launch {
  const DevJob* jobs;  // device array
  int njobs;
  const int* off;      // device prefix table for the launch's item kind
  int total;           // total items
};

// SumPool of both measures with their block moments and the input checks
// (k_moments, which = 2), over the plan's moment items.
// SumPool with the block moments and input checks; upscale: also f^ for the
// jobs with k <= 64 (launch_upscale with skip_small does the others).
int launch_pool(const DevJob* jobs, int njobs, const int* off_mom, int total_mom, int upscale, void* stream);
int launch_upscale(const DevJob* jobs, int njobs, const int* off, int total, int skip_small, void* stream);
constexpr int kQueues = 8;  // XCDs: the planner groups c-transform items per XCD
// Waves of k_ctransform resident per compute unit (0 if the runtime cannot say).
int ctransform_waves_per_cu();
// Entries of the context's integer square-root table: RN32(sqrt(n)) for
// 0 <= n < kSqrtTab, filled once with the kernels' own correctly rounded
// square root.  p = 1 jobs with d (N-1)^2 < kSqrtTab read their table rows
// from it instead of taking square roots.
constexpr int kSqrtTab = 65536;
int launch_sqrt_table(float* t, int n, void* stream);
// Exact separable c-transform (p = 2): squares table of kXsSquares doubles
// ((i - 2904)^2); stage k (0 .. d-1) over the items of table `off` (jobs with
// d > k), then the re-evaluation of the targets the last stage could not
// certify.  `list` holds 2 ints per queued target (capacity: the jobs' total
// pixel count) and `count` their number (zero before stage 0).
constexpr int kXsSquares = 2 * 2904 + 1;
int launch_xs_squares(double* t, void* stream);
// T: the plan's targets per lane (every job's xs_T; for xt 2 the item's
// targets, xs_T times the group factor); argmin: the plan wants arg-mins;
// waves: waves per work-group splitting an item's sources (1, 2, 4; 1 with
// arg-mins; up to 8 for xt 2).
// xt: 0 axis d-1 first (xs_item), 1 two-dimensional axis 0 first over every
// source (xs_item_xt), 2 the same by argmin windows (xs_item_win)
int launch_xs_stage(const DevJob* jobs, int njobs, const int* off, int total, int phase, int k, const double* sqt,
                    int* list, int* count, int T, int argmin, int waves, int xt, void* stream);
int launch_xs_fallback(const DevJob* jobs, const int* list, const int* count, int phase, int grid, void* stream);
int launch_ctransform(const DevJob* jobs, const CtItem* items, int n_items, int* counter, int phase, int grid,
                      void* stream);
int launch_merge(const DevJob* jobs, int njobs, const int* off, int total, int phase, void* stream);
int launch_argmin(const DevJob* jobs, int njobs, const int* off, int total, int phase, void* stream);
// Coarse kernels (one work-group per job) stage the coupling and nvec
// per-block vectors in LDS when the job's bytes fit the launch's allocation.
constexpr size_t kCoarseLdsMax = 160 * 1024;
constexpr size_t coarse_lds_need(int Q, int nnz, int nvec) {
  return 8 * ((size_t)nvec * Q + (size_t)nnz) + 4 * (2 * (size_t)(Q + 1) + 3 * (size_t)nnz) + 16;
}
// flags: bit 0 p = 2 plan-cost entries, bit 1 also the reverse pass (the
// coarse part of the backward; scratch holds 4 x stride doubles per job for
// jobs whose coupling is not staged in LDS).
int launch_ipf(const DevJob* jobs, int njobs, size_t lds_bytes, int flags, double* scratch, int stride,
               void* stream);
int launch_scalings(const DevJob* jobs, int njobs, const int* off, int total, void* stream);
int launch_tv_partial(const DevJob* jobs, int njobs, const int* off, int total, void* stream);
// p = 1 plan cost and upper-bound gradient on blocks of m = k^d pixels: the
// work-group size of the distance-table kernels (every pair distance of a
// block pair is one of (2k-1)^d values, tabulated in LDS), or 0 where the
// direct kernels are used (m <= 32: several entries per wave; table larger
// than 4096 entries or m > 1024).
constexpr int p1_table_nt(int k, int d) {
  return ((d == 2 ? k * k : k * k * k) <= 32 || (d == 2 ? k * k : k * k * k) > 1024 ||
          (d == 2 ? (2 * k - 1) * (2 * k - 1) : (2 * k - 1) * (2 * k - 1) * (2 * k - 1)) > 4096)
             ? 0
             : ((d == 2 ? k * k : k * k * k) <= 64 ? 64 : 256);
}
// Item tables of the three p = 1 kernel kinds: [0] direct, [1] table with 64
// threads, [2] table with 256 threads (device prefix tables and totals).
struct P1Items {
  const int* off[3];
  int total[3];
};
int launch_plancost(const DevJob* jobs, int njobs, const P1Items& items, void* stream);
int launch_finalize(const DevJob* jobs, int njobs, void* stream);
int launch_moments(const DevJob* jobs, int njobs, const int* off, int total, int which,
                   void* stream);
int launch_plancost2(const DevJob* jobs, int njobs, const int* off, int total, void* stream);
int launch_cbar2(const DevJob* jobs, int njobs, const int* off, int total, double* const* outs,
                 void* stream);
int launch_lb_grad(const DevJob* jobs, int njobs, const int* off, int total, const double* dl,
                   void* stream);
// The coarse reverse pass of the fitting; for p = 2 jobs it also writes the
// per-block quadratics of the direct gradient term (block moments of mu, nu
// must be current).
int launch_ub_coarse_bwd2(const DevJob* jobs, int njobs, double* scratch, int stride, size_t lds_bytes,
                          int skip_p2, void* stream);
int launch_ub_grad(const DevJob* jobs, int njobs, const P1Items& items, const double* du, int side,
                   void* stream);
int launch_fhat_grad2(const DevJob* jobs, int njobs, const int* off, int total, const double* dl,
                      double* const* outs, void* stream);
// The forward pixel sweep; it also zeroes clear[0 .. nclear) (the c-transform
// counters, for the next step).
int launch_fwd_pixels(const DevJob* jobs, int njobs, const int* off, int total, int* clear, int nclear,
                      void* stream);
int launch_pc1_sum(const DevJob* jobs, int njobs, void* stream);
int launch_ub_grad_sum(const DevJob* jobs, int njobs, const int* off, int total, const double* du, int side,
                       void* stream);
int launch_grad2(const DevJob* jobs, int njobs, const int* off, int total, const double* dl, const double* du,
                 void* stream);
int launch_tv_prep(const DevJob* jobs, int njobs, void* stream);
int launch_ct1d(const DevJob* jobs, int njobs, const int* off, int total, int phase, int pass,
                void* stream);
// Targets per lane of the register-window 1-D pass for lines of length N
// (power of two, 32 <= N <= 1024), 0 where it does not apply.
constexpr int ct1d_fast_R(int N) {
  return (N >= 128 && N <= 1024 && (N & (N - 1)) == 0) ? 16 : N == 64 ? 8 : N == 32 ? 4 : 0;
}
int launch_ct1d_fast(const DevJob* jobs, int njobs, const int* off, int total, int phase, int pass, int R,
                     void* stream);
int launch_sep_argmin(const DevJob* jobs, int njobs, const int* off, int total, int phase,
                      void* stream);
int launch_reset_counter(int* counter, int n, void* stream);

// Static device scratch of the allocation-free c-transform (bytes per GPU) and
// its device address on `device`, which must be the current device; the
// address is looked up once per device and kept.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxScratchDevices = 64;
int scratch_address(int device, void** out);
int launch_noalloc_setup(const DevJob& D, DevJob* dj, int* off, CtItem* items, int n_items, int tiles, int* ints,
                         int n_ints, void* stream);

}  // namespace qbw
