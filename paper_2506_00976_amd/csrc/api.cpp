// Host orchestration of libqbw: validation, workspace planning, the C ABI.
//
// One "plan" describes a set of jobs (one pair, or a batch of pairs of uneven
// sizes): it lays out every per-job device buffer in one arena, uploads the
// job table, the coarse couplings (entry list + CSR/CSC views) and the work
// tables, and enqueues the forward and backward kernel sequences.  The
// single-pair calls and the batched calls share it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <numeric>
#include <queue>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "qbw_internal.h"

namespace qbw {

static thread_local std::string g_err = "no error";

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

#define HIPCHK(x)                                                         \
  do {                                                                    \
    hipError_t e_ = (x);                                                  \
    if (e_ != hipSuccess) {                                               \
      set_error("%s failed: %s", #x, hipGetErrorString(e_));              \
      return QBW_E_HIP;                                                   \
    }                                                                     \
  } while (0)
#define CHK(x)                        \
  do {                                \
    int r_ = (x);                     \
    if (r_ != QBW_OK) return (qbw_status)r_; \
  } while (0)

static inline hipStream_t S(qbw_stream s) { return (hipStream_t)s; }

static int ipow(int b, int e) {
  int r = 1;
  while (e--) r *= b;
  return r;
}

static int check_grid(const qbw_grid* g) {
  if (!g) { set_error("grid is NULL"); return QBW_E_INVAL; }
  if (g->d != 2 && g->d != 3) { set_error("d must be 2 or 3 (got %d)", g->d); return QBW_E_GRID; }
  if (g->p != 1 && g->p != 2) { set_error("p must be 1 or 2 (got %d)", g->p); return QBW_E_GRID; }
  if (g->N < 1 || g->k < 1 || g->k > g->N || g->N % g->k) {
    set_error("need 1 <= k <= N and N %% k == 0 (N=%d k=%d)", g->N, g->k);
    return QBW_E_GRID;
  }
  const double P = std::pow((double)g->N, g->d);
  if (P > (double)(1 << 26)) { set_error("grid too large (N^d = %.0f > 2^26)", P); return QBW_E_GRID; }
  if (g->d * (double)(g->N - 1) * (g->N - 1) >= 16777216.0) {
    set_error("squared distances must stay below 2^24 (float32-exact)");
    return QBW_E_GRID;
  }
  return QBW_OK;
}

void centre_cost(const qbw_grid& g, double* out) {
  const int n = g.N / g.k;
  const int Q = ipow(n, g.d);
  for (int K = 0; K < Q; ++K) {
    int kc[3] = {0, 0, 0}, t = K;
    for (int a = g.d - 1; a >= 0; --a) { kc[a] = t % n; t /= n; }
    for (int L = 0; L < Q; ++L) {
      int lc[3] = {0, 0, 0}, s = L;
      for (int a = g.d - 1; a >= 0; --a) { lc[a] = s % n; s /= n; }
      long long d2 = 0;
      for (int a = 0; a < g.d; ++a) {
        long long e = (long long)g.k * (kc[a] - lc[a]);
        d2 += e * e;
      }
      out[(size_t)K * Q + L] = g.p == 2 ? (double)d2 : std::sqrt((double)d2);
    }
  }
}

// ------------------------------------------------------------------ device arena

struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  Arena(Arena&& o) noexcept : base(o.base), cap(o.cap) { o.base = nullptr; o.cap = 0; }
  Arena& operator=(Arena&& o) noexcept {
    if (this != &o) {
      if (base) (void)hipFree(base);
      base = o.base; cap = o.cap;
      o.base = nullptr; o.cap = 0;
    }
    return *this;
  }
  ~Arena() { if (base) (void)hipFree(base); }
  int reserve(size_t bytes) {
    if (bytes <= cap) return QBW_OK;
    if (base) { HIPCHK(hipFree(base)); base = nullptr; cap = 0; }
    size_t want = std::max(bytes, cap * 3 / 2);
    if (hipMalloc(&base, want) != hipSuccess) {
      base = nullptr;
      if (hipMalloc(&base, bytes) != hipSuccess) {
        base = nullptr;
        set_error("device allocation of %zu bytes failed", bytes);
        return QBW_E_NOMEM;
      }
      want = bytes;
    }
    cap = want;
    return QBW_OK;
  }
};

// Byte layout builder: records (offset) for each named buffer.
struct Layout {
  size_t size = 0;
  size_t add(size_t bytes) {
    size_t off = (size + 255) & ~size_t(255);
    size = off + bytes;
    return off;
  }
};

// ------------------------------------------------------------------ tuning

struct Tiling { int R, S; };

static int default_R(int N) {
  for (int r : {32, 16, 8, 4, 2})
    if (N % r == 0) return r;
  return 1;
}

// ------------------------------------------------------------------ context

}  // namespace qbw

struct qbw_ctx {
  int device = 0;
  int num_cu = 256;
  qbw::Arena work;      // scratch for single-pair calls that keep nothing
  std::map<std::tuple<int, int, int>, qbw::Tiling> tuned;  // (d, N, p) -> tiling
  int target_waves = 4096;
  float* sqrt_tab = nullptr;  // kSqrtTab entries, filled at creation, read-only after
  double* xs_sq = nullptr;    // kXsSquares entries (exact separable c-transform), likewise
  char* scratch = nullptr;    // this device's static scratch (kScratchBytes), shared by all contexts on it
  // pinned staging for the planner's one host-to-device copy; `staged` marks
  // a copy in flight (completion recorded in `staged_ev`)
  char* stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t staged_ev = nullptr;
  bool staged = false;
  // Device arenas of freed saved-for-backward records, reused by the next
  // ones (a forward + backward per call would otherwise allocate and free
  // each time), and the live records, detached when the context goes first.
  // Saved records may be freed from another thread: both lists take `mu`.
  std::mutex mu;
  std::vector<qbw::Arena> spare;
  std::set<qbw_saved*> live;
  ~qbw_ctx();
};

namespace qbw {

struct CoarseHost {
  int Q = 0, nnz = 0;
  std::vector<int> rows, cols;  // sorted by row
  std::vector<double> vals, f;
  std::vector<int> csr_ptr, csc_ptr, csc_idx;
  double obj = 0;
};

static int make_coarse(const qbw_grid& g, const qbw_coarse* c, CoarseHost* out) {
  const int n = g.N / g.k, Q = ipow(n, g.d);
  if (!c || !c->rows || !c->cols || !c->vals || !c->f) { set_error("coarse solution has NULL arrays"); return QBW_E_INVAL; }
  if (c->Q != Q) { set_error("coarse solution has Q=%d, grid needs %d", c->Q, Q); return QBW_E_INVAL; }
  if (c->nnz < 1 || c->nnz > Q * Q) { set_error("coarse coupling has %d entries", c->nnz); return QBW_E_INVAL; }
  out->Q = Q;
  out->nnz = c->nnz;
  std::vector<int> ord(c->nnz);
  std::iota(ord.begin(), ord.end(), 0);
  for (int e = 0; e < c->nnz; ++e) {
    if (c->rows[e] < 0 || c->rows[e] >= Q || c->cols[e] < 0 || c->cols[e] >= Q) {
      set_error("coarse coupling entry %d has an index out of range", e);
      return QBW_E_INVAL;
    }
    if (!(c->vals[e] >= 0.0) || !std::isfinite(c->vals[e])) {
      set_error("coarse coupling entry %d is negative or not finite", e);
      return QBW_E_INVAL;
    }
  }
  for (int K = 0; K < Q; ++K)
    if (!std::isfinite(c->f[K])) { set_error("coarse potential is not finite"); return QBW_E_INVAL; }
  const auto by_row = [&](int a, int b) { return c->rows[a] < c->rows[b]; };
  if (!std::is_sorted(ord.begin(), ord.end(), by_row)) std::stable_sort(ord.begin(), ord.end(), by_row);
  out->rows.resize(c->nnz); out->cols.resize(c->nnz); out->vals.resize(c->nnz);
  double obj = 0;
  std::vector<double> Ct;
  for (int q = 0; q < c->nnz; ++q) {
    out->rows[q] = c->rows[ord[q]];
    out->cols[q] = c->cols[ord[q]];
    out->vals[q] = c->vals[ord[q]];
  }
  out->csr_ptr.assign(Q + 1, 0);
  out->csc_ptr.assign(Q + 1, 0);
  for (int q = 0; q < c->nnz; ++q) { out->csr_ptr[out->rows[q] + 1]++; out->csc_ptr[out->cols[q] + 1]++; }
  for (int K = 0; K < Q; ++K) { out->csr_ptr[K + 1] += out->csr_ptr[K]; out->csc_ptr[K + 1] += out->csc_ptr[K]; }
  out->csc_idx.resize(c->nnz);
  std::vector<int> fill(out->csc_ptr.begin(), out->csc_ptr.end() - 1);
  for (int q = 0; q < c->nnz; ++q) out->csc_idx[fill[out->cols[q]]++] = q;
  out->f.assign(c->f, c->f + Q);
  // objective <pi~, C~> (reported only)
  const int n_ = n;
  for (int q = 0; q < c->nnz; ++q) {
    int K = out->rows[q], L = out->cols[q];
    long long d2 = 0;
    int tk = K, tl = L;
    for (int a = 0; a < g.d; ++a) {
      long long e = (long long)g.k * ((tk % n_) - (tl % n_));
      d2 += e * e;
      tk /= n_; tl /= n_;
    }
    obj += out->vals[q] * (g.p == 2 ? (double)d2 : std::sqrt((double)d2));
  }
  out->obj = obj;
  return QBW_OK;
}

// A job as given to the planner.
struct JobIn {
  qbw_grid g;
  const double* a;
  const double* b;
  double* ga;
  double* gb;
  const CoarseHost* coarse;  // may be null (stage-only plans)
  Tiling tiling;
};

enum PlanMode : unsigned {
  PM_FORWARD = 1, PM_ARGMIN = 2, PM_BACKWARD = 4, PM_CBAR = 8, PM_SEP = 16, PM_XS = 32,
};

struct Plan {
  int njobs = 0;
  unsigned mode = 0;
  int max_iter = 50;
  double xi = 1e-12;
  std::vector<DevJob> hj;
  std::vector<JobIn> in;
  Arena own;         // used when the plan owns its memory
  char* base = nullptr;
  DevJob* djobs = nullptr;
  int *off_chunk = nullptr, *off_pool = nullptr, *off_entry = nullptr, *off_block = nullptr,
      *off_cbar = nullptr, *off_mom = nullptr, *off_pc1 = nullptr, *off_pc2 = nullptr,
      *off_sep = nullptr, *off_ubg = nullptr;
  int tot_chunk = 0, tot_pool = 0, tot_entry = 0, tot_block = 0, tot_cbar = 0, tot_mom = 0,
      tot_pc1 = 0, tot_pc2 = 0, tot_sep = 0, max_sep_d = 0, tot_ubg = 0;
  bool has_p1 = false, has_p2 = false;  // grid cost exponents present
  unsigned sep_kinds = 0;  // separable passes present: bit 0 k_ct1d, bits 4, 8, 16 k_ct1d_fast<R>
  // exact separable c-transforms: stage items of all such jobs and of the 3D
  // ones (third stage), the brute-force queue and its length (all pixels)
  int *off_xs = nullptr, *off_xs3 = nullptr;
  int tot_xs = 0, tot_xs3 = 0;
  int* xs_list = nullptr;
  int xs_pixels = 0;
  int xs_T = 8, xs_W = 1;  // targets per lane and waves per work-group of the stages
  int xs_W0 = 1;           // waves per work-group of the first stage
  bool xs_has_xt = false, xs_has_std = false;   // jobs on xs_item_xt (2D, axis 0 first) / on xs_item
  int xs_xt_kind = 2;   // the axis-0-first jobs' kind: 2 argmin windows (xs_item_win), 1 every source
  int xs_wg = 2;        // argmin windows: targets and waves of a work-group, in multiples of xs_T, xs_W
  size_t ipf_lds = 0;      // dynamic LDS of the coarse fitting kernel (jobs that do not fit use global memory)
  size_t bwd_lds = 0;      // the same for the coarse backward kernel
  bool fwd_rev = false;    // a backward pass follows: the forward's coarse kernel runs its p = 2 reverse pass
  const double* xs_sq = nullptr;
  P1Items p1_tab{};        // p = 1 plan-cost / gradient items per kernel kind
  CtItem* items = nullptr;
  int n_items = 0;
  int ct_grid = 1;
  // ints[0], ints[kQueues]: the two phases' tail counters; ints[2 kQueues + 0,
  // 1]: the phases' brute-force queue lengths (all zeroed by the pixel sweep
  // for the next step); then njobs input flags
  int* ints = nullptr;
  int n_ints = 0;
  double* dl = nullptr;  // per-job upstream gradients
  double* du = nullptr;
  double* bwd_scratch = nullptr;
  int max_q = 1;              // row stride of bwd_scratch (per job: 4 x max_q doubles)
  double* results = nullptr;  // njobs x RS_COUNT
  double** cbar_out = nullptr;  // device array of njobs pointers
  double** fhat_grad_out = nullptr;
  std::vector<double> host_results;
  bool timing = false;                                  // event pairs around c-transforms
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  ~Plan() {
    for (auto& e : ev_pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  }
};

// Relative time of one c-transform pair: p = 1 builds a row of correctly
// rounded square roots per source row and target row (R per lane) and reads
// the window from it, measured at 1.1x the p = 2 time on 256-pixel rows, 1.3x
// on 128 and 1.55x on 32-pixel rows; the split sizing balances time, not pairs.
static double pair_weight(const qbw_grid& g) {
  return g.p == 1 ? 1.05 + 16.0 / g.N : 1.0;
}

static int choose_splits(std::vector<JobIn>& in, int target_waves) {
  // Items (tile, split) of one launch should end together: starting from one
  // split per tile, the next split goes to the job whose items take longest
  // (pairs per item times the pair weight) while one round of target_waves
  // resident waves has room for that job's tiles.  Jobs with a given S keep it.
  const int nj = (int)in.size();
  std::vector<int> tiles(nj), rows(nj);
  std::vector<double> work(nj);
  std::priority_queue<std::pair<double, int>> heap;   // (time of one item, job)
  long long used = 0;
  for (int j = 0; j < nj; ++j) {
    JobIn& J = in[j];
    const int P = ipow(J.g.N, J.g.d);
    rows[j] = ipow(J.g.N, J.g.d - 1);
    if (J.tiling.R <= 0) J.tiling.R = default_R(J.g.N);
    tiles[j] = (P + 64 * J.tiling.R - 1) / (64 * J.tiling.R);
    work[j] = (double)P * (double)P * pair_weight(J.g) / tiles[j];   // per tile
    if (J.tiling.S > 0) {
      J.tiling.S = std::min(J.tiling.S, rows[j]);
    } else {
      J.tiling.S = 1;
      heap.push({work[j], j});
    }
    used += (long long)tiles[j] * J.tiling.S;
  }
  while (!heap.empty()) {
    const int j = heap.top().second;
    JobIn& J = in[j];
    if (J.tiling.S >= rows[j] || used + tiles[j] > target_waves) break;   // the longest item stays
    heap.pop();
    ++J.tiling.S;
    used += tiles[j];
    heap.push({work[j] / J.tiling.S, j});
  }
  for (int j = 0; j < nj; ++j) {
    JobIn& J = in[j];
    // splits take whole source rows: with r = ceil(rows / S) rows per split,
    // use no more splits than needed, so no split is longer than r rows
    const int r = (rows[j] + J.tiling.S - 1) / J.tiling.S;
    J.tiling.S = (rows[j] + r - 1) / r;
  }
  return QBW_OK;
}

// c-transform work items of the all-pairs jobs of `in`, laid out for the
// persistent launch (position b < G is work-group b's item); returns G.
static int build_ct_items(const qbw_ctx* ctx, const std::vector<JobIn>& in, unsigned mode,
                          std::vector<CtItem>& items) {
  const int NJ = (int)in.size();
  // c-transform work items, grouped per XCD.  Jobs get a home XCD by
  // longest-processing-time assignment of their pair counts; a lone job (or one
  // too big for a single XCD's share) spreads its target tiles over all XCDs.
  // modelled cost of one item of each job (all of a job's items are alike)
  std::vector<double> job_item_cost(NJ);
  for (int j = 0; j < NJ; ++j) {
    const auto& J = in[j];
    const double rows = std::pow((double)J.g.N, J.g.d - 1);
    job_item_cost[j] = 64.0 * J.tiling.R * (rows / J.tiling.S) * J.g.N * (J.g.p == 1 ? 1.4 : 1.0);
  }
  auto item_cost = [&](const CtItem& w) { return job_item_cost[w.job]; };
  std::vector<std::vector<CtItem>> queues(kQueues);
  {
    std::vector<double> load(kQueues, 0.0);
    std::vector<int> order(NJ);
    std::iota(order.begin(), order.end(), 0);
    auto work = [&](int j) { return std::pow((double)in[j].g.N, 2.0 * in[j].g.d); };
    double total = 0;
    for (int j = 0; j < NJ; ++j) total += work(j);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    for (int j : order) {
      const auto& J = in[j];
      if ((mode & (PM_SEP | PM_XS)) && J.g.p == 2) continue;   // separable jobs use the 1-D passes
      const int P = ipow(J.g.N, J.g.d);
      const int tiles = (P + 64 * J.tiling.R - 1) / (64 * J.tiling.R);
      const bool spread = work(j) > total / kQueues;
      int home = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      for (int s = 0; s < J.tiling.S; ++s)
        for (int t = 0; t < tiles; ++t) {
          CtItem w{j, t, s, 0};
          const int q = spread ? (t % kQueues) : home;
          queues[q].push_back(w);
          load[q] += item_cost(w);
        }
    }
  }
  // Item table: position b < G (the grid) is the item work-group b takes in
  // the static round.  The dispatcher deals work-groups to the XCDs in turn,
  // so positions b = q (mod kQueues) are XCD q's: they get queue q's items
  // (largest first); surplus items of longer queues fill the positions left
  // free by shorter ones, and what exceeds the grid forms the dynamic tail.
  int n_all = 0;
  const auto larger = [&](const CtItem& x, const CtItem& y) { return item_cost(x) > item_cost(y); };
  for (int q = 0; q < kQueues; ++q) {
    // items enter in (split, tile) order, usually already by decreasing cost
    if (!std::is_sorted(queues[q].begin(), queues[q].end(), larger))
      std::stable_sort(queues[q].begin(), queues[q].end(), larger);
    n_all += (int)queues[q].size();
  }
  // persistent grid: one work-group per item, at most 32 per compute unit
  const int G = std::min(n_all, ctx->num_cu * 4 * 8);
  items.assign(n_all, CtItem{});
  std::vector<CtItem> surplus;
  std::vector<int> free_pos;
  for (int q = 0; q < kQueues; ++q) {
    size_t used = 0;
    for (int b = q; b < G; b += kQueues) {
      if (used < queues[q].size()) items[b] = queues[q][used++];
      else free_pos.push_back(b);
    }
    surplus.insert(surplus.end(), queues[q].begin() + used, queues[q].end());
  }
  if (!std::is_sorted(surplus.begin(), surplus.end(), larger))
    std::stable_sort(surplus.begin(), surplus.end(), larger);
  size_t si = 0;
  for (int b : free_pos) items[b] = surplus[si++];
  for (int b = G; b < n_all; ++b) items[b] = surplus[si++];
  return G;
}

// Build the layout, allocate (or reuse) device memory, upload tables.
static int plan_build(qbw_ctx* ctx, Plan& pl, std::vector<JobIn> in, unsigned mode,
                      const qbw_opts& o, bool own_memory, hipStream_t st) {
  pl.in = std::move(in);
  pl.njobs = (int)pl.in.size();
  pl.mode = mode;
  pl.fwd_rev = (mode & PM_BACKWARD) != 0;
  pl.max_iter = o.max_ipf_iter;
  pl.xi = o.xi;
  const int NJ = pl.njobs;
  CHK(choose_splits(pl.in, ctx->target_waves));
  Layout L;
  struct Offs {
    size_t mu_t, nu_t, ftil, fhat, g, f, part, win, arg_g, arg_f, e_row, e_col, e_val, csr, csc,
        csc_idx, ipf_u, ipf_v, a_s, b_s, red_lb, red_tv, red_pc, red_pm, gbar_mu, gbar_nu, coef, gquad, part1, mom_mu, mom_nu,
        mom_as, mom_bs, sep_tmp, sep_arg, xs_v, xs_i;
  };
  std::vector<Offs> offs(NJ);
  const bool ub = true;
  for (int j = 0; j < NJ; ++j) {
    const auto& J = pl.in[j];
    const int N = J.g.N, d = J.g.d, n = N / J.g.k;
    const int P = ipow(N, d), Q = ipow(n, d);
    const int chunks = (P + kChunk - 1) / kChunk;
    const int nnz = J.coarse ? J.coarse->nnz : 1;
    Offs& O = offs[j];
    O.mu_t = L.add(8 * Q);
    O.nu_t = L.add(8 * Q);
    O.fhat = L.add(4 * (size_t)P);
    O.g = L.add(4 * (size_t)P);
    O.f = L.add(4 * (size_t)P);
    O.part = L.add(4 * (size_t)P * J.tiling.S);
    O.win = L.add(4 * (size_t)P);
    O.arg_g = (mode & PM_ARGMIN) ? L.add(4 * (size_t)P) : 0;
    O.arg_f = (mode & PM_ARGMIN) ? L.add(4 * (size_t)P) : 0;
    O.ipf_u = L.add(8 * (size_t)Q * (o.max_ipf_iter + 2));
    O.ipf_v = L.add(8 * (size_t)Q * (o.max_ipf_iter + 2));
    O.a_s = ub ? L.add(8 * (size_t)P) : 0;
    O.b_s = ub ? L.add(8 * (size_t)P) : 0;
    O.red_lb = L.add(8 * (size_t)chunks * kRedSlotsLB);
    O.red_tv = L.add(8 * (size_t)chunks * kRedSlotsTV);
    O.red_pc = L.add(8 * (size_t)nnz);
    O.red_pm = L.add(8 * (size_t)nnz);
    O.gbar_mu = L.add(8 * (size_t)Q);
    O.gbar_nu = L.add(8 * (size_t)Q);
    O.coef = L.add(8 * (size_t)nnz);
    O.gquad = L.add(8 * 10 * (size_t)Q);
    {
      const int mb = ipow(J.g.k, d);
      O.part1 = J.g.p == 1 ? L.add(8 * (size_t)nnz * ((mb + 63) / 64) * 64) : 0;
    }
    O.mom_mu = L.add(8 * 5 * (size_t)Q);
    O.mom_nu = L.add(8 * 5 * (size_t)Q);
    O.mom_as = L.add(8 * 5 * (size_t)Q);
    O.mom_bs = L.add(8 * 5 * (size_t)Q);
    const bool sep = (mode & PM_SEP) && J.g.p == 2;
    O.sep_tmp = sep ? L.add(4 * 2 * (size_t)P) : 0;
    O.sep_arg = (sep && (mode & PM_ARGMIN)) ? L.add(4 * (size_t)d * P) : 0;
    const bool xs = (mode & PM_XS) && J.g.p == 2;
    O.xs_v = xs ? L.add(8 * 4 * (size_t)P) : 0;
    O.xs_i = xs ? L.add(4 * 2 * (size_t)P) : 0;
    if (xs) pl.xs_pixels += P;
  }
  const size_t o_xs_list = pl.xs_pixels ? L.add(8 * (size_t)pl.xs_pixels) : 0;
  constexpr int kTables = 14;
  std::vector<CtItem> items;
  const int G = build_ct_items(ctx, pl.in, mode, items);
  pl.n_items = (int)items.size();
  pl.n_ints = 2 * kQueues + 2 + NJ;
  const size_t o_res = L.add(8 * (size_t)RS_COUNT * NJ);
  size_t maxQ = 1;
  for (auto& J : pl.in) maxQ = std::max<size_t>(maxQ, ipow(J.g.N / J.g.k, J.g.d));
  const size_t o_bwd = L.add(8 * 4 * maxQ * NJ);
  pl.max_q = (int)maxQ;
  // Everything the host supplies sits in one contiguous region [u0, u1),
  // filled in pinned staging memory and copied with a single transfer.
  const size_t u0 = L.add(0);
  const size_t o_jobs = L.add(sizeof(DevJob) * NJ);
  const size_t o_offs = L.add(sizeof(int) * kTables * (NJ + 1));
  const size_t o_items = L.add(sizeof(CtItem) * std::max(1, pl.n_items));
  const size_t o_dl = L.add(8 * NJ), o_du = L.add(8 * NJ);
  const size_t o_ptrs = L.add(sizeof(double*) * 4 * NJ);
  const size_t o_ints = L.add(sizeof(int) * pl.n_ints);   // zero at the start
  for (int j = 0; j < NJ; ++j) {
    const auto& J = pl.in[j];
    const int Q = ipow(J.g.N / J.g.k, J.g.d);
    const int nnz = J.coarse ? J.coarse->nnz : 1;
    Offs& O = offs[j];
    O.ftil = L.add(8 * (size_t)Q);
    O.e_row = L.add(4 * (size_t)nnz);
    O.e_col = L.add(4 * (size_t)nnz);
    O.e_val = L.add(8 * (size_t)nnz);
    O.csr = L.add(4 * (size_t)(Q + 1));
    O.csc = L.add(4 * (size_t)(Q + 1));
    O.csc_idx = L.add(4 * (size_t)nnz);
  }
  const size_t u1 = L.size;

  if (own_memory) {
    CHK(pl.own.reserve(L.size));
    pl.base = pl.own.base;
  } else {
    CHK(ctx->work.reserve(L.size));
    pl.base = ctx->work.base;
  }
  char* B = pl.base;
  // host images of the uploaded region
  pl.hj.resize(NJ);
  std::vector<int> off(kTables * (NJ + 1), 0);
  // exact separable stages: the most targets per lane (fewest loads per
  // candidate) that still give a launch about four waves per SIMD; 16 only
  // without arg-mins (one running minimum per target) and for N <= 2048 (the
  // squares table's reach)
  int xs_max_N = 0;
  for (const auto& J : pl.in)
    if ((mode & PM_XS) && J.g.p == 2) xs_max_N = std::max(xs_max_N, J.g.N);
  const bool xs16 = !(mode & PM_ARGMIN) && xs_max_N <= 2048;
  // QBW_XS_XT=0 keeps two-dimensional jobs on the last-axis-first order
  const char* xte = std::getenv("QBW_XS_XT");
  const bool xs_xt_on = !(xte && std::strcmp(xte, "0") == 0);
  // QBW_XS_WIN=0 scans every source of those jobs (no argmin windows)
  const char* xwe = std::getenv("QBW_XS_WIN");
  const bool xs_win_on = !(xwe && std::strcmp(xwe, "0") == 0);
  // QBW_XS_WG (1 or 2): an argmin-window item spans that many target groups
  // of xs_T targets, on as many times the waves (one scan of the item's
  // lines serves all of its targets' windows)
  int xs_wg = 2;
  if (const char* e = std::getenv("QBW_XS_WG")) {
    const int v = std::atoi(e);
    if (v == 1 || v == 2) xs_wg = v;
  }
  int xs_T = xs16 ? 16 : 8;
  {
    auto waves = [&](int T) {
      long long w = 0;
      for (const auto& J : pl.in)
        if ((mode & PM_XS) && J.g.p == 2) {
          const long long rows = ipow(J.g.N, J.g.d - 1);
          w += ((rows + 63) / 64) * ((J.g.N + T - 1) / T);
        }
      return w;
    };
    const long long want = 4LL * 4 * ctx->num_cu;
    // without arg-mins a work-group's waves can split an item's sources
    // (up to four), which counts toward the waves a launch has
    const int max_split = (mode & PM_ARGMIN) ? 1 : 4;
    while (xs_T > 2 && waves(xs_T) * max_split < want) xs_T /= 2;
    // QBW_XS_T (2, 4, 8, or 16 without arg-mins) overrides the choice
    if (const char* e = std::getenv("QBW_XS_T")) {
      const int v = std::atoi(e);
      if (v == 2 || v == 4 || v == 8 || (v == 16 && xs16)) xs_T = v;
    }
    // splits up to about eight waves per SIMD requested (fewer fit at 16
    // targets per lane; the surplus queues behind, which still measured
    // faster than stopping at four)
    pl.xs_W = 1;
    while (pl.xs_W < max_split && waves(xs_T) * pl.xs_W < 2 * want) pl.xs_W *= 2;
    // QBW_XS_W (1, 2 or 4 without arg-mins) overrides the split
    if (const char* e = std::getenv("QBW_XS_W")) {
      const int v = std::atoi(e);
      if (v == 1 || ((v == 2 || v == 4) && max_split == 4)) pl.xs_W = v;
    }
    pl.xs_W0 = pl.xs_W;
    if (const char* e = std::getenv("QBW_XS_W0")) {   // the first stage's alone
      const int v = std::atoi(e);
      if (v == 1 || ((v == 2 || v == 4) && max_split == 4)) pl.xs_W0 = v;
    }
    pl.xs_T = xs_T;
  }
  for (int j = 0; j < NJ; ++j) {
    const auto& J = pl.in[j];
    const Offs& O = offs[j];
    DevJob& D = pl.hj[j];
    std::memset(&D, 0, sizeof(D));
    D.d = J.g.d; D.N = J.g.N; D.k = J.g.k; D.p = J.g.p;
    D.n = J.g.N / J.g.k;
    D.P = ipow(D.N, D.d);
    D.Q = ipow(D.n, D.d);
    D.rows = ipow(D.N, D.d - 1);
    D.R = J.tiling.R;
    D.S = J.tiling.S;
    D.chunks = (D.P + kChunk - 1) / kChunk;
    D.nnz = J.coarse ? J.coarse->nnz : 0;
    D.max_iter = o.max_ipf_iter;
    D.want_argmin = (mode & PM_ARGMIN) ? 1 : 0;
    D.interp = (o.flags & QBW_INTERP_CUBIC) ? 2 : (o.flags & QBW_INTERP_NEAREST) ? 1 : 0;
    D.xi = o.xi;
    D.coarse_obj = J.coarse ? J.coarse->obj : 0.0;
    D.mu = J.a;
    D.nu = J.b;
    D.mu_t = (double*)(B + O.mu_t);
    D.nu_t = (double*)(B + O.nu_t);
    D.ftil = (const double*)(B + O.ftil);
    D.fhat = (float*)(B + O.fhat);
    D.g = (float*)(B + O.g);
    D.f = (float*)(B + O.f);
    D.part = (float*)(B + O.part);
    D.win = (int*)(B + O.win);
    D.arg_g = (mode & PM_ARGMIN) ? (int*)(B + O.arg_g) : nullptr;
    D.arg_f = (mode & PM_ARGMIN) ? (int*)(B + O.arg_f) : nullptr;
    D.e_row = (const int*)(B + O.e_row);
    D.e_col = (const int*)(B + O.e_col);
    D.e_val = (const double*)(B + O.e_val);
    D.csr_ptr = (const int*)(B + O.csr);
    D.csc_ptr = (const int*)(B + O.csc);
    D.csc_idx = (const int*)(B + O.csc_idx);
    D.ipf_u = (double*)(B + O.ipf_u);
    D.ipf_v = (double*)(B + O.ipf_v);
    D.a_s = (double*)(B + O.a_s);
    D.b_s = (double*)(B + O.b_s);
    D.red_lb = (double*)(B + O.red_lb);
    D.red_tv = (double*)(B + O.red_tv);
    D.red_pc = (double*)(B + O.red_pc);
    D.red_pm = (double*)(B + O.red_pm);
    if (J.coarse) {
      const CoarseHost& C = *J.coarse;
      for (int K = 0; K < C.Q; ++K) {
        D.row_max = std::max(D.row_max, C.csr_ptr[K + 1] - C.csr_ptr[K]);
        D.col_max = std::max(D.col_max, C.csc_ptr[K + 1] - C.csc_ptr[K]);
      }
    }
    D.result = (double*)(B + o_res) + (size_t)RS_COUNT * j;
    D.flags = (int*)(B + o_ints) + 2 * kQueues + 2 + j;
    D.grad_a = J.ga;
    D.grad_b = J.gb;
    D.gbar_mu = (double*)(B + O.gbar_mu);
    D.gbar_nu = (double*)(B + O.gbar_nu);
    D.coef = (double*)(B + O.coef);
    D.gquad = (double*)(B + O.gquad);
    D.part1 = D.p == 1 ? (double*)(B + O.part1) : nullptr;
    D.mom_mu = (double*)(B + O.mom_mu);
    D.mom_nu = (double*)(B + O.mom_nu);
    D.mom_as = (double*)(B + O.mom_as);
    D.mom_bs = (double*)(B + O.mom_bs);
    D.sep = ((mode & PM_SEP) && D.p == 2) ? 1 : 0;
    D.sep_tmp = D.sep ? (float*)(B + O.sep_tmp) : nullptr;
    D.sep_arg = (D.sep && (mode & PM_ARGMIN)) ? (int*)(B + O.sep_arg) : nullptr;
    D.sep_R = (D.sep && !(mode & PM_ARGMIN)) ? ct1d_fast_R(D.N) : 0;
    if (D.sep) pl.sep_kinds |= D.sep_R ? (unsigned)D.sep_R : 1u;
    D.xs = ((mode & PM_XS) && D.p == 2) ? 1 : 0;
    D.xs_v = D.xs ? (double*)(B + O.xs_v) : nullptr;
    D.xs_i = D.xs ? (int*)(B + O.xs_i) : nullptr;
    {
      // exact separable stages: one wave per (64 lines, xs_T targets along the axis)
      D.xs_T = xs_T;
      D.xs_xt = (D.xs && D.d == 2 && !(mode & PM_ARGMIN) && xs_T >= 8 && xs_xt_on) ? (xs_win_on ? 2 : 1) : 0;
      pl.xs_xt_kind = xs_win_on ? 2 : 1;
      pl.xs_wg = xs_wg;
      if (D.xs) (D.xs_xt ? pl.xs_has_xt : pl.xs_has_std) = true;
      const int Tj = D.xs_xt == 2 ? xs_T * xs_wg : xs_T;   // targets per item
      const int xs_items = D.xs ? ((D.rows + 63) / 64) * ((D.N + Tj - 1) / Tj) : 0;
      off[12 * (NJ + 1) + j + 1] = off[12 * (NJ + 1) + j] + xs_items;
      off[13 * (NJ + 1) + j + 1] = off[13 * (NJ + 1) + j] + (D.d == 3 ? xs_items : 0);
    }
    off[0 * (NJ + 1) + j + 1] = off[0 * (NJ + 1) + j] + D.chunks;
    const int bpw = 64 / reduce_group(ipow(D.k, D.d));   // blocks per wave in pooling / moments
    off[1 * (NJ + 1) + j + 1] = off[1 * (NJ + 1) + j] + (D.Q + 4 * bpw - 1) / (4 * bpw);
    off[2 * (NJ + 1) + j + 1] = off[2 * (NJ + 1) + j] + D.nnz;
    off[3 * (NJ + 1) + j + 1] = off[3 * (NJ + 1) + j] + D.Q;
    off[4 * (NJ + 1) + j + 1] = off[4 * (NJ + 1) + j] + (int)(((long long)D.Q * D.Q + 255) / 256);
    // block moments: one item per strip of blocks along the last axis (k <= 64),
    // else per 4 waves of (side, block) lane groups
    off[5 * (NJ + 1) + j + 1] = off[5 * (NJ + 1) + j] +
                                (D.k <= 64 ? ipow(D.n, D.d - 1) : (2 * D.Q + 4 * bpw - 1) / (4 * bpw));
    // p = 1 plan cost and upper-bound gradient: one item per (entry, 64 pixels
    // of its block), or per 64 / reduce_group(k^d) entries when k^d <= 32
    const int mblk = ipow(D.k, D.d);
    D.p1_nt = D.p == 1 ? p1_table_nt(D.k, D.d) : 0;
    D.sqrt_tab = (D.p == 1 && (int64_t)D.d * (D.N - 1) * (D.N - 1) < kSqrtTab) ? ctx->sqrt_tab : nullptr;
    // direct kernels (table 6): per (entry, 64 pixels), or 64 / g entries per
    // item when k^d <= 32; distance-table kernels (tables 10, 11): per
    // (entry, 64 or 256 pixels)
    const int p1_items = D.p != 1 || D.p1_nt ? 0
                         : mblk <= 32 ? (D.nnz + 64 / reduce_group(mblk) - 1) / (64 / reduce_group(mblk))
                                      : D.nnz * ((mblk + 63) / 64);
    off[6 * (NJ + 1) + j + 1] = off[6 * (NJ + 1) + j] + p1_items;
    off[10 * (NJ + 1) + j + 1] = off[10 * (NJ + 1) + j] + (D.p1_nt == 64 ? D.nnz * ((mblk + 63) / 64) : 0);
    off[11 * (NJ + 1) + j + 1] = off[11 * (NJ + 1) + j] + (D.p1_nt == 256 ? D.nnz * ((mblk + 255) / 256) : 0);
    off[7 * (NJ + 1) + j + 1] = off[7 * (NJ + 1) + j] + (D.p == 2 ? (D.nnz + 255) / 256 : 0);
    // separable passes: one item per line (fast kernel) or per (line, 64 targets)
    off[8 * (NJ + 1) + j + 1] = off[8 * (NJ + 1) + j] + (D.sep ? D.rows * (D.sep_R ? 1 : (D.N + 63) / 64) : 0);
    off[9 * (NJ + 1) + j + 1] = off[9 * (NJ + 1) + j] + p1_items;
    if (D.sep) pl.max_sep_d = std::max(pl.max_sep_d, D.d);
    (D.p == 1 ? pl.has_p1 : pl.has_p2) = true;
  }
  pl.djobs = (DevJob*)(B + o_jobs);
  int* offd = (int*)(B + o_offs);
  pl.off_chunk = offd;
  pl.off_pool = offd + (NJ + 1);
  pl.off_entry = offd + 2 * (NJ + 1);
  pl.off_block = offd + 3 * (NJ + 1);
  pl.off_cbar = offd + 4 * (NJ + 1);
  pl.off_mom = offd + 5 * (NJ + 1);
  pl.off_pc1 = offd + 6 * (NJ + 1);
  pl.off_pc2 = offd + 7 * (NJ + 1);
  pl.tot_pc1 = off[6 * (NJ + 1) + NJ];
  pl.tot_pc2 = off[7 * (NJ + 1) + NJ];
  pl.off_sep = offd + 8 * (NJ + 1);
  pl.tot_sep = off[8 * (NJ + 1) + NJ];
  pl.off_ubg = offd + 9 * (NJ + 1);
  pl.tot_ubg = off[9 * (NJ + 1) + NJ];
  for (int q = 0; q < 2; ++q) {
    pl.p1_tab.off[1 + q] = offd + (10 + q) * (NJ + 1);
    pl.p1_tab.total[1 + q] = off[(10 + q) * (NJ + 1) + NJ];
  }
  pl.off_xs = offd + 12 * (NJ + 1);
  pl.tot_xs = off[12 * (NJ + 1) + NJ];
  pl.off_xs3 = offd + 13 * (NJ + 1);
  pl.tot_xs3 = off[13 * (NJ + 1) + NJ];
  pl.xs_list = pl.xs_pixels ? (int*)(B + o_xs_list) : nullptr;
  pl.xs_sq = ctx->xs_sq;
  pl.p1_tab.off[0] = pl.off_pc1;
  pl.p1_tab.total[0] = pl.tot_pc1;
  pl.tot_chunk = off[0 * (NJ + 1) + NJ];
  pl.tot_pool = off[1 * (NJ + 1) + NJ];
  pl.tot_entry = off[2 * (NJ + 1) + NJ];
  pl.tot_block = off[3 * (NJ + 1) + NJ];
  pl.tot_cbar = off[4 * (NJ + 1) + NJ];
  pl.tot_mom = off[5 * (NJ + 1) + NJ];
  pl.items = (CtItem*)(B + o_items);
  pl.ints = (int*)(B + o_ints);
  pl.dl = (double*)(B + o_dl);
  pl.du = (double*)(B + o_du);
  pl.results = (double*)(B + o_res);
  pl.bwd_scratch = (double*)(B + o_bwd);
  double** ptrs = (double**)(B + o_ptrs);
  pl.cbar_out = ptrs;
  pl.fhat_grad_out = ptrs + 3 * NJ;
  pl.ct_grid = std::max(1, G);
  for (const auto& D : pl.hj) {   // jobs that do not fit keep their coarse data in global memory
    const size_t ni = coarse_lds_need(D.Q, D.nnz, 6), nb = coarse_lds_need(D.Q, D.nnz, 4);
    if (ni <= kCoarseLdsMax) pl.ipf_lds = std::max(pl.ipf_lds, ni);
    if (nb <= kCoarseLdsMax) pl.bwd_lds = std::max(pl.bwd_lds, nb);
  }

  // uploads: the previous staged copy must have landed before the staging
  // memory is rewritten
  if (ctx->staged) {
    HIPCHK(hipEventSynchronize(ctx->staged_ev));
    ctx->staged = false;
  }
  const size_t ubytes = u1 - u0;
  if (ubytes > ctx->stage_cap) {
    if (ctx->stage) HIPCHK(hipHostFree(ctx->stage));
    ctx->stage = nullptr;
    ctx->stage_cap = 0;
    const size_t want = std::max(ubytes, (size_t)1 << 20);
    if (hipHostMalloc((void**)&ctx->stage, want, hipHostMallocDefault) != hipSuccess) {
      ctx->stage = nullptr;
      set_error("pinned host allocation of %zu bytes failed", want);
      return QBW_E_NOMEM;
    }
    ctx->stage_cap = want;
  }
  if (!ctx->staged_ev) HIPCHK(hipEventCreateWithFlags(&ctx->staged_ev, hipEventDisableTiming));
  // host image of the region: at(off) mirrors B + off
  auto at = [&](size_t off) { return ctx->stage + (off - u0); };
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(at(off), src, bytes);
  };
  put(o_jobs, pl.hj.data(), sizeof(DevJob) * NJ);
  put(o_offs, off.data(), sizeof(int) * off.size());
  put(o_items, items.data(), sizeof(CtItem) * items.size());
  std::memset(at(o_ptrs), 0, sizeof(double*) * 4 * NJ);
  std::memset(at(o_ints), 0, sizeof(int) * pl.n_ints);
  {
    const std::vector<double> ones(NJ, 1.0);
    put(o_dl, ones.data(), 8 * (size_t)NJ);
    put(o_du, ones.data(), 8 * (size_t)NJ);
  }
  for (int j = 0; j < NJ; ++j) {
    const CoarseHost* C = pl.in[j].coarse;
    if (!C) continue;
    const Offs& O = offs[j];
    put(O.ftil, C->f.data(), 8 * (size_t)C->Q);
    put(O.e_row, C->rows.data(), 4 * (size_t)C->nnz);
    put(O.e_col, C->cols.data(), 4 * (size_t)C->nnz);
    put(O.e_val, C->vals.data(), 8 * (size_t)C->nnz);
    put(O.csr, C->csr_ptr.data(), 4 * (size_t)(C->Q + 1));
    put(O.csc, C->csc_ptr.data(), 4 * (size_t)(C->Q + 1));
    put(O.csc_idx, C->csc_idx.data(), 4 * (size_t)C->nnz);
  }
  HIPCHK(hipMemcpyAsync(B + u0, ctx->stage, ubytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(ctx->staged_ev, st));
  ctx->staged = true;
  return QBW_OK;
}

static int enqueue_sep(Plan& pl, int phase, hipStream_t st) {
  const int NJ = pl.njobs;
  for (int pass = 0; pass < pl.max_sep_d; ++pass) {
    if (pl.sep_kinds & 1u) CHK(launch_ct1d(pl.djobs, NJ, pl.off_sep, pl.tot_sep, phase, pass, st));
    for (int R : {4, 8, 16})
      if (pl.sep_kinds & (unsigned)R) CHK(launch_ct1d_fast(pl.djobs, NJ, pl.off_sep, pl.tot_sep, phase, pass, R, st));
  }
  if (pl.mode & PM_ARGMIN) CHK(launch_sep_argmin(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, phase, st));
  return QBW_OK;
}

// The queue lengths sit after the jobs' flags in pl.ints and are cleared with
// the other counters at the start of a forward pass.
static int* xs_count(Plan& pl, int phase) { return pl.ints + 2 * kQueues + phase; }

// Events around a launch when the batch's c-transform timing is on.
template <typename F>
static int timed_launch(Plan& pl, hipStream_t st, F launch) {
  std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
  if (pl.timing) {
    if (pl.ev_used == pl.ev_pool.size()) {
      hipEvent_t a, b;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&b));
      pl.ev_pool.push_back({a, b});
    }
    ev = &pl.ev_pool[pl.ev_used++];
    HIPCHK(hipEventRecord(ev->first, st));
  }
  CHK(launch());
  if (ev) HIPCHK(hipEventRecord(ev->second, st));
  return QBW_OK;
}

static int enqueue_xs(Plan& pl, int phase, hipStream_t st) {
  int* cnt = xs_count(pl, phase);
  for (int k = 0; k < 3; ++k) {
    const int* off = k < 2 ? pl.off_xs : pl.off_xs3;
    const int total = k < 2 ? pl.tot_xs : pl.tot_xs3;
    if (!total) continue;
    // two-dimensional value-only jobs take axis 0 first (their own kernel
    // instance), the others axis d-1 first; a plan may hold both
    for (int xt = 0; xt < 2; ++xt) {
      if (!(xt ? pl.xs_has_xt && k < 2 : pl.xs_has_std)) continue;
      CHK(timed_launch(pl, st, [&] {
        const int kind = xt ? pl.xs_xt_kind : 0;
        const int f = kind == 2 ? pl.xs_wg : 1;
        return launch_xs_stage(pl.djobs, pl.njobs, off, total, phase, k, pl.xs_sq, pl.xs_list, cnt, pl.xs_T * f,
                               (pl.mode & PM_ARGMIN) ? 1 : 0, (k == 0 ? pl.xs_W0 : pl.xs_W) * f, kind, st);
      }));
    }
  }
  return launch_xs_fallback(pl.djobs, pl.xs_list, cnt, phase, std::max(1, std::min(pl.xs_pixels, 4096)), st);
}

static int enqueue_plancost_p1(Plan& pl, hipStream_t st) {
  const int NJ = pl.njobs;
  if (pl.p1_tab.total[0] + pl.p1_tab.total[1] + pl.p1_tab.total[2]) {
    CHK(launch_plancost(pl.djobs, NJ, pl.p1_tab, st));
    CHK(launch_pc1_sum(pl.djobs, NJ, st));
  }
  return QBW_OK;
}

static int enqueue_ctransforms(Plan& pl, hipStream_t st) {
  const int NJ = pl.njobs;
  for (int phase = 0; phase < 2; ++phase) {
    if (pl.tot_sep) CHK(enqueue_sep(pl, phase, st));
    if (pl.tot_xs) CHK(enqueue_xs(pl, phase, st));
    if (!pl.n_items) continue;
    CHK(timed_launch(pl, st, [&] {
      return launch_ctransform(pl.djobs, pl.items, pl.n_items, pl.ints + phase * kQueues, phase, pl.ct_grid, st);
    }));
    CHK(launch_merge(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, phase, st));
    if (pl.mode & PM_ARGMIN) CHK(launch_argmin(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, phase, st));
  }
  return QBW_OK;
}

// Plan cost from caller-supplied scalings: their block moments, then the
// entries (p = 2); the pixel-pair sums (p = 1).
static int enqueue_plancost(Plan& pl, hipStream_t st) {
  const int NJ = pl.njobs;
  if (pl.tot_pc2) {
    CHK(launch_moments(pl.djobs, NJ, pl.off_mom, pl.tot_mom, 1, st));
    CHK(launch_plancost2(pl.djobs, NJ, pl.off_pc2, pl.tot_pc2, st));
  }
  return enqueue_plancost_p1(pl, st);
}

// A second stream for the coarse kernel of a step: it depends only on the
// pooled measures and overlaps the c-transforms.  Null members: one stream.
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// The plan's counters are zero when it is built and the pixel sweep zeroes
// the c-transform counters again for the next step.
static int enqueue_forward(Plan& pl, hipStream_t st, const SideStream* side = nullptr) {
  const int NJ = pl.njobs;
  // SumPool, block moments and f^ (Algorithm 5's upscaled potential) in one
  // pass over the block strips
  bool big_k = false;
  for (const auto& D : pl.hj) big_k |= D.k > 64;
  CHK(launch_pool(pl.djobs, NJ, pl.off_mom, pl.tot_mom, 1, st));
  if (big_k) CHK(launch_upscale(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, 1, st));
  // upper bound (Algorithm 4), coarse part: the fitting, the p = 2 plan-cost
  // entries from the pooled moments and, when a backward pass follows, its
  // coarse reverse pass, all in one launch that needs only the pooled measures
  hipStream_t cs = st;
  if (side && side->st) {
    HIPCHK(hipEventRecord(side->fork, st));
    HIPCHK(hipStreamWaitEvent(side->st, side->fork, 0));
    cs = side->st;
  }
  CHK(launch_ipf(pl.djobs, NJ, pl.ipf_lds, 1 | (pl.fwd_rev ? 2 : 0), pl.bwd_scratch, pl.max_q, cs));
  if (cs != st) HIPCHK(hipEventRecord(side->join, cs));
  // lower bound (Algorithm 5): the c-transforms of f^
  CHK(enqueue_ctransforms(pl, st));
  if (cs != st) HIPCHK(hipStreamWaitEvent(st, side->join, 0));
  // one sweep over the pixels for the lower-bound sums, the fine scalings and
  // the weighted-TV sums; the p = 1 plan cost; the bounds
  CHK(launch_fwd_pixels(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, pl.ints, 2 * kQueues + 2, st));
  CHK(enqueue_plancost_p1(pl, st));
  CHK(launch_finalize(pl.djobs, NJ, st));
  return QBW_OK;
}

static int enqueue_backward(Plan& pl, hipStream_t st) {
  const int NJ = pl.njobs;
  // p = 1 jobs: separate lower- and upper-bound passes (the latter over
  // support blocks); p = 2 jobs: one fused pass over pixels after the moments
  if (pl.has_p1) CHK(launch_lb_grad(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, pl.dl, st));
  // the coarse reverse pass, unless the forward's coarse kernel ran it (p = 2)
  if (pl.has_p1 || !pl.fwd_rev)
    CHK(launch_ub_coarse_bwd2(pl.djobs, NJ, pl.bwd_scratch, pl.max_q, pl.bwd_lds, pl.fwd_rev ? 1 : 0, st));
  if (pl.has_p1) {
    for (int side = 0; side < 2; ++side) {   // per-entry partials, then per-pixel sums
      P1Items ubg = pl.p1_tab;
      ubg.off[0] = pl.off_ubg;
      ubg.total[0] = pl.tot_ubg;
      CHK(launch_ub_grad(pl.djobs, NJ, ubg, pl.du, side, st));
      CHK(launch_ub_grad_sum(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, pl.du, side, st));
    }
  }
  if (pl.has_p2) CHK(launch_grad2(pl.djobs, NJ, pl.off_chunk, pl.tot_chunk, pl.dl, pl.du, st));
  return QBW_OK;
}

static void to_result(const double* r, qbw_result* out) {
  out->lower = r[RS_LOWER];
  out->upper = r[RS_UPPER];
  out->lower_S = r[RS_LOWER_S];
  out->feas_shift = r[RS_SHIFT];
  out->upper_cost = r[RS_UPPER_COST];
  out->tv_mu = r[RS_TV_MU];
  out->tv_nu = r[RS_TV_NU];
  out->ipf_residual = r[RS_IPF_RESID];
  out->coarse_objective = r[RS_COARSE_OBJ];
  out->ipf_iters = (int32_t)r[RS_IPF_ITERS];
  out->warn = (uint32_t)r[RS_WARN];
}

static int fetch_results(Plan& pl, hipStream_t st) {
  pl.host_results.resize((size_t)RS_COUNT * pl.njobs);
  HIPCHK(hipMemcpyAsync(pl.host_results.data(), pl.results, 8 * pl.host_results.size(),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

// Pool on the device, validate on the host (negative / NaN entries, masses).
static int pool_and_check(qbw_ctx* ctx, const std::vector<JobIn>& jobs, std::vector<std::vector<double>>* mt,
                          std::vector<std::vector<double>>* nt, hipStream_t st) {
  Plan pl;
  qbw_opts o = qbw_default_opts();
  o.max_ipf_iter = 1;
  CHK(plan_build(ctx, pl, jobs, 0, o, true, st));
  CHK(launch_reset_counter(pl.ints, pl.n_ints, st));
  CHK(launch_pool(pl.djobs, pl.njobs, pl.off_mom, pl.tot_mom, 0, st));
  std::vector<int> flags(pl.n_ints);
  mt->resize(pl.njobs);
  nt->resize(pl.njobs);
  for (int j = 0; j < pl.njobs; ++j) {
    const DevJob& D = pl.hj[j];
    (*mt)[j].resize(D.Q);
    (*nt)[j].resize(D.Q);
    HIPCHK(hipMemcpyAsync((*mt)[j].data(), D.mu_t, 8 * D.Q, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync((*nt)[j].data(), D.nu_t, 8 * D.Q, hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipMemcpyAsync(flags.data(), pl.ints, 4 * pl.n_ints, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int j = 0; j < pl.njobs; ++j) {
    const int fl = flags[2 * kQueues + 2 + j];
    if (fl & 2) { set_error("job %d: a measure contains NaN", j); return QBW_E_MASS; }
    if (fl & 1) { set_error("job %d: a measure has a negative entry", j); return QBW_E_MASS; }
    double sa = 0, sb = 0;
    for (double v : (*mt)[j]) sa += v;
    for (double v : (*nt)[j]) sb += v;
    if (!(sa > 0) || !(sb > 0) || !std::isfinite(sa) || !std::isfinite(sb)) {
      set_error("job %d: a measure has no mass", j);
      return QBW_E_MASS;
    }
    if (std::fabs(sa - sb) > 1e-10 * std::max(sa, sb)) {
      set_error("job %d: unequal masses %.17g vs %.17g", j, sa, sb);
      return QBW_E_MASS;
    }
  }
  return QBW_OK;
}

static int solve_coarse_host(const qbw_grid& g, const std::vector<double>& mt, const std::vector<double>& nt,
                             CoarseSolution* sol) {
  const int Q = (int)mt.size();
  std::vector<double> C((size_t)Q * Q);
  centre_cost(g, C.data());
  CoarseProblem P{Q, mt.data(), nt.data(), C.data(), g.p == 2};
  // multiscale start by default; QBW_COARSE_SOLVER=dense prices every block
  // pair from the first pivot (the same optimum either way)
  const char* e = std::getenv("QBW_COARSE_SOLVER");
  const bool dense = e && std::strcmp(e, "dense") == 0;
  int rc = dense ? coarse_solve(P, sol) : coarse_solve_multiscale(P, g.N / g.k, g.d, g.p, sol);
  if (rc != QBW_OK) set_error("coarse network simplex failed (Q=%d)", Q);
  return rc;
}

static int to_coarse_host(const qbw_grid& g, const CoarseSolution& s, CoarseHost* out) {
  qbw_coarse c;
  c.Q = (int)s.f.size();
  c.nnz = (int)s.vals.size();
  c.rows = s.rows.data();
  c.cols = s.cols.data();
  c.vals = s.vals.data();
  c.f = s.f.data();
  return make_coarse(g, &c, out);
}

// Parallel host solves over jobs.
static int solve_all(const std::vector<qbw_grid>& grids, const std::vector<std::vector<double>>& mt,
                     const std::vector<std::vector<double>>& nt, std::vector<CoarseHost>* out) {
  const int NJ = (int)grids.size();
  out->resize(NJ);
  std::vector<int> rcs(NJ, QBW_OK);
  std::vector<std::string> errs(NJ);
  std::atomic<int> next{0};
  // one host thread per core (QBW_HOST_THREADS overrides), at most one per job
  int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  if (const char* e = std::getenv("QBW_HOST_THREADS")) {
    const int t = std::atoi(e);
    if (t > 0) hw = t;
  }
  const int nthreads = std::max(1, std::min(NJ, hw));
  auto worker = [&]() {
    for (;;) {
      int j = next.fetch_add(1);
      if (j >= NJ) break;
      CoarseSolution sol;
      int rc = solve_coarse_host(grids[j], mt[j], nt[j], &sol);
      if (rc == QBW_OK) rc = to_coarse_host(grids[j], sol, &(*out)[j]);
      rcs[j] = rc;
      if (rc != QBW_OK) errs[j] = g_err;
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nthreads; ++t) th.emplace_back(worker);
  worker();
  for (auto& t : th) t.join();
  for (int j = 0; j < NJ; ++j)
    if (rcs[j] != QBW_OK) { set_error("job %d: %s", j, errs[j].c_str()); return rcs[j]; }
  return QBW_OK;
}

// Single-pair tiling: the environment override QBW_TILE_R (targets per lane,
// one of 32, 16, 8, 4, 2, 1, used where it divides N), else the tuned value,
// else the default.
static Tiling lookup_tiling(qbw_ctx* ctx, const qbw_grid& g) {
  if (const char* e = std::getenv("QBW_TILE_R")) {
    const int R = std::atoi(e);
    if ((R == 32 || R == 16 || R == 8 || R == 4 || R == 2 || R == 1) && g.N % R == 0) return {R, 0};
  }
  auto it = ctx->tuned.find({g.d, g.N, g.p});
  if (it != ctx->tuned.end()) return it->second;
  return {default_R(g.N), 0};
}

}  // namespace qbw

using namespace qbw;

struct qbw_saved {
  Plan plan;
  std::vector<CoarseHost> coarse;
  qbw_ctx* ctx = nullptr;   // where the arena goes back to; null once detached
};

qbw_ctx::~qbw_ctx() {
  {
    std::lock_guard<std::mutex> lk(mu);
    for (qbw_saved* sv : live) sv->ctx = nullptr;
    live.clear();
  }
  if (staged_ev) { (void)hipEventSynchronize(staged_ev); (void)hipEventDestroy(staged_ev); }
  if (stage) (void)hipHostFree(stage);
  if (sqrt_tab) (void)hipFree(sqrt_tab);
  if (xs_sq) (void)hipFree(xs_sq);
}

struct qbw_batch {
  qbw_ctx* ctx = nullptr;
  Plan plan;
  std::vector<CoarseHost> coarse;
  uint32_t flags = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double* pinned = nullptr;  // 2 * njobs upstream gradients
  // completion of the last copy out of `pinned`: a run waits for it before it
  // rewrites the staging memory, so back-to-back runs cannot change the
  // upstream gradients of a copy that is still pending
  hipEvent_t pinned_ev = nullptr;
  bool pinned_busy = false;
  // the upstream gradients last copied to the device: a run with the same
  // values copies nothing (the device copy is still current)
  std::vector<double> last_grads;
  SideStream side;   // the coarse kernel's stream and its fork / join events
};

extern "C" {

const char* qbw_last_error(void) { return g_err.c_str(); }
const char* qbw_version(void) { return "qbw 0.1 (gfx950)"; }

qbw_opts qbw_default_opts(void) {
  qbw_opts o;
  o.xi = 1e-12;
  o.max_ipf_iter = 50;
  o.flags = 0;
  return o;
}

qbw_status qbw_create(qbw_ctx** ctx, int32_t device) {
  if (!ctx) { set_error("ctx is NULL"); return QBW_E_INVAL; }
  *ctx = nullptr;
  int cnt = 0;
  HIPCHK(hipGetDeviceCount(&cnt));
  if (device < 0 || device >= cnt) { set_error("device %d not available (%d devices)", device, cnt); return QBW_E_HIP; }
  HIPCHK(hipSetDevice(device));
  auto* c = new (std::nothrow) qbw_ctx();
  if (!c) { set_error("out of host memory"); return QBW_E_NOMEM; }
  c->device = device;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
    c->num_cu = cu;
  // one full round of resident c-transform waves: equal-sized work items then
  // finish together instead of leaving a partly filled last round
  const int occ = qbw::ctransform_waves_per_cu();
  c->target_waves = c->num_cu * (occ > 0 ? occ : 16);
  // the integer square-root and squares tables, filled once and never
  // written again, so plans on any stream (and captured graphs) may read them
  if (hipMalloc(&c->sqrt_tab, sizeof(float) * qbw::kSqrtTab) != hipSuccess) {
    c->sqrt_tab = nullptr;
    delete c;
    set_error("device allocation of the square-root table failed");
    return QBW_E_NOMEM;
  }
  if (hipMalloc(&c->xs_sq, sizeof(double) * qbw::kXsSquares) != hipSuccess) {
    c->xs_sq = nullptr;
    delete c;
    set_error("device allocation of the squares table failed");
    return QBW_E_NOMEM;
  }
  int rc = qbw::launch_sqrt_table(c->sqrt_tab, qbw::kSqrtTab, nullptr);
  if (rc == QBW_OK) rc = qbw::launch_xs_squares(c->xs_sq, nullptr);
  // the device address of the static scratch array, with `device` current
  if (rc == QBW_OK) {
    void* sp = nullptr;
    rc = qbw::scratch_address(device, &sp);
    c->scratch = (char*)sp;
  }
  if (rc == QBW_OK && hipDeviceSynchronize() != hipSuccess) {
    set_error("filling the square-root table failed");
    rc = QBW_E_HIP;
  }
  if (rc != QBW_OK) { delete c; return (qbw_status)rc; }
  *ctx = c;
  return QBW_OK;
}

void qbw_destroy(qbw_ctx* ctx) { delete ctx; }

static int check_opts(const qbw_opts* o) {
  if (!o) return QBW_OK;
  if (o->max_ipf_iter < 1 || o->max_ipf_iter > 100000) { set_error("max_ipf_iter must be in [1, 1e5]"); return QBW_E_INVAL; }
  if (!(o->xi > 0) && !(o->xi <= 0)) { set_error("xi is NaN"); return QBW_E_INVAL; }
  if ((o->flags & QBW_SEPARABLE) && (o->flags & QBW_SEPARABLE_EXACT)) {
    set_error("QBW_SEPARABLE and QBW_SEPARABLE_EXACT are exclusive");
    return QBW_E_INVAL;
  }
  if ((o->flags & QBW_INTERP_NEAREST) && (o->flags & QBW_INTERP_CUBIC)) {
    set_error("QBW_INTERP_NEAREST and QBW_INTERP_CUBIC are exclusive");
    return QBW_E_INVAL;
  }
  return QBW_OK;
}

static qbw_status bounds_impl(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                              const CoarseHost* C, const qbw_opts* opts, qbw_result* out, qbw_saved** saved,
                              qbw_stream stream, std::vector<CoarseHost>* keep) {
  qbw_opts o = opts ? *opts : qbw_default_opts();
  const bool save = (o.flags & QBW_SAVE_FOR_BWD) && saved;
  unsigned mode = PM_FORWARD | ((o.flags & QBW_WANT_ARGMIN) ? PM_ARGMIN : 0u) |
                  ((o.flags & QBW_SEPARABLE) ? PM_SEP : 0u) | ((o.flags & QBW_SEPARABLE_EXACT) ? PM_XS : 0u);
  JobIn J{*grid, a, b, nullptr, nullptr, nullptr, lookup_tiling(ctx, *grid)};
  hipStream_t st = S(stream);
  if (save) {
    auto* sv = new (std::nothrow) qbw_saved();
    if (!sv) { set_error("out of host memory"); return QBW_E_NOMEM; }
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (!ctx->spare.empty()) {
        sv->plan.own = std::move(ctx->spare.back());
        ctx->spare.pop_back();
      }
      ctx->live.insert(sv);
      sv->ctx = ctx;
    }
    sv->coarse = std::move(*keep);
    J.coarse = &sv->coarse[0];
    int rc = plan_build(ctx, sv->plan, {J}, mode | PM_BACKWARD, o, true, st);
    if (rc == QBW_OK) rc = enqueue_forward(sv->plan, st);
    if (rc == QBW_OK) rc = fetch_results(sv->plan, st);
    if (rc != QBW_OK) { qbw_saved_free(sv); return (qbw_status)rc; }
    to_result(sv->plan.host_results.data(), out);
    *saved = sv;
    return QBW_OK;
  }
  J.coarse = C;
  Plan pl;
  CHK(plan_build(ctx, pl, {J}, mode, o, false, st));
  CHK(enqueue_forward(pl, st));
  CHK(fetch_results(pl, st));
  to_result(pl.host_results.data(), out);
  if (saved) *saved = nullptr;
  return QBW_OK;
}

qbw_status qbw_bounds_with_coarse(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                                  const qbw_coarse* coarse, const qbw_opts* opts, qbw_result* out,
                                  qbw_saved** saved, qbw_stream stream) {
  if (!ctx || !a || !b || !out || !coarse) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  CHK(check_opts(opts));
  std::vector<CoarseHost> ch(1);
  CHK(make_coarse(*grid, coarse, &ch[0]));
  return bounds_impl(ctx, grid, a, b, &ch[0], opts, out, saved, stream, &ch);
}

qbw_status qbw_bounds(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                      const qbw_opts* opts, qbw_result* out, qbw_saved** saved, qbw_stream stream) {
  if (!ctx || !a || !b || !out) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  CHK(check_opts(opts));
  std::vector<std::vector<double>> mt, nt;
  JobIn J{*grid, a, b, nullptr, nullptr, nullptr, {default_R(grid->N), 1}};
  CHK(pool_and_check(ctx, {J}, &mt, &nt, S(stream)));
  std::vector<CoarseHost> ch;
  CHK(solve_all({*grid}, mt, nt, &ch));
  return bounds_impl(ctx, grid, a, b, &ch[0], opts, out, saved, stream, &ch);
}

qbw_status qbw_bounds_backward(qbw_ctx* ctx, const qbw_saved* saved, double dlower, double dupper,
                               double* grad_a, double* grad_b, double* grad_fhat, qbw_stream stream) {
  if (!ctx || !saved) { set_error("NULL argument"); return QBW_E_INVAL; }
  if (!grad_a || !grad_b) { set_error("grad_a and grad_b are required"); return QBW_E_INVAL; }
  auto* sv = const_cast<qbw_saved*>(saved);
  Plan& pl = sv->plan;
  hipStream_t st = S(stream);
  pl.hj[0].grad_a = grad_a;
  pl.hj[0].grad_b = grad_b;
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  double g2[2] = {dlower, dupper};
  HIPCHK(hipMemcpyAsync(pl.dl, &g2[0], 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(pl.du, &g2[1], 8, hipMemcpyHostToDevice, st));
  CHK(enqueue_backward(pl, st));
  if (grad_fhat) {
    if (!(pl.mode & PM_ARGMIN)) { set_error("grad_fhat needs QBW_WANT_ARGMIN in the forward pass"); return QBW_E_STATE; }
    HIPCHK(hipMemcpyAsync(pl.fhat_grad_out, &grad_fhat, sizeof(double*), hipMemcpyHostToDevice, st));
    CHK(launch_fhat_grad2(pl.djobs, 1, pl.off_chunk, pl.tot_chunk, pl.dl, pl.fhat_grad_out, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

void qbw_saved_free(qbw_saved* saved) {
  if (!saved) return;
  if (qbw_ctx* ctx = saved->ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->live.erase(saved);
    // keep a few arenas for reuse; the plan's work on them has finished (every
    // entry point that uses a saved record synchronizes before returning)
    if (saved->plan.own.base && ctx->spare.size() < 4) ctx->spare.push_back(std::move(saved->plan.own));
  }
  delete saved;
}

// ---------------------------------------------------------------- stages

static JobIn stage_job(const qbw_grid* g, const double* a, const double* b) {
  return JobIn{*g, a, b, nullptr, nullptr, nullptr, {default_R(g->N), 0}};
}

qbw_status qbw_sumpool(qbw_ctx* ctx, const qbw_grid* grid, const double* m, double* out, qbw_stream stream) {
  if (!ctx || !m || !out) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  Plan pl;
  hipStream_t st = S(stream);
  CHK(plan_build(ctx, pl, {stage_job(grid, m, m)}, 0, qbw_default_opts(), false, st));
  pl.hj[0].mu_t = out;
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  CHK(launch_reset_counter(pl.ints, pl.n_ints, st));
  CHK(launch_pool(pl.djobs, 1, pl.off_mom, pl.tot_mom, 0, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

qbw_status qbw_coarse_cost(const qbw_grid* grid, double* out) {
  if (!out) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  centre_cost(*grid, out);
  return QBW_OK;
}

qbw_status qbw_cbar(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b, double* out,
                    qbw_stream stream) {
  if (!ctx || !a || !b || !out) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  Plan pl;
  hipStream_t st = S(stream);
  CHK(plan_build(ctx, pl, {stage_job(grid, a, b)}, PM_CBAR, qbw_default_opts(), false, st));
  HIPCHK(hipMemcpyAsync(pl.cbar_out, &out, sizeof(double*), hipMemcpyHostToDevice, st));
  CHK(launch_reset_counter(pl.ints, pl.n_ints, st));
  CHK(launch_pool(pl.djobs, 1, pl.off_mom, pl.tot_mom, 0, st));
  CHK(launch_cbar2(pl.djobs, 1, pl.off_cbar, pl.tot_cbar, pl.cbar_out, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

static void min_cost_matrix(const qbw_grid& g, double* out) {
  const int n = g.N / g.k;
  const int Q = ipow(n, g.d);
  for (int K = 0; K < Q; ++K) {
    int kc[3] = {0, 0, 0}, t = K;
    for (int a = g.d - 1; a >= 0; --a) { kc[a] = t % n; t /= n; }
    for (int L = 0; L < Q; ++L) {
      int lc[3] = {0, 0, 0}, s = L;
      for (int a = g.d - 1; a >= 0; --a) { lc[a] = s % n; s /= n; }
      long long d2 = 0;
      for (int a = 0; a < g.d; ++a) {
        // closest pixels of two blocks along one axis: k |K - L| - (k - 1) apart, or 0
        long long gap = (long long)g.k * std::llabs((long long)kc[a] - lc[a]) - (g.k - 1);
        if (gap < 0) gap = 0;
        d2 += gap * gap;
      }
      out[(size_t)K * Q + L] = g.p == 2 ? (double)d2 : std::sqrt((double)d2);
    }
  }
}

qbw_status qbw_weighted_cost_upper(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                                   double* upper, double* objective, qbw_stream stream) {
  if (!ctx || !a || !b || !upper) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  hipStream_t st = S(stream);
  std::vector<std::vector<double>> mt, nt;
  JobIn J{*grid, a, b, nullptr, nullptr, nullptr, {default_R(grid->N), 1}};
  CHK(pool_and_check(ctx, {J}, &mt, &nt, st));
  const int Q = (int)mt[0].size();
  Plan pl;
  CHK(plan_build(ctx, pl, {stage_job(grid, a, b)}, PM_CBAR, qbw_default_opts(), false, st));
  double* dC = nullptr;
  HIPCHK(hipMalloc(&dC, 8 * (size_t)Q * Q));
  std::unique_ptr<double, void (*)(double*)> guard(dC, [](double* p) { (void)hipFree(p); });
  HIPCHK(hipMemcpyAsync(pl.cbar_out, &dC, sizeof(double*), hipMemcpyHostToDevice, st));
  CHK(launch_reset_counter(pl.ints, pl.n_ints, st));
  CHK(launch_pool(pl.djobs, 1, pl.off_mom, pl.tot_mom, 0, st));
  CHK(launch_cbar2(pl.djobs, 1, pl.off_cbar, pl.tot_cbar, pl.cbar_out, st));
  std::vector<double> C((size_t)Q * Q);
  HIPCHK(hipMemcpyAsync(C.data(), dC, 8 * C.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  CoarseProblem P{Q, mt[0].data(), nt[0].data(), C.data(), false};
  CoarseSolution sol;
  if (coarse_solve(P, &sol) != QBW_OK) { set_error("network simplex failed on C-bar (Q=%d)", Q); return QBW_E_LP; }
  const double obj = std::max(sol.objective, 0.0) * (1.0 + 9.094947017729282e-13);
  *upper = grid->p == 2 ? std::sqrt(obj) : obj;
  if (objective) *objective = sol.objective;
  return QBW_OK;
}

qbw_status qbw_min_cost_lower(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                              double* lower, double* objective, qbw_stream stream) {
  if (!ctx || !a || !b || !lower) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  std::vector<std::vector<double>> mt, nt;
  JobIn J{*grid, a, b, nullptr, nullptr, nullptr, {default_R(grid->N), 1}};
  CHK(pool_and_check(ctx, {J}, &mt, &nt, S(stream)));
  const int Q = (int)mt[0].size();
  std::vector<double> C((size_t)Q * Q);
  min_cost_matrix(*grid, C.data());
  CoarseProblem P{Q, mt[0].data(), nt[0].data(), C.data(), grid->p == 2};
  CoarseSolution sol;
  if (coarse_solve(P, &sol) != QBW_OK) { set_error("network simplex failed on C^min (Q=%d)", Q); return QBW_E_LP; }
  // dual objective of admissible potentials is a lower bound whatever the rounding
  double viol = 0.0, dual = 0.0, ma = 0.0, mb = 0.0;
  for (int K = 0; K < Q; ++K)
    for (int L = 0; L < Q; ++L) viol = std::max(viol, sol.f[K] + sol.g[L] - C[(size_t)K * Q + L]);
  for (int K = 0; K < Q; ++K) {
    dual += sol.f[K] * mt[0][K] + sol.g[K] * nt[0][K];
    ma += mt[0][K];
    mb += nt[0][K];
  }
  double s = dual - viol * std::max(ma, mb);
  s -= std::fabs(s) * 9.094947017729282e-13;
  s = std::max(s, 0.0);
  *lower = grid->p == 2 ? std::sqrt(s) : s;
  if (objective) *objective = sol.objective;
  return QBW_OK;
}

qbw_status qbw_coarse_solve_host(const qbw_grid* grid, const double* a_t, const double* b_t, int32_t* rows,
                                 int32_t* cols, double* vals, int32_t* nnz, double* f, double* g,
                                 double* objective) {
  if (!a_t || !b_t || !rows || !cols || !vals || !nnz || !f || !g) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  const int Q = ipow(grid->N / grid->k, grid->d);
  std::vector<double> mt(a_t, a_t + Q), nt(b_t, b_t + Q);
  double sa = 0, sb = 0;
  for (int K = 0; K < Q; ++K) {
    if (!(mt[K] >= 0) || !(nt[K] >= 0)) { set_error("coarse masses must be nonnegative"); return QBW_E_MASS; }
    sa += mt[K]; sb += nt[K];
  }
  if (!(sa > 0) || std::fabs(sa - sb) > 1e-10 * std::max(sa, sb)) { set_error("unequal or zero coarse masses"); return QBW_E_MASS; }
  CoarseSolution sol;
  CHK(solve_coarse_host(*grid, mt, nt, &sol));
  if ((int)sol.vals.size() > 2 * Q - 1) { set_error("internal: basis larger than 2Q-1"); return QBW_E_LP; }
  *nnz = (int)sol.vals.size();
  for (int e = 0; e < *nnz; ++e) { rows[e] = sol.rows[e]; cols[e] = sol.cols[e]; vals[e] = sol.vals[e]; }
  for (int K = 0; K < Q; ++K) { f[K] = sol.f[K]; g[K] = sol.g[K]; }
  if (objective) *objective = sol.objective;
  return QBW_OK;
}

qbw_status qbw_upscale_potential(qbw_ctx* ctx, const qbw_grid* grid, const double* ftil, float* fhat,
                                 qbw_stream stream) {
  return qbw_upscale_potential_interp(ctx, grid, 0u, ftil, fhat, stream);
}

qbw_status qbw_upscale_potential_interp(qbw_ctx* ctx, const qbw_grid* grid, uint32_t interp,
                                        const double* ftil, float* fhat, qbw_stream stream) {
  if (!ctx || !ftil || !fhat) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  if (interp != 0u && interp != QBW_INTERP_NEAREST && interp != QBW_INTERP_CUBIC) {
    set_error("interp must be 0, QBW_INTERP_NEAREST or QBW_INTERP_CUBIC (got %u)", interp);
    return QBW_E_INVAL;
  }
  Plan pl;
  hipStream_t st = S(stream);
  qbw_opts o = qbw_default_opts();
  o.flags = interp;
  CHK(plan_build(ctx, pl, {stage_job(grid, nullptr, nullptr)}, 0, o, false, st));
  pl.hj[0].ftil = ftil;
  pl.hj[0].fhat = fhat;
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  CHK(launch_upscale(pl.djobs, 1, pl.off_chunk, pl.tot_chunk, 0, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

qbw_status qbw_ctransform(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst, int32_t* argmin,
                          qbw_stream stream) {
  if (!ctx || !src || !dst) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  Plan pl;
  hipStream_t st = S(stream);
  JobIn J = stage_job(grid, nullptr, nullptr);
  J.tiling = lookup_tiling(ctx, *grid);
  CHK(plan_build(ctx, pl, {J}, argmin ? PM_ARGMIN : 0u, qbw_default_opts(), false, st));
  pl.hj[0].fhat = const_cast<float*>(src);
  pl.hj[0].g = dst;
  if (argmin) pl.hj[0].arg_g = argmin;
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  CHK(launch_reset_counter(pl.ints, pl.n_ints, st));
  CHK(launch_ctransform(pl.djobs, pl.items, pl.n_items, pl.ints, 0, pl.ct_grid, st));
  CHK(launch_merge(pl.djobs, 1, pl.off_chunk, pl.tot_chunk, 0, st));
  if (argmin) CHK(launch_argmin(pl.djobs, 1, pl.off_chunk, pl.tot_chunk, 0, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

qbw_status qbw_ctransform_noalloc(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst,
                                  int32_t* argmin, qbw_stream stream) {
  if (!ctx || !src || !dst) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  if (!ctx->scratch) { set_error("the context has no static scratch address"); return QBW_E_HIP; }
  hipStream_t st = S(stream);
  std::vector<JobIn> in{stage_job(grid, nullptr, nullptr)};
  in[0].tiling = lookup_tiling(ctx, *grid);
  CHK(choose_splits(in, ctx->target_waves));
  const int N = grid->N, d = grid->d;
  const int P = ipow(N, d), rows = ipow(N, d - 1);
  const int R = in[0].tiling.R;
  const int tiles = (P + 64 * R - 1) / (64 * R);
  const int chunks = (P + kChunk - 1) / kChunk;
  constexpr int kInts = 64;
  // scratch layout: [job][prefix table][items][counters][winning split]
  // [S partial-minimum rows]; the first four are written by the set-up kernel
  struct Offs { size_t job, off, items, ints, win, part, end; };
  auto layout = [&](int S) {
    Layout L;
    Offs o;
    o.job = L.add(sizeof(DevJob));
    o.off = L.add(sizeof(int) * 2);
    o.items = L.add(sizeof(CtItem) * (size_t)tiles * S);
    o.ints = L.add(sizeof(int) * kInts);
    o.win = L.add(4 * (size_t)P);
    o.part = L.add(4 * (size_t)P * S);
    o.end = L.size;
    return o;
  };
  // fewer source splits when the planned ones do not fit (results do not
  // depend on the split count); whole source rows per split, as planned
  int S = in[0].tiling.S;
  while (S > 1 && layout(S).end > kScratchBytes) {
    const int want = S - 1;
    const int r = (rows + want - 1) / want;
    S = (rows + r - 1) / r;
  }
  const Offs o = layout(S);
  if (o.end > kScratchBytes) {
    set_error("qbw_ctransform_noalloc: N^d = %d needs %zu bytes of scratch, the static scratch holds %zu "
              "(about %zu pixels at most)", P, o.end, kScratchBytes, kScratchBytes / 8 - 64);
    return QBW_E_INVAL;
  }
  const int n_items = tiles * S;
  const int G = std::min(n_items, ctx->num_cu * 4 * 8);
  char* B = ctx->scratch;
  DevJob D;
  std::memset(&D, 0, sizeof(D));
  D.d = d; D.N = N; D.k = grid->k; D.p = grid->p;
  D.n = N / grid->k;
  D.P = P;
  D.Q = ipow(D.n, d);
  D.rows = rows;
  D.R = R;
  D.S = S;
  D.chunks = chunks;
  D.want_argmin = argmin ? 1 : 0;
  D.fhat = const_cast<float*>(src);
  D.g = dst;
  D.arg_g = argmin;
  D.part = (float*)(B + o.part);
  D.win = (int*)(B + o.win);
  D.sqrt_tab = (D.p == 1 && (int64_t)d * (N - 1) * (N - 1) < kSqrtTab) ? ctx->sqrt_tab : nullptr;
  DevJob* dj = (DevJob*)(B + o.job);
  int* doff = (int*)(B + o.off);
  CtItem* items = (CtItem*)(B + o.items);
  int* ints = (int*)(B + o.ints);
  CHK(launch_noalloc_setup(D, dj, doff, items, n_items, tiles, ints, kInts, st));
  CHK(launch_ctransform(dj, items, n_items, ints, 0, std::max(1, G), st));
  CHK(launch_merge(dj, 1, doff, chunks, 0, st));
  if (argmin) CHK(launch_argmin(dj, 1, doff, chunks, 0, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

qbw_status qbw_ctransform_separable(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst,
                                    int32_t* argmin, qbw_stream stream) {
  if (!ctx || !src || !dst) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  if (grid->p != 2) { set_error("the separable c-transform needs p = 2"); return QBW_E_GRID; }
  Plan pl;
  hipStream_t st = S(stream);
  CHK(plan_build(ctx, pl, {stage_job(grid, nullptr, nullptr)}, PM_SEP | (argmin ? PM_ARGMIN : 0u),
                 qbw_default_opts(), false, st));
  pl.hj[0].fhat = const_cast<float*>(src);
  pl.hj[0].g = dst;
  if (argmin) pl.hj[0].arg_g = argmin;
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  CHK(enqueue_sep(pl, 0, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

qbw_status qbw_ctransform_exact(qbw_ctx* ctx, const qbw_grid* grid, const float* src, float* dst,
                                int32_t* argmin, int32_t* n_fallback, qbw_stream stream) {
  if (!ctx || !src || !dst) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  if (grid->p != 2) { set_error("the exact separable c-transform needs p = 2"); return QBW_E_GRID; }
  Plan pl;
  hipStream_t st = S(stream);
  CHK(plan_build(ctx, pl, {stage_job(grid, nullptr, nullptr)}, PM_XS | (argmin ? PM_ARGMIN : 0u),
                 qbw_default_opts(), false, st));
  pl.hj[0].fhat = const_cast<float*>(src);
  pl.hj[0].g = dst;
  pl.hj[0].arg_g = argmin;
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  CHK(launch_reset_counter(pl.ints, pl.n_ints, st));
  CHK(enqueue_xs(pl, 0, st));
  if (n_fallback) HIPCHK(hipMemcpyAsync(n_fallback, xs_count(pl, 0), sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

static qbw_status coarse_stage_plan(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                                    const qbw_coarse* coarse, const qbw_opts* opts, Plan& pl, CoarseHost& ch,
                                    hipStream_t st) {
  if (!ctx || !coarse) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  CHK(check_opts(opts));
  CHK(make_coarse(*grid, coarse, &ch));
  JobIn J = stage_job(grid, a, b);
  J.coarse = &ch;
  return (qbw_status)plan_build(ctx, pl, {J}, 0, opts ? *opts : qbw_default_opts(), false, st);
}

qbw_status qbw_ipf(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                   const qbw_coarse* coarse, const qbw_opts* opts, double* a_s, double* b_s, int32_t* iters,
                   double* residual, qbw_stream stream) {
  if (!a || !b || !a_s || !b_s) { set_error("NULL argument"); return QBW_E_INVAL; }
  Plan pl;
  CoarseHost ch;
  hipStream_t st = S(stream);
  CHK(coarse_stage_plan(ctx, grid, a, b, coarse, opts, pl, ch, st));
  pl.hj[0].a_s = a_s;
  pl.hj[0].b_s = b_s;
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  CHK(launch_reset_counter(pl.ints, pl.n_ints, st));
  CHK(launch_pool(pl.djobs, 1, pl.off_mom, pl.tot_mom, 0, st));
  CHK(launch_ipf(pl.djobs, 1, pl.ipf_lds, 0, nullptr, 0, st));
  CHK(launch_scalings(pl.djobs, 1, pl.off_chunk, pl.tot_chunk, st));
  CHK(fetch_results(pl, st));
  if (iters) *iters = (int32_t)pl.host_results[RS_IPF_ITERS];
  if (residual) *residual = pl.host_results[RS_IPF_RESID];
  return QBW_OK;
}

qbw_status qbw_plan_cost(qbw_ctx* ctx, const qbw_grid* grid, const qbw_coarse* coarse, const double* a_s,
                         const double* b_s, double* cost, qbw_stream stream) {
  if (!a_s || !b_s || !cost) { set_error("NULL argument"); return QBW_E_INVAL; }
  Plan pl;
  CoarseHost ch;
  hipStream_t st = S(stream);
  CHK(coarse_stage_plan(ctx, grid, a_s, b_s, coarse, nullptr, pl, ch, st));
  DevJob& D = pl.hj[0];
  D.a_s = const_cast<double*>(a_s);
  D.b_s = const_cast<double*>(b_s);
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(D.red_lb, 0, 8 * (size_t)D.chunks * kRedSlotsLB, st));
  HIPCHK(hipMemsetAsync(D.red_tv, 0, 8 * (size_t)D.chunks * kRedSlotsTV, st));
  HIPCHK(hipMemsetAsync(D.result, 0, 8 * RS_COUNT, st));
  CHK(enqueue_plancost(pl, st));
  CHK(launch_finalize(pl.djobs, 1, st));
  CHK(fetch_results(pl, st));
  *cost = pl.host_results[RS_PCOST_RAW];
  return QBW_OK;
}

qbw_status qbw_tv(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                  const qbw_coarse* coarse, const double* a_s, const double* b_s, double* tv_mu, double* tv_nu,
                  qbw_stream stream) {
  if (!a || !b || !a_s || !b_s || !tv_mu || !tv_nu) { set_error("NULL argument"); return QBW_E_INVAL; }
  Plan pl;
  CoarseHost ch;
  hipStream_t st = S(stream);
  CHK(coarse_stage_plan(ctx, grid, a, b, coarse, nullptr, pl, ch, st));
  DevJob& D = pl.hj[0];
  D.a_s = const_cast<double*>(a_s);
  D.b_s = const_cast<double*>(b_s);
  HIPCHK(hipMemcpyAsync(pl.djobs, pl.hj.data(), sizeof(DevJob), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(D.red_lb, 0, 8 * (size_t)D.chunks * kRedSlotsLB, st));
  HIPCHK(hipMemsetAsync(D.red_pc, 0, 8 * (size_t)std::max(1, D.nnz), st));
  HIPCHK(hipMemsetAsync(D.red_pm, 0, 8 * (size_t)std::max(1, D.nnz), st));
  HIPCHK(hipMemsetAsync(D.result, 0, 8 * RS_COUNT, st));
  CHK(launch_tv_prep(pl.djobs, 1, st));
  CHK(launch_tv_partial(pl.djobs, 1, pl.off_chunk, pl.tot_chunk, st));
  CHK(launch_finalize(pl.djobs, 1, st));
  CHK(fetch_results(pl, st));
  *tv_mu = pl.host_results[RS_TV_RAW_MU];
  *tv_nu = pl.host_results[RS_TV_RAW_NU];
  return QBW_OK;
}

// ---------------------------------------------------------------- upper bound with any upscaling kernel

constexpr int kMaxKernelOffsets = 4096;  // k^d: the kernel matrix is k^d x k^d float64

static int check_plan_kernel(int m, const double* K) {
  // compensated (Neumaier) sum, so that the 1e-12 test does not depend on m
  double sum = 0.0, comp = 0.0;
  for (size_t q = 0; q < (size_t)m * m; ++q) {
    const double v = K[q];
    if (!(v >= 0.0) || !std::isfinite(v)) {
      set_error("kernel entry %zu is negative or not finite", q);
      return QBW_E_INVAL;
    }
    const double t = sum + v;
    comp += std::fabs(sum) >= v ? (sum - t) + v : (v - t) + sum;
    sum = t;
  }
  sum += comp;
  if (!(std::fabs(sum - 1.0) <= 1e-12)) {
    set_error("kernel entries sum to %.17g, not 1", sum);
    return QBW_E_INVAL;
  }
  return QBW_OK;
}

qbw_status qbw_upper_kernel(qbw_ctx* ctx, const qbw_grid* grid, const double* a, const double* b,
                            const qbw_coarse* coarse, const double* kernel, const qbw_opts* opts,
                            qbw_result* out, double* a_s, double* b_s, double dupper, double* grad_a,
                            double* grad_b, qbw_stream stream) {
  if (!ctx || !grid || !a || !b || !coarse || !kernel || !out) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  CHK(check_opts(opts));
  const qbw_opts o = opts ? *opts : qbw_default_opts();
  const int m = ipow(grid->k, grid->d);
  if (m > kMaxKernelOffsets) {
    set_error("kernel upscaling needs k^d <= %d, got %d", kMaxKernelOffsets, m);
    return QBW_E_GRID;
  }
  CHK(check_plan_kernel(m, kernel));
  CoarseHost ch;
  CHK(make_coarse(*grid, coarse, &ch));
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = S(stream);

  KubJob J{};
  J.d = grid->d; J.N = grid->N; J.k = grid->k; J.p = grid->p;
  J.n = J.N / J.k; J.P = ipow(J.N, J.d); J.Q = ch.Q; J.m = m; J.nnz = ch.nnz;
  J.max_iter = o.max_ipf_iter;
  J.nt = m <= 64 ? 64 : 256;
  J.cpb = (m + J.nt - 1) / J.nt;
  J.chunks = (J.P + kChunk - 1) / kChunk;
  J.xi = o.xi;
  J.coarse_obj = ch.obj;
  J.mu = a;
  J.nu = b;
  // uploaded tables first (one copy), device-only buffers after them
  Layout lay;
  const size_t mm = (size_t)m * m, P = J.P, Q = J.Q, nnz = J.nnz;
  const size_t oKst = lay.add(8 * mm), oKts = lay.add(8 * mm), oVal = lay.add(8 * nnz),
               oRes = lay.add(8 * RS_COUNT), oRow = lay.add(4 * nnz), oCol = lay.add(4 * nnz),
               oCsr = lay.add(4 * (Q + 1)), oCsc = lay.add(4 * (Q + 1)), oIdx = lay.add(4 * nnz),
               oState = lay.add(4 * 2);
  const size_t up = lay.size;
  const size_t oA0 = lay.add(8 * P), oA1 = lay.add(8 * P), oB = lay.add(8 * P), oMuh = lay.add(8 * P),
               oNuh = lay.add(8 * P), oPm = lay.add(8 * Q * J.cpb), oPn = lay.add(8 * Q * J.cpb),
               oPc = lay.add(8 * nnz * J.cpb), oTv = lay.add(8 * (size_t)J.chunks * kRedSlotsTV);
  // gradient: every iterate u^t, v^t is kept, plus five adjoint vectors
  const bool grad = grad_a || grad_b;
  size_t oHu = 0, oHv = 0, oG = 0;
  if (grad) {
    const double hist = 8.0 * P * (2.0 * J.max_iter + 8.0);
    if (hist > 32.0 * (1ull << 30)) {
      set_error("gradient needs %.1f GiB of checkpointed iterates (max_ipf_iter %d); the cap is 32 GiB",
                hist / (1ull << 30), J.max_iter);
      return QBW_E_NOMEM;
    }
    oHu = lay.add(8 * P * (size_t)(J.max_iter + 2));
    oHv = lay.add(8 * P * (size_t)(J.max_iter + 1));
    oG = lay.add(8 * P * 5);
  }
  CHK(ctx->work.reserve(lay.size));
  char* base = ctx->work.base;
  std::vector<char> blob(up, 0);
  double* kst = (double*)(blob.data() + oKst);
  double* kts = (double*)(blob.data() + oKts);
  for (int s = 0; s < m; ++s)
    for (int t = 0; t < m; ++t) {
      kst[(size_t)s * m + t] = kernel[(size_t)s * m + t];
      kts[(size_t)t * m + s] = kernel[(size_t)s * m + t];
    }
  std::memcpy(blob.data() + oVal, ch.vals.data(), 8 * nnz);
  std::memcpy(blob.data() + oRow, ch.rows.data(), 4 * nnz);
  std::memcpy(blob.data() + oCol, ch.cols.data(), 4 * nnz);
  std::memcpy(blob.data() + oCsr, ch.csr_ptr.data(), 4 * (Q + 1));
  std::memcpy(blob.data() + oCsc, ch.csc_ptr.data(), 4 * (Q + 1));
  std::memcpy(blob.data() + oIdx, ch.csc_idx.data(), 4 * nnz);
  HIPCHK(hipMemcpyAsync(base, blob.data(), up, hipMemcpyHostToDevice, st));
  J.Kst = (const double*)(base + oKst);
  J.Kts = (const double*)(base + oKts);
  J.e_val = (const double*)(base + oVal);
  J.result = (double*)(base + oRes);
  J.e_row = (const int*)(base + oRow);
  J.e_col = (const int*)(base + oCol);
  J.csr_ptr = (const int*)(base + oCsr);
  J.csc_ptr = (const int*)(base + oCsc);
  J.csc_idx = (const int*)(base + oIdx);
  J.state = (int*)(base + oState);
  J.a0 = (double*)(base + oA0);
  J.a1 = (double*)(base + oA1);
  J.b = (double*)(base + oB);
  J.muh = (double*)(base + oMuh);
  J.nuh = (double*)(base + oNuh);
  J.part_mu = (double*)(base + oPm);
  J.part_nu = (double*)(base + oPn);
  J.pc_part = (double*)(base + oPc);
  J.red_tv = (double*)(base + oTv);
  if (grad) {
    J.hist_u = (double*)(base + oHu);
    J.hist_v = (double*)(base + oHv);
    double* g = (double*)(base + oG);
    J.g_mu = g;
    J.g_nu = g + P;
    J.g_abar = g + 2 * P;
    J.g_ubar = g + 3 * P;
    J.g_vbar = g + 4 * P;
  }

  // Algorithm 4's fitting: row(0) gives a^1; then col(t), row(t), check(t).
  // The host looks at the stop flag every kGroup iterations; passes enqueued
  // after the stop return at once.
  constexpr int kGroup = 16;
  CHK(launch_kub_row(J, 0, st));
  for (int t0 = 1; t0 <= J.max_iter; t0 += kGroup) {
    const int t1 = std::min(J.max_iter, t0 + kGroup - 1);
    for (int t = t0; t <= t1; ++t) {
      CHK(launch_kub_col(J, t, st));
      CHK(launch_kub_row(J, t, st));
      CHK(launch_kub_check(J, t, st));
    }
    int stopped = 0;
    HIPCHK(hipMemcpyAsync(&stopped, J.state, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (stopped) break;
  }
  CHK(launch_kub_plancost(J, st));
  CHK(launch_kub_tv(J, st));
  CHK(launch_kub_finalize(J, st));
  std::vector<double> res(RS_COUNT);
  HIPCHK(hipMemcpyAsync(res.data(), J.result, 8 * RS_COUNT, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  to_result(res.data(), out);
  const int T = out->ipf_iters;
  if (grad) CHK(launch_kub_backward(J, T, dupper, grad_a, grad_b, st));
  if (a_s) HIPCHK(hipMemcpyAsync(a_s, (T & 1) ? J.a1 : J.a0, 8 * P, hipMemcpyDeviceToDevice, st));
  if (b_s) HIPCHK(hipMemcpyAsync(b_s, J.b, 8 * P, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return QBW_OK;
}

qbw_status qbw_plan_kernel_gaussian(int32_t k, int32_t d, double sigma, double* out) {
  if (!out || k < 1 || (d != 2 && d != 3) || !(sigma > 0.0)) {
    set_error("plan kernel needs k >= 1, d in {2, 3}, sigma > 0 and an output array");
    return QBW_E_INVAL;
  }
  const int m = ipow(k, d);
  if (m > kMaxKernelOffsets) {
    set_error("kernel upscaling needs k^d <= %d, got %d", kMaxKernelOffsets, m);
    return QBW_E_GRID;
  }
  // one factor per axis, exp(-(u - v)^2 / (2 sigma^2)); the kernel is their product
  std::vector<double> g1((size_t)k * k);
  for (int u = 0; u < k; ++u)
    for (int v = 0; v < k; ++v) g1[(size_t)u * k + v] = std::exp(-(double)((u - v) * (u - v)) / (2.0 * sigma * sigma));
  double tot = 0.0;
  for (int s = 0; s < m; ++s)
    for (int t = 0; t < m; ++t) {
      double w = 1.0;
      int rs = s, rt = t;
      for (int a = 0; a < d; ++a) {
        w *= g1[(size_t)(rs % k) * k + (rt % k)];
        rs /= k;
        rt /= k;
      }
      out[(size_t)s * m + t] = w;
      tot += w;
    }
  for (size_t q = 0; q < (size_t)m * m; ++q) out[q] /= tot;
  return QBW_OK;
}

// ---------------------------------------------------------------- batches

static qbw_status batch_enqueue(qbw_batch* B, hipStream_t st) {
  CHK(enqueue_forward(B->plan, st, &B->side));
  if (B->flags & QBW_BATCH_BACKWARD) CHK(enqueue_backward(B->plan, st));
  return QBW_OK;
}

static double time_ctransform(qbw_ctx* ctx, Plan& pl, hipStream_t st, int reps) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 1e30;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return 1e30; }
  double best = 1e30;
  for (int r = 0; r < reps; ++r) {
    (void)launch_reset_counter(pl.ints, pl.n_ints, st);
    (void)hipEventRecord(e0, st);
    (void)launch_ctransform(pl.djobs, pl.items, pl.n_items, pl.ints, 0, pl.ct_grid, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) break;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)ctx;
  return best;
}

static std::string tune_cache_path() {
  const char* p = std::getenv("QBW_TUNE_CACHE");
  if (p && *p) return p;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : ".") + "/.cache/qbw_tune.txt";
}

static void load_tune_cache(qbw_ctx* ctx) {
  std::ifstream in(tune_cache_path());
  int d, N, p, R, Sp;
  std::string arch;
  while (in >> arch >> d >> N >> p >> R >> Sp)
    if (arch == "gfx950" && !ctx->tuned.count({d, N, p})) ctx->tuned[{d, N, p}] = {R, Sp};
}

static void save_tune_entry(int d, int N, int p, Tiling t) {
  std::ofstream out(tune_cache_path(), std::ios::app);
  if (out) out << "gfx950 " << d << " " << N << " " << p << " " << t.R << " " << t.S << "\n";
}

qbw_status qbw_autotune_ctransform(qbw_ctx* ctx, const qbw_grid* grid, int32_t* targets_per_lane,
                                   int32_t* splits, double* best_ms, qbw_stream stream) {
  if (!ctx) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(check_grid(grid));
  hipStream_t st = S(stream);
  const int N = grid->N, d = grid->d;
  const int P = ipow(N, d), rows = ipow(N, d - 1);
  Tiling best{default_R(N), 1};
  double best_t = 1e30;
  for (int R : {32, 16, 8, 4}) {
    if (N % R) continue;
    const int tiles = (P + 64 * R - 1) / (64 * R);
    for (int waves : {ctx->num_cu * 4, ctx->num_cu * 8, ctx->num_cu * 16, ctx->num_cu * 32}) {
      int Sp = std::max(1, std::min(rows, (waves + tiles - 1) / tiles));
      Plan pl;
      JobIn J = stage_job(grid, nullptr, nullptr);
      J.tiling = {R, Sp};
      CHK(plan_build(ctx, pl, {J}, 0, qbw_default_opts(), false, st));
      HIPCHK(hipMemsetAsync(pl.hj[0].fhat, 0, 4 * (size_t)P, st));
      const double t = time_ctransform(ctx, pl, st, 3);
      if (t < best_t) { best_t = t; best = {R, Sp}; }
    }
  }
  ctx->tuned[{d, N, grid->p}] = best;
  save_tune_entry(d, N, grid->p, best);
  if (targets_per_lane) *targets_per_lane = best.R;
  if (splits) *splits = best.S;
  if (best_ms) *best_ms = best_t;
  return QBW_OK;
}

qbw_status qbw_batch_create(qbw_ctx* ctx, const qbw_job* jobs, int32_t njobs, const qbw_coarse* coarse,
                            const qbw_opts* opts, uint32_t batch_flags, qbw_batch** out, qbw_stream stream) {
  if (!ctx || !jobs || njobs < 1 || !out) { set_error("NULL argument or empty batch"); return QBW_E_INVAL; }
  *out = nullptr;
  CHK(check_opts(opts));
  qbw_opts o = opts ? *opts : qbw_default_opts();
  hipStream_t st = S(stream);
  std::vector<JobIn> in(njobs);
  std::vector<qbw_grid> grids(njobs);
  for (int j = 0; j < njobs; ++j) {
    CHK(check_grid(&jobs[j].grid));
    if (!jobs[j].a || !jobs[j].b) { set_error("job %d has NULL measures", j); return QBW_E_INVAL; }
    if ((batch_flags & QBW_BATCH_BACKWARD) && (!jobs[j].grad_a || !jobs[j].grad_b)) {
      set_error("job %d: backward batches need grad_a and grad_b", j);
      return QBW_E_INVAL;
    }
    in[j] = JobIn{jobs[j].grid, jobs[j].a, jobs[j].b, jobs[j].grad_a, jobs[j].grad_b, nullptr, {0, 0}};
    grids[j] = jobs[j].grid;
  }
  auto* B = new (std::nothrow) qbw_batch();
  if (!B) { set_error("out of host memory"); return QBW_E_NOMEM; }
  std::unique_ptr<qbw_batch, void (*)(qbw_batch*)> guard(B, qbw_batch_destroy);
  B->ctx = ctx;
  B->flags = batch_flags;
  B->coarse.resize(njobs);
  if (coarse) {
    for (int j = 0; j < njobs; ++j) CHK(make_coarse(grids[j], &coarse[j], &B->coarse[j]));
  } else {
    std::vector<std::vector<double>> mt, nt;
    std::vector<JobIn> pin = in;
    for (auto& J : pin) J.tiling = {default_R(J.g.N), 1};
    CHK(pool_and_check(ctx, pin, &mt, &nt, st));
    CHK(solve_all(grids, mt, nt, &B->coarse));
  }
  for (int j = 0; j < njobs; ++j) in[j].coarse = &B->coarse[j];
  const unsigned mode = PM_FORWARD | ((batch_flags & QBW_BATCH_BACKWARD) ? PM_BACKWARD : 0u) |
                        ((o.flags & QBW_WANT_ARGMIN) ? PM_ARGMIN : 0u) |
                        ((o.flags & QBW_SEPARABLE) ? PM_SEP : 0u) |
                        ((o.flags & QBW_SEPARABLE_EXACT) ? PM_XS : 0u);
  load_tune_cache(ctx);
  if (batch_flags & QBW_BATCH_AUTOTUNE) {
    // batch-level tuning: targets per lane and the total number of waves the
    // source splits aim for; every candidate times the whole batch's c-transform
    double best_t = 1e30;
    int best_R = 0, best_w = ctx->target_waves;
    for (int R : {32, 16, 8}) {
      for (int waves : {ctx->num_cu * 4, ctx->num_cu * 8, ctx->num_cu * 16, ctx->num_cu * 32, ctx->num_cu * 48,
                        ctx->num_cu * 64}) {
        std::vector<JobIn> cand = in;
        for (auto& J : cand) J.tiling = {(J.g.N % R == 0) ? R : default_R(J.g.N), 0};
        const int keep = ctx->target_waves;
        ctx->target_waves = waves;
        Plan pl;
        int rc = plan_build(ctx, pl, cand, mode, o, false, st);
        ctx->target_waves = keep;
        if (rc != QBW_OK) return (qbw_status)rc;
        for (auto& D : pl.hj) HIPCHK(hipMemsetAsync(D.fhat, 0, 4 * (size_t)D.P, st));
        const double t = time_ctransform(ctx, pl, st, 2);
        if (t < best_t) { best_t = t; best_R = R; best_w = waves; }
      }
    }
    for (auto& J : in) J.tiling = {(J.g.N % best_R == 0) ? best_R : default_R(J.g.N), 0};
    const int keep = ctx->target_waves;
    ctx->target_waves = best_w;
    int rc = plan_build(ctx, B->plan, in, mode, o, true, st);
    ctx->target_waves = keep;
    CHK(rc);
  } else {
    for (auto& J : in) {
      auto it = ctx->tuned.find({J.g.d, J.g.N, J.g.p});
      J.tiling = {it != ctx->tuned.end() ? it->second.R : default_R(J.g.N), 0};
    }
    CHK(plan_build(ctx, B->plan, in, mode, o, true, st));
  }
  HIPCHK(hipHostMalloc((void**)&B->pinned, 16 * (size_t)njobs, hipHostMallocDefault));
  // the coarse kernel's own stream (QBW_COARSE_STREAM=main: the batch's stream)
  const char* cse = std::getenv("QBW_COARSE_STREAM");
  if (!(cse && std::strcmp(cse, "main") == 0)) {
    HIPCHK(hipStreamCreateWithFlags(&B->side.st, hipStreamNonBlocking));
    // the fork and the join order work between two streams of this device
    // only (the host never waits on them): no system-scope fence (QBW_EVENT_FENCE=1 keeps it)
    const char* efe = std::getenv("QBW_EVENT_FENCE");
    const unsigned ef = hipEventDisableTiming | ((efe && std::strcmp(efe, "1") == 0) ? 0u : hipEventDisableSystemFence);
    HIPCHK(hipEventCreateWithFlags(&B->side.fork, ef));
    HIPCHK(hipEventCreateWithFlags(&B->side.join, ef));
  }
  if (batch_flags & QBW_BATCH_GRAPH) {
    HIPCHK(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
    qbw_status rc = batch_enqueue(B, B->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(B->cap_stream, &g);
    if (rc != QBW_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e2 != hipSuccess) { set_error("graph capture failed: %s", hipGetErrorString(e2)); return QBW_E_HIP; }
    B->graph = g;
    HIPCHK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  }
  *out = guard.release();
  return QBW_OK;
}

qbw_status qbw_batch_run(qbw_batch* B, const double* dlower, const double* dupper, qbw_stream stream) {
  if (!B) { set_error("NULL batch"); return QBW_E_INVAL; }
  hipStream_t st = S(stream);
  const int NJ = B->plan.njobs;
  if (B->flags & QBW_BATCH_BACKWARD) {
    std::vector<double> want(2 * (size_t)NJ);
    for (int j = 0; j < NJ; ++j) {
      want[j] = dlower ? dlower[j] : 1.0;
      want[NJ + j] = dupper ? dupper[j] : 1.0;
    }
    // plan building wrote 1 for every job; otherwise the last run's values
    if (B->last_grads.empty()) B->last_grads.assign(2 * (size_t)NJ, 1.0);
    if (std::memcmp(want.data(), B->last_grads.data(), 8 * want.size()) != 0) {
      if (B->pinned_busy) {
        HIPCHK(hipEventSynchronize(B->pinned_ev));
        B->pinned_busy = false;
      }
      std::memcpy(B->pinned, want.data(), 8 * want.size());
      HIPCHK(hipMemcpyAsync(B->plan.dl, B->pinned, 8 * NJ, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(B->plan.du, B->pinned + NJ, 8 * NJ, hipMemcpyHostToDevice, st));
      if (!B->pinned_ev) HIPCHK(hipEventCreateWithFlags(&B->pinned_ev, hipEventDisableTiming));
      HIPCHK(hipEventRecord(B->pinned_ev, st));
      B->pinned_busy = true;
      B->last_grads = want;
    }
  }
  if (B->exec) {
    HIPCHK(hipGraphLaunch(B->exec, st));
    return QBW_OK;
  }
  return batch_enqueue(B, st);
}

qbw_status qbw_batch_results(qbw_batch* B, qbw_result* out, qbw_stream stream) {
  if (!B || !out) { set_error("NULL argument"); return QBW_E_INVAL; }
  CHK(fetch_results(B->plan, S(stream)));
  for (int j = 0; j < B->plan.njobs; ++j) to_result(B->plan.host_results.data() + (size_t)RS_COUNT * j, &out[j]);
  return QBW_OK;
}

qbw_status qbw_batch_set_timing(qbw_batch* B, int32_t enable) {
  if (!B) { set_error("NULL batch"); return QBW_E_INVAL; }
  B->plan.timing = enable != 0;
  B->plan.ev_used = 0;
  return QBW_OK;
}

qbw_status qbw_batch_ctransform_time(qbw_batch* B, double* mean_ms, int32_t* launches) {
  if (!B || !mean_ms || !launches) { set_error("NULL argument"); return QBW_E_INVAL; }
  Plan& pl = B->plan;
  double tot = 0;
  for (size_t i = 0; i < pl.ev_used; ++i) {
    HIPCHK(hipEventSynchronize(pl.ev_pool[i].second));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, pl.ev_pool[i].first, pl.ev_pool[i].second));
    tot += ms;
  }
  *launches = (int32_t)pl.ev_used;
  *mean_ms = pl.ev_used ? tot / pl.ev_used : 0.0;
  pl.ev_used = 0;
  return QBW_OK;
}

qbw_status qbw_batch_ctransform_pairs(const qbw_batch* B, double* pairs) {
  if (!B || !pairs) { set_error("NULL argument"); return QBW_E_INVAL; }
  // per phase: one all-pairs launch over the other jobs (P^2 each), and d
  // exact separable stages (P N candidates per job and stage)
  double evals = 0, launches = 0, ap = 0, s01 = 0, s2 = 0;
  for (const auto& D : B->plan.hj) {
    if (D.xs) {
      s01 += (double)D.P * D.N;
      if (D.d == 3) s2 += (double)D.P * D.N;
    } else {
      ap += (double)D.P * (double)D.P;
    }
  }
  if (ap > 0) { evals += ap; launches += 1; }
  if (s01 > 0) { evals += 2 * s01; launches += 2; }
  if (s2 > 0) { evals += s2; launches += 1; }
  *pairs = launches > 0 ? evals / launches : 0.0;
  return QBW_OK;
}

qbw_status qbw_batch_tiling(const qbw_batch* B, int32_t job, int32_t* targets_per_lane, int32_t* splits) {
  if (!B || job < 0 || job >= B->plan.njobs) { set_error("bad batch or job index"); return QBW_E_INVAL; }
  if (targets_per_lane) *targets_per_lane = B->plan.hj[job].R;
  if (splits) *splits = B->plan.hj[job].S;
  return QBW_OK;
}

void qbw_batch_destroy(qbw_batch* B) {
  if (!B) return;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
  if (B->side.st) { (void)hipStreamSynchronize(B->side.st); (void)hipStreamDestroy(B->side.st); }
  if (B->side.fork) (void)hipEventDestroy(B->side.fork);
  if (B->side.join) (void)hipEventDestroy(B->side.join);
  if (B->pinned_ev) { (void)hipEventSynchronize(B->pinned_ev); (void)hipEventDestroy(B->pinned_ev); }
  if (B->pinned) (void)hipHostFree(B->pinned);
  delete B;
}

qbw_status qbw_bounds_batched(qbw_ctx* ctx, const qbw_job* jobs, int32_t njobs, const qbw_opts* opts,
                              qbw_result* out, qbw_stream stream) {
  qbw_batch* B = nullptr;
  CHK(qbw_batch_create(ctx, jobs, njobs, nullptr, opts, 0, &B, stream));
  qbw_status rc = qbw_batch_run(B, nullptr, nullptr, stream);
  if (rc == QBW_OK) rc = qbw_batch_results(B, out, stream);
  qbw_batch_destroy(B);
  return rc;
}

}  // extern "C"
