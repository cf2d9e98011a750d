// Host network simplex for the coarse Kantorovich problem.
//
// The coarse problem of the primal- and dual-upscaling bounds (Algorithms 4
// and 5, "Solve" step) is a dense transportation problem between the n^d
// coarse blocks of mu and of nu with the centre cost C~.  It is small and
// serial, so it runs on the host.
//
// Method: primal network simplex on the bipartite graph plus an artificial
// root (every node starts on an artificial arc of big cost), block-search
// pricing over the implicit dense arc set, and the leaving-arc rule of
// strongly feasible spanning trees (ties on the source side resolved to the
// first blocking arc, on the target side to the last), which rules out
// cycling on degenerate pivots.  Supplies are integerised (scale 2^52,
// largest entry adjusted so both sides balance exactly) so that ratio tests
// are exact; after the optimal basis is found, its flows are re-derived in
// float64 from the actual block masses on the spanning tree (leaf peeling),
// so the returned coupling's marginals match mu~ and nu~ to float64
// rounding.  Duals come from the tree potentials: f_k = -pi_k, g_l = pi_l;
// with an integer cost (p = 2) they are exact integers.
//
// Blocks of zero mass are left out of the LP.  Their potentials are then
// completed by c-transforms of the solved ones, which keeps (f~, g~)
// admissible for every block pair: first f~_k = min_l C~_kl - g~_l for empty
// source blocks, then g~_l = min_k C~_kl - f~_k for empty target blocks.
// Finally f~ is shifted so that sum_k mu~_k f~_k = 0 (g~ the other way).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <type_traits>
#include <utility>
#include <vector>

#include "qbw_internal.h"

namespace qbw {

namespace {

// Smallest reduced cost c_j + pk - pl_j over one cost row segment.  Built for
// several instruction sets and picked at load time by the CPU's features.
__attribute__((target_clones("avx512f", "avx2", "default")))
int64_t row_min(const int64_t* cr, int64_t pk, const int64_t* pl, int len) {
  int64_t v = std::numeric_limits<int64_t>::max();
  for (int j = 0; j < len; ++j) v = std::min(v, cr[j] + pk - pl[j]);
  return v;
}
// The same with the costs stored in 32 bits (half the bytes streamed).
__attribute__((target_clones("avx512f", "avx2", "default")))
int64_t row_min(const int32_t* cr, int64_t pk, const int64_t* pl, int len) {
  int64_t v = std::numeric_limits<int64_t>::max();
  for (int j = 0; j < len; ++j) v = std::min(v, (int64_t)cr[j] + pk - pl[j]);
  return v;
}
// Eight independent running minima so that the loop vectorises: a minimum
// is exact, so the grouping cannot change the result.
__attribute__((target_clones("avx512f", "avx2", "default")))
double row_min(const double* cr, double pk, const double* pl, int len) {
  constexpr double inf = std::numeric_limits<double>::infinity();
  double v[8] = {inf, inf, inf, inf, inf, inf, inf, inf};
  int j = 0;
  for (; j + 8 <= len; j += 8)
    for (int u = 0; u < 8; ++u) {
      const double r = cr[j + u] + pk - pl[j + u];
      v[u] = r < v[u] ? r : v[u];
    }
  double w = inf;
  for (; j < len; ++j) {
    const double r = cr[j] + pk - pl[j];
    w = r < w ? r : w;
  }
  for (int u = 0; u < 8; ++u) w = v[u] < w ? v[u] : w;
  return w;
}

// Cost: arithmetic of costs and potentials; Stored: how the cost matrix is
// held (32-bit integers when every cost fits, to halve the pricing stream).
template <typename Cost, typename Stored = Cost>
struct TransportSimplex {
  // Problem: n sources (supply s_k > 0), m sinks (demand t_l > 0), dense
  // cost c[k*m + l].  Nodes 0..n-1 sources, n..n+m-1 sinks, root = n+m.
  int n, m, root;
  const Stored* c;
  std::vector<int64_t> supply;  // +s for sources, -t for sinks, 0 for the root
  Cost art;                     // cost of artificial arcs

  struct Edge {
    int a, b;        // arc a -> b
    int64_t arc;     // real arc id k*m + l, or -1 for an artificial arc
    int64_t flow;
  };
  std::vector<Edge> edges;  // tree edges (n + m of them)
  // Spanning tree: parent and the edge to it (pred); a circular preorder list
  // (thread / rthread) with, per node, its subtree size and the last node of
  // its subtree in that order.  A subtree is a contiguous run of the list.
  std::vector<int> parent, pred, thread, rthread, size, last;
  std::vector<Cost> pi;
  std::vector<int> path;
  std::vector<std::pair<int, int>> runs;  // (first, last) node of each run
  int64_t next_arc = 0;
  int64_t pivots = 0;

  Cost arc_cost(const Edge& e) const { return e.arc >= 0 ? Cost(c[e.arc]) : art; }

  void init() {
    const int N = n + m + 1;
    root = n + m;
    parent.assign(N, -1);
    pred.assign(N, -1);
    thread.assign(N, 0);
    rthread.assign(N, 0);
    size.assign(N, 1);
    last.assign(N, 0);
    pi.assign(N, Cost(0));
    edges.clear();
    for (int v = 0; v < n + m; ++v) {
      Edge e;
      if (v < n) { e.a = v; e.b = root; e.flow = supply[v]; }
      else       { e.a = root; e.b = v; e.flow = -supply[v]; }
      e.arc = -1;
      pred[v] = (int)edges.size();
      edges.push_back(e);
      parent[v] = root;
      last[v] = v;
      // tree arcs have zero reduced cost: cost + pi[a] - pi[b] = 0
      pi[v] = (v < n) ? Cost(-art) : art;
    }
    // preorder: root, 0, 1, ..., n+m-1, back to root
    for (int v = 0; v < N; ++v) {
      const int nx = v == root ? 0 : (v + 1 == n + m ? root : v + 1);
      thread[v] = nx;
      rthread[nx] = v;
    }
    size[root] = N;
    last[root] = n + m - 1;
  }

  Cost reduced(int64_t arc) const {
    int k = (int)(arc / m), l = (int)(arc % m);
    return Cost(c[arc]) + pi[k] - pi[n + l];
  }

  // Block search pricing: scan arcs cyclically in blocks of about sqrt(n m),
  // return the most negative reduced cost of the first block that has one
  // (lowest arc in scan order on ties).  Arcs are visited row by row, so the
  // inner loop runs over one contiguous cost row with one source potential.
  int64_t find_entering(Cost eps) {
    const int64_t A = (int64_t)n * m;
    const int64_t block = std::max<int64_t>(64, (int64_t)std::sqrt((double)A));
    const Cost* pl = pi.data() + n;
    int k = (int)(next_arc / m), l = (int)(next_arc % m);
    for (int64_t scanned = 0; scanned < A;) {
      const int64_t len = std::min(block, A - scanned);
      Cost best = -eps;
      int bk = -1, bl = -1;
      for (int64_t left = len; left > 0;) {
        const int seg = (int)std::min<int64_t>(left, m - l);
        const Stored* cr = c + (int64_t)k * m;
        const Cost pk = pi[k];
        const Cost smin = row_min(cr + l, pk, pl + l, seg);
        if (smin < best) {
          int j = l;
          while (Cost(cr[j]) + pk - pl[j] != smin) ++j;   // first arc attaining it
          best = smin; bk = k; bl = j;
        }
        left -= seg;
        l += seg;
        if (l == m) { l = 0; if (++k == n) k = 0; }
      }
      scanned += len;
      if (bk >= 0) {
        next_arc = (int64_t)k * m + l;
        return (int64_t)bk * m + bl;
      }
    }
    return -1;
  }

  bool up(int v) const { return edges[pred[v]].a == v; }  // pred edge points v -> parent

  void pivot(int64_t in_arc) {
    const int first = (int)(in_arc / m), second = n + (int)(in_arc % m);
    // join node of the cycle: climb from the endpoint with the smaller
    // subtree (an ancestor always has the larger one)
    int u = first, v = second;
    while (u != v) {
      if (size[u] < size[v]) u = parent[u];
      else v = parent[v];
    }
    const int join = u;
    // leaving edge: the cycle runs first -> second -> ... -> join -> ... -> first
    int64_t delta = std::numeric_limits<int64_t>::max();
    int out = -1;        // node whose pred edge leaves
    bool out_first = false;
    for (int x = first; x != join; x = parent[x]) {
      if (up(x)) {       // traversed backwards: limited by its flow
        int64_t d = edges[pred[x]].flow;
        if (d < delta) { delta = d; out = x; out_first = true; }
      }
    }
    for (int x = second; x != join; x = parent[x]) {
      if (!up(x)) {
        int64_t d = edges[pred[x]].flow;
        if (d <= delta) { delta = d; out = x; out_first = false; }
      }
    }
    // push delta around the cycle
    if (delta > 0) {
      for (int x = first; x != join; x = parent[x])
        edges[pred[x]].flow += up(x) ? -delta : delta;
      for (int x = second; x != join; x = parent[x])
        edges[pred[x]].flow += up(x) ? delta : -delta;
    }
    // The subtree S below `out` is cut off and re-hung, rooted at the
    // entering arc's endpoint inside it, below the other endpoint.
    const int u_in = out_first ? first : second;   // endpoint inside S
    const int v_in = out_first ? second : first;   // endpoint outside S
    const int eid = pred[out];
    const int pout = parent[out];
    const int nS = size[out];
    // path u_in = w_0, w_1, ..., w_k = out
    path.clear();
    for (int x = u_in; ; x = parent[x]) { path.push_back(x); if (x == out) break; }
    // S in its new preorder is a sequence of runs of the old list: the
    // subtree of w_0, then for each i >= 1 the run of w_i's subtree with the
    // run of w_{i-1}'s subtree taken out (w_i up to just before w_{i-1}, and
    // what follows w_{i-1}'s subtree up to w_i's last node, if anything).
    // Each run keeps its inner links; only the run ends are relinked.
    runs.clear();
    runs.push_back({u_in, last[u_in]});
    for (size_t i = 1; i < path.size(); ++i) {
      const int w = path[i], wc = path[i - 1];
      runs.push_back({w, rthread[wc]});
      if (last[wc] != last[w]) runs.push_back({thread[last[wc]], last[w]});
    }
    const int lastS = runs.back().second;
    // unlink S's old run from the preorder and fix the subtree ends above it
    {
      const int before = rthread[out], after = thread[last[out]];
      thread[before] = after;
      rthread[after] = before;
      const int oldlast = last[out];
      for (int a = pout; a >= 0 && last[a] == oldlast; a = parent[a]) last[a] = before;
    }
    for (int a = pout; a != join; a = parent[a]) size[a] -= nS;
    // link S's new run right after v_in
    {
      const int after = thread[v_in];
      int prev = v_in;
      for (const auto& r : runs) { thread[prev] = r.first; rthread[r.first] = prev; prev = r.second; }
      thread[lastS] = after;
      rthread[after] = lastS;
      for (int a = v_in; a >= 0 && last[a] == v_in; a = parent[a]) last[a] = lastS;
    }
    for (int a = v_in; a != join; a = parent[a]) size[a] += nS;
    // re-root S along the path (sizes and preds from the old values, top down)
    for (size_t i = path.size() - 1; i >= 1; --i) {
      const int w = path[i], wc = path[i - 1];
      size[w] = nS - size[wc];
      parent[w] = wc;
      pred[w] = pred[wc];
      last[w] = lastS;
    }
    size[u_in] = nS;
    last[u_in] = lastS;
    parent[u_in] = v_in;
    pred[u_in] = eid;
    Edge& E = edges[eid];
    E.a = first; E.b = second; E.arc = in_arc; E.flow = delta;
    // potentials of S shift so that the entering arc has zero reduced cost
    // (first in S: pi[first] -= rc).  Reduced costs only see differences, and
    // a constant added to every potential cancels in the returned duals, so
    // with integer costs the other side is shifted instead when it is the
    // smaller one (floating-point potentials always shift S, so that their
    // rounding does not depend on which side is smaller).
    const Cost rc = Cost(c[in_arc]) + pi[first] - pi[second];
    const Cost sigma = out_first ? Cost(-rc) : rc;
    if (std::is_integral<Cost>::value && 2 * nS > n + m + 1) {
      for (int x = thread[lastS]; x != u_in; x = thread[x]) pi[x] -= sigma;
    } else {
      for (int x = u_in; ; x = thread[x]) { pi[x] += sigma; if (x == lastS) break; }
    }
    ++pivots;
  }

  bool solve(int64_t max_pivots, Cost eps) {
    init();
    for (;;) {
      int64_t e = find_entering(eps);
      if (e < 0) return true;
      if (pivots >= max_pivots) return false;
      pivot(e);
    }
  }

  // Pricing over a candidate subset of the arcs (source k, sink l), cyclic
  // blocks of about sqrt(size) candidates, most negative reduced cost of the
  // first block that has one (first in scan order on ties).
  std::vector<int> ck, cl;
  size_t next_cand = 0;
  int64_t find_entering_sparse(Cost eps) {
    const size_t A = ck.size();
    if (!A) return -1;
    const size_t block = std::max<size_t>(64, (size_t)std::sqrt((double)A));
    size_t pos = next_cand % A;
    for (size_t scanned = 0; scanned < A;) {
      const size_t len = std::min(block, A - scanned);
      Cost best = -eps;
      int64_t barc = -1;
      for (size_t q = 0; q < len; ++q) {
        const int k = ck[pos], l = cl[pos];
        const int64_t a = (int64_t)k * m + l;
        const Cost r = Cost(c[a]) + pi[k] - pi[n + l];
        if (r < best) { best = r; barc = a; }
        if (++pos == A) pos = 0;
      }
      scanned += len;
      if (barc >= 0) { next_cand = pos; return barc; }
    }
    return -1;
  }

  // Arcs of the whole dense set with a reduced cost below -eps, appended to
  // the candidates; returns how many.
  int64_t add_violators(Cost eps) {
    const Cost* pl = pi.data() + n;
    int64_t added = 0;
    for (int k = 0; k < n; ++k) {
      const Stored* cr = c + (int64_t)k * m;
      const Cost pk = pi[k];
      if (!(row_min(cr, pk, pl, m) < -eps)) continue;
      for (int l = 0; l < m; ++l)
        if (Cost(cr[l]) + pk - pl[l] < -eps) { ck.push_back(k); cl.push_back(l); ++added; }
    }
    return added;
  }

  // Optimal on the candidate arcs, then checked against every arc: arcs with
  // a negative reduced cost join the candidates and pivoting continues from
  // the current tree, until no arc of the dense set prices out (the basis is
  // then optimal for the whole problem, whatever the first candidates were).
  bool solve_sparse(int64_t max_pivots, Cost eps, int* rounds) {
    init();
    for (*rounds = 1;; ++*rounds) {
      for (;;) {
        const int64_t e = find_entering_sparse(eps);
        if (e < 0) break;
        if (pivots >= max_pivots) return false;
        pivot(e);
      }
      if (add_violators(eps) == 0) return true;
    }
  }
};

template <typename Cost, typename Stored = Cost>
int solve_typed(int n, int m, const Stored* cost, const double* a, const double* b,
                const std::vector<int>& src_ids, const std::vector<int>& dst_ids,
                CoarseSolution* out, Cost eps, const std::vector<std::pair<int, int>>* cand = nullptr) {
  TransportSimplex<Cost, Stored> S;
  S.n = n; S.m = m; S.c = cost;
  if (cand) {
    S.ck.reserve(cand->size());
    S.cl.reserve(cand->size());
    for (const auto& kl : *cand) { S.ck.push_back(kl.first); S.cl.push_back(kl.second); }
  }
  // integerise supplies
  const double scale = 4503599627370496.0;  // 2^52
  double ta = 0, tb = 0;
  for (int i = 0; i < n; ++i) ta += a[i];
  for (int j = 0; j < m; ++j) tb += b[j];
  S.supply.assign(n + m + 1, 0);
  int64_t sa = 0, sb = 0;
  int ia = 0, ib = 0;
  for (int i = 0; i < n; ++i) {
    int64_t v = std::max<int64_t>(1, (int64_t)std::llround(a[i] / ta * scale));
    S.supply[i] = v; sa += v;
    if (a[i] > a[ia]) ia = i;
  }
  for (int j = 0; j < m; ++j) {
    int64_t v = std::max<int64_t>(1, (int64_t)std::llround(b[j] / tb * scale));
    S.supply[n + j] = -v; sb += v;
    if (b[j] > b[ib]) ib = j;
  }
  // balance exactly on the larger side's largest entry
  if (sa > sb) S.supply[ia] -= (sa - sb);
  else if (sb > sa) S.supply[n + ib] += (sb - sa);
  Cost cmax = 0;
  for (int64_t e = 0; e < (int64_t)n * m; ++e) cmax = std::max(cmax, Cost(cost[e]));
  S.art = (cmax + 1) * (Cost)(n + m + 1);
  const int64_t max_pivots = int64_t(200) * (n + m) * (n + m) + 100000;
  if (cand) {
    int rounds = 0;
    if (!S.solve_sparse(max_pivots, eps, &rounds)) return QBW_E_LP;
    out->rounds = rounds;
  } else if (!S.solve(max_pivots, eps)) {
    return QBW_E_LP;
  }
  // every artificial arc must carry no flow
  for (const auto& e : S.edges)
    if (e.arc < 0 && e.flow != 0) return QBW_E_LP;
  out->pivots = S.pivots;
  // float64 flows from the tree: peel leaves in reverse preorder
  const int NN = n + m + 1;
  std::vector<int> order;
  order.reserve(NN);
  for (int x = S.root; ; ) { order.push_back(x); x = S.thread[x]; if (x == S.root) break; }
  if ((int)order.size() != NN) return QBW_E_LP;
  std::vector<double> ex(NN, 0.0);
  for (int i = 0; i < n; ++i) ex[i] = a[i];
  for (int j = 0; j < m; ++j) ex[n + j] = -b[j];
  std::vector<double> fl(S.edges.size(), 0.0);
  for (int qi = (int)order.size() - 1; qi > 0; --qi) {
    int x = order[qi];
    int id = S.pred[x];
    const auto& ed = S.edges[id];
    fl[id] = (ed.a == x) ? ex[x] : -ex[x];
    ex[S.parent[x]] += ex[x];
  }
  out->rows.clear(); out->cols.clear(); out->vals.clear();
  for (size_t id = 0; id < S.edges.size(); ++id) {
    const auto& ed = S.edges[id];
    if (ed.arc < 0) continue;
    double v = fl[id];
    if (!(v > 0)) continue;
    out->rows.push_back(src_ids[(int)(ed.arc / m)]);
    out->cols.push_back(dst_ids[(int)(ed.arc % m)]);
    out->vals.push_back(v);
  }
  // duals
  for (int i = 0; i < n; ++i) out->f[src_ids[i]] = -(double)S.pi[i];
  for (int j = 0; j < m; ++j) out->g[dst_ids[j]] = (double)S.pi[n + j];
  return QBW_OK;
}

}  // namespace

// `cand` (may be null): candidate block pairs (source block, target block) for
// pricing first; the solve still ends optimal for every pair.
static int coarse_solve_cand(const CoarseProblem& P, const std::vector<std::pair<int, int>>* cand_blocks,
                             CoarseSolution* out) {
  const int Q = P.Q;
  std::vector<int> src, dst;
  for (int i = 0; i < Q; ++i) if (P.mu[i] > 0) src.push_back(i);
  for (int j = 0; j < Q; ++j) if (P.nu[j] > 0) dst.push_back(j);
  if (src.empty() || dst.empty()) return QBW_E_MASS;
  const int n = (int)src.size(), m = (int)dst.size();
  std::vector<double> a(n), b(m);
  for (int i = 0; i < n; ++i) a[i] = P.mu[src[i]];
  for (int j = 0; j < m; ++j) b[j] = P.nu[dst[j]];
  // candidates in the solver's numbering (blocks of zero mass are not in the LP)
  std::vector<std::pair<int, int>> cand;
  const std::vector<std::pair<int, int>>* cp = nullptr;
  if (cand_blocks) {
    std::vector<int> si(Q, -1), di(Q, -1);
    for (int i = 0; i < n; ++i) si[src[i]] = i;
    for (int j = 0; j < m; ++j) di[dst[j]] = j;
    cand.reserve(cand_blocks->size());
    for (const auto& kl : *cand_blocks)
      if (si[kl.first] >= 0 && di[kl.second] >= 0) cand.push_back({si[kl.first], di[kl.second]});
    cp = &cand;
  }
  out->f.assign(Q, 0.0);
  out->g.assign(Q, 0.0);
  std::vector<char> fset(Q, 0), gset(Q, 0);
  int rc;
  if (P.integer_cost) {
    // integer costs are held in 32 bits when they all fit (arithmetic stays 64-bit)
    double cm = 0;
    for (int i : src)
      for (int j : dst) cm = std::max(cm, std::fabs(P.cost[(size_t)i * Q + j]));
    if (std::llround(cm) <= std::numeric_limits<int32_t>::max()) {
      std::vector<int32_t> c((size_t)n * m);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) c[(size_t)i * m + j] = (int32_t)std::llround(P.cost[(size_t)src[i] * Q + dst[j]]);
      rc = solve_typed<int64_t, int32_t>(n, m, c.data(), a.data(), b.data(), src, dst, out, 0, cp);
    } else {
      std::vector<int64_t> c((size_t)n * m);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) c[(size_t)i * m + j] = (int64_t)std::llround(P.cost[(size_t)src[i] * Q + dst[j]]);
      rc = solve_typed<int64_t>(n, m, c.data(), a.data(), b.data(), src, dst, out, 0, cp);
    }
  } else {
    std::vector<double> c((size_t)n * m);
    double cm = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < m; ++j) {
        c[(size_t)i * m + j] = P.cost[(size_t)src[i] * Q + dst[j]];
        cm = std::max(cm, c[(size_t)i * m + j]);
      }
    rc = solve_typed<double>(n, m, c.data(), a.data(), b.data(), src, dst, out, 1e-11 * (cm + 1.0), cp);
  }
  if (rc != QBW_OK) return rc;
  for (int i : src) fset[i] = 1;
  for (int j : dst) gset[j] = 1;
  // complete potentials of empty blocks by c-transforms (keeps admissibility)
  for (int k = 0; k < Q; ++k) {
    if (fset[k]) continue;
    double best = std::numeric_limits<double>::infinity();
    for (int j : dst) best = std::min(best, P.cost[(size_t)k * Q + j] - out->g[j]);
    out->f[k] = best;
  }
  for (int l = 0; l < Q; ++l) {
    if (gset[l]) continue;
    double best = std::numeric_limits<double>::infinity();
    for (int k = 0; k < Q; ++k) best = std::min(best, P.cost[(size_t)k * Q + l] - out->f[k]);
    out->g[l] = best;
  }
  // normalise: sum_k mu~_k f~_k = 0
  double tot = 0, s = 0;
  for (int k = 0; k < Q; ++k) { s += P.mu[k] * out->f[k]; tot += P.mu[k]; }
  double shift = s / tot;
  if (P.integer_cost) shift = std::nearbyint(shift);   // keep integer duals integer
  for (int k = 0; k < Q; ++k) out->f[k] -= shift;
  for (int l = 0; l < Q; ++l) out->g[l] += shift;
  double obj = 0;
  for (size_t e = 0; e < out->vals.size(); ++e)
    obj += out->vals[e] * P.cost[(size_t)out->rows[e] * Q + out->cols[e]];
  out->objective = obj;
  return QBW_OK;
}

int coarse_solve(const CoarseProblem& P, CoarseSolution* out) { return coarse_solve_cand(P, nullptr, out); }

// Multiscale start (coarse-to-fine, as the paper suggests for the coarse solve
// itself): the problem on the n^d blocks is pooled once more, 2^d blocks to
// one, and solved (recursively, down to a few hundred blocks); the pairs of
// children of that solution's support are priced first.  (Widening each
// target to its 3^d neighbours made the first set larger and the solve
// slower: the arcs the start set lacks come in through the checks.)  The result is optimal for the whole
// dense problem: the solve only stops when no block pair has a negative
// reduced cost (solve_sparse), so the start set affects the time, not the
// objective.
int coarse_solve_multiscale(const CoarseProblem& P, int n, int d, int p, CoarseSolution* out) {
  const int Q = P.Q;
  if (n % 2 != 0 || Q <= kMultiscaleMinQ) return coarse_solve(P, out);
  const int h = n / 2;
  const int Q2 = d == 2 ? h * h : h * h * h;
  auto coords = [&](int K, int side, int* x) {
    for (int a = d - 1; a >= 0; --a) { x[a] = K % side; K /= side; }
  };
  auto index = [&](const int* x, int side) {
    int K = 0;
    for (int a = 0; a < d; ++a) K = K * side + x[a];
    return K;
  };
  // pooled masses and a cost of the same form on the half-resolution blocks
  std::vector<double> mu2(Q2, 0.0), nu2(Q2, 0.0);
  for (int K = 0; K < Q; ++K) {
    int x[3];
    coords(K, n, x);
    for (int a = 0; a < d; ++a) x[a] /= 2;
    const int K2 = index(x, h);
    mu2[K2] += P.mu[K];
    nu2[K2] += P.nu[K];
  }
  std::vector<double> C2((size_t)Q2 * Q2);
  for (int K = 0; K < Q2; ++K) {
    int x[3];
    coords(K, h, x);
    for (int L = 0; L < Q2; ++L) {
      int y[3];
      coords(L, h, y);
      long long d2 = 0;
      for (int a = 0; a < d; ++a) d2 += (long long)(x[a] - y[a]) * (x[a] - y[a]);
      C2[(size_t)K * Q2 + L] = p == 2 ? (double)d2 : std::sqrt((double)d2);
    }
  }
  CoarseProblem P2{Q2, mu2.data(), nu2.data(), C2.data(), p == 2};
  CoarseSolution s2;
  int rc = coarse_solve_multiscale(P2, h, d, p, &s2);
  if (rc != QBW_OK) return coarse_solve(P, out);
  // candidate pairs: the children of the support's block pairs
  const int nc = 1 << d;
  std::vector<std::vector<int>> tg(Q);
  for (size_t e = 0; e < s2.vals.size(); ++e) {
    int xs[3], xt[3];
    coords(s2.rows[e], h, xs);
    coords(s2.cols[e], h, xt);
    for (int cs = 0; cs < nc; ++cs) {
      int u[3];
      for (int a = 0; a < d; ++a) u[a] = 2 * xs[a] + ((cs >> a) & 1);
      std::vector<int>& T = tg[index(u, n)];
      for (int ct = 0; ct < nc; ++ct) {
        int v[3];
        for (int a = 0; a < d; ++a) v[a] = 2 * xt[a] + ((ct >> a) & 1);
        T.push_back(index(v, n));
      }
    }
  }
  std::vector<std::pair<int, int>> cand;
  for (int K = 0; K < Q; ++K) {
    std::vector<int>& T = tg[K];
    std::sort(T.begin(), T.end());
    T.erase(std::unique(T.begin(), T.end()), T.end());
    for (int L : T) cand.push_back({K, L});
  }
  rc = coarse_solve_cand(P, &cand, out);
  if (rc == QBW_OK) out->pivots += s2.pivots;
  return rc;
}

}  // namespace qbw
