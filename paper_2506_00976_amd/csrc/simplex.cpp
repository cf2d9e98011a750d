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
#include <vector>

#include "qbw_internal.h"

namespace qbw {

namespace {

template <typename Cost>
struct TransportSimplex {
  // Problem: n sources (supply s_k > 0), m sinks (demand t_l > 0), dense
  // cost c[k*m + l].  Nodes 0..n-1 sources, n..n+m-1 sinks, root = n+m.
  int n, m, root;
  const Cost* c;
  std::vector<int64_t> supply;  // +s for sources, -t for sinks, 0 for the root
  Cost art;                     // cost of artificial arcs

  struct Edge {
    int a, b;        // arc a -> b
    int64_t arc;     // real arc id k*m + l, or -1 for an artificial arc
    int64_t flow;
  };
  std::vector<Edge> edges;                 // tree edges (n + m of them)
  std::vector<int> parent, pred, depth;    // pred = edge index to the parent
  std::vector<Cost> pi;
  std::vector<std::vector<int>> adj;       // tree edges incident to each node
  std::vector<int> queue;
  int64_t next_arc = 0;
  int64_t pivots = 0;

  Cost arc_cost(const Edge& e) const { return e.arc >= 0 ? c[e.arc] : art; }

  void init() {
    const int N = n + m + 1;
    root = n + m;
    parent.assign(N, -1);
    pred.assign(N, -1);
    depth.assign(N, 0);
    pi.assign(N, Cost(0));
    adj.assign(N, {});
    edges.clear();
    for (int v = 0; v < n + m; ++v) {
      Edge e;
      if (v < n) { e.a = v; e.b = root; e.flow = supply[v]; }
      else       { e.a = root; e.b = v; e.flow = -supply[v]; }
      e.arc = -1;
      int id = (int)edges.size();
      edges.push_back(e);
      parent[v] = root;
      pred[v] = id;
      depth[v] = 1;
      // tree arcs have zero reduced cost: cost + pi[a] - pi[b] = 0
      pi[v] = (v < n) ? Cost(-art) : art;
      adj[v].push_back(id);
      adj[root].push_back(id);
    }
  }

  Cost reduced(int64_t arc) const {
    int k = (int)(arc / m), l = (int)(arc % m);
    return c[arc] + pi[k] - pi[n + l];
  }

  // Block search pricing: scan arcs cyclically in blocks, return the most
  // negative reduced cost found in the first block that has one.
  int64_t find_entering(Cost eps) {
    const int64_t A = (int64_t)n * m;
    int64_t block = std::max<int64_t>(64, (int64_t)std::sqrt((double)A));
    Cost best = -eps;
    int64_t best_arc = -1, cnt = 0;
    int64_t e = next_arc;
    for (int64_t scanned = 0; scanned < A; ++scanned) {
      int k = (int)(e / m), l = (int)(e % m);
      Cost rc = c[e] + pi[k] - pi[n + l];
      if (rc < best) { best = rc; best_arc = e; }
      if (++cnt == block) {
        if (best_arc >= 0) { next_arc = e + 1 == A ? 0 : e + 1; return best_arc; }
        cnt = 0;
      }
      if (++e == A) e = 0;
    }
    if (best_arc >= 0) next_arc = best_arc + 1 == A ? 0 : best_arc + 1;
    return best_arc;
  }

  bool up(int v) const { return edges[pred[v]].a == v; }  // pred edge points v -> parent

  void pivot(int64_t in_arc) {
    const int first = (int)(in_arc / m), second = n + (int)(in_arc % m);
    // join node of the cycle
    int u = first, v = second;
    while (u != v) {
      if (depth[u] > depth[v]) u = parent[u];
      else if (depth[v] > depth[u]) v = parent[v];
      else { u = parent[u]; v = parent[v]; }
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
    // replace the leaving edge by the entering arc
    const int eid = pred[out];
    const int pout = parent[out];
    auto& ao = adj[out];
    ao.erase(std::find(ao.begin(), ao.end(), eid));
    auto& ap = adj[pout];
    ap.erase(std::find(ap.begin(), ap.end(), eid));
    // subtree S hanging below `out` contains `first` or `second`
    const int u_in = out_first ? first : second;   // endpoint inside S
    const int v_in = out_first ? second : first;   // endpoint outside S
    Edge& E = edges[eid];
    E.a = first; E.b = second; E.arc = in_arc; E.flow = delta;
    adj[u_in].push_back(eid);
    adj[v_in].push_back(eid);
    // potentials of S shift so that the entering arc has zero reduced cost
    const Cost rc = c[in_arc] + pi[first] - pi[second];
    const Cost sigma = out_first ? Cost(-rc) : rc;   // first in S: pi[first] -= rc
    parent[u_in] = v_in;
    pred[u_in] = eid;
    depth[u_in] = depth[v_in] + 1;
    pi[u_in] += sigma;
    queue.clear();
    queue.push_back(u_in);
    for (size_t qi = 0; qi < queue.size(); ++qi) {
      const int x = queue[qi];
      for (int id : adj[x]) {
        if (id == pred[x]) continue;
        const Edge& ed = edges[id];
        const int y = ed.a == x ? ed.b : ed.a;
        parent[y] = x;
        pred[y] = id;
        depth[y] = depth[x] + 1;
        pi[y] += sigma;
        queue.push_back(y);
      }
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
};

template <typename Cost>
int solve_typed(int n, int m, const Cost* cost, const double* a, const double* b,
                const std::vector<int>& src_ids, const std::vector<int>& dst_ids,
                CoarseSolution* out, Cost eps) {
  TransportSimplex<Cost> S;
  S.n = n; S.m = m; S.c = cost;
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
  for (int64_t e = 0; e < (int64_t)n * m; ++e) cmax = std::max(cmax, cost[e]);
  S.art = (cmax + 1) * (Cost)(n + m + 1);
  if (!S.solve(int64_t(200) * (n + m) * (n + m) + 100000, eps)) return QBW_E_LP;
  // every artificial arc must carry no flow
  for (const auto& e : S.edges)
    if (e.arc < 0 && e.flow != 0) return QBW_E_LP;
  out->pivots = S.pivots;
  // float64 flows from the tree: peel leaves in reverse BFS order from the root
  const int NN = n + m + 1;
  std::vector<int> order;
  order.reserve(NN);
  order.push_back(S.root);
  std::vector<int> par(NN, -1);
  par[S.root] = S.root;
  for (size_t qi = 0; qi < order.size(); ++qi) {
    int x = order[qi];
    for (int id : S.adj[x]) {
      const auto& ed = S.edges[id];
      int y = ed.a == x ? ed.b : ed.a;
      if (par[y] >= 0) continue;
      par[y] = x;
      order.push_back(y);
    }
  }
  std::vector<double> ex(NN, 0.0);
  for (int i = 0; i < n; ++i) ex[i] = a[i];
  for (int j = 0; j < m; ++j) ex[n + j] = -b[j];
  std::vector<double> fl(S.edges.size(), 0.0);
  for (int qi = (int)order.size() - 1; qi > 0; --qi) {
    int x = order[qi];
    int id = S.pred[x];
    const auto& ed = S.edges[id];
    fl[id] = (ed.a == x) ? ex[x] : -ex[x];
    ex[par[x]] += ex[x];
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

int coarse_solve(const CoarseProblem& P, CoarseSolution* out) {
  const int Q = P.Q;
  std::vector<int> src, dst;
  for (int i = 0; i < Q; ++i) if (P.mu[i] > 0) src.push_back(i);
  for (int j = 0; j < Q; ++j) if (P.nu[j] > 0) dst.push_back(j);
  if (src.empty() || dst.empty()) return QBW_E_MASS;
  const int n = (int)src.size(), m = (int)dst.size();
  std::vector<double> a(n), b(m);
  for (int i = 0; i < n; ++i) a[i] = P.mu[src[i]];
  for (int j = 0; j < m; ++j) b[j] = P.nu[dst[j]];
  out->f.assign(Q, 0.0);
  out->g.assign(Q, 0.0);
  std::vector<char> fset(Q, 0), gset(Q, 0);
  int rc;
  if (P.integer_cost) {
    std::vector<int64_t> c((size_t)n * m);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < m; ++j) c[(size_t)i * m + j] = (int64_t)std::llround(P.cost[(size_t)src[i] * Q + dst[j]]);
    rc = solve_typed<int64_t>(n, m, c.data(), a.data(), b.data(), src, dst, out, 0);
  } else {
    std::vector<double> c((size_t)n * m);
    double cm = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < m; ++j) {
        c[(size_t)i * m + j] = P.cost[(size_t)src[i] * Q + dst[j]];
        cm = std::max(cm, c[(size_t)i * m + j]);
      }
    rc = solve_typed<double>(n, m, c.data(), a.data(), b.data(), src, dst, out, 1e-11 * (cm + 1.0));
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

}  // namespace qbw
