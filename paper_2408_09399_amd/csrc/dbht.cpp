// DBHT clustering of a finished TMFG, on the host (Section 2, Background: the directed
// bubble hierarchy tree; Section 5, Evaluation: the dendrogram cut into as many clusters as
// the ground truth has).
//
// Steps: shortest paths on the TMFG with edge lengths sqrt(2 (1 - W)) (one Dijkstra per
// source, sources spread over threads); the bubble tree read off the insertion record (the
// seed clique and one bubble per insertion, each joined to the bubble that made the face it
// split); each tree edge pointed to the side whose vertices are more strongly tied to the
// separating triangle; converging bubbles (no outgoing edge); each vertex's group (the
// reachable converging bubble its TMFG edges favour) and bubble (the containing bubble that
// reaches its group, nearest by summed path lengths); complete linkage over the path lengths,
// first inside each (group, bubble) cell, then over the cells of each group, then over the
// groups; the cut. Every choice that the paper leaves open is fixed in tmfg.h, and every
// floating-point sum runs in a fixed order, so the result is one well-defined record.
#include "../../include/tmfg.h"
#include "common.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <queue>
#include <thread>
#include <tuple>
#include <vector>

namespace {

struct Graph {
  std::vector<int> off, nbr;      // CSR, neighbours ascending
  std::vector<double> len;        // edge length per CSR entry
};

Graph make_graph(int n, const float* W, const int32_t* edges, int ne) {
  std::vector<std::vector<int>> adj(n);
  for (int e = 0; e < ne; ++e) {
    const int a = edges[2 * e], b = edges[2 * e + 1];
    adj[a].push_back(b);
    adj[b].push_back(a);
  }
  Graph G;
  G.off.assign(n + 1, 0);
  for (int v = 0; v < n; ++v) {
    std::sort(adj[v].begin(), adj[v].end());
    adj[v].erase(std::unique(adj[v].begin(), adj[v].end()), adj[v].end());
    G.off[v + 1] = G.off[v] + (int)adj[v].size();
  }
  G.nbr.resize(G.off[n]);
  G.len.resize(G.off[n]);
  for (int v = 0; v < n; ++v)
    for (int q = 0; q < (int)adj[v].size(); ++q) {
      const int w = adj[v][q];
      G.nbr[G.off[v] + q] = w;
      G.len[G.off[v] + q] = std::sqrt(2.0 * std::max(1.0 - (double)W[(size_t)v * n + w], 0.0));
    }
  return G;
}

bool adjacent(const Graph& G, int v, int w) {
  return std::binary_search(G.nbr.begin() + G.off[v], G.nbr.begin() + G.off[v + 1], w);
}

// One source: distances are the smallest path sums taken from the source outward.
void dijkstra(const Graph& G, int n, int s, double* dist) {
  std::fill(dist, dist + n, INFINITY);
  std::vector<char> done(n, 0);
  using Item = std::pair<double, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> h;
  dist[s] = 0.0;
  h.push({0.0, s});
  while (!h.empty()) {
    const auto [d, v] = h.top();
    h.pop();
    if (done[v]) continue;
    done[v] = 1;
    for (int q = G.off[v]; q < G.off[v + 1]; ++q) {
      const int w = G.nbr[q];
      const double nd = d + G.len[q];
      if (nd < dist[w]) {
        dist[w] = nd;
        h.push({nd, w});
      }
    }
  }
}

struct Merge {
  int lo, hi;
  double d;
  int size;
};

// Complete linkage over m clusters (ids, sizes, distance matrix Dc, row-major m x m): the
// closest pair merges, ties to the lowest (smaller id, larger id); the merged cluster takes
// the next id. Returns the last cluster's id. Each slot keeps its nearest other slot; merged
// distances never shrink, so only slots whose nearest was merged need a new search.
int complete_linkage(std::vector<double>& Dc, int m, std::vector<int> ids, std::vector<int> sizes, int& next_id,
                     std::vector<Merge>& out) {
  if (m == 1) return ids[0];
  std::vector<char> alive(m, 1);
  auto key_less = [&](int a, int b, int c, int d) {     // pair (a, b) before pair (c, d)?
    const double x = Dc[(size_t)a * m + b], y = Dc[(size_t)c * m + d];
    if (x != y) return x < y;
    const int l1 = std::min(ids[a], ids[b]), h1 = std::max(ids[a], ids[b]);
    const int l2 = std::min(ids[c], ids[d]), h2 = std::max(ids[c], ids[d]);
    return l1 != l2 ? l1 < l2 : h1 < h2;
  };
  std::vector<int> nn(m, -1);
  auto find_nn = [&](int a) {
    int best = -1;
    for (int b = 0; b < m; ++b)
      if (b != a && alive[b] && (best < 0 || key_less(a, b, a, best))) best = b;
    nn[a] = best;
  };
  for (int a = 0; a < m; ++a) find_nn(a);
  for (int step = 0; step < m - 1; ++step) {
    int ba = -1;
    for (int a = 0; a < m; ++a)
      if (alive[a] && (ba < 0 || key_less(a, nn[a], ba, nn[ba]))) ba = a;
    const int a = ba, b = nn[ba];
    const double d = Dc[(size_t)a * m + b];
    out.push_back({std::min(ids[a], ids[b]), std::max(ids[a], ids[b]), d, sizes[a] + sizes[b]});
    for (int c = 0; c < m; ++c) {
      const double v = std::max(Dc[(size_t)a * m + c], Dc[(size_t)b * m + c]);
      Dc[(size_t)a * m + c] = v;
      Dc[(size_t)c * m + a] = v;
    }
    alive[b] = 0;
    ids[a] = next_id++;
    sizes[a] += sizes[b];
    for (int c = 0; c < m; ++c)
      if (alive[c] && (c == a || nn[c] == a || nn[c] == b)) find_nn(c);
  }
  for (int a = 0; a < m; ++a)
    if (alive[a]) return ids[a];
  return -1;
}

// Largest distance between every two blocks of vertices (m x m, zero diagonal).
std::vector<double> block_max(const double* D, int n, const std::vector<std::vector<int>>& blocks) {
  const int m = (int)blocks.size();
  std::vector<double> out((size_t)m * m, 0.0);
  for (int a = 0; a < m; ++a)
    for (int b = a + 1; b < m; ++b) {
      double v = -INFINITY;
      for (int i : blocks[a])
        for (int j : blocks[b]) v = std::max(v, D[(size_t)i * n + j]);
      out[(size_t)a * m + b] = out[(size_t)b * m + a] = v;
    }
  return out;
}

}  // namespace

extern "C" tmfg_status tmfg_dbht(int32_t n, const float* W, const int32_t* order, const int32_t* edges,
                                 const int32_t* steps, int32_t k, int32_t n_threads, int32_t* labels,
                                 double* linkage, int32_t* group_out, int32_t* bubble_out) {
  if (!W || !order || !edges || !labels || (n > 4 && !steps)) return TMFG_E_INVALID;
  if (n < tmfg::kMinN || n > tmfg::kMaxN || k < 1 || k > n) return TMFG_E_SIZE;
  const int ne = 3 * n - 6, ns = n - 4;
  {
    std::vector<char> seen(n, 0);
    for (int i = 0; i < n; ++i) {
      if (order[i] < 0 || order[i] >= n || seen[order[i]]) return TMFG_E_INVALID;
      seen[order[i]] = 1;
    }
    for (int i = 0; i < 2 * ne; ++i)
      if (edges[i] < 0 || edges[i] >= n) return TMFG_E_INVALID;
    for (int s = 0; s < ns; ++s) {
      if (steps[4 * s] < 0 || steps[4 * s] >= 2 * n - 4) return TMFG_E_INVALID;
      for (int j = 1; j < 4; ++j)
        if (steps[4 * s + j] < 0 || steps[4 * s + j] >= n) return TMFG_E_INVALID;
    }
  }
  const Graph G = make_graph(n, W, edges, ne);

  // Shortest paths, one Dijkstra per source.
  std::vector<double> D;
  try {
    D.resize((size_t)n * n);
  } catch (...) {
    return TMFG_E_NOMEM;
  }
  int nt = n_threads > 0 ? n_threads : (int)std::thread::hardware_concurrency();
  nt = std::max(1, std::min(nt, 64));
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&, t] {
        for (int s = t; s < n; s += nt) dijkstra(G, n, s, D.data() + (size_t)s * n);
      });
    for (auto& x : th) x.join();
  }
  // Path sums from the two ends of a pair can differ in the last bit: a pair's distance is
  // the one from its smaller id (copied into the lower triangle in 64 x 64 tiles).
  {
    constexpr int T = 64;
    const int nt_ = (n + T - 1) / T;
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&, t] {
        for (int bi = t; bi < nt_; bi += nt)
          for (int bj = bi; bj < nt_; ++bj)
            for (int i = bi * T; i < std::min(n, bi * T + T); ++i)
              for (int j = std::max(bj * T, i + 1); j < std::min(n, bj * T + T); ++j)
                D[(size_t)j * n + i] = D[(size_t)i * n + j];
      });
    for (auto& x : th) x.join();
  }

  // The bubble tree: bubble 0 is the seed, bubble s + 1 the clique of insertion s, whose
  // parent made the face that insertion split.
  const int nb = ns + 1;
  std::vector<std::array<int, 4>> bub(nb);
  std::vector<int> parent(nb, -1), creator(n, 0);
  std::vector<std::array<int, 3>> tri(nb);
  {
    std::array<int, 4> seed = {order[0], order[1], order[2], order[3]};
    std::sort(seed.begin(), seed.end());
    bub[0] = seed;
    std::vector<int> owner(2 * n, 0);
    int nfaces = 4;
    for (int s = 0; s < ns; ++s) {
      const int b = s + 1, f = steps[4 * s], u = order[4 + s];
      const int x = steps[4 * s + 1], y = steps[4 * s + 2], z = steps[4 * s + 3];
      std::array<int, 4> q = {u, x, y, z};
      std::sort(q.begin(), q.end());
      bub[b] = q;
      parent[b] = owner[f];
      tri[b] = {x, y, z};
      owner[f] = b;
      owner[nfaces] = b;
      owner[nfaces + 1] = b;
      nfaces += 2;
      creator[u] = b;
    }
  }
  std::vector<std::vector<int>> children(nb);
  for (int b = 1; b < nb; ++b) children[parent[b]].push_back(b);
  std::vector<int> tin(nb), tout(nb);
  {
    int clock = 0;
    std::vector<std::pair<int, bool>> st = {{0, false}};
    while (!st.empty()) {
      const auto [b, leaving] = st.back();
      st.pop_back();
      if (leaving) {
        tout[b] = clock;
        continue;
      }
      tin[b] = clock++;
      st.push_back({b, true});
      for (auto it = children[b].rbegin(); it != children[b].rend(); ++it) st.push_back({*it, false});
    }
  }
  // Edge directions: to the strictly stronger side, a tie to the parent.
  std::vector<char> to_child(nb, 0);
  for (int b = 1; b < nb; ++b) {
    std::array<int, 3> t = tri[b];
    std::sort(t.begin(), t.end());
    double sc = 0.0, sp = 0.0;
    for (int i : t)
      for (int q = G.off[i]; q < G.off[i + 1]; ++q) {
        const int j = G.nbr[q];
        if (j == t[0] || j == t[1] || j == t[2]) continue;
        const int c = creator[j];
        if (tin[b] <= tin[c] && tin[c] < tout[b])
          sc += (double)W[(size_t)i * n + j];
        else
          sp += (double)W[(size_t)i * n + j];
      }
    to_child[b] = sc > sp;
  }
  // Converging bubbles and the converging bubbles each bubble reaches.
  std::vector<std::vector<int>> out(nb);
  for (int b = 1; b < nb; ++b) {
    if (to_child[b])
      out[parent[b]].push_back(b);
    else
      out[b].push_back(parent[b]);
  }
  std::vector<std::vector<int>> reach(nb);
  std::vector<char> have(nb, 0);
  for (int s0 = 0; s0 < nb; ++s0) {
    if (have[s0]) continue;
    std::vector<int> st = {s0};
    while (!st.empty()) {
      const int b = st.back();
      bool pend = false;
      for (int y : out[b])
        if (!have[y]) {
          st.push_back(y);
          pend = true;
        }
      if (pend) continue;
      st.pop_back();
      if (have[b]) continue;
      if (out[b].empty()) {
        reach[b] = {b};
      } else {
        std::vector<int> r;
        for (int y : out[b]) r.insert(r.end(), reach[y].begin(), reach[y].end());
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        reach[b] = std::move(r);
      }
      have[b] = 1;
    }
  }
  // Each vertex's group and bubble.
  std::vector<std::vector<int>> homes(n);
  for (int b = 0; b < nb; ++b)
    for (int v : bub[b]) homes[v].push_back(b);
  std::vector<int> group(n), bubble(n);
  for (int v = 0; v < n; ++v) {
    std::vector<int> cands;
    for (int h : homes[v]) cands.insert(cands.end(), reach[h].begin(), reach[h].end());
    std::sort(cands.begin(), cands.end());
    cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
    int bc = -1;
    double bs = -INFINITY;
    for (int c : cands) {
      double s = 0.0;
      for (int w : bub[c])
        if (w != v && adjacent(G, v, w)) s += (double)W[(size_t)v * n + w];
      if (bc < 0 || s > bs) {
        bc = c;
        bs = s;
      }
    }
    group[v] = bc;
    int bh = -1;
    double bd = INFINITY;
    for (int h : homes[v]) {                        // ascending bubble ids
      if (!std::binary_search(reach[h].begin(), reach[h].end(), bc)) continue;
      double d = 0.0;
      for (int w : bub[h]) d += D[(size_t)v * n + w];
      if (bh < 0 || d < bd) {
        bh = h;
        bd = d;
      }
    }
    bubble[v] = bh;
  }

  // Complete linkage: cells, then the cells of each group, then the groups.
  std::vector<Merge> merges;
  merges.reserve(n - 1);
  int next_id = n;
  // vertices by (group, bubble, id): each group and each of its cells is one run
  std::vector<int> byc(n);
  std::iota(byc.begin(), byc.end(), 0);
  std::sort(byc.begin(), byc.end(), [&](int x, int y) {
    return std::tie(group[x], bubble[x], x) < std::tie(group[y], bubble[y], y);
  });
  std::vector<int> group_top;
  std::vector<std::vector<int>> group_members;
  for (int i = 0; i < n;) {
    const int g = group[byc[i]];
    int j = i;
    while (j < n && group[byc[j]] == g) ++j;
    std::vector<int> cell_top;
    std::vector<std::vector<int>> cell_members;
    for (int a = i; a < j;) {
      const int c = bubble[byc[a]];
      int b = a;
      while (b < j && bubble[byc[b]] == c) ++b;
      std::vector<int> mem(byc.begin() + a, byc.begin() + b);
      const int m = (int)mem.size();
      std::vector<double> Dc((size_t)m * m);
      for (int x = 0; x < m; ++x)
        for (int y = 0; y < m; ++y) Dc[(size_t)x * m + y] = D[(size_t)mem[x] * n + mem[y]];
      cell_top.push_back(complete_linkage(Dc, m, mem, std::vector<int>(m, 1), next_id, merges));
      cell_members.push_back(std::move(mem));
      a = b;
    }
    std::vector<double> Dc = block_max(D.data(), n, cell_members);
    std::vector<int> sz;
    for (auto& mm : cell_members) sz.push_back((int)mm.size());
    group_top.push_back(complete_linkage(Dc, (int)cell_members.size(), cell_top, sz, next_id, merges));
    std::vector<int> all(byc.begin() + i, byc.begin() + j);
    std::sort(all.begin(), all.end());
    group_members.push_back(std::move(all));
    i = j;
  }
  {
    std::vector<double> Dc = block_max(D.data(), n, group_members);
    std::vector<int> sz;
    for (auto& mm : group_members) sz.push_back((int)mm.size());
    complete_linkage(Dc, (int)group_members.size(), group_top, sz, next_id, merges);
  }
  if ((int)merges.size() != n - 1) return TMFG_E_INTERNAL;

  // The cut into k clusters: the first n - k merges; clusters numbered by smallest vertex.
  std::vector<int> uf(2 * n);
  std::iota(uf.begin(), uf.end(), 0);
  std::function<int(int)> find = [&](int x) {
    while (uf[x] != x) {
      uf[x] = uf[uf[x]];
      x = uf[x];
    }
    return x;
  };
  for (int m = 0; m < n - k; ++m) {
    uf[find(merges[m].lo)] = n + m;
    uf[find(merges[m].hi)] = n + m;
  }
  std::vector<int> first(2 * n, -1);
  int nl = 0;
  for (int v = 0; v < n; ++v) {
    const int r = find(v);
    if (first[r] < 0) first[r] = nl++;
    labels[v] = first[r];
  }
  if (linkage)
    for (int m = 0; m < n - 1; ++m) {
      linkage[4 * m] = merges[m].lo;
      linkage[4 * m + 1] = merges[m].hi;
      linkage[4 * m + 2] = merges[m].d;
      linkage[4 * m + 3] = merges[m].size;
    }
  if (group_out)
    for (int v = 0; v < n; ++v) group_out[v] = group[v];
  if (bubble_out)
    for (int v = 0; v < n; ++v) bubble_out[v] = bubble[v];
  return TMFG_OK;
}
