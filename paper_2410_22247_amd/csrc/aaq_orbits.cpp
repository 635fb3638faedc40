// Edge orbits of Aut(G) on the host (Algorithm 1 of the paper, "Automorphism-Based
// Graph Processing" section), without nauty.
//
// Algorithm 1 closes the edge list under a set of automorphism generators: scanning the
// edges in order, each edge not yet classified seeds a new class, and a breadth-first
// search adds the images of the class's edges under every generator (an image edge
// (phi(u), phi(v)) is normalised to (min, max) before lookup).  The paper takes the
// generators from nauty; here they come from an individualisation-refinement search:
// whenever two classes whose seed edges have equal colour-refinement invariants are
// still apart, the search looks for an automorphism mapping one seed onto the other,
// adds it to the generators and closes again.  The result is the orbit partition of the
// edges under the whole group Aut(G) (the group generated, the reading taken for the
// paper's "mapped onto each other via a generator").  With integer edge weights (the
// w_ij of the MaxCut H_P) the group is the weight-preserving automorphisms: refinement
// sees (neighbour colour, edge weight) pairs, a permutation must map every edge onto
// one of equal weight, and only seeds of equal weight are compared.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "aaq_launch.h"
#include "aaqaoa.h"

namespace aaq_orbits {

using Adj = std::vector<std::vector<int>>;

// colour refinement (1-dimensional Weisfeiler-Leman) to a stable colouring; wadj[v][k]
// is the weight of the edge to adj[v][k].  Colour names are canonical (ranks of sorted
// signatures), so the two copies of a disjoint union refined together get comparable
// colours
std::vector<int> refine(const Adj& adj, const Adj& wadj, std::vector<int> cur) {
  const int n = (int)adj.size();
  size_t ncls = std::set<int>(cur.begin(), cur.end()).size();
  using Sig = std::pair<int, std::vector<std::pair<int, int>>>;
  for (;;) {
    std::vector<Sig> sig(n);
    for (int v = 0; v < n; ++v) {
      sig[v].first = cur[v];
      for (size_t k = 0; k < adj[v].size(); ++k) sig[v].second.push_back({cur[adj[v][k]], wadj[v][k]});
      std::sort(sig[v].second.begin(), sig[v].second.end());
    }
    std::vector<Sig> uniq = sig;
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    std::vector<int> nxt(n);
    for (int v = 0; v < n; ++v) nxt[v] = (int)(std::lower_bound(uniq.begin(), uniq.end(), sig[v]) - uniq.begin());
    if (uniq.size() == ncls) return nxt;
    cur.swap(nxt);
    ncls = uniq.size();
  }
}

// Finds automorphisms of G that extend a partial vertex mapping: the graph and a copy
// are refined together, individualising one more vertex pair per level until every
// colour class is a singleton, which defines the mapping.
struct Searcher {
  int n;
  Adj adj, wadj, adj2, wadj2;
  std::vector<std::set<std::pair<int, int>>> nbs;  // (neighbour, edge weight)
  std::vector<int> base;                           // stable colouring of G alone (edge invariants)

  Searcher(const Adj& a, const Adj& w)
      : n((int)a.size()), adj(a), wadj(w), adj2(2 * a.size()), wadj2(2 * a.size()), nbs(a.size()) {
    for (int v = 0; v < n; ++v) {
      for (size_t k = 0; k < adj[v].size(); ++k) nbs[v].insert({adj[v][k], wadj[v][k]});
      adj2[v] = adj[v];
      wadj2[v] = wadj2[n + v] = wadj[v];
      for (int x : adj[v]) adj2[n + v].push_back(n + x);
    }
    base = refine(adj, wadj, std::vector<int>(n, 0));
  }

  bool is_automorphism(const std::vector<int>& phi) const {
    for (int v = 0; v < n; ++v) {
      std::set<std::pair<int, int>> img;
      for (size_t k = 0; k < adj[v].size(); ++k) img.insert({phi[adj[v][k]], wadj[v][k]});
      if (img != nbs[phi[v]]) return false;
    }
    return true;
  }

  bool search(std::vector<int> colors, std::vector<int>& phi) const {
    std::vector<int> col = refine(adj2, wadj2, std::move(colors));
    std::map<int, int> c0, c1;
    for (int v = 0; v < n; ++v) {
      c0[col[v]]++;
      c1[col[n + v]]++;
    }
    if (c0 != c1) return false;
    // target cell: the smallest non-singleton class (ties: smallest colour)
    int cell = -1, best = 0;
    for (auto& kv : c0)
      if (kv.second > 1 && (cell < 0 || kv.second < best)) {
        cell = kv.first;
        best = kv.second;
      }
    if (cell < 0) {
      std::map<int, int> where;
      for (int v = 0; v < n; ++v) where[col[n + v]] = v;
      phi.assign(n, 0);
      for (int v = 0; v < n; ++v) phi[v] = where[col[v]];
      return is_automorphism(phi);
    }
    int x = -1;
    for (int v = 0; v < n && x < 0; ++v)
      if (col[v] == cell) x = v;
    for (int y = 0; y < n; ++y) {
      if (col[n + y] != cell) continue;
      std::vector<int> c2(col);
      for (int& c : c2) c += 1;  // the individualised pair gets the fresh colour 0
      c2[x] = 0;
      c2[n + y] = 0;
      if (search(std::move(c2), phi)) return true;
    }
    return false;
  }

  // an automorphism phi with phi[a] = b for every pair, if one exists
  bool extend(const std::vector<std::pair<int, int>>& pairs, std::vector<int>& phi) const {
    std::vector<int> colors(2 * n, 1);
    for (size_t i = 0; i < pairs.size(); ++i) {
      colors[pairs[i].first] = (int)i + 2;
      colors[n + pairs[i].second] = (int)i + 2;
    }
    return search(std::move(colors), phi);
  }
};

// Algorithm 1's classification: breadth-first closure of the edge list under the
// generators; classes are seeded in edge order
void close(const std::vector<std::pair<int, int>>& edges, const std::map<std::pair<int, int>, int>& index,
           const std::vector<std::vector<int>>& gens, std::vector<int>& orbit_of, std::vector<std::vector<int>>& orbits) {
  const int m = (int)edges.size();
  orbit_of.assign(m, -1);
  orbits.clear();
  for (int e0 = 0; e0 < m; ++e0) {
    if (orbit_of[e0] >= 0) continue;
    const int cid = (int)orbits.size();
    std::vector<int> cls{e0};
    orbit_of[e0] = cid;
    std::deque<int> q{e0};
    while (!q.empty()) {
      const auto [u, v] = edges[q.front()];
      q.pop_front();
      for (const auto& g : gens) {
        const int a = g[u], b = g[v];
        const int e2 = index.at({std::min(a, b), std::max(a, b)});
        if (orbit_of[e2] < 0) {
          orbit_of[e2] = cid;
          cls.push_back(e2);
          q.push_back(e2);
        }
      }
    }
    orbits.push_back(std::move(cls));
  }
}

}  // namespace aaq_orbits


extern "C" aaq_status aaq_edge_orbits(int n, int num_edges, const int32_t* edges, const int32_t* edge_weight,
                                      int32_t* orbit_of, int32_t* num_orbits, int32_t* orbit_rep, int32_t* orbit_size) {
  using namespace aaq_orbits;
  if (n < 1 || n > 4096) return aaq::set_error(AAQ_ERR_INVALID_ARG, "n must be in [1, 4096]");
  if (num_edges < 0) return aaq::set_error(AAQ_ERR_GRAPH, "num_edges < 0");
  if (num_edges > 0 && (!edges || !orbit_of || !orbit_rep || !orbit_size))
    return aaq::set_error(AAQ_ERR_INVALID_ARG, "edges / output arrays are NULL");
  if (!num_orbits) return aaq::set_error(AAQ_ERR_INVALID_ARG, "num_orbits is NULL");
  std::vector<std::pair<int, int>> es(num_edges);
  std::map<std::pair<int, int>, int> index;
  Adj adj(n), wadj(n);
  std::vector<int> wt(num_edges, 1);
  for (int e = 0; e < num_edges; ++e) {
    const int u = edges[2 * e], v = edges[2 * e + 1];
    if (u < 0 || u >= n || v < 0 || v >= n)
      return aaq::set_error(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " has a vertex out of range");
    if (u == v) return aaq::set_error(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " is a self-loop");
    es[e] = {std::min(u, v), std::max(u, v)};
    if (!index.emplace(es[e], e).second)
      return aaq::set_error(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " is a duplicate");
    if (edge_weight) {
      if (edge_weight[e] < 1) return aaq::set_error(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " has a weight < 1");
      wt[e] = edge_weight[e];
    }
    adj[u].push_back(v);
    adj[v].push_back(u);
    wadj[u].push_back(wt[e]);
    wadj[v].push_back(wt[e]);
  }
  if (num_edges == 0) {
    *num_orbits = 0;
    return AAQ_OK;
  }
  Searcher S(adj, wadj);
  std::vector<std::vector<int>> gens;
  std::set<std::pair<int, int>> tested;
  std::vector<int> of;
  std::vector<std::vector<int>> orbits;
  for (;;) {
    close(es, index, gens, of, orbits);
    bool merged = false;
    for (size_t i = 0; i < orbits.size() && !merged; ++i)
      for (size_t j = i + 1; j < orbits.size() && !merged; ++j) {
        const int ei = orbits[i][0], ej = orbits[j][0];
        const auto [a, b] = es[ei];
        const auto [c, d] = es[ej];
        const auto inv_i = std::minmax(S.base[a], S.base[b]), inv_j = std::minmax(S.base[c], S.base[d]);
        if (inv_i != inv_j || wt[ei] != wt[ej] || !tested.insert({ei, ej}).second) continue;
        std::vector<int> phi;
        if (S.extend({{a, c}, {b, d}}, phi) || S.extend({{a, d}, {b, c}}, phi)) {
          gens.push_back(phi);
          merged = true;
        }
      }
    if (!merged) break;
  }
  for (int e = 0; e < num_edges; ++e) orbit_of[e] = of[e];
  *num_orbits = (int32_t)orbits.size();
  for (size_t o = 0; o < orbits.size(); ++o) {
    orbit_rep[o] = orbits[o][0];
    orbit_size[o] = (int32_t)orbits[o].size();
  }
  return AAQ_OK;
}

// ---------------------------------------------------------------- combined-RCC coverage
// eta_p = 1 - |U_{e in R} RCC_p(e)| / |E| (the structural descriptor of the paper's
// combined-RCC coverage subsection).  RCC_p(e), e = (i, j), holds the cost gates that do
// not commute through to Z_i Z_j in p layers: the edges with an endpoint within graph
// distance p - 1 of {i, j} (layer p: the gates on i or j; each earlier layer one hop
// further); its qubits are the vertices within distance p.  The qubit-elimination
// fraction is the share of the n qubits outside the union of the cones' qubits.
extern "C" aaq_status aaq_rcc_eta(int n, int num_edges, const int32_t* edges, const int32_t* orbit_of,
                                  int num_orbits, const int32_t* rep, int p, double* eta_out,
                                  double* qubit_elim_out, uint8_t* vertex_cover_out) {
  if (n < 1 || n > 4096) return aaq::set_error(AAQ_ERR_INVALID_ARG, "n must be in [1, 4096]");
  if (num_edges < 1 || num_edges > (1 << 16)) return aaq::set_error(AAQ_ERR_GRAPH, "num_edges must be in [1, 65536]");
  if (!edges || !orbit_of || !eta_out) return aaq::set_error(AAQ_ERR_INVALID_ARG, "edges / orbit_of / eta_out is NULL");
  if (p < 1) return aaq::set_error(AAQ_ERR_INVALID_ARG, "p must be >= 1");
  if (vertex_cover_out && !rep)
    return aaq::set_error(AAQ_ERR_INVALID_ARG, "the vertex cover is defined for given representatives");
  if (num_orbits < 1 || num_orbits > num_edges) return aaq::set_error(AAQ_ERR_ORBITS, "num_orbits must be in [1, |E|]");
  std::vector<std::vector<int>> adj(n);
  std::set<std::pair<int, int>> seen;
  for (int e = 0; e < num_edges; ++e) {
    const int u = edges[2 * e], v = edges[2 * e + 1];
    if (u < 0 || u >= n || v < 0 || v >= n)
      return aaq::set_error(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " has a vertex out of range");
    if (u == v) return aaq::set_error(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " is a self-loop");
    if (!seen.emplace(std::min(u, v), std::max(u, v)).second)
      return aaq::set_error(AAQ_ERR_GRAPH, "edge " + std::to_string(e) + " is a duplicate");
    adj[u].push_back(v);
    adj[v].push_back(u);
  }
  std::vector<std::vector<int>> members(num_orbits);
  for (int e = 0; e < num_edges; ++e) {
    if (orbit_of[e] < 0 || orbit_of[e] >= num_orbits)
      return aaq::set_error(AAQ_ERR_ORBITS, "edge " + std::to_string(e) + " has an orbit id out of range");
    members[orbit_of[e]].push_back(e);
  }
  for (int m = 0; m < num_orbits; ++m) {
    if (members[m].empty()) return aaq::set_error(AAQ_ERR_ORBITS, "orbit " + std::to_string(m) + " is empty");
    if (rep && (rep[m] < 0 || rep[m] >= num_edges || orbit_of[rep[m]] != m))
      return aaq::set_error(AAQ_ERR_ORBITS, "representative of orbit " + std::to_string(m) + " is not in it");
  }
  // distances from {i, j} of edge e by breadth-first search, up to p
  const int far = p + 1;
  std::vector<int> dist(n), queue(n);
  auto cone = [&](int e) {
    std::fill(dist.begin(), dist.end(), far);
    int head = 0, tail = 0;
    for (int s : {edges[2 * e], edges[2 * e + 1]}) {
      dist[s] = 0;
      queue[tail++] = s;
    }
    while (head < tail) {
      const int u = queue[head++];
      if (dist[u] + 1 > p) continue;
      for (int w : adj[u])
        if (dist[w] == far) {
          dist[w] = dist[u] + 1;
          queue[tail++] = w;
        }
    }
  };
  auto in_cone = [&](int f) { return std::min(dist[edges[2 * f]], dist[edges[2 * f + 1]]) <= p - 1; };
  double outside = 0.0, qout = 0.0;  // edges / qubits outside the union (expected counts without rep)
  if (rep) {
    std::vector<char> covered(num_edges, 0), vcov(n, 0);
    for (int m = 0; m < num_orbits; ++m) {
      cone(rep[m]);
      for (int f = 0; f < num_edges; ++f)
        if (in_cone(f)) covered[f] = 1;
      for (int v = 0; v < n; ++v)
        if (dist[v] <= p) vcov[v] = 1;
    }
    for (int f = 0; f < num_edges; ++f) outside += covered[f] ? 0.0 : 1.0;
    for (int v = 0; v < n; ++v) qout += vcov[v] ? 0.0 : 1.0;
    if (vertex_cover_out)
      for (int v = 0; v < n; ++v) vertex_cover_out[v] = (uint8_t)vcov[v];
  } else {
    // representatives drawn uniformly and independently per orbit: edge f lies outside
    // the union with probability prod_m (1 - c_mf / |m|), c_mf = the edges of orbit m
    // whose cone holds f
    // (and qubit v likewise, with the edges whose cone's qubits hold v)
    std::vector<double> miss(num_edges, 1.0), vmiss(n, 1.0);
    std::vector<int> cnt(num_edges), vcnt(n);
    for (int m = 0; m < num_orbits; ++m) {
      std::fill(cnt.begin(), cnt.end(), 0);
      std::fill(vcnt.begin(), vcnt.end(), 0);
      for (int e : members[m]) {
        cone(e);
        for (int f = 0; f < num_edges; ++f) cnt[f] += in_cone(f) ? 1 : 0;
        for (int v = 0; v < n; ++v) vcnt[v] += dist[v] <= p ? 1 : 0;
      }
      const double sz = (double)members[m].size();
      for (int f = 0; f < num_edges; ++f) miss[f] *= 1.0 - cnt[f] / sz;
      for (int v = 0; v < n; ++v) vmiss[v] *= 1.0 - vcnt[v] / sz;
    }
    for (int f = 0; f < num_edges; ++f) outside += miss[f];
    for (int v = 0; v < n; ++v) qout += vmiss[v];
  }
  *eta_out = outside / num_edges;
  if (qubit_elim_out) *qubit_elim_out = qout / n;
  return AAQ_OK;
}
