// Nested-dissection ordering of the adjacency graph (host; the independent
// parts below the top separators are ordered in parallel threads).
//
// The paper's land-ice runs reorder each subdomain matrix with METIS nested
// dissection before the factorization (Tacho section; the nested-dissection
// picture is drawn in the Basker section).  METIS is not available here, so
// this file implements a multilevel nested dissection of its own:
//
//   1. coarsen the part by heavy-edge matching until it is small;
//   2. bisect the coarsest graph by greedy region growing from several
//      seeds, keeping the smallest balanced edge cut;
//   3. project back level by level, improving the cut at every level with
//      Fiduccia-Mattheyses moves under a balance constraint;
//   4. turn the edge separator into a vertex separator: a minimum vertex
//      cover of the bipartite graph of cut edges (maximum matching + Koenig);
//   5. number the separator after both sides and recurse on the connected
//      components of each side.
//
// Minimum edge cuts give connected, plane-like separators on grid graphs, so
// every separator becomes one dense supernode.  Parts of at most `leaf_size`
// vertices are numbered in ascending original order.  All choices depend only
// on a part's local structure (vertices in ascending order, a generator
// seeded by the part's size), so the ordering of a connected component does
// not depend on what else is in the graph.
#include <algorithm>
#include <cstdint>
#include <exception>
#include <queue>
#include <thread>
#include <vector>

#include "symbolic.hpp"

namespace tacho {
namespace {

struct Graph {
  int32_t n = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
  std::vector<int32_t> ew;  // edge weights (1 on the input graph)
  std::vector<int32_t> vw;  // vertex weights
  int64_t total_vw = 0;
};

Graph adjacency(const Pattern& P) {
  Graph G;
  G.n = (int32_t)P.n;
  G.xadj.assign(P.n + 1, 0);
  for (int64_t i = 0; i < P.n; ++i)
    for (int64_t k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k)
      if (P.colind[k] != i) G.xadj[i + 1]++;
  for (int64_t i = 0; i < P.n; ++i) G.xadj[i + 1] += G.xadj[i];
  G.adj.resize(G.xadj[P.n]);
  for (int64_t i = 0, q = 0; i < P.n; ++i)
    for (int64_t k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k)
      if (P.colind[k] != i) G.adj[q++] = P.colind[k];
  G.ew.assign(G.adj.size(), 1);
  G.vw.assign(P.n, 1);
  G.total_vw = P.n;
  return G;
}

// splitmix64: small deterministic generator
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint32_t below(uint32_t n) { return (uint32_t)(next() % n); }
};

// Subgraph induced by `verts` (ascending global ids), local ids 0..|verts|-1.
Graph induced(const Graph& G, const std::vector<int32_t>& verts, std::vector<int32_t>& local) {
  Graph H;
  H.n = (int32_t)verts.size();
  for (int32_t i = 0; i < H.n; ++i) local[verts[i]] = i;
  H.xadj.assign(H.n + 1, 0);
  for (int32_t i = 0; i < H.n; ++i) {
    const int32_t v = verts[i];
    int64_t c = 0;
    for (int64_t k = G.xadj[v]; k < G.xadj[v + 1]; ++k) c += local[G.adj[k]] >= 0;
    H.xadj[i + 1] = H.xadj[i] + c;
  }
  H.adj.resize(H.xadj[H.n]);
  H.ew.resize(H.xadj[H.n]);
  H.vw.resize(H.n);
  H.total_vw = 0;
  for (int32_t i = 0; i < H.n; ++i) {
    const int32_t v = verts[i];
    int64_t q = H.xadj[i];
    for (int64_t k = G.xadj[v]; k < G.xadj[v + 1]; ++k) {
      const int32_t u = local[G.adj[k]];
      if (u >= 0) {
        H.adj[q] = u;
        H.ew[q] = G.ew[k];
        ++q;
      }
    }
    H.vw[i] = G.vw[v];
    H.total_vw += H.vw[i];
  }
  for (int32_t v : verts) local[v] = -1;
  return H;
}

// One level of heavy-edge matching; cmap maps fine -> coarse vertices.
Graph coarsen(const Graph& g, std::vector<int32_t>& cmap, Rng& rng) {
  const int32_t n = g.n;
  std::vector<int32_t> order(n), match(n, -1);
  for (int32_t i = 0; i < n; ++i) order[i] = i;
  for (int32_t i = n - 1; i > 0; --i) std::swap(order[i], order[rng.below((uint32_t)i + 1)]);
  for (int32_t v : order) {
    if (match[v] >= 0) continue;
    int32_t best = -1, bw = -1;
    for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
      const int32_t u = g.adj[k];
      if (match[u] < 0 && u != v && g.ew[k] > bw) {
        bw = g.ew[k];
        best = u;
      }
    }
    if (best >= 0) {
      match[v] = best;
      match[best] = v;
    } else {
      match[v] = v;
    }
  }
  cmap.assign(n, -1);
  int32_t nc = 0;
  for (int32_t v = 0; v < n; ++v)
    if (cmap[v] < 0) {
      cmap[v] = nc;
      cmap[match[v]] = nc;
      ++nc;
    }
  Graph c;
  c.n = nc;
  c.vw.assign(nc, 0);
  c.total_vw = g.total_vw;
  c.xadj.assign(nc + 1, 0);
  std::vector<int32_t> fine_of(2 * (size_t)nc, -1);
  for (int32_t v = 0; v < n; ++v) {
    const int32_t cv = cmap[v];
    c.vw[cv] += g.vw[v];
    if (fine_of[2 * cv] < 0) fine_of[2 * cv] = v;
    else if (fine_of[2 * cv] != v) fine_of[2 * cv + 1] = v;
  }
  std::vector<int32_t> slot(nc, -1);
  c.adj.reserve(g.adj.size());
  c.ew.reserve(g.adj.size());
  for (int32_t cv = 0; cv < nc; ++cv) {
    const int64_t start = (int64_t)c.adj.size();
    for (int t = 0; t < 2; ++t) {
      const int32_t v = fine_of[2 * cv + t];
      if (v < 0) continue;
      for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
        const int32_t cu = cmap[g.adj[k]];
        if (cu == cv) continue;
        if (slot[cu] < start || slot[cu] >= (int64_t)c.adj.size() || c.adj[slot[cu]] != cu) {
          slot[cu] = (int32_t)c.adj.size();
          c.adj.push_back(cu);
          c.ew.push_back(g.ew[k]);
        } else {
          c.ew[slot[cu]] += g.ew[k];
        }
      }
    }
    c.xadj[cv + 1] = (int64_t)c.adj.size();
  }
  return c;
}

int64_t cut_of(const Graph& g, const std::vector<uint8_t>& side) {
  int64_t cut = 0;
  for (int32_t v = 0; v < g.n; ++v)
    for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k)
      if (side[g.adj[k]] != side[v]) cut += g.ew[k];
  return cut / 2;
}

// Fiduccia-Mattheyses refinement of a two-way edge cut.  Each pass moves
// unlocked vertices by best gain (ties: lowest id) from a side that may give
// weight away, and keeps the best prefix of moves.
void fm_refine(const Graph& g, std::vector<uint8_t>& side, int64_t maxw, int passes) {
  const int32_t n = g.n;
  std::vector<int64_t> gain(n);
  std::vector<uint8_t> locked(n);
  int64_t w[2] = {0, 0};
  for (int32_t v = 0; v < n; ++v) w[side[v]] += g.vw[v];
  int64_t cut = cut_of(g, side);
  typedef std::pair<int64_t, int32_t> Entry;  // (gain, -id) max-heap
  for (int pass = 0; pass < passes; ++pass) {
    std::priority_queue<Entry> heap[2];
    for (int32_t v = 0; v < n; ++v) {
      int64_t ext = 0, in = 0;
      for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k)
        (side[g.adj[k]] != side[v] ? ext : in) += g.ew[k];
      gain[v] = ext - in;
      locked[v] = 0;
      if (ext > 0) heap[side[v]].push({gain[v], -v});
    }
    std::vector<int32_t> moves;
    int64_t best_cut = cut, cur = cut;
    int64_t best_imb = std::max(w[0], w[1]);
    size_t best_len = 0;
    const size_t limit = std::max<size_t>(64, (size_t)n / 20);
    size_t since_best = 0;
    while (since_best < limit) {
      int from = -1;
      Entry top[2];
      bool have[2] = {false, false};
      for (int s = 0; s < 2; ++s) {
        while (!heap[s].empty()) {
          Entry e = heap[s].top();
          const int32_t v = -e.second;
          if (locked[v] || side[v] != s || e.first != gain[v]) {
            heap[s].pop();
            continue;
          }
          top[s] = e;
          have[s] = true;
          break;
        }
      }
      for (int s = 0; s < 2; ++s) {
        if (!have[s]) continue;
        const int32_t v = -top[s].second;
        if (w[1 - s] + g.vw[v] > maxw) have[s] = false;  // would overload the other side
      }
      if (have[0] && have[1])
        from = top[0] > top[1] ? 0 : 1;
      else if (have[0])
        from = 0;
      else if (have[1])
        from = 1;
      if (from < 0) break;
      const int32_t v = -top[from].second;
      heap[from].pop();
      locked[v] = 1;
      cur -= gain[v];
      side[v] = (uint8_t)(1 - from);
      w[from] -= g.vw[v];
      w[1 - from] += g.vw[v];
      moves.push_back(v);
      for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
        const int32_t u = g.adj[k];
        if (locked[u]) continue;
        gain[u] += side[u] == side[v] ? -2 * g.ew[k] : 2 * g.ew[k];
        heap[side[u]].push({gain[u], -u});
      }
      const int64_t imb = std::max(w[0], w[1]);
      if (cur < best_cut || (cur == best_cut && imb < best_imb)) {
        best_cut = cur;
        best_imb = imb;
        best_len = moves.size();
        since_best = 0;
      } else {
        ++since_best;
      }
    }
    for (size_t i = moves.size(); i > best_len; --i) {
      const int32_t v = moves[i - 1];
      w[side[v]] -= g.vw[v];
      side[v] = (uint8_t)(1 - side[v]);
      w[side[v]] += g.vw[v];
    }
    const bool improved = best_cut < cut;
    cut = best_cut;
    if (!improved) break;
  }
}

// Greedy region growing from a seed: repeatedly add the frontier vertex with
// the largest (edges into the region - edges out) until half the weight.
void grow(const Graph& g, int32_t seed, std::vector<uint8_t>& side) {
  const int32_t n = g.n;
  side.assign(n, 1);
  std::vector<int64_t> conn(n, 0);
  std::vector<uint8_t> inq(n, 0);
  typedef std::pair<int64_t, int32_t> Entry;
  std::priority_queue<Entry> heap;
  int64_t w0 = 0;
  const int64_t half = g.total_vw / 2;
  heap.push({0, -seed});
  inq[seed] = 1;
  int32_t next_unvisited = 0;
  while (w0 < half) {
    int32_t v = -1;
    while (!heap.empty()) {
      Entry e = heap.top();
      heap.pop();
      const int32_t u = -e.second;
      if (side[u] == 0 || e.first != conn[u]) continue;
      v = u;
      break;
    }
    if (v < 0) {  // disconnected remainder: continue from the lowest unvisited vertex
      while (next_unvisited < n && side[next_unvisited] == 0) ++next_unvisited;
      if (next_unvisited >= n) break;
      v = next_unvisited;
    }
    side[v] = 0;
    w0 += g.vw[v];
    for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
      const int32_t u = g.adj[k];
      if (side[u] == 0) continue;
      conn[u] += g.ew[k];
      heap.push({conn[u], -u});
    }
  }
}

// Bisection of g: multilevel coarsening, best of several grown seeds on the
// coarsest graph, FM at every level.  Returns side[v] in {0, 1}.
std::vector<uint8_t> bisect(const Graph& g0, Rng& rng) {
  std::vector<Graph> levels;
  std::vector<std::vector<int32_t>> maps;
  const Graph* cur = &g0;
  while (cur->n > 120) {
    std::vector<int32_t> cmap;
    Graph c = coarsen(*cur, cmap, rng);
    if (c.n > cur->n * 0.92) break;  // matching no longer shrinks the graph
    maps.push_back(std::move(cmap));
    levels.push_back(std::move(c));
    cur = &levels.back();
  }
  const Graph& cg = *cur;
  const int64_t maxw_c = (int64_t)(0.55 * (double)cg.total_vw) + 1;
  std::vector<uint8_t> best, side;
  int64_t best_cut = -1;
  const int tries = std::min<int32_t>(8, cg.n);
  for (int t = 0; t < tries; ++t) {
    const int32_t seed = t == 0 ? 0 : (int32_t)rng.below((uint32_t)cg.n);
    grow(cg, seed, side);
    fm_refine(cg, side, maxw_c, 6);
    const int64_t c = cut_of(cg, side);
    if (best_cut < 0 || c < best_cut) {
      best_cut = c;
      best = side;
    }
  }
  // project back
  for (int lv = (int)levels.size() - 1; lv >= 0; --lv) {
    const Graph& fine = lv == 0 ? g0 : levels[lv - 1];
    const std::vector<int32_t>& cmap = maps[lv];
    std::vector<uint8_t> fs(fine.n);
    for (int32_t v = 0; v < fine.n; ++v) fs[v] = best[cmap[v]];
    fm_refine(fine, fs, (int64_t)(0.55 * (double)fine.total_vw) + 1, 4);
    best.swap(fs);
  }
  return best;
}

// Minimum vertex cover of the bipartite graph of cut edges (Kuhn's
// augmenting paths + Koenig's construction).  Returns the cover as a 0/1 mask.
std::vector<uint8_t> separator_from_cut(const Graph& g, const std::vector<uint8_t>& side) {
  const int32_t n = g.n;
  std::vector<int32_t> mate(n, -1);
  std::vector<int32_t> stamp(n, -1);
  std::vector<int32_t> left;  // side-0 boundary vertices
  for (int32_t v = 0; v < n; ++v) {
    if (side[v] != 0) continue;
    for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k)
      if (side[g.adj[k]] == 1) {
        left.push_back(v);
        break;
      }
  }
  // iterative augmenting path search from each left vertex
  std::vector<int32_t> stk, via;
  std::vector<int64_t> it(n);
  for (size_t li = 0; li < left.size(); ++li) {
    const int32_t root = left[li];
    stk.clear();
    via.clear();
    stk.push_back(root);
    it[root] = g.xadj[root];
    stamp[root] = (int32_t)li;
    bool found = false;
    while (!stk.empty() && !found) {
      const int32_t v = stk.back();
      if (it[v] >= g.xadj[v + 1]) {
        stk.pop_back();
        if (!via.empty()) via.pop_back();
        continue;
      }
      const int32_t u = g.adj[it[v]++];
      if (side[u] != 1 || stamp[u] == (int32_t)li) continue;
      stamp[u] = (int32_t)li;
      if (mate[u] < 0) {
        // augment along stk (left vertices) and via (right vertices) + u
        via.push_back(u);
        for (size_t t = stk.size(); t-- > 0;) {
          const int32_t lv = stk[t], rv = via[t];
          mate[lv] = rv;
          mate[rv] = lv;
        }
        found = true;
      } else {
        const int32_t w = mate[u];
        if (stamp[w] == (int32_t)li) continue;
        stamp[w] = (int32_t)li;
        via.push_back(u);
        stk.push_back(w);
        it[w] = g.xadj[w];
      }
    }
  }
  // Koenig: Z = vertices reachable from unmatched left vertices by alternating
  // paths (left -> right over any cut edge, right -> left over matched edges).
  std::vector<uint8_t> inZ(n, 0);
  std::vector<int32_t> q;
  for (int32_t v : left)
    if (mate[v] < 0) {
      inZ[v] = 1;
      q.push_back(v);
    }
  for (size_t h = 0; h < q.size(); ++h) {
    const int32_t v = q[h];
    for (int64_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
      const int32_t u = g.adj[k];
      if (side[u] != 1 || inZ[u]) continue;
      inZ[u] = 1;
      const int32_t w = mate[u];
      if (w >= 0 && !inZ[w]) {
        inZ[w] = 1;
        q.push_back(w);
      }
    }
  }
  std::vector<uint8_t> cover(n, 0);
  for (int32_t v : left)
    if (!inZ[v]) cover[v] = 1;
  for (int32_t v = 0; v < n; ++v)
    if (side[v] == 1 && inZ[v]) cover[v] = 1;
  return cover;
}

// Per-thread scratch: local ids of induced() and component marks (indexed by
// global vertex; a part touches only its own vertices and reads its
// neighbours', so concurrent parts need their own copies).
struct Work {
  std::vector<int32_t> local, mark;
  int32_t epoch = 0;
  explicit Work(int32_t n) : local(n, -1), mark(n, 0) {}
};

// The order of a part is a function of the part alone: its components are
// ordered one by one (the component holding the largest vertex first) and the
// separator comes last.  Large parts near the top of the recursion hand one of
// their components to another thread; the result does not depend on it.
class Dissector {
 public:
  Dissector(const Graph& G, int leaf) : G_(G), leaf_(std::max(leaf, 1)) {}

  std::vector<int32_t> run() {
    Work w(G_.n);
    std::vector<int32_t> all(G_.n);
    for (int32_t v = 0; v < G_.n; ++v) all[v] = v;
    std::vector<int32_t> out;
    out.reserve(G_.n);
    order_components(all, w, 0, out);
    return out;
  }

 private:
  static constexpr int32_t kParallelMin = 20000;  // vertices of a part worth a thread
  static constexpr int kParallelDepth = 4;        // at most 2^4 concurrent parts

  // Append the order of `verts` (ascending, one connected component).
  void order_part(const std::vector<int32_t>& verts, Work& w, int depth,
                  std::vector<int32_t>& out) const {
    if ((int64_t)verts.size() <= leaf_) {
      out.insert(out.end(), verts.begin(), verts.end());
      return;
    }
    Graph g = induced(G_, verts, w.local);
    Rng rng(0x5eed0000ull ^ (uint64_t)verts.size() * 0x9E3779B97F4A7C15ull);
    std::vector<uint8_t> side = bisect(g, rng);
    std::vector<uint8_t> cover = separator_from_cut(g, side);
    std::vector<int32_t> sep, rest;
    for (int32_t i = 0; i < g.n; ++i) (cover[i] ? sep : rest).push_back(verts[i]);
    if (sep.empty() || rest.empty()) {  // no split found: treat as a leaf
      out.insert(out.end(), verts.begin(), verts.end());
      return;
    }
    order_components(rest, w, depth + 1, out);
    out.insert(out.end(), sep.begin(), sep.end());
  }

  // Append the orders of the connected components of `verts` (ascending),
  // the component holding the largest smallest vertex first.
  void order_components(const std::vector<int32_t>& verts, Work& w, int depth,
                        std::vector<int32_t>& out) const {
    std::vector<std::vector<int32_t>> comps = components(verts, w);
    std::vector<std::vector<int32_t>> parts(comps.size());
    std::vector<std::thread> helpers;
    std::vector<std::exception_ptr> errs(comps.size());
    for (size_t c = comps.size(); c-- > 0;) {
      const bool spawn = depth < kParallelDepth && c > 0 &&
                         (int32_t)comps[c].size() >= kParallelMin;
      if (spawn) {
        helpers.emplace_back([this, &comps, &parts, &errs, c, depth]() {
          try {
            Work wc(G_.n);
            order_part(comps[c], wc, depth, parts[c]);
          } catch (...) {
            errs[c] = std::current_exception();
          }
        });
      } else {
        order_part(comps[c], w, depth, parts[c]);
      }
    }
    for (auto& t : helpers) t.join();
    for (auto& e : errs)
      if (e) std::rethrow_exception(e);
    for (size_t c = comps.size(); c-- > 0;) out.insert(out.end(), parts[c].begin(), parts[c].end());
  }

  // Connected components of the subgraph induced by `verts`, each ascending,
  // in the order of their smallest vertex.
  std::vector<std::vector<int32_t>> components(const std::vector<int32_t>& verts, Work& w) const {
    ++w.epoch;
    for (int32_t v : verts) w.mark[v] = w.epoch;  // members of this set
    std::vector<std::vector<int32_t>> comps;
    for (int32_t s : verts) {
      if (w.mark[s] != w.epoch) continue;
      std::vector<int32_t> comp{s};
      w.mark[s] = -w.epoch;
      for (size_t h = 0; h < comp.size(); ++h) {
        const int32_t v = comp[h];
        for (int64_t k = G_.xadj[v]; k < G_.xadj[v + 1]; ++k) {
          const int32_t u = G_.adj[k];
          if (w.mark[u] == w.epoch) {
            w.mark[u] = -w.epoch;
            comp.push_back(u);
          }
        }
      }
      std::sort(comp.begin(), comp.end());
      comps.push_back(std::move(comp));
    }
    return comps;
  }

  const Graph& G_;
  int leaf_;
};

}  // namespace

std::vector<int32_t> nested_dissection(const Pattern& P, int leaf_size) {
  Graph G = adjacency(P);
  Dissector D(G, leaf_size);
  return D.run();
}

}  // namespace tacho
