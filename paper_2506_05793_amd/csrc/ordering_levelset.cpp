// Level-structure nested dissection (host, one core), the alternative to the
// multilevel ordering in ordering.cpp.
//
// An automatic nested dissection in the style of George and Liu:
// a pseudo-peripheral vertex roots a breadth-first level structure, a level
// near the middle (the smallest one inside a balance window) gives the
// separator, refined to the vertices that touch the next level, and the
// separator is numbered after both remaining parts.  Parts of at most
// `leaf_size` vertices, or with fewer than three levels, are numbered in
// ascending original order.  All tie-breaks use the lowest vertex index, so
// the result is deterministic.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "symbolic.hpp"

namespace tacho {
namespace levelset {

struct Graph {
  int64_t n;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
};

Graph adjacency(const Pattern& P) {
  Graph G;
  G.n = P.n;
  G.xadj.assign(P.n + 1, 0);
  for (int64_t i = 0; i < P.n; ++i)
    for (int64_t k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k)
      if (P.colind[k] != i) G.xadj[i + 1]++;
  for (int64_t i = 0; i < P.n; ++i) G.xadj[i + 1] += G.xadj[i];
  G.adj.resize(G.xadj[P.n]);
  for (int64_t i = 0, q = 0; i < P.n; ++i)
    for (int64_t k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k)
      if (P.colind[k] != i) G.adj[q++] = P.colind[k];
  return G;
}

class Dissector {
 public:
  Dissector(const Graph& G, int leaf) : G_(G), leaf_(std::max(leaf, 1)) {
    part_.assign(G.n, 0);
    stamp_.assign(G.n, 0);
    lev_.assign(G.n, -1);
    perm_.assign(G.n, -1);
    queue_.reserve(G.n);
  }

  std::vector<int32_t> run() {
    hi_ = G_.n;
    // Initial parts: connected components of the whole graph, part id 1.
    std::vector<int32_t> all(G_.n);
    for (int64_t v = 0; v < G_.n; ++v) { all[v] = (int32_t)v; part_[v] = 1; }
    next_part_ = 2;
    push_components(all, 1);
    while (!stack_.empty()) {
      Item it = std::move(stack_.back());
      stack_.pop_back();
      dissect(it.verts, it.part);
    }
    return perm_;
  }

 private:
  struct Item {
    std::vector<int32_t> verts;  // sorted ascending, connected
    int32_t part;
  };

  // Number `verts` (ascending) into the highest free positions.
  void number(const std::vector<int32_t>& verts) {
    int64_t base = hi_ - (int64_t)verts.size();
    for (size_t k = 0; k < verts.size(); ++k) {
      perm_[base + k] = verts[k];
      part_[verts[k]] = 0;
    }
    hi_ = base;
  }

  int degree_in(int32_t v, int32_t p) const {
    int d = 0;
    for (int64_t k = G_.xadj[v]; k < G_.xadj[v + 1]; ++k) d += part_[G_.adj[k]] == p;
    return d;
  }

  // Breadth-first level structure of part p from root r: fills queue_ (vertices by
  // level) and lptr_ (level starts).  Returns the number of levels.
  int bfs(int32_t r, int32_t p) {
    ++cur_stamp_;
    queue_.clear();
    lptr_.clear();
    queue_.push_back(r);
    stamp_[r] = cur_stamp_;
    size_t head = 0;
    while (head < queue_.size()) {
      lptr_.push_back((int64_t)head);
      size_t end = queue_.size();
      int32_t L = (int32_t)lptr_.size() - 1;
      for (; head < end; ++head) {
        int32_t v = queue_[head];
        lev_[v] = L;
        for (int64_t k = G_.xadj[v]; k < G_.xadj[v + 1]; ++k) {
          int32_t u = G_.adj[k];
          if (part_[u] == p && stamp_[u] != cur_stamp_) {
            stamp_[u] = cur_stamp_;
            queue_.push_back(u);
          }
        }
      }
    }
    lptr_.push_back((int64_t)queue_.size());
    return (int)lptr_.size() - 1;
  }

  void dissect(const std::vector<int32_t>& verts, int32_t p) {
    const int64_t nv = (int64_t)verts.size();
    if (nv <= leaf_) { number(verts); return; }
    // Pseudo-peripheral root: start at a vertex of minimum degree, move to a
    // minimum-degree vertex of the last level while the eccentricity grows.
    int32_t r = verts[0];
    int best = degree_in(r, p);
    for (int32_t v : verts) {
      int d = degree_in(v, p);
      if (d < best) { best = d; r = v; }
    }
    int nlev = bfs(r, p);
    for (int iter = 0; iter < 8; ++iter) {
      int32_t x = -1;
      int xd = 0;
      for (int64_t q = lptr_[nlev - 1]; q < lptr_[nlev]; ++q) {
        int32_t v = queue_[q];
        int d = degree_in(v, p);
        if (x < 0 || d < xd || (d == xd && v < x)) { x = v; xd = d; }
      }
      int nx = bfs(x, p);
      if (nx > nlev) { r = x; nlev = nx; continue; }
      nlev = bfs(r, p);  // restore the structure of r
      break;
    }
    if (nlev < 3) { number(verts); return; }

    // Separator level: the smallest refined level among those whose split keeps
    // each side at least a fifth of the part; ties go to the most balanced.
    auto refined = [&](int L, std::vector<int32_t>* out) {
      int64_t cnt = 0;
      for (int64_t q = lptr_[L]; q < lptr_[L + 1]; ++q) {
        int32_t v = queue_[q];
        bool touches = false;
        for (int64_t k = G_.xadj[v]; k < G_.xadj[v + 1] && !touches; ++k) {
          int32_t u = G_.adj[k];
          touches = part_[u] == p && stamp_[u] == cur_stamp_ && lev_[u] == L + 1;
        }
        if (touches) {
          ++cnt;
          if (out) out->push_back(v);
        }
      }
      return cnt;
    };
    int mid = nlev / 2;
    int chosen = mid;
    int64_t best_sz = refined(mid, nullptr);
    int64_t best_imb = 0;
    {
      int64_t below = lptr_[mid];
      int64_t above = nv - lptr_[mid + 1];
      best_imb = below > above ? below - above : above - below;
    }
    for (int L = 1; L + 1 < nlev; ++L) {
      if (L == mid) continue;
      int64_t below = lptr_[L];
      int64_t above = nv - lptr_[L + 1];
      if (below * 5 < nv || above * 5 < nv) continue;
      int64_t sz = refined(L, nullptr);
      int64_t imb = below > above ? below - above : above - below;
      if (sz < best_sz || (sz == best_sz && imb < best_imb)) {
        best_sz = sz;
        best_imb = imb;
        chosen = L;
      }
    }
    std::vector<int32_t> sep;
    refined(chosen, &sep);
    std::sort(sep.begin(), sep.end());
    for (int32_t v : sep) part_[v] = -1;  // mark removed
    // Remaining vertices of the part, ascending.
    std::vector<int32_t> rest;
    rest.reserve(nv - sep.size());
    for (int32_t v : verts)
      if (part_[v] == p) rest.push_back(v);
    number(sep);
    push_components(rest, p);
  }

  // Split `verts` (all in part p, ascending) into connected components and push
  // them so that the component holding the smallest vertex is dissected first.
  void push_components(const std::vector<int32_t>& verts, int32_t p) {
    std::vector<Item> comps;
    for (int32_t s : verts) {
      if (part_[s] != p) continue;
      int32_t np = next_part_++;
      Item it;
      it.part = np;
      part_[s] = np;
      it.verts.push_back(s);
      for (size_t h = 0; h < it.verts.size(); ++h) {
        int32_t v = it.verts[h];
        for (int64_t k = G_.xadj[v]; k < G_.xadj[v + 1]; ++k) {
          int32_t u = G_.adj[k];
          if (part_[u] == p) {
            part_[u] = np;
            it.verts.push_back(u);
          }
        }
      }
      std::sort(it.verts.begin(), it.verts.end());
      comps.push_back(std::move(it));
    }
    for (size_t c = comps.size(); c-- > 0;) stack_.push_back(std::move(comps[c]));
  }

  const Graph& G_;
  int leaf_;
  int64_t hi_ = 0;
  int32_t next_part_ = 1;
  int32_t cur_stamp_ = 0;
  std::vector<int32_t> part_, stamp_, lev_, perm_, queue_;
  std::vector<int64_t> lptr_;
  std::vector<Item> stack_;
};

}  // namespace levelset

using levelset::adjacency;
using levelset::Dissector;

std::vector<int32_t> levelset_dissection(const Pattern& P, int leaf_size) {
  levelset::Graph G = adjacency(P);
  Dissector D(G, leaf_size);
  return D.run();
}

}  // namespace tacho
