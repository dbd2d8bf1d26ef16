// Host symbolic analysis of the supernodal multifrontal Cholesky.
//
// Paper, Trilinos section (step 1): the analysis uses only the pattern,
// reorders to reduce fill and expose parallelism, and sets up the data
// structures of the factors; it runs on one host core and is reused across
// value changes.  Tacho section: the factorization is multifrontal and
// level-set scheduled, over dense supernodal blocks.
//
// Steps: validate the CSR pattern and add missing diagonals; nested
// dissection; elimination tree (Liu) of the reordered pattern; postorder and
// composition into the final permutation; column counts by the
// Gilbert-Ng-Peyton skeleton/least-common-ancestor method; relaxed
// supernodes; supernodal row structures by merging children; child-to-parent
// relative maps; A-entry-to-front maps; height levels.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <exception>
#include <mutex>
#include <numeric>
#include <stdexcept>
#include <thread>
#include <unordered_map>
#include <vector>

#include "symbolic.hpp"

namespace tacho {

int build_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind, Pattern& P,
                  std::string& err) {
  if (n < 0 || (n > 0 && (!rowptr || !colind && rowptr[n] > 0))) {
    err = "invalid CSR arguments";
    return kInvalid;
  }
  if (n > INT32_MAX - 1) {
    err = "n exceeds the int32 index range";
    return kInvalid;
  }
  P.n = n;
  if (n == 0) {
    P.rowptr.assign(1, 0);
    return kOk;
  }
  if (rowptr[0] != 0) {
    err = "rowptr[0] must be 0";
    return kInvalid;
  }
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) {
      err = "rowptr is not monotone";
      return kInvalid;
    }
  const int64_t nnz = rowptr[n];
  // Rows sorted with their source positions, diagonal added where missing.
  P.rowptr.assign(n + 1, 0);
  std::vector<std::pair<int32_t, int64_t>> row;
  std::vector<int32_t> cols;
  std::vector<int64_t> srcs;
  cols.reserve(nnz + n);
  srcs.reserve(nnz + n);
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    bool diag = false;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      int32_t c = colind[k];
      if (c < 0 || c >= n) {
        err = "column index out of range in row " + std::to_string(i);
        return kInvalid;
      }
      diag |= c == i;
      row.emplace_back(c, k);
    }
    if (!diag) row.emplace_back((int32_t)i, -1);
    std::sort(row.begin(), row.end());
    for (size_t q = 1; q < row.size(); ++q)
      if (row[q].first == row[q - 1].first) {
        err = "duplicate entry (" + std::to_string(i) + ", " + std::to_string(row[q].first) + ")";
        return kInvalid;
      }
    for (auto& e : row) {
      cols.push_back(e.first);
      srcs.push_back(e.second);
    }
    P.rowptr[i + 1] = (int64_t)cols.size();
  }
  P.colind = std::move(cols);
  P.src = std::move(srcs);
  // Structural symmetry: every (i, j) needs (j, i).  Count per column and
  // compare sorted transposes row by row.
  std::vector<int64_t> tptr(n + 1, 0);
  for (int64_t k = 0; k < P.rowptr[n]; ++k) tptr[P.colind[k] + 1]++;
  for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
  for (int64_t i = 0; i < n; ++i)
    if (tptr[i + 1] - tptr[i] != P.rowptr[i + 1] - P.rowptr[i]) {
      err = "pattern is not structurally symmetric (row " + std::to_string(i) + ")";
      return kPattern;
    }
  std::vector<int32_t> tind(P.rowptr[n]);
  std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k) tind[fill[P.colind[k]]++] = (int32_t)i;
  // tind rows are produced in ascending i, hence sorted; compare with colind.
  if (!std::equal(tind.begin(), tind.end(), P.colind.begin())) {
    err = "pattern is not structurally symmetric";
    return kPattern;
  }
  return kOk;
}

namespace {

// Upper-triangle adjacency of C = P A P^T by columns: for column j the rows i < j.
void upper_by_column(const Pattern& A, const std::vector<int32_t>& pinv, std::vector<int64_t>& ptr,
                     std::vector<int32_t>& ind) {
  const int64_t n = A.n;
  ptr.assign(n + 1, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      int32_t i = pinv[r], j = pinv[A.colind[k]];
      if (i < j) ptr[j + 1]++;
    }
  for (int64_t j = 0; j < n; ++j) ptr[j + 1] += ptr[j];
  ind.resize(ptr[n]);
  std::vector<int64_t> pos(ptr.begin(), ptr.end() - 1);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      int32_t i = pinv[r], j = pinv[A.colind[k]];
      if (i < j) ind[pos[j]++] = i;
    }
}

// Elimination tree: for each column j, climb from every i < j adjacent to j
// through the current forest roots (with path halving) and hang the root under j.
std::vector<int32_t> etree(int64_t n, const std::vector<int64_t>& ptr,
                           const std::vector<int32_t>& ind) {
  std::vector<int32_t> parent(n, -1), root(n);
  for (int64_t j = 0; j < n; ++j) {
    root[j] = (int32_t)j;
    for (int64_t q = ptr[j]; q < ptr[j + 1]; ++q) {
      int32_t v = ind[q];
      // find the representative of v's current tree with path halving
      while (root[v] != v) {
        root[v] = root[root[v]];
        v = root[v];
      }
      if (v != j) {
        parent[v] = (int32_t)j;
        root[v] = (int32_t)j;
      }
    }
  }
  return parent;
}

// Postorder of a forest; children visited in ascending order, roots ascending.
std::vector<int32_t> postorder(const std::vector<int32_t>& parent) {
  const int64_t n = (int64_t)parent.size();
  std::vector<int32_t> head(n, -1), next(n, -1), post;
  post.reserve(n);
  for (int64_t j = n - 1; j >= 0; --j)
    if (parent[j] >= 0) {
      next[j] = head[parent[j]];
      head[parent[j]] = (int32_t)j;
    }
  std::vector<int32_t> stack;
  for (int64_t r = 0; r < n; ++r) {
    if (parent[r] >= 0) continue;
    stack.push_back((int32_t)r);
    while (!stack.empty()) {
      int32_t v = stack.back();
      int32_t c = head[v];
      if (c >= 0) {
        head[v] = next[c];
        stack.push_back(c);
      } else {
        stack.pop_back();
        post.push_back(v);
      }
    }
  }
  return post;
}

// Column counts of L for a postordered etree (descendants of j are the
// contiguous labels [first[j], j]).  Each row subtree T_i (rows of L that
// column j contributes to, plus i itself) is encoded by +1 at its leaves,
// -1 at the least common ancestor of consecutive leaves and -1 at parent(i);
// subtree sums of that weight give eta_j.
// With vertex weights wt (row i standing for wt[i] rows), the same encoding
// with +-wt[i] in place of +-1 gives sum over the rows i of column j of wt[i].
std::vector<int64_t> column_counts(int64_t n, const std::vector<int32_t>& parent,
                                   const std::vector<int64_t>& lptr,
                                   const std::vector<int32_t>& lind,
                                   const std::vector<int32_t>* wt = nullptr) {
  std::vector<int32_t> first(n), prev_nbr(n, -1), prev_leaf(n, -1), uf(n);
  std::vector<int64_t> w(n, 0);
  auto weight = [&](int64_t i) -> int64_t { return wt ? (*wt)[i] : 1; };
  for (int64_t j = 0; j < n; ++j) first[j] = (int32_t)j;
  for (int64_t j = 0; j < n; ++j)
    if (parent[j] >= 0) first[parent[j]] = std::min(first[parent[j]], first[j]);
  for (int64_t j = 0; j < n; ++j) {
    uf[j] = (int32_t)j;
    if (first[j] == j) w[j] = weight(j);  // etree leaf: T_j = {j}
  }
  for (int64_t j = 0; j < n; ++j) {
    if (parent[j] >= 0) w[parent[j]] -= weight(j);
    // rows i > j with C_ij != 0: j may be a leaf of T_i
    for (int64_t q = lptr[j]; q < lptr[j + 1]; ++q) {
      int32_t i = lind[q];
      if (first[j] > prev_nbr[i]) {
        w[j] += weight(i);
        int32_t pl = prev_leaf[i];
        if (pl >= 0) {
          int32_t a = pl;
          while (uf[a] != a) a = uf[a];
          for (int32_t v = pl; v != a;) {  // compress
            int32_t nx = uf[v];
            uf[v] = a;
            v = nx;
          }
          w[a] -= weight(i);
        }
        prev_leaf[i] = (int32_t)j;
      }
      prev_nbr[i] = (int32_t)j;
    }
    if (parent[j] >= 0) uf[j] = parent[j];
  }
  for (int64_t j = 0; j < n; ++j)
    if (parent[j] >= 0) w[parent[j]] += w[j];
  return w;
}

}  // namespace

// The permuted pattern and its elimination quantities for one candidate order.
struct Ordered {
  std::vector<int32_t> perm, pinv, parent;
  std::vector<int64_t> lptr;  // lower triangle of C by columns (rows i > j)
  std::vector<int32_t> lind;
  std::vector<int64_t> colcount;
  int64_t nnzL = 0, flops = 0;
};

// Lower-triangle adjacency of C = P A P^T by columns: for column j the rows i > j.
void lower_by_column(const Pattern& A, const std::vector<int32_t>& pinv, std::vector<int64_t>& lptr,
                     std::vector<int32_t>& lind) {
  const int64_t n = A.n;
  lptr.assign(n + 1, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      const int32_t i = pinv[r], j = pinv[A.colind[k]];
      if (i > j) lptr[j + 1]++;
    }
  for (int64_t j = 0; j < n; ++j) lptr[j + 1] += lptr[j];
  lind.resize(lptr[n]);
  std::vector<int64_t> pos(lptr.begin(), lptr.end() - 1);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      const int32_t i = pinv[r], j = pinv[A.colind[k]];
      if (i > j) lind[pos[j]++] = i;
    }
}

// Etree of the reordered pattern, postorder composed into the final
// permutation, lower-triangle adjacency and column counts (weighted by wt,
// indexed by original vertex, when given).
Ordered order_and_count(const Pattern& A, const std::vector<int32_t>& perm0,
                        const std::vector<int32_t>* wt = nullptr) {
  const int64_t n = A.n;
  Ordered O;
  std::vector<int32_t> pinv0(n);
  for (int64_t k = 0; k < n; ++k) pinv0[perm0[k]] = (int32_t)k;
  std::vector<int32_t> par0;
  {
    std::vector<int64_t> uptr;
    std::vector<int32_t> uind;
    upper_by_column(A, pinv0, uptr, uind);
    par0 = etree(n, uptr, uind);
  }
  std::vector<int32_t> post = postorder(par0);
  O.perm.resize(n);
  O.pinv.resize(n);
  for (int64_t k = 0; k < n; ++k) O.perm[k] = perm0[post[k]];
  for (int64_t k = 0; k < n; ++k) O.pinv[O.perm[k]] = (int32_t)k;
  {
    std::vector<int32_t> postinv(n);
    for (int64_t k = 0; k < n; ++k) postinv[post[k]] = (int32_t)k;
    O.parent.assign(n, -1);
    for (int64_t k = 0; k < n; ++k) {
      const int32_t p = par0[post[k]];
      O.parent[k] = p < 0 ? -1 : postinv[p];
    }
  }
  lower_by_column(A, O.pinv, O.lptr, O.lind);
  std::vector<int32_t> wpost;
  if (wt) {  // weights in permuted numbering
    wpost.resize(n);
    for (int64_t k = 0; k < n; ++k) wpost[k] = (*wt)[O.perm[k]];
  }
  O.colcount = column_counts(n, O.parent, O.lptr, O.lind, wt ? &wpost : nullptr);
  for (int64_t j = 0; j < n; ++j) {
    O.nnzL += O.colcount[j];
    O.flops += O.colcount[j] * O.colcount[j];
  }
  return O;
}

// Relaxed supernodes.  Start from the fundamental supernodes (j, j+1 share
// one iff parent(j) = j+1, j+1 has one child and eta_j = eta_{j+1} + 1) and,
// in column order, merge a supernode p into the group that ends right
// before it when that group is p's child, provided the explicit zeros of
// the merged dense block stay small: with w and m the merged width and
// order, padded = w*m - w(w-1)/2 entries against sum eta_j true ones, merge
// when zeros <= padded/2 (m <= 16), padded/5 (m <= 64) or padded/20.
std::vector<int32_t> relaxed_supernodes(int64_t n, const std::vector<int32_t>& parent,
                                        const std::vector<int64_t>& colcount) {
  std::vector<int32_t> nkids(n, 0);
  for (int64_t j = 0; j < n; ++j)
    if (parent[j] >= 0) nkids[parent[j]]++;
  std::vector<int32_t> fund;
  for (int64_t j = 0; j < n; ++j) {
    const bool extend = j > 0 && parent[j - 1] == j && nkids[j] == 1 &&
                        colcount[j - 1] == colcount[j] + 1;
    if (!extend) fund.push_back((int32_t)j);
  }
  fund.push_back((int32_t)n);
  std::vector<int32_t> start;  // group starts
  int64_t g_true = 0;          // true entries of the last group
  for (size_t p = 0; p + 1 < fund.size(); ++p) {
    const int64_t f = fund[p], l = fund[p + 1];
    int64_t true_p = 0;
    for (int64_t j = f; j < l; ++j) true_p += colcount[j];
    if (!start.empty() && parent[f - 1] == f) {
      const int64_t w = l - start.back();
      const int64_t m = w + colcount[l - 1] - 1;  // rows below l are the last column's
      const int64_t padded = w * m - w * (w - 1) / 2;
      const int64_t zeros = padded - (g_true + true_p);
      const int64_t div = m <= 16 ? 2 : (m <= 64 ? 5 : 20);
      if (zeros * div <= padded) {
        g_true += true_p;
        continue;
      }
    }
    start.push_back((int32_t)f);
    g_true = true_p;
  }
  start.push_back((int32_t)n);
  return start;
}

// Indistinguishable vertices: u and v with the same closed adjacency set
// (row u of the pattern, diagonal included, equals row v).  Multi-DOF
// meshes have one such class per node (both DOFs couple to the same nodes).
// The quotient graph has one vertex per class, numbered by ascending smallest
// member; ordering it and expanding each class into its members (ascending,
// consecutive) gives an order of the full graph at a fraction of the cost.
// Returns false when every class is a single vertex.
bool compress_indistinguishable(const Pattern& A, Pattern& Q, std::vector<int32_t>& cls_ptr,
                                std::vector<int32_t>& cls_members) {
  const int64_t n = A.n;
  auto mix = [](uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  std::vector<uint64_t> h(n);
  for (int64_t v = 0; v < n; ++v) {
    uint64_t s = (uint64_t)(A.rowptr[v + 1] - A.rowptr[v]) * 0x100000001B3ull;
    for (int64_t k = A.rowptr[v]; k < A.rowptr[v + 1]; ++k) s += mix((uint64_t)A.colind[k]);
    h[v] = s;
  }
  auto same_row = [&](int64_t u, int64_t v) {
    const int64_t du = A.rowptr[u + 1] - A.rowptr[u];
    if (du != A.rowptr[v + 1] - A.rowptr[v]) return false;
    return std::equal(A.colind.begin() + A.rowptr[u], A.colind.begin() + A.rowptr[u + 1],
                      A.colind.begin() + A.rowptr[v]);
  };
  // class representative = smallest member; candidates share the hash
  std::vector<int32_t> rep(n, -1);
  std::unordered_map<uint64_t, std::vector<int32_t>> seen;
  seen.reserve((size_t)n);
  int64_t ncls = 0;
  for (int64_t v = 0; v < n; ++v) {
    std::vector<int32_t>& reps = seen[h[v]];
    for (int32_t r : reps)
      if (same_row(r, v)) {
        rep[v] = r;
        break;
      }
    if (rep[v] < 0) {
      rep[v] = (int32_t)v;
      reps.push_back((int32_t)v);
      ++ncls;
    }
  }
  if (ncls == n) return false;
  std::vector<int32_t> cls(n);
  cls_ptr.assign(ncls + 1, 0);
  std::vector<int32_t> reps_in_order;
  reps_in_order.reserve(ncls);
  {
    std::vector<int32_t> id(n, -1);
    for (int64_t v = 0; v < n; ++v) {
      if (rep[v] == v) {
        id[v] = (int32_t)reps_in_order.size();
        reps_in_order.push_back((int32_t)v);
      }
      cls[v] = id[rep[v]];
      cls_ptr[cls[v] + 1]++;
    }
  }
  for (int64_t c = 0; c < ncls; ++c) cls_ptr[c + 1] += cls_ptr[c];
  cls_members.resize(n);
  {
    std::vector<int32_t> pos(cls_ptr.begin(), cls_ptr.end() - 1);
    for (int64_t v = 0; v < n; ++v) cls_members[pos[cls[v]]++] = (int32_t)v;
  }
  Q = Pattern();
  Q.n = ncls;
  Q.rowptr.assign(ncls + 1, 0);
  std::vector<int32_t> row;
  for (int64_t c = 0; c < ncls; ++c) {
    const int32_t r = reps_in_order[c];
    row.clear();
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) row.push_back(cls[A.colind[k]]);
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    Q.colind.insert(Q.colind.end(), row.begin(), row.end());
    Q.rowptr[c + 1] = (int64_t)Q.colind.size();
  }
  return true;
}

// Quotient pattern of a partition of the vertices into classes (members
// ascending, classes numbered by ascending smallest member when the partition
// comes from indistinguishable vertices, by the caller's ids otherwise), and
// whether every class is a set of indistinguishable vertices (equal rows of
// the pattern, diagonal included).
struct Condensed {
  Pattern Q;
  std::vector<int32_t> cptr, cmem, size;
  bool exact = false;
};

namespace {

bool quotient_by_map(const Pattern& A, const std::vector<int32_t>& cls, int64_t ncls,
                     Condensed& C, std::string& err) {
  const int64_t n = A.n;
  C.cptr.assign(ncls + 1, 0);
  for (int64_t v = 0; v < n; ++v) C.cptr[cls[v] + 1]++;
  for (int64_t c = 0; c < ncls; ++c) {
    if (C.cptr[c + 1] == 0) {
      err = "dof map: condensed vertex " + std::to_string(c) + " has no DOF";
      return false;
    }
    C.cptr[c + 1] += C.cptr[c];
  }
  C.cmem.resize(n);
  {
    std::vector<int32_t> pos(C.cptr.begin(), C.cptr.end() - 1);
    for (int64_t v = 0; v < n; ++v) C.cmem[pos[cls[v]]++] = (int32_t)v;
  }
  C.Q = Pattern();
  C.Q.n = ncls;
  C.Q.rowptr.assign(ncls + 1, 0);
  std::vector<int32_t> row;
  C.exact = true;
  for (int64_t c = 0; c < ncls; ++c) {
    row.clear();
    const int32_t r0 = C.cmem[C.cptr[c]];
    for (int32_t q = C.cptr[c]; q < C.cptr[c + 1]; ++q) {
      const int32_t r = C.cmem[q];
      for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) row.push_back(cls[A.colind[k]]);
      if (C.exact && r != r0 &&
          !(A.rowptr[r + 1] - A.rowptr[r] == A.rowptr[r0 + 1] - A.rowptr[r0] &&
            std::equal(A.colind.begin() + A.rowptr[r], A.colind.begin() + A.rowptr[r + 1],
                       A.colind.begin() + A.rowptr[r0])))
        C.exact = false;
    }
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    C.Q.colind.insert(C.Q.colind.end(), row.begin(), row.end());
    C.Q.rowptr[c + 1] = (int64_t)C.Q.colind.size();
  }
  return true;
}

// The condensed graph the options ask for: indistinguishable vertices
// (dof_block 0), none (1), blocks of dof_block consecutive rows, or the
// caller's DOF map.  Returns false when there is nothing to condense (or on
// an error, with err set).
bool condense(const Pattern& A, const SymOptions& opt, Condensed& C, std::string& err) {
  const int64_t n = A.n;
  if (opt.dof_map) {
    if (opt.dof_map_n != n) {
      err = "dof map has " + std::to_string(opt.dof_map_n) + " entries for " + std::to_string(n) +
            " rows";
      return false;
    }
    int64_t ncls = 0;
    for (int64_t v = 0; v < n; ++v) {
      if (opt.dof_map[v] < 0 || opt.dof_map[v] >= n) {
        err = "dof map entry " + std::to_string(v) + " out of range";
        return false;
      }
      ncls = std::max<int64_t>(ncls, opt.dof_map[v] + 1);
    }
    if (ncls == n) return false;
    std::vector<int32_t> cls(opt.dof_map, opt.dof_map + n);
    if (!quotient_by_map(A, cls, ncls, C, err)) return false;
  } else if (opt.dof_block >= 2) {
    const int64_t b = opt.dof_block;
    if (n % b != 0) {
      err = "dof_block " + std::to_string(b) + " does not divide n = " + std::to_string(n);
      return false;
    }
    std::vector<int32_t> cls(n);
    for (int64_t v = 0; v < n; ++v) cls[v] = (int32_t)(v / b);
    if (!quotient_by_map(A, cls, n / b, C, err)) return false;
  } else if (opt.dof_block == 1) {
    return false;
  } else {
    if (!compress_indistinguishable(A, C.Q, C.cptr, C.cmem)) return false;
    C.exact = true;
  }
  C.size.resize(C.Q.n);
  for (int64_t c = 0; c < C.Q.n; ++c) C.size[c] = C.cptr[c + 1] - C.cptr[c];
  return true;
}

std::vector<int32_t> dissection(const Pattern& P, int method, int leaf) {
  return method == 1 ? nested_dissection(P, leaf) : levelset_dissection(P, leaf);
}

// One ordering candidate.  On a condensed graph the dissection runs on the
// quotient and each class's members stay consecutive (ascending), and the
// elimination tree, postorder and column counts follow from the quotient's
// (counts weighted by class sizes): the t-th member of class v has eta =
// W_v - t with W_v the weighted count of v, its parent is the next member,
// and the last member's parent is the first member of v's parent class.
// That is the exact structure of P A P^T when the classes are
// indistinguishable, and otherwise the structure of the class-expanded
// pattern (every member's row the union of its class's rows), whose extra
// entries the factorization stores as exact zeros.  The full lower adjacency
// is built once, for the candidate that is kept.
Ordered order_candidate(const Pattern& A, const Condensed* C, int method, int leaf) {
  if (!C) return order_and_count(A, dissection(A, method, leaf));
  const Pattern& Q = C->Q;
  const int qleaf = std::max(1, (int)(leaf * (int64_t)Q.n / std::max<int64_t>(1, A.n)));
  std::vector<int32_t> pq = dissection(Q, method, qleaf);
  Ordered Oq = order_and_count(Q, pq, &C->size);
  const int64_t nq = Q.n, n = A.n;
  std::vector<int64_t> off(nq + 1, 0);
  for (int64_t k = 0; k < nq; ++k) off[k + 1] = off[k] + C->size[Oq.perm[k]];
  Ordered O;
  O.perm.resize(n);
  O.pinv.resize(n);
  O.parent.resize(n);
  O.colcount.resize(n);
  for (int64_t k = 0; k < nq; ++k) {
    const int32_t c = Oq.perm[k];
    const int64_t b = C->size[c];
    for (int64_t t = 0; t < b; ++t) {
      const int64_t j = off[k] + t;
      O.perm[j] = C->cmem[C->cptr[c] + t];
      O.parent[j] = t + 1 < b ? (int32_t)(j + 1) : (Oq.parent[k] < 0 ? -1 : (int32_t)off[Oq.parent[k]]);
      O.colcount[j] = Oq.colcount[k] - t;
    }
  }
  for (int64_t j = 0; j < n; ++j) {
    O.pinv[O.perm[j]] = (int32_t)j;
    O.nnzL += O.colcount[j];
    O.flops += O.colcount[j] * O.colcount[j];
  }
  return O;
}

}  // namespace

// Pattern with every member's row replaced by the union of its class's rows
// (classes adjacent in the quotient become dense blocks).
Pattern expand_classes(const Pattern& A, const Condensed& C) {
  Pattern B;
  B.n = A.n;
  B.rowptr.assign(A.n + 1, 0);
  const int64_t nq = C.Q.n;
  std::vector<int32_t> row;
  std::vector<std::vector<int32_t>> rows(nq);
  for (int64_t c = 0; c < nq; ++c) {
    row.clear();
    for (int64_t k = C.Q.rowptr[c]; k < C.Q.rowptr[c + 1]; ++k) {
      const int32_t u = C.Q.colind[k];
      row.insert(row.end(), C.cmem.begin() + C.cptr[u], C.cmem.begin() + C.cptr[u + 1]);
    }
    std::sort(row.begin(), row.end());
    rows[c] = row;
    for (int32_t q = C.cptr[c]; q < C.cptr[c + 1]; ++q) B.rowptr[C.cmem[q] + 1] = (int64_t)row.size();
  }
  for (int64_t i = 0; i < A.n; ++i) B.rowptr[i + 1] += B.rowptr[i];
  B.colind.resize(B.rowptr[A.n]);
  for (int64_t c = 0; c < nq; ++c)
    for (int32_t q = C.cptr[c]; q < C.cptr[c + 1]; ++q)
      std::copy(rows[c].begin(), rows[c].end(), B.colind.begin() + B.rowptr[C.cmem[q]]);
  return B;
}

// One system's order: the requested dissection, or both candidates run
// concurrently (they share only the read-only pattern) and the one with
// fewer flops kept; `used` receives the method.  With a condensed graph whose
// classes are not indistinguishable, the result (counts and lower adjacency)
// describes the class-expanded pattern.
Ordered choose_order(const Pattern& A, const SymOptions& opt, int& used) {
  Condensed C;
  std::string err;
  const bool cond = condense(A, opt, C, err);
  if (!err.empty()) throw std::invalid_argument(err);
  const Condensed* cp = cond ? &C : nullptr;
  Ordered O;
  if (opt.ordering == 1 || opt.ordering == 2) {
    used = opt.ordering;
    O = order_candidate(A, cp, opt.ordering, opt.nd_leaf_size);
  } else {
    Ordered O2;
    std::exception_ptr failed;
    std::thread t2([&] {
      try {
        O2 = order_candidate(A, cp, 2, opt.nd_leaf_size);
      } catch (...) {
        failed = std::current_exception();
      }
    });
    try {
      O = order_candidate(A, cp, 1, opt.nd_leaf_size);
    } catch (...) {
      t2.join();
      throw;
    }
    t2.join();
    if (failed) std::rethrow_exception(failed);
    used = 1;
    if (O2.flops < O.flops) {
      used = 2;
      O = std::move(O2);
    }
  }
  if (cond && !C.exact) {
    lower_by_column(expand_classes(A, C), O.pinv, O.lptr, O.lind);
  } else if (O.lptr.empty()) {
    lower_by_column(A, O.pinv, O.lptr, O.lind);
  }
  return O;
}

int analyze_pattern(Symbolic& S, const SymOptions& opt, std::string& err) {
  const Pattern& A = S.A;
  const int64_t n = A.n;
  S.n = n;
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();

  // 1. fill-reducing order: nested dissection (multilevel and/or level
  // structure), composed with an etree postorder; with both candidates the
  // one with fewer factorization flops is kept.  The systems of a batch are
  // ordered one by one, exactly as each would be alone, so that a system's
  // ordering (and with it every later result) does not depend on the other
  // systems; their postordered orders concatenated are a postorder of the
  // block-diagonal union, which order_and_count keeps as it is.
  Ordered O;
  if (S.nsys > 1) {
    const int64_t nsys = S.nsys;
    std::vector<std::vector<int32_t>> sub_perm(nsys);
    std::vector<int> sub_used(nsys, 0);
    std::atomic<int64_t> next{0};
    std::exception_ptr failed;
    std::mutex failed_mu;
    auto worker = [&]() {
      for (int64_t k = next++; k < nsys; k = next++) {
        try {
          const int64_t r0 = S.sys_ptr[k], r1 = S.sys_ptr[k + 1];
          Pattern Ak;
          Ak.n = r1 - r0;
          Ak.rowptr.resize(Ak.n + 1);
          const int64_t q0 = A.rowptr[r0];
          for (int64_t i = 0; i <= Ak.n; ++i) Ak.rowptr[i] = A.rowptr[r0 + i] - q0;
          Ak.colind.resize(A.rowptr[r1] - q0);
          for (int64_t q = q0; q < A.rowptr[r1]; ++q) Ak.colind[q - q0] = (int32_t)(A.colind[q] - r0);
          Ordered Ok = choose_order(Ak, opt, sub_used[k]);
          sub_perm[k] = std::move(Ok.perm);
        } catch (...) {
          std::lock_guard<std::mutex> g(failed_mu);
          if (!failed) failed = std::current_exception();
        }
      }
    };
    const int nw = (int)std::max<int64_t>(1, std::min<int64_t>(
        nsys, std::max(1u, std::thread::hardware_concurrency()) / 2));
    std::vector<std::thread> pool;
    for (int t = 1; t < nw; ++t) pool.emplace_back(worker);
    worker();
    for (auto& t : pool) t.join();
    if (failed) std::rethrow_exception(failed);
    std::vector<int32_t> perm;
    perm.reserve(n);
    int used_mask = 0;
    for (int64_t k = 0; k < nsys; ++k) {
      for (int32_t v : sub_perm[k]) perm.push_back((int32_t)(v + S.sys_ptr[k]));
      used_mask |= sub_used[k] > 0 ? 1 << (sub_used[k] - 1) : 0;
    }
    O = order_and_count(A, perm);
    S.ordering_used = used_mask;  // 1, 2, or 3 when the systems used both methods
  } else {
    O = choose_order(A, opt, S.ordering_used);
  }
  S.perm = std::move(O.perm);
  S.pinv = std::move(O.pinv);
  S.parent = std::move(O.parent);
  S.colcount = std::move(O.colcount);
  S.nnzL = O.nnzL;
  S.flops = O.flops;
  std::vector<int64_t> lptr = std::move(O.lptr);
  std::vector<int32_t> lind = std::move(O.lind);
  const auto t1 = clk::now();
  S.t_order_us = std::chrono::duration_cast<std::chrono::microseconds>(t1 - t0).count();

  // 2. relaxed supernodes and the supernodal tree.
  S.sptr = relaxed_supernodes(n, S.parent, S.colcount);
  S.ns = (int32_t)S.sptr.size() - 1;
  S.col2sn.assign(n, 0);
  for (int32_t s = 0; s < S.ns; ++s)
    for (int32_t j = S.sptr[s]; j < S.sptr[s + 1]; ++j) S.col2sn[j] = s;
  const int32_t ns = S.ns;
  S.sparent.assign(ns, -1);
  for (int32_t s = 0; s < ns; ++s) {
    int32_t last = S.sptr[s + 1] - 1;
    S.sparent[s] = S.parent[last] < 0 ? -1 : S.col2sn[S.parent[last]];
  }
  S.child_ptr.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s)
    if (S.sparent[s] >= 0) S.child_ptr[S.sparent[s] + 1]++;
  for (int32_t s = 0; s < ns; ++s) S.child_ptr[s + 1] += S.child_ptr[s];
  S.child_list.resize(S.child_ptr[ns]);
  {
    std::vector<int32_t> pos(S.child_ptr.begin(), S.child_ptr.end() - 1);
    for (int32_t s = 0; s < ns; ++s)  // ascending child ids
      if (S.sparent[s] >= 0) S.child_list[pos[S.sparent[s]]++] = s;
  }

  // 5. row structures: pivots, A's rows below the supernode, children's update rows.
  // A supernode's rows below its last pivot are those of its last column, so
  // m_s = w_s + eta_{l_s - 1} - 1 (explicit zeros of relaxed supernodes
  // included).
  S.front_m.assign(ns, 0);
  S.rows_ptr.assign(ns + 1, 0);
  for (int32_t s = 0; s < ns; ++s)
    S.front_m[s] = (S.sptr[s + 1] - S.sptr[s]) + (int32_t)S.colcount[S.sptr[s + 1] - 1] - 1;
  S.nnz_front = 0;
  for (int32_t s = 0; s < ns; ++s) {
    S.rows_ptr[s + 1] = S.rows_ptr[s] + S.front_m[s];
    const int64_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
    S.nnz_front += w * m - w * (w - 1) / 2;
  }
  S.rows.assign(S.rows_ptr[ns], 0);
  S.rmap.assign(S.rows_ptr[ns], -1);
  {
    std::vector<int32_t> mark(n, -1);
    std::vector<int32_t> tmp;
    for (int32_t s = 0; s < ns; ++s) {
      const int32_t f = S.sptr[s], l = S.sptr[s + 1];
      tmp.clear();
      for (int32_t j = f; j < l; ++j) { mark[j] = s; tmp.push_back(j); }
      for (int32_t j = f; j < l; ++j)
        for (int64_t q = lptr[j]; q < lptr[j + 1]; ++q) {
          int32_t i = lind[q];
          if (mark[i] != s) { mark[i] = s; tmp.push_back(i); }
        }
      for (int32_t q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
        int32_t c = S.child_list[q];
        int32_t wc = S.sptr[c + 1] - S.sptr[c];
        for (int64_t k = S.rows_ptr[c] + wc; k < S.rows_ptr[c + 1]; ++k) {
          int32_t i = S.rows[k];
          if (mark[i] != s) { mark[i] = s; tmp.push_back(i); }
        }
      }
      std::sort(tmp.begin(), tmp.end());
      if ((int64_t)tmp.size() != S.front_m[s]) {
        err = "internal error: row structure of supernode " + std::to_string(s) +
              " disagrees with the column count";
        return kInvalid;
      }
      std::copy(tmp.begin(), tmp.end(), S.rows.begin() + S.rows_ptr[s]);
    }
  }
  // relative maps of each child's update rows into the parent's rows
  {
    std::vector<int32_t> where(n, -1);
    for (int32_t s = 0; s < ns; ++s) {
      for (int64_t k = S.rows_ptr[s]; k < S.rows_ptr[s + 1]; ++k)
        where[S.rows[k]] = (int32_t)(k - S.rows_ptr[s]);
      for (int32_t q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
        int32_t c = S.child_list[q];
        int32_t wc = S.sptr[c + 1] - S.sptr[c];
        for (int64_t k = S.rows_ptr[c] + wc; k < S.rows_ptr[c + 1]; ++k) {
          int32_t pos = where[S.rows[k]];
          if (pos < 0) {
            err = "internal error: child row missing from parent front";
            return kInvalid;
          }
          S.rmap[k] = pos;
        }
      }
      for (int64_t k = S.rows_ptr[s]; k < S.rows_ptr[s + 1]; ++k) where[S.rows[k]] = -1;
    }
  }

  // 6. A-entry -> front maps: lower triangle of C by permuted column, values
  // from the original lower triangle (row >= col).
  S.acol_ptr.assign(n + 1, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k)
      if (r >= A.colind[k]) {
        int32_t a = S.pinv[r], b = S.pinv[A.colind[k]];
        S.acol_ptr[std::min(a, b) + 1]++;
      }
  for (int64_t j = 0; j < n; ++j) S.acol_ptr[j + 1] += S.acol_ptr[j];
  S.a_src.assign(S.acol_ptr[n], -1);
  S.a_row.assign(S.acol_ptr[n], 0);
  {
    std::vector<int64_t> pos(S.acol_ptr.begin(), S.acol_ptr.end() - 1);
    std::vector<int32_t> rowat(n, -1);
    for (int64_t r = 0; r < n; ++r)
      for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k)
        if (r >= A.colind[k]) {
          int32_t a = S.pinv[r], b = S.pinv[A.colind[k]];
          int32_t col = std::min(a, b), row = std::max(a, b);
          S.a_src[pos[col]] = A.src[k];
          S.a_row[pos[col]] = row;  // global row for now
          pos[col]++;
        }
    for (int32_t s = 0; s < ns; ++s) {
      for (int64_t k = S.rows_ptr[s]; k < S.rows_ptr[s + 1]; ++k)
        rowat[S.rows[k]] = (int32_t)(k - S.rows_ptr[s]);
      for (int32_t j = S.sptr[s]; j < S.sptr[s + 1]; ++j)
        for (int64_t q = S.acol_ptr[j]; q < S.acol_ptr[j + 1]; ++q) S.a_row[q] = rowat[S.a_row[q]];
      for (int64_t k = S.rows_ptr[s]; k < S.rows_ptr[s + 1]; ++k) rowat[S.rows[k]] = -1;
    }
  }

  // 7. levels by height (leaves 0); children have smaller ids than parents.
  S.height.assign(ns, 0);
  for (int32_t s = 0; s < ns; ++s)
    if (S.sparent[s] >= 0)
      S.height[S.sparent[s]] = std::max(S.height[S.sparent[s]], S.height[s] + 1);
  S.nlevels = 0;
  for (int32_t s = 0; s < ns; ++s) S.nlevels = std::max(S.nlevels, S.height[s] + 1);
  S.level_ptr.assign(S.nlevels + 1, 0);
  for (int32_t s = 0; s < ns; ++s) S.level_ptr[S.height[s] + 1]++;
  for (int32_t h = 0; h < S.nlevels; ++h) S.level_ptr[h + 1] += S.level_ptr[h];
  S.level_list.resize(ns);
  {
    std::vector<int32_t> pos(S.level_ptr.begin(), S.level_ptr.end() - 1);
    for (int32_t s = 0; s < ns; ++s) S.level_list[pos[S.height[s]]++] = s;
  }
  S.max_m = S.max_w = S.max_child_r = 0;
  for (int32_t s = 0; s < ns; ++s) {
    S.max_m = std::max<int64_t>(S.max_m, S.front_m[s]);
    S.max_w = std::max<int64_t>(S.max_w, S.sptr[s + 1] - S.sptr[s]);
  }
  S.t_structure_us =
      std::chrono::duration_cast<std::chrono::microseconds>(clk::now() - t1).count();
  return kOk;
}

// LU of a matrix with a symmetric pattern: for every A entry q of the
// assembly maps (the lower triangle of C = P A P^T, in the maps' order), the
// caller's index of C(row, col) (lo) and of its transposed twin C(col, row)
// (up; -1 on the diagonal and where the caller's pattern lacks the entry).
// The loop visits the entries in the order the maps were filled.
void lu_value_sources(const Symbolic& S, std::vector<int64_t>& lo, std::vector<int64_t>& up) {
  const Pattern& A = S.A;
  const int64_t n = A.n;
  lo.assign(S.acol_ptr[n], -1);
  up.assign(S.acol_ptr[n], -1);
  std::vector<int64_t> pos(S.acol_ptr.begin(), S.acol_ptr.end() - 1);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      const int32_t c = A.colind[k];
      if (r < c) continue;
      const int32_t a = S.pinv[r], b = S.pinv[c];
      const int64_t q = pos[std::min(a, b)]++;
      int64_t twin = -1;
      if (r != c) {
        const int32_t* b0 = A.colind.data() + A.rowptr[c];
        const int32_t* e0 = A.colind.data() + A.rowptr[c + 1];
        const int32_t* p = std::lower_bound(b0, e0, (int32_t)r);
        if (p != e0 && *p == (int32_t)r) twin = A.src[A.rowptr[c] + (p - b0)];
      }
      // C(a, b) = A(r, c) and C(b, a) = A(c, r)
      lo[q] = a >= b ? A.src[k] : twin;
      up[q] = a >= b ? twin : A.src[k];
    }
}

}  // namespace tacho
