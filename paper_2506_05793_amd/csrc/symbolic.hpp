// Host symbolic analysis: ordering, elimination tree, column counts,
// fundamental supernodes, front row structures and maps, level schedule.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"

namespace tacho {

struct SymOptions {
  int nd_leaf_size = 8;
  int ordering = 0;  // 0: the better of 1 and 2 (fewer flops), 1: multilevel ND, 2: level-structure ND
  // condensed graph: 0 indistinguishable vertices, 1 none, b >= 2 blocks of b
  // consecutive rows; dof_map (n entries, condensed vertex of each row)
  // overrides dof_block
  int dof_block = 0;
  const int32_t* dof_map = nullptr;
  int64_t dof_map_n = 0;
};

// Pattern of the full symmetric matrix, validated, diagonal present.
struct Pattern {
  int64_t n = 0;
  std::vector<int64_t> rowptr;  // n+1
  std::vector<int32_t> colind;  // rows sorted ascending
  std::vector<int64_t> src;     // for each entry: index into the caller's values, -1 if added
};

struct Symbolic {
  int64_t n = 0;
  int64_t nsys = 1;
  std::vector<int64_t> sys_ptr;  // nsys+1, row ranges of the independent systems
  Pattern A;                     // validated input pattern (original numbering)
  int64_t nnz_input = 0;         // length of the caller's values array

  std::vector<int32_t> perm, pinv;  // perm: new -> old
  std::vector<int32_t> parent;      // etree of P A P^T
  std::vector<int64_t> colcount;    // eta_j
  int64_t nnzL = 0, flops = 0;
  int64_t nnz_front = 0;  // stored factor entries incl. explicit zeros of relaxed supernodes
  int ordering_used = 0;  // 1 multilevel, 2 level-structure
  int64_t t_order_us = 0, t_structure_us = 0, t_plan_us = 0;  // analysis phase times

  // supernodes
  int32_t ns = 0;
  std::vector<int32_t> sptr;     // ns+1
  std::vector<int32_t> sparent;  // ns
  std::vector<int32_t> col2sn;   // n
  std::vector<int32_t> front_m;  // ns, m_s = |rows(s)|
  std::vector<int64_t> rows_ptr;  // ns+1
  std::vector<int32_t> rows;      // rows(s): sorted permuted row indices, first w are pivots
  std::vector<int32_t> rmap;      // same indexing as rows; for k >= w_s the position of
                                  // rows(s)[k] within rows(parent(s))
  std::vector<int32_t> child_ptr, child_list;  // children ascending

  // assembly of A: per permuted column j, the lower-triangle entries of C
  std::vector<int64_t> acol_ptr;  // n+1
  std::vector<int64_t> a_src;     // index into the caller's values
  std::vector<int32_t> a_row;     // row position inside the front of col2sn[j]

  // level schedule (height: leaves 0)
  std::vector<int32_t> height;    // ns
  int32_t nlevels = 0;
  std::vector<int32_t> level_ptr, level_list;  // supernodes of each level, ascending

  int64_t max_m = 0, max_w = 0;
  int64_t max_child_r = 0;
};

int build_pattern(int64_t n, const int64_t* rowptr, const int32_t* colind, Pattern& P,
                  std::string& err);

// Fill-reducing ordering (new -> old) by nested dissection on the adjacency
// graph of P (self loops ignored).
std::vector<int32_t> nested_dissection(const Pattern& P, int leaf_size);
std::vector<int32_t> levelset_dissection(const Pattern& P, int leaf_size);

// Classes of indistinguishable vertices (equal rows of the pattern) and the
// quotient pattern; false when there is nothing to compress.
bool compress_indistinguishable(const Pattern& A, Pattern& Q, std::vector<int32_t>& cls_ptr,
                                std::vector<int32_t>& cls_members);

int analyze_pattern(Symbolic& S, const SymOptions& opt, std::string& err);

void lu_value_sources(const Symbolic& S, std::vector<int64_t>& lo, std::vector<int64_t>& up);

}  // namespace tacho
