// Memory layout and launch plan of the numeric phase (host).
//
// Factor storage: one dense column-major panel of m_s x w_s per supernode
// (the paper's dense supernodal blocks L_ii / L_ki, Tacho section), leading
// dimension m_s rounded up to kLdAlign elements.  Update matrices U_s
// (r_s x r_s, r_s = m_s - w_s) live in a workspace whose blocks are reused
// across levels: U_s is created at its own level and released once its
// parent's level has assembled it, placed best-fit.
//
// Launch plan, per level of the supernodal elimination tree (level-set
// scheduling, Tacho section), leaves first:
//   small fronts (m <= kSmallMax, and for Cholesky m <= kPackedMax with one
//     pivot block): one launch, one workgroup per front, the whole front
//     assembled and partially factored in LDS;
//   large fronts: assembly into the panels / update matrices, then
//     front_mode 0 (Cholesky): one dataflow launch of 64-row tile tasks per
//     level (per group of chain fronts where a level has many);
//     front_mode 1 (LDL^T): for every panel of kPanel columns a
//     diagonal-block launch, a triangular solve launch for the rows below and
//     an update launch of the remaining columns of its kOuter-wide outer
//     panel; after each outer panel one update launch with K = kOuter of the
//     remaining pivot columns; finally one update launch U -= L21 L21^T.
#include <algorithm>
#include <array>
#include <climits>
#include <map>
#include <set>

#include "plan.hpp"

namespace tacho {
namespace {

// Best-fit allocator over a growing arena: a request takes the smallest free
// block that holds it (lowest offset among equals), freed blocks coalesce
// with their neighbours.  O(log blocks) per call.
class BestFit {
 public:
  int64_t alloc(int64_t size) {
    auto it = by_size_.lower_bound({size, INT64_MIN});
    if (it == by_size_.end()) {
      // grow: a free block at the top of the arena is extended
      if (!by_off_.empty()) {
        auto last = std::prev(by_off_.end());
        if (last->first + last->second == top_) {
          const int64_t off = last->first;
          by_size_.erase({last->second, off});
          by_off_.erase(last);
          top_ = off + size;
          return off;
        }
      }
      const int64_t off = top_;
      top_ += size;
      return off;
    }
    const int64_t bsize = it->first, off = it->second;
    by_size_.erase(it);
    by_off_.erase(off);
    if (bsize > size) insert(off + size, bsize - size);
    return off;
  }
  void release(int64_t off, int64_t size) {
    auto nx = by_off_.lower_bound(off);
    if (nx != by_off_.end() && off + size == nx->first) {
      size += nx->second;
      by_size_.erase({nx->second, nx->first});
      nx = by_off_.erase(nx);
    }
    if (nx != by_off_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        size += pv->second;
        by_size_.erase({pv->second, pv->first});
        by_off_.erase(pv);
      }
    }
    insert(off, size);
  }
  int64_t peak() const { return top_; }

 private:
  void insert(int64_t off, int64_t size) {
    by_off_.emplace(off, size);
    by_size_.insert({size, off});
  }
  std::map<int64_t, int64_t> by_off_;
  std::set<std::pair<int64_t, int64_t>> by_size_;
  int64_t top_ = 0;
};

// Algorithmic flops of the partial factorization of front s: sum_{j<w} (m-j)^2.
double front_flops(const Symbolic& S, int32_t s) {
  const double m = S.front_m[s], w = S.sptr[s + 1] - S.sptr[s];
  double f = 0;
  for (double j = 0; j < w; ++j) f += (m - j) * (m - j);
  return f;
}

// Algorithmic element traffic of assembling and writing front s: its A
// entries, its children's update matrices (lower triangles), the L
// trapezoid and its own update matrix written once.
double front_io(const Symbolic& S, int32_t s) {
  const double m = S.front_m[s], w = S.sptr[s + 1] - S.sptr[s], r = m - w;
  double e = (double)(S.acol_ptr[S.sptr[s + 1]] - S.acol_ptr[S.sptr[s]]);
  for (int32_t q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int32_t c = S.child_list[q];
    const double rc = S.front_m[c] - (S.sptr[c + 1] - S.sptr[c]);
    e += rc * (rc + 1) / 2;
  }
  e += w * m - w * (w - 1) / 2 + r * (r + 1) / 2;
  return e;
}

}  // namespace

int build_plan(const Symbolic& S, Plan& P, std::string& err, int front_mode,
               const PlanTuning& tune) {
  const int32_t urange = tune.u_range > 0 ? tune.u_range : kURange;
  const int32_t chain_min = tune.chain_min == 0 ? kChainMin : tune.chain_min;
  const int32_t level_fronts = tune.level_fronts > 0 ? tune.level_fronts : kLevelFronts;
  const int32_t asm_cols = tune.asm_cols > 0 ? tune.asm_cols : kAsmCols;
  const int32_t solo_m = tune.solo_m == 0 ? kSoloM : tune.solo_m;  // negative: never
  const bool inplace = tune.chain_inplace >= 0;  // default: in place
  const int32_t ns = S.ns;
  P.front_mode = front_mode;
  static_assert(kPanel == 64, "front task tiling assumes 64-column pivot blocks");
  P.L_off.assign(ns, 0);
  P.U_off.assign(ns, -1);
  P.u_off.assign(ns, 0);
  P.ldL.assign(ns, 0);
  P.ldU.assign(ns, 0);
  int64_t off = 0, uoff = 0;
  for (int32_t s = 0; s < ns; ++s) {
    const int64_t m = S.front_m[s], w = S.sptr[s + 1] - S.sptr[s], r = m - w;
    if (m > 46000) {
      err = "front of order " + std::to_string(m) + " exceeds the supported maximum";
      return kInvalid;
    }
    P.ldL[s] = (int32_t)round_up(m, kLdAlign);
    P.ldU[s] = (int32_t)round_up(std::max<int64_t>(r, 1), kLdAlign);
    P.L_off[s] = off;
    off += (int64_t)P.ldL[s] * w;
    P.u_off[s] = uoff;
    uoff += r;
  }
  P.L_elems = off;
  P.u_elems = uoff;

  // update-matrix workspace, best-fit by level
  BestFit ff;
  for (int32_t h = 0; h < S.nlevels; ++h) {
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
      int32_t s = S.level_list[q];
      int64_t r = S.front_m[s] - (S.sptr[s + 1] - S.sptr[s]);
      if (r > 0) P.U_off[s] = ff.alloc(round_up((int64_t)P.ldU[s] * r, 64));
    }
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
      int32_t s = S.level_list[q];
      for (int32_t c = S.child_ptr[s]; c < S.child_ptr[s + 1]; ++c) {
        int32_t ch = S.child_list[c];
        int64_t r = S.front_m[ch] - (S.sptr[ch + 1] - S.sptr[ch]);
        if (r > 0) ff.release(P.U_off[ch], round_up((int64_t)P.ldU[ch] * r, 64));
      }
    }
  }
  P.U_elems = ff.peak();

  // A-entry positions inside front panels, diagonal entry per column
  P.a_pos.assign(S.a_row.size(), 0);
  P.diag_q.assign(S.n, -1);
  for (int32_t s = 0; s < ns; ++s) {
    const int32_t f = S.sptr[s];
    for (int32_t j = f; j < S.sptr[s + 1]; ++j)
      for (int64_t q = S.acol_ptr[j]; q < S.acol_ptr[j + 1]; ++q) {
        P.a_pos[q] = S.a_row[q] + (j - f) * P.ldL[s];
        if (S.a_row[q] == j - f && S.a_src[q] >= 0) P.diag_q[j] = (int32_t)q;
      }
  }

  // launch sequence
  P.steps.clear();
  P.small_list.clear();
  P.asm_items.clear();
  P.asm_rng.clear();
  P.diag_items.clear();
  P.panel_items.clear();
  // diagonal-block inverse storage of every large front
  P.wbase.assign(ns, -1);
  P.woff.clear();
  P.W_elems = 0;
  P.tbase.assign(1, 0);
  for (int32_t s = 0; s < ns; ++s) {
    if (S.front_m[s] <= kSmallMax) continue;
    const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
    P.wbase[s] = (int32_t)P.woff.size();
    for (int32_t k = 0; k < w; k += kPanel) {
      const int64_t kb = std::min(kPanel, w - k);
      P.woff.push_back(P.W_elems);
      P.W_elems += kb * kb;
      const int64_t next = (int64_t)P.tbase.back() + front_block_tiles(m, w, k / kPanel);
      if (next > INT32_MAX) {
        err = "too many factorization tiles";
        return kInvalid;
      }
      P.tbase.push_back((int32_t)next);
    }
  }
  P.probs.clear();
  P.tiles.clear();
  P.ftasks.clear();
  P.nucount = 0;
  P.front_launches = 0;
  P.pt1base.assign(P.woff.size(), -1);
  P.pt1_slots = 0;
  // Problems of one update launch group; tiles are emitted per tile size so
  // that every launch uses a single tile shape.
  std::vector<int32_t> group;
  auto add_gemm = [&](const GemmProb& g) {
    group.push_back((int32_t)P.probs.size());
    P.probs.push_back(g);
  };
  auto add_gemm_step = [&](int32_t h) {
    for (int pass = 0; pass < 2; ++pass) {
      const int T = pass == 0 ? kGemmTileBig : kGemmTile;
      Step st{kStepGemm, h, (int64_t)P.tiles.size(), 0};
      st.tile = T;
      for (int32_t pid : group) {
        const GemmProb& g = P.probs[pid];
        const bool big = (int64_t)g.M * g.N >= kGemmBigMin;
        if (big != (pass == 0)) continue;
        const int32_t nti = (g.M + T - 1) / T, ntj = (g.N + T - 1) / T;
        for (int32_t tj = 0; tj < ntj; ++tj)
          for (int32_t ti = 0; ti < nti; ++ti)
            if ((int64_t)ti * T + T - 1 >= (int64_t)tj * T) P.tiles.push_back({pid, ti, tj, T});
        const double Nn = g.N, Mm = g.M, Kk = g.K;
        const double lower = Nn * (Nn + 1) / 2 + (Mm - Nn) * Nn;  // outputs with row >= col
        st.flops += 2.0 * Kk * lower;
        st.elems += Mm * Kk + 2.0 * lower;
      }
      st.end = (int64_t)P.tiles.size();
      if (st.end > st.begin) P.steps.push_back(st);
    }
    group.clear();
  };
  std::vector<int32_t> big;
  for (int32_t h = 0; h < S.nlevels; ++h) {
    big.clear();
    int64_t b0 = (int64_t)P.small_list.size();
    // leaves with one pivot column first (one thread each), then the rest
    auto leaf = [&](int32_t s) {
      return S.sptr[s + 1] - S.sptr[s] == 1 && S.child_ptr[s] == S.child_ptr[s + 1] &&
             S.front_m[s] <= kLeafMax;
    };
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q)
      if (leaf(S.level_list[q])) P.small_list.push_back(S.level_list[q]);
    const int32_t nleaf = (int32_t)((int64_t)P.small_list.size() - b0);
    // Cholesky fronts a little larger than kSmallMax with one pivot block
    // (a decision of the front's shape alone) go to the packed-LDS kernel
    auto packed = [&](int32_t s) {
      return front_mode == 0 && S.front_m[s] > kSmallMax && S.front_m[s] <= kPackedMax &&
             S.sptr[s + 1] - S.sptr[s] <= kSmallMax;
    };
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
      int32_t s = S.level_list[q];
      if (leaf(s) || packed(s))
        continue;
      else if (S.front_m[s] <= kSmallMax)
        P.small_list.push_back(s);
      else
        big.push_back(s);
    }
    // the smaller-LDS instance holds the front and, after it, the inverse of
    // its diagonal block: w (m + 1) entries
    auto packed_mid = [&](int32_t s) {
      const int64_t m = S.front_m[s], w = S.sptr[s + 1] - S.sptr[s];
      return m <= kPackedMid && w * (m + 1) <= (int64_t)kPackedMid * (kPackedMid + 1) / 2;
    };
    const int64_t p0 = (int64_t)P.small_list.size();
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q)
      if (packed(S.level_list[q]) && packed_mid(S.level_list[q])) P.small_list.push_back(S.level_list[q]);
    const int64_t p1 = (int64_t)P.small_list.size();
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q)
      if (packed(S.level_list[q]) && !packed_mid(S.level_list[q])) P.small_list.push_back(S.level_list[q]);
    if ((int64_t)P.small_list.size() > b0) {
      Step st{kStepSmall, h, b0, (int64_t)P.small_list.size()};
      st.tile = nleaf;
      st.packed = p0;
      st.packed_big = p1;
      for (int64_t q = b0; q < st.end; ++q) {
        const int32_t s = P.small_list[q];
        st.flops += front_flops(S, s);
        st.elems += front_io(S, s);
      }
      P.steps.push_back(st);
    }
    if (big.empty()) continue;
    int64_t a0 = (int64_t)P.asm_items.size();
    int32_t wmax = 0;
    for (int32_t s : big) {
      const int32_t m = S.front_m[s], w = S.sptr[s + 1] - S.sptr[s];
      // front row space: the panel's rows [0, ldL), the update matrix's
      // rows [w, w + ldU); a U column c is kept from row w + ((c - w) & ~63)
      const int32_t R = m > w ? std::max(P.ldL[s], w + P.ldU[s]) : P.ldL[s];
      // Blocks of columns of full height when kAsmTile entries hold at
      // least one column (as many columns as fit, at most 64); otherwise
      // asm_cols columns in chunks of rows.
      for (int32_t c = 0; c < m;) {
        const int32_t r0 = c < w ? 0 : w + ((c - w) & ~(kPanel - 1));
        const int32_t height = R - r0;
        int32_t cols, rows;
        if (height <= kAsmTile) {
          cols = std::min(std::min(64, kAsmTile / height), m - c);
          rows = height;
        } else {
          cols = std::min(std::min(asm_cols, 64), m - c);
          rows = kAsmTile / cols;
        }
        const int32_t c1 = c + cols;
        for (int32_t ra = r0; ra < R; ra += rows) {
          const int32_t rb = std::min(R, ra + rows);
          const int32_t rbase = (int32_t)(P.asm_rng.size() / 4);
          for (int32_t q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
            // child rows (front positions in s, ascending) past its pivots
            const int32_t ch = S.child_list[q];
            const int32_t wc = S.sptr[ch + 1] - S.sptr[ch];
            const int32_t* rm = S.rmap.data() + S.rows_ptr[ch] + wc;
            const int32_t rc = S.front_m[ch] - wc;
            P.asm_rng.push_back((int32_t)(std::lower_bound(rm, rm + rc, c) - rm));
            P.asm_rng.push_back((int32_t)(std::lower_bound(rm, rm + rc, c1) - rm));
            P.asm_rng.push_back((int32_t)(std::lower_bound(rm, rm + rc, ra) - rm));
            P.asm_rng.push_back((int32_t)(std::lower_bound(rm, rm + rc, rb) - rm));
          }
          P.asm_items.push_back({s, c, c1, rbase, ra, rb});
        }
        c = c1;
      }
      wmax = std::max(wmax, w);
    }
    {
      Step st{kStepAssemble, h, a0, (int64_t)P.asm_items.size()};
      for (int32_t s : big) st.elems += front_io(S, s);
      P.steps.push_back(st);
    }
    if (front_mode == 0) {
      // Fronts with one pivot block and at most solo_m rows run as one task
      // each (diagonal block, row tiles, update-matrix tiles in order, no
      // flags); the others as tile tasks below.
      std::vector<int32_t> flow_all, solo;
      for (int32_t s : big)
        ((S.sptr[s + 1] - S.sptr[s] <= kPanel && S.front_m[s] <= solo_m) ? solo : flow_all).push_back(s);
      // Fronts with at least chain_min pivot blocks run their diagonal blocks
      // as one chain task (a decision of the front's shape alone, so that its
      // summation order never depends on the other fronts of the level).  A
      // chain holds a workgroup slot while it waits for later tickets, so a
      // level with more than kMaxChains of them is split into several
      // launches of at most kMaxChains chains each.
      auto is_chain = [&](int32_t s) {
        return chain_min > 0 && (S.sptr[s + 1] - S.sptr[s] + kPanel - 1) / kPanel >= chain_min;
      };
      // A front with one pivot block and at most kPanelTaskMax rows factors
      // its whole panel in one task (no flags between its row tiles); its
      // update matrix is left to the update-matrix tasks.
      auto whole_panel = [&](int32_t s) {
        return S.sptr[s + 1] - S.sptr[s] <= kPanel && S.front_m[s] <= kPanelTaskMax;
      };
      std::vector<std::vector<int32_t>> groups(1);
      {
        int nchain = 0;
        for (int32_t s : flow_all) {
          if (is_chain(s) && nchain == kMaxChains) {
            groups.emplace_back();
            nchain = 0;
          }
          nchain += is_chain(s) ? 1 : 0;
          groups.back().push_back(s);
        }
      }
      for (size_t gi = 0; gi < groups.size(); ++gi) {
      const std::vector<int32_t>& flow = groups[gi];
      const bool last_group = gi + 1 == groups.size();
      int32_t gwmax = 0;
      for (int32_t s : flow) gwmax = std::max(gwmax, S.sptr[s + 1] - S.sptr[s]);
      // Dataflow: pivot blocks in column order across the group's fronts;
      // the update-matrix tiles of a front in ranges of u_range pivot
      // blocks, each range right after the last column it needs.  Every task
      // depends only on tasks with smaller tickets.
      Step st{kStepFront, h, (int64_t)P.ftasks.size(), 0};
      st.ticket = P.front_launches++;
      // Update matrices of more than 64 rows go in kUBlock x kUBlock blocks
      // (twice the products per operand byte of a 64 x 64 tile; a decision
      // of the front's shape alone).
      auto ublock = [&](int32_t s) {
        return S.front_m[s] - (S.sptr[s + 1] - S.sptr[s]) > kPanel ? kUBlock : kPanel;
      };
      std::vector<int32_t> ubase(flow.size());
      for (size_t bi = 0; bi < flow.size(); ++bi) {
        const int32_t s = flow[bi];
        const int32_t r = S.front_m[s] - (S.sptr[s + 1] - S.sptr[s]);
        const int32_t ub = ublock(s);
        const int32_t nt = (r + ub - 1) / ub;
        ubase[bi] = (int32_t)P.nucount;
        P.nucount += (int64_t)nt * (nt + 1) / 2;
      }
      // Range k of a front (pivot blocks [8k, 8k+8)) is emitted in u_range
      // chunks after the columns 8k+8 ... 8k+15, so that its tasks take
      // workgroup slots when their inputs are complete and interleave with
      // the pivot-block tasks that carry the critical path; what is left
      // when the level's columns end is emitted then.
      std::vector<std::vector<FrontTask>> pending(flow.size());
      std::vector<size_t> pending_pos(flow.size(), 0);
      auto emit_u = [&](size_t bi, size_t upto) {
        upto = std::min(upto, pending[bi].size());
        for (; pending_pos[bi] < upto; ++pending_pos[bi]) P.ftasks.push_back(pending[bi][pending_pos[bi]]);
      };
      const int32_t ncols = (gwmax + kPanel - 1) / kPanel;
      // chain tasks first in ticket order; block j >= 2 of a chain is
      // pre-accumulated by a task issued right after column j - 2
      std::vector<char> chain(flow.size(), 0);
      for (size_t bi = 0; bi < flow.size(); ++bi) {
        const int32_t s = flow[bi];
        if (is_chain(s)) {
          chain[bi] = 1;
          P.ftasks.push_back({s, 0, 0, 2, inplace ? 1 : 0, kPdRange, 0, 0});
          const int32_t nbs = (S.sptr[s + 1] - S.sptr[s] + kPanel - 1) / kPanel;
          for (int32_t b = 1; b < nbs; ++b) P.pt1base[P.wbase[s] + b] = (int32_t)P.pt1_slots++;
        }
      }
      for (int32_t j = 0; j < ncols; ++j) {
        for (size_t bi = 0; bi < flow.size(); ++bi) {
          const int32_t s = flow[bi];
          const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
          if (j * kPanel >= w) continue;
          if (whole_panel(s)) {
            P.ftasks.push_back({s, 0, 0, 6, 0, 0, 0, 0});
            continue;
          }
          // the diagonal task (t = 0) also produces row tile 1
          const int nt = front_block_tiles(m, w, j);
          for (int t = chain[bi] ? 2 : 0; t < nt; ++t)
            if (t != 1) P.ftasks.push_back({s, j, t, 0, chain[bi] ? (inplace ? 2 : 1) : 0, 0, 0, 0});
          if (chain[bi]) {
            // pre-accumulation ranges that end with pivot block j: for block
            // b >= 2, [b - 2, b - 1) and before it [e - kPdRange, e) for e =
            // b - 2, b - 2 - kPdRange, ... (the first one cut at 0), applied
            // in order of their start (rk)
            const int32_t nbs = (w + kPanel - 1) / kPanel;
            for (int32_t b = j + 2; b < nbs; ++b) {
              const int32_t e = b - 2, before = (e + kPdRange - 1) / kPdRange;
              int32_t p0, p1, rk;
              if (b == j + 2) {
                p0 = j;
                p1 = j + 1;
                rk = before;
              } else {
                const int32_t d = e - (j + 1);  // distance of this end below b - 2
                if (d % kPdRange != 0) continue;
                p1 = j + 1;
                p0 = std::max(0, p1 - kPdRange);
                rk = before - 1 - d / kPdRange;
              }
              P.ftasks.push_back({s, b, 0, 3, p0, p1, 0, rk});
            }
          }
        }
        for (size_t bi = 0; bi < flow.size(); ++bi) {
          const int32_t s = flow[bi];
          const int32_t w = S.sptr[s + 1] - S.sptr[s], r = S.front_m[s] - w;
          const int32_t pb = (w + kPanel - 1) / kPanel;
          if (r <= 0 || kUSplit) continue;
          const int32_t ub = ublock(s);
          if (j < pb && ((j + 1) % urange == 0 || j + 1 == pb)) {
            // range ending at column j: queue its tasks
            const int32_t rk = j / urange, p0 = rk * urange, p1 = j + 1;
            const int32_t nt = (r + ub - 1) / ub;
            for (int32_t b = 0; b < nt; ++b)
              for (int32_t a = b; a < nt; ++a) {
                const int32_t ui = ubase[bi] + a * (a + 1) / 2 + b;
                pending[bi].push_back({s, b, a, ub == kUBlock ? 5 : 1, p0, p1, ui, rk});
              }
          }
          // release the queued tasks of the range that ended u_range columns
          // ago in proportion to the columns passed since
          const int32_t per = (int32_t)((r + ub - 1) / ub);
          const size_t range_tasks = (size_t)per * (per + 1) / 2;
          if (j >= urange) {
            const int32_t rk = (j - urange) / urange;       // range being released
            const int32_t q = (j - urange) % urange + 1;    // chunks released so far
            const size_t base = (size_t)rk * range_tasks;
            if (rk * urange < pb) emit_u(bi, base + range_tasks * q / urange);
          }
        }
      }
      for (size_t bi = 0; bi < flow.size(); ++bi) emit_u(bi, pending[bi].size());
      if (last_group)
        for (int32_t s : solo) P.ftasks.push_back({s, 0, 0, 4, 0, 1, 0, 0});
      st.end = (int64_t)P.ftasks.size();
      std::vector<int32_t> members(flow);
      if (last_group) members.insert(members.end(), solo.begin(), solo.end());
      for (int32_t s : members) {
        const double m = S.front_m[s], w = S.sptr[s + 1] - S.sptr[s], r = m - w;
        const bool split = kUSplit && std::find(flow.begin(), flow.end(), s) != flow.end();
        st.flops += front_flops(S, s) - (split ? w * r * r : 0.0);
        // front read once (panel trapezoid + update triangle), written once
        st.elems += 2.0 * ((w * m - w * (w - 1) / 2) + (split ? 0.0 : r * (r + 1) / 2));
      }
      if (st.end > st.begin) P.steps.push_back(st);
      if (kUSplit) {
        // the update matrices of the group's flow fronts, in a launch of
        // their own once every panel is done: kUBlock x kUBlock blocks over
        // all pivot columns, no flags; blocks sharing rows get neighbouring
        // tickets
        Step us{kStepFront, h, (int64_t)P.ftasks.size(), 0};
        us.ticket = P.front_launches++;
        for (int32_t s : flow) {
          const int32_t w = S.sptr[s + 1] - S.sptr[s], r = S.front_m[s] - w;
          if (r <= 0) continue;
          const int32_t nt = (r + kUBlock - 1) / kUBlock, pb = (w + kPanel - 1) / kPanel;
          for (int32_t a = 0; a < nt; ++a)
            for (int32_t b = 0; b <= a; ++b) P.ftasks.push_back({s, b, a, 7, 0, pb, 0, 0});
          us.flops += (double)w * r * r;
          us.elems += (double)r * w + (double)r * (r + 1);
        }
        us.end = (int64_t)P.ftasks.size();
        if (us.end > us.begin) P.steps.push_back(us);
      }
      }
      continue;
    }
    for (int32_t k = 0; k < wmax; k += kPanel) {
      int64_t d0 = (int64_t)P.diag_items.size();
      for (int32_t s : big) {
        const int32_t w = S.sptr[s + 1] - S.sptr[s];
        if (w <= k) continue;
        P.diag_items.push_back({s, k, std::min(kPanel, w - k), 0, P.wbase[s] + k / kPanel, 0});
      }
      {
        Step st{kStepDiag, h, d0, (int64_t)P.diag_items.size()};
        for (int64_t q = d0; q < st.end; ++q) {
          const double kb = P.diag_items[q].kb;
          st.flops += kb * (kb + 1) * (2 * kb + 1) / 6.0;
          st.elems += kb * (kb + 1) + kb * kb;
        }
        P.steps.push_back(st);
      }
      int64_t p0 = (int64_t)P.panel_items.size();
      for (size_t bi = 0; bi < big.size(); ++bi) {
        const int32_t s = big[bi];
        const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
        if (w <= k) continue;
        const int32_t kb = std::min(kPanel, w - k);
        const int32_t below = m - k - kb;
        const int32_t chunks = (below + kPanelRows - 1) / kPanelRows;
        for (int32_t c = 0; c < chunks; ++c)
          P.panel_items.push_back({s, k, kb, c, P.wbase[s] + k / kPanel, 0});
      }
      if ((int64_t)P.panel_items.size() > p0) {
        Step st{kStepPanel, h, p0, (int64_t)P.panel_items.size()};
        for (int32_t s : big) {
          const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
          if (w <= k) continue;
          const double kb = std::min(kPanel, w - k), rows = m - k - kb;
          st.flops += rows * kb * kb;
          st.elems += 2 * rows * kb + kb * kb;
        }
        P.steps.push_back(st);
      }
      // Two-level blocking: a kPanel step updates only the columns of its
      // kOuter-wide outer panel (all rows below); once an outer panel is
      // done, one update with K = kOuter covers the rest of the front's
      // pivot columns.
      const int32_t k_outer = (k / kOuter) * kOuter;
      const bool outer_end = k + kPanel >= k_outer + kOuter;
      for (int32_t s : big) {
        const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
        const int32_t panel_end = std::min(w, k_outer + kOuter);
        if (panel_end <= k + kPanel) continue;
        const int32_t kb = kPanel;
        GemmProb g;
        g.a_off = P.L_off[s] + (int64_t)k * P.ldL[s] + (k + kb);
        g.c_off = P.L_off[s] + (int64_t)(k + kb) * P.ldL[s] + (k + kb);
        g.lda = g.ldc = P.ldL[s];
        g.M = m - k - kb;
        g.N = panel_end - k - kb;
        g.K = kb;
        g.c_in_u = 0;
        add_gemm(g);
      }
      add_gemm_step(h);
      if (outer_end) {
        const int32_t k1 = k_outer + kOuter;
        for (int32_t s : big) {
          const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
          if (w <= k1) continue;
          GemmProb g;
          g.a_off = P.L_off[s] + (int64_t)k_outer * P.ldL[s] + k1;
          g.c_off = P.L_off[s] + (int64_t)k1 * P.ldL[s] + k1;
          g.lda = g.ldc = P.ldL[s];
          g.M = m - k1;
          g.N = w - k1;
          g.K = kOuter;
          g.c_in_u = 0;
          add_gemm(g);
        }
        add_gemm_step(h);
      }
    }
    for (int32_t s : big) {
      const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s], r = m - w;
      if (r <= 0) continue;
      GemmProb g;
      g.a_off = P.L_off[s] + w;
      g.c_off = P.U_off[s];
      g.lda = P.ldL[s];
      g.ldc = P.ldU[s];
      g.M = g.N = r;
      g.K = w;
      g.c_in_u = 1;
      add_gemm(g);
    }
    add_gemm_step(h);
  }
  // Solves: backward partial-product slots of every large front, the
  // level-by-level phase, then the dataflow phase.
  P.fsolve.clear();
  P.bsolve.clear();
  P.wave_list.clear();
  P.lwave.clear();
  P.llarge.clear();
  P.part_base.assign(P.woff.size(), 0);
  P.part_slots = 0;
  for (int32_t s = 0; s < ns; ++s) {
    if (S.front_m[s] <= kSmallMax) continue;
    const int32_t w = S.sptr[s + 1] - S.sptr[s], r = S.front_m[s] - w;
    const int32_t nch = (r + kBwdChunk - 1) / kBwdChunk;
    for (int32_t b = 0; b * kPanel < w; ++b) {
      if (P.part_slots + nch > INT32_MAX) {
        err = "too many partial products for the solve plan";
        return kInvalid;
      }
      P.part_base[P.wbase[s] + b] = (int32_t)P.part_slots;
      P.part_slots += nch;
    }
  }
  {
    int32_t H = 0;
    for (int32_t h = S.nlevels - 1; h >= 0; --h)
      if (S.level_ptr[h + 1] - S.level_ptr[h] > level_fronts) {
        H = h + 1;
        break;
      }
    P.solve_split = H;
    P.lwave_ptr.assign(H + 1, 0);
    P.llarge_ptr.assign(H + 1, 0);
    for (int32_t h = 0; h < H; ++h) {
      for (int g = 8; g <= 64; g *= 2) {
        std::vector<int32_t> sel;
        for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
          const int32_t s = S.level_list[q], m = S.front_m[s];
          if (m <= g && (g == 8 || m > g / 2)) sel.push_back(s);
        }
        const int per = 64 / g;
        for (size_t i = 0; i < sel.size(); i += per) {
          WaveItem it{};
          it.first = (int32_t)P.wave_list.size();
          it.count = (int32_t)std::min<size_t>(per, sel.size() - i);
          it.g = (int16_t)g;
          for (int32_t k = 0; k < it.count; ++k) {
            const int32_t s = sel[i + k], w = S.sptr[s + 1] - S.sptr[s];
            it.wmax = (int16_t)std::max<int32_t>(it.wmax, w);
            it.rmax = (int16_t)std::max<int32_t>(it.rmax, S.front_m[s] - w);
            P.wave_list.push_back(s);
          }
          P.lwave.push_back(it);
        }
      }
      for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q)
        if (S.front_m[S.level_list[q]] > kSmallMax) P.llarge.push_back(S.level_list[q]);
      P.lwave_ptr[h + 1] = (int64_t)P.lwave.size();
      P.llarge_ptr[h + 1] = (int64_t)P.llarge.size();
    }
    // Dataflow phase.  Forward, per level from the split: the diagonal
    // blocks of the large fronts, then the wave groups, then the L21 row
    // blocks.  Backward, per level from the root: the L21 partial products,
    // the diagonal blocks from the last, then the wave groups.  A task waits
    // only on its front's children (forward) or parent (backward) and on
    // earlier blocks of its own front, all of which have smaller tickets or
    // belong to the level-by-level phase.
    std::vector<std::vector<std::pair<int64_t, int32_t>>> level_groups(S.nlevels);
    for (int32_t h = H; h < S.nlevels; ++h) {
      int64_t first = (int64_t)P.wave_list.size();
      for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
        const int32_t s = S.level_list[q];
        if (S.front_m[s] <= kSmallMax) P.wave_list.push_back(s);
      }
      const int64_t last = (int64_t)P.wave_list.size();
      for (int64_t g = first; g < last; g += kWaveFronts)
        level_groups[h].push_back({g, (int32_t)std::min<int64_t>(kWaveFronts, last - g)});
    }
    if ((int64_t)P.wave_list.size() > INT32_MAX) {
      err = "too many fronts for the solve plan";
      return kInvalid;
    }
    for (int32_t h = H; h < S.nlevels; ++h) {
      for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
        const int32_t s = S.level_list[q];
        if (S.front_m[s] <= kSmallMax) continue;
        const int32_t w = S.sptr[s + 1] - S.sptr[s];
        for (int32_t b = 0; b * kPanel < w; ++b) P.fsolve.push_back({s, kSolveTri, b, 0});
      }
      for (const auto& g : level_groups[h]) P.fsolve.push_back({-1, kSolveWave, (int32_t)g.first, g.second});
      for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
        const int32_t s = S.level_list[q];
        if (S.front_m[s] <= kSmallMax) continue;
        const int32_t r = S.front_m[s] - (S.sptr[s + 1] - S.sptr[s]);
        for (int32_t k = 0; k * kPanel < r; ++k) P.fsolve.push_back({s, kSolveRows, k, 0});
      }
    }
    for (int32_t h = S.nlevels - 1; h >= H; --h) {
      for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
        const int32_t s = S.level_list[q];
        if (S.front_m[s] <= kSmallMax) continue;
        const int32_t w = S.sptr[s + 1] - S.sptr[s], r = S.front_m[s] - w;
        const int32_t nb = (w + kPanel - 1) / kPanel, nch = (r + kBwdChunk - 1) / kBwdChunk;
        for (int32_t b = nb - 1; b >= 0; --b)
          for (int32_t c = 0; c < nch; ++c) P.bsolve.push_back({s, kSolveRows, b, c});
      }
      for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
        const int32_t s = S.level_list[q];
        if (S.front_m[s] <= kSmallMax) continue;
        const int32_t w = S.sptr[s + 1] - S.sptr[s];
        for (int32_t b = (w + kPanel - 1) / kPanel - 1; b >= 0; --b) P.bsolve.push_back({s, kSolveTri, b, 0});
      }
      for (const auto& g : level_groups[h]) P.bsolve.push_back({-1, kSolveWave, (int32_t)g.first, g.second});
    }
    if ((int64_t)P.fsolve.size() > INT32_MAX || (int64_t)P.bsolve.size() > INT32_MAX) {
      err = "too many solve tasks";
      return kInvalid;
    }
  }
  // forward extend-add sources, children in ascending order
  {
    const int64_t nrow = S.rows_ptr[ns];
    std::vector<int64_t> cnt(nrow + 1, 0);
    for (int32_t c = 0; c < ns; ++c) {
      const int32_t p = S.sparent[c];
      if (p < 0) continue;
      const int32_t wc = S.sptr[c + 1] - S.sptr[c];
      for (int64_t k = S.rows_ptr[c] + wc; k < S.rows_ptr[c + 1]; ++k) ++cnt[S.rows_ptr[p] + S.rmap[k] + 1];
    }
    for (int64_t q = 0; q < nrow; ++q) cnt[q + 1] += cnt[q];
    if (cnt[nrow] > INT32_MAX || P.u_elems > INT32_MAX) {
      err = "update vectors too large for the solve plan";
      return kInvalid;
    }
    P.pull_ptr.assign(cnt.begin(), cnt.end());
    P.pull_src.assign(cnt[nrow], 0);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t p = 0; p < ns; ++p)
      for (int32_t q = S.child_ptr[p]; q < S.child_ptr[p + 1]; ++q) {
        const int32_t c = S.child_list[q];
        const int32_t wc = S.sptr[c + 1] - S.sptr[c];
        for (int64_t k = S.rows_ptr[c] + wc; k < S.rows_ptr[c + 1]; ++k)
          P.pull_src[fill[S.rows_ptr[p] + S.rmap[k]]++] = (int32_t)(P.u_off[c] + (k - S.rows_ptr[c] - wc));
      }
  }
  P.level_lentries.assign(S.nlevels, 0.0);
  P.level_rows.assign(S.nlevels, 0.0);
  for (int32_t s = 0; s < ns; ++s) {
    const double m = S.front_m[s], w = S.sptr[s + 1] - S.sptr[s];
    P.level_lentries[S.height[s]] += w * m - w * (w - 1) / 2;
    P.level_rows[S.height[s]] += m;
  }
  return kOk;
}

void build_pinv_plan(const Symbolic& S, PinvPlan& Q) {
  const int32_t ns = S.ns;
  Q.setup.clear();
  Q.setup_ptr.assign(1, 0);
  Q.flops = 0;
  int32_t nbmax = 0;
  for (int32_t s = 0; s < ns; ++s) nbmax = std::max(nbmax, (S.sptr[s + 1] - S.sptr[s] + kPanel - 1) / kPanel);
  for (int32_t q = 0; q < nbmax; ++q) {
    for (int32_t s = 0; s < ns; ++s) {
      const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
      const int32_t nb = (w + kPanel - 1) / kPanel, nt = (m + kPanel - 1) / kPanel;
      if (q >= nb) continue;
      if (q == 0) {
        for (int32_t a = nb - 1; a < nt; ++a) Q.setup.push_back({s, a, nb - 1, -1});
        continue;
      }
      const int32_t j = nb - q;  // finished by the previous launch
      for (int32_t i = 0; i < j; ++i) {
        if (i == j - 1) Q.setup.push_back({s, j - 1, i, -1});  // nothing from block j
        for (int32_t a = j; a < nt; ++a) {
          Q.setup.push_back({s, a, i, j});
          Q.flops += 2.0 * kPanel * kPanel * std::min<int32_t>(kPanel, w - j * kPanel);
        }
      }
    }
    Q.setup_ptr.push_back((int64_t)Q.setup.size());
  }
  Q.tiles.clear();
  for (int32_t s = 0; s < ns; ++s)
    for (int32_t c = 0; c * kPanel < S.sptr[s + 1] - S.sptr[s]; ++c) Q.tiles.push_back({s, c});
  Q.frow.clear();
  Q.bcol.clear();
  Q.frow_ptr.assign(1, 0);
  Q.bcol_ptr.assign(1, 0);
  Q.small.clear();
  Q.large.clear();
  Q.small_ptr.assign(1, 0);
  Q.large_ptr.assign(1, 0);
  Q.slots = 0;
  Q.gchunks.clear();
  Q.fsum.clear();
  Q.bsum.clear();
  Q.fsum_ptr.assign(1, 0);
  Q.bsum_ptr.assign(1, 0);
  auto add = [&](std::vector<PinvSweepTask>& v, std::vector<PinvSweepTask>& sum, int32_t s, int32_t t,
                 int32_t len) {
    const int32_t nch = (len + kPinvChunk - 1) / kPinvChunk;
    const int32_t slot = nch > 1 ? (int32_t)Q.slots : -1;
    if (nch > 1) {
      Q.slots += nch;
      sum.push_back({s, t, nch, slot});
    }
    for (int32_t c = 0; c < nch; ++c) v.push_back({s, t, c, slot});
  };
  for (int32_t h = 0; h < S.nlevels; ++h) {
    int32_t gch = 1;
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
      const int32_t s = S.level_list[q];
      const int32_t w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s];
      if (m <= kPinvSmallM && w <= kSmallMax) {
        Q.small.push_back(s);
        continue;
      }
      Q.large.push_back(s);
      gch = std::max(gch, std::min(kPinvGatherMax, (m + kPinvGatherRows - 1) / kPinvGatherRows));
      // forward: rows of Z11 see only the columns up to their own
      for (int32_t a = 0; a * kPanel < m; ++a) add(Q.frow, Q.fsum, s, a, std::min(w, (a + 1) * kPanel));
      // backward: Z is zero above a column's diagonal
      for (int32_t c = 0; c * kPanel < w; ++c) add(Q.bcol, Q.bsum, s, c, m - c * kPanel);
    }
    Q.frow_ptr.push_back((int64_t)Q.frow.size());
    Q.bcol_ptr.push_back((int64_t)Q.bcol.size());
    Q.small_ptr.push_back((int64_t)Q.small.size());
    Q.large_ptr.push_back((int64_t)Q.large.size());
    Q.gchunks.push_back(gch);
    Q.fsum_ptr.push_back((int64_t)Q.fsum.size());
    Q.bsum_ptr.push_back((int64_t)Q.bsum.size());
  }
}

void build_level_csr(const Symbolic& S, LevelCsr& C) {
  C.rows.clear();
  C.rptr.assign(1, 0);
  C.segs.clear();
  C.fwd_ptr.clear();
  C.b_ptr.clear();
  int64_t pos = 0;
  auto add_row = [&](int32_t row) {
    C.rows.push_back(row);
    C.rptr.push_back(pos);
  };
  std::vector<std::array<int32_t, 3>> anc;  // (ancestor row, front, local row)
  // forward matrices of every level (ancestor rows, then pivot rows)
  for (int32_t h = 0; h < S.nlevels; ++h) {
    C.fwd_ptr.push_back((int64_t)C.rows.size());
    anc.clear();
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
      const int32_t s = S.level_list[q];
      const int32_t w = S.sptr[s + 1] - S.sptr[s];
      for (int32_t k = w; k < S.front_m[s]; ++k) anc.push_back({S.rows[S.rows_ptr[s] + k], s, k});
    }
    std::sort(anc.begin(), anc.end());  // by row, then front
    for (size_t a = 0; a < anc.size();) {
      const int32_t row = anc[a][0];
      for (; a < anc.size() && anc[a][0] == row; ++a) {
        const int32_t s = anc[a][1];
        C.segs.push_back({pos, s, anc[a][2], 1, 0});
        pos += S.sptr[s + 1] - S.sptr[s];
      }
      add_row(row);
    }
    C.fwd_ptr.push_back((int64_t)C.rows.size());
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
      const int32_t s = S.level_list[q];
      for (int32_t c = 0; c < S.sptr[s + 1] - S.sptr[s]; ++c) {
        C.segs.push_back({pos, s, c, 0, 0});
        pos += c + 1;
        add_row(S.sptr[s] + c);
      }
    }
  }
  C.fwd_ptr.push_back((int64_t)C.rows.size());
  // backward matrices
  for (int32_t h = 0; h < S.nlevels; ++h) {
    C.b_ptr.push_back((int64_t)C.rows.size());
    for (int32_t q = S.level_ptr[h]; q < S.level_ptr[h + 1]; ++q) {
      const int32_t s = S.level_list[q];
      for (int32_t c = 0; c < S.sptr[s + 1] - S.sptr[s]; ++c) {
        C.segs.push_back({pos, s, c, 2, 0});
        pos += S.front_m[s] - c;
        add_row(S.sptr[s] + c);
      }
    }
  }
  C.b_ptr.push_back((int64_t)C.rows.size());
  C.nnz = pos;
}

}  // namespace tacho
