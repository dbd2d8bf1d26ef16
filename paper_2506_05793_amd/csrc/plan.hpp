// Device memory layout and per-level launch plan of the numeric phase.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "symbolic.hpp"

namespace tacho {

// Work item of the large-front assembly: the entries of front s in columns
// [c0, c1) and front rows [r0, r1) (at most kAsmTile of them, summed in LDS
// and written once); for the q-th child of s, the child's update-matrix
// columns that land in [c0, c1) are [asm_rng[4 (rbase + q)],
// asm_rng[4 (rbase + q) + 1]) and its rows that land in [r0, r1) are
// [asm_rng[4 (rbase + q) + 2], asm_rng[4 (rbase + q) + 3]).
struct AsmItem {
  int32_t s, c0, c1, rbase, r0, r1;
};

// Work item of the panel kernels: diagonal block [k, k+kb) of front s (one
// item per front for the diagonal Cholesky), rows below it handled in chunks
// of kPanelRows (one item per chunk for the triangular solve).  `wblk` is the
// global index of the diagonal block, whose inverse is kept for the solves.
struct PanelItem {
  int32_t s, k, kb, chunk, wblk, pad;
};

// Update C[M x N] -= A[M x K] * A[0:N, :]^T, lower part (row >= col) only.
// A lives in the factor panels; C in the panels (c_in_u = 0) or in the
// update matrices (c_in_u = 1).  Offsets are in elements.
struct GemmProb {
  int64_t a_off, c_off;
  int32_t lda, ldc, M, N, K, c_in_u;
};

// Task of the dataflow solves (one workgroup each, taken in ticket order).
// Fronts with m <= kSmallMax are solved by one wave each; a kSolveWave task
// holds up to kWaveFronts of them: wave_list[a, a + b).  A larger front is
// split into 64-row blocks: kSolveTri, block a of the diagonal part (forward:
// rows [64a, 64a + kb) of L11, backward: columns of it); forward kSolveRows,
// block a of L21 (rows w + 64a ...); backward kSolveRows, the partial product
// of L21 rows [kBwdChunk b, ...) with column block a.
struct SolveTask {
  int32_t s, kind, a, b;
};
enum SolveKind : int32_t { kSolveWave = 0, kSolveTri = 1, kSolveRows = 2 };
constexpr int kWaveFronts = 4;   // one per wave of a 256-thread workgroup
constexpr int kBwdChunk = 256;   // L21 rows per backward partial product

// Solve levels below the last level with more than kLevelFronts fronts run
// level by level (one launch each, no flags); the levels above run as one
// dataflow launch.  In the level-by-level phase the fronts with m <=
// kSmallMax share waves: a WaveItem is wave_list[first, first + count), each
// front in its own group of g lanes (g = 8, 16, 32 or 64, at least its m),
// with wmax / rmax the largest w / r among them.
struct WaveItem {
  int32_t first, count;
  int16_t g, wmax, rmax, pad;
};
constexpr int kLevelFronts = 256;  // default of PlanTuning::level_fronts

#if defined(__HIP__)
#define TACHO_HOST_DEVICE __host__ __device__
#else
#define TACHO_HOST_DEVICE
#endif

struct GemmTile {
  int32_t prob, ti, tj, size;  // size: kGemmTile or kGemmTileBig
};

// Task of the dataflow large-front kernel (one workgroup each, taken in
// ticket order).  kind 0: pivot block j of front s (columns [64j, 64j+kb)),
// row tile t: t = 0 is the diagonal block (kb rows) together with row tile
// 1, t >= 2 the 64 rows starting at 64j + kb + 64(t-1).  kind 1: tile (t, j)
// of the update matrix U_s (rows 64t.., columns 64j..), t >= j, for the
// pivot blocks [p0, p1): the rk-th such range of the tile, applied after
// range rk-1 (counter ui of the tile orders them).  kind 2: the chain of
// diagonal blocks of front s (all its t = 0 work, in order; p1 holds the
// pre-accumulation range length).  kind 3: pre-accumulation of diagonal
// block j and row tile 1 of front s over the pivot blocks [p0, p1), the
// rk-th such range of block j (ranges cover the blocks before j - 1, the
// last one is [j - 2, j - 1) and they are applied in order), for the chain.
// kind 4: the whole front s (one pivot block): the diagonal block, its row
// tiles and the update-matrix tiles, in order, by one workgroup.  kind 5:
// as kind 1 for a block of kUBlock x kUBlock entries (rows kUBlock t..,
// columns kUBlock j..), used for every update matrix of more than 64 rows.
// kind 6: the whole panel of front s (one pivot block, at most
// kPanelTaskMax rows): the diagonal block and all row tiles, in order, by one
// workgroup, which then raises the flags of all its row tiles.
// kind 7: update-matrix block (t, j) of front s (as kind 5) over all its
// pivot blocks [0, p1), in a launch after the one that factors the panels
// (nothing awaited or published).
// A kind 0 task of a chain front
// has p0 = 1 or 2: its rows that are row tile 1 of block j + 1 also get
// their product with row tile 1 of block j, for the chain's step j + 1,
// stored in a slot (1) or subtracted in place (2, and the chain task has
// p0 = 1).
struct FrontTask {
  int32_t s, j, t, kind;
  int32_t p0, p1, ui, rk;
};

constexpr int kURange = 8;     // default pivot blocks per update-matrix task
constexpr int kUBlock = 128;   // rows and columns of an update-matrix block task (kind 5)
constexpr int kPanelTaskMax = 1024;  // rows of the largest front whose panel is one task (kind 6)
constexpr bool kUSplit = true;  // update matrices of the flow fronts in a launch after their panels'
constexpr int kChainMin = 3;   // default pivot blocks from which a front's diagonal blocks form a chain
constexpr int kPdRange = 4;    // pivot blocks per pre-accumulation range of a chain's diagonal block
constexpr int kAsmTile = 4096;   // front entries per assembly work item (its LDS tile)
constexpr int kSoloM = 192;    // default: fronts with one pivot block and m <= this run as one task
// Chains per front launch: each holds a workgroup slot while it waits for
// later tickets.  The FP64 front kernel keeps two workgroups per CU resident
// (512 on 256 CUs), so four concurrent factorizations (the serving slots)
// still leave slots for the tasks the chains wait on.
constexpr int kMaxChains = 96;

// Batching parameters of the plan (task grouping only; the arithmetic of a
// front does not depend on them).
struct PlanTuning {
  int32_t u_range = 8;        // pivot blocks per update-matrix range
  int32_t chain_min = 3;      // chain fronts: at least this many pivot blocks (<= 0: none)
  int32_t level_fronts = 256; // solve level-by-level phase threshold
  int32_t asm_cols = 8;       // front columns per assembly workgroup
  int32_t solo_m = 0;         // one-task fronts: one pivot block, at most this many rows (0: default, < 0: none)
  int32_t chain_inplace = 0;  // chain fronts: next-block product subtracted in place (>= 0) or via a slot (< 0)
};

enum StepKind : int32_t {
  kStepSmall = 0,
  kStepAssemble = 1,
  kStepDiag = 2,
  kStepPanel = 3,
  kStepGemm = 4,
  kStepFront = 5,
};

// One kernel launch: [begin, end) into the matching item array; for
// kStepGemm, [begin, end) indexes tiles (all of size `tile`) and the problems
// are those tiles' own.
struct Step {
  int32_t kind;
  int32_t level;
  int64_t begin, end;
  double flops = 0;  // algorithmic flops of the launch
  double elems = 0;  // algorithmic element traffic (reads + writes) of the launch
  int32_t tile = 0;  // update steps: tile size; small-front steps: leading one-thread leaves
  int32_t ticket = 0;  // dataflow front steps: index of the launch's ticket counter
  int64_t packed = 0;      // small-front steps: [packed, packed_big) go to the packed-LDS
  int64_t packed_big = 0;  // kernel for m <= kPackedMid, [packed_big, end) to the larger one
};

constexpr int kSmallMax = 64;     // fronts with m <= kSmallMax go to the LDS kernel
constexpr int kLeafMax = 16;      // ... leaves with one pivot column and m <= kLeafMax to one thread each
constexpr int kPackedMax = 128;   // Cholesky fronts with m <= kPackedMax and w <= kSmallMax: packed LDS kernel
constexpr int kPackedMid = 96;    // ... its smaller-LDS instance: m <= kPackedMid, w (m + 1) <= 96 * 97 / 2
// every front of the class (w <= kSmallMax) fits with its diagonal-block inverse
static_assert(kPackedMax * (kPackedMax + 1) / 2 >= kSmallMax * (kPackedMax + 1),
              "packed front and inverse exceed the LDS array");
constexpr int kPanel = 64;        // panel width of the blocked large-front path
constexpr int kOuter = 256;       // outer panel width (trailing updates with K = kOuter)
constexpr int kPanelRows = 64;    // rows per triangular-solve workgroup
constexpr int kAsmCols = 8;       // front columns per assembly work item of a tall front
constexpr int kGemmTile = 64;     // output tile of the update kernel
constexpr int kGemmTileBig = 128; // output tile for large updates
constexpr int64_t kGemmBigMin = 256 * 256;  // M*N from which the large tile is used
constexpr int kLdAlign = 16;      // leading dimensions rounded to this many elements (128-byte FP64 columns)

struct Plan {
  // memory layout (elements; identical for FP32 and FP64)
  std::vector<int64_t> L_off, U_off, u_off;
  std::vector<int32_t> ldL, ldU;
  int64_t L_elems = 0, U_elems = 0, u_elems = 0;  // u_elems per right-hand side
  // inverses of the kPanel diagonal blocks of large fronts (kb x kb each,
  // column-major): per supernode its first block (-1: none), per block the
  // element offset
  std::vector<int32_t> wbase;
  std::vector<int64_t> woff;
  int64_t W_elems = 0;
  // dataflow factorization: per pivot block the index of its first row tile's
  // completion flag (prefix sums of front_block_tiles; one entry past the end)
  std::vector<int32_t> tbase;
  int64_t nucount = 0;  // update-matrix task counters (one per tile or block of every large front)
  // chain fronts: per pivot block j >= 1 (woff indexing) a 64 x 64 slot for the
  // product of block j - 1's rows of row tile 1 of block j with row tile 1 of
  // block j - 1 (-1: none)
  std::vector<int32_t> pt1base;
  int64_t pt1_slots = 0;
  std::vector<int32_t> a_pos;   // per A entry: row + col*ldL inside the front panel
  std::vector<int32_t> diag_q;  // per permuted column: A entry of the diagonal (-1: absent)

  // launch sequence
  std::vector<int32_t> small_list;  // supernodes factored in LDS, grouped by level
  std::vector<AsmItem> asm_items;
  std::vector<PanelItem> diag_items;
  std::vector<PanelItem> panel_items;
  std::vector<GemmProb> probs;
  std::vector<GemmTile> tiles;
  std::vector<FrontTask> ftasks;  // dataflow large-front tasks, per launch in ticket order
  int32_t front_launches = 0;     // dataflow front launches (one ticket counter each)
  std::vector<Step> steps;
  int front_mode = 0;             // 0: dataflow large-front kernel, 1: stepwise launches

  // solve, per level: factor entries read (sum over fronts of the lower
  // trapezoid of the panel) and front rows touched
  std::vector<double> level_lentries, level_rows;
  // dataflow solves: tasks of the forward and backward sweeps in ticket
  // order, the fronts solved by one wave, and the forward extend-add
  // sources: for row i of front s, entries [pull_ptr[q], pull_ptr[q + 1]) of
  // pull_src with q = rows_ptr[s] + i, each the index of an update-vector
  // entry of a child (children in ascending order)
  std::vector<SolveTask> fsolve, bsolve;
  std::vector<int32_t> wave_list;
  // level-by-level phase of the solves: levels [0, solve_split); per level
  // h its wave items [lwave_ptr[h], lwave_ptr[h + 1]) and its fronts with m >
  // kSmallMax [llarge_ptr[h], llarge_ptr[h + 1]) (one workgroup each)
  int32_t solve_split = 0;
  std::vector<WaveItem> lwave;
  std::vector<int64_t> lwave_ptr;
  std::vector<int32_t> llarge;
  std::vector<int64_t> llarge_ptr;
  std::vector<int32_t> pull_ptr, pull_src;
  // assembly: per item and child, the child's column and row ranges (see AsmItem)
  std::vector<int32_t> asm_rng;
  // backward partial products: per diagonal block (woff indexing) the first
  // of its ceil(r / kBwdChunk) slots of kPanel x 16 elements
  std::vector<int32_t> part_base;
  int64_t part_slots = 0;
};

// Rows of pivot block j of a front of order m and width w: the diagonal
// block plus 64-row tiles below it.
TACHO_HOST_DEVICE inline int front_block_tiles(int m, int w, int j) {
  const int c0 = j * 64, kb = (w - c0 < 64) ? (w - c0) : 64;
  return 1 + (m - c0 - kb + 63) / 64;
}

// Row tile of pivot block j that holds front row r (r >= 64 j).
TACHO_HOST_DEVICE inline int front_row_tile(int w, int j, int r) {
  const int c0 = j * 64, kb = (w - c0 < 64) ? (w - c0) : 64;
  return r < c0 + kb ? 0 : 1 + (r - c0 - kb) / 64;
}

int build_plan(const Symbolic& S, Plan& P, std::string& err, int front_mode = 0,
               const PlanTuning& tune = PlanTuning());

// Partitioned inverse (SpTRSV variant 3 of the Tacho section).  Every
// supernode's panel [L11; L21] (m x w, the layout of L) is replaced in a
// second buffer by Z = [L11^-1; L21 L11^-1], the solution of Z L11 = [I; L21],
// so that a sweep applies one product per supernode.  Z is formed right to
// left in 64-column blocks j: Z_j = (B_j - sum_{k > j} Z_k L_kj) W_j with W_j
// = L_jj^-1 the factorization's diagonal-block inverse and B = [I; L21].
// Row tile a (rows [64a, 64a + 64) of the panel) of block column i is
// nonzero only for a >= i, and Z_ak is nonzero only for a >= k.
struct PinvTask {
  int32_t s, a, i, j;  // tile (a, i) of front s: R_ai -= Z_aj L_ji, then Z_ai = R_ai W_ii if
                       // i == j - 1; j < 0: Z_ai = R_ai W_ii alone
};
struct FrontTile {
  int32_t s, t;  // front s, 64-column tile t
};
// A sweep task: tile t of front s (forward: 64 rows, backward: 64 columns),
// the chunk c of its reduction dimension (kPinvChunk columns forward, rows
// backward).  A tile with one chunk writes its result itself (slot < 0);
// otherwise chunk c stores a partial product in slot slot + c, and a sum
// task {s, t, nch, slot} of the next launch adds the tile's nch partial
// products in chunk order and writes the result.
struct PinvSweepTask {
  int32_t s, t, c, slot;
};
constexpr int kPinvChunk = 512;
constexpr int kPinvSmallM = 128;  // wave-per-front sweeps: two rows per lane
constexpr int kPinvGatherRows = 256;  // front rows per workgroup of the forward gather (its threads)
constexpr int kPinvGatherMax = 16;    // workgroups per front of the forward gather
struct PinvPlan {
  // setup: launch q runs tasks [setup_ptr[q], setup_ptr[q + 1]); launch 0
  // scales every front's last block column, launch q >= 1 applies the block
  // column finished by launch q - 1; `tiles` lists every 64-column tile
  std::vector<PinvTask> setup;
  std::vector<int64_t> setup_ptr;
  std::vector<FrontTile> tiles;
  // solves, per level h: fronts with at most kPinvSmallM rows and kSmallMax
  // pivot columns [small_ptr[h], small_ptr[h + 1]) of `small` (one wave
  // each, both sweeps); the other fronts [large_ptr[h], ...) of `large`, their
  // forward tasks [frow_ptr[h], frow_ptr[h + 1]) and backward tasks
  // [bcol_ptr[h], bcol_ptr[h + 1])
  std::vector<int32_t> small, large;
  std::vector<int64_t> small_ptr, large_ptr;
  std::vector<PinvSweepTask> frow, bcol;
  std::vector<int64_t> frow_ptr, bcol_ptr;
  // per level: sum tasks of the tiles with several chunks [fsum_ptr[h],
  // fsum_ptr[h + 1]) forward, [bsum_ptr[h], ...) backward
  std::vector<PinvSweepTask> fsum, bsum;
  std::vector<int64_t> fsum_ptr, bsum_ptr;
  // per level: workgroups per large front of the forward gather (one per
  // kPinvGatherRows rows of its largest front, at most kPinvGatherMax)
  std::vector<int32_t> gchunks;
  int64_t slots = 0;  // partial-product slots of the sweeps
  double flops = 0;   // setup flops (2 per multiply-add of the tile products)
};

void build_pinv_plan(const Symbolic& S, PinvPlan& Q);

// Level CSR form of the partitioned inverse (SpTRSV variant 4 of the Tacho
// section): for every level, the inverse of L's level part as sparse rows
// over the solve vector, one sparse matrix-vector product per level and
// sweep.  All matrices live back to back in one CSR (row r holds entries
// [rptr[r], rptr[r + 1]) and acts on solve row rows[r]).  Level h's forward
// ancestor rows are CSR rows [fwd_ptr[2h], fwd_ptr[2h + 1]) (y[i] += the
// sum of -Z21 y over the level's pivot columns, every front of the level
// whose rows hold i in ascending order), its forward pivot rows
// [fwd_ptr[2h + 1], fwd_ptr[2h + 2]) (yfwd[p] = Z11 y), its backward rows
// [b_ptr[h], b_ptr[h + 1]) (x[j] = Z11^T yfwd - Z21^T x, where a column
// index c >= n stands for x[c - n]).  The values come from the inverse
// panels Z, copied by segments, a segment being one front's part of a row.
struct CsrSeg {
  int64_t pos;     // first entry of the segment
  int32_t s, k;    // front; local row (forward) or local column (backward)
  int32_t kind;    // 0 forward pivot row, 1 forward ancestor row, 2 backward row
  int32_t pad;
};
struct LevelCsr {
  std::vector<int32_t> rows;
  std::vector<int64_t> rptr;
  std::vector<int64_t> fwd_ptr, b_ptr;
  std::vector<CsrSeg> segs;
  int64_t nnz = 0;
};
void build_level_csr(const Symbolic& S, LevelCsr& C);

}  // namespace tacho
