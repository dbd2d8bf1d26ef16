// Device-side views shared by the kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace tacho {

// Symbolic arrays resident in HBM (one copy per symbolic handle).
struct DevSym {
  int64_t n;
  const int32_t* sptr;       // ns+1
  const int32_t* front_m;    // ns
  const int64_t* rows_ptr;   // ns+1
  const int32_t* rows;       // rows(s), permuted indices
  const int32_t* rmap;       // child -> parent front positions (rows indexing)
  const int32_t* child_ptr;  // ns+1
  const int32_t* child_list;
  const int64_t* acol_ptr;   // n+1
  const int32_t* a_pos;      // row + col*ldL inside the front panel
  const int64_t* a_src;      // index into the caller's values (-1: added diagonal)
  const int32_t* a_prc;      // 2 per entry: permuted row, permuted column
  const int64_t* L_off;
  const int32_t* ldL;
  const int64_t* U_off;
  const int32_t* ldU;
  const int64_t* u_off;
  const int32_t* perm;       // new -> old
  const int32_t* pinv;       // old -> new
  const int32_t* diag_q;     // per permuted column: A entry of the diagonal or -1
  const int32_t* wbase;      // per supernode: first diagonal-inverse block (-1: none)
  const int64_t* woff;       // per diagonal-inverse block: element offset
  const int32_t* tbase;      // per pivot block: first row-tile completion flag
  const int32_t* sparent;    // per supernode: parent (-1: root)
  const int32_t* pull_ptr;   // per front row (rows_ptr indexing): first extend-add source
  const int32_t* pull_src;   // update-vector entry of each source
  const int32_t* part_base;  // per diagonal block: first backward partial-product slot
  const int32_t* pt1base;    // per pivot block of a chain front: 64 x 64 product slot (-1: none)
  const int32_t* asm_rng;    // per assembly item and child: child column and row ranges
  // LDL^T solves (nullptr otherwise): pivot order lq (L row i is row lq[i] of
  // P A P^T; it moves rows only within a diagonal block) and its inverse.  A
  // front's interchanges act on its own front vector after the children's
  // contributions arrive, so the forward sweep reads pivot position i from
  // front row lq[f + i] - f, and the backward sweep finds the solution of an
  // ancestor's row r at position lqinv[r].
  const int32_t* lq;
  const int32_t* lqinv;
};

template <typename T>
struct DevNum {
  T* L;             // factor panels
  T* U;             // update matrices
  T* avals;         // A entries in assembly order (scaled for FP32)
  const double* scale;  // Jacobi scaling per permuted column (FP32 path) or nullptr
  int32_t* fail;    // smallest failing permuted column, INT32_MAX if none
  T* pt1;           // chain products, 64 x 64 per slot (column-major)
};

// LDL^T factorization outputs (FP64): D as its diagonal d and first
// subdiagonal e (e[k] != 0 marks a 2x2 pivot on permuted columns k, k + 1),
// the pivot order q (row i of L is row q[i] of P A P^T; q moves a column only
// within its diagonal block), and the panels L D of the columns eliminated so
// far, laid out like L (the trailing updates read them).
struct DevLdlt {
  double* d;
  double* e;
  int32_t* q;
  double* ld;
};

// Host launchers (kernels.hip).
template <typename T>
void launch_gather(const DevSym& S, const DevNum<T>& N, const double* vals, int64_t nentries,
                   hipStream_t st);
void launch_scale(const DevSym& S, const double* vals, double* scale, hipStream_t st);
void launch_mirror(const int64_t* idx, const double* src, double* dst, int64_t count,
                   hipStream_t st);
void launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st);
template <typename T>
void launch_leaf(const DevSym& S, const DevNum<T>& N, const int32_t* list, int64_t count,
                 hipStream_t st);
template <typename T>
void launch_small(const DevSym& S, const DevNum<T>& N, const int32_t* list, int64_t count,
                  hipStream_t st);
// big: the kernel for fronts up to kPackedMax rows, else up to kPackedMid
template <typename T>
void launch_packed(const DevSym& S, const DevNum<T>& N, T* winv, const int32_t* list,
                   int64_t count, bool big, hipStream_t st);
// Partitioned inverse (PinvPlan): Z = [I; L21] per front, the setup steps,
// and one level of each sweep (forward: gather, then the merged product).
template <typename T>
void launch_pinv_init(const DevSym& S, T* Z, const T* L, const FrontTile* tiles, int64_t count,
                      hipStream_t st);
template <typename T>
void launch_pinv_step(const DevSym& S, T* Z, const T* L, const T* winv, const PinvTask* tasks,
                      int64_t count, hipStream_t st);
// the fronts of PinvPlan::small, one wave each: forward (y, yfwd, uvec) or
// backward (solution into y)
template <typename T>
void launch_pinv_small(const DevSym& S, const T* Z, T* y, T* yfwd, T* uvec, const int32_t* fronts,
                       int64_t count, bool forward, int nrhs, hipStream_t st);
template <typename T>
void launch_pinv_fwd(const DevSym& S, const T* Z, T* y, T* yout, T* uvec, const int32_t* fronts,
                     int64_t nfronts, int gchunks, const PinvSweepTask* tasks, int64_t ntasks,
                     const PinvSweepTask* sums, int64_t nsums, T* part, int nrhs, hipStream_t st);
template <typename T>
void launch_pinv_bwd(const DevSym& S, const T* Z, const T* yfwd, T* x, const PinvSweepTask* tasks,
                     int64_t ntasks, const PinvSweepTask* sums, int64_t nsums, T* part, int nrhs,
                     hipStream_t st);
template <typename T>
void launch_csr_fill(const DevSym& S, const T* Z, const CsrSeg* segs, int64_t count, int32_t* cols,
                     T* vals, hipStream_t st);
template <typename T>
void launch_level_spmv(const int32_t* rows, const int64_t* rptr, const int32_t* cols, const T* vals,
                       int64_t r0, int64_t r1, int64_t n, const T* a, const T* b, T* out, bool beta,
                       int nrhs, hipStream_t st);
template <typename T>
void launch_assemble(const DevSym& S, const DevNum<T>& N, const AsmItem* items, int64_t count,
                     hipStream_t st);
template <typename T>
void launch_diag(const DevSym& S, const DevNum<T>& N, const PanelItem* items, int64_t count,
                 T* winv, hipStream_t st);
template <typename T>
void launch_panel(const DevSym& S, const DevNum<T>& N, const PanelItem* items, int64_t count,
                  const T* winv, hipStream_t st);
template <typename T>
void launch_gemm(const DevNum<T>& N, const GemmProb* probs, const GemmTile* tiles, int64_t count,
                 int tile, hipStream_t st, const T* bsrc = nullptr, const DevNum<T>* N2 = nullptr,
                 const T* bsrc2 = nullptr);
// Dataflow factorization of one level's large fronts.  flow holds one
// completion flag per row tile of every pivot block (ntiles, indexed through
// DevSym::tbase), one pre-accumulation flag per pivot block (nblocks), one
// range counter per update-matrix tile (nucount), one ticket counter per
// level and the hang flag; all zero before the factorization starts.
template <typename T>
void launch_front(const DevSym& S, const DevNum<T>& N, T* winv, const FrontTask* tasks,
                  int64_t count, int32_t* flow, int64_t ntiles, int64_t nblocks, int64_t nucount,
                  int ticket, int nticket, hipStream_t st);

// Dataflow solves of nrhs <= 16 right-hand sides.  y (n rows of 1 value
// when nrhs = 1, else of 16) receives P b in solve_in, is solved forward and
// backward in place, and x = P^T y leaves in solve_out.  uvec holds the
// update vectors (u_elems rows of the same width), part the backward partial
// products (part_slots x 64 x 16).  counters: 3 ns + nblk + 2 ints, cleared
// by solve_in; hang is raised (never cleared here) if a wait times out.
template <typename T>
void launch_solve_in(const DevSym& S, const double* b, int64_t ldb, T* y, int nrhs,
                     const double* scale, int32_t* counters, int64_t ns, int64_t nblk,
                     hipStream_t st);
template <typename T>
void launch_solve_fwd(const DevSym& S, const T* L, const T* winv, T* y, T* uvec,
                      const SolveTask* tasks, int64_t count, const int32_t* wave_list, int nrhs,
                      int32_t* counters, int64_t ns, int64_t nblk, int32_t* hang, hipStream_t st);
template <typename T>
void launch_solve_bwd(const DevSym& S, const T* L, const T* winv, T* y, T* part,
                      const SolveTask* tasks, int64_t count, const int32_t* wave_list, int nrhs,
                      int32_t* counters, int64_t ns, int64_t nblk, int32_t* hang, hipStream_t st);
// Level-by-level phase of the solves: one launch per level (wave items and
// large fronts of that level); forward before the dataflow launch, backward
// after it.
template <typename T>
void launch_level_fwd(const DevSym& S, const T* L, const T* winv, T* y, T* uvec,
                      const WaveItem* items, int64_t nitems, const int32_t* large, int64_t nlarge,
                      const int32_t* wave_list, int nrhs, int32_t* counters, int64_t ns,
                      int64_t nblk, int32_t* hang, hipStream_t st);
template <typename T>
void launch_level_bwd(const DevSym& S, const T* L, const T* winv, T* y, T* part,
                      const WaveItem* items, int64_t nitems, const int32_t* large, int64_t nlarge,
                      const int32_t* wave_list, int nrhs, int32_t* counters, int64_t ns,
                      int64_t nblk, int32_t* hang, hipStream_t st);
template <typename T>
void launch_solve_out(const DevSym& S, const T* y, double* x, int64_t ldx, int nrhs,
                      const double* scale, int accumulate, hipStream_t st);

// FP64 refinement helpers: r = b - A x (original numbering, CSR), column norms.
void launch_residual(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                     const double* b, int64_t ldb, const double* x, int64_t ldx, double* r,
                     int64_t nrhs, double* xt, hipStream_t st);
void launch_colnorms(int64_t n, const double* v, int64_t ldv, int64_t nrhs, double* out,
                     hipStream_t st);
// out[k + c*nsys] = || v[sys_ptr[k]:sys_ptr[k+1], c] ||_2, each summed in
// kNormParts parts (partial: kNormParts doubles per (system, column))
// added in a fixed order
constexpr int kNormParts = 128;
void launch_segnorms(int64_t nsys, const int64_t* sys_ptr, const double* v, int64_t ldv,
                     int64_t nrhs, double* out, double* partial, hipStream_t st);
// v[sys k rows, c] = 0 where mask[k + c*nsys] != 0
void launch_zero_units(int64_t nsys, const int64_t* sys_ptr, double* v, int64_t ldv, int64_t nrhs,
                       const uint8_t* mask, hipStream_t st);

// v[sys k rows, c] = src[sys k rows, c] where mask[k + c*nsys] != 0 (both with ld)
void launch_select_units(int64_t nsys, const int64_t* sys_ptr, double* v, const double* src,
                         int64_t ld, int64_t nrhs, const uint8_t* mask, hipStream_t st);

// LDL^T (FP64) with Bunch-Kaufman pivoting restricted to diagonal blocks.
void launch_small_ldlt(const DevSym& S, const DevNum<double>& N, const DevLdlt& D,
                       const int32_t* list, int64_t count, hipStream_t st);
void launch_diag_ldlt(const DevSym& S, const DevNum<double>& N, const DevLdlt& D,
                      const PanelItem* items, int64_t count, double* winv, hipStream_t st);
void launch_panel_ldlt(const DevSym& S, const DevNum<double>& N, const DevLdlt& D,
                       const PanelItem* items, int64_t count, const double* winv, hipStream_t st);
// y <- D^{-1} y on the solve vector (permuted rows, kRowLd stride); and the
// permutations of the numeric handle: perm_num[i] = perm[q[i]], pinv_num its
// inverse, qinv the inverse of q.
void launch_apply_dinv(int64_t n, const double* d, const double* e, double* y, int nrhs,
                       hipStream_t st);
// LU (restricted row pivoting): N is the L half (L panels, lower update
// matrices, lower A entries), Nt the U^T half laid out the same way; q gets
// the row order (row i of L U is row q[i] of P A P^T).
void launch_small_lu(const DevSym& S, const DevNum<double>& N, const DevNum<double>& Nt,
                     int32_t* q, const int32_t* list, int64_t count, hipStream_t st);
void launch_diag_lu(const DevSym& S, const DevNum<double>& N, const DevNum<double>& Nt, int32_t* q,
                    const PanelItem* items, int64_t count, double* winv, double* vinv,
                    hipStream_t st);
void launch_lu_rowperm(const DevSym& S, const DevNum<double>& N, const int32_t* q,
                       const PanelItem* items, int64_t count, hipStream_t st);
void launch_panel_lu(const DevSym& S, const DevNum<double>& N, const DevNum<double>& Nt,
                     const int32_t* q, const PanelItem* items, int64_t count, const double* winv,
                     const double* vinv, hipStream_t st);
void launch_ldlt_perm(int64_t n, const int32_t* perm, const int32_t* q, int32_t* perm_num,
                      int32_t* pinv_num, int32_t* qinv, hipStream_t st);
// p[i] = i (the identity pivot order an LDL^T factorization starts from, so
// that a block left unfactored after a failure still holds valid indices).
void launch_iota(int32_t* p, int64_t n, hipStream_t st);

// Scratch of the no-allocation entry points: a file-scope device array of
// kNoAllocScratchBytes per GPU.  Returns its address on the current device
// (looked up once per device).  Calls that overlap on one GPU share it.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch(void** ptr);

}  // namespace tacho
