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
  const int32_t* diag_q;     // per permuted column: A entry of the diagonal or -1
  const int32_t* wbase;      // per supernode: first diagonal-inverse block (-1: none)
  const int64_t* woff;       // per diagonal-inverse block: element offset
  const int32_t* tbase;      // per pivot block: first row-tile completion flag
};

template <typename T>
struct DevNum {
  T* L;             // factor panels
  T* U;             // update matrices
  T* avals;         // A entries in assembly order (scaled for FP32)
  const double* scale;  // Jacobi scaling per permuted column (FP32 path) or nullptr
  int32_t* fail;    // smallest failing permuted column, INT32_MAX if none
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
void launch_small(const DevSym& S, const DevNum<T>& N, const int32_t* list, int64_t count,
                  hipStream_t st);
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
                 int tile, hipStream_t st);
// Dataflow factorization of one level's large fronts.  flow holds one
// completion flag per row tile of every pivot block (ntiles, indexed through
// DevSym::tbase), one pre-accumulation flag per pivot block (nblocks), one
// range counter per update-matrix tile (nucount), one ticket counter per
// level and the hang flag; all zero before the factorization starts.
template <typename T>
void launch_front(const DevSym& S, const DevNum<T>& N, T* winv, const FrontTask* tasks,
                  int64_t count, int32_t* flow, int64_t ntiles, int64_t nblocks, int64_t nucount,
                  int level, int nlevels, hipStream_t st);

// Solves: y is the permuted right-hand side / solution (n x nrhs, ld n).
template <typename T>
void launch_permute_in(const DevSym& S, const double* b, int64_t ldb, T* y, int64_t nrhs,
                       const double* scale, hipStream_t st);
template <typename T>
void launch_permute_out(const DevSym& S, const T* y, double* x, int64_t ldx, int64_t nrhs,
                        const double* scale, int accumulate, hipStream_t st);
template <typename T>
void launch_fwd(const DevSym& S, const T* L, T* y, T* uvec, const int32_t* list, int64_t count,
                int32_t nrhs, hipStream_t st);
template <typename T>
void launch_bwd(const DevSym& S, const T* L, T* y, const int32_t* list, int64_t count,
                int32_t nrhs, hipStream_t st);

// L21 products of split fronts (matrix-core tiles into `part`, then a
// fixed-order reduction): forward uvec -= L21 x_s, backward y_s -= L21^T u_s.
template <typename T>
void launch_fwd_gemv(const DevSym& S, const T* L, const T* y, T* part, const GemvItem* items,
                     int64_t count, const ReduceItem* red, int64_t nred, T* uvec, int32_t nrhs,
                     hipStream_t st);
template <typename T>
void launch_bwd_gemv(const DevSym& S, const T* L, const T* uvec, T* part, const GemvItem* items,
                     int64_t count, const ReduceItem* red, int64_t nred, T* y, int32_t nrhs,
                     hipStream_t st);
template <typename T>
void launch_bwd_gather(const DevSym& S, const T* y, T* uvec, const int32_t* list, int64_t count,
                       int32_t nrhs, hipStream_t st);

template <typename T>
void launch_fwd_tri(const DevSym& S, const T* L, const T* winv, T* y, const TriItem* items,
                    int64_t count, int32_t* counter, int32_t* flags, int32_t nrhs, hipStream_t st);
template <typename T>
void launch_bwd_tri(const DevSym& S, const T* L, const T* winv, T* y, const TriItem* items,
                    int64_t count, int32_t* counter, int32_t* flags, int32_t nrhs, hipStream_t st);

// FP64 refinement helpers: r = b - A x (original numbering, CSR), column norms.
void launch_residual(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                     const double* b, int64_t ldb, const double* x, int64_t ldx, double* r,
                     int64_t nrhs, hipStream_t st);
void launch_colnorms(int64_t n, const double* v, int64_t ldv, int64_t nrhs, double* out,
                     hipStream_t st);
// out[k + c*nsys] = || v[sys_ptr[k]:sys_ptr[k+1], c] ||_2
void launch_segnorms(int64_t nsys, const int64_t* sys_ptr, const double* v, int64_t ldv,
                     int64_t nrhs, double* out, hipStream_t st);
// v[sys k rows, c] = 0 where mask[k + c*nsys] != 0
void launch_zero_units(int64_t nsys, const int64_t* sys_ptr, double* v, int64_t ldv, int64_t nrhs,
                       const uint8_t* mask, hipStream_t st);

}  // namespace tacho
