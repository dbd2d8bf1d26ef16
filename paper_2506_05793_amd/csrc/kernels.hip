// HIP kernels of the numeric phase and the solves (gfx950, wave64).
//
// Multifrontal Cholesky (Tacho section of the paper): every supernode s owns
// a dense front F_s of order m_s over its row set rows(s).  F_s receives the
// entries of C = P A P^T of its w_s pivot columns and the update matrices
// U_c of its children (extend-add), then a partial Cholesky eliminates the
// pivot columns: L11 = chol(F11), L21 = F21 L11^{-T}, U_s = F22 - L21 L21^T.
// Fronts are processed level by level of the supernodal elimination tree.
//
// Determinism: no floating-point atomics anywhere.  Each front pulls its
// children's contributions in ascending child order, and every output element
// is owned by one thread per step, so the result depends only on the front
// sizes, never on how fronts are batched into launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>

#include "device.hpp"

namespace tacho {

namespace {

constexpr int kThreads = 256;
static_assert(kPinvGatherRows == kThreads, "the forward gather takes one front row per thread");
constexpr int kDiagLd = kPanel + 1;  // LDS leading dimension of diagonal blocks

// Row stride of the solve vectors (y and the update vectors): one 128-byte
// cache line per row, whatever the number of right-hand sides, so that rows
// written by different workgroups never share a line.  The L2 caches of the
// XCDs are not coherent with each other, and with 8-byte rows (one
// right-hand side) the dataflow solves gave intermittently wrong results,
// which this layout removed.
template <typename T>
constexpr int kRowLd = 128 / (int)sizeof(T);

template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};
template <>
struct Vec4<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};

// One 16x16x4 matrix-core step: D = A(16x4) * B(4x16) + C.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Its four results are column
// l % 16 of D at rows mfma_row<T>(l, v), v = 0..3: rows l/16 + 4v for the
// FP64 instruction, rows 4(l/16) + v for the FP32 one (checked on gfx950).
__device__ inline Vec4<double>::type mfma16(double a, double b, Vec4<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline Vec4<float>::type mfma16(float a, float b, Vec4<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
__device__ inline int mfma_row(int lane, int v);
template <>
__device__ inline int mfma_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }
template <>
__device__ inline int mfma_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }

// Value of `v` in lane `l` (uniform result).
__device__ inline double readlane(double v, int l) {
  union {
    double d;
    int i[2];
  } u;
  u.d = v;
  u.i[0] = __builtin_amdgcn_readlane(u.i[0], l);
  u.i[1] = __builtin_amdgcn_readlane(u.i[1], l);
  return u.d;
}
__device__ inline float readlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 1/sqrt(x) from the hardware estimate refined by two Newton steps
// (r <- r + r (1 - x r^2) / 2); accurate to about an ulp for normal x > 0,
// NaN or infinite otherwise (the caller flags non-positive pivots).
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double e = __builtin_fma(-x * r, r, 1.0);
  r = __builtin_fma(0.5 * r, e, r);
  e = __builtin_fma(-x * r, r, 1.0);
  return __builtin_fma(0.5 * r, e, r);
}
__device__ inline float rsqrt_nr(float x) {
  float r = __builtin_amdgcn_rsqf(x);
  const float e = __builtin_fmaf(-x * r, r, 1.0f);
  return __builtin_fmaf(0.5f * r, e, r);
}

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// value gather: avals[q] = A entry q of the lower triangle of C, in the order
// of the assembly maps; the FP32 path applies Jacobi scaling d_i d_j.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(DevSym S, DevNum<T> N, const double* vals,
                                                     int64_t count) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= count) return;
  const int64_t src = S.a_src[q];
  double v = src >= 0 ? vals[src] : 0.0;
  if (N.scale) v = v * N.scale[S.a_prc[2 * q]] * N.scale[S.a_prc[2 * q + 1]];
  N.avals[q] = (T)v;
}

// scale[j] = 1/sqrt(C_jj) (1 where the diagonal is not positive, which the
// factorization then reports).
__global__ __launch_bounds__(kThreads) void k_scale(DevSym S, const double* vals, double* scale) {
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= S.n) return;
  const int32_t q = S.diag_q[j];
  const double d = q >= 0 ? vals[S.a_src[q]] : 0.0;
  scale[j] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
}

__global__ __launch_bounds__(kThreads) void k_mirror(const int64_t* idx, const double* src,
                                                     double* dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < count) dst[i] = idx[i] >= 0 ? src[idx[i]] : 0.0;
}

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// Small fronts (m <= kSmallMax): one workgroup assembles the whole front in
// LDS (A entries, then each child's update matrix in ascending child order),
// eliminates the w pivot columns right-looking, and writes the L panel and
// the update matrix U.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_small(DevSym S, DevNum<T> N, const int32_t* list) {
  __shared__ T F[kSmallMax * kSmallMax];
  const int s = list[blockIdx.x];
  const int tid = threadIdx.x;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ld = S.ldL[s];
  for (int t = tid; t < ld * m; t += kThreads) F[t] = T(0);
  __syncthreads();
  {
    const int64_t q0 = S.acol_ptr[f], q1 = S.acol_ptr[f + w];
    for (int64_t q = q0 + tid; q < q1; q += kThreads) F[S.a_pos[q]] = N.avals[q];
  }
  __syncthreads();
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int c = S.child_list[q];
    const int wc = S.sptr[c + 1] - S.sptr[c], rc = S.front_m[c] - wc;
    const T* Uc = N.U + S.U_off[c];
    const int ldc = S.ldU[c];
    const int32_t* rm = S.rmap + S.rows_ptr[c] + wc;
    for (int t = tid; t < rc * rc; t += kThreads) {
      const int jj = t / rc, ii = t - jj * rc;
      if (ii >= jj) F[rm[ii] + rm[jj] * ld] += Uc[ii + (int64_t)jj * ldc];
    }
    __syncthreads();
  }
  for (int j = 0; j < w; ++j) {
    const T d = F[j + j * ld];
    __syncthreads();
    const T ljj = sqrt(d);
    if (tid == 0) {
      F[j + j * ld] = ljj;
      if (!(d > T(0))) atomicMin(N.fail, f + j);
    }
    for (int i = j + 1 + tid; i < m; i += kThreads) F[i + j * ld] = F[i + j * ld] / ljj;
    __syncthreads();
    const int nt = m - j - 1;
    for (int t = tid; t < nt * nt; t += kThreads) {
      const int cc = t / nt, rr = t - cc * nt;
      if (rr >= cc) {
        const int i = j + 1 + rr, k = j + 1 + cc;
        F[i + k * ld] -= F[i + j * ld] * F[k + j * ld];
      }
    }
    __syncthreads();
  }
  T* Lp = N.L + S.L_off[s];
  for (int t = tid; t < ld * w; t += kThreads) Lp[t] = F[t];
  if (r > 0) {
    T* Us = N.U + S.U_off[s];
    const int ldu = S.ldU[s];
    for (int t = tid; t < ldu * r; t += kThreads) {
      const int jj = t / ldu, ii = t - jj * ldu;
      Us[t] = ii < r ? F[(w + ii) + (w + jj) * ld] : T(0);
    }
  }
}

// Cholesky fronts with kSmallMax < m <= kPackedMax and w <= kSmallMax: one
// workgroup assembles the front in LDS as a packed lower triangle (column j
// holds rows j..m-1 from col(j) = j m - j (j - 1) / 2), eliminates the w
// pivot columns right-looking within the pivot panel, writes the L panel, and
// forms every update-matrix entry from its assembled value by subtracting
// the pivot columns' products in column order: the operations of k_small,
// with the trailing updates of one entry applied together.  Last, the
// inverse W = L11^-1 that the solves apply to the diagonal block, by forward
// substitution (one column per thread).
template <typename T, int MAXM>
__global__ __launch_bounds__(kThreads) void k_packed(DevSym S, DevNum<T> N, T* winv,
                                                     const int32_t* list) {
  __shared__ T F[MAXM * (MAXM + 1) / 2];
  __shared__ T dinv[kSmallMax];
  const int s = list[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ld = S.ldL[s];
  auto col = [m](int j) { return j * m - (j * (j - 1)) / 2; };
  for (int t = tid; t < m * (m + 1) / 2; t += kThreads) F[t] = T(0);
  __syncthreads();
  {
    const int64_t q0 = S.acol_ptr[f], q1 = S.acol_ptr[f + w];
    for (int64_t q = q0 + tid; q < q1; q += kThreads) {
      const int pos = S.a_pos[q], j = pos / ld, i = pos - j * ld;
      F[col(j) + i - j] = N.avals[q];
    }
  }
  __syncthreads();
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int c = S.child_list[q];
    const int wc = S.sptr[c + 1] - S.sptr[c], rc = S.front_m[c] - wc;
    const T* Uc = N.U + S.U_off[c];
    const int ldc = S.ldU[c];
    const int32_t* rm = S.rmap + S.rows_ptr[c] + wc;
    for (int t = tid; t < rc * rc; t += kThreads) {
      const int jj = t / rc, ii = t - jj * rc;
      if (ii >= jj) F[col(rm[jj]) + rm[ii] - rm[jj]] += Uc[ii + (int64_t)jj * ldc];
    }
    __syncthreads();
  }
  for (int j = 0; j < w; ++j) {
    const int cj = col(j);
    const T d = F[cj];
    __syncthreads();
    const T ljj = sqrt(d);
    if (tid == 0) {
      F[cj] = ljj;
      if (!(d > T(0))) atomicMin(N.fail, f + j);
    }
    for (int i = j + 1 + tid; i < m; i += kThreads) F[cj + i - j] = F[cj + i - j] / ljj;
    __syncthreads();
    // the pivot panel's later columns now; the update matrix after the loop
    for (int k = j + 1 + wave; k < w; k += kThreads / 64) {
      const int ck = col(k);
      const T lkj = F[cj + k - j];
      for (int i = k + lane; i < m; i += 64) F[ck + i - k] -= F[cj + i - j] * lkj;
    }
    __syncthreads();
  }
  T* Lp = N.L + S.L_off[s];
  for (int t = tid; t < ld * w; t += kThreads) {
    const int j = t / ld, i = t - j * ld;
    Lp[t] = (i >= j && i < m) ? F[col(j) + i - j] : T(0);
  }
  if (r > 0) {
    T* Us = N.U + S.U_off[s];
    const int ldu = S.ldU[s];
    for (int t = tid; t < ldu * r; t += kThreads) {
      const int kk = t / ldu, ii = t - kk * ldu;
      T v = T(0);
      if (ii < r && ii >= kk) {
        const int i = w + ii, k = w + kk;
        v = F[col(k) + i - k];
        int cs = 0;  // col(j)
        for (int j = 0; j < w; ++j) {
          v -= F[cs + i - j] * F[cs + k - j];
          cs += m - j;
        }
      }
      Us[t] = v;
    }
  }
  // W, packed by columns (column c at wc(c) = c w - c (c - 1) / 2) in the
  // space from col(w) on, no longer needed: the plan sends a front here only
  // if w (m + 1) <= MAXM (MAXM + 1) / 2, so it fits.
  for (int i = tid; i < w; i += kThreads) dinv[i] = T(1) / F[col(i)];
  __syncthreads();
  T* Wl = F + col(w);
  if (tid < w) {
    const int c = tid, wc = c * w - (c * (c - 1)) / 2;
    Wl[wc] = dinv[c];
    for (int i = c + 1; i < w; ++i) {
      T acc = T(0);
      int ck = col(c);
      for (int k = c; k < i; ++k) {
        acc += F[ck + i - k] * Wl[wc + k - c];
        ck += m - k;
      }
      Wl[wc + i - c] = -(acc * dinv[i]);
    }
  }
  __syncthreads();
  T* Wout = winv + S.woff[S.wbase[s]];  // w x w, column-major
  for (int t = tid; t < w * w; t += kThreads) {
    const int c = t / w, i = t - c * w;
    Wout[t] = i >= c ? Wl[c * w - (c * (c - 1)) / 2 + i - c] : T(0);
  }
}

// Leaf fronts with one pivot column, no children and m <= kLeafMax, one
// thread each: the same operations as k_small (A entries into a zero
// column, pivot square root, column scaled by it, update matrix 0 - l l^T),
// in registers.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_leaf(DevSym S, DevNum<T> N, const int32_t* list,
                                                   int count) {
  const int idx = blockIdx.x * kThreads + threadIdx.x;
  if (idx >= count) return;
  const int s = list[idx];
  const int f = S.sptr[s], m = S.front_m[s], r = m - 1;
  const int ld = S.ldL[s];
  T x[kLeafMax];
#pragma unroll
  for (int i = 0; i < kLeafMax; ++i) x[i] = T(0);
  for (int64_t q = S.acol_ptr[f]; q < S.acol_ptr[f + 1]; ++q) {
    const int pos = S.a_pos[q];
    const T v = N.avals[q];
#pragma unroll
    for (int i = 0; i < kLeafMax; ++i) x[i] = pos == i ? v : x[i];
  }
  const T d = x[0];
  const T l0 = sqrt(d);
  if (!(d > T(0))) atomicMin(N.fail, f);
  x[0] = l0;
#pragma unroll
  for (int i = 1; i < kLeafMax; ++i) x[i] = x[i] / l0;
  T* Lp = N.L + S.L_off[s];
#pragma unroll
  for (int i = 0; i < kLeafMax; ++i)
    if (i < ld) Lp[i] = i < m ? x[i] : T(0);
  if (r > 0) {
    T* Us = N.U + S.U_off[s];
    const int ldu = S.ldU[s];
#pragma unroll
    for (int jj = 0; jj < kLeafMax - 1; ++jj) {
      if (jj < r) {
#pragma unroll
        for (int ii = 0; ii < kLeafMax; ++ii)
          if (ii < ldu) Us[ii + (int64_t)jj * ldu] = (ii < r && ii >= jj) ? T(0) - x[1 + ii] * x[1 + jj] : T(0);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Large fronts, assembly: the workgroup owns the entries of front s in
// columns [c0, c1) and front rows [r0, r1) (at most kAsmTile).  It sums them
// in LDS -- zero, the A entries, then every child's update matrix in
// ascending child order -- and writes each entry once.  The child's
// relative map is increasing, so its columns landing in [c0, c1) and its
// rows landing in [r0, r1) are contiguous ranges (from the plan).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_assemble(DevSym S, DevNum<T> N,
                                                       const AsmItem* items) {
  __shared__ T tile[kAsmTile];  // tile[(c - c0) nr + (row - r0)]
  const AsmItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int s = it.s;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f;
  const int ldl = S.ldL[s], ldu = S.ldU[s];
  const int nr = it.r1 - it.r0, nc = it.c1 - it.c0;
  T* Lp = N.L + S.L_off[s];
  T* Us = w < S.front_m[s] ? N.U + S.U_off[s] : nullptr;
  for (int t = tid; t < nr * nc; t += kThreads) tile[t] = T(0);
  __syncthreads();
  for (int c = it.c0; c < min(it.c1, w); ++c) {
    const int64_t q0 = S.acol_ptr[f + c], q1 = S.acol_ptr[f + c + 1];
    for (int64_t q = q0 + tid; q < q1; q += kThreads) {
      const int row = (int)(S.a_pos[q] - (int64_t)c * ldl);
      if (row >= it.r0 && row < it.r1) tile[(c - it.c0) * nr + row - it.r0] = N.avals[q];
    }
  }
  __syncthreads();
  // one wave per child column, rows in lanes, four rows per lane fetched
  // before their sums are stored (the row map is injective, so the targets
  // of one child are distinct)
  const int32_t* rg = S.asm_rng + 4 * (int64_t)it.rbase;
  const int lane = tid & 63, wave = tid >> 6;
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q, rg += 4) {
    const int lo = rg[0], hi = rg[1], ilo = rg[2], ihi = rg[3];
    if (lo >= hi || ilo >= ihi) continue;  // same for the whole workgroup
    const int c = S.child_list[q];
    const int wc = S.sptr[c + 1] - S.sptr[c];
    const T* Uc = N.U + S.U_off[c];
    const int ldc = S.ldU[c];
    const int32_t* rm = S.rmap + S.rows_ptr[c] + wc;
    for (int jj = lo + wave; jj < hi; jj += kThreads / 64) {
      T* col = tile + (rm[jj] - it.c0) * nr - it.r0;  // indexed by front row
      const T* src = Uc + (int64_t)jj * ldc;
      for (int i0 = max(jj, ilo) + lane; i0 < ihi; i0 += 4 * 64) {
        int tr[4];
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ii = i0 + 64 * u;
          tr[u] = ii < ihi ? rm[ii] : -1;
          v[u] = ii < ihi ? src[ii] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (tr[u] >= 0) col[tr[u]] += v[u];
      }
    }
    __syncthreads();
  }
  // Write-out: panel columns rows [0, ldl), update-matrix columns from row
  // (c - w) & ~63 of U (what the front kernel's tiles and the parent's
  // lower-triangle pull read).
  for (int t = tid; t < nr * nc; t += kThreads) {
    const int cc = t / nr, row = it.r0 + (t - cc * nr), c = it.c0 + cc;
    if (c < w) {
      if (row < ldl) Lp[row + (int64_t)c * ldl] = tile[t];
    } else if (row >= w + ((c - w) & ~(kPanel - 1)) && row < w + ldu) {
      Us[(row - w) + (int64_t)(c - w) * ldu] = tile[t];
    }
  }
}

// ---------------------------------------------------------------------------
// Diagonal blocks of large fronts: Cholesky of a 64 x 64 block in LDS,
// blocked by 16 columns (a 16x16 block by one wave, its rows below by one
// thread each, a rank-16 update of the rest), and its inverse W = L_kk^{-1},
// kept per block for the triangular solves of the rows below and for the
// solve phase.  Non-positive or NaN pivots go to the failure flag.
constexpr int kSub = 16;

// 16x16x16 product on the matrix cores: acc += A B, with lane l supplying
// A(l % 16, k) and B(k, l % 16) for k = l / 16 + 4 s through the accessors.
template <typename T, typename FA, typename FB>
__device__ inline typename Vec4<T>::type mm16(FA a, FB b, typename Vec4<T>::type acc) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma16(a(i, 4 * s + kq), b(4 * s + kq, i), acc);
  return acc;
}

// Cholesky of the kb x kb diagonal block held in D (column-major, ld
// kDiagLd, entries past kb set to the identity), in place, and its inverse W
// = L^{-1} (same layout).  Blocked by 16 columns up to kb rounded to 16:
// per block, one wave factors the 16-column panel in registers (all of its
// rows, one per lane; pivots and column entries broadcast with readlane) and
// the trailing lower triangle is updated on the matrix cores.  Then each
// 16x16 diagonal block is inverted by its own wave (one lane per row), and
// the off-diagonal blocks of W follow by distance from the diagonal: W_ib =
// -W_ii sum_{q=b}^{i-1} L_iq W_qb.  A non-positive or NaN pivot j records
// col0 + j in *fail.  Every thread of the workgroup takes part; Tmp holds
// 3 x 256 scratch elements.
template <typename T>
__device__ __forceinline__ void diag_factor_inverse(T* D, T* W, T (*Tmp)[kSub * kSub], int kb,
                                                    int col0, int32_t* fail) {
  typedef typename Vec4<T>::type V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kr = (kb + kSub - 1) / kSub * kSub;
  const int nb = kr / kSub;
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    W[c * kDiagLd + r] = (r == c && r >= kr) ? T(1) : T(0);
  }
  __syncthreads();
  for (int jb = 0; jb < kr; jb += kSub) {
    // (1) 16-column panel, rows jb..kr-1, wave 0: lane i holds row jb + i.
    // Updates run on every lane: entries above the diagonal become garbage
    // that is never broadcast or stored, which keeps the pivot chain free of
    // lane masks.  The reciprocal pivots go to the diagonal of W, where the
    // inversion below picks them up.
    if (wave == 0) {
      const int row = jb + lane;
      const bool valid = row < kr;
      T a[kSub];
#pragma unroll
      for (int c = 0; c < kSub; ++c) a[c] = valid ? D[(jb + c) * kDiagLd + row] : T(0);
      T myinv = T(0);
      uint32_t bad = 0;  // pivots that are not positive (or NaN), bit j
#pragma unroll
      for (int j = 0; j < kSub; ++j) {
        const T piv = readlane(a[j], j);
        bad |= (piv > T(0)) ? 0u : (1u << j);
        const T rinv = rsqrt_nr(piv);
        if (lane == j) myinv = rinv;
        a[j] = lane == j ? piv * rinv : a[j] * rinv;
#pragma unroll
        for (int c = j + 1; c < kSub; ++c) a[c] -= a[j] * readlane(a[j], c);
      }
      if (kb - jb < kSub) bad &= (1u << (kb - jb)) - 1u;  // identity padding past kb
      if (lane == 0 && bad != 0) atomicMin(fail, col0 + jb + __builtin_ctz(bad));
      if (valid) {
#pragma unroll
        for (int c = 0; c < kSub; ++c)
          if (c <= lane) D[(jb + c) * kDiagLd + row] = a[c];
      }
      if (lane < kSub) W[row * kDiagLd + row] = myinv;
    }
    __syncthreads();
    const int below = (kr - jb - kSub) / kSub;  // 16-row blocks below
    if (below == 0) break;
    // (2) trailing lower triangle: D_ij -= X_i X_j^T over 16x16 blocks i >= j
    for (int q = wave; q < below * (below + 1) / 2; q += kThreads / 64) {
      int bi = 0;
      while ((bi + 1) * (bi + 2) / 2 <= q) ++bi;
      const int bj = q - bi * (bi + 1) / 2;
      const int ri = jb + kSub + bi * kSub, rj = jb + kSub + bj * kSub;
      V4 acc = V4{0, 0, 0, 0};
      acc = mm16<T>([&](int m, int k) { return D[(jb + k) * kDiagLd + ri + m]; },
                    [&](int k, int n) { return D[(jb + k) * kDiagLd + rj + n]; }, acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T* p = D + (rj + (lane & 15)) * kDiagLd + ri + mfma_row<T>(lane, v);
        *p -= acc[v];
      }
    }
    __syncthreads();
  }
  // (3) inverses of the 16x16 diagonal blocks, wave b for block b (lane i
  // holds row i of L_bb in a[] and, afterwards, row i of W_bb in x[]): row q
  // of W_bb is final once rows < q are subtracted; it is scaled by 1 / L_qq
  // and subtracted from the rows below.
  if (wave < nb && lane < kSub) {
    const int o = wave * kSub;
    T a[kSub];
#pragma unroll
    for (int c = 0; c < kSub; ++c) a[c] = D[(o + c) * kDiagLd + o + lane];
    const T myinv = W[(o + lane) * kDiagLd + o + lane];
    T x[kSub];
#pragma unroll
    for (int k = 0; k < kSub; ++k) x[k] = lane == k ? T(1) : T(0);
#pragma unroll
    for (int q = 0; q < kSub; ++q) {
#pragma unroll
      for (int k = 0; k <= q; ++k) x[k] = lane == q ? x[k] * myinv : x[k];
#pragma unroll
      for (int k = 0; k <= q; ++k) x[k] -= (lane > q ? a[q] : T(0)) * readlane(x[k], q);
    }
#pragma unroll
    for (int k = 0; k < kSub; ++k) W[(o + k) * kDiagLd + o + lane] = x[k];
  }
  __syncthreads();
  // off-diagonal blocks of W, by distance d from the diagonal
  for (int d = 1; d < nb; ++d) {
    const int b = wave, i = wave + d;
    const bool act = b + d < nb;
    if (act) {
      V4 acc = V4{0, 0, 0, 0};
      for (int q = b; q < i; ++q)
        acc = mm16<T>([&](int m, int k) { return D[(kSub * q + k) * kDiagLd + kSub * i + m]; },
                      [&](int k, int n) { return W[(kSub * b + n) * kDiagLd + kSub * q + k]; },
                      acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) Tmp[wave][mfma_row<T>(lane, v) * kSub + (lane & 15)] = acc[v];
    }
    __syncthreads();
    if (act) {
      V4 acc = V4{0, 0, 0, 0};
      acc = mm16<T>([&](int m, int k) { return W[(kSub * i + k) * kDiagLd + kSub * i + m]; },
                    [&](int k, int n) { return Tmp[wave][k * kSub + n]; }, acc);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        W[(kSub * b + (lane & 15)) * kDiagLd + kSub * i + mfma_row<T>(lane, v)] = -acc[v];
    }
    __syncthreads();
  }
}

// Large fronts, panel step 1 (stepwise path): Cholesky of the diagonal
// block [k, k+kb) of front s and its inverse, kept for the solves.
template <typename T>
__global__ __launch_bounds__(kThreads, 2) void k_diag(DevSym S, DevNum<T> N, const PanelItem* items,
                                                   T* winv) {
  __shared__ T D[kPanel * kDiagLd];  // column-major, D[c * kDiagLd + r]
  __shared__ T W[kPanel * kDiagLd];
  __shared__ T Tmp[3][kSub * kSub];
  const PanelItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int s = it.s, k = it.k, kb = it.kb;
  const int f = S.sptr[s], ld = S.ldL[s];
  T* Lp = N.L + S.L_off[s];
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    T v;
    if (r < kb && c < kb)
      v = r >= c ? Lp[(k + r) + (int64_t)(k + c) * ld] : T(0);
    else
      v = r == c ? T(1) : T(0);
    D[c * kDiagLd + r] = v;
  }
  __syncthreads();
  diag_factor_inverse<T>(D, W, Tmp, kb, f + k, N.fail);
  for (int t = tid; t < kb * kb; t += kThreads) {
    const int c = t / kb, r = t - c * kb;
    if (r >= c) Lp[(k + r) + (int64_t)(k + c) * ld] = D[c * kDiagLd + r];
  }
  T* Wout = winv + S.woff[it.wblk];  // kb x kb, column-major
  for (int t = tid; t < kb * kb; t += kThreads) {
    const int c = t / kb, r = t - c * kb;
    Wout[t] = W[c * kDiagLd + r];
  }
}

// Large fronts, panel step 2: the rows below the diagonal block, 64 per
// workgroup, X = B W^T on the matrix cores (W = L_kk^{-1} from step 1),
// written in place.  B's columns past kb are read as zeros.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_panel(DevSym S, DevNum<T> N, const PanelItem* items,
                                                    const T* winv) {
  constexpr int PAD = 4;
  __shared__ T Bs[kPanel][kPanel + PAD];  // Bs[c][r] = B[r][c]
  __shared__ T Ws[kPanel][kPanel + PAD];  // Ws[c'][c] = W[c][c']
  const PanelItem it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = it.s, k = it.k, kb = it.kb;
  const int m = S.front_m[s], ld = S.ldL[s];
  T* Lp = N.L + S.L_off[s];
  const int r0 = k + kb + it.chunk * kPanel;
  const T* Win = winv + S.woff[it.wblk];  // kb x kb column-major: Win[c * kb + r] = W[r][c]
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    Ws[c][r] = (r < kb && c < kb) ? Win[c * kb + r] : T(0);
    const int row = r0 + r;
    Bs[c][r] = (row < m && c < kb) ? Lp[row + (int64_t)(k + c) * ld] : T(0);
  }
  __syncthreads();
  typedef typename Vec4<T>::type V4;
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int ks = 0; ks < kPanel / 4; ++ks) {
    const int kk = ks * 4 + (lane >> 4);
    T av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = Bs[kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = Ws[kk][wc * 32 + b * 16 + (lane & 15)];
    // D[m][n] = sum_kk W[m][kk] B[n][kk] = X[n][m]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr * 32 + a * 16 + (lane & 15);
        const int c = wc * 32 + b * 16 + mfma_row<T>(lane, v);
        const int row = r0 + r;
        if (row < m && c < kb) Lp[row + (int64_t)(k + c) * ld] = acc[a][b][v];
      }
}

// ---------------------------------------------------------------------------
// LDL^T of a symmetric indefinite C (Tacho section: besides Cholesky, LDL^T of
// a symmetric indefinite matrix with pivots searched only within each
// diagonal block).  The diagonal blocks are the supernodes' pivot columns cut
// into blocks of at most kPanel columns; inside a block, Bunch-Kaufman
// partial pivoting with the candidate rows and columns limited to the
// block's columns not yet eliminated.  L is stored unit lower triangular
// (explicit ones on the diagonal, a zero below the first column of a 2x2
// pivot), D as d / e, the interchanges as the pivot order q.  FP64 only.

constexpr double kBkAlpha = 0x1.47e0f66afed07p-1;  // (1 + sqrt(17)) / 8, rounded to nearest

// Pivot choice for position k among the block's positions [k, b1) of the
// symmetric matrix whose lower triangle is F (element (i, j), i >= j, at
// F[j * ld + i]): .x = size (1 or 2; 0: no usable pivot), .y = the position
// moved to k (size 1) or to k + 1 (size 2).  Ties go to the smallest index.
__device__ inline int2 bk_choose(const double* F, int ld, int k, int b1) {
  double lam = 0.0;
  int r = k;
  for (int i = k + 1; i < b1; ++i) {
    const double v = fabs(F[k * ld + i]);
    if (v > lam) {
      lam = v;
      r = i;
    }
  }
  const double akk = fabs(F[k * ld + k]);
  if (lam == 0.0) return make_int2(F[k * ld + k] == 0.0 ? 0 : 1, k);
  if (akk >= kBkAlpha * lam) return make_int2(1, k);
  double sigma = 0.0;
  for (int j = k; j < b1; ++j) {
    if (j == r) continue;
    const double v = fabs(j < r ? F[j * ld + r] : F[r * ld + j]);
    sigma = v > sigma ? v : sigma;
  }
  if (akk * sigma >= kBkAlpha * lam * lam) return make_int2(1, k);
  if (fabs(F[r * ld + r]) >= kBkAlpha * sigma) return make_int2(1, r);
  return make_int2(2, r);
}

// Symmetric interchange of rows and columns p < r of the order-m matrix whose
// lower triangle is F; the columns before p (eliminated pivots) exchange
// their rows p and r too.  Every thread touches its own elements.
__device__ inline void sym_swap(double* F, int ld, int m, int p, int r) {
  for (int t = threadIdx.x; t < m; t += kThreads) {
    double* a = nullptr;
    double* b = nullptr;
    if (t == p) {
      a = F + p * ld + p;
      b = F + r * ld + r;
    } else if (t < p) {
      a = F + t * ld + p;
      b = F + t * ld + r;
    } else if (t < r) {
      a = F + p * ld + t;
      b = F + t * ld + r;
    } else if (t > r) {
      a = F + p * ld + t;
      b = F + r * ld + t;
    }
    if (a) {
      const double v = *a;
      *a = *b;
      *b = v;
    }
  }
}

// Right-looking restricted Bunch-Kaufman elimination of positions [0, w) of
// the order-m matrix F in LDS (lower triangle, leading dimension ld); every
// position of [0, w) is one block.  On return F holds the unit lower L in
// columns [0, w) and the Schur complement below; pivots go to d / e at
// col0 + position, the order to qloc.  Returns the failing position, or -1.
// c0 / c1 hold kSmallMax (or kPanel) entries of scratch each.
__device__ inline int ldlt_eliminate(double* F, int ld, int m, int w, int* qloc, double* c0,
                                     double* c1, double* d, double* e, int2* choice) {
  const int tid = threadIdx.x;
  for (int t = tid; t < w; t += kThreads) qloc[t] = t;
  __syncthreads();
  int k = 0;
  while (k < w) {
    if (tid == 0) *choice = bk_choose(F, ld, k, w);
    __syncthreads();
    const int2 ch = *choice;
    __syncthreads();
    if (ch.x == 0) return k;
    const int p = ch.x == 1 ? k : k + 1;
    if (ch.y != p) {
      sym_swap(F, ld, m, p, ch.y);
      if (tid == 0) {
        const int t = qloc[p];
        qloc[p] = qloc[ch.y];
        qloc[ch.y] = t;
      }
    }
    __syncthreads();
    if (ch.x == 1) {
      const double piv = F[k * ld + k];
      for (int i = k + 1 + tid; i < m; i += kThreads) c0[i] = F[k * ld + i];
      __syncthreads();
      const int nt = m - k - 1;
      for (int t = tid; t < nt * nt; t += kThreads) {
        const int cc = t / nt, rr = t - cc * nt;
        if (rr >= cc) {
          const int i = k + 1 + rr, j = k + 1 + cc;
          F[j * ld + i] -= (c0[i] / piv) * c0[j];
        }
      }
      for (int i = k + 1 + tid; i < m; i += kThreads) F[k * ld + i] = c0[i] / piv;
      if (tid == 0) {
        d[k] = piv;
        e[k] = 0.0;
        F[k * ld + k] = 1.0;
      }
      __syncthreads();
      k += 1;
    } else {
      const double a = F[k * ld + k], b = F[k * ld + k + 1], c = F[(k + 1) * ld + k + 1];
      const double det = a * c - b * b;
      for (int i = k + 2 + tid; i < m; i += kThreads) {
        c0[i] = F[k * ld + i];
        c1[i] = F[(k + 1) * ld + i];
      }
      __syncthreads();
      const int nt = m - k - 2;
      for (int t = tid; t < nt * nt; t += kThreads) {
        const int cc = t / nt, rr = t - cc * nt;
        if (rr >= cc) {
          const int i = k + 2 + rr, j = k + 2 + cc;
          const double l0 = (c0[i] * c - c1[i] * b) / det, l1 = (c1[i] * a - c0[i] * b) / det;
          F[j * ld + i] -= l0 * c0[j] + l1 * c1[j];
        }
      }
      for (int i = k + 2 + tid; i < m; i += kThreads) {
        F[k * ld + i] = (c0[i] * c - c1[i] * b) / det;
        F[(k + 1) * ld + i] = (c1[i] * a - c0[i] * b) / det;
      }
      if (tid == 0) {
        d[k] = a;
        d[k + 1] = c;
        e[k] = b;
        e[k + 1] = 0.0;
        F[k * ld + k] = 1.0;
        F[k * ld + k + 1] = 0.0;
        F[(k + 1) * ld + k + 1] = 1.0;
      }
      __syncthreads();
      k += 2;
    }
  }
  return -1;
}

// Small fronts (m <= kSmallMax), LDL^T: assembly as in k_small, elimination
// of the w pivot positions (one diagonal block), L panel and U written out.
__global__ __launch_bounds__(kThreads) void k_small_ldlt(DevSym S, DevNum<double> N, DevLdlt D,
                                                         const int32_t* list) {
  __shared__ double F[kSmallMax * kSmallMax];
  __shared__ double c0[kSmallMax], c1[kSmallMax], dd[kSmallMax], ee[kSmallMax];
  __shared__ int qloc[kSmallMax];
  __shared__ int2 choice;
  const int s = list[blockIdx.x];
  const int tid = threadIdx.x;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ld = S.ldL[s];
  for (int t = tid; t < ld * m; t += kThreads) F[t] = 0.0;
  __syncthreads();
  {
    const int64_t q0 = S.acol_ptr[f], q1 = S.acol_ptr[f + w];
    for (int64_t q = q0 + tid; q < q1; q += kThreads) F[S.a_pos[q]] = N.avals[q];
  }
  __syncthreads();
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int c = S.child_list[q];
    const int wc = S.sptr[c + 1] - S.sptr[c], rc = S.front_m[c] - wc;
    const double* Uc = N.U + S.U_off[c];
    const int ldc = S.ldU[c];
    const int32_t* rm = S.rmap + S.rows_ptr[c] + wc;
    for (int t = tid; t < rc * rc; t += kThreads) {
      const int jj = t / rc, ii = t - jj * rc;
      if (ii >= jj) F[rm[ii] + rm[jj] * ld] += Uc[ii + (int64_t)jj * ldc];
    }
    __syncthreads();
  }
  const int bad = ldlt_eliminate(F, ld, m, w, qloc, c0, c1, dd, ee, &choice);
  if (bad >= 0) {
    if (tid == 0) atomicMin(N.fail, f + bad);
    return;
  }
  for (int c = tid; c < w; c += kThreads) {
    D.d[f + c] = dd[c];
    D.e[f + c] = ee[c];
    D.q[f + c] = f + qloc[c];
  }
  double* Lp = N.L + S.L_off[s];
  for (int t = tid; t < ld * w; t += kThreads) Lp[t] = F[t];
  if (r > 0) {
    double* Us = N.U + S.U_off[s];
    const int ldu = S.ldU[s];
    for (int t = tid; t < ldu * r; t += kThreads) {
      const int jj = t / ldu, ii = t - jj * ldu;
      Us[t] = ii < r ? F[(w + ii) + (w + jj) * ld] : 0.0;
    }
  }
}

// Large fronts, LDL^T step 1 (stepwise launches): elimination of diagonal
// block [k, k + kb) of front s (already updated by the blocks before it),
// the block's interchanges applied to the rows of the front's earlier
// columns (L and L D), and W = L_kk^{-1} (unit lower) kept for the panel and
// the solves.
__global__ __launch_bounds__(kThreads) void k_diag_ldlt(DevSym S, DevNum<double> N, DevLdlt D,
                                                        const PanelItem* items, double* winv) {
  __shared__ double F[kPanel * kDiagLd];
  __shared__ double c0[kPanel], c1[kPanel], dd[kPanel], ee[kPanel];
  __shared__ int qloc[kPanel];
  __shared__ int2 choice;
  const PanelItem it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = it.s, k = it.k, kb = it.kb;
  const int f = S.sptr[s], ld = S.ldL[s];
  double* Lp = N.L + S.L_off[s];
  double* LDp = D.ld + S.L_off[s];
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    F[c * kDiagLd + r] = (r < kb && c < kb && r >= c) ? Lp[(k + r) + (int64_t)(k + c) * ld] : 0.0;
  }
  __syncthreads();
  const int bad = ldlt_eliminate(F, kDiagLd, kb, kb, qloc, c0, c1, dd, ee, &choice);
  if (bad >= 0) {
    if (tid == 0) atomicMin(N.fail, f + k + bad);
    return;
  }
  for (int c = tid; c < kb; c += kThreads) {
    D.d[f + k + c] = dd[c];
    D.e[f + k + c] = ee[c];
    D.q[f + k + c] = f + k + qloc[c];
  }
  for (int t = tid; t < kb * kb; t += kThreads) {
    const int c = t / kb, r = t - c * kb;
    if (r >= c) Lp[(k + r) + (int64_t)(k + c) * ld] = F[c * kDiagLd + r];
  }
  // rows of this block in the earlier columns: new row r <- old row qloc[r]
  for (int p = wave; p < k; p += kThreads / 64) {
    double* lc = Lp + (int64_t)p * ld + k;
    double* dc = LDp + (int64_t)p * ld + k;
    const double lv = lane < kb ? lc[qloc[lane]] : 0.0;
    const double dv = lane < kb ? dc[qloc[lane]] : 0.0;
    if (lane < kb) {
      lc[lane] = lv;
      dc[lane] = dv;
    }
  }
  // W = L_kk^{-1}: column c by forward substitution (one thread per column)
  __syncthreads();
  double* Wout = winv + S.woff[it.wblk];  // kb x kb, column-major
  if (tid < kb) {
    const int c = tid;
    for (int r = 0; r < kb; ++r) {
      double v = r == c ? 1.0 : 0.0;
      if (r > c)
        for (int j = c; j < r; ++j) v -= F[j * kDiagLd + r] * Wout[c * kb + j];
      Wout[c * kb + r] = r < c ? 0.0 : v;
    }
  }
}

// Large fronts, LDL^T step 2: 64 rows below the diagonal block, X = B W^T
// with B the rows' entries in the block's columns taken in pivot order (the
// block's interchanges permute these columns), on the matrix cores; X is
// their L D, stored, and L = X D^{-1} replaces them.
__global__ __launch_bounds__(kThreads) void k_panel_ldlt(DevSym S, DevNum<double> N, DevLdlt D,
                                                         const PanelItem* items,
                                                         const double* winv) {
  constexpr int PAD = 4;
  __shared__ double Bs[kPanel][kPanel + PAD];  // Bs[c][r] = B[r][c]
  __shared__ double Ws[kPanel][kPanel + PAD];  // Ws[c'][c] = W[c][c']
  const PanelItem it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = it.s, k = it.k, kb = it.kb;
  const int f = S.sptr[s], m = S.front_m[s], ld = S.ldL[s];
  double* Lp = N.L + S.L_off[s];
  double* LDp = D.ld + S.L_off[s];
  const int r0 = k + kb + it.chunk * kPanel;
  const double* Win = winv + S.woff[it.wblk];
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    Ws[c][r] = (r < kb && c < kb) ? Win[c * kb + r] : 0.0;
    const int row = r0 + r;
    const int src = c < kb ? D.q[f + k + c] - f : 0;  // front column in pivot order
    Bs[c][r] = (row < m && c < kb) ? Lp[row + (int64_t)src * ld] : 0.0;
  }
  __syncthreads();
  typedef Vec4<double>::type V4;
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int ks = 0; ks < kPanel / 4; ++ks) {
    const int kk = ks * 4 + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = Bs[kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = Ws[kk][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
  }
  __syncthreads();
  // X[r][c] into Bs[c][r] (B is no longer needed)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr * 32 + a * 16 + (lane & 15);
        const int c = wc * 32 + b * 16 + mfma_row<double>(lane, v);
        Bs[c][r] = acc[a][b][v];
      }
  __syncthreads();
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    const int row = r0 + r;
    if (row >= m || c >= kb) continue;
    const double x = Bs[c][r];
    const double ec = D.e[f + k + c];
    double l;
    if (ec != 0.0) {  // first column of a 2x2 pivot
      const double d0 = D.d[f + k + c], d1 = D.d[f + k + c + 1];
      l = (x * d1 - Bs[c + 1][r] * ec) / (d0 * d1 - ec * ec);
    } else if (c > 0 && D.e[f + k + c - 1] != 0.0) {  // second column
      const double ep = D.e[f + k + c - 1];
      const double d0 = D.d[f + k + c - 1], d1 = D.d[f + k + c];
      l = (x * d0 - Bs[c - 1][r] * ep) / (d0 * d1 - ep * ep);
    } else {
      l = x / D.d[f + k + c];
    }
    LDp[row + (int64_t)(k + c) * ld] = x;
    Lp[row + (int64_t)(k + c) * ld] = l;
  }
}

// y <- D^{-1} y, rows in pivot order, kRowLd values per row.
__global__ __launch_bounds__(kThreads) void k_apply_dinv(int64_t n, const double* d,
                                                         const double* e, double* y, int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  constexpr int ldy = kRowLd<double>;
  if (e[i] != 0.0) {
    const double a = d[i], b = e[i], c = d[i + 1], det = a * c - b * b;
    for (int r = 0; r < nrhs; ++r) {
      const double y0 = y[i * ldy + r], y1 = y[(i + 1) * ldy + r];
      y[i * ldy + r] = (c * y0 - b * y1) / det;
      y[(i + 1) * ldy + r] = (a * y1 - b * y0) / det;
    }
  } else if (i == 0 || e[i - 1] == 0.0) {
    for (int r = 0; r < nrhs; ++r) y[i * ldy + r] /= d[i];
  }
}

__global__ __launch_bounds__(kThreads) void k_iota(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

__global__ __launch_bounds__(kThreads) void k_ldlt_perm(int64_t n, const int32_t* perm,
                                                        const int32_t* q, int32_t* perm_num,
                                                        int32_t* pinv_num, int32_t* qinv) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int32_t o = perm[q[i]];
  perm_num[i] = o;
  pinv_num[o] = (int32_t)i;
  qinv[q[i]] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// LU of a matrix with a symmetric pattern, row pivoting restricted to the
// diagonal blocks.  A front is kept as two halves laid out like a Cholesky
// front: the L half (N: unit lower L panel, lower triangle of the update
// matrix, the lower A entries) and the U^T half (Nt: U^T panel, the update
// matrix's upper triangle stored transposed, the upper A entries
// transposed).  The assembly and the trailing updates run once per half with
// the halves' roles swapped; the diagonal entries live in the L half (the
// U^T half's diagonal is never read before the factorization stores U's
// diagonal there).

// Pivot of one column by wave 0 (lane = row, a = the lane's entry): the
// largest magnitude among lanes [lo, hi), ties to the first; *piv = its row
// (-1 if all are zero), *pval = its signed value.
__device__ inline void lu_pick(double a, int lane, int lo, int hi, int* piv, double* pval) {
  double v = (lane >= lo && lane < hi) ? fabs(a) : -1.0;
  int idx = lane;
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o, 64);
    const int oi = __shfl_xor(idx, o, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
  const double sv = __shfl(a, idx, 64);
  if (lane == 0) {
    *piv = v > 0.0 ? idx : -1;
    *pval = sv;
  }
}

// Right-looking elimination of columns [0, w) of the order-m matrix F in LDS
// (m <= 64; all entries, column-major, leading dimension ld), the pivot of
// column k being the largest magnitude among rows [k, w) (ties to the first
// row).  Rows are interchanged over all m columns.  On return F holds L
// (below the diagonal, unit diagonal implied) and U (on and above) in
// columns / rows [0, w) and the Schur complement in [w, m)^2; the order goes
// to qloc.  Returns the first column without a usable pivot, or -1.
// Two barriers per column: interchange + scaling, then the rank-1 update
// (lane = row, waves stride the columns), during which wave 0 picks the
// next pivot from the column it has just updated.
__device__ inline int lu_eliminate(double* F, int ld, int m, int w, int* qloc, int* piv,
                                   double* pval) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int t = tid; t < w; t += kThreads) qloc[t] = t;
  if (wave == 0) lu_pick(lane < m ? F[lane] : 0.0, lane, 0, w, piv, pval);
  __syncthreads();
  for (int k = 0; k < w; ++k) {
    const int p = *piv;
    if (p < 0) return k;
    const double pv = *pval;
    if (p != k) {
      for (int t = tid; t < m; t += kThreads)
        if (t != k) {
          const double a = F[k + t * ld];
          F[k + t * ld] = F[p + t * ld];
          F[p + t * ld] = a;
        }
      if (tid == 0) {
        const int t = qloc[k];
        qloc[k] = qloc[p];
        qloc[p] = t;
      }
    }
    // column k: the pivot moves to row k, the old diagonal to row p
    for (int i = k + 1 + tid; i < m; i += kThreads) {
      if (i == p) {
        const double a = F[k + k * ld];
        F[k + k * ld] = pv;
        F[p + k * ld] = a / pv;
      } else {
        F[i + k * ld] = F[i + k * ld] / pv;
      }
    }
    __syncthreads();
    if (lane > k && lane < m) {
      const double l = F[lane + k * ld];
      for (int j = k + 1 + wave; j < m; j += kThreads / 64) F[lane + j * ld] -= l * F[k + j * ld];
    }
    if (wave == 0 && k + 1 < w)
      lu_pick((lane > k && lane < m) ? F[lane + (k + 1) * ld] : 0.0, lane, k + 1, w, piv, pval);
    __syncthreads();
  }
  return -1;
}

static_assert(kSmallMax <= 64 && kPanel <= 64, "lu_eliminate maps the rows to one wave's lanes");

// Small fronts (m <= kSmallMax), LU: both halves assembled into one full
// matrix in LDS, the w pivot columns eliminated, L and U^T panels and both
// update-matrix halves written out.
__global__ __launch_bounds__(kThreads) void k_small_lu(DevSym S, DevNum<double> N,
                                                       DevNum<double> Nt, int32_t* qout,
                                                       const int32_t* list) {
  __shared__ double F[kSmallMax * kSmallMax];
  __shared__ int qloc[kSmallMax];
  __shared__ int piv;
  __shared__ double pval;
  const int s = list[blockIdx.x];
  const int tid = threadIdx.x;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ld = S.ldL[s];
  for (int t = tid; t < ld * m; t += kThreads) F[t] = 0.0;
  __syncthreads();
  {
    const int64_t q0 = S.acol_ptr[f], q1 = S.acol_ptr[f + w];
    for (int64_t q = q0 + tid; q < q1; q += kThreads) {
      const int pos = S.a_pos[q];
      const int c = pos / ld, i = pos - c * ld;  // front row i >= column c
      F[pos] = N.avals[q];
      if (i != c) F[c + i * ld] = Nt.avals[q];
    }
  }
  __syncthreads();
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int c = S.child_list[q];
    const int wc = S.sptr[c + 1] - S.sptr[c], rc = S.front_m[c] - wc;
    const double* Uc = N.U + S.U_off[c];
    const double* Vc = Nt.U + S.U_off[c];
    const int ldc = S.ldU[c];
    const int32_t* rm = S.rmap + S.rows_ptr[c] + wc;
    for (int t = tid; t < rc * rc; t += kThreads) {
      const int jj = t / rc, ii = t - jj * rc;
      if (ii >= jj) F[rm[ii] + rm[jj] * ld] += Uc[ii + (int64_t)jj * ldc];
      if (ii > jj) F[rm[jj] + rm[ii] * ld] += Vc[ii + (int64_t)jj * ldc];
    }
    __syncthreads();
  }
  const int bad = lu_eliminate(F, ld, m, w, qloc, &piv, &pval);
  if (bad >= 0) {
    if (tid == 0) atomicMin(N.fail, f + bad);
    return;
  }
  for (int c = tid; c < w; c += kThreads) qout[f + c] = f + qloc[c];
  double* Lp = N.L + S.L_off[s];
  double* Tp = Nt.L + S.L_off[s];
  for (int t = tid; t < ld * w; t += kThreads) {
    const int c = t / ld, i = t - c * ld;
    Lp[t] = i > c ? F[t] : (i == c ? 1.0 : 0.0);
    Tp[t] = (i >= c && i < m) ? F[c + i * ld] : 0.0;
  }
  if (r > 0) {
    double* Us = N.U + S.U_off[s];
    double* Vs = Nt.U + S.U_off[s];
    const int ldu = S.ldU[s];
    for (int t = tid; t < ldu * r; t += kThreads) {
      const int jj = t / ldu, ii = t - jj * ldu;
      Us[t] = ii < r ? F[(w + ii) + (w + jj) * ld] : 0.0;
      Vs[t] = ii < r ? F[(w + jj) + (w + ii) * ld] : 0.0;
    }
  }
}

// Large fronts, LU step 1: diagonal block [k, k + kb) of front s (already
// updated by the blocks before it; its lower part from the L half, its upper
// part from the U^T half) factored with row interchanges inside the block;
// the interchanges applied to the block's rows of L's earlier columns;
// W = L_kk^{-1} (unit lower) and V = (U_kk^T)^{-1} (lower) kept for the
// panels and the solves.  The block's rows of U in later columns are
// permuted by the panel step (it reads them in pivot order).
__global__ __launch_bounds__(kThreads) void k_diag_lu(DevSym S, DevNum<double> N,
                                                      DevNum<double> Nt, int32_t* qout,
                                                      const PanelItem* items, double* winv,
                                                      double* vinv) {
  __shared__ double F[kPanel * kDiagLd];
  __shared__ double Xs[2 * kPanel * kDiagLd];  // W, then V, row-major by r
  __shared__ int qloc[kPanel];
  __shared__ int piv;
  __shared__ double pval;
  const PanelItem it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = it.s, k = it.k, kb = it.kb;
  const int f = S.sptr[s], ld = S.ldL[s];
  double* Lp = N.L + S.L_off[s];
  double* Tp = Nt.L + S.L_off[s];
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    double v = 0.0;
    if (r < kb && c < kb)
      v = r >= c ? Lp[(k + r) + (int64_t)(k + c) * ld] : Tp[(k + c) + (int64_t)(k + r) * ld];
    F[c * kDiagLd + r] = v;
  }
  __syncthreads();
  const int bad = lu_eliminate(F, kDiagLd, kb, kb, qloc, &piv, &pval);
  if (bad >= 0) {
    if (tid == 0) atomicMin(N.fail, f + k + bad);
    return;
  }
  for (int c = tid; c < kb; c += kThreads) qout[f + k + c] = f + k + qloc[c];
  for (int t = tid; t < kb * kb; t += kThreads) {
    const int c = t / kb, r = t - c * kb;
    if (r >= c) {
      Lp[(k + r) + (int64_t)(k + c) * ld] = r > c ? F[c * kDiagLd + r] : 1.0;
      Tp[(k + r) + (int64_t)(k + c) * ld] = F[r * kDiagLd + c];  // U^T(r, c) = U(c, r)
    }
  }
  // (the block's rows of L's earlier columns are permuted by k_lu_rowperm
  // once the factorization is done: nothing reads them before)
  // W column c (wave 0, lane c) and V column c (wave 1, lane c) by forward
  // substitution into LDS (U^T_kk(r, j) = F(j, r)), then written out
  if (wave < 2 && lane < kb) {
    const int c = lane;
    double* X = Xs + wave * kPanel * kDiagLd;  // X[r * kDiagLd + c]
    for (int r = 0; r < kb; ++r) {
      double v = r == c ? 1.0 : 0.0;
      if (wave == 0) {
        if (r > c)
          for (int j = c; j < r; ++j) v -= F[j * kDiagLd + r] * X[j * kDiagLd + c];
      } else if (r >= c) {
        for (int j = c; j < r; ++j) v -= F[r * kDiagLd + j] * X[j * kDiagLd + c];
        v = v / F[r * kDiagLd + r];
      }
      X[r * kDiagLd + c] = r < c ? 0.0 : v;
    }
  }
  __syncthreads();
  double* Wout = winv + S.woff[it.wblk];
  double* Vout = vinv + S.woff[it.wblk];
  for (int t = tid; t < kb * kb; t += kThreads) {
    const int c = t / kb, r = t - c * kb;
    Wout[t] = Xs[r * kDiagLd + c];
    Vout[t] = Xs[kPanel * kDiagLd + r * kDiagLd + c];
  }
}

// After the LU factorization: the interchanges of every diagonal block
// applied to its rows of L's earlier columns.  One workgroup per diagonal
// block (s, k, kb); wave v handles the block's columns k + v, k + v + 4, ...
// and, for each, the later blocks of the front, four at a time (their rows
// move only within their block: new row kk + r <- old row q[f + kk + r] - f).
__global__ __launch_bounds__(kThreads) void k_lu_rowperm(DevSym S, DevNum<double> N,
                                                         const int32_t* q,
                                                         const PanelItem* items) {
  const PanelItem it = items[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s = it.s, f = S.sptr[s], w = S.sptr[s + 1] - f, ld = S.ldL[s];
  double* Lp = N.L + S.L_off[s];
  const int first = it.k + kPanel;  // the blocks after this one
  for (int p = it.k + wave; p < it.k + it.kb; p += kThreads / 64) {
    double* lc = Lp + (int64_t)p * ld;
    for (int kk = first; kk < w; kk += 4 * kPanel) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = kk + u * kPanel + lane;
        v[u] = row < w ? lc[q[f + row] - f] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = kk + u * kPanel + lane;
        if (row < w) lc[row] = v[u];
      }
    }
  }
}

// Large fronts, LU step 2: 64 rows below the diagonal block, on the matrix
// cores.  blockIdx.y = 0: L21 = F21 U_kk^{-1} = B V^T with B the rows' L-half
// entries; blockIdx.y = 1: U12^T = (Q F12)^T L_kk^{-T} = B W^T with B the
// rows' U^T-half entries in the block's columns taken in pivot order.  The
// result replaces the block's columns of the same rows.
__global__ __launch_bounds__(kThreads) void k_panel_lu(DevSym S, DevNum<double> N,
                                                       DevNum<double> Nt, const int32_t* q,
                                                       const PanelItem* items,
                                                       const double* winv, const double* vinv) {
  constexpr int PAD = 4;
  __shared__ double Bs[kPanel][kPanel + PAD];  // Bs[c][r] = B[r][c]
  __shared__ double Ws[kPanel][kPanel + PAD];  // Ws[c'][c] = M[c][c']
  const PanelItem it = items[blockIdx.x];
  const bool upper = blockIdx.y == 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = it.s, k = it.k, kb = it.kb;
  const int f = S.sptr[s], m = S.front_m[s], ld = S.ldL[s];
  double* Pp = (upper ? Nt.L : N.L) + S.L_off[s];
  const double* Min = (upper ? winv : vinv) + S.woff[it.wblk];
  const int r0 = k + kb + it.chunk * kPanel;
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    Ws[c][r] = (r < kb && c < kb) ? Min[c * kb + r] : 0.0;
    const int row = r0 + r;
    const int src = c < kb ? (upper ? q[f + k + c] - f : k + c) : 0;
    Bs[c][r] = (row < m && c < kb) ? Pp[row + (int64_t)src * ld] : 0.0;
  }
  __syncthreads();
  typedef Vec4<double>::type V4;
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
  const int wr = wave >> 1, wc = wave & 1;
#pragma unroll
  for (int ks = 0; ks < kPanel / 4; ++ks) {
    const int kk = ks * 4 + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = Bs[kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = Ws[kk][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr * 32 + a * 16 + (lane & 15);
        const int c = wc * 32 + b * 16 + mfma_row<double>(lane, v);
        Bs[c][r] = acc[a][b][v];
      }
  __syncthreads();
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    const int row = r0 + r;
    if (row < m && c < kb) Pp[row + (int64_t)(k + c) * ld] = Bs[c][r];
  }
}

// ---------------------------------------------------------------------------
// Update on the matrix cores: C[M x N] -= A[M x K] * A[0:N, :]^T for the
// elements with row >= col.  One TT x TT output tile per workgroup, four
// waves of (TT/2) x (TT/2) built from 16x16x4 MFMA blocks, K staged through
// double-buffered LDS 16 at a time with the next stage prefetched into
// registers while the current one is multiplied.  The MFMA computes the
// transposed tile so that a lane's outputs run down a column of the
// column-major C (coalesced read-modify-write).
// With Bsrc (the L D panels of an LDL^T factorization, laid out like L) the
// second operand is read from there: C -= A * B[0:N, :]^T.
// A paired launch (gridDim.y = 2) runs the same tiles a second time on
// (N2, Bsrc2): the two halves of an LU front.
template <typename T, int TT>
__global__ __launch_bounds__(kThreads) void k_gemm(DevNum<T> N, const GemmProb* probs,
                                                   const GemmTile* tiles, const T* Bsrc,
                                                   DevNum<T> N2, const T* Bsrc2) {
  if (blockIdx.y != 0) {
    N = N2;
    Bsrc = Bsrc2;
  }
  constexpr int KT = 16, PAD = 4;
  constexpr int BL = TT / 32;               // 16x16 blocks per wave dimension
  constexpr int LPT = TT * KT / kThreads;   // elements per thread per stage and operand
  constexpr int RSTEP = kThreads / TT;      // k rows covered per load round
  __shared__ T As[2][KT][TT + PAD];
  __shared__ T Bs[2][KT][TT + PAD];
  const GemmTile tl = tiles[blockIdx.x];
  const GemmProb g = probs[tl.prob];
  const T* A = N.L + g.a_off;
  T* C = (g.c_in_u ? N.U : N.L) + g.c_off;
  const int i0 = tl.ti * TT, j0 = tl.tj * TT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  typedef typename Vec4<T>::type V4;
  V4 acc[BL][BL];
#pragma unroll
  for (int a = 0; a < BL; ++a)
#pragma unroll
    for (int b = 0; b < BL; ++b) acc[a][b] = V4{0, 0, 0, 0};
  const int lrow = tid % TT, lk = tid / TT;
  const bool arow_ok = i0 + lrow < g.M, brow_ok = j0 + lrow < g.N;
  const T* pa = A + (i0 + lrow);
  const T* pb = (Bsrc ? Bsrc + g.a_off : A) + (j0 + lrow);
  T ra[LPT], rb[LPT];
  auto load_stage = [&](int k0) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      const int kg = k0 + lk + RSTEP * u;
      const bool kok = kg < g.K;
      ra[u] = (arow_ok && kok) ? pa[(int64_t)kg * g.lda] : T(0);
      rb[u] = (brow_ok && kok) ? pb[(int64_t)kg * g.lda] : T(0);
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int u = 0; u < LPT; ++u) {
      As[buf][lk + RSTEP * u][lrow] = ra[u];
      Bs[buf][lk + RSTEP * u][lrow] = rb[u];
    }
  };
  const int nstage = (g.K + KT - 1) / KT;
  load_stage(0);
  store_stage(0);
  __syncthreads();
  for (int st = 0; st < nstage; ++st) {
    const int buf = st & 1;
    if (st + 1 < nstage) load_stage((st + 1) * KT);
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      T av[BL], bv[BL];
#pragma unroll
      for (int a = 0; a < BL; ++a) av[a] = As[buf][kr][wr * (TT / 2) + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < BL; ++b) bv[b] = Bs[buf][kr][wc * (TT / 2) + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
    }
    if (st + 1 < nstage) store_stage(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < BL; ++a)
#pragma unroll
    for (int b = 0; b < BL; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * (TT / 2) + a * 16 + (lane & 15);
        const int j = j0 + wc * (TT / 2) + b * 16 + mfma_row<T>(lane, v);
        if (i < g.M && j < g.N && i >= j) {
          T* p = C + i + (int64_t)j * g.ldc;
          *p = *p - acc[a][b][v];
        }
      }
}

// ---------------------------------------------------------------------------
// Solve input and output: y (row-major, NR values per row) = P b, scaled by
// the Jacobi factors on the FP32 path; x = P^T y (or x += P^T y).
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_permute_in(DevSym S, const double* b, int64_t ldb,
                                                         T* y, int64_t nrhs,
                                                         const double* scale) {
  // thread per original row: coalesced reads of each column of b, one whole
  // row of y (its own cache line) written per thread
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= S.n) return;
  const int64_t i = S.pinv[j];
  const double d = scale ? scale[i] : 1.0;
#pragma unroll
  for (int c = 0; c < NR; ++c) y[i * kRowLd<T> + c] = c < nrhs ? (T)(b[j + c * ldb] * d) : T(0);
}

template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_permute_out(DevSym S, const T* y, double* x,
                                                          int64_t ldx, int64_t nrhs,
                                                          const double* scale, int accumulate) {
  // thread per original row: one row of y read, coalesced writes of each
  // column of x
  const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (j >= S.n) return;
  const int64_t i = S.pinv[j];
  const double d = scale ? scale[i] : 1.0;
  for (int64_t c = 0; c < nrhs; ++c) {
    const double v = (double)y[i * kRowLd<T> + c] * d;
    if (accumulate)
      x[j + c * ldx] += v;
    else
      x[j + c * ldx] = v;
  }
}

// Cross-workgroup ordering at agent scope.  The L2 caches of the XCDs are
// not coherent with each other: a producer writes its L2 back before
// raising a flag, a consumer invalidates its caches after seeing one.  The
// sequences are written out so that the wait after the writeback (or the
// invalidate) is always there; the compiler drops that wait when the wave
// has no stores of its own pending, and the flag could then overtake the
// writeback.
__device__ inline void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ inline void release_agent() {
  asm volatile("buffer_wbl2 sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
}
__device__ inline void acquire_agent() {
  asm volatile("s_waitcnt vmcnt(0)\n\tbuffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
}

// Stores of the front kernel's results (factor tiles, inverses, update
// tiles, pre-accumulations): agent-scope relaxed atomic stores, which write
// through to memory, so that a publishing workgroup's L2 writeback has little
// dirty data to flush.
template <typename T>
__device__ __forceinline__ void st_out(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup barrier after which thread 0 publishes the workgroup's global
// stores: every wave first waits until its stores have reached its L2, so
// the one writeback that thread 0 issues after the barrier covers them all.
__device__ inline void publish_barrier() {
  wait_vm();
  __syncthreads();
}

// Stores of this workgroup visible to its own later loads: every wave waits
// for its stores, then (after the barrier) drops its stale L1 lines.
__device__ inline void local_publish() {
  wait_vm();
  __syncthreads();
  asm volatile("buffer_inv sc0\n\ts_waitcnt vmcnt(0)" ::: "memory");
}

__device__ inline void set_flag(int32_t* flag, int32_t value) {
  release_agent();
  __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait for *flag >= value (acquire).  A dependency of the dataflow
// factorization is satisfied within one level's run time, far below the
// bound; on timeout the hang flag is raised (the host reports it as an
// error) and every other wait of the launch gives up as soon as it sees the
// flag, so the launch drains.
constexpr int kFlowSpinLimit = 1 << 21;

// Relaxed polling only: the caller issues one acquire fence after its last
// wait, then a workgroup barrier hands the ordering to the other threads.
__device__ inline void wait_at_least(const int32_t* flag, int32_t value, int32_t* hang) {
  int spins = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < value) {
    __builtin_amdgcn_s_sleep(1);
    ++spins;
    if ((spins & 255) == 0 && __hip_atomic_load(hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      break;
    if (spins > kFlowSpinLimit) {
      __hip_atomic_store(hang, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
}

__device__ inline bool flag_set(const int32_t* flag) {
  return __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Update-matrix block task (kind 5): the kUBlock x kUBlock block (tk.t, tk.j)
// of U_s loses sum_p L(a rows, p) L(b rows, p)^T over the pivot blocks
// [p0, p1), formed on the matrix cores.  Both operands are staged through
// double-buffered LDS 16 columns at a time (the next stage prefetched into
// registers while the current one is multiplied), and each wave owns a 64 x 64
// quadrant, so a staged byte feeds twice the products it feeds in a 64 x 64
// tile.  Per output entry the products are added in the same column order as
// in a 64 x 64 tile.  The block's ranges are applied in order (counter ui).
//
// With local set the block belongs to a whole-front task whose own earlier
// steps wrote the operands: nothing is awaited or published.
template <typename T>
__device__ __forceinline__ void front_ublock(const DevSym& S, const DevNum<T>& N, const FrontTask& tk,
                                             T* lds, const int32_t* tile_done, int32_t* ucount,
                                             int32_t* hang, int* s_ready, bool local) {
  constexpr int UB = kUBlock, UK = 16, PAD = 4, QB = UB / 2 / 16;  // 16 x 16 tiles per quadrant side
  constexpr int RS = kThreads / UB;          // k rows covered per load round
  constexpr int SL = UB * UK / kThreads;     // staged elements per thread and operand
  typedef typename Vec4<T>::type V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int s = tk.s;
  const int w = S.sptr[s + 1] - S.sptr[s], m = S.front_m[s], ld = S.ldL[s], wb = S.wbase[s];
  const T* Lp = N.L + S.L_off[s];
  T* Cu = N.U + S.U_off[s];
  const int ldc = S.ldU[s];
  const int a0 = w + tk.t * UB, b0 = w + tk.j * UB;  // front rows of the block's rows / columns
  const int arows = min(UB, m - a0), bcols = min(UB, m - b0);
  const int kstart = tk.p0 * kPanel, K = min(w, tk.p1 * kPanel);
  // the upper right quadrant of a diagonal block lies above the diagonal
  const bool idle = tk.t == tk.j && wr == 0 && wc == 1;
  V4 acc[QB][QB];
#pragma unroll
  for (int a = 0; a < QB; ++a)
#pragma unroll
    for (int b = 0; b < QB; ++b) acc[a][b] = V4{0, 0, 0, 0};
  T* As = lds;  // [2][UK][UB + PAD]: As[buf][k][row]
  T* Bs = lds + 2 * UK * (UB + PAD);
  const int lrow = tid % UB, lk = tid / UB;
  const bool aok = lrow < arows, bok = lrow < bcols;
  const T* pa = Lp + a0 + lrow;
  const T* pb = Lp + b0 + lrow;
  T ra[SL], rb[SL];
  // Pivot blocks [0, ready) are known complete (see the front kernel).
  int ready = kstart / kPanel;
  const int nblk = (K + kPanel - 1) / kPanel;
  auto rows_done = [&](int p, int r0, int nr, bool wait) {
    const int32_t* fl = tile_done + S.tbase[wb + p];
    const int t1 = front_row_tile(w, p, r0 + nr - 1);
    for (int t = front_row_tile(w, p, r0); t <= t1; ++t) {
      if (wait)
        wait_at_least(fl + t, 1, hang);
      else if (!flag_set(fl + t))
        return false;
    }
    return true;
  };
  auto block_done = [&](int p, bool wait) {
    return rows_done(p, a0, arows, wait) && rows_done(p, b0, bcols, wait);
  };
  auto load_stage = [&](int st) {
    const int k0 = kstart + st * UK;
    if (!local && k0 % kPanel == 0 && k0 / kPanel >= ready) {
      if (tid == 0) {
        int q = k0 / kPanel;
        block_done(q, true);
        ++q;
        while (q < nblk && block_done(q, false)) ++q;
        acquire_agent();
        *s_ready = q;
      }
      __syncthreads();
      ready = *s_ready;
    }
#pragma unroll
    for (int u = 0; u < SL; ++u) {
      const int kg = k0 + lk + RS * u;
      const bool kok = kg < K;
      ra[u] = *((aok && kok) ? pa + (int64_t)kg * ld : Lp);
      rb[u] = *((bok && kok) ? pb + (int64_t)kg * ld : Lp);
    }
  };
  // masked-off values become zero only here, so that the loads of the
  // next stage stay in flight while the current one is multiplied
  auto store_stage = [&](int buf, int st) {
    const int k0 = kstart + st * UK;
#pragma unroll
    for (int u = 0; u < SL; ++u) {
      const bool kok = k0 + lk + RS * u < K;
      As[(buf * UK + lk + RS * u) * (UB + PAD) + lrow] = (aok && kok) ? ra[u] : T(0);
      Bs[(buf * UK + lk + RS * u) * (UB + PAD) + lrow] = (bok && kok) ? rb[u] : T(0);
    }
  };
  const int nstage = (K - kstart + UK - 1) / UK;
  if (nstage > 0) {
    load_stage(0);
    store_stage(0, 0);
    __syncthreads();
  }
  for (int st = 0; st < nstage; ++st) {
    const int buf = st & 1;
    if (st + 1 < nstage) load_stage(st + 1);
    if (!idle) {
#pragma unroll
      for (int ks = 0; ks < UK / 4; ++ks) {
        const int kr = buf * UK + ks * 4 + (lane >> 4);
        T av[QB], bv[QB];
#pragma unroll
        for (int a = 0; a < QB; ++a) av[a] = As[kr * (UB + PAD) + wr * (UB / 2) + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < QB; ++b) bv[b] = Bs[kr * (UB + PAD) + wc * (UB / 2) + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < QB; ++a)
#pragma unroll
          for (int b = 0; b < QB; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
      }
    }
    if (st + 1 < nstage) store_stage(buf ^ 1, st + 1);
    __syncthreads();
  }
  if (tk.rk > 0) {
    if (tid == 0) {
      wait_at_least(ucount + tk.ui, tk.rk, hang);
      acquire_agent();
    }
    __syncthreads();
  }
  // U <- U - acc over the block's lower part, one row of 16 x 16 tiles at a
  // time; masked-off entries read the block's first entry (the loads of a
  // row issue before their first use)
  const int gi0 = tk.t * UB, gj0 = tk.j * UB;
#pragma unroll
  for (int a = 0; a < QB; ++a) {
    const int i = wr * (UB / 2) + a * 16 + (lane & 15);
    T f[QB][4];
#pragma unroll
    for (int b = 0; b < QB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = wc * (UB / 2) + b * 16 + mfma_row<T>(lane, v);
        const bool ok = i < arows && jj < bcols && gi0 + i >= gj0 + jj;
        f[b][v] = *(ok ? Cu + (gi0 + i) + (int64_t)(gj0 + jj) * ldc : Cu);
      }
#pragma unroll
    for (int b = 0; b < QB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = wc * (UB / 2) + b * 16 + mfma_row<T>(lane, v);
        if (i < arows && jj < bcols && gi0 + i >= gj0 + jj)
          st_out(&Cu[(gi0 + i) + (int64_t)(gj0 + jj) * ldc], f[b][v] - acc[a][b][v]);
      }
  }
  if (tk.p1 * kPanel < w) {  // a later range of this block follows
    publish_barrier();
    if (tid == 0) set_flag(ucount + tk.ui, tk.rk + 1);
  }
}

// ---------------------------------------------------------------------------
// Dataflow factorization of the large fronts of one level (one launch).
// Left-looking over 64-column pivot blocks: the task of pivot block j, row
// tile t accumulates L(rows, p) L(block j rows, p)^T over the completed
// blocks p < j in registers on the matrix cores, subtracts it from the
// assembled front, then either factors the diagonal block (t = 0: Cholesky
// and inverse W_j, published through a ready flag) or solves its rows
// against it (X = C W_j^T on the matrix cores).  Update-matrix tiles
// accumulate over all pivot blocks of their front, each as soon as it is
// complete, and subtract the sum from the assembled U.  Every row tile has a
// completion flag; a consumer of rows [r0, r1) of pivot block p waits for
// the (at most three) tiles of p that hold them, so the next diagonal block
// waits only for the one tile that holds its rows, not for a whole column.
//
// Workgroups take tasks from a ticket counter in the plan's order, in which
// every task depends only on tasks with smaller tickets; those belong to
// workgroups that already run, so the waits end (and are bounded anyway).
template <typename T>
__global__ __launch_bounds__(kThreads, sizeof(T) == 8 ? 2 : 3) void k_front(DevSym S, DevNum<T> N, T* winv,
                                                    const FrontTask* tasks, int count,
                                                    int32_t* tile_done, int32_t* pd_done,
                                                    int32_t* ucount, int32_t* counter,
                                                    int32_t* hang) {
  constexpr int TT = kPanel, PAD = 4, BL = 2;
  constexpr int RSTEP = kThreads / TT;     // k rows covered per load round
  constexpr int STAGE = TT * (TT + PAD);   // one operand, double-buffered half blocks
  constexpr int POST = 2 * kPanel * kDiagLd + 3 * kSub * kSub;
  constexpr int UBLDS = 4 * 16 * (kUBlock + PAD);  // update-matrix block stages
  constexpr int LDS0 = POST > 2 * STAGE ? POST : 2 * STAGE;
  constexpr int LDS = LDS0 > UBLDS ? LDS0 : UBLDS;
  typedef typename Vec4<T>::type V4;
  __shared__ T lds[LDS];
  __shared__ int s_ticket, s_ready;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  if (tid == 0) s_ticket = atomicAdd(counter, 1);
  __syncthreads();
  const int ticket = s_ticket;
  if (ticket >= count) return;
  const FrontTask tk = tasks[ticket];
  // Update-matrix blocks run after the other steps, from one call site (one
  // inlined copy): the task's own block (kind 5, or kind 7 in a launch of
  // its own, which awaits nothing) or, for a whole-front task of an update
  // matrix of more than 64 rows, all of them.
  bool ublocks = tk.kind == 5 || tk.kind == 7;
  if (!ublocks) {
  const int s = tk.s;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], ld = S.ldL[s];
  const int wb = S.wbase[s];
  T* Lp = N.L + S.L_off[s];
  // One task step.  mode 0: row tile tt of pivot block tj (tt = 0: the
  // diagonal block with row tile 1); mode 1: update-matrix tile (tt, tj);
  // mode 3: pre-accumulation of the diagonal block tj and its row tile 1
  // (no factorization).  Pivot blocks [kstart / 64, K / 64) are applied.
  auto step = [&](int mode, int tj, int tt, int kstart, int K) {
  // Lane-dependent index arithmetic is redone in every step rather than
  // kept in registers across the task loop (it would push the kernel past
  // its register budget into scratch spills).
  int lane = tid & 63;
  asm volatile("" : "+v"(lane));
  const bool utile = mode == 1;
  const bool pre = mode == 3;
  // whole-front or whole-panel task: every operand comes from this
  // workgroup's own earlier steps, so there are no flags to wait for or
  // raise between them
  const bool solo = tk.kind == 4 || tk.kind == 6;
  const bool diag = (mode == 0 && tt == 0) || pre;
  const int c0 = tj * TT;
  const int kb = utile ? TT : min(TT, w - c0);
  // Output rows [a0, a0 + arows) against operand rows [b0, b0 + bcols); a
  // diagonal task also produces row tile 1 (rows [c0 + kb, ...)) when it
  // exists, so the next diagonal block does not wait for another workgroup.
  int a0, arows, b0, bcols;
  if (utile) {
    a0 = w + tt * TT;
    b0 = w + tj * TT;
    arows = min(TT, m - a0);
    bcols = min(TT, m - b0);
  } else {
    b0 = c0;
    bcols = kb;
    a0 = diag ? c0 + kb : c0 + kb + (tt - 1) * TT;  // diagonal: row tile 1 (may be empty)
    arows = min(TT, m - a0);
  }
  const bool fuse1 = diag && arows > 0;
  T* Lc0 = Lp + (int64_t)c0 * ld;  // pivot block j's columns (32-bit offsets from here)
  T* Cu = N.U + (utile ? S.U_off[s] : 0);
  const int ldc = utile ? S.ldU[s] : 0;

  // Output element (a, b, v) of this thread: row i(a) of the tile, column j(b, v).
  auto oi = [&](int a) { return wr * (TT / 2) + a * 16 + (lane & 15); };
  auto oj = [&](int b, int v) { return wc * (TT / 2) + b * 16 + mfma_row<T>(lane, v); };
  V4 acc[BL][BL], dacc[BL][BL];
#pragma unroll
  for (int a = 0; a < BL; ++a)
#pragma unroll
    for (int b = 0; b < BL; ++b) acc[a][b] = dacc[a][b] = V4{0, 0, 0, 0};
  // Assembled front values F of the outputs are folded into the
  // accumulators after the products: acc <- F - acc for rows a0.. (or the U
  // tile), dacc <- F - dacc for the diagonal block.  Branch-free:
  // masked-off elements read the front's first entry and give zero.
  const T* fbase = utile ? Cu + tt * TT + (int64_t)(tj * TT) * ldc : Lp + a0 + (int64_t)c0 * ld;
  const int fld = utile ? ldc : ld;
  const int fcols = utile ? bcols : kb;
  const int tri_off = utile ? (tt - tj) * TT : INT_MAX / 2;  // U: keep gi >= gj
  const T* dbase = Lp + c0 + (int64_t)c0 * ld;
  auto fold_acc = [&]() {
    if constexpr (sizeof(T) == 8) {
      // FP64: all loads in flight before the first use (on the chain's
      // critical path); the FP32 instance has no registers to spare for it
      T va[BL][BL][4];
#pragma unroll
      for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = oi(a), jj = oj(b, v);
            const bool ma = i < arows && jj < fcols && i + tri_off >= jj;
            va[a][b][v] = *(ma ? fbase + (i + jj * fld) : (const T*)Lp);
          }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = oi(a), jj = oj(b, v);
            const bool ma = i < arows && jj < fcols && i + tri_off >= jj;
            acc[a][b][v] = (ma ? T(1) : T(0)) * (va[a][b][v] - acc[a][b][v]);
          }
      return;
    }
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = oi(a), jj = oj(b, v);
          // unconditional loads from a selected address (masked-off ones read
          // the front's first entry): the loads of one thread all issue
          // before the first use instead of one branch and wait each
          // (a multiplicative mask keeps the compiler from turning them
          // back into branches around each load)
          const bool ma = i < arows && jj < fcols && i + tri_off >= jj;
          const T va = *(ma ? fbase + (i + jj * fld) : (const T*)Lp);
          acc[a][b][v] = (ma ? T(1) : T(0)) * (va - acc[a][b][v]);
        }
  };
  auto fold_dacc = [&]() {
    // on the chain's critical path: all loads in flight before the first use
    T vd[BL][BL][4];
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = oi(a), jj = oj(b, v);
          const bool md = i < kb && jj < kb && i >= jj;
          vd[a][b][v] = *(md ? dbase + (i + jj * ld) : (const T*)Lp);
        }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = oi(a), jj = oj(b, v);
          const bool md = i < kb && jj < kb && i >= jj;
          dacc[a][b][v] = (md ? T(1) : T(0)) * (vd[a][b][v] - dacc[a][b][v]);
        }
  };
  auto fold_f = [&]() {
    fold_acc();
    if (diag) fold_dacc();
  };

  T* Cs = lds;                      // C tile, column-major, ld kDiagLd
  T* Ws = lds + kPanel * kDiagLd;   // W_j, column-major, ld kDiagLd
  T(*Tmp)[kSub * kSub] = reinterpret_cast<T(*)[kSub * kSub]>(lds + 2 * kPanel * kDiagLd);
  int32_t* done = tile_done + S.tbase[wb + tj];  // flags of pivot block j's row tiles

  // rows [a0, a0 + arows): X = C W_j^T with C in Cs and W_j in Ws; with
  // keep, X also replaces C in Cs (column-major, zero outside the tile)
  auto trsm_rows = [&](bool keep) {
    V4 x[BL][BL];
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b) x[a][b] = V4{0, 0, 0, 0};
#pragma unroll 4
    for (int ks = 0; ks < kPanel / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      T av[BL], bv[BL];
#pragma unroll
      for (int a = 0; a < BL; ++a) av[a] = Cs[kk * kDiagLd + wr * (TT / 2) + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < BL; ++b) bv[b] = Ws[kk * kDiagLd + wc * (TT / 2) + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b) x[a][b] = mfma16(bv[b], av[a], x[a][b]);
    }
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = oi(a), c = oj(b, v);
          if (r < arows && c < kb) st_out(&Lc0[(a0 + r) + c * ld], x[a][b][v]);
        }
    if (keep) {
      __syncthreads();
#pragma unroll
      for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = oi(a), c = oj(b, v);
            Cs[c * kDiagLd + r] = (r < arows && c < kb) ? x[a][b][v] : T(0);
          }
    }
  };
  // C = F - acc of the row tile into Cs (zero outside the tile)
  auto stage_rows = [&]() {
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) Cs[oj(b, v) * kDiagLd + oi(a)] = acc[a][b][v];
  };
  // diagonal block: F - Y Y^T into Cs (identity past kb, zero above the
  // diagonal), Cholesky and inverse, L_jj and W_j stored and published
  auto factor_diag = [&](bool publish) {
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = oi(a), c = oj(b, v);
          T val;
          if (r < kb && c < kb && r >= c)
            val = dacc[a][b][v];
          else
            val = (r == c && r >= kb) ? T(1) : T(0);
          Cs[c * kDiagLd + r] = val;
        }
    __syncthreads();
    diag_factor_inverse<T>(Cs, Ws, Tmp, kb, f + c0, N.fail);
    T* Wout = winv + S.woff[wb + tj];  // kb x kb, column-major
    if (kb == TT) {
      // full block: a column per wave and round, four rounds in flight
#pragma unroll 4
      for (int q = 0; q < TT / (kThreads / 64); ++q) {
        const int c = wave + q * (kThreads / 64);
        const T lv = Cs[c * kDiagLd + lane], wv = Ws[c * kDiagLd + lane];
        if (lane >= c) st_out(&Lc0[(c0 + lane) + c * ld], lv);
        st_out(&Wout[c * TT + lane], wv);
      }
    } else {
      for (int t = tid; t < kb * kb; t += kThreads) {
        const int c = t / kb, r = t - c * kb;
        if (r >= c) st_out(&Lc0[(c0 + r) + c * ld], Cs[c * kDiagLd + r]);
      }
      for (int t = tid; t < kb * kb; t += kThreads) {
        const int c = t / kb, r = t - c * kb;
        st_out(&Wout[t], Ws[c * kDiagLd + r]);
      }
    }
    if (publish) {
      publish_barrier();
      if (tid == 0) set_flag(done, 1);
    } else {
      __syncthreads();
    }
  };
  // out[a][b] += sum_k B(rb0 + row, k) A(ra0 + row, k) over columns k in
  // [k0, k1), both operands loaded from the front panel
  auto gemm_direct = [&](V4 (&out)[BL][BL], int ra0, int na, int rb0, int nbr, int k0, int k1) {
#pragma unroll 1
    for (int k4 = k0; k4 < k1; k4 += 16) {
      T av[4][BL], bv[4][BL];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k4 + 4 * u + (lane >> 4);
        const int kc = min(k, k1 - 1);
#pragma unroll
        for (int a = 0; a < BL; ++a) {
          const int r = wr * (TT / 2) + a * 16 + (lane & 15);
          const bool ok = k < k1 && r < na;
          av[u][a] = Lp[(ra0 + min(r, na - 1)) + (int64_t)kc * ld] * (ok ? T(1) : T(0));
        }
#pragma unroll
        for (int b = 0; b < BL; ++b) {
          const int r = wc * (TT / 2) + b * 16 + (lane & 15);
          const bool ok = k < k1 && r < nbr;
          bv[u][b] = Lp[(rb0 + min(r, nbr - 1)) + (int64_t)kc * ld] * (ok ? T(1) : T(0));
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int a = 0; a < BL; ++a)
#pragma unroll
          for (int b = 0; b < BL; ++b) out[a][b] = mfma16(bv[u][b], av[u][a], out[a][b]);
    }
  };

  if (mode == 0 && tk.kind == 2) {
    // Chain step: one pivot block (j - 1) to apply.  Its rows of block j
    // (row tile 1 of block j - 1) are this workgroup's previous result,
    // still in Cs; the product of its rows of row tile 1 of block j with
    // them was formed by the tasks of block j - 1 that own those rows (for a
    // full block j), into slot pt1 of block j or, with p0 = 1, subtracted
    // in place.  So the diagonal block is updated from LDS, factored, and
    // only then are those tasks awaited; both row tiles of block j are
    // published together at the end.
    if (K > kstart) {
#pragma unroll 4
      for (int ks = 0; ks < TT / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        T yv[BL], bv[BL];
#pragma unroll
        for (int a = 0; a < BL; ++a) yv[a] = Cs[kk * kDiagLd + wr * (TT / 2) + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < BL; ++b) bv[b] = Cs[kk * kDiagLd + wc * (TT / 2) + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < BL; ++a)
#pragma unroll
          for (int b = 0; b < BL; ++b) dacc[a][b] = mfma16(bv[b], yv[a], dacc[a][b]);
      }
      __syncthreads();
    }
    if (tj >= 2) {
      // the pre-accumulated part of the diagonal block and row tile 1: all
      // ranges of block j applied (tk.p1 blocks per range before [j-2, j-1))
      if (tid == 0) {
        wait_at_least(pd_done + wb + tj, (tj - 2 + tk.p1 - 1) / tk.p1 + 1, hang);
        acquire_agent();
      }
      __syncthreads();
    }
    fold_dacc();
    factor_diag(false);
    if (!fuse1) {
      if (tid == 0) set_flag(done, 1);
      return;
    }
    if (K > kstart) {
      if (tid == 0) {
        const int32_t* fl = tile_done + S.tbase[wb + tj - 1];
        const int t1 = front_row_tile(w, tj - 1, a0 + arows - 1);
        for (int t = front_row_tile(w, tj - 1, a0); t <= t1; ++t) wait_at_least(fl + t, 1, hang);
        acquire_agent();
      }
      __syncthreads();
      if (kb == TT && tk.p0 == 0) {
        const T* P1 = N.pt1 + (int64_t)S.pt1base[wb + tj] * (TT * TT);
#pragma unroll
        for (int a = 0; a < BL; ++a)
#pragma unroll
          for (int b = 0; b < BL; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = oi(a), c = oj(b, v);
              const bool ok = r < arows && c < kb;
              acc[a][b][v] = P1[ok ? r + c * TT : 0] * (ok ? T(1) : T(0));
            }
      } else if (kb < TT) {
        // last (partial) block: part of its row tile 1 lies in row tile 1
        // of block j - 1, which no other task owns; apply block j - 1 here
        gemm_direct(acc, a0, arows, b0, bcols, kstart, K);
      }
    }
    fold_acc();
    stage_rows();
    __syncthreads();
    trsm_rows(true);
    publish_barrier();
    if (tid == 0) {
      release_agent();
      __hip_atomic_store(done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(done + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }

  // acc = X Y^T over the completed pivot blocks (X: rows a0.., Y: rows b0..);
  // a diagonal task accumulates Y Y^T in dacc as well.  Half a pivot block
  // (32 columns of both operands) per stage through double-buffered LDS, the
  // next stage prefetched into registers while the current one is multiplied.
  {
    constexpr int KT = TT / 2;
    constexpr int SLPT = TT * KT / kThreads;  // staged elements per thread and operand
    T* As = lds;                  // [2][KT][TT + PAD]: As[buf][k][row]
    T* Bs = lds + 2 * KT * (TT + PAD);
    const int lrow = tid % TT, lk = tid / TT;
    const bool aok = lrow < arows, bok = lrow < bcols;
    const T* pa = Lp + a0 + lrow;
    const T* pb = Lp + b0 + lrow;
    T ra[SLPT], rb[SLPT];
    // Pivot blocks [0, ready) are known complete.  Before reading block p,
    // thread 0 waits for the row tiles of p that hold the operand rows, then
    // extends `ready` over the following blocks that are already complete,
    // and issues one acquire fence for all of them.
    int ready = kstart / TT;
    const int nblk = (K + TT - 1) / TT;
    auto rows_done = [&](int p, int r0, int nr, bool wait) {
      const int32_t* fl = tile_done + S.tbase[wb + p];
      const int t1 = front_row_tile(w, p, r0 + nr - 1);
      for (int t = front_row_tile(w, p, r0); t <= t1; ++t) {
        if (wait)
          wait_at_least(fl + t, 1, hang);
        else if (!flag_set(fl + t))
          return false;
      }
      return true;
    };
    auto block_done = [&](int p, bool wait) {
      return (arows <= 0 || rows_done(p, a0, arows, wait)) && rows_done(p, b0, bcols, wait);
    };
    auto load_stage = [&](int st) {
      const int k0 = kstart + st * KT;
      if (!solo && k0 % TT == 0 && k0 / TT >= ready) {
        if (tid == 0) {
          int q = k0 / TT;
          block_done(q, true);
          ++q;
          while (q < nblk && block_done(q, false)) ++q;
          acquire_agent();
          s_ready = q;
        }
        __syncthreads();
        ready = s_ready;
      }
#pragma unroll
      for (int u = 0; u < SLPT; ++u) {
        const int kg = k0 + lk + RSTEP * u;
        const bool kok = kg < K;
        ra[u] = *((aok && kok) ? pa + (int64_t)kg * ld : (const T*)Lp);
        rb[u] = *((bok && kok) ? pb + (int64_t)kg * ld : (const T*)Lp);
      }
    };
    // masked-off values become zero only here, so that the loads of the
    // next stage stay in flight while the current one is multiplied
    auto store_stage = [&](int buf, int st) {
      const int k0 = kstart + st * KT;
#pragma unroll
      for (int u = 0; u < SLPT; ++u) {
        const bool kok = k0 + lk + RSTEP * u < K;
        As[(buf * KT + lk + RSTEP * u) * (TT + PAD) + lrow] = (aok && kok) ? ra[u] : T(0);
        Bs[(buf * KT + lk + RSTEP * u) * (TT + PAD) + lrow] = (bok && kok) ? rb[u] : T(0);
      }
    };
    const int nstage = (K - kstart + KT - 1) / KT;
    if (nstage > 0) {
      load_stage(0);
      store_stage(0, 0);
      __syncthreads();
    }
    for (int st = 0; st < nstage; ++st) {
      const int buf = st & 1;
      if (st + 1 < nstage) load_stage(st + 1);
#pragma unroll 4
      for (int ks = 0; ks < KT / 4; ++ks) {
        const int kr = buf * KT + ks * 4 + (lane >> 4);
        T av[BL], bv[BL];
#pragma unroll
        for (int a = 0; a < BL; ++a) av[a] = As[kr * (TT + PAD) + wr * (TT / 2) + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < BL; ++b) bv[b] = Bs[kr * (TT + PAD) + wc * (TT / 2) + b * 16 + (lane & 15)];
        if (!diag || fuse1) {
#pragma unroll
          for (int a = 0; a < BL; ++a)
#pragma unroll
            for (int b = 0; b < BL; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
        }
        if (diag) {
          T yv[BL];
#pragma unroll
          for (int a = 0; a < BL; ++a) yv[a] = Bs[kr * (TT + PAD) + wr * (TT / 2) + a * 16 + (lane & 15)];
#pragma unroll
          for (int a = 0; a < BL; ++a)
#pragma unroll
            for (int b = 0; b < BL; ++b) dacc[a][b] = mfma16(bv[b], yv[a], dacc[a][b]);
        }
      }
      if (st + 1 < nstage) store_stage(buf ^ 1, st + 1);
      __syncthreads();
    }
  }
  if ((utile || pre) && tk.rk > 0) {
    // ranges of one update-matrix tile, or of one pre-accumulated diagonal
    // block, are applied in order
    if (tid == 0) {
      wait_at_least(utile ? ucount + tk.ui : pd_done + wb + tj, tk.rk, hang);
      acquire_agent();
    }
    __syncthreads();
  }
  fold_f();

  if (utile) {
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = oi(a), jj = oj(b, v);
          const int gi = tt * TT + i, gj = tj * TT + jj;
          if (i < arows && jj < bcols && gi >= gj) st_out(&Cu[gi + (int64_t)gj * ldc], acc[a][b][v]);
        }
    if (tk.p1 * TT < w) {  // a later range of this tile follows
      publish_barrier();
      if (tid == 0) set_flag(ucount + tk.ui, tk.rk + 1);
    }
    return;
  }

  if (pre) {
    // pre-accumulated diagonal block and row tile 1 go back in place; the
    // chain applies the last pivot block and factors
#pragma unroll
    for (int a = 0; a < BL; ++a)
#pragma unroll
      for (int b = 0; b < BL; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = oi(a), c = oj(b, v);
          if (r < kb && c < kb && r >= c) st_out(&Lc0[(c0 + r) + c * ld], dacc[a][b][v]);
          if (r < arows && c < kb) st_out(&Lc0[(a0 + r) + c * ld], acc[a][b][v]);
        }
    publish_barrier();
    if (tid == 0) set_flag(pd_done + wb + tj, tk.rk + 1);
    return;
  }
  if (diag) {
    factor_diag(!solo);
    if (!fuse1) return;
    // row tile 1 (still in registers) against the inverse in LDS
    stage_rows();
    __syncthreads();
    trsm_rows(false);
    if (solo) {
      local_publish();
    } else {
      publish_barrier();
      if (tid == 0) set_flag(done + 1, 1);
    }
    return;
  }
  // rows below the diagonal block: X = C W_j^T
  stage_rows();
  if (solo) {
    // W_j is still in LDS from the diagonal step
    __syncthreads();
    trsm_rows(false);
    local_publish();
    return;
  }
  if (tid == 0) {
    wait_at_least(done, 1, hang);
    acquire_agent();
  }
  __syncthreads();
  {
    const T* Win = winv + S.woff[wb + tj];  // Win[c * kb + r] = W[r][c]
    for (int t = tid; t < kPanel * kPanel; t += kThreads) {
      const int kk = t / kPanel, c = t - kk * kPanel;
      Ws[kk * kDiagLd + c] = (kk < kb && c < kb) ? Win[kk * kb + c] : T(0);  // W[c][kk]
    }
  }
  __syncthreads();
  trsm_rows(false);
  if (tk.p0 && c0 + kb + TT <= w) {
    // chain front: rows of this tile that are row tile 1 of block j + 1 also
    // get their product with row tile 1 of block j (the chain's result), for
    // the chain's step j + 1 (a full block j + 1; the last, partial one
    // applies block j itself)
    const int c1 = c0 + kb, kb1 = min(TT, w - c1);
    const int t1lo = c1 + kb1, t1hi = min(m, t1lo + TT);
    const int lo = max(a0, t1lo), hi = min(a0 + arows, t1hi);
    if (lo < hi) {
      if (tid == 0) {
        wait_at_least(done + 1, 1, hang);
        acquire_agent();
      }
      __syncthreads();
#pragma unroll
      for (int a = 0; a < BL; ++a)
#pragma unroll
        for (int b = 0; b < BL; ++b) acc[a][b] = V4{0, 0, 0, 0};
      gemm_direct(acc, a0, arows, c1, kb1, c0, c0 + kb);
      if (tk.p0 == 2) {
        // in place, after the pre-accumulation of block j + 1 (its ranges
        // have smaller tickets), so that the chain reads one value
        if (tj + 1 >= 2) {
          if (tid == 0) {
            wait_at_least(pd_done + wb + tj + 1, (tj + 1 - 2 + kPdRange - 1) / kPdRange + 1, hang);
            acquire_agent();
          }
          __syncthreads();
        }
#pragma unroll
        for (int a = 0; a < BL; ++a)
#pragma unroll
          for (int b = 0; b < BL; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = a0 + oi(a), c = oj(b, v);
              if (r >= lo && r < hi && c < kb1) {
                T* p = Lp + r + (int64_t)(c1 + c) * ld;
                st_out(p, *p - acc[a][b][v]);
              }
            }
      } else {
        // into block j + 1's slot
        T* P1 = N.pt1 + (int64_t)S.pt1base[wb + tj + 1] * (TT * TT);
#pragma unroll
        for (int a = 0; a < BL; ++a)
#pragma unroll
          for (int b = 0; b < BL; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = a0 + oi(a), c = oj(b, v);
              if (r >= lo && r < hi && c < kb1) st_out(&P1[(r - t1lo) + c * TT], acc[a][b][v]);
            }
      }
    }
  }
  publish_barrier();
  if (tid == 0) set_flag(done + tt, 1);
  };

  // Chain of the diagonal blocks of one front (kind 2): block j applies
  // only block j - 1 (the rest was pre-accumulated in place), factors, and
  // solves its row tile 1, which is block j + 1's last operand.  Other
  // kinds run one step.  (One call site keeps a single inlined copy.)
  // A whole-front task (kind 4, one pivot block) runs the diagonal step,
  // the steps of row tiles 2.. and then the update matrix: one 64 x 64
  // tile, or kUBlock x kUBlock blocks when it has more than 64 rows.  A
  // whole-panel task (kind 6) runs the same steps up to the update matrix
  // and then raises the flags of all its row tiles at once.
  const bool whole = tk.kind == 4 || tk.kind == 6;
  const int nrt = whole ? max(1, front_block_tiles(m, w, 0) - 1) : 0;
  const int nut = tk.kind == 4 && m - w <= TT ? (m - w + TT - 1) / TT : 0;
  const int nsteps = tk.kind == 2 ? (w + TT - 1) / TT : whole ? nrt + nut * (nut + 1) / 2 : 1;
  for (int it = 0; it < nsteps; ++it) {
    int mode = 0, tj = tk.j, tt = tk.t, kstart = 0, kend = tk.j * TT;
    if (whole) {
      if (it < nrt) {
        tj = 0;
        tt = it == 0 ? 0 : it + 1;
        kend = 0;
      } else {
        // update-matrix tile (a, b), a >= b, in row-major lower order
        const int u = it - nrt;
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= u) ++a;
        mode = 1;
        tt = a;
        tj = u - a * (a + 1) / 2;
        kend = w;
      }
    } else if (tk.kind == 2) {
      tj = it;
      tt = 0;
      kstart = it > 0 ? (it - 1) * TT : 0;
      kend = it * TT;
    } else if (tk.kind == 1) {
      mode = 1;
      kstart = tk.p0 * TT;
      kend = min(w, tk.p1 * TT);
    } else if (tk.kind == 3) {
      mode = 3;
      tt = 0;
      kstart = tk.p0 * TT;
      kend = tk.p1 * TT;
    }
    step(mode, tj, tt, kstart, kend);
  }
  if (tk.kind == 6) {
    publish_barrier();
    if (tid == 0) {
      release_agent();
      int32_t* done = tile_done + S.tbase[wb];
      const int nt = front_block_tiles(m, w, 0);
      for (int t = 0; t < nt; ++t) __hip_atomic_store(done + t, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  ublocks = tk.kind == 4 && m - w > TT;
  }
  if (!ublocks) return;
  // a whole-front task: blocks (a, b), a >= b, in row-major lower order, on
  // the row tiles its own steps stored (visible to it after local_publish)
  const bool whole = tk.kind == 4;
  const int r = S.front_m[tk.s] - (S.sptr[tk.s + 1] - S.sptr[tk.s]);
  const int nub = whole ? (r + kUBlock - 1) / kUBlock : 1;
  const int nblk = whole ? nub * (nub + 1) / 2 : 1;
  for (int q = 0; q < nblk; ++q) {
    FrontTask u = tk;
    if (whole) {
      int a = 0;
      while ((a + 1) * (a + 2) / 2 <= q) ++a;
      u = FrontTask{tk.s, q - a * (a + 1) / 2, a, 5, 0, 1, 0, 0};
    }
    front_ublock<T>(S, N, u, lds, tile_done, ucount, hang, &s_ready, tk.kind != 5);
  }
}

// ---------------------------------------------------------------------------
// Dataflow solves (forward L y = P b, backward L^T x = y; the paper's
// supernodal triangular solves with the inverted diagonal blocks of the
// factorization, ordered by dependencies instead of by levels).
//
// y holds P b and receives P x, row-major with NR values per row (NR = 1 or
// 16, columns past the caller's count are zero); the update vector u_s of a
// front (r_s rows of NR) sits at uvec + u_off[s] NR.  One launch per sweep:
// workgroups take tasks in the plan's ticket order, and a task waits only on
// tasks with smaller tickets (children before parents forward, parents
// before children backward, earlier blocks of its own front), so every wait
// ends; the waits are bounded all the same and raise the hang flag.
//
// Completion counters (zero when a solve starts): xcnt[s] forward diagonal
// blocks of s solved, in order; ucnt[s] forward L21 row blocks of s done (a
// wave-solved front counts one); bcnt[s] backward diagonal blocks of s
// solved, from the last (a wave-solved front counts one); pcnt[blk] backward
// partial products of diagonal block blk done.
struct SolveFlags {
  int32_t* xcnt;
  int32_t* ucnt;
  int32_t* bcnt;
  int32_t* pcnt;
  int32_t* ticket;
  int32_t* hang;
};

// Forward results of front c are complete when ucnt[c] reaches this.
__device__ inline int fwd_need(const DevSym& S, int c) {
  const int m = S.front_m[c], w = S.sptr[c + 1] - S.sptr[c];
  return m <= kSmallMax ? 1 : (m - w + kPanel - 1) / kPanel;
}
// Backward results of front p are complete when bcnt[p] reaches this.
__device__ inline int bwd_need(const DevSym& S, int p) {
  const int m = S.front_m[p], w = S.sptr[p + 1] - S.sptr[p];
  return m <= kSmallMax ? 1 : (w + kPanel - 1) / kPanel;
}

// One thread: relaxed polls until every child of s has its update vector.
__device__ inline void wait_children(const DevSym& S, int s, const int32_t* ucnt, int32_t* hang) {
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int c = S.child_list[q];
    wait_at_least(ucnt + c, fwd_need(S, c), hang);
  }
}

__device__ inline void add_release(int32_t* p) {
  release_agent();
  __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 waits until *cnt >= need and publishes the value it saw in
// s_ready[par] after one acquire fence; every thread returns that value.
// The two LDS slots alternate, so a slow reader of one wait never sees the
// next wait's write.
__device__ inline int wait_ready(const int32_t* cnt, int need, int32_t* hang, int* s_ready,
                                 int& par) {
  if (threadIdx.x == 0) {
    wait_at_least(cnt, need, hang);
    const int v = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    acquire_agent();
    s_ready[par] = v;
  }
  __syncthreads();
  const int v = s_ready[par];
  par ^= 1;
  return v;
}

// Forward solve of a front with m <= kSmallMax by one wave, lane = front
// row: gather the children's contributions, eliminate the w pivot columns
// with register broadcasts, write x (rows < w) to y and the rest to u_s.
template <typename T, int NR>
__device__ __forceinline__ void fwd_wave(const DevSym& S, const T* L, T* y, T* uvec, int s,
                                         const SolveFlags& F, int lane) {
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ldl = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  if (lane == 0) wait_children(S, s, F.ucnt, F.hang);
  acquire_agent();
  const int i = lane;
  const int ic = i < m ? i : m - 1;
  const int isrc = (S.lq && i < w) ? S.lq[f + i] - f : ic;  // LDL^T: row taken in pivot order
  const int64_t q = S.rows_ptr[s] + isrc;
  const int p0 = S.pull_ptr[q], p1 = i < m ? S.pull_ptr[q + 1] : p0;
  T z[NR];
  {
    const T* yr = y + (int64_t)(f + (i < w ? isrc : 0)) * kRowLd<T>;
    const T own = i < w ? T(1) : T(0);
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] = yr[c] * own;
  }
  for (int p = p0; p < p1; ++p) {
    const T* ur = uvec + (int64_t)S.pull_src[p] * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] += ur[c];
  }
#pragma unroll 2
  for (int k = 0; k < w; ++k) {
    const T inv = T(1) / Lp[k + (int64_t)k * ldl];
    const T lik = Lp[(i > k && i < m ? i : k) + (int64_t)k * ldl];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const T xk = readlane(z[c], k) * inv;
      z[c] = i == k ? xk : (i > k ? z[c] - lik * xk : z[c]);
    }
  }
  if (i < w) {
    T* yr = y + (int64_t)(f + i) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) yr[c] = z[c];
  } else if (i < m) {
    T* ur = uvec + (S.u_off[s] + (i - w)) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) ur[c] = z[c];
  }
  release_agent();
  if (lane == 0) __hip_atomic_store(F.ucnt + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Backward solve of a front with m <= kSmallMax by one wave, lane = pivot
// column: subtract L21^T x[rows] (the rows' solutions are final once the
// parent is done), then back-substitute through L11^T.
template <typename T, int NR>
__device__ __forceinline__ void bwd_wave(const DevSym& S, const T* L, T* y, int s,
                                         const SolveFlags& F, int lane) {
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ldl = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  const int p = S.sparent[s];
  if (lane == 0 && p >= 0) wait_at_least(F.bcnt + p, bwd_need(S, p), F.hang);
  acquire_agent();
  const int i = lane;
  const int ic = i < w ? i : 0;
  T z[NR];
  {
    const T* yr = y + (int64_t)(f + ic) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] = yr[c];
  }
  const int32_t* rws = S.rows + S.rows_ptr[s] + w;
  const T* lc = Lp + (int64_t)ic * ldl + w;  // L21 column ic
#pragma unroll 2
  for (int k = 0; k < r; ++k) {
    const T* xr = y + (int64_t)(S.lqinv ? S.lqinv[rws[k]] : rws[k]) * kRowLd<T>;
    const T l = lc[k];
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] -= l * xr[c];
  }
#pragma unroll 2
  for (int k = w - 1; k >= 0; --k) {
    const T inv = T(1) / Lp[k + (int64_t)k * ldl];
    const T lki = Lp[k + (int64_t)ic * ldl];  // L11[k][i], used for i < k
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const T xk = readlane(z[c], k) * inv;
      z[c] = i == k ? xk : (i < k ? z[c] - lki * xk : z[c]);
    }
  }
  if (i < w) {
    T* yr = y + (int64_t)(f + i) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) yr[c] = z[c];
  }
  release_agent();
  if (lane == 0) __hip_atomic_store(F.bcnt + s, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Forward, one 64-row block of a front with m > kSmallMax.  Diagonal block
// (tri): rows [64 blk, 64 blk + kb) of L11, z = y + pulled - sum_{j<blk}
// L(blk, j) x_j, x_blk = W_blk z.  L21 block (!tri): rows w + 64 blk ...,
// u = pulled - sum_j L21(blk, j) x_j over all diagonal blocks.  The products
// run on the matrix cores, 16 rows x 16 right-hand sides per wave; the block
// of x_j is taken as soon as xcnt says it is solved.
template <typename T, int NR, bool DF>
__device__ __forceinline__ void fwd_block(const DevSym& S, const T* L, const T* winv, T* y,
                                          T* uvec, int s, bool tri, int blk, const SolveFlags& F,
                                          T* Zs, int* s_ready) {
  typedef typename Vec4<T>::type V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ldl = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  const int row0 = tri ? blk * kPanel : w + blk * kPanel;
  const int nrows = min(kPanel, (tri ? w : m) - row0);
  const int nj = tri ? blk : (w + kPanel - 1) / kPanel;
  const int li = 16 * wave + (lane & 15);  // A-operand row of this lane
  const int lk = lane >> 4;                // k offset within a 4-step
  const int col = lane & 15;               // B / result column
  T wa[16];
  if (tri) {  // W_blk (lower triangular, nrows x nrows, column-major)
    const T* Wb = winv + S.woff[S.wbase[s] + blk];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 4 * q + lk;
      const bool ok = k <= li && li < nrows;
      wa[q] = Wb[ok ? li + k * nrows : 0] * (ok ? T(1) : T(0));
    }
  }
  if (DF && tid == 0) {
    wait_children(S, s, F.ucnt, F.hang);
    acquire_agent();
  }
  __syncthreads();
  {
    for (int t = tid; t < kPanel * 16; t += kThreads) {
      const int i = t >> 4, c = t & 15;
      T v = T(0);
      if (i < nrows && c < NR) {
        // LDL^T: a pivot row is taken in the block's pivot order
        const int src = (tri && S.lq) ? S.lq[f + row0 + i] - f : row0 + i;
        const int64_t qi = S.rows_ptr[s] + src;
        if (tri) v = y[(int64_t)(f + src) * kRowLd<T> + c];
        for (int p = S.pull_ptr[qi]; p < S.pull_ptr[qi + 1]; ++p)
          v += uvec[(int64_t)S.pull_src[p] * kRowLd<T> + c];
      }
      Zs[t] = v;
    }
  }
  __syncthreads();
  V4 acc = V4{0, 0, 0, 0};
  const int arow = row0 + min(li, nrows - 1);
  const T amask = li < nrows ? T(1) : T(0);
  const int bcol = col < NR ? col : NR - 1;
  const T cmask = col < NR ? T(1) : T(0);
  int ready = 0, par = 0;
  for (int j = 0; j < nj; ++j) {
    const int kbj = min(kPanel, w - j * kPanel);
    T a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 4 * q + lk;
      a[q] = Lp[arow + (int64_t)(j * kPanel + min(k, kbj - 1)) * ldl] * (k < kbj ? amask : T(0));
    }
    if (DF && j >= ready) ready = wait_ready(F.xcnt + s, j + 1, F.hang, s_ready, par);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 4 * q + lk;
      const T b = y[(int64_t)(f + j * kPanel + min(k, kbj - 1)) * kRowLd<T> + bcol] * (k < kbj ? cmask : T(0));
      acc = mfma16(a[q], b, acc);
    }
  }
  if (tri) {
#pragma unroll
    for (int v = 0; v < 4; ++v) Zs[(16 * wave + mfma_row<T>(lane, v)) * 16 + col] -= acc[v];
    __syncthreads();
    V4 xv = V4{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 16; ++q) xv = mfma16(wa[q], Zs[(4 * q + lk) * 16 + col], xv);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * wave + mfma_row<T>(lane, v);
      if (i < nrows && col < NR) y[(int64_t)(f + row0 + i) * kRowLd<T> + col] = xv[v];
    }
    if (DF) {
      publish_barrier();
      if (tid == 0) set_flag(F.xcnt + s, blk + 1);
    } else {
      __syncthreads();
    }
  } else {
    T* us = uvec + (S.u_off[s] + blk * kPanel) * kRowLd<T>;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * wave + mfma_row<T>(lane, v);
      if (i < nrows && col < NR) us[(int64_t)i * kRowLd<T> + col] = Zs[i * 16 + col] - acc[v];
    }
    if (DF) {
      publish_barrier();
      if (tid == 0) add_release(F.ucnt + s);
    } else {
      __syncthreads();
    }
  }
}

// Backward partial product of a front with m > kSmallMax: column block blk
// of L21 against the solutions of L21 rows [kBwdChunk ch, ...) (available
// once the parent is done), written to the block's slot ch.  L21 tiles are
// staged through LDS with coalesced column reads.
template <typename T, int NR, bool DF>
__device__ __forceinline__ void bwd_part(const DevSym& S, const T* L, const T* y, T* part, int s,
                                         int blk, int ch, const SolveFlags& F, T* Ls, T* Vs) {
  typedef typename Vec4<T>::type V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ldl = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  const int p = S.sparent[s];
  if (DF && tid == 0) {
    if (p >= 0) wait_at_least(F.bcnt + p, bwd_need(S, p), F.hang);
    acquire_agent();
  }
  __syncthreads();
  const int c0 = blk * kPanel, kb = min(kPanel, w - c0);
  const int i0 = ch * kBwdChunk, i1 = min(r, i0 + kBwdChunk);
  const int32_t* rws = S.rows + S.rows_ptr[s] + w;
  const int li = 16 * wave + (lane & 15), lk = lane >> 4, col = lane & 15;
  V4 acc = V4{0, 0, 0, 0};
  for (int k0 = i0; k0 < i1; k0 += kPanel) {
    const int kw = min(kPanel, i1 - k0);
    const int rr = min(lane, kw - 1);
    const T rmask = lane < kw ? T(1) : T(0);
#pragma unroll
    for (int c4 = 0; c4 < 16; ++c4) {
      const int cc = wave * 16 + c4;
      Ls[cc * kDiagLd + lane] =
          Lp[(w + k0 + rr) + (int64_t)(c0 + min(cc, kb - 1)) * ldl] * (cc < kb ? rmask : T(0));
    }
    for (int t = tid; t < kPanel * 16; t += kThreads) {
      const int i = t >> 4, c = t & 15;
      const int32_t rr = i < kw ? rws[k0 + i] : 0;
      Vs[t] = (i < kw && c < NR) ? y[(int64_t)(S.lqinv ? S.lqinv[rr] : rr) * kRowLd<T> + c] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = 4 * q + lk;
      acc = mfma16(Ls[li * kDiagLd + i], Vs[i * 16 + col], acc);
    }
    __syncthreads();
  }
  T* P = part + ((int64_t)S.part_base[S.wbase[s] + blk] + ch) * (kPanel * 16);
#pragma unroll
  for (int v = 0; v < 4; ++v) P[(16 * wave + mfma_row<T>(lane, v)) * 16 + col] = acc[v];
  if (DF) {
    publish_barrier();
    if (tid == 0) add_release(F.pcnt + S.wbase[s] + blk);
  } else {
    __syncthreads();
  }
}

// Backward, diagonal block blk of a front with m > kSmallMax (columns
// [64 blk, 64 blk + kb)): z = y - sum of the block's partial products (in
// slot order, taken before the chain since they need only the parent) -
// sum_{c > blk} L(c, blk)^T x_c, x_blk = W_blk^T z.
template <typename T, int NR, bool DF>
__device__ __forceinline__ void bwd_tri(const DevSym& S, const T* L, const T* winv, T* y,
                                        const T* part, int s, int blk, const SolveFlags& F,
                                        T* Zs, int* s_ready) {
  typedef typename Vec4<T>::type V4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ldl = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  const int nb = (w + kPanel - 1) / kPanel;
  const int c0 = blk * kPanel, kb = min(kPanel, w - c0);
  const int li = 16 * wave + (lane & 15), lk = lane >> 4, col = lane & 15;
  const int wblk = S.wbase[s] + blk;
  T wa[16];  // A[i][k] = W_blk[k][i], nonzero for i <= k < kb
  {
    const T* Wb = winv + S.woff[wblk];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 4 * q + lk;
      const bool ok = li <= k && k < kb;
      wa[q] = Wb[ok ? k + li * kb : 0] * (ok ? T(1) : T(0));
    }
  }
  int ready = 0, par = 0;
  const int nch = (r + kBwdChunk - 1) / kBwdChunk;
  if (DF && nch > 0) (void)wait_ready(F.pcnt + wblk, nch, F.hang, s_ready, par);
  {
    const T* P = part + (int64_t)S.part_base[wblk] * (kPanel * 16);
    for (int t = tid; t < kPanel * 16; t += kThreads) {
      const int i = t >> 4, c = t & 15;
      T v = T(0);
      if (i < kb && c < NR) {
        v = y[(int64_t)(f + c0 + i) * kRowLd<T> + c];
        int q = 0;
        for (; q + 4 <= nch; q += 4) {
          const T p0 = P[(int64_t)q * (kPanel * 16) + t], p1 = P[(int64_t)(q + 1) * (kPanel * 16) + t];
          const T p2 = P[(int64_t)(q + 2) * (kPanel * 16) + t], p3 = P[(int64_t)(q + 3) * (kPanel * 16) + t];
          v = (((v - p0) - p1) - p2) - p3;
        }
        for (; q < nch; ++q) v -= P[(int64_t)q * (kPanel * 16) + t];
      }
      Zs[t] = v;
    }
  }
  V4 acc = V4{0, 0, 0, 0};
  const int lcol = c0 + min(li, kb - 1);
  const T amask = li < kb ? T(1) : T(0);
  const int bcol = col < NR ? col : NR - 1;
  const T cmask = col < NR ? T(1) : T(0);
  for (int c = nb - 1; c > blk; --c) {
    const int kc = min(kPanel, w - c * kPanel);
    T a[16];  // A[i][k] = L(c, blk)[k][i]
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 4 * q + lk;
      a[q] = Lp[(c * kPanel + min(k, kc - 1)) + (int64_t)lcol * ldl] * (k < kc ? amask : T(0));
    }
    if (DF && nb - c > ready) ready = wait_ready(F.bcnt + s, nb - c, F.hang, s_ready, par);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = 4 * q + lk;
      const T b = y[(int64_t)(f + c * kPanel + min(k, kc - 1)) * kRowLd<T> + bcol] * (k < kc ? cmask : T(0));
      acc = mfma16(a[q], b, acc);
    }
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < 4; ++v) Zs[(16 * wave + mfma_row<T>(lane, v)) * 16 + col] -= acc[v];
  __syncthreads();
  V4 xv = V4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 16; ++q) xv = mfma16(wa[q], Zs[(4 * q + lk) * 16 + col], xv);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * wave + mfma_row<T>(lane, v);
    if (i < kb && col < NR) y[(int64_t)(f + c0 + i) * kRowLd<T> + col] = xv[v];
  }
  if (DF) {
    publish_barrier();
    if (tid == 0) set_flag(F.bcnt + s, nb - blk);
  } else {
    __syncthreads();
  }
}

// Forward solve of small fronts (m <= g) several per wave in the
// level-by-level phase: lane li of group grp handles row li of front
// wave_list[first + grp]; pivots are broadcast inside the group.
template <typename T, int NR>
__device__ __forceinline__ void fwd_group(const DevSym& S, const T* L, T* y, T* uvec,
                                          const int32_t* wave_list, const WaveItem it, int lane,
                                          int32_t* ucnt) {
  const int g = it.g;
  const int grp = lane / g, i = lane - grp * g, base = grp * g;
  const bool act = grp < it.count;
  const int s = wave_list[it.first + (act ? grp : 0)];
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ldl = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  const int ic = i < m ? i : m - 1;
  const int isrc = (S.lq && i < w) ? S.lq[f + i] - f : ic;  // LDL^T: row taken in pivot order
  const int64_t q = S.rows_ptr[s] + isrc;
  const int p0 = S.pull_ptr[q], p1 = (act && i < m) ? S.pull_ptr[q + 1] : p0;
  T z[NR];
  {
    const T* yr = y + (int64_t)(f + (i < w ? isrc : 0)) * kRowLd<T>;
    const T own = i < w ? T(1) : T(0);
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] = yr[c] * own;
  }
  for (int p = p0; p < p1; ++p) {
    const T* ur = uvec + (int64_t)S.pull_src[p] * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] += ur[c];
  }
  for (int k = 0; k < it.wmax; ++k) {
    const bool kv = k < w;
    const int kk = kv ? k : w - 1;
    const T inv = T(1) / Lp[kk + (int64_t)kk * ldl];
    const T lik = Lp[(i > kk && i < m ? i : kk) + (int64_t)kk * ldl];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const T xk = __shfl(z[c], base + kk, 64) * inv;
      z[c] = !kv ? z[c] : (i == k ? xk : (i > k ? z[c] - lik * xk : z[c]));
    }
  }
  if (act && i < w) {
    T* yr = y + (int64_t)(f + i) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) yr[c] = z[c];
  } else if (act && i < m) {
    T* ur = uvec + (S.u_off[s] + (i - w)) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) ur[c] = z[c];
  }
  if (act && i == 0) ucnt[s] = 1;
}

// Backward counterpart of fwd_group: lane li of group grp handles pivot
// column li of its front.
template <typename T, int NR>
__device__ __forceinline__ void bwd_group(const DevSym& S, const T* L, T* y,
                                          const int32_t* wave_list, const WaveItem it, int lane) {
  const int g = it.g;
  const int grp = lane / g, i = lane - grp * g, base = grp * g;
  const bool act = grp < it.count;
  const int s = wave_list[it.first + (act ? grp : 0)];
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ldl = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  const int ic = i < w ? i : 0;
  T z[NR];
  {
    const T* yr = y + (int64_t)(f + ic) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] = yr[c];
  }
  const int r0 = r > 0 ? w : 0;  // keeps the row pointer inside rows(s) when r = 0
  const int32_t* rws = S.rows + S.rows_ptr[s] + r0;
  const T* lc = Lp + (int64_t)ic * ldl + r0;
  for (int k = 0; k < it.rmax; ++k) {
    const bool kv = k < r;
    const int kk = kv ? k : 0;
    const T l = lc[kk] * (kv ? T(1) : T(0));
    const T* xr = y + (int64_t)(S.lqinv ? S.lqinv[rws[kk]] : rws[kk]) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) z[c] -= l * xr[c];
  }
  for (int k = it.wmax - 1; k >= 0; --k) {
    const bool kv = k < w;
    const int kk = kv ? k : 0;
    const T inv = T(1) / Lp[kk + (int64_t)kk * ldl];
    const T lki = Lp[kk + (int64_t)ic * ldl];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      const T xk = __shfl(z[c], base + kk, 64) * inv;
      z[c] = !kv ? z[c] : (i == k ? xk : (i < k ? z[c] - lki * xk : z[c]));
    }
  }
  if (act && i < w) {
    T* yr = y + (int64_t)(f + i) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) yr[c] = z[c];
  }
}

template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_solve_fwd(DevSym S, const T* L, const T* winv, T* y,
                                                        T* uvec, const SolveTask* tasks,
                                                        int count, const int32_t* wave_list,
                                                        SolveFlags F) {
  __shared__ T Zs[kPanel * 16];
  __shared__ int s_ready[2];
  __shared__ int s_ticket;
  if (threadIdx.x == 0) s_ticket = atomicAdd(F.ticket, 1);
  __syncthreads();
  const int ticket = s_ticket;
  if (ticket >= count) return;
  const SolveTask tk = tasks[ticket];
  if (tk.kind == kSolveWave) {
    const int wave = threadIdx.x >> 6;
    if (wave < tk.b) fwd_wave<T, NR>(S, L, y, uvec, wave_list[tk.a + wave], F, threadIdx.x & 63);
  } else {
    fwd_block<T, NR, true>(S, L, winv, y, uvec, tk.s, tk.kind == kSolveTri, tk.a, F, Zs, s_ready);
  }
}

template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_solve_bwd(DevSym S, const T* L, const T* winv, T* y,
                                                        T* part, const SolveTask* tasks,
                                                        int count, const int32_t* wave_list,
                                                        SolveFlags F) {
  __shared__ T Ls[kPanel * kDiagLd];
  __shared__ T Zs[kPanel * 16];
  __shared__ int s_ready[2];
  __shared__ int s_ticket;
  if (threadIdx.x == 0) s_ticket = atomicAdd(F.ticket, 1);
  __syncthreads();
  const int ticket = s_ticket;
  if (ticket >= count) return;
  const SolveTask tk = tasks[ticket];
  if (tk.kind == kSolveWave) {
    const int wave = threadIdx.x >> 6;
    if (wave < tk.b) bwd_wave<T, NR>(S, L, y, wave_list[tk.a + wave], F, threadIdx.x & 63);
  } else if (tk.kind == kSolveRows) {
    bwd_part<T, NR, true>(S, L, y, part, tk.s, tk.a, tk.b, F, Ls, Zs);
  } else {
    bwd_tri<T, NR, true>(S, L, winv, y, part, tk.s, tk.a, F, Zs, s_ready);
  }
}

// Level-by-level phase: one launch per level; the first (nitems + 3) / 4
// workgroups take four wave items each, the others one large front each,
// whose blocks they solve in order (no flags: the launch boundaries order
// the levels).  Forward also records the fronts as complete for the
// dataflow phase.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_level_fwd(DevSym S, const T* L, const T* winv, T* y,
                                                        T* uvec, const WaveItem* items, int nitems,
                                                        const int32_t* large, const int32_t* wave_list,
                                                        SolveFlags F) {
  __shared__ T Zs[kPanel * 16];
  __shared__ int s_ready[2];
  const int nwg = (nitems + 3) / 4;
  if ((int)blockIdx.x < nwg) {
    const int it = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (it < nitems) fwd_group<T, NR>(S, L, y, uvec, wave_list, items[it], threadIdx.x & 63, F.ucnt);
    return;
  }
  const int s = large[blockIdx.x - nwg];
  const int w = S.sptr[s + 1] - S.sptr[s], r = S.front_m[s] - w;
  for (int b = 0; b * kPanel < w; ++b) fwd_block<T, NR, false>(S, L, winv, y, uvec, s, true, b, F, Zs, s_ready);
  for (int k = 0; k * kPanel < r; ++k) fwd_block<T, NR, false>(S, L, winv, y, uvec, s, false, k, F, Zs, s_ready);
  if (threadIdx.x == 0) F.ucnt[s] = (r + kPanel - 1) / kPanel;
}

template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_level_bwd(DevSym S, const T* L, const T* winv, T* y,
                                                        T* part, const WaveItem* items, int nitems,
                                                        const int32_t* large, const int32_t* wave_list,
                                                        SolveFlags F) {
  __shared__ T Ls[kPanel * kDiagLd];
  __shared__ T Zs[kPanel * 16];
  __shared__ int s_ready[2];
  const int nwg = (nitems + 3) / 4;
  if ((int)blockIdx.x < nwg) {
    const int it = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (it < nitems) bwd_group<T, NR>(S, L, y, wave_list, items[it], threadIdx.x & 63);
    return;
  }
  const int s = large[blockIdx.x - nwg];
  const int w = S.sptr[s + 1] - S.sptr[s], r = S.front_m[s] - w;
  const int nch = (r + kBwdChunk - 1) / kBwdChunk;
  for (int b = (w + kPanel - 1) / kPanel - 1; b >= 0; --b) {
    for (int c = 0; c < nch; ++c) bwd_part<T, NR, false>(S, L, y, part, s, b, c, F, Ls, Zs);
    bwd_tri<T, NR, false>(S, L, winv, y, part, s, b, F, Zs, s_ready);
  }
}

// ---------------------------------------------------------------------------
// Partitioned inverse (SpTRSV variant 3 of the Tacho section).  Z holds, in
// the layout of L, every supernode's [L11^-1; L21 L11^-1] (PinvPlan).

// Z = [I; L21] before the setup steps: one workgroup per 64-column tile of a
// front (rows past m stay zero).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pinv_init(DevSym S, T* Z, const T* L,
                                                        const FrontTile* tiles) {
  const FrontTile ft = tiles[blockIdx.x];
  const int s = ft.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s], c0 = kPanel * ft.t, kb = min(kPanel, w - c0);
  const T* Lp = L + S.L_off[s];
  T* Zp = Z + S.L_off[s];
  for (int t = threadIdx.x; t < ld * kb; t += kThreads) {
    const int c = t / ld, r = t - c * ld;
    const int64_t q = r + (int64_t)(c0 + c) * ld;
    Zp[q] = r < w ? (r == c0 + c ? T(1) : T(0)) : (r < m ? Lp[q] : T(0));
  }
}

// One setup task (PinvTask): tile (a, i) of front s, 64 x 64, wave v owning
// rows 16v..16v+15.  R_ai -= Z_aj L_ji on the matrix cores; when block
// column i has all its terms, Z_ai = R_ai W_ii, with W_ii the stored inverse
// of the diagonal block, or for a front without one (m <= kSmallMax, one
// block) by substitution through L_ii, columns right to left.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pinv_step(DevSym S, T* Z, const T* L,
                                                        const T* winv, const PinvTask* tasks) {
  typedef typename Vec4<T>::type V4;
  __shared__ T Rs[kPanel][kPanel + 1];
  const PinvTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = tk.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s];
  const T* Lp = L + S.L_off[s];
  T* Zp = Z + S.L_off[s];
  const int r0 = kPanel * tk.a, nrows = min(kPanel, m - r0);
  const int c0 = kPanel * tk.i, kbi = min(kPanel, w - c0);
  const int li = 16 * wave + (lane & 15), lk = lane >> 4, col = lane & 15;
  V4 acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * wave + mfma_row<T>(lane, v), cc = 16 * nb + col;
      acc[nb][v] = (row < nrows && cc < kbi) ? Zp[(r0 + row) + (int64_t)(c0 + cc) * ld] : T(0);
    }
  if (tk.j >= 0) {
    const int j0 = kPanel * tk.j, kbj = min(kPanel, w - j0);
    const int arow = r0 + min(li, nrows - 1);
    const T amask = li < nrows ? T(1) : T(0);
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
      const int k = 4 * q + lk, kc = j0 + min(k, kbj - 1);
      const T av = -Zp[arow + (int64_t)kc * ld] * (k < kbj ? amask : T(0));
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int cc = 16 * nb + col;
        const T bv = Lp[kc + (int64_t)(c0 + min(cc, kbi - 1)) * ld] * ((k < kbj && cc < kbi) ? T(1) : T(0));
        acc[nb] = mfma16(av, bv, acc[nb]);
      }
    }
  }
  if (tk.j < 0 || tk.i == tk.j - 1) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) Rs[16 * wave + mfma_row<T>(lane, v)][16 * nb + col] = acc[nb][v];
    __syncthreads();
    if (S.wbase[s] >= 0) {
      const T* Wb = winv + S.woff[S.wbase[s] + tk.i];  // W[k][c] = Wb[c * kbi + k]
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[nb] = V4{0, 0, 0, 0};
#pragma unroll 4
      for (int q = 0; q < 16; ++q) {
        const int k = 4 * q + lk;
        const T av = Rs[li][k];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const int cc = 16 * nb + col;
          const bool ok = k < kbi && cc < kbi;
          const T bv = Wb[ok ? cc * kbi + k : 0] * (ok ? T(1) : T(0));
          acc[nb] = mfma16(av, bv, acc[nb]);
        }
      }
    } else {
      if (tid < nrows) {
        for (int c = kbi - 1; c >= 0; --c) {
          T v = Rs[tid][c];
          for (int k = c + 1; k < kbi; ++k) v -= Rs[tid][k] * Lp[(c0 + k) + (int64_t)(c0 + c) * ld];
          Rs[tid][c] = v / Lp[(c0 + c) + (int64_t)(c0 + c) * ld];
        }
      }
      __syncthreads();
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[nb][v] = Rs[16 * wave + mfma_row<T>(lane, v)][16 * nb + col];
    }
  }
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * wave + mfma_row<T>(lane, v), cc = 16 * nb + col;
      if (row < nrows && cc < kbi) Zp[(r0 + row) + (int64_t)(c0 + cc) * ld] = acc[nb][v];
    }
}

// Forward sweep, one level, step 1: each front's vector z = [y_s; 0] plus
// its children's update vectors (pull map), written back over y_s (pivot
// rows) and u_s (the other rows).  gridDim.y workgroups per front,
// interleaved by kThreads rows.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_pinv_gather_fwd(DevSym S, T* y, T* uvec,
                                                              const int32_t* fronts) {
  const int s = fronts[blockIdx.x];
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  // rows [kThreads y, ...) of the front, kThreads gridDim.y apart
  for (int i = blockIdx.y * kThreads + threadIdx.x; i < m; i += kThreads * gridDim.y) {
    const int64_t q = S.rows_ptr[s] + i;
    T z[NR];
    {
      const T* yr = y + (int64_t)(f + (i < w ? i : 0)) * kRowLd<T>;
      const T own = i < w ? T(1) : T(0);
#pragma unroll
      for (int c = 0; c < NR; ++c) z[c] = yr[c] * own;
    }
    for (int p = S.pull_ptr[q]; p < S.pull_ptr[q + 1]; ++p) {
      const T* ur = uvec + (int64_t)S.pull_src[p] * kRowLd<T>;
#pragma unroll
      for (int c = 0; c < NR; ++c) z[c] += ur[c];
    }
    T* out = i < w ? y + (int64_t)(f + i) * kRowLd<T> : uvec + (S.u_off[s] + (i - w)) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) out[c] = z[c];
  }
}

// Sweeps of a front with m <= kPinvSmallM and w <= kSmallMax by one wave
// (four fronts per workgroup), lane l holding front rows l and l + 64.
// Forward: gather z (own rows of y, children's update vectors), then
// out = Z_s z_s from registers (pivot entries broadcast from their lanes);
// rows < w go to yout, the others are z - out in the update vector.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_pinv_small_fwd(DevSym S, const T* Z, T* y, T* yout,
                                                             T* uvec, const int32_t* fronts,
                                                             int count) {
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (idx >= count) return;
  const int s = fronts[idx];
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s];
  const T* Zp = Z + S.L_off[s];
  T z[2][NR], out[2][NR];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int i = lane + 64 * t;
    const int ic = i < m ? i : m - 1;
    const int64_t q = S.rows_ptr[s] + ic;
    const T* yr = y + (int64_t)(f + (i < w ? i : 0)) * kRowLd<T>;
    const T own = i < w ? T(1) : T(0);
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      z[t][c] = yr[c] * own;
      out[t][c] = T(0);
    }
    const int p0 = S.pull_ptr[q], p1 = i < m ? S.pull_ptr[q + 1] : p0;
    for (int p = p0; p < p1; ++p) {
      const T* ur = uvec + (int64_t)S.pull_src[p] * kRowLd<T>;
#pragma unroll
      for (int c = 0; c < NR; ++c) z[t][c] += ur[c];
    }
  }
#pragma unroll 4
  for (int k = 0; k < w; ++k) {
    T zk[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) zk[c] = readlane(z[0][c], k);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = lane + 64 * t;
      const bool ok = i < m && (i >= w || k <= i);
      const T zik = Zp[(ok ? i : k) + (int64_t)k * ld] * (ok ? T(1) : T(0));
#pragma unroll
      for (int c = 0; c < NR; ++c) out[t][c] += zik * zk[c];
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int i = lane + 64 * t;
    if (i < w) {
      T* yr = yout + (int64_t)(f + i) * kRowLd<T>;
#pragma unroll
      for (int c = 0; c < NR; ++c) yr[c] = out[t][c];
    } else if (i < m) {
      T* ur = uvec + (S.u_off[s] + (i - w)) * kRowLd<T>;
#pragma unroll
      for (int c = 0; c < NR; ++c) ur[c] = z[t][c] - out[t][c];
    }
  }
}

// Backward, same fronts: lane j < w forms x_j = sum_i Z[i][j] v_i with
// v = [yfwd_s; -x_rows] held by the lanes of the rows and broadcast.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_pinv_small_bwd(DevSym S, const T* Z, const T* yfwd,
                                                             T* x, const int32_t* fronts,
                                                             int count) {
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (idx >= count) return;
  const int s = fronts[idx];
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s];
  const T* Zp = Z + S.L_off[s];
  const int32_t* rws = S.rows + S.rows_ptr[s];
  T v[2][NR], acc[NR];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int i = lane + 64 * t;
    const T* src = i < w ? yfwd + (int64_t)(f + i) * kRowLd<T>
                         : x + (int64_t)rws[i < m ? i : m - 1] * kRowLd<T>;
    const T sg = i < w ? T(1) : (i < m ? T(-1) : T(0));
#pragma unroll
    for (int c = 0; c < NR; ++c) v[t][c] = src[c] * sg;
  }
#pragma unroll
  for (int c = 0; c < NR; ++c) acc[c] = T(0);
  const int jc = lane < w ? lane : 0;
  const T jmask = lane < w ? T(1) : T(0);
  for (int i = 0; i < m; ++i) {
    const T zij = Zp[i + (int64_t)jc * ld] * jmask;
#pragma unroll
    for (int c = 0; c < NR; ++c) acc[c] += zij * readlane(i < 64 ? v[0][c] : v[1][c], i & 63);
  }
  if (lane < w) {
    T* xr = x + (int64_t)(f + lane) * kRowLd<T>;
#pragma unroll
    for (int c = 0; c < NR; ++c) xr[c] = acc[c];
  }
}

// Partial product of one chunk of a sweep tile with several chunks (the
// matrix-core layout of the tile's 64 x 16 results): value (i, col) goes to
// part[slot kPanel 16 + i 16 + col].
template <typename T>
__device__ inline void pinv_partial(const typename Vec4<T>::type& acc, T* part, int slot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T* P = part + (int64_t)slot * (kPanel * 16);
#pragma unroll
  for (int v = 0; v < 4; ++v) P[(16 * wave + mfma_row<T>(lane, v)) * 16 + (lane & 15)] = acc[v];
}

// Sum tasks of a sweep (a launch after the chunks'): tile t of front s had
// tk.c chunks; their partial products (slots tk.slot, tk.slot + 1, ...) are
// added in chunk order and written as a one-chunk tile writes its result.
// Forward: rows of Z11 to yout, the others subtracted from the update vector.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_pinv_fsum(DevSym S, T* yout, T* uvec,
                                                        const PinvSweepTask* tasks, const T* part) {
  const PinvSweepTask tk = tasks[blockIdx.x];
  const int s = tk.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int r0 = kPanel * tk.t, nrows = min(kPanel, m - r0);
  for (int q = threadIdx.x; q < nrows * NR; q += kThreads) {
    const int li = q / NR, col = q - li * NR;
    const T* P = part + (int64_t)tk.slot * (kPanel * 16) + li * 16 + col;
    T sum = T(0);
    for (int c = 0; c < tk.c; ++c) sum += P[(int64_t)c * (kPanel * 16)];
    const int i = r0 + li;
    if (i < w) {
      yout[(int64_t)(f + i) * kRowLd<T> + col] = sum;
    } else {
      T* ur = uvec + (S.u_off[s] + (i - w)) * kRowLd<T> + col;
      *ur = *ur - sum;
    }
  }
}

// Backward: columns [64t, 64t + kb) of the front's solution.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_pinv_bsum(DevSym S, T* x, const PinvSweepTask* tasks,
                                                        const T* part) {
  const PinvSweepTask tk = tasks[blockIdx.x];
  const int s = tk.s, f = S.sptr[s], w = S.sptr[s + 1] - f;
  const int c0 = kPanel * tk.t, kb = min(kPanel, w - c0);
  for (int q = threadIdx.x; q < kb * NR; q += kThreads) {
    const int c = q / NR, col = q - c * NR;
    const T* P = part + (int64_t)tk.slot * (kPanel * 16) + c * 16 + col;
    T sum = T(0);
    for (int k = 0; k < tk.c; ++k) sum += P[(int64_t)k * (kPanel * 16)];
    x[(int64_t)(f + c0 + c) * kRowLd<T> + col] = sum;
  }
}

// Forward sweep, one level, step 2: 64 rows of Z_s times z_s (pivot rows of
// y) on the matrix cores (16 rows x 16 right-hand sides per wave), over one
// chunk of the columns; rows < w are the front's solution rows (to yout),
// the others are subtracted from the update vector in place.  Rows of Z11
// see only the columns up to their own.
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_pinv_fwd(DevSym S, const T* Z, const T* y, T* yout,
                                                       T* uvec, const PinvSweepTask* tasks,
                                                       T* part) {
  typedef typename Vec4<T>::type V4;
  const PinvSweepTask tk = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s = tk.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s];
  const T* Zp = Z + S.L_off[s];
  const int r0 = kPanel * tk.t, nrows = min(kPanel, m - r0);
  const int kend = min(w, r0 + kPanel);
  const int klo = tk.c * kPinvChunk, khi = min(kend, klo + kPinvChunk);
  const int li = 16 * wave + (lane & 15), lk = lane >> 4, col = lane & 15;
  const int arow = r0 + min(li, nrows - 1);
  const T amask = li < nrows ? T(1) : T(0);
  const int bcol = col < NR ? col : NR - 1;
  const T cmask = col < NR ? T(1) : T(0);
  V4 acc = V4{0, 0, 0, 0};
  for (int k0 = klo; k0 < khi; k0 += kPanel) {
    T a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = k0 + 4 * q + lk;
      a[q] = Zp[arow + (int64_t)min(k, khi - 1) * ld] * (k < khi ? amask : T(0));
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int k = k0 + 4 * q + lk;
      const T b = y[(int64_t)(f + min(k, khi - 1)) * kRowLd<T> + bcol] * (k < khi ? cmask : T(0));
      acc = mfma16(a[q], b, acc);
    }
  }
  if (tk.slot >= 0) {
    pinv_partial<T>(acc, part, tk.slot + tk.c);
    return;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = r0 + 16 * wave + mfma_row<T>(lane, v);
    if (i - r0 < nrows && col < NR) {
      if (i < w) {
        yout[(int64_t)(f + i) * kRowLd<T> + col] = acc[v];
      } else {
        T* ur = uvec + (S.u_off[s] + (i - w)) * kRowLd<T> + col;
        *ur = *ur - acc[v];
      }
    }
  }
}

// Backward sweep, one level: columns [64t, 64t + kb) of the front's
// solution, x = Z11^T yfwd_s - Z21^T x_rows, over one chunk of the rows from
// 64t on (Z tiles staged through LDS with coalesced column reads; the rows'
// solutions, final once the ancestors are done, read in place).
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_pinv_bwd(DevSym S, const T* Z, const T* yfwd, T* x,
                                                       const PinvSweepTask* tasks, T* part) {
  typedef typename Vec4<T>::type V4;
  __shared__ T Ls[kPanel * kDiagLd];
  __shared__ T Vs[kPanel * 16];
  const PinvSweepTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = tk.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s];
  const T* Zp = Z + S.L_off[s];
  const int32_t* rws = S.rows + S.rows_ptr[s];
  const int c0 = kPanel * tk.t, kb = min(kPanel, w - c0);
  const int ilo = c0 + tk.c * kPinvChunk, ihi = min(m, ilo + kPinvChunk);
  const int li = 16 * wave + (lane & 15), lk = lane >> 4, col = lane & 15;
  V4 acc = V4{0, 0, 0, 0};
  for (int i0 = ilo; i0 < ihi; i0 += kPanel) {
    const int kw = min(kPanel, ihi - i0);
    const int rr = min(lane, kw - 1);
    const T rmask = lane < kw ? T(1) : T(0);
#pragma unroll
    for (int c4 = 0; c4 < 16; ++c4) {
      const int cc = wave * 16 + c4;
      Ls[cc * kDiagLd + lane] = Zp[(i0 + rr) + (int64_t)(c0 + min(cc, kb - 1)) * ld] * (cc < kb ? rmask : T(0));
    }
    for (int t = tid; t < kPanel * 16; t += kThreads) {
      const int i = i0 + (t >> 4), c = t & 15;
      T v = T(0);
      if (i < ihi && c < NR)
        v = i < w ? yfwd[(int64_t)(f + i) * kRowLd<T> + c] : -x[(int64_t)rws[i] * kRowLd<T> + c];
      Vs[t] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int i = 4 * q + lk;
      acc = mfma16(Ls[li * kDiagLd + i], Vs[i * 16 + col], acc);
    }
    __syncthreads();
  }
  if (tk.slot >= 0) {
    pinv_partial<T>(acc, part, tk.slot + tk.c);
    return;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int c = 16 * wave + mfma_row<T>(lane, v);
    if (c < kb && col < NR) x[(int64_t)(f + c0 + c) * kRowLd<T> + col] = acc[v];
  }
}

// Forward sweep, one level, step 2, one right-hand side, on the vector
// units: one lane per row of the 64-row tile, the chunk's columns in four
// contiguous quarters (one per wave), 32 column loads in flight per lane;
// the quarters are added in wave order.  Same outputs as k_pinv_fwd.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pinv_fwd1(DevSym S, const T* Z, const T* y, T* yout,
                                                        T* uvec, const PinvSweepTask* tasks, T* part) {
  constexpr int U = 16;
  __shared__ T xs[kPinvChunk];
  __shared__ T red[kThreads / 64][kPanel];
  const PinvSweepTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = tk.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s];
  const int r0 = kPanel * tk.t, nrows = min(kPanel, m - r0);
  const int kend = min(w, r0 + kPanel);
  const int klo = tk.c * kPinvChunk, khi = min(kend, klo + kPinvChunk);
  for (int k = klo + tid; k < khi; k += kThreads) xs[k - klo] = y[(int64_t)(f + k) * kRowLd<T>];
  __syncthreads();
  const int n = khi - klo, per = (n + 4 * U - 1) / (4 * U) * U;
  const int q0 = min(n, wave * per), q1 = min(n, q0 + per);
  const T* zr = Z + S.L_off[s] + r0 + min(lane, nrows - 1) + (int64_t)klo * ld;
  T acc = T(0);
  for (int k = q0; k < q1; k += U) {
    T z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) z[u] = zr[(int64_t)min(k + u, q1 - 1) * ld];
    __builtin_amdgcn_sched_barrier(0);  // all U loads in flight before the first use
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T xv = xs[min(k + u, q1 - 1)];
      acc += z[u] * (k + u < q1 ? xv : T(0));
    }
  }
  red[wave][lane] = acc;
  __syncthreads();
  T v = T(0);
  if (wave == 0) v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
  if (tk.slot >= 0) {
    if (wave == 0) part[(int64_t)(tk.slot + tk.c) * (kPanel * 16) + lane * 16] = v;
    return;
  }
  if (wave == 0 && lane < nrows) {
    const int i = r0 + lane;
    if (i < w) {
      yout[(int64_t)(f + i) * kRowLd<T>] = v;
    } else {
      T* ur = uvec + (S.u_off[s] + (i - w)) * kRowLd<T>;
      *ur = *ur - v;
    }
  }
}

// Backward sweep, one level, one right-hand side, on the vector units:
// columns [64t, 64t + kb) of the front's solution, x = Z11^T yfwd_s - Z21^T
// x_rows over one chunk of the rows from 64t on.  One lane per row, 16 of
// the block's columns per wave, two 64-row groups (32 column loads) in flight
// per lane; every column's 64 lane sums are added in a fixed order.  Same
// outputs as k_pinv_bwd.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pinv_bwd1(DevSym S, const T* Z, const T* yfwd, T* x,
                                                        const PinvSweepTask* tasks, T* part) {
  __shared__ T vs[kPinvChunk];
  __shared__ T red[kPanel][kPanel + 1];  // [column][lane]
  __shared__ T red2[kPanel][4];
  const PinvSweepTask tk = tasks[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int s = tk.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ld = S.ldL[s];
  const int32_t* rws = S.rows + S.rows_ptr[s];
  const int c0 = kPanel * tk.t, kb = min(kPanel, w - c0);
  const int ilo = c0 + tk.c * kPinvChunk, ihi = min(m, ilo + kPinvChunk);
  for (int i = ilo + tid; i < ihi; i += kThreads)
    vs[i - ilo] = i < w ? yfwd[(int64_t)(f + i) * kRowLd<T>] : -x[(int64_t)rws[i] * kRowLd<T>];
  __syncthreads();
  const int cb = wave * 16;
  const T* zc = Z + S.L_off[s] + (int64_t)c0 * ld;
  T acc[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = T(0);
  for (int i0 = ilo; i0 < ihi; i0 += 2 * kPanel) {
    T z[2][16], v[2];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int i = i0 + g * kPanel + lane;
      const int ic = min(i, ihi - 1);
      v[g] = vs[ic - ilo] * (i < ihi ? T(1) : T(0));
#pragma unroll
      for (int u = 0; u < 16; ++u) z[g][u] = zc[ic + (int64_t)min(cb + u, kb - 1) * ld];
    }
    __builtin_amdgcn_sched_barrier(0);  // all 32 loads in flight before the first use
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += z[g][u] * v[g];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) red[cb + u][lane] = acc[u];
  __syncthreads();
  {
    // four threads per column, 16 lanes each, then the four in order
    const int c = tid >> 2, pq = tid & 3;
    T sum = T(0);
#pragma unroll
    for (int l = 0; l < 16; ++l) sum += red[c][pq * 16 + l];
    red2[c][pq] = sum;
  }
  __syncthreads();
  T v = T(0);
  if (tid < kPanel) v = ((red2[tid][0] + red2[tid][1]) + red2[tid][2]) + red2[tid][3];
  if (tk.slot >= 0) {
    if (tid < kPanel) part[(int64_t)(tk.slot + tk.c) * (kPanel * 16) + tid * 16] = v;
    return;
  }
  if (tid < kb) x[(int64_t)(f + c0 + tid) * kRowLd<T>] = v;
}

// ---------------------------------------------------------------------------
// Level CSR form of the partitioned inverse (SpTRSV variant 4 of the Tacho
// section): the inverse panels Z copied into one CSR per level and sweep,
// then one sparse matrix-vector product per level.
//
// Copy of the segments (one front's part of one CSR row; a wave each):
// forward pivot row (kind 0): row k of Z11 up to its diagonal, columns f + t;
// forward ancestor row (kind 1): row k of Z21, negated, columns f + t;
// backward row (kind 2) of pivot column c: column c of Z_s from row c down,
// the Z11 part reading yfwd (column f + row), the Z21 part negated and
// reading the solution (column n + solve row).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_csr_fill(DevSym S, const T* Z, const CsrSeg* segs,
                                                       int64_t count, int32_t* cols, T* vals) {
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (g >= count) return;
  const CsrSeg sg = segs[g];
  const int s = sg.s, f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], ld = S.ldL[s];
  const T* Zp = Z + S.L_off[s];
  if (sg.kind == 2) {
    const int c = sg.k;
    const int32_t* rws = S.rows + S.rows_ptr[s];
    for (int t = lane; t < m - c; t += 64) {
      const int kr = c + t;
      const T z = Zp[kr + (int64_t)c * ld];
      vals[sg.pos + t] = kr < w ? z : -z;
      cols[sg.pos + t] = kr < w ? f + kr : (int32_t)S.n + rws[kr];
    }
  } else {
    const int len = sg.kind == 0 ? sg.k + 1 : w;
    for (int t = lane; t < len; t += 64) {
      const T z = Zp[sg.k + (int64_t)t * ld];
      vals[sg.pos + t] = sg.kind == 0 ? z : -z;
      cols[sg.pos + t] = f + t;
    }
  }
}

// CSR rows [r0, r1) of one level: out[rows[r]] = (beta ? out[rows[r]] : 0)
// + sum_k vals[k] v(cols[k]), with v(c) = a[c] for c < n and b[c - n]
// otherwise (solve rows of kRowLd values, NR of them used).  A group of
// kSpmvLanes lanes owns a row: the lanes stride its entries (coalesced values
// and indices), each accumulating NR columns, and the group adds its
// partial sums in a fixed order (xor butterfly).
constexpr int kSpmvLanes = 16;
template <typename T, int NR>
__global__ __launch_bounds__(kThreads) void k_level_spmv(const int32_t* rows, const int64_t* rptr,
                                                         const int32_t* cols, const T* vals,
                                                         int64_t r0, int64_t r1, int64_t n,
                                                         const T* a, const T* b, T* out, int beta) {
  const int lane = threadIdx.x & (kSpmvLanes - 1);
  const int64_t r = r0 + (int64_t)blockIdx.x * (kThreads / kSpmvLanes) + threadIdx.x / kSpmvLanes;
  if (r >= r1) return;  // whole groups
  const int64_t k0 = rptr[r], k1 = rptr[r + 1];
  T acc[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = T(0);
  for (int64_t k = k0 + lane; k < k1; k += kSpmvLanes) {
    const int64_t c = cols[k];
    const T v = vals[k];
    const T* src = c < n ? a + c * kRowLd<T> : b + (c - n) * kRowLd<T>;
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] += v * src[q];
  }
#pragma unroll
  for (int q = 0; q < NR; ++q)
    for (int o = kSpmvLanes / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, kSpmvLanes);
  T* dst = out + (int64_t)rows[r] * kRowLd<T>;
#pragma unroll
  for (int q = 0; q < NR; ++q)
    if (lane == q) dst[q] = (beta ? dst[q] : T(0)) + acc[q];
}

// ---------------------------------------------------------------------------
// FP64 refinement: r = b - A x with the full symmetric CSR whose values come
// from the lower triangle (mirror index), one thread per row and column.
// r = b - A x for up to 16 right-hand sides per pass, with x given by rows
// (xt[i * ldt + c] = x[i][c], so the right-hand sides of one unknown share a
// cache line).  A group of kResLanes lanes owns a row: the lanes step through
// its entries together (coalesced reads of values and column indices, each
// read once for every right-hand side), accumulate all columns in registers,
// and the group sum gives lane c the result of column c.  Groups step over
// rows.
constexpr int kResLanes = 16;
__global__ __launch_bounds__(kThreads) void k_residual(int64_t n, const int64_t* rowptr,
                                                       const int32_t* colind, const double* vals,
                                                       const double* b, int64_t ldb,
                                                       const double* xt, int64_t ldt, double* r,
                                                       int64_t nrhs) {
  const int lane = threadIdx.x & (kResLanes - 1);
  const int64_t groups = (int64_t)gridDim.x * (kThreads / kResLanes);
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / kResLanes) + threadIdx.x / kResLanes; i < n;
       i += groups) {
    const int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
    for (int64_t c0 = 0; c0 < nrhs; c0 += kResLanes) {
      const int nc = (int)(nrhs - c0 < kResLanes ? nrhs - c0 : kResLanes);
      double acc[kResLanes];
#pragma unroll
      for (int c = 0; c < kResLanes; ++c) acc[c] = 0.0;
      for (int64_t k = k0 + lane; k < k1; k += kResLanes) {
        const double v = vals[k];
        const double* xc = xt + (int64_t)colind[k] * ldt + c0;
#pragma unroll
        for (int c = 0; c < kResLanes; ++c)
          if (c < nc) acc[c] += v * xc[c];
      }
      // group sums of the columns in use only (nc is the same for the whole
      // workgroup, so the skipped columns cost nothing)
      double mine = 0.0;
#pragma unroll
      for (int c = 0; c < kResLanes; ++c) {
        if (c >= nc) break;
        double t = acc[c];
        for (int o = kResLanes / 2; o > 0; o >>= 1) t += __shfl_xor(t, o, kResLanes);
        mine = lane == c ? t : mine;
      }
      if (lane < nc) r[i + (c0 + lane) * n] = b[i + (c0 + lane) * ldb] - mine;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_colnorms(int64_t n, const double* v, int64_t ldv,
                                                       double* out) {
  __shared__ double part[kThreads / 64];
  const int64_t c = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    const double t = v[i + c * ldv];
    acc += t * t;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) t += part[k];
    out[c] = sqrt(t);
  }
}

// xt[i * nrhs + c] = x[i + c * ldx]: the refinement's iterate by rows.
__global__ __launch_bounds__(kThreads) void k_to_rows(int64_t n, const double* x, int64_t ldx,
                                                      int64_t nrhs, double* xt) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  for (int64_t c = 0; c < nrhs; ++c) xt[i * nrhs + c] = x[i + c * ldx];
}

// Norms of each (system, column) segment of v in two passes, both in a fixed
// order: kNormParts workgroups per segment each sum the squares of one part
// (four independent partial sums per thread keep four loads in flight), then
// one thread per segment adds the parts in order.
__global__ __launch_bounds__(kThreads) void k_segnorms_part(const int64_t* sys_ptr, const double* v,
                                                            int64_t ldv, int64_t nsys,
                                                            double* partial) {
  __shared__ double part[kThreads / 64];
  const int64_t u = blockIdx.x / kNormParts, p = blockIdx.x % kNormParts;
  const int64_t k = u % nsys, c = u / nsys;
  const int64_t s0 = sys_ptr[k], len = sys_ptr[k + 1] - s0;
  const int64_t i0 = s0 + len * p / kNormParts, i1 = s0 + len * (p + 1) / kNormParts;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const double* vc = v + c * ldv;
  int64_t i = i0 + threadIdx.x;
  for (; i + 3 * kThreads < i1; i += 4 * kThreads) {
    const double t0 = vc[i], t1 = vc[i + kThreads], t2 = vc[i + 2 * kThreads], t3 = vc[i + 3 * kThreads];
    a0 += t0 * t0;
    a1 += t1 * t1;
    a2 += t2 * t2;
    a3 += t3 * t3;
  }
  for (; i < i1; i += kThreads) a0 += vc[i] * vc[i];
  double acc = (a0 + a1) + (a2 + a3);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) t += part[q];
    partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kThreads) void k_segnorms_sum(const double* partial, int64_t units,
                                                           double* out) {
  const int64_t u = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (u >= units) return;
  double t = 0.0;
  for (int p = 0; p < kNormParts; ++p) t += partial[u * kNormParts + p];
  out[u] = sqrt(t);
}

__global__ __launch_bounds__(kThreads) void k_zero_units(const int64_t* sys_ptr, double* v,
                                                         int64_t ldv, int64_t nsys,
                                                         const uint8_t* mask) {
  const int64_t k = blockIdx.x, c = blockIdx.y;
  if (!mask[k + c * nsys]) return;
  for (int64_t i = sys_ptr[k] + threadIdx.x; i < sys_ptr[k + 1]; i += kThreads) v[i + c * ldv] = 0.0;
}

__global__ __launch_bounds__(kThreads) void k_select_units(const int64_t* sys_ptr, double* v,
                                                           const double* src, int64_t ld,
                                                           int64_t nsys, const uint8_t* mask) {
  const int64_t k = blockIdx.x, c = blockIdx.y;
  if (!mask[k + c * nsys]) return;
  for (int64_t i = sys_ptr[k] + threadIdx.x; i < sys_ptr[k + 1]; i += kThreads)
    v[i + c * ld] = src[i + c * ld];
}

inline unsigned blocks_for(int64_t count) { return (unsigned)((count + kThreads - 1) / kThreads); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers

template <typename T>
void launch_gather(const DevSym& S, const DevNum<T>& N, const double* vals, int64_t nentries,
                   hipStream_t st) {
  if (nentries > 0) hipLaunchKernelGGL(k_gather<T>, dim3(blocks_for(nentries)), dim3(kThreads), 0, st, S, N, vals, nentries);
}

void launch_scale(const DevSym& S, const double* vals, double* scale, hipStream_t st) {
  if (S.n > 0) hipLaunchKernelGGL(k_scale, dim3(blocks_for(S.n)), dim3(kThreads), 0, st, S, vals, scale);
}

void launch_mirror(const int64_t* idx, const double* src, double* dst, int64_t count,
                   hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_mirror, dim3(blocks_for(count)), dim3(kThreads), 0, st, idx, src, dst, count);
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(count)), dim3(kThreads), 0, st, p, v, count);
}

template <typename T>
void launch_small(const DevSym& S, const DevNum<T>& N, const int32_t* list, int64_t count,
                  hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_small<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, list);
}

template <typename T>
void launch_packed(const DevSym& S, const DevNum<T>& N, T* winv, const int32_t* list,
                   int64_t count, bool big, hipStream_t st) {
  if (count <= 0) return;
  if (big)
    hipLaunchKernelGGL((k_packed<T, kPackedMax>), dim3((unsigned)count), dim3(kThreads), 0, st, S, N, winv, list);
  else
    hipLaunchKernelGGL((k_packed<T, kPackedMid>), dim3((unsigned)count), dim3(kThreads), 0, st, S, N, winv, list);
}

template <typename T>
void launch_leaf(const DevSym& S, const DevNum<T>& N, const int32_t* list, int64_t count,
                 hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_leaf<T>, dim3((unsigned)((count + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                       S, N, list, (int)count);
}

template <typename T>
void launch_assemble(const DevSym& S, const DevNum<T>& N, const AsmItem* items, int64_t count,
                     hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_assemble<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, items);
}

template <typename T>
void launch_diag(const DevSym& S, const DevNum<T>& N, const PanelItem* items, int64_t count,
                 T* winv, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_diag<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, items, winv);
}

template <typename T>
void launch_panel(const DevSym& S, const DevNum<T>& N, const PanelItem* items, int64_t count,
                  const T* winv, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_panel<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, items, winv);
}

template <typename T>
void launch_front(const DevSym& S, const DevNum<T>& N, T* winv, const FrontTask* tasks,
                  int64_t count, int32_t* flow, int64_t ntiles, int64_t nblocks, int64_t nucount,
                  int ticket, int nticket, hipStream_t st) {
  if (count <= 0) return;
  int32_t* pd_done = flow + ntiles;
  int32_t* ucount = pd_done + nblocks;
  int32_t* tickets = ucount + nucount;
  k_front<T><<<(unsigned)count, kThreads, 0, st>>>(S, N, winv, tasks, (int)count, flow, pd_done,
                                                   ucount, tickets + ticket, tickets + nticket);
}

template <typename T>
void launch_gemm(const DevNum<T>& N, const GemmProb* probs, const GemmTile* tiles, int64_t count,
                 int tile, hipStream_t st, const T* bsrc, const DevNum<T>* N2, const T* bsrc2) {
  if (count <= 0) return;
  const dim3 grid((unsigned)count, N2 ? 2 : 1);
  const DevNum<T>& M2 = N2 ? *N2 : N;
  if (tile == kGemmTileBig)
    hipLaunchKernelGGL((k_gemm<T, kGemmTileBig>), grid, dim3(kThreads), 0, st, N, probs, tiles, bsrc, M2, bsrc2);
  else
    hipLaunchKernelGGL((k_gemm<T, kGemmTile>), grid, dim3(kThreads), 0, st, N, probs, tiles, bsrc, M2, bsrc2);
}

void launch_small_ldlt(const DevSym& S, const DevNum<double>& N, const DevLdlt& D,
                       const int32_t* list, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_small_ldlt, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, D, list);
}

void launch_diag_ldlt(const DevSym& S, const DevNum<double>& N, const DevLdlt& D,
                      const PanelItem* items, int64_t count, double* winv, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_diag_ldlt, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, D, items, winv);
}

void launch_panel_ldlt(const DevSym& S, const DevNum<double>& N, const DevLdlt& D,
                       const PanelItem* items, int64_t count, const double* winv, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_panel_ldlt, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, D, items, winv);
}

void launch_apply_dinv(int64_t n, const double* d, const double* e, double* y, int nrhs,
                       hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_apply_dinv, dim3(blocks_for(n)), dim3(kThreads), 0, st, n, d, e, y, nrhs);
}

void launch_iota(int32_t* p, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3(blocks_for(n)), dim3(kThreads), 0, st, p, n);
}

void launch_small_lu(const DevSym& S, const DevNum<double>& N, const DevNum<double>& Nt,
                     int32_t* q, const int32_t* list, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_small_lu, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, Nt, q, list);
}

void launch_diag_lu(const DevSym& S, const DevNum<double>& N, const DevNum<double>& Nt, int32_t* q,
                    const PanelItem* items, int64_t count, double* winv, double* vinv,
                    hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_diag_lu, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, Nt, q, items, winv,
                       vinv);
}

void launch_lu_rowperm(const DevSym& S, const DevNum<double>& N, const int32_t* q,
                       const PanelItem* items, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_lu_rowperm, dim3((unsigned)count), dim3(kThreads), 0, st, S, N, q, items);
}

void launch_panel_lu(const DevSym& S, const DevNum<double>& N, const DevNum<double>& Nt,
                     const int32_t* q, const PanelItem* items, int64_t count, const double* winv,
                     const double* vinv, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_panel_lu, dim3((unsigned)count, 2), dim3(kThreads), 0, st, S, N, Nt, q, items,
                       winv, vinv);
}

void launch_ldlt_perm(int64_t n, const int32_t* perm, const int32_t* q, int32_t* perm_num,
                      int32_t* pinv_num, int32_t* qinv, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_ldlt_perm, dim3(blocks_for(n)), dim3(kThreads), 0, st, n, perm, q, perm_num, pinv_num, qinv);
}

// Counters of the dataflow solves: [xcnt ns][ucnt ns][bcnt ns][pcnt nblk][2 tickets].
inline SolveFlags solve_flags(int32_t* counters, int64_t ns, int64_t nblk, int32_t* hang, int bwd) {
  SolveFlags F;
  F.xcnt = counters;
  F.ucnt = counters + ns;
  F.bcnt = counters + 2 * ns;
  F.pcnt = counters + 3 * ns;
  F.ticket = counters + 3 * ns + nblk + bwd;
  F.hang = hang;
  return F;
}

template <typename T>
void launch_solve_in(const DevSym& S, const double* b, int64_t ldb, T* y, int nrhs,
                     const double* scale, int32_t* counters, int64_t ns, int64_t nblk,
                     hipStream_t st) {
  launch_fill_i32(counters, 0, 3 * ns + nblk + 2, st);
  if (S.n <= 0) return;
  if (nrhs == 1)
    hipLaunchKernelGGL((k_permute_in<T, 1>), dim3(blocks_for(S.n)), dim3(kThreads), 0, st, S, b, ldb, y, (int64_t)nrhs, scale);
  else
    hipLaunchKernelGGL((k_permute_in<T, 16>), dim3(blocks_for(S.n)), dim3(kThreads), 0, st, S, b, ldb, y, (int64_t)nrhs, scale);
}

template <typename T>
void launch_solve_fwd(const DevSym& S, const T* L, const T* winv, T* y, T* uvec,
                      const SolveTask* tasks, int64_t count, const int32_t* wave_list, int nrhs,
                      int32_t* counters, int64_t ns, int64_t nblk, int32_t* hang, hipStream_t st) {
  if (count <= 0) return;
  const SolveFlags F = solve_flags(counters, ns, nblk, hang, 0);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_solve_fwd<T, 1>), dim3((unsigned)count), dim3(kThreads), 0, st, S, L, winv, y, uvec, tasks, (int)count, wave_list, F);
  else
    hipLaunchKernelGGL((k_solve_fwd<T, 16>), dim3((unsigned)count), dim3(kThreads), 0, st, S, L, winv, y, uvec, tasks, (int)count, wave_list, F);
}

template <typename T>
void launch_solve_bwd(const DevSym& S, const T* L, const T* winv, T* y, T* part,
                      const SolveTask* tasks, int64_t count, const int32_t* wave_list, int nrhs,
                      int32_t* counters, int64_t ns, int64_t nblk, int32_t* hang, hipStream_t st) {
  if (count <= 0) return;
  const SolveFlags F = solve_flags(counters, ns, nblk, hang, 1);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_solve_bwd<T, 1>), dim3((unsigned)count), dim3(kThreads), 0, st, S, L, winv, y, part, tasks, (int)count, wave_list, F);
  else
    hipLaunchKernelGGL((k_solve_bwd<T, 16>), dim3((unsigned)count), dim3(kThreads), 0, st, S, L, winv, y, part, tasks, (int)count, wave_list, F);
}

template <typename T>
void launch_level_fwd(const DevSym& S, const T* L, const T* winv, T* y, T* uvec,
                      const WaveItem* items, int64_t nitems, const int32_t* large, int64_t nlarge,
                      const int32_t* wave_list, int nrhs, int32_t* counters, int64_t ns,
                      int64_t nblk, int32_t* hang, hipStream_t st) {
  const int64_t grid = (nitems + 3) / 4 + nlarge;
  if (grid <= 0) return;
  const SolveFlags F = solve_flags(counters, ns, nblk, hang, 0);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_level_fwd<T, 1>), dim3((unsigned)grid), dim3(kThreads), 0, st, S, L, winv, y, uvec, items, (int)nitems, large, wave_list, F);
  else
    hipLaunchKernelGGL((k_level_fwd<T, 16>), dim3((unsigned)grid), dim3(kThreads), 0, st, S, L, winv, y, uvec, items, (int)nitems, large, wave_list, F);
}

template <typename T>
void launch_level_bwd(const DevSym& S, const T* L, const T* winv, T* y, T* part,
                      const WaveItem* items, int64_t nitems, const int32_t* large, int64_t nlarge,
                      const int32_t* wave_list, int nrhs, int32_t* counters, int64_t ns,
                      int64_t nblk, int32_t* hang, hipStream_t st) {
  const int64_t grid = (nitems + 3) / 4 + nlarge;
  if (grid <= 0) return;
  const SolveFlags F = solve_flags(counters, ns, nblk, hang, 1);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_level_bwd<T, 1>), dim3((unsigned)grid), dim3(kThreads), 0, st, S, L, winv, y, part, items, (int)nitems, large, wave_list, F);
  else
    hipLaunchKernelGGL((k_level_bwd<T, 16>), dim3((unsigned)grid), dim3(kThreads), 0, st, S, L, winv, y, part, items, (int)nitems, large, wave_list, F);
}

template <typename T>
void launch_pinv_init(const DevSym& S, T* Z, const T* L, const FrontTile* tiles, int64_t count,
                      hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_pinv_init<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, Z, L, tiles);
}

template <typename T>
void launch_pinv_step(const DevSym& S, T* Z, const T* L, const T* winv, const PinvTask* tasks,
                      int64_t count, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_pinv_step<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, Z, L, winv, tasks);
}

template <typename T>
void launch_pinv_small(const DevSym& S, const T* Z, T* y, T* yfwd, T* uvec, const int32_t* fronts,
                       int64_t count, bool forward, int nrhs, hipStream_t st) {
  if (count <= 0) return;
  const unsigned grid = (unsigned)((count + kThreads / 64 - 1) / (kThreads / 64));
  if (forward) {
    if (nrhs == 1)
      hipLaunchKernelGGL((k_pinv_small_fwd<T, 1>), dim3(grid), dim3(kThreads), 0, st, S, Z, y, yfwd, uvec, fronts, (int)count);
    else
      hipLaunchKernelGGL((k_pinv_small_fwd<T, 16>), dim3(grid), dim3(kThreads), 0, st, S, Z, y, yfwd, uvec, fronts, (int)count);
  } else {
    if (nrhs == 1)
      hipLaunchKernelGGL((k_pinv_small_bwd<T, 1>), dim3(grid), dim3(kThreads), 0, st, S, Z, yfwd, y, fronts, (int)count);
    else
      hipLaunchKernelGGL((k_pinv_small_bwd<T, 16>), dim3(grid), dim3(kThreads), 0, st, S, Z, yfwd, y, fronts, (int)count);
  }
}

template <typename T>
void launch_pinv_fwd(const DevSym& S, const T* Z, T* y, T* yout, T* uvec, const int32_t* fronts,
                     int64_t nfronts, int gchunks, const PinvSweepTask* tasks, int64_t ntasks,
                     const PinvSweepTask* sums, int64_t nsums, T* part, int nrhs, hipStream_t st) {
  if (nfronts <= 0) return;
  const dim3 ggrid((unsigned)nfronts, (unsigned)std::max(1, gchunks));
  if (nrhs == 1) {
    hipLaunchKernelGGL((k_pinv_gather_fwd<T, 1>), ggrid, dim3(kThreads), 0, st, S, y, uvec, fronts);
    hipLaunchKernelGGL((k_pinv_fwd1<T>), dim3((unsigned)ntasks), dim3(kThreads), 0, st, S, Z, y, yout, uvec, tasks, part);
    if (nsums > 0)
      hipLaunchKernelGGL((k_pinv_fsum<T, 1>), dim3((unsigned)nsums), dim3(kThreads), 0, st, S, yout, uvec, sums, (const T*)part);
  } else {
    hipLaunchKernelGGL((k_pinv_gather_fwd<T, 16>), ggrid, dim3(kThreads), 0, st, S, y, uvec, fronts);
    hipLaunchKernelGGL((k_pinv_fwd<T, 16>), dim3((unsigned)ntasks), dim3(kThreads), 0, st, S, Z, y, yout, uvec, tasks, part);
    if (nsums > 0)
      hipLaunchKernelGGL((k_pinv_fsum<T, 16>), dim3((unsigned)nsums), dim3(kThreads), 0, st, S, yout, uvec, sums, (const T*)part);
  }
}

template <typename T>
void launch_pinv_bwd(const DevSym& S, const T* Z, const T* yfwd, T* x, const PinvSweepTask* tasks,
                     int64_t ntasks, const PinvSweepTask* sums, int64_t nsums, T* part, int nrhs,
                     hipStream_t st) {
  if (ntasks <= 0) return;
  if (nrhs == 1) {
    hipLaunchKernelGGL((k_pinv_bwd1<T>), dim3((unsigned)ntasks), dim3(kThreads), 0, st, S, Z, yfwd, x, tasks, part);
    if (nsums > 0)
      hipLaunchKernelGGL((k_pinv_bsum<T, 1>), dim3((unsigned)nsums), dim3(kThreads), 0, st, S, x, sums, (const T*)part);
  } else {
    hipLaunchKernelGGL((k_pinv_bwd<T, 16>), dim3((unsigned)ntasks), dim3(kThreads), 0, st, S, Z, yfwd, x, tasks, part);
    if (nsums > 0)
      hipLaunchKernelGGL((k_pinv_bsum<T, 16>), dim3((unsigned)nsums), dim3(kThreads), 0, st, S, x, sums, (const T*)part);
  }
}

template <typename T>
void launch_csr_fill(const DevSym& S, const T* Z, const CsrSeg* segs, int64_t count, int32_t* cols,
                     T* vals, hipStream_t st) {
  if (count <= 0) return;
  const int64_t per = kThreads / 64;
  hipLaunchKernelGGL(k_csr_fill<T>, dim3((unsigned)((count + per - 1) / per)), dim3(kThreads), 0, st, S, Z,
                     segs, count, cols, vals);
}

template <typename T>
void launch_level_spmv(const int32_t* rows, const int64_t* rptr, const int32_t* cols, const T* vals,
                       int64_t r0, int64_t r1, int64_t n, const T* a, const T* b, T* out, bool beta,
                       int nrhs, hipStream_t st) {
  if (r1 <= r0) return;
  const int64_t per = kThreads / kSpmvLanes;
  const dim3 grid((unsigned)((r1 - r0 + per - 1) / per));
  if (nrhs == 1)
    hipLaunchKernelGGL((k_level_spmv<T, 1>), grid, dim3(kThreads), 0, st, rows, rptr, cols, vals, r0, r1, n, a, b, out, (int)beta);
  else
    hipLaunchKernelGGL((k_level_spmv<T, 16>), grid, dim3(kThreads), 0, st, rows, rptr, cols, vals, r0, r1, n, a, b, out, (int)beta);
}

template <typename T>
void launch_solve_out(const DevSym& S, const T* y, double* x, int64_t ldx, int nrhs,
                      const double* scale, int accumulate, hipStream_t st) {
  if (S.n <= 0) return;
  if (nrhs == 1)
    hipLaunchKernelGGL((k_permute_out<T, 1>), dim3(blocks_for(S.n)), dim3(kThreads), 0, st, S, y, x, ldx, (int64_t)nrhs, scale, accumulate);
  else
    hipLaunchKernelGGL((k_permute_out<T, 16>), dim3(blocks_for(S.n)), dim3(kThreads), 0, st, S, y, x, ldx, (int64_t)nrhs, scale, accumulate);
}

void launch_residual(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                     const double* b, int64_t ldb, const double* x, int64_t ldx, double* r,
                     int64_t nrhs, double* xt, hipStream_t st) {
  if (n > 0 && nrhs > 0) {
    const double* rows = x;
    int64_t ldt = 1;
    if (nrhs > 1) {
      hipLaunchKernelGGL(k_to_rows, dim3(blocks_for(n)), dim3(kThreads), 0, st, n, x, ldx, nrhs, xt);
      rows = xt;
      ldt = nrhs;
    }
    const int64_t rows_per_block = kThreads / kResLanes;
    const int64_t blocks = std::min<int64_t>((n + rows_per_block - 1) / rows_per_block, 8192);
    hipLaunchKernelGGL(k_residual, dim3((unsigned)blocks), dim3(kThreads), 0, st, n, rowptr, colind,
                       vals, b, ldb, rows, ldt, r, nrhs);
  }
}

void launch_colnorms(int64_t n, const double* v, int64_t ldv, int64_t nrhs, double* out,
                     hipStream_t st) {
  if (nrhs > 0) hipLaunchKernelGGL(k_colnorms, dim3((unsigned)nrhs), dim3(kThreads), 0, st, n, v, ldv, out);
}

void launch_segnorms(int64_t nsys, const int64_t* sys_ptr, const double* v, int64_t ldv,
                     int64_t nrhs, double* out, double* partial, hipStream_t st) {
  const int64_t units = nsys * nrhs;
  if (units <= 0) return;
  hipLaunchKernelGGL(k_segnorms_part, dim3((unsigned)(units * kNormParts)), dim3(kThreads), 0, st,
                     sys_ptr, v, ldv, nsys, partial);
  hipLaunchKernelGGL(k_segnorms_sum, dim3(blocks_for(units)), dim3(kThreads), 0, st, partial, units,
                     out);
}

void launch_zero_units(int64_t nsys, const int64_t* sys_ptr, double* v, int64_t ldv, int64_t nrhs,
                       const uint8_t* mask, hipStream_t st) {
  if (nsys > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_zero_units, dim3((unsigned)nsys, (unsigned)nrhs), dim3(kThreads), 0, st,
                       sys_ptr, v, ldv, nsys, mask);
}

void launch_select_units(int64_t nsys, const int64_t* sys_ptr, double* v, const double* src,
                         int64_t ld, int64_t nrhs, const uint8_t* mask, hipStream_t st) {
  if (nsys > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_select_units, dim3((unsigned)nsys, (unsigned)nrhs), dim3(kThreads), 0, st,
                       sys_ptr, v, src, ld, nsys, mask);
}

#define TACHO_INSTANTIATE(T)                                                                     \
  template void launch_gather<T>(const DevSym&, const DevNum<T>&, const double*, int64_t,         \
                                 hipStream_t);                                                   \
  template void launch_small<T>(const DevSym&, const DevNum<T>&, const int32_t*, int64_t,         \
                                hipStream_t);                                                    \
  template void launch_packed<T>(const DevSym&, const DevNum<T>&, T*, const int32_t*, int64_t,    \
                                 bool, hipStream_t);                                             \
  template void launch_pinv_init<T>(const DevSym&, T*, const T*, const FrontTile*, int64_t,       \
                                    hipStream_t);                                                \
  template void launch_pinv_step<T>(const DevSym&, T*, const T*, const T*, const PinvTask*,       \
                                    int64_t, hipStream_t);                                       \
  template void launch_pinv_small<T>(const DevSym&, const T*, T*, T*, T*, const int32_t*, int64_t, \
                                     bool, int, hipStream_t);                                    \
  template void launch_pinv_fwd<T>(const DevSym&, const T*, T*, T*, T*, const int32_t*, int64_t,  \
                                   int, const PinvSweepTask*, int64_t, const PinvSweepTask*,     \
                                   int64_t, T*, int, hipStream_t);                               \
  template void launch_pinv_bwd<T>(const DevSym&, const T*, const T*, T*, const PinvSweepTask*,   \
                                   int64_t, const PinvSweepTask*, int64_t, T*, int, hipStream_t); \
  template void launch_csr_fill<T>(const DevSym&, const T*, const CsrSeg*, int64_t, int32_t*, T*,  \
                                   hipStream_t);                                                 \
  template void launch_level_spmv<T>(const int32_t*, const int64_t*, const int32_t*, const T*,     \
                                     int64_t, int64_t, int64_t, const T*, const T*, T*, bool, int, \
                                     hipStream_t);                                               \
  template void launch_leaf<T>(const DevSym&, const DevNum<T>&, const int32_t*, int64_t,          \
                               hipStream_t);                                                     \
  template void launch_assemble<T>(const DevSym&, const DevNum<T>&, const AsmItem*, int64_t,      \
                                   hipStream_t);                                                 \
  template void launch_diag<T>(const DevSym&, const DevNum<T>&, const PanelItem*, int64_t, T*,    \
                               hipStream_t);                                                     \
  template void launch_panel<T>(const DevSym&, const DevNum<T>&, const PanelItem*, int64_t,       \
                                const T*, hipStream_t);                                          \
  template void launch_gemm<T>(const DevNum<T>&, const GemmProb*, const GemmTile*, int64_t, int,  \
                               hipStream_t, const T*, const DevNum<T>*, const T*);               \
  template void launch_front<T>(const DevSym&, const DevNum<T>&, T*, const FrontTask*, int64_t,   \
                                int32_t*, int64_t, int64_t, int64_t, int, int, hipStream_t);     \
  template void launch_solve_in<T>(const DevSym&, const double*, int64_t, T*, int,              \
                                   const double*, int32_t*, int64_t, int64_t, hipStream_t);      \
  template void launch_solve_fwd<T>(const DevSym&, const T*, const T*, T*, T*, const SolveTask*,  \
                                    int64_t, const int32_t*, int, int32_t*, int64_t, int64_t,    \
                                    int32_t*, hipStream_t);                                      \
  template void launch_solve_bwd<T>(const DevSym&, const T*, const T*, T*, T*, const SolveTask*,  \
                                    int64_t, const int32_t*, int, int32_t*, int64_t, int64_t,    \
                                    int32_t*, hipStream_t);                                      \
  template void launch_solve_out<T>(const DevSym&, const T*, double*, int64_t, int,               \
                                    const double*, int, hipStream_t);                            \
  template void launch_level_fwd<T>(const DevSym&, const T*, const T*, T*, T*, const WaveItem*,   \
                                    int64_t, const int32_t*, int64_t, const int32_t*, int,       \
                                    int32_t*, int64_t, int64_t, int32_t*, hipStream_t);          \
  template void launch_level_bwd<T>(const DevSym&, const T*, const T*, T*, T*, const WaveItem*,   \
                                    int64_t, const int32_t*, int64_t, const int32_t*, int,       \
                                    int32_t*, int64_t, int64_t, int32_t*, hipStream_t);

TACHO_INSTANTIATE(double)
TACHO_INSTANTIATE(float)

// ---------------------------------------------------------------------------
// Device scratch of the entry points that allocate nothing: one file-scope
// array per GPU (the runtime gives every device its own copy when it loads
// the code object; each holds it until the process ends).  In host code the
// array's name is not a device address: its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current.

namespace {
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace tacho
