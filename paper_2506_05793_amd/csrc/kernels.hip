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

#include <climits>
#include <cstdint>

#include "device.hpp"

namespace tacho {

namespace {

constexpr int kThreads = 256;
constexpr int kDiagLd = kPanel + 1;  // LDS leading dimension of diagonal blocks

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

// ---------------------------------------------------------------------------
// Large fronts, assembly: the workgroup owns front columns [c0, c1).  It
// zeroes them, writes the A entries, then adds every child's update matrix
// (ascending child order).  The child's relative map is increasing, so the
// child columns landing in [c0, c1) form one contiguous range.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_assemble(DevSym S, DevNum<T> N,
                                                       const AsmItem* items) {
  const AsmItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const int s = it.s;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f;
  const int ldl = S.ldL[s], ldu = S.ldU[s];
  T* Lp = N.L + S.L_off[s];
  T* Us = w < S.front_m[s] ? N.U + S.U_off[s] : nullptr;
  for (int c = it.c0; c < it.c1; ++c) {
    if (c < w) {
      for (int i = tid; i < ldl; i += kThreads) Lp[i + (int64_t)c * ldl] = T(0);
    } else {
      for (int i = tid; i < ldu; i += kThreads) Us[i + (int64_t)(c - w) * ldu] = T(0);
    }
  }
  __syncthreads();
  if (it.c0 < w) {
    const int64_t q0 = S.acol_ptr[f + it.c0], q1 = S.acol_ptr[f + min(it.c1, w)];
    for (int64_t q = q0 + tid; q < q1; q += kThreads) Lp[S.a_pos[q]] = N.avals[q];
  }
  __syncthreads();
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int c = S.child_list[q];
    const int wc = S.sptr[c + 1] - S.sptr[c], rc = S.front_m[c] - wc;
    const T* Uc = N.U + S.U_off[c];
    const int ldc = S.ldU[c];
    const int32_t* rm = S.rmap + S.rows_ptr[c] + wc;
    int lo = 0, hi = rc;  // first jj with rm[jj] >= c0
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (rm[mid] < it.c0) lo = mid + 1; else hi = mid;
    }
    for (int jj = lo; jj < rc; ++jj) {
      const int tc = rm[jj];
      if (tc >= it.c1) break;
      for (int ii = jj + tid; ii < rc; ii += kThreads) {
        const int tr = rm[ii];
        const T v = Uc[ii + (int64_t)jj * ldc];
        if (tc < w)
          Lp[tr + (int64_t)tc * ldl] += v;
        else
          Us[(tr - w) + (int64_t)(tc - w) * ldu] += v;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Large fronts, panel step 1 (one workgroup per front): Cholesky of the
// diagonal block [k, k+kb) in LDS, blocked by 16 columns (a 16x16 block by
// one wave, its rows below by one thread each, a rank-16 update of the rest),
// written back in place, and its inverse W = L_kk^{-1} (identity-padded to
// kPanel) written to the scratch slot of the item for the triangular solve
// of the rows below.  Non-positive or NaN pivots go to the failure flag.
constexpr int kSub = 16;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_diag(DevSym S, DevNum<T> N, const PanelItem* items,
                                                   T* winv) {
  __shared__ T D[kPanel * kDiagLd];  // column-major, D[c * kDiagLd + r]
  __shared__ T W[kPanel * kDiagLd];
  const PanelItem it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
  for (int jb = 0; jb < kPanel; jb += kSub) {
    // (1) 16x16 diagonal block by wave 0; lanes own rows jb + (lane & 15)
    if (wave == 0) {
      for (int j = jb; j < jb + kSub; ++j) {
        const T d = D[j * kDiagLd + j];
        const T ljj = sqrt(d);
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
          if (j < kb && !(d > T(0))) atomicMin(N.fail, f + k + j);
          D[j * kDiagLd + j] = ljj;
        }
        const int i = jb + (lane & 15);
        if (lane < kSub && i > j) D[j * kDiagLd + i] = D[j * kDiagLd + i] / ljj;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // rank-1 update inside the 16x16 block: lanes cover (row, col) pairs
        for (int t = lane; t < kSub * kSub; t += 64) {
          const int r = jb + (t & 15), c = jb + (t >> 4);
          if (c > j && r >= c) D[c * kDiagLd + r] -= D[j * kDiagLd + r] * D[j * kDiagLd + c];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    // (2) rows below the block: one thread per row, forward substitution
    const int below = kPanel - jb - kSub;
    if (tid < below) {
      const int r = jb + kSub + tid;
      T x[kSub];
#pragma unroll
      for (int c = 0; c < kSub; ++c) x[c] = D[(jb + c) * kDiagLd + r];
#pragma unroll
      for (int c = 0; c < kSub; ++c) {
        T acc = x[c];
#pragma unroll
        for (int c2 = 0; c2 < c; ++c2) acc -= x[c2] * D[(jb + c2) * kDiagLd + jb + c];
        x[c] = acc / D[(jb + c) * kDiagLd + jb + c];
      }
#pragma unroll
      for (int c = 0; c < kSub; ++c) D[(jb + c) * kDiagLd + r] = x[c];
    }
    __syncthreads();
    // (3) rank-16 update of the trailing lower triangle
    for (int t = tid; t < below * below; t += kThreads) {
      const int cc = t / below, rr = t - cc * below;
      if (rr >= cc) {
        const int r = jb + kSub + rr, c = jb + kSub + cc;
        T acc = D[c * kDiagLd + r];
#pragma unroll
        for (int q = 0; q < kSub; ++q) acc -= D[(jb + q) * kDiagLd + r] * D[(jb + q) * kDiagLd + c];
        D[c * kDiagLd + r] = acc;
      }
    }
    __syncthreads();
  }
  for (int t = tid; t < kb * kb; t += kThreads) {
    const int c = t / kb, r = t - c * kb;
    if (r >= c) Lp[(k + r) + (int64_t)(k + c) * ld] = D[c * kDiagLd + r];
  }
  // W = L^{-1} by 16x16 blocks.  Diagonal blocks first (one thread per
  // column of each block, forward substitution down its own column), then
  // the off-diagonal blocks by distance d = 1..3 from the diagonal:
  // W_ib = -W_ii * sum_{q=b}^{i-1} L_iq W_qb.
  __shared__ T rd[kPanel];
  __shared__ T Tmp[3][kSub * kSub];
  if (tid < kPanel) rd[tid] = T(1) / D[tid * kDiagLd + tid];
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
    W[c * kDiagLd + r] = T(0);
  }
  __syncthreads();
  if (tid < kPanel) {
    const int col = tid, b0 = (col / kSub) * kSub;
    for (int r = col; r < b0 + kSub; ++r) {
      T acc = r == col ? T(1) : T(0);
      for (int q = col; q < r; ++q) acc -= D[q * kDiagLd + r] * W[col * kDiagLd + q];
      W[col * kDiagLd + r] = acc * rd[r];
    }
  }
  __syncthreads();
  for (int d = 1; d < kPanel / kSub; ++d) {
    const int nblk = kPanel / kSub - d;  // blocks (b + d, b), b < nblk
    for (int t = tid; t < nblk * kSub * kSub; t += kThreads) {
      const int bb = t / (kSub * kSub), e = t - bb * kSub * kSub;
      const int rr = e % kSub, cc = e / kSub;
      const int i0 = (bb + d) * kSub, c = bb * kSub + cc;
      T acc = T(0);
      for (int q = bb * kSub; q < i0; ++q) acc += D[q * kDiagLd + i0 + rr] * W[c * kDiagLd + q];
      Tmp[bb][rr + cc * kSub] = acc;
    }
    __syncthreads();
    for (int t = tid; t < nblk * kSub * kSub; t += kThreads) {
      const int bb = t / (kSub * kSub), e = t - bb * kSub * kSub;
      const int rr = e % kSub, cc = e / kSub;
      const int i0 = (bb + d) * kSub, c = bb * kSub + cc;
      T acc = T(0);
      for (int q = 0; q < kSub; ++q) acc += W[(i0 + q) * kDiagLd + i0 + rr] * Tmp[bb][q + cc * kSub];
      W[c * kDiagLd + i0 + rr] = -acc;
    }
    __syncthreads();
  }
  T* Wout = winv + (int64_t)it.wslot * kPanel * kPanel;
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;
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
  const T* Win = winv + (int64_t)it.wslot * kPanel * kPanel;
  for (int t = tid; t < kPanel * kPanel; t += kThreads) {
    const int c = t / kPanel, r = t - c * kPanel;  // W stored column-major: Win[c * 64 + r] = W[r][c]
    Ws[c][r] = Win[t];
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
// Update on the matrix cores: C[M x N] -= A[M x K] * A[0:N, :]^T for the
// elements with row >= col.  One 64x64 output tile per workgroup, four waves
// of 32x32 (2x2 blocks of 16x16x4 MFMA), K staged through LDS 16 at a time.
// The MFMA computes the transposed tile so that a lane's outputs run down a
// column of the column-major C (coalesced read-modify-write).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gemm(DevNum<T> N, const GemmProb* probs,
                                                   const GemmTile* tiles) {
  constexpr int TT = kGemmTile, KT = 16, PAD = 4;
  __shared__ T As[KT][TT + PAD];
  __shared__ T Bs[KT][TT + PAD];
  const GemmTile tl = tiles[blockIdx.x];
  const GemmProb g = probs[tl.prob];
  const T* A = N.L + g.a_off;
  T* C = (g.c_in_u ? N.U : N.L) + g.c_off;
  const int i0 = tl.ti * TT, j0 = tl.tj * TT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  typedef typename Vec4<T>::type V4;
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
  const int lrow = tid & 63, lk = tid >> 6;
  const bool arow_ok = i0 + lrow < g.M, brow_ok = j0 + lrow < g.N;
  for (int k0 = 0; k0 < g.K; k0 += KT) {
#pragma unroll
    for (int u = 0; u < KT / 4; ++u) {
      const int kk = lk + 4 * u, kg = k0 + kk;
      const bool kok = kg < g.K;
      As[kk][lrow] = (arow_ok && kok) ? A[(i0 + lrow) + (int64_t)kg * g.lda] : T(0);
      Bs[kk][lrow] = (brow_ok && kok) ? A[(j0 + lrow) + (int64_t)kg * g.lda] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KT / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      T av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kr][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kr][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma16(bv[b], av[a], acc[a][b]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * 32 + a * 16 + (lane & 15);
        const int j = j0 + wc * 32 + b * 16 + mfma_row<T>(lane, v);
        if (i < g.M && j < g.N && i >= j) {
          T* p = C + i + (int64_t)j * g.ldc;
          *p = *p - acc[a][b][v];
        }
      }
}

// ---------------------------------------------------------------------------
// Solves.  y holds P b (n x nrhs, ld n) and receives P x.  Forward: each
// front pulls its children's update vectors (ascending), solves its diagonal
// block in 64-column blocks (one wave per right-hand side, register shuffles)
// and subtracts L21 x from the rows below; rows >= w go to its own update
// vector u_s (r x nrhs in uvec).  Backward: x_s = L11^{-T}(y_s - L21^T x[rows]).
constexpr int kRhsBlock = 16;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_permute_in(DevSym S, const double* b, int64_t ldb,
                                                         T* y, int64_t nrhs,
                                                         const double* scale) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= S.n) return;
  const int64_t src = S.perm[i];
  const double d = scale ? scale[i] : 1.0;
  for (int64_t c = 0; c < nrhs; ++c) y[i + c * S.n] = (T)(b[src + c * ldb] * d);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_permute_out(DevSym S, const T* y, double* x,
                                                          int64_t ldx, int64_t nrhs,
                                                          const double* scale, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= S.n) return;
  const int64_t dst = S.perm[i];
  const double d = scale ? scale[i] : 1.0;
  for (int64_t c = 0; c < nrhs; ++c) {
    const double v = (double)y[i + c * S.n] * d;
    if (accumulate)
      x[dst + c * ldx] += v;
    else
      x[dst + c * ldx] = v;
  }
}

// Fronts with r_s * w_s >= kSolveSplit leave the L21 products of the solves
// to the multi-workgroup kernels k_fwd_gemv / k_bwd_gemv.
__device__ inline bool solve_split(int w, int r) { return (int64_t)r * w >= kSolveSplit; }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fwd(DevSym S, const T* L, T* y, T* uvec,
                                                  const int32_t* list, int nrhs) {
  __shared__ T D[kPanel * kDiagLd];
  __shared__ T X[kPanel * kRhsBlock];
  const int s = list[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ldl = S.ldL[s];
  const int64_t n = S.n;
  const T* Lp = L + S.L_off[s];
  T* us = uvec + S.u_off[s] * nrhs;
  const int mrow = solve_split(w, r) ? w : m;  // rows updated here
  for (int t = tid; t < r * nrhs; t += kThreads) us[t] = T(0);
  __syncthreads();
  for (int q = S.child_ptr[s]; q < S.child_ptr[s + 1]; ++q) {
    const int c = S.child_list[q];
    const int wc = S.sptr[c + 1] - S.sptr[c], rc = S.front_m[c] - wc;
    const T* uc = uvec + S.u_off[c] * nrhs;
    const int32_t* rm = S.rmap + S.rows_ptr[c] + wc;
    for (int t = tid; t < rc * nrhs; t += kThreads) {
      const int col = t / rc, i = t - col * rc;
      const int tr = rm[i];
      const T v = uc[i + col * rc];
      if (tr < w)
        y[f + tr + col * n] += v;
      else
        us[(tr - w) + col * r] += v;
    }
    __syncthreads();
  }
  for (int jb = 0; jb < w; jb += kPanel) {
    const int kb = min(kPanel, w - jb);
    for (int t = tid; t < kb * kb; t += kThreads) {
      const int c = t / kb, rr = t - c * kb;
      if (rr >= c) D[c * kDiagLd + rr] = Lp[(jb + rr) + (int64_t)(jb + c) * ldl];
    }
    for (int t = tid; t < kb * nrhs; t += kThreads) {
      const int col = t / kb, rr = t - col * kb;
      X[rr + col * kPanel] = y[f + jb + rr + col * n];
    }
    __syncthreads();
    for (int col = wave; col < nrhs; col += kThreads / 64) {
      T z = lane < kb ? X[lane + col * kPanel] : T(0);
      for (int c = 0; c < kb; ++c) {
        const T xc = __shfl(z, c, 64) / D[c * kDiagLd + c];
        if (lane == c)
          z = xc;
        else if (lane > c && lane < kb)
          z -= D[c * kDiagLd + lane] * xc;
      }
      if (lane < kb) {
        X[lane + col * kPanel] = z;
        y[f + jb + lane + col * n] = z;
      }
    }
    __syncthreads();
    for (int i = jb + kb + tid; i < mrow; i += kThreads) {
      T acc[kRhsBlock];
#pragma unroll
      for (int col = 0; col < kRhsBlock; ++col) acc[col] = T(0);
      for (int c = 0; c < kb; ++c) {
        const T l = Lp[i + (int64_t)(jb + c) * ldl];
#pragma unroll
        for (int col = 0; col < kRhsBlock; ++col)
          if (col < nrhs) acc[col] += l * X[c + col * kPanel];
      }
#pragma unroll
      for (int col = 0; col < kRhsBlock; ++col) {
        if (col < nrhs) {
          if (i < w)
            y[f + i + col * n] -= acc[col];
          else
            us[(i - w) + col * r] -= acc[col];
        }
      }
    }
    __syncthreads();
  }
}

// Forward solve, L21 part of a split front: u_s[rows] -= L21[rows, :] x_s for
// kPanel rows per workgroup; lanes own rows, the four waves split the
// columns, x_s is staged through LDS kSolveChunk columns at a time.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fwd_gemv(DevSym S, const T* L, const T* y, T* uvec,
                                                       const SolveItem* items, int nrhs) {
  __shared__ T X[kSolveChunk * kRhsBlock];
  __shared__ T part[kThreads / 64][kPanel * kRhsBlock];
  const SolveItem it = items[blockIdx.x];
  const int s = it.s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ldl = S.ldL[s];
  const int64_t n = S.n;
  const T* Lp = L + S.L_off[s];
  const int row = w + it.chunk * kPanel + lane;
  const bool valid = row < m;
  T acc[kRhsBlock];
#pragma unroll
  for (int col = 0; col < kRhsBlock; ++col) acc[col] = T(0);
  for (int cb = 0; cb < w; cb += kSolveChunk) {
    const int cw = min(kSolveChunk, w - cb);
    __syncthreads();
    for (int t = tid; t < cw * nrhs; t += kThreads) {
      const int col = t / cw, c = t - col * cw;
      X[c + col * kSolveChunk] = y[f + cb + c + col * n];
    }
    __syncthreads();
    if (valid) {
      for (int c = wave; c < cw; c += kThreads / 64) {
        const T l = Lp[row + (int64_t)(cb + c) * ldl];
#pragma unroll
        for (int col = 0; col < kRhsBlock; ++col)
          if (col < nrhs) acc[col] += l * X[c + col * kSolveChunk];
      }
    }
  }
#pragma unroll
  for (int col = 0; col < kRhsBlock; ++col) part[wave][lane + col * kPanel] = acc[col];
  __syncthreads();
  if (wave == 0 && valid) {
    T* us = uvec + S.u_off[s] * nrhs;
    for (int col = 0; col < nrhs; ++col) {
      T t = T(0);
#pragma unroll
      for (int q = 0; q < kThreads / 64; ++q) t += part[q][lane + col * kPanel];
      us[(row - w) + col * r] -= t;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd(DevSym S, const T* L, T* y, const int32_t* list,
                                                  int nrhs) {
  __shared__ T D[kPanel * kDiagLd];
  __shared__ T X[kPanel * kRhsBlock];
  const int s = list[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s];
  const int ldl = S.ldL[s];
  const int64_t n = S.n;
  const T* Lp = L + S.L_off[s];
  const int32_t* rws = S.rows + S.rows_ptr[s];
  if (w == 0) return;
  const int mrow = solve_split(w, m - w) ? w : m;  // L21^T x already applied when split
  for (int jb = ((w - 1) / kPanel) * kPanel; jb >= 0; jb -= kPanel) {
    const int kb = min(kPanel, w - jb);
    for (int t = tid; t < kb * kb; t += kThreads) {
      const int c = t / kb, rr = t - c * kb;
      if (rr >= c) D[c * kDiagLd + rr] = Lp[(jb + rr) + (int64_t)(jb + c) * ldl];
    }
    for (int p = wave; p < kb * nrhs; p += kThreads / 64) {
      const int col = p / kb, j = p - col * kb;
      T acc = T(0);
      const T* lc = Lp + (int64_t)(jb + j) * ldl;
      for (int i = jb + kb + lane; i < mrow; i += 64) {
        const int64_t gi = i < w ? (int64_t)(f + i) : (int64_t)rws[i];
        acc += lc[i] * y[gi + col * n];
      }
      acc = wave_sum(acc);
      if (lane == 0) X[j + col * kPanel] = y[f + jb + j + col * n] - acc;
    }
    __syncthreads();
    for (int col = wave; col < nrhs; col += kThreads / 64) {
      T z = lane < kb ? X[lane + col * kPanel] : T(0);
      for (int c = kb - 1; c >= 0; --c) {
        const T xc = __shfl(z, c, 64) / D[c * kDiagLd + c];
        if (lane == c)
          z = xc;
        else if (lane < c)
          z -= D[lane * kDiagLd + c] * xc;
      }
      if (lane < kb) y[f + jb + lane + col * n] = z;
    }
    __syncthreads();
  }
}

// Backward solve, L21 part of a split front: y_s[cols] -= L21[:, cols]^T x[rows(s)[w:]]
// for kPanel columns per workgroup; lanes own columns (each lane walks its
// column down, the 64 columns of a wave share cache lines), the four waves
// split the rows, the gathered x is staged through LDS.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_gemv(DevSym S, const T* L, T* y,
                                                       const SolveItem* items, int nrhs) {
  __shared__ T XG[kSolveChunk * kRhsBlock];
  __shared__ T part[kThreads / 64][kPanel * kRhsBlock];
  const SolveItem it = items[blockIdx.x];
  const int s = it.s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int f = S.sptr[s], w = S.sptr[s + 1] - f, m = S.front_m[s], r = m - w;
  const int ldl = S.ldL[s];
  const int64_t n = S.n;
  const T* Lp = L + S.L_off[s];
  const int32_t* rws = S.rows + S.rows_ptr[s] + w;
  const int j = it.chunk * kPanel + lane;
  const bool valid = j < w;
  const T* lc = Lp + (int64_t)(valid ? j : 0) * ldl + w;
  T acc[kRhsBlock];
#pragma unroll
  for (int col = 0; col < kRhsBlock; ++col) acc[col] = T(0);
  for (int rb = 0; rb < r; rb += kSolveChunk) {
    const int rw = min(kSolveChunk, r - rb);
    __syncthreads();
    for (int t = tid; t < rw * nrhs; t += kThreads) {
      const int col = t / rw, i = t - col * rw;
      XG[i + col * kSolveChunk] = y[(int64_t)rws[rb + i] + col * n];
    }
    __syncthreads();
    if (valid) {
      for (int i = wave; i < rw; i += kThreads / 64) {
        const T l = lc[rb + i];
#pragma unroll
        for (int col = 0; col < kRhsBlock; ++col)
          if (col < nrhs) acc[col] += l * XG[i + col * kSolveChunk];
      }
    }
  }
#pragma unroll
  for (int col = 0; col < kRhsBlock; ++col) part[wave][lane + col * kPanel] = acc[col];
  __syncthreads();
  if (wave == 0 && valid) {
    for (int col = 0; col < nrhs; ++col) {
      T t = T(0);
#pragma unroll
      for (int q = 0; q < kThreads / 64; ++q) t += part[q][lane + col * kPanel];
      y[f + j + col * n] -= t;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 refinement: r = b - A x with the full symmetric CSR whose values come
// from the lower triangle (mirror index), one thread per row and column.
__global__ __launch_bounds__(kThreads) void k_residual(int64_t n, const int64_t* rowptr,
                                                       const int32_t* colind, const double* vals,
                                                       const double* b, int64_t ldb,
                                                       const double* x, int64_t ldx, double* r,
                                                       int64_t nrhs) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t c = blockIdx.y;
  double acc = 0.0;
  for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += vals[k] * x[colind[k] + c * ldx];
  r[i + c * n] = b[i + c * ldb] - acc;
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
void launch_gemm(const DevNum<T>& N, const GemmProb* probs, const GemmTile* tiles, int64_t count,
                 hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_gemm<T>, dim3((unsigned)count), dim3(kThreads), 0, st, N, probs, tiles);
}

template <typename T>
void launch_permute_in(const DevSym& S, const double* b, int64_t ldb, T* y, int64_t nrhs,
                       const double* scale, hipStream_t st) {
  if (S.n > 0) hipLaunchKernelGGL(k_permute_in<T>, dim3(blocks_for(S.n)), dim3(kThreads), 0, st, S, b, ldb, y, nrhs, scale);
}

template <typename T>
void launch_permute_out(const DevSym& S, const T* y, double* x, int64_t ldx, int64_t nrhs,
                        const double* scale, int accumulate, hipStream_t st) {
  if (S.n > 0) hipLaunchKernelGGL(k_permute_out<T>, dim3(blocks_for(S.n)), dim3(kThreads), 0, st, S, y, x, ldx, nrhs, scale, accumulate);
}

template <typename T>
void launch_fwd(const DevSym& S, const T* L, T* y, T* uvec, const int32_t* list, int64_t count,
                int32_t nrhs, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fwd<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, L, y, uvec, list, nrhs);
}

template <typename T>
void launch_fwd_gemv(const DevSym& S, const T* L, const T* y, T* uvec, const SolveItem* items,
                     int64_t count, int32_t nrhs, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fwd_gemv<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, L, y, uvec, items, nrhs);
}

template <typename T>
void launch_bwd_gemv(const DevSym& S, const T* L, T* y, const SolveItem* items, int64_t count,
                     int32_t nrhs, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_bwd_gemv<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, L, y, items, nrhs);
}

template <typename T>
void launch_bwd(const DevSym& S, const T* L, T* y, const int32_t* list, int64_t count,
                int32_t nrhs, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_bwd<T>, dim3((unsigned)count), dim3(kThreads), 0, st, S, L, y, list, nrhs);
}

void launch_residual(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* vals,
                     const double* b, int64_t ldb, const double* x, int64_t ldx, double* r,
                     int64_t nrhs, hipStream_t st) {
  if (n > 0 && nrhs > 0)
    hipLaunchKernelGGL(k_residual, dim3(blocks_for(n), (unsigned)nrhs), dim3(kThreads), 0, st, n,
                       rowptr, colind, vals, b, ldb, x, ldx, r, nrhs);
}

void launch_colnorms(int64_t n, const double* v, int64_t ldv, int64_t nrhs, double* out,
                     hipStream_t st) {
  if (nrhs > 0) hipLaunchKernelGGL(k_colnorms, dim3((unsigned)nrhs), dim3(kThreads), 0, st, n, v, ldv, out);
}

#define TACHO_INSTANTIATE(T)                                                                     \
  template void launch_gather<T>(const DevSym&, const DevNum<T>&, const double*, int64_t,         \
                                 hipStream_t);                                                   \
  template void launch_small<T>(const DevSym&, const DevNum<T>&, const int32_t*, int64_t,         \
                                hipStream_t);                                                    \
  template void launch_assemble<T>(const DevSym&, const DevNum<T>&, const AsmItem*, int64_t,      \
                                   hipStream_t);                                                 \
  template void launch_diag<T>(const DevSym&, const DevNum<T>&, const PanelItem*, int64_t, T*,    \
                               hipStream_t);                                                     \
  template void launch_panel<T>(const DevSym&, const DevNum<T>&, const PanelItem*, int64_t,       \
                                const T*, hipStream_t);                                          \
  template void launch_gemm<T>(const DevNum<T>&, const GemmProb*, const GemmTile*, int64_t,       \
                               hipStream_t);                                                     \
  template void launch_permute_in<T>(const DevSym&, const double*, int64_t, T*, int64_t,          \
                                     const double*, hipStream_t);                                \
  template void launch_permute_out<T>(const DevSym&, const T*, double*, int64_t, int64_t,         \
                                      const double*, int, hipStream_t);                          \
  template void launch_fwd<T>(const DevSym&, const T*, T*, T*, const int32_t*, int64_t, int32_t,  \
                              hipStream_t);                                                      \
  template void launch_bwd<T>(const DevSym&, const T*, T*, const int32_t*, int64_t, int32_t,      \
                              hipStream_t);                                                      \
  template void launch_fwd_gemv<T>(const DevSym&, const T*, const T*, T*, const SolveItem*,       \
                                   int64_t, int32_t, hipStream_t);                               \
  template void launch_bwd_gemv<T>(const DevSym&, const T*, T*, const SolveItem*, int64_t,        \
                                   int32_t, hipStream_t);

TACHO_INSTANTIATE(double)
TACHO_INSTANTIATE(float)

}  // namespace tacho
