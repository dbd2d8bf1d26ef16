// C ABI of the library: handles, device memory, launch sequences.
//
// Three phases as in the paper's Trilinos section: tacho_analyze (pattern
// only, host), tacho_factorize / tacho_refactorize (numeric, GPU, level by
// level of the supernodal elimination tree), tacho_solve (forward and
// backward supernodal substitution by levels, Tacho section variant 1), plus
// FP32 factors with FP64 iterative refinement (templated precisions,
// Trilinos section; refinement with computed factors, Basker section).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/tacho.h"
#include "device.hpp"
#include "plan.hpp"
#include "symbolic.hpp"
#include "tuning.hpp"

using namespace tacho;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      if (e_ == hipErrorOutOfMemory)                                                   \
        return fail(TACHO_ERR_NOMEM, std::string("out of device memory: ") + #expr);  \
      return fail(TACHO_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    }                                                                                  \
  } while (0)

// Owning device allocation.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { reset(); }
  void reset() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t b) {
    reset();
    if (b == 0) b = 64;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    else p = nullptr;
    return e;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// The library's own host transfers (symbolic uploads, counter clearing) run
// on a private non-blocking stream per device and wait for it, never on the
// legacy default stream: a legacy-stream operation is refused while another
// thread captures a graph on a blocking stream.
hipError_t aux_stream(hipStream_t* out) {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev]) {
    e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  *out = streams[dev];
  return hipSuccess;
}

hipError_t copy_to_device(void* dst, const void* src, size_t bytes) {
  hipStream_t st = nullptr;
  hipError_t e = aux_stream(&st);
  if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

hipError_t clear_device(void* dst, size_t bytes) {
  hipStream_t st = nullptr;
  hipError_t e = aux_stream(&st);
  if (e == hipSuccess) e = hipMemsetAsync(dst, 0, bytes, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

template <typename T>
hipError_t upload(DBuf& d, const std::vector<T>& v) {
  hipError_t e = d.alloc(v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  if (!v.empty()) e = copy_to_device(d.p, v.data(), v.size() * sizeof(T));
  return e;
}

}  // namespace

struct tacho_sym {
  tacho_options opt;
  Symbolic S;
  Plan P;
  PlanTuning tune;                // plan parameters in effect (defaults resolved)
  std::vector<int64_t> mirror;    // per pattern entry: caller index of the lower twin (-1: none)
  std::vector<int32_t> a_prc;     // per assembly entry: permuted row, permuted column
  std::vector<int32_t> solve_levels;  // level_list copy (supernodes by level)
  // device copies
  bool uploaded = false;
  int device = -1;
  DBuf d_sptr, d_front_m, d_rows_ptr, d_rows, d_rmap, d_child_ptr, d_child_list, d_acol_ptr,
      d_a_pos, d_a_src, d_a_prc, d_L_off, d_ldL, d_U_off, d_ldU, d_u_off, d_perm, d_pinv, d_diag_q,
      d_wbase, d_woff, d_tbase, d_sparent, d_pull_ptr, d_pull_src, d_part_base, d_pt1base, d_asm_rng;
  DBuf d_small, d_asm, d_diag, d_panel, d_probs, d_tiles, d_ftasks, d_levels, d_fsolve, d_bsolve,
      d_wave_list, d_lwave, d_llarge;
  DBuf d_rowptr, d_colind, d_mirror, d_sys_ptr;
  DevSym view{};
  std::mutex mu;
  // LDL^T runs the stepwise large-front launches (diagonal block, panel,
  // trailing updates): their plan, built on the first LDL^T factorization,
  // and the device view with that plan's assembly ranges
  std::unique_ptr<Plan> P1;
  DBuf d1_small, d1_asm, d1_asm_rng, d1_diag, d1_panel, d1_probs, d1_tiles;
  DBuf d_lu_lo, d_lu_up;  // LU: caller indices of each A entry and of its transposed twin
  DevSym view1{};
  // partitioned-inverse solves: their plan, built on first use
  std::unique_ptr<PinvPlan> Q;
  DBuf dq_setup, dq_tiles, dq_frow, dq_bcol, dq_fsum, dq_bsum, dq_small, dq_large;
  // level CSR form of the partitioned inverse (built on first use)
  std::unique_ptr<LevelCsr> C;
  DBuf dc_rows, dc_rptr, dc_segs;
};

// Per-launch timing of the library's kernels on the caller's stream (hipEvents
// around each launch while profiling is enabled), with the algorithmic flops
// and bytes of each launch taken from the plan.
struct KernelProfile {
  struct Rec {
    int kind;
    int ev;
    double flops, bytes;
  };
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<Rec> recs;
  int64_t launches[TACHO_PROFILE_KINDS] = {};
  double ms[TACHO_PROFILE_KINDS] = {}, flops[TACHO_PROFILE_KINDS] = {},
         bytes[TACHO_PROFILE_KINDS] = {};
  ~KernelProfile() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  void clear() {
    recs.clear();
    for (int k = 0; k < TACHO_PROFILE_KINDS; ++k) {
      launches[k] = 0;
      ms[k] = flops[k] = bytes[k] = 0;
    }
  }
  int begin(hipStream_t st) {
    if (!on) return -1;
    const size_t e = recs.size() * 2;
    while (pool.size() < e + 2) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) return -1;
      pool.push_back(ev);
    }
    if (hipEventRecord(pool[e], st) != hipSuccess) return -1;
    return (int)e;
  }
  void end(int e, hipStream_t st, int kind, double fl, double by) {
    if (e < 0) return;
    if (hipEventRecord(pool[e + 1], st) != hipSuccess) return;
    recs.push_back({kind, e, fl, by});
  }
  hipError_t collect() {
    if (recs.empty()) return hipSuccess;
    hipError_t err = hipEventSynchronize(pool[recs.back().ev + 1]);
    if (err != hipSuccess) return err;
    for (const Rec& r : recs) {
      float t = 0;
      err = hipEventElapsedTime(&t, pool[r.ev], pool[r.ev + 1]);
      if (err != hipSuccess) return err;
      launches[r.kind] += 1;
      ms[r.kind] += t;
      flops[r.kind] += r.flops;
      bytes[r.kind] += r.bytes;
    }
    recs.clear();
    return hipSuccess;
  }
};

// Host bookkeeping of one refinement, per unit (system x right-hand side).
struct RefineHost {
  std::vector<double> hn, rho, prev;
  std::vector<int> stalls;
  std::vector<uint8_t> done, bad, mask;
  void resize(int64_t units) {
    hn.resize(2 * units);
    rho.resize(units);
    prev.resize(units);
    stalls.resize(units);
    done.resize(units);
    bad.resize(units);
    mask.resize(units);
  }
};

struct tacho_num {
  tacho_sym* sym = nullptr;
  RefineHost rh;
  KernelProfile prof;
  int precision = TACHO_FP64;
  DBuf L, U, avals, vals, fullvals, scale, fail, winv, pt1;
  DBuf y, uvec;             // solve workspace (kRhs columns)
  DBuf part;                // partial L21 products of the split solves
  DBuf sync;                // solve tickets (2 per level) and block ready flags
  DBuf flow;                // dataflow factorization counters, flags, tickets, hang flag
  DBuf bdev, xdev;          // host-pointer staging
  DBuf rws;                 // refinement scratch (residual, norms, mask)
  DBuf ld_d, ld_e, ld_q, ld_qinv, ld_perm, ld_pinv, ld_panels;  // LDL^T: D, pivot orders, L D panels
  DBuf lu_t, lu_u2, lu_avals, lu_vinv;  // LU: U^T panels, upper update halves, upper A entries, (U_kk^T)^{-1}
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool pending = false;     // factorization queued, flag not yet read
  int last_status = TACHO_OK;
  int64_t last_fail = -1;
  hipStream_t last_stream = nullptr;
  tacho_num* fallback = nullptr;  // FP64 refactorization after a refinement stall
  bool fp32_broken = false;       // FP32 pivot breakdown: the breaking system uses `fallback`
  int32_t fp32_fail_col = -1;     // permuted column of the first FP32 pivot breakdown
  hipStream_t last_solve_stream = nullptr;  // stream of the last solve (queued or finished)
  bool solve_queued = false;      // a solve was queued without reading its hang flag
  hipGraphExec_t fgraph = nullptr;  // captured factorization launch sequence
  int solve_variant = TACHO_SOLVE_BLOCK_INVERSE;
  bool csr_pending = false;  // the level CSR copy is being set up for a variant switch
  DBuf Z, yfwd;                   // partitioned inverse (layout of L) and forward result rows
  DBuf zpart;                     // its sweeps' chunk partial products
  DBuf cvals, ccols;              // level CSR form of Z (TACHO_SOLVE_LEVEL_CSR)
  ~tacho_num() {
    if (fgraph) (void)hipGraphExecDestroy(fgraph);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    delete fallback;
  }
};

namespace {

constexpr int kRhs = 16;  // right-hand sides per solve sweep
constexpr int kRowBytes = 128;  // bytes per row of the solve vectors (one cache line, >= kRhs doubles)

tacho_options defaults() {
  tacho_options o;
  std::memset(&o, 0, sizeof(o));
  o.nd_leaf_size = 8;
  o.small_front = 0;
  o.scale_fp32 = 1;
  o.refine_max = 10;
  o.refine_tol = 1e-10;
  o.stall_ratio = 0.5;
  o.hbm_budget_bytes = 0;
  o.block_size = 0;
  o.ordering = 0;
  o.graphs = 1;
  o.front_kernel = 0;
  return o;
}

int finish_analysis(tacho_sym* h, int64_t nnz_input) {
  std::string err;
  if (h->opt.small_front != 0 || h->opt.block_size != 0)
    return fail(TACHO_ERR_INVALID, "small_front and block_size are reserved and must be 0");
  h->S.nnz_input = nnz_input;
  SymOptions so;
  so.nd_leaf_size = h->opt.nd_leaf_size > 0 ? h->opt.nd_leaf_size : 8;
  so.ordering = h->opt.ordering;
  if (h->opt.dof_block < 0) return fail(TACHO_ERR_INVALID, "dof_block must be >= 0");
  so.dof_block = h->opt.dof_block;
  if (h->opt.dof_map) {
    if (h->S.nsys > 1) return fail(TACHO_ERR_INVALID, "dof_map is not accepted for a batch");
    so.dof_map = h->opt.dof_map;
    so.dof_map_n = h->S.A.n;
  }
  int rc;
  try {
    rc = analyze_pattern(h->S, so, err);
  } catch (const std::bad_alloc&) {
    return fail(TACHO_ERR_NOMEM, "host memory exhausted during the analysis");
  } catch (const std::exception& e) {
    return fail(TACHO_ERR_INVALID, e.what());
  }
  if (rc != kOk) return fail(rc, err);
  const auto t_plan = std::chrono::steady_clock::now();
  PlanTuning tune;
  tune.u_range = h->opt.u_range;
  tune.chain_min = h->opt.chain_min;
  tune.level_fronts = h->opt.solve_level_fronts;
  tune.asm_cols = h->opt.asm_cols;
  tune.solo_m = h->opt.solo_m;
  tune.chain_inplace = h->opt.chain_inplace;
  if (h->opt.autotune_path && h->opt.autotune_path[0]) {
    // parameters left at 0 take the table's value for this workload class
    // and precision (order-changing ones from the precision's entry)
    TunedParams tp;
    if (load_tuned(h->opt.autotune_path, h->S.n, nnz_input,
                   h->opt.autotune_precision == TACHO_FP32 ? 1 : 0, tp, err) != 0)
      return fail(TACHO_ERR_INVALID, err);
    if (tune.u_range == 0) tune.u_range = tp.u_range;
    if (tune.chain_min == 0) tune.chain_min = tp.chain_min;
    if (tune.level_fronts == 0) tune.level_fronts = tp.solve_level_fronts;
    if (tune.asm_cols == 0) tune.asm_cols = tp.asm_cols;
    if (tune.solo_m == 0) tune.solo_m = tp.solo_m;
    if (tune.chain_inplace == 0) tune.chain_inplace = tp.chain_inplace;
  }
  // effective values (0 = the plan's default)
  h->tune.u_range = tune.u_range > 0 ? tune.u_range : kURange;
  h->tune.chain_min = tune.chain_min == 0 ? kChainMin : tune.chain_min;
  h->tune.level_fronts = tune.level_fronts > 0 ? tune.level_fronts : kLevelFronts;
  h->tune.asm_cols = tune.asm_cols > 0 ? tune.asm_cols : kAsmCols;
  h->tune.solo_m = tune.solo_m == 0 ? kSoloM : tune.solo_m;
  h->tune.chain_inplace = tune.chain_inplace >= 0 ? 1 : -1;
  rc = build_plan(h->S, h->P, err, h->opt.front_kernel == 1 ? 1 : 0, tune);
  if (rc != kOk) return fail(rc, err);
  const Symbolic& S = h->S;
  // lower-twin index of every pattern entry, for the refinement residual
  const Pattern& A = S.A;
  h->mirror.assign(A.colind.size(), -1);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
      const int32_t j = A.colind[k];
      if (i >= j) {
        h->mirror[k] = A.src[k];
      } else {
        // twin (j, i) lies in row j, sorted
        const int32_t* b = A.colind.data() + A.rowptr[j];
        const int32_t* e = A.colind.data() + A.rowptr[j + 1];
        const int32_t* p = std::lower_bound(b, e, (int32_t)i);
        h->mirror[k] = A.src[A.rowptr[j] + (p - b)];
      }
    }
  h->a_prc.resize(2 * S.a_src.size());
  for (int32_t s = 0; s < S.ns; ++s)
    for (int32_t j = S.sptr[s]; j < S.sptr[s + 1]; ++j)
      for (int64_t q = S.acol_ptr[j]; q < S.acol_ptr[j + 1]; ++q) {
        h->a_prc[2 * q] = S.rows[S.rows_ptr[s] + S.a_row[q]];
        h->a_prc[2 * q + 1] = j;
      }
  h->S.t_plan_us = std::chrono::duration_cast<std::chrono::microseconds>(
                       std::chrono::steady_clock::now() - t_plan).count();
  return TACHO_OK;
}

int ensure_uploaded(tacho_sym* h) {
  std::lock_guard<std::mutex> lock(h->mu);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (h->uploaded) {
    if (dev != h->device) return fail(TACHO_ERR_INVALID, "symbolic handle used on another device");
    return TACHO_OK;
  }
  const Symbolic& S = h->S;
  const Plan& P = h->P;
  HIP_TRY(upload(h->d_sptr, S.sptr));
  HIP_TRY(upload(h->d_front_m, S.front_m));
  HIP_TRY(upload(h->d_rows_ptr, S.rows_ptr));
  HIP_TRY(upload(h->d_rows, S.rows));
  HIP_TRY(upload(h->d_rmap, S.rmap));
  HIP_TRY(upload(h->d_child_ptr, S.child_ptr));
  HIP_TRY(upload(h->d_child_list, S.child_list));
  HIP_TRY(upload(h->d_acol_ptr, S.acol_ptr));
  HIP_TRY(upload(h->d_a_pos, P.a_pos));
  HIP_TRY(upload(h->d_a_src, S.a_src));
  HIP_TRY(upload(h->d_a_prc, h->a_prc));
  HIP_TRY(upload(h->d_L_off, P.L_off));
  HIP_TRY(upload(h->d_ldL, P.ldL));
  HIP_TRY(upload(h->d_U_off, P.U_off));
  HIP_TRY(upload(h->d_ldU, P.ldU));
  HIP_TRY(upload(h->d_u_off, P.u_off));
  HIP_TRY(upload(h->d_perm, S.perm));
  {
    std::vector<int32_t> pinv(S.perm.size());
    for (size_t i = 0; i < S.perm.size(); ++i) pinv[S.perm[i]] = (int32_t)i;
    HIP_TRY(upload(h->d_pinv, pinv));
  }
  HIP_TRY(upload(h->d_diag_q, P.diag_q));
  HIP_TRY(upload(h->d_wbase, P.wbase));
  HIP_TRY(upload(h->d_woff, P.woff));
  HIP_TRY(upload(h->d_tbase, P.tbase));
  HIP_TRY(upload(h->d_sparent, S.sparent));
  HIP_TRY(upload(h->d_pull_ptr, P.pull_ptr));
  HIP_TRY(upload(h->d_pull_src, P.pull_src));
  HIP_TRY(upload(h->d_part_base, P.part_base));
  HIP_TRY(upload(h->d_pt1base, P.pt1base));
  HIP_TRY(upload(h->d_asm_rng, P.asm_rng));
  HIP_TRY(upload(h->d_small, P.small_list));
  HIP_TRY(upload(h->d_asm, P.asm_items));
  HIP_TRY(upload(h->d_diag, P.diag_items));
  HIP_TRY(upload(h->d_panel, P.panel_items));
  HIP_TRY(upload(h->d_probs, P.probs));
  HIP_TRY(upload(h->d_tiles, P.tiles));
  HIP_TRY(upload(h->d_ftasks, P.ftasks));
  HIP_TRY(upload(h->d_levels, S.level_list));
  HIP_TRY(upload(h->d_fsolve, P.fsolve));
  HIP_TRY(upload(h->d_bsolve, P.bsolve));
  HIP_TRY(upload(h->d_wave_list, P.wave_list));
  HIP_TRY(upload(h->d_lwave, P.lwave));
  HIP_TRY(upload(h->d_llarge, P.llarge));
  HIP_TRY(upload(h->d_rowptr, S.A.rowptr));
  HIP_TRY(upload(h->d_colind, S.A.colind));
  HIP_TRY(upload(h->d_mirror, h->mirror));
  HIP_TRY(upload(h->d_sys_ptr, S.sys_ptr));
  DevSym& v = h->view;
  v.n = S.n;
  v.sptr = h->d_sptr.as<int32_t>();
  v.front_m = h->d_front_m.as<int32_t>();
  v.rows_ptr = h->d_rows_ptr.as<int64_t>();
  v.rows = h->d_rows.as<int32_t>();
  v.rmap = h->d_rmap.as<int32_t>();
  v.child_ptr = h->d_child_ptr.as<int32_t>();
  v.child_list = h->d_child_list.as<int32_t>();
  v.acol_ptr = h->d_acol_ptr.as<int64_t>();
  v.a_pos = h->d_a_pos.as<int32_t>();
  v.a_src = h->d_a_src.as<int64_t>();
  v.a_prc = h->d_a_prc.as<int32_t>();
  v.L_off = h->d_L_off.as<int64_t>();
  v.ldL = h->d_ldL.as<int32_t>();
  v.U_off = h->d_U_off.as<int64_t>();
  v.ldU = h->d_ldU.as<int32_t>();
  v.u_off = h->d_u_off.as<int64_t>();
  v.perm = h->d_perm.as<int32_t>();
  v.pinv = h->d_pinv.as<int32_t>();
  v.diag_q = h->d_diag_q.as<int32_t>();
  v.wbase = h->d_wbase.as<int32_t>();
  v.woff = h->d_woff.as<int64_t>();
  v.tbase = h->d_tbase.as<int32_t>();
  v.sparent = h->d_sparent.as<int32_t>();
  v.pull_ptr = h->d_pull_ptr.as<int32_t>();
  v.pull_src = h->d_pull_src.as<int32_t>();
  v.part_base = h->d_part_base.as<int32_t>();
  v.pt1base = h->d_pt1base.as<int32_t>();
  v.asm_rng = h->d_asm_rng.as<int32_t>();
  h->device = dev;
  h->uploaded = true;
  return TACHO_OK;
}

// The stepwise launch plan that LDL^T factorizations run (built once per
// symbolic handle, with the same batching parameters).
// LU value maps (built once per symbolic handle, on first use).
int ensure_lu_maps(tacho_sym* h) {
  if (h->d_lu_lo.p) return TACHO_OK;
  std::vector<int64_t> lo, up;
  lu_value_sources(h->S, lo, up);
  HIP_TRY(upload(h->d_lu_lo, lo));
  HIP_TRY(upload(h->d_lu_up, up));
  return TACHO_OK;
}

int ensure_stepwise(tacho_sym* h) {
  std::lock_guard<std::mutex> lock(h->mu);
  if (h->P1) return TACHO_OK;
  std::unique_ptr<Plan> P1(new Plan());
  std::string err;
  if (build_plan(h->S, *P1, err, 1, h->tune) != kOk) return fail(TACHO_ERR_INVALID, err);
  // the rest of the device view (layout of L, U and the diagonal-block
  // inverses) is shared with the Cholesky plan
  if (P1->wbase != h->P.wbase || P1->woff != h->P.woff || P1->U_off != h->P.U_off ||
      P1->L_off != h->P.L_off)
    return fail(TACHO_ERR_INVALID, "stepwise plan does not share the factor layout");
  HIP_TRY(upload(h->d1_small, P1->small_list));
  HIP_TRY(upload(h->d1_asm, P1->asm_items));
  HIP_TRY(upload(h->d1_asm_rng, P1->asm_rng));
  HIP_TRY(upload(h->d1_diag, P1->diag_items));
  HIP_TRY(upload(h->d1_panel, P1->panel_items));
  HIP_TRY(upload(h->d1_probs, P1->probs));
  HIP_TRY(upload(h->d1_tiles, P1->tiles));
  // the stepwise plan's assembly items index its own child column ranges
  h->view1 = h->view;
  h->view1.asm_rng = h->d1_asm_rng.as<int32_t>();
  h->P1 = std::move(P1);
  return TACHO_OK;
}

int ensure_pinv(tacho_sym* h) {
  std::lock_guard<std::mutex> lock(h->mu);
  if (h->Q) return TACHO_OK;
  std::unique_ptr<PinvPlan> Q(new PinvPlan());
  build_pinv_plan(h->S, *Q);
  if ((int64_t)Q->setup.size() > INT32_MAX || (int64_t)Q->frow.size() > INT32_MAX)
    return fail(TACHO_ERR_INVALID, "too many partitioned-inverse tiles");
  HIP_TRY(upload(h->dq_setup, Q->setup));
  HIP_TRY(upload(h->dq_tiles, Q->tiles));
  HIP_TRY(upload(h->dq_frow, Q->frow));
  HIP_TRY(upload(h->dq_bcol, Q->bcol));
  HIP_TRY(upload(h->dq_fsum, Q->fsum));
  HIP_TRY(upload(h->dq_bsum, Q->bsum));
  HIP_TRY(upload(h->dq_small, Q->small));
  HIP_TRY(upload(h->dq_large, Q->large));
  h->Q = std::move(Q);
  return TACHO_OK;
}

size_t elem_size(int precision) { return precision == TACHO_FP32 ? 4 : 8; }

bool valid_precision(int precision) {
  return precision == TACHO_FP64 || precision == TACHO_FP32 || precision == TACHO_LDLT ||
         precision == TACHO_LU;
}

// Device bytes a numeric handle needs (factor, update workspace, values,
// solve workspace for kRhs columns).
// Dataflow factorization: one completion flag per row tile, one
// pre-accumulation flag per pivot block, one counter per update-matrix tile,
// one ticket counter per level, one hang flag.
int64_t flow_ntiles(const tacho_sym* h) { return h->P.tbase.empty() ? 0 : h->P.tbase.back(); }
int64_t flow_ints(const tacho_sym* h) {
  return flow_ntiles(h) + (int64_t)h->P.woff.size() + h->P.nucount + h->P.front_launches + 1;
}

// Dataflow solves: three completion counters per supernode, one
// partial-product counter per diagonal block, two tickets, then the hang
// flag (cleared once, when the handle is created).
int64_t solve_counters(const tacho_sym* h) { return 3 * (int64_t)h->S.ns + (int64_t)h->P.woff.size() + 2; }

int64_t numeric_bytes(const tacho_sym* h, int precision) {
  const size_t es = elem_size(precision);
  const Symbolic& S = h->S;
  const Plan& P = h->P;
  int64_t b = 0;
  b += (int64_t)es * P.L_elems + (int64_t)es * P.U_elems + (int64_t)es * (int64_t)S.a_src.size();
  b += 8 * S.nnz_input + 4;
  b += (int64_t)kRowBytes * (S.n + P.u_elems);
  b += (int64_t)es * std::max<int64_t>(P.part_slots, 1) * kPanel * kRhs;
  b += (int64_t)es * P.W_elems;
  b += (int64_t)es * kPanel * kPanel * P.pt1_slots;
  b += 4 * (solve_counters(h) + 1);
  b += 4 * flow_ints(h);
  if (precision == TACHO_FP32) b += 8 * (int64_t)S.A.colind.size() + 8 * S.n;  // values, scaling
  if (precision == TACHO_LDLT) b += 8 * h->P.L_elems + 16 * S.n + 16 * S.n;    // L D, D, orders
  if (precision == TACHO_LU)  // U^T panels and update halves, upper values and maps, V blocks, orders
    b += 8 * h->P.L_elems + 8 * h->P.U_elems + 24 * (int64_t)S.a_src.size() + 8 * P.W_elems + 16 * S.n;
  return b;
}

template <typename T>
DevNum<T> num_view(tacho_num* f) {
  DevNum<T> N;
  N.L = f->L.as<T>();
  N.U = f->U.as<T>();
  N.avals = f->avals.as<T>();
  N.scale = f->precision == TACHO_FP32 && f->sym->opt.scale_fp32 ? f->scale.as<double>() : nullptr;
  N.fail = f->fail.as<int32_t>();
  N.pt1 = f->pt1.as<T>();
  return N;
}

int step_kind(int kind) {
  switch (kind) {
    case kStepSmall: return TACHO_K_SMALL_FRONT;
    case kStepAssemble: return TACHO_K_ASSEMBLE;
    case kStepDiag: return TACHO_K_DIAG;
    case kStepPanel: return TACHO_K_PANEL;
    case kStepFront: return TACHO_K_FRONT;
    default: return TACHO_K_UPDATE;
  }
}

template <typename T>
void run_factor_steps(tacho_num* f, hipStream_t st) {
  tacho_sym* h = f->sym;
  const DevSym& S = h->view;
  const Plan& P = h->P;
  DevNum<T> N = num_view<T>(f);
  const int32_t* small = h->d_small.as<int32_t>();
  const AsmItem* asmi = h->d_asm.as<AsmItem>();
  const PanelItem* dia = h->d_diag.as<PanelItem>();
  const PanelItem* pan = h->d_panel.as<PanelItem>();
  const GemmProb* probs = h->d_probs.as<GemmProb>();
  const GemmTile* tiles = h->d_tiles.as<GemmTile>();
  const FrontTask* ftasks = h->d_ftasks.as<FrontTask>();
  const int64_t ntiles = flow_ntiles(h);
  for (const Step& s : P.steps) {
    const int64_t cnt = s.end - s.begin;
    const int pe = f->prof.begin(st);
    switch (s.kind) {
      case kStepSmall:
        launch_leaf<T>(S, N, small + s.begin, s.tile, st);
        launch_small<T>(S, N, small + s.begin + s.tile, s.packed - s.begin - s.tile, st);
        launch_packed<T>(S, N, f->winv.as<T>(), small + s.packed, s.packed_big - s.packed, false, st);
        launch_packed<T>(S, N, f->winv.as<T>(), small + s.packed_big, s.end - s.packed_big, true, st);
        break;
      case kStepAssemble: launch_assemble<T>(S, N, asmi + s.begin, cnt, st); break;
      case kStepDiag: launch_diag<T>(S, N, dia + s.begin, cnt, f->winv.as<T>(), st); break;
      case kStepPanel: launch_panel<T>(S, N, pan + s.begin, cnt, f->winv.as<T>(), st); break;
      case kStepGemm: launch_gemm<T>(N, probs, tiles + s.begin, cnt, s.tile, st); break;
      case kStepFront:
        launch_front<T>(S, N, f->winv.as<T>(), ftasks + s.begin, cnt, f->flow.as<int32_t>(), ntiles,
                        (int64_t)P.woff.size(), P.nucount, s.ticket, P.front_launches, st);
        break;
    }
    f->prof.end(pe, st, step_kind(s.kind), s.flops, s.elems * sizeof(T));
  }
}

// LDL^T: the stepwise plan's launches with the LDL^T kernels for the small
// fronts, the diagonal blocks and the panels; the trailing updates subtract
// L (L D)^T.
void run_ldlt_steps(tacho_num* f, hipStream_t st) {
  tacho_sym* h = f->sym;
  const DevSym& S = h->view1;
  const Plan& P = *h->P1;
  DevNum<double> N = num_view<double>(f);
  DevLdlt D{f->ld_d.as<double>(), f->ld_e.as<double>(), f->ld_q.as<int32_t>(),
            f->ld_panels.as<double>()};
  const int32_t* small = h->d1_small.as<int32_t>();
  const AsmItem* asmi = h->d1_asm.as<AsmItem>();
  const PanelItem* dia = h->d1_diag.as<PanelItem>();
  const PanelItem* pan = h->d1_panel.as<PanelItem>();
  const GemmProb* probs = h->d1_probs.as<GemmProb>();
  const GemmTile* tiles = h->d1_tiles.as<GemmTile>();
  launch_iota(D.q, h->S.n, st);
  for (const Step& s : P.steps) {
    const int64_t cnt = s.end - s.begin;
    const int pe = f->prof.begin(st);
    switch (s.kind) {
      case kStepSmall: launch_small_ldlt(S, N, D, small + s.begin, cnt, st); break;
      case kStepAssemble: launch_assemble<double>(S, N, asmi + s.begin, cnt, st); break;
      case kStepDiag: launch_diag_ldlt(S, N, D, dia + s.begin, cnt, f->winv.as<double>(), st); break;
      case kStepPanel: launch_panel_ldlt(S, N, D, pan + s.begin, cnt, f->winv.as<double>(), st); break;
      case kStepGemm: launch_gemm<double>(N, probs, tiles + s.begin, cnt, s.tile, st, D.ld); break;
      default: break;
    }
    f->prof.end(pe, st, step_kind(s.kind), s.flops, s.elems * sizeof(double));
  }
  launch_ldlt_perm(h->S.n, h->d_perm.as<int32_t>(), D.q, f->ld_perm.as<int32_t>(),
                   f->ld_pinv.as<int32_t>(), f->ld_qinv.as<int32_t>(), st);
}

// LU: the stepwise plan's launches with the LU kernels; assembly and
// trailing updates run once for the L half and once for the U^T half
// (C -= L (U^T)^T there, C -= U^T L^T here).
void run_lu_steps(tacho_num* f, hipStream_t st) {
  tacho_sym* h = f->sym;
  const DevSym& S = h->view1;
  const Plan& P = *h->P1;
  DevNum<double> N = num_view<double>(f);
  DevNum<double> Nt = N;
  Nt.L = f->lu_t.as<double>();
  Nt.U = f->lu_u2.as<double>();
  Nt.avals = f->lu_avals.as<double>();
  int32_t* q = f->ld_q.as<int32_t>();
  double* winv = f->winv.as<double>();
  double* vinv = f->lu_vinv.as<double>();
  const int32_t* small = h->d1_small.as<int32_t>();
  const AsmItem* asmi = h->d1_asm.as<AsmItem>();
  const PanelItem* dia = h->d1_diag.as<PanelItem>();
  const PanelItem* pan = h->d1_panel.as<PanelItem>();
  const GemmProb* probs = h->d1_probs.as<GemmProb>();
  const GemmTile* tiles = h->d1_tiles.as<GemmTile>();
  launch_iota(q, h->S.n, st);
  for (const Step& s : P.steps) {
    const int64_t cnt = s.end - s.begin;
    const int pe = f->prof.begin(st);
    double mult = 1.0;
    switch (s.kind) {
      case kStepSmall: launch_small_lu(S, N, Nt, q, small + s.begin, cnt, st); break;
      case kStepAssemble:
        launch_assemble<double>(S, N, asmi + s.begin, cnt, st);
        launch_assemble<double>(S, Nt, asmi + s.begin, cnt, st);
        mult = 2.0;
        break;
      case kStepDiag: launch_diag_lu(S, N, Nt, q, dia + s.begin, cnt, winv, vinv, st); break;
      case kStepPanel:
        launch_panel_lu(S, N, Nt, q, pan + s.begin, cnt, winv, vinv, st);
        mult = 2.0;
        break;
      case kStepGemm:
        launch_gemm<double>(N, probs, tiles + s.begin, cnt, s.tile, st, Nt.L, &Nt, N.L);
        mult = 2.0;
        break;
      default: break;
    }
    f->prof.end(pe, st, step_kind(s.kind), mult * s.flops, mult * s.elems * sizeof(double));
  }
  launch_lu_rowperm(S, N, q, dia, (int64_t)P.diag_items.size(), st);
  launch_ldlt_perm(h->S.n, h->d_perm.as<int32_t>(), q, f->ld_perm.as<int32_t>(),
                   f->ld_pinv.as<int32_t>(), f->ld_qinv.as<int32_t>(), st);
}

int refactor(tacho_num* f, const double* values, int on_device, hipStream_t st, int sync,
             int64_t* fail_index);
int fp64_fallback(tacho_num* f, hipStream_t st, int64_t* fail_index);

int read_fail_flag(tacho_num* f, int64_t* fail_index, bool may_allocate = true) {
  int32_t flag = INT32_MAX, hang = 0;
  HIP_TRY(hipMemcpyAsync(&flag, f->fail.p, sizeof(int32_t), hipMemcpyDeviceToHost, f->last_stream));
  if (!f->sym->P.ftasks.empty() && f->precision != TACHO_LDLT && f->precision != TACHO_LU)
    HIP_TRY(hipMemcpyAsync(&hang, f->flow.as<int32_t>() + flow_ints(f->sym) - 1, sizeof(int32_t),
                           hipMemcpyDeviceToHost, f->last_stream));
  HIP_TRY(hipStreamSynchronize(f->last_stream));
  f->pending = false;
  if (hang != 0) {
    f->last_status = TACHO_ERR_HIP;
    return fail(TACHO_ERR_HIP, "dataflow factorization: a dependency wait timed out");
  }
  if (flag != INT32_MAX && f->precision == TACHO_FP32) {
    // FP32 pivot breakdown: the FP64 factorization of the same values on the
    // same symbolic handle serves the solves of the system that broke down
    // (reported as a fallback); the other systems of a batch keep their FP32
    // factors, which do not depend on it.
    f->fp32_fail_col = flag;
    int64_t fi = -1;
    if (!f->fallback && !may_allocate) {
      f->last_status = TACHO_ERR_NOMEM;
      return fail(TACHO_ERR_NOMEM, "the FP32 factorization broke down and its FP64 fallback "
                                   "factor would need device memory; use tacho_solve");
    }
    const int rc = fp64_fallback(f, f->last_stream, &fi);
    f->last_status = rc;
    f->last_fail = rc == TACHO_OK ? -1 : fi;
    if (fail_index) *fail_index = f->last_fail;
    if (rc == TACHO_OK) f->fp32_broken = true;
    return rc;
  }
  if (flag != INT32_MAX && (f->precision == TACHO_LDLT || f->precision == TACHO_LU)) {
    f->last_fail = f->sym->S.perm[flag];
    f->last_status = TACHO_ERR_SINGULAR;
    if (fail_index) *fail_index = f->last_fail;
    return fail(TACHO_ERR_SINGULAR, "no usable pivot within the diagonal block of column " +
                                        std::to_string(f->last_fail));
  }
  if (flag != INT32_MAX) {
    f->last_fail = f->sym->S.perm[flag];
    f->last_status = TACHO_ERR_NOT_SPD;
    if (fail_index) *fail_index = f->last_fail;
    return fail(TACHO_ERR_NOT_SPD, "matrix is not positive definite (pivot " +
                                       std::to_string(f->last_fail) + ")");
  }
  f->last_fail = -1;
  f->last_status = TACHO_OK;
  if (fail_index) *fail_index = -1;
  return TACHO_OK;
}

int ensure_level_csr(tacho_sym* h) {
  std::lock_guard<std::mutex> lock(h->mu);
  if (h->C) return TACHO_OK;
  if (2 * h->S.n >= (int64_t)INT32_MAX)
    return fail(TACHO_ERR_INVALID, "the level CSR form needs 2 n below 2^31");
  std::unique_ptr<LevelCsr> C(new LevelCsr());
  build_level_csr(h->S, *C);
  HIP_TRY(upload(h->dc_rows, C->rows));
  HIP_TRY(upload(h->dc_rptr, C->rptr));
  HIP_TRY(upload(h->dc_segs, C->segs));
  h->C = std::move(C);
  return TACHO_OK;
}

// Partitioned-inverse setup for the factor in f: Z = [I; L21] per front,
// then the right-to-left block-column steps of the plan.
template <typename T>
void run_pinv_setup(tacho_num* f, hipStream_t st) {
  tacho_sym* h = f->sym;
  const PinvPlan& Q = *h->Q;
  const DevSym& S = h->view;
  T* Z = f->Z.as<T>();
  const T* L = f->L.as<T>();
  const int pe = f->prof.begin(st);
  launch_pinv_init<T>(S, Z, L, h->dq_tiles.as<FrontTile>(), (int64_t)Q.tiles.size(), st);
  const PinvTask* tasks = h->dq_setup.as<PinvTask>();
  for (size_t q = 0; q + 1 < Q.setup_ptr.size(); ++q)
    launch_pinv_step<T>(S, Z, L, f->winv.as<T>(), tasks + Q.setup_ptr[q],
                        Q.setup_ptr[q + 1] - Q.setup_ptr[q], st);
  f->prof.end(pe, st, TACHO_K_PINV, Q.flops, 3.0 * sizeof(T) * (double)h->P.L_elems);
  if (f->solve_variant == TACHO_SOLVE_LEVEL_CSR || f->csr_pending) {
    const LevelCsr& C = *h->C;
    const int pc = f->prof.begin(st);
    launch_csr_fill<T>(S, Z, h->dc_segs.as<CsrSeg>(), (int64_t)C.segs.size(), f->ccols.as<int32_t>(),
                       f->cvals.as<T>(), st);
    f->prof.end(pc, st, TACHO_K_PINV, 0, (sizeof(T) * 2.0 + 4.0) * (double)C.nnz);
  }
}

// Device work of one factorization after the values are resident: failure
// flag reset, value gather (and for FP32 the scaling and the FP64 values of
// the refinement residual), then every level's launches.
void enqueue_factor(tacho_num* f, hipStream_t st) {
  tacho_sym* h = f->sym;
  const Symbolic& S = h->S;
  launch_fill_i32(f->fail.as<int32_t>(), INT32_MAX, 1, st);
  if (!h->P.ftasks.empty()) launch_fill_i32(f->flow.as<int32_t>(), 0, flow_ints(h), st);
  const double* vals = f->vals.as<double>();
  const int64_t nq = (int64_t)S.a_src.size();
  if (f->precision == TACHO_FP32) {
    launch_mirror(h->d_mirror.as<int64_t>(), vals, f->fullvals.as<double>(),
                  (int64_t)S.A.colind.size(), st);
    if (h->opt.scale_fp32) launch_scale(h->view, vals, f->scale.as<double>(), st);
    const int pe = f->prof.begin(st);
    launch_gather<float>(h->view, num_view<float>(f), vals, nq, st);
    f->prof.end(pe, st, TACHO_K_GATHER, 0, nq * (8.0 + 8.0 + 4.0));
    run_factor_steps<float>(f, st);
  } else {
    const int pe = f->prof.begin(st);
    DevSym G = h->view;
    if (f->precision == TACHO_LU) G.a_src = h->d_lu_lo.as<int64_t>();
    launch_gather<double>(G, num_view<double>(f), vals, nq, st);
    if (f->precision == TACHO_LU) {
      DevNum<double> Nt = num_view<double>(f);
      Nt.avals = f->lu_avals.as<double>();
      G.a_src = h->d_lu_up.as<int64_t>();
      launch_gather<double>(G, Nt, vals, nq, st);
    }
    f->prof.end(pe, st, TACHO_K_GATHER, 0,
                (f->precision == TACHO_LU ? 2.0 : 1.0) * nq * (8.0 + 8.0 + 8.0));
    if (f->precision == TACHO_LDLT)
      run_ldlt_steps(f, st);
    else if (f->precision == TACHO_LU)
      run_lu_steps(f, st);
    else
      run_factor_steps<double>(f, st);
  }
}

// The factorization's launch sequence captured once into a graph on a
// private stream; replays go to the caller's stream.
int build_factor_graph(tacho_num* f) {
  hipStream_t cs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    enqueue_factor(f, cs);
    e = hipStreamEndCapture(cs, &g);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&f->fgraph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    f->fgraph = nullptr;
    return fail(TACHO_ERR_HIP, std::string("factorization graph: ") + hipGetErrorString(e));
  }
  return TACHO_OK;
}

int refactor(tacho_num* f, const double* values, int on_device, hipStream_t st, int sync,
             int64_t* fail_index) {
  tacho_sym* h = f->sym;
  const Symbolic& S = h->S;
  const int64_t nv = S.nnz_input;
  if (nv > 0 && !values) return fail(TACHO_ERR_INVALID, "values is NULL");
  f->fp32_broken = false;
  f->fp32_fail_col = -1;
  if (nv > 0)
    HIP_TRY(hipMemcpyAsync(f->vals.p, values, nv * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(f->ev[0], st));
  if (h->opt.graphs != 0 && !f->prof.on && f->precision != TACHO_LDLT && f->precision != TACHO_LU) {
    if (!f->fgraph) {
      const int rc = build_factor_graph(f);
      if (rc != TACHO_OK) return rc;
    }
    HIP_TRY(hipGraphLaunch(f->fgraph, st));
  } else {
    enqueue_factor(f, st);
  }
  HIP_TRY(hipEventRecord(f->ev[1], st));
  if (f->solve_variant == TACHO_SOLVE_PARTITIONED_INVERSE || f->solve_variant == TACHO_SOLVE_LEVEL_CSR) {
    if (f->precision == TACHO_FP32)
      run_pinv_setup<float>(f, st);
    else
      run_pinv_setup<double>(f, st);
  }
  HIP_TRY(hipGetLastError());
  f->pending = true;
  f->last_stream = st;
  if (sync) return read_fail_flag(f, fail_index);
  return TACHO_OK;
}

int create_numeric(tacho_sym* h, int precision, tacho_num** out) {
  int rc = ensure_uploaded(h);
  if (rc != TACHO_OK) return rc;
  const Symbolic& S = h->S;
  const Plan& P = h->P;
  const int64_t need = numeric_bytes(h, precision);
  if (h->opt.hbm_budget_bytes > 0 && (uint64_t)need > h->opt.hbm_budget_bytes)
    return fail(TACHO_ERR_NOMEM, "numeric handle needs " + std::to_string(need) +
                                     " bytes, over the HBM budget");
  std::unique_ptr<tacho_num> f(new tacho_num());
  f->sym = h;
  f->precision = precision;
  const size_t es = elem_size(precision);
  HIP_TRY(f->L.alloc(es * P.L_elems));
  HIP_TRY(f->U.alloc(es * P.U_elems));
  HIP_TRY(f->avals.alloc(es * S.a_src.size()));
  HIP_TRY(f->vals.alloc(sizeof(double) * S.nnz_input));
  HIP_TRY(f->fail.alloc(sizeof(int32_t)));
  HIP_TRY(f->winv.alloc(es * std::max<int64_t>(P.W_elems, 1)));
  HIP_TRY(f->pt1.alloc(es * kPanel * kPanel * std::max<int64_t>(P.pt1_slots, 1)));
  HIP_TRY(f->y.alloc((size_t)kRowBytes * S.n));
  HIP_TRY(f->uvec.alloc((size_t)kRowBytes * std::max<int64_t>(P.u_elems, 1)));
  HIP_TRY(f->part.alloc(es * std::max<int64_t>(P.part_slots, 1) * kPanel * kRhs));
  HIP_TRY(f->sync.alloc(sizeof(int32_t) * (solve_counters(h) + 1)));
  HIP_TRY(clear_device(f->sync.p, sizeof(int32_t) * (solve_counters(h) + 1)));
  HIP_TRY(f->flow.alloc(sizeof(int32_t) * flow_ints(h)));
  if (precision == TACHO_FP32) {
    HIP_TRY(f->scale.alloc(sizeof(double) * S.n));
    HIP_TRY(f->fullvals.alloc(sizeof(double) * S.A.colind.size()));
  }
  for (auto& e : f->ev) HIP_TRY(hipEventCreate(&e));
  if (precision == TACHO_FP32) f->rh.resize(S.nsys * kRhs);
  if (precision == TACHO_LDLT) {
    rc = ensure_stepwise(h);
    if (rc != TACHO_OK) return rc;
    HIP_TRY(f->ld_d.alloc(sizeof(double) * S.n));
    HIP_TRY(f->ld_e.alloc(sizeof(double) * S.n));
    HIP_TRY(f->ld_q.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->ld_qinv.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->ld_perm.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->ld_pinv.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->ld_panels.alloc(sizeof(double) * std::max<int64_t>(P.L_elems, 1)));
  }
  if (precision == TACHO_LU) {
    rc = ensure_stepwise(h);
    if (rc != TACHO_OK) return rc;
    rc = ensure_lu_maps(h);
    if (rc != TACHO_OK) return rc;
    HIP_TRY(f->ld_q.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->ld_qinv.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->ld_perm.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->ld_pinv.alloc(sizeof(int32_t) * S.n));
    HIP_TRY(f->lu_t.alloc(sizeof(double) * std::max<int64_t>(P.L_elems, 1)));
    HIP_TRY(f->lu_u2.alloc(sizeof(double) * std::max<int64_t>(P.U_elems, 1)));
    HIP_TRY(f->lu_avals.alloc(sizeof(double) * std::max<size_t>(S.a_src.size(), 1)));
    HIP_TRY(f->lu_vinv.alloc(sizeof(double) * std::max<int64_t>(P.W_elems, 1)));
  }
  *out = f.release();
  return TACHO_OK;
}

// FP64 refactorization of an FP32 handle's values on the same symbolic
// handle, used after an FP32 pivot breakdown or a refinement stall.
int fp64_fallback(tacho_num* f, hipStream_t st, int64_t* fail_index) {
  if (!f->fallback) {
    tacho_num* g = nullptr;
    const int rc = create_numeric(f->sym, TACHO_FP64, &g);
    if (rc != TACHO_OK) return rc;
    f->fallback = g;
  }
  return refactor(f->fallback, f->vals.as<double>(), 1, st, 1, fail_index);
}

// Error if a wait of this handle's dataflow solves (or of its FP64
// fallback's) timed out.  Synchronizes st.  A raised flag is reported once
// and then cleared, so the handle's next solve waits normally again.
int check_solve_hang(tacho_num* f, hipStream_t st) {
  int32_t hang[2] = {0, 0};
  int32_t* flags[2] = {f->sync.as<int32_t>() + solve_counters(f->sym),
                       f->fallback ? f->fallback->sync.as<int32_t>() + solve_counters(f->sym)
                                   : nullptr};
  HIP_TRY(hipMemcpyAsync(&hang[0], flags[0], sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (flags[1])
    HIP_TRY(hipMemcpyAsync(&hang[1], flags[1], sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  f->solve_queued = false;
  if (hang[0] || hang[1]) {
    for (int k = 0; k < 2; ++k)
      if (hang[k]) launch_fill_i32(flags[k], 0, 1, st);
    HIP_TRY(hipStreamSynchronize(st));
    return fail(TACHO_ERR_HIP, "dataflow solve: a dependency wait timed out");
  }
  return TACHO_OK;
}

// One sweep of forward + backward substitution for up to kRhs columns,
// b (FP64, ld ldb) -> x (FP64, ld ldx), x += result when accumulate.
template <typename T>
void solve_sweep(tacho_num* f, const double* b, int64_t ldb, double* x, int64_t ldx, int nrhs,
                 int accumulate, hipStream_t st) {
  tacho_sym* h = f->sym;
  const Symbolic& S = h->S;
  // LDL^T: the sweeps apply each block's pivot order (lq, lqinv) to their
  // front vectors; the result comes out in pivot order, so the output
  // permutation is P composed with it
  DevSym Vq = h->view, Vout = h->view;
  if (f->precision == TACHO_LDLT || f->precision == TACHO_LU) {
    Vq.lq = f->ld_q.as<int32_t>();
    Vq.lqinv = f->ld_qinv.as<int32_t>();
    Vout.perm = f->ld_perm.as<int32_t>();
    Vout.pinv = f->ld_pinv.as<int32_t>();
  }
  // LU: the forward sweeps take the pivot rows in pivot order (L, W); the
  // backward sweeps run on U^T with V = (U_kk^T)^{-1}, read the ancestors'
  // solutions in the analysis order and leave the result in that order
  DevSym Vb = Vq;
  if (f->precision == TACHO_LU) {
    Vq.lqinv = nullptr;
    Vb.lq = nullptr;
    Vb.lqinv = nullptr;
    Vout = h->view;
  }
  const DevSym& V = Vq;
  const Plan& P = h->P;
  const double* scale = f->precision == TACHO_FP32 && h->opt.scale_fp32 ? f->scale.as<double>() : nullptr;
  T* y = f->y.as<T>();
  const T* L = f->L.as<T>();
  const T* winv = f->winv.as<T>();
  const T* Lb = L;
  const T* winvb = winv;
  if (f->precision == TACHO_LU) {
    Lb = f->lu_t.as<T>();
    winvb = f->lu_vinv.as<T>();
  }
  const double es = sizeof(T);
  const int width = nrhs == 1 ? 1 : kRhs;  // values per row of y and of the update vectors
  const int64_t ns = S.ns, nblk = (int64_t)P.woff.size();
  int32_t* counters = f->sync.as<int32_t>();
  int32_t* hang = counters + solve_counters(h);
  const int32_t* waves = h->d_wave_list.as<int32_t>();
  double lentries = 0, rows = 0;
  for (int32_t lvl = 0; lvl < S.nlevels; ++lvl) {
    lentries += P.level_lentries[lvl];
    rows += P.level_rows[lvl];
  }
  int pe = f->prof.begin(st);
  launch_solve_in<T>(V, b, ldb, y, nrhs, scale, counters, ns, nblk, st);
  // test hook: raise the hang flag so that every dependency wait of this
  // sweep gives up at once (the kernels still run to the end)
  if (h->opt.debug_flags & TACHO_DEBUG_SOLVE_GIVE_UP) launch_fill_i32(hang, 1, 1, st);
  f->prof.end(pe, st, TACHO_K_PERMUTE, 0, (double)S.n * (8.0 * nrhs + es * width) + 4.0 * S.n);
  if (f->solve_variant == TACHO_SOLVE_LEVEL_CSR) {
    // one CSR product per level and sweep on the whole solve vector:
    // forward, the level's ancestor rows of y get the -Z21 y terms and its
    // pivot rows Z11 y go to yfwd; backward, x = Z11^T yfwd - Z21^T x for
    // the level's pivot rows, back into y
    const LevelCsr& C = *h->C;
    const int32_t* rws = h->dc_rows.as<int32_t>();
    const int64_t* rp = h->dc_rptr.as<int64_t>();
    const int32_t* cc = f->ccols.as<int32_t>();
    const T* cv = f->cvals.as<T>();
    T* yf = f->yfwd.as<T>();
    const int64_t n = S.n;
    pe = f->prof.begin(st);
    for (int32_t lvl = 0; lvl < S.nlevels; ++lvl) {
      launch_level_spmv<T>(rws, rp, cc, cv, C.fwd_ptr[2 * lvl], C.fwd_ptr[2 * lvl + 1], n, y, y, y, true,
                           nrhs, st);
      launch_level_spmv<T>(rws, rp, cc, cv, C.fwd_ptr[2 * lvl + 1], C.fwd_ptr[2 * lvl + 2], n, y, y, yf,
                           false, nrhs, st);
    }
    const double half = (double)C.nnz / 2;  // about half the entries per sweep
    f->prof.end(pe, st, TACHO_K_FORWARD, 2.0 * half * nrhs, (es + 4.0) * half + es * 2.0 * rows * nrhs);
    pe = f->prof.begin(st);
    for (int32_t lvl = S.nlevels - 1; lvl >= 0; --lvl)
      launch_level_spmv<T>(rws, rp, cc, cv, C.b_ptr[lvl], C.b_ptr[lvl + 1], n, yf, y, y, false, nrhs, st);
    f->prof.end(pe, st, TACHO_K_BACKWARD, 2.0 * half * nrhs, (es + 4.0) * half + es * 2.0 * rows * nrhs);
    pe = f->prof.begin(st);
    launch_solve_out<T>(Vout, y, x, ldx, nrhs, scale, accumulate, st);
    f->prof.end(pe, st, TACHO_K_PERMUTE, 0, (double)S.n * (8.0 * nrhs + es * width) + 4.0 * S.n);
    return;
  }
  if (f->solve_variant == TACHO_SOLVE_PARTITIONED_INVERSE) {
    // one gather and one merged product per level and sweep; the forward
    // result goes to yfwd, the solution back into y
    const PinvPlan& Q = *h->Q;
    const T* Z = f->Z.as<T>();
    T* yf = f->yfwd.as<T>();
    T* uv = f->uvec.as<T>();
    const int32_t* sm = h->dq_small.as<int32_t>();
    const int32_t* lg = h->dq_large.as<int32_t>();
    const PinvSweepTask* fr = h->dq_frow.as<PinvSweepTask>();
    const PinvSweepTask* bc = h->dq_bcol.as<PinvSweepTask>();
    const PinvSweepTask* fs = h->dq_fsum.as<PinvSweepTask>();
    const PinvSweepTask* bs = h->dq_bsum.as<PinvSweepTask>();
    T* part = f->zpart.as<T>();
    pe = f->prof.begin(st);
    for (int32_t lvl = 0; lvl < S.nlevels; ++lvl) {
      launch_pinv_small<T>(V, Z, y, yf, uv, sm + Q.small_ptr[lvl], Q.small_ptr[lvl + 1] - Q.small_ptr[lvl],
                           true, nrhs, st);
      launch_pinv_fwd<T>(V, Z, y, yf, uv, lg + Q.large_ptr[lvl], Q.large_ptr[lvl + 1] - Q.large_ptr[lvl],
                         Q.gchunks[lvl], fr + Q.frow_ptr[lvl], Q.frow_ptr[lvl + 1] - Q.frow_ptr[lvl],
                         fs + Q.fsum_ptr[lvl], Q.fsum_ptr[lvl + 1] - Q.fsum_ptr[lvl], part, nrhs, st);
    }
    f->prof.end(pe, st, TACHO_K_FORWARD, 2.0 * lentries * nrhs, es * (lentries + 2.0 * rows * nrhs));
    pe = f->prof.begin(st);
    for (int32_t lvl = S.nlevels - 1; lvl >= 0; --lvl) {
      launch_pinv_small<T>(V, Z, y, yf, uv, sm + Q.small_ptr[lvl], Q.small_ptr[lvl + 1] - Q.small_ptr[lvl],
                           false, nrhs, st);
      launch_pinv_bwd<T>(V, Z, yf, y, bc + Q.bcol_ptr[lvl], Q.bcol_ptr[lvl + 1] - Q.bcol_ptr[lvl],
                         bs + Q.bsum_ptr[lvl], Q.bsum_ptr[lvl + 1] - Q.bsum_ptr[lvl], part, nrhs, st);
    }
    f->prof.end(pe, st, TACHO_K_BACKWARD, 2.0 * lentries * nrhs, es * (lentries + 2.0 * rows * nrhs));
    pe = f->prof.begin(st);
    launch_solve_out<T>(Vout, y, x, ldx, nrhs, scale, accumulate, st);
    f->prof.end(pe, st, TACHO_K_PERMUTE, 0, (double)S.n * (8.0 * nrhs + es * width) + 4.0 * S.n);
    return;
  }
  const WaveItem* items = h->d_lwave.as<WaveItem>();
  const int32_t* large = h->d_llarge.as<int32_t>();
  pe = f->prof.begin(st);
  for (int32_t lvl = 0; lvl < P.solve_split; ++lvl)
    launch_level_fwd<T>(V, L, winv, y, f->uvec.as<T>(), items + P.lwave_ptr[lvl],
                        P.lwave_ptr[lvl + 1] - P.lwave_ptr[lvl], large + P.llarge_ptr[lvl],
                        P.llarge_ptr[lvl + 1] - P.llarge_ptr[lvl], waves, nrhs, counters, ns, nblk,
                        hang, st);
  launch_solve_fwd<T>(V, L, winv, y, f->uvec.as<T>(), h->d_fsolve.as<SolveTask>(),
                      (int64_t)P.fsolve.size(), waves, nrhs, counters, ns, nblk, hang, st);
  f->prof.end(pe, st, TACHO_K_FORWARD, 2.0 * lentries * nrhs, es * (lentries + 2.0 * rows * nrhs));
  if constexpr (std::is_same<T, double>::value)
    if (f->precision == TACHO_LDLT)
      launch_apply_dinv(S.n, f->ld_d.as<double>(), f->ld_e.as<double>(), y, nrhs, st);
  pe = f->prof.begin(st);
  launch_solve_bwd<T>(Vb, Lb, winvb, y, f->part.as<T>(), h->d_bsolve.as<SolveTask>(),
                      (int64_t)P.bsolve.size(), waves, nrhs, counters, ns, nblk, hang, st);
  for (int32_t lvl = P.solve_split - 1; lvl >= 0; --lvl)
    launch_level_bwd<T>(Vb, Lb, winvb, y, f->part.as<T>(), items + P.lwave_ptr[lvl],
                        P.lwave_ptr[lvl + 1] - P.lwave_ptr[lvl], large + P.llarge_ptr[lvl],
                        P.llarge_ptr[lvl + 1] - P.llarge_ptr[lvl], waves, nrhs, counters, ns, nblk,
                        hang, st);
  f->prof.end(pe, st, TACHO_K_BACKWARD, 2.0 * lentries * nrhs, es * (lentries + 2.0 * rows * nrhs));
  pe = f->prof.begin(st);
  launch_solve_out<T>(Vout, y, x, ldx, nrhs, scale, accumulate, st);
  f->prof.end(pe, st, TACHO_K_PERMUTE, 0, (double)S.n * (8.0 * nrhs + es * width) + 4.0 * S.n);
}

template <typename T>
void solve_all(tacho_num* f, const double* b, int64_t ldb, double* x, int64_t ldx, int64_t nrhs,
               int accumulate, hipStream_t st) {
  for (int64_t c = 0; c < nrhs; c += kRhs) {
    const int nb = (int)std::min<int64_t>(kRhs, nrhs - c);
    solve_sweep<T>(f, b + c * ldb, ldb, x + c * ldx, ldx, nb, accumulate, st);
  }
}

// Device scratch of one refinement: residual r (n x nrhs), per-unit norms
// (2 x units) and a per-unit byte mask.
struct RefineScratch {
  double* r = nullptr;
  double* xt = nullptr;  // the iterate by rows (several right-hand sides)
  double* nrm = nullptr;
  double* npart = nullptr;  // partial sums of the norms
  uint8_t* mask = nullptr;
};

int64_t refine_scratch_bytes(int64_t n, int64_t nrhs, int64_t nsys) {
  const int64_t units = nsys * nrhs;
  const int64_t rows = nrhs > 1 ? n * nrhs : 0;
  return (int64_t)sizeof(double) * (n * nrhs + rows + (2 + kNormParts) * units) + units;
}

RefineScratch carve_refine_scratch(void* base, int64_t n, int64_t nrhs, int64_t nsys) {
  RefineScratch w;
  w.r = static_cast<double*>(base);
  w.xt = w.r + n * nrhs;
  w.nrm = w.xt + (nrhs > 1 ? n * nrhs : 0);
  w.npart = w.nrm + 2 * nsys * nrhs;
  w.mask = reinterpret_cast<uint8_t*>(w.npart + kNormParts * nsys * nrhs);
  return w;
}

// FP32 factor + FP64 refinement on device buffers b (ld n) -> x (ld n).
// Convergence is tracked per independent system and right-hand side (one
// unit each): a converged unit gets a zero correction from then on, and a
// unit that stalls (or whose system's FP32 factorization broke down) takes
// the FP64 factor's solution while the others keep their refined FP32
// results, so a system's result does not depend on the other systems of a
// batch.  The host bookkeeping lives in the handle (sized for 16 columns when
// the handle is created).
int refine_solve(tacho_num* f, const double* b, double* x, int64_t nrhs, hipStream_t st,
                 tacho_solve_info* info, const RefineScratch& ws, bool may_allocate) {
  tacho_sym* h = f->sym;
  const Symbolic& S = h->S;
  const int64_t n = S.n;
  const int64_t nsys = S.nsys;
  const int64_t units = nsys * nrhs;
  double* r = ws.r;
  double* nrm = ws.nrm;
  uint8_t* mask = ws.mask;
  const int64_t* sysp = h->d_sys_ptr.as<int64_t>();
  RefineHost& H = f->rh;
  if ((int64_t)H.rho.size() < units) {
    if (!may_allocate) return fail(TACHO_ERR_INVALID, "too many right-hand sides for this call");
    H.resize(units);
  }
  double* hn = H.hn.data();
  double* rho = H.rho.data();
  for (int64_t u = 0; u < units; ++u) {
    H.prev[u] = INFINITY;
    H.stalls[u] = 0;
    H.done[u] = 0;
    H.bad[u] = 0;
  }
  if (f->fp32_broken) {
    // the system holding the first failing pivot goes to the FP64 factor at
    // once; any other system that broke down shows a non-finite residual
    const int32_t orig = S.perm[f->fp32_fail_col];
    const int64_t k = std::upper_bound(S.sys_ptr.begin(), S.sys_ptr.end(), (int64_t)orig) -
                      S.sys_ptr.begin() - 1;
    for (int64_t c = 0; c < nrhs; ++c) H.bad[k + c * nsys] = 1;
  }
  int64_t active = 0;
  for (int64_t u = 0; u < units; ++u) active += H.bad[u] ? 0 : 1;
  launch_segnorms(nsys, sysp, b, n, nrhs, nrm + units, ws.npart, st);
  if (active > 0) solve_all<float>(f, b, n, x, n, nrhs, 0, st);
  const double tol = h->opt.refine_tol > 0 ? h->opt.refine_tol : 1e-10;
  const int maxit = h->opt.refine_max > 0 ? h->opt.refine_max : 10;
  const double ratio = h->opt.stall_ratio > 0 ? h->opt.stall_ratio : 0.5;
  int iters = 0;
  const double nnz = (double)S.A.colind.size();
  auto residual_norms = [&]() -> int {
    const int pe = f->prof.begin(st);
    launch_residual(n, h->d_rowptr.as<int64_t>(), h->d_colind.as<int32_t>(),
                    f->fullvals.as<double>(), b, n, x, n, r, nrhs, ws.xt, st);
    launch_segnorms(nsys, sysp, r, n, nrhs, nrm, ws.npart, st);
    f->prof.end(pe, st, TACHO_K_REFINE, (2.0 * nnz + 2.0 * n) * nrhs,
                nnz * 12.0 + 8.0 * n + 8.0 * 3.0 * n * nrhs);
    HIP_TRY(hipMemcpyAsync(hn, nrm, sizeof(double) * 2 * units, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t u = 0; u < units; ++u) {
      const double bn = hn[units + u];
      rho[u] = bn > 0 ? hn[u] / bn : hn[u];
      if (!(rho[u] == rho[u])) rho[u] = INFINITY;
    }
    return TACHO_OK;
  };
  while (active > 0) {
    int rc = residual_norms();
    if (rc != TACHO_OK) return rc;
    for (int64_t u = 0; u < units; ++u) {
      if (H.done[u] || H.bad[u]) continue;
      if (rho[u] <= tol) {
        H.done[u] = 1;
        --active;
        continue;
      }
      if (!std::isfinite(rho[u])) {
        H.bad[u] = 1;
        --active;
        continue;
      }
      if (rho[u] > ratio * H.prev[u]) {
        if (++H.stalls[u] >= 2) {
          H.bad[u] = 1;
          --active;
        }
      } else {
        H.stalls[u] = 0;
      }
      H.prev[u] = rho[u];
    }
    if (active == 0) break;
    if (iters >= maxit) {
      for (int64_t u = 0; u < units; ++u)
        if (!H.done[u]) H.bad[u] = 1;
      active = 0;
      break;
    }
    // finished units (converged or handed to FP64) get a zero correction
    for (int64_t u = 0; u < units; ++u) H.mask[u] = H.done[u] | H.bad[u];
    HIP_TRY(hipMemcpyAsync(mask, H.mask.data(), units, hipMemcpyHostToDevice, st));
    launch_zero_units(nsys, sysp, r, n, nrhs, mask, st);
    solve_all<float>(f, r, n, x, n, nrhs, 1, st);
    ++iters;
  }
  int64_t nbad = 0;
  for (int64_t u = 0; u < units; ++u) nbad += H.bad[u];
  if (nbad > 0) {
    // FP64 refactorization with the same values (already done after an FP32
    // pivot breakdown), an FP64 solve of every unit into r, and its columns
    // copied into x for the units that fell back.
    if (!f->fallback) {
      if (!may_allocate)
        return fail(TACHO_ERR_NOMEM, "refinement stalled and the FP64 fallback factor would "
                                     "need device memory; use tacho_solve");
      int64_t fi = -1;
      const int rc = fp64_fallback(f, st, &fi);
      if (rc != TACHO_OK) return rc;
    }
    solve_all<double>(f->fallback, b, n, r, n, nrhs, 0, st);
    HIP_TRY(hipMemcpyAsync(mask, H.bad.data(), units, hipMemcpyHostToDevice, st));
    launch_select_units(nsys, sysp, x, r, n, nrhs, mask, st);
    const int rc = residual_norms();
    if (rc != TACHO_OK) return rc;
  }
  if (info) {
    info->iters = iters;
    info->fell_back = nbad > 0 ? 1 : 0;
    double mx = 0;
    for (int64_t c = 0; c < nrhs; ++c) {
      double col = 0;
      for (int64_t k = 0; k < nsys; ++k) col = std::max(col, rho[k + c * nsys]);
      mx = std::max(mx, col);
      if (info->relres) info->relres[c] = col;
    }
    info->relres_max = mx;
    if (info->fell_back_units)
      for (int64_t u = 0; u < units; ++u) info->fell_back_units[u] = H.bad[u];
  }
  return check_solve_hang(f, st);
}

}  // namespace

extern "C" {

void tacho_default_options(tacho_options* opt) {
  if (opt) *opt = defaults();
}

const char* tacho_strerror(int code) {
  switch (code) {
    case TACHO_OK: return "success";
    case TACHO_ERR_INVALID: return "invalid argument";
    case TACHO_ERR_PATTERN: return "pattern is not structurally symmetric";
    case TACHO_ERR_NOT_SPD: return "matrix is not positive definite";
    case TACHO_ERR_NOMEM: return "out of device memory or over the HBM budget";
    case TACHO_ERR_HIP: return "HIP runtime error";
    case TACHO_ERR_SINGULAR: return "no usable pivot within a diagonal block";
    default: return "unknown error";
  }
}

const char* tacho_last_error(void) { return g_last_error.c_str(); }

int tacho_analyze(int64_t n, const int64_t* rowptr, const int32_t* colind,
                  const tacho_options* opt, tacho_sym_t* out) {
  if (!out) return fail(TACHO_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 0 || (n > 0 && (!rowptr || (!colind && rowptr[n] > 0))))
    return fail(TACHO_ERR_INVALID, "invalid CSR arguments");
  std::unique_ptr<tacho_sym> h(new tacho_sym());
  h->opt = opt ? *opt : defaults();
  std::string err;
  int rc = build_pattern(n, rowptr, colind, h->S.A, err);
  if (rc != kOk) return fail(rc, err);
  h->S.nsys = 1;
  h->S.sys_ptr = {0, n};
  rc = finish_analysis(h.get(), n > 0 ? rowptr[n] : 0);
  if (rc != TACHO_OK) return rc;
  *out = h.release();
  return TACHO_OK;
}

int tacho_analyze_batch(int64_t nsys, const int64_t* n, const int64_t* const* rowptr,
                        const int32_t* const* colind, const tacho_options* opt,
                        tacho_sym_t* out) {
  if (!out) return fail(TACHO_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (nsys < 1 || !n || !rowptr || !colind) return fail(TACHO_ERR_INVALID, "invalid batch");
  int64_t ntot = 0, nnz = 0;
  for (int64_t k = 0; k < nsys; ++k) {
    if (n[k] < 0 || (n[k] > 0 && !rowptr[k])) return fail(TACHO_ERR_INVALID, "invalid system");
    if (n[k] > 0) {
      if (rowptr[k][0] != 0)
        return fail(TACHO_ERR_INVALID, "system " + std::to_string(k) + ": rowptr[0] != 0");
      for (int64_t i = 0; i < n[k]; ++i)
        if (rowptr[k][i + 1] < rowptr[k][i])
          return fail(TACHO_ERR_INVALID, "system " + std::to_string(k) + ": rowptr decreases");
      if (rowptr[k][n[k]] > 0 && !colind[k])
        return fail(TACHO_ERR_INVALID, "system " + std::to_string(k) + ": colind is NULL");
    }
    ntot += n[k];
    nnz += n[k] > 0 ? rowptr[k][n[k]] : 0;
  }
  if (ntot > INT32_MAX - 1) return fail(TACHO_ERR_INVALID, "batch too large");
  std::vector<int64_t> rp(ntot + 1, 0);
  std::vector<int32_t> ci;
  ci.reserve(nnz);
  std::vector<int64_t> sys_ptr(nsys + 1, 0);
  int64_t roff = 0, koff = 0;
  for (int64_t k = 0; k < nsys; ++k) {
    for (int64_t i = 0; i < n[k]; ++i) {
      for (int64_t q = rowptr[k][i]; q < rowptr[k][i + 1]; ++q) {
        const int32_t c = colind[k][q];
        if (c < 0 || c >= n[k]) return fail(TACHO_ERR_INVALID, "column index out of range");
        ci.push_back((int32_t)(c + roff));
      }
      rp[roff + i + 1] = koff + rowptr[k][i + 1];
    }
    roff += n[k];
    koff += n[k] > 0 ? rowptr[k][n[k]] : 0;
    sys_ptr[k + 1] = roff;
  }
  std::unique_ptr<tacho_sym> h(new tacho_sym());
  h->opt = opt ? *opt : defaults();
  std::string err;
  int rc = build_pattern(ntot, rp.data(), ci.data(), h->S.A, err);
  if (rc != kOk) return fail(rc, err);
  h->S.nsys = nsys;
  h->S.sys_ptr = sys_ptr;
  rc = finish_analysis(h.get(), nnz);
  if (rc != TACHO_OK) return rc;
  *out = h.release();
  return TACHO_OK;
}

int tacho_query_symbolic(tacho_sym_t h, tacho_sym_info* info) {
  if (!h || !info) return fail(TACHO_ERR_INVALID, "NULL argument");
  const Symbolic& S = h->S;
  info->n = S.n;
  info->nnz_a = (int64_t)S.A.colind.size();
  info->nnz_l = S.nnzL;
  info->flops = S.flops;
  info->nsuper = S.ns;
  info->nlevels = S.nlevels;
  info->max_front = S.max_m;
  info->max_width = S.max_w;
  info->factor_bytes_fp64 = 8 * h->P.L_elems;
  info->work_bytes_fp64 = 8 * h->P.U_elems;
  info->device_bytes_fp64 = numeric_bytes(h, TACHO_FP64);
  info->nsystems = S.nsys;
  info->nnz_factor = S.nnz_front;
  info->ordering = S.ordering_used;
  info->t_order_us = S.t_order_us;
  info->t_structure_us = S.t_structure_us;
  info->t_plan_us = S.t_plan_us;
  info->plan_u_range = h->tune.u_range;
  info->plan_chain_min = h->tune.chain_min;
  info->plan_solve_level_fronts = h->tune.level_fronts;
  info->plan_asm_cols = h->tune.asm_cols;
  info->plan_solo_m = h->tune.solo_m;
  info->plan_chain_inplace = h->tune.chain_inplace;
  return TACHO_OK;
}

int tacho_get_symbolic(tacho_sym_t h, int32_t* perm, int32_t* parent, int64_t* colcount,
                       int32_t* super_ptr, int32_t* super_parent, int32_t* level) {
  if (!h) return fail(TACHO_ERR_INVALID, "NULL handle");
  const Symbolic& S = h->S;
  if (perm) std::copy(S.perm.begin(), S.perm.end(), perm);
  if (parent) std::copy(S.parent.begin(), S.parent.end(), parent);
  if (colcount) std::copy(S.colcount.begin(), S.colcount.end(), colcount);
  if (super_ptr) std::copy(S.sptr.begin(), S.sptr.end(), super_ptr);
  if (super_parent) std::copy(S.sparent.begin(), S.sparent.end(), super_parent);
  if (level) std::copy(S.height.begin(), S.height.end(), level);
  return TACHO_OK;
}

int tacho_factorize(tacho_sym_t h, const double* values, int values_on_device, int precision,
                    void* hip_stream, tacho_num_t* out, int64_t* fail_index) {
  if (!h || !out) return fail(TACHO_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (fail_index) *fail_index = -1;
  if (!valid_precision(precision)) return fail(TACHO_ERR_INVALID, "unknown precision");
  tacho_num* f = nullptr;
  int rc = create_numeric(h, precision, &f);
  if (rc != TACHO_OK) return rc;
  rc = refactor(f, values, values_on_device, (hipStream_t)hip_stream, 1, fail_index);
  if (rc != TACHO_OK) {
    delete f;
    return rc;
  }
  *out = f;
  return TACHO_OK;
}

int tacho_numeric_create(tacho_sym_t h, int precision, tacho_num_t* out) {
  if (!h || !out) return fail(TACHO_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (!valid_precision(precision)) return fail(TACHO_ERR_INVALID, "unknown precision");
  tacho_num* f = nullptr;
  const int rc = create_numeric(h, precision, &f);
  if (rc != TACHO_OK) return rc;
  f->last_status = TACHO_ERR_INVALID;  // no factor until the first refactorization
  *out = f;
  return TACHO_OK;
}

int tacho_numeric_bytes(tacho_sym_t h, int precision, int64_t* bytes) {
  if (!h || !bytes) return fail(TACHO_ERR_INVALID, "NULL argument");
  *bytes = numeric_bytes(h, precision);
  return TACHO_OK;
}

int tacho_refactorize(tacho_num_t f, const double* values, int values_on_device, void* hip_stream,
                      int sync, int64_t* fail_index) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  if (fail_index) *fail_index = -1;
  return refactor(f, values, values_on_device, (hipStream_t)hip_stream, sync, fail_index);
}

int tacho_check_factor(tacho_num_t f, int64_t* fail_index) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  if (f->pending) {
    const int rc = read_fail_flag(f, fail_index);
    if (rc != TACHO_OK) return rc;
  }
  if (f->sync.p) {
    // the last solve may have been queued on another stream than the factorization
    const int rc = check_solve_hang(f, f->last_solve_stream ? f->last_solve_stream : f->last_stream);
    if (rc != TACHO_OK) return rc;
  }
  if (fail_index) *fail_index = f->last_fail;
  return f->last_status;
}

}  // extern "C"

namespace {

// tacho_solve and tacho_solve_noalloc.  With `noalloc` the caller's blocks
// are on the device and used in place, and the refinement scratch is the
// file-scope device array of kernels.hip instead of the handle's buffer.
int solve_impl(tacho_num_t f, const double* b, double* x, int64_t nrhs, int64_t ld, int on_device,
               void* hip_stream, tacho_solve_info* info, bool noalloc) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  tacho_sym* h = f->sym;
  const int64_t n = h->S.n;
  if (nrhs < 0 || ld < std::max<int64_t>(n, 1) || (nrhs > 0 && n > 0 && (!b || !x)))
    return fail(TACHO_ERR_INVALID, "invalid solve arguments");
  if (info) {
    info->iters = 0;
    info->fell_back = 0;
    info->relres_max = 0;
  }
  const bool refine = f->precision == TACHO_FP32;
  const bool dense_ld = ld == n;
  if (noalloc) {
    if (refine && (!dense_ld || b == x))
      return fail(TACHO_ERR_INVALID, "tacho_solve_noalloc with an FP32 factor needs ld == n "
                                     "and x != b");
    if (refine && nrhs > kRhs)
      return fail(TACHO_ERR_INVALID, "tacho_solve_noalloc with an FP32 factor takes at most 16 "
                                     "right-hand sides");
    if (refine && refine_scratch_bytes(n, nrhs, h->S.nsys) > (int64_t)kNoAllocScratchBytes)
      return fail(TACHO_ERR_INVALID, "refinement scratch of " +
                                         std::to_string(refine_scratch_bytes(n, nrhs, h->S.nsys)) +
                                         " bytes exceeds the no-allocation maximum of " +
                                         std::to_string(kNoAllocScratchBytes));
  }
  // A factorization queued without waiting is not checked here when the solve
  // stays on the device in FP64: the solve is queued behind it and
  // tacho_check_factor tells whether the result is valid.
  const bool queue_only = on_device && f->precision != TACHO_FP32;
  if (f->pending && !queue_only) {
    int rc = read_fail_flag(f, nullptr, !noalloc);
    if (rc != TACHO_OK) return rc;
  } else if (!f->pending && f->last_status != TACHO_OK) {
    return fail(f->last_status, "no valid factor in this handle");
  }
  if (nrhs == 0 || n == 0) return TACHO_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  f->last_solve_stream = st;
  f->solve_queued = true;
  const double* bd = b;
  double* xd = x;
  // the refinement path works on dense (ld = n) device blocks
  if (!on_device || (refine && !dense_ld) || (refine && b == x)) {
    const size_t bytes = sizeof(double) * n * nrhs;
    if (f->bdev.bytes < bytes) HIP_TRY(f->bdev.alloc(bytes));
    if (f->xdev.bytes < bytes) HIP_TRY(f->xdev.alloc(bytes));
    HIP_TRY(hipMemcpy2DAsync(f->bdev.p, n * sizeof(double), b, ld * sizeof(double),
                             n * sizeof(double), nrhs,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    bd = f->bdev.as<double>();
    xd = f->xdev.as<double>();
  }
  const int64_t ldi = (bd == b) ? ld : n;
  HIP_TRY(hipEventRecord(f->ev[2], st));
  if (refine) {
    void* base = nullptr;
    if (noalloc) {
      HIP_TRY(noalloc_scratch(&base));
    } else {
      const int64_t need = refine_scratch_bytes(n, nrhs, h->S.nsys);
      if (f->rws.bytes < (size_t)need) HIP_TRY(f->rws.alloc(need));
      base = f->rws.p;
    }
    const int rc = refine_solve(f, bd, xd, nrhs, st, info,
                                carve_refine_scratch(base, n, nrhs, h->S.nsys), !noalloc);
    if (rc != TACHO_OK) return rc;
  } else {
    solve_all<double>(f, bd, ldi, xd, (xd == x) ? ld : n, nrhs, 0, st);
  }
  HIP_TRY(hipEventRecord(f->ev[3], st));
  if (xd != x) {
    HIP_TRY(hipMemcpy2DAsync(x, ld * sizeof(double), xd, n * sizeof(double), n * sizeof(double),
                             nrhs, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             st));
    if (!on_device) HIP_TRY(hipStreamSynchronize(st));
  }
  if (!on_device) {
    const int rc = check_solve_hang(f, st);
    if (rc != TACHO_OK) return rc;
  }
  HIP_TRY(hipGetLastError());
  return TACHO_OK;
}

}  // namespace

extern "C" {

int tacho_solve(tacho_num_t f, const double* b, double* x, int64_t nrhs, int64_t ld, int on_device,
                void* hip_stream, tacho_solve_info* info) {
  return solve_impl(f, b, x, nrhs, ld, on_device, hip_stream, info, false);
}

int tacho_solve_noalloc(tacho_num_t f, const double* b, double* x, int64_t nrhs, int64_t ld,
                        void* hip_stream, tacho_solve_info* info) {
  return solve_impl(f, b, x, nrhs, ld, 1, hip_stream, info, true);
}

int tacho_set_solve_variant(tacho_num_t f, int variant, void* hip_stream) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  if (variant != TACHO_SOLVE_BLOCK_INVERSE && variant != TACHO_SOLVE_PARTITIONED_INVERSE &&
      variant != TACHO_SOLVE_LEVEL_CSR)
    return fail(TACHO_ERR_INVALID, "unknown solve variant " + std::to_string(variant));
  if (variant == f->solve_variant) return TACHO_OK;
  if (variant == TACHO_SOLVE_BLOCK_INVERSE) {
    f->solve_variant = variant;
    return TACHO_OK;
  }
  if (f->precision == TACHO_LDLT || f->precision == TACHO_LU)
    return fail(TACHO_ERR_INVALID, "the partitioned inverse needs a Cholesky factor");
  if (f->pending) {
    const int rc = read_fail_flag(f, nullptr);
    if (rc != TACHO_OK) return rc;
  } else if (f->last_status != TACHO_OK) {
    return fail(f->last_status, "no valid factor in this handle");
  }
  tacho_sym* h = f->sym;
  const size_t es = elem_size(f->precision);
  const size_t zbytes = es * (size_t)std::max<int64_t>(h->P.L_elems, 1);
  const size_t ybytes = (size_t)kRowBytes * (size_t)std::max<int64_t>(h->S.n, 1);
  const bool csr = variant == TACHO_SOLVE_LEVEL_CSR;
  int rc = TACHO_OK;
  if (csr) {
    rc = ensure_level_csr(h);
    if (rc != TACHO_OK) return rc;
  }
  const size_t cbytes = csr ? (es + sizeof(int32_t)) * (size_t)std::max<int64_t>(h->C->nnz, 1) : 0;
  if (h->opt.hbm_budget_bytes > 0 &&
      (uint64_t)numeric_bytes(h, f->precision) + zbytes + ybytes + cbytes > h->opt.hbm_budget_bytes)
    return fail(TACHO_ERR_NOMEM, "the partitioned inverse would exceed the HBM budget");
  rc = ensure_pinv(h);
  if (rc != TACHO_OK) return rc;
  if (csr) {
    if (f->cvals.bytes < es * (size_t)h->C->nnz) HIP_TRY(f->cvals.alloc(es * (size_t)h->C->nnz));
    if (f->ccols.bytes < sizeof(int32_t) * (size_t)h->C->nnz)
      HIP_TRY(f->ccols.alloc(sizeof(int32_t) * (size_t)h->C->nnz));
  }
  if (f->Z.bytes < zbytes) HIP_TRY(f->Z.alloc(zbytes));
  if (f->yfwd.bytes < ybytes) HIP_TRY(f->yfwd.alloc(ybytes));
  {
    const int64_t slots = std::max<int64_t>(h->Q->slots, 1);
    const size_t pbytes = es * (size_t)slots * kPanel * kRhs;
    if (f->zpart.bytes < pbytes) HIP_TRY(f->zpart.alloc(pbytes));
  }
  hipStream_t st = (hipStream_t)hip_stream;
  f->csr_pending = csr;
  if (f->precision == TACHO_FP32)
    run_pinv_setup<float>(f, st);
  else
    run_pinv_setup<double>(f, st);
  f->csr_pending = false;
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipGetLastError());
  f->solve_variant = variant;
  return TACHO_OK;
}

// Panels of one factor half (L, or U^T of an LU factorization) as CSC by
// permuted column.  remap: a front's pivot rows are stored in its pivot
// order, the rows of its ancestors keep their analysis numbering and map
// through the inverse pivot order (columns re-sorted by row).
int export_panels(tacho_num* f, const DBuf& src, bool remap, int64_t* Lp, int32_t* Li, double* Lx) {
  const Symbolic& S = f->sym->S;
  const Plan& P = f->sym->P;
  const size_t es = elem_size(f->precision);
  std::vector<char> host(es * P.L_elems);
  HIP_TRY(hipDeviceSynchronize());
  if (!host.empty()) HIP_TRY(hipMemcpy(host.data(), src.p, host.size(), hipMemcpyDeviceToHost));
  Lp[0] = 0;
  for (int32_t s = 0; s < S.ns; ++s)
    for (int32_t j = S.sptr[s]; j < S.sptr[s + 1]; ++j)
      Lp[j + 1] = Lp[j] + (S.front_m[s] - (j - S.sptr[s]));
  std::vector<int32_t> qinv;
  if (remap && S.n > 0) {
    qinv.resize(S.n);
    HIP_TRY(hipMemcpy(qinv.data(), f->ld_qinv.p, sizeof(int32_t) * S.n, hipMemcpyDeviceToHost));
  }
  std::vector<std::pair<int32_t, double>> col;
  for (int32_t s = 0; s < S.ns; ++s) {
    const int32_t f0 = S.sptr[s], w = S.sptr[s + 1] - f0, m = S.front_m[s];
    for (int32_t c = 0; c < w; ++c) {
      const int64_t q0 = Lp[f0 + c];
      int64_t q = q0;
      for (int32_t i = c; i < m; ++i, ++q) {
        const int64_t off = P.L_off[s] + (int64_t)c * P.ldL[s] + i;
        const int32_t row = S.rows[S.rows_ptr[s] + i];
        Li[q] = qinv.empty() || i < w ? row : qinv[row];
        Lx[q] = f->precision == TACHO_FP32 ? (double)reinterpret_cast<const float*>(host.data())[off]
                                           : reinterpret_cast<const double*>(host.data())[off];
      }
      if (!qinv.empty()) {
        col.clear();
        for (int64_t k = q0; k < q; ++k) col.emplace_back(Li[k], Lx[k]);
        std::sort(col.begin(), col.end(),
                  [](const std::pair<int32_t, double>& a, const std::pair<int32_t, double>& b) {
                    return a.first < b.first;
                  });
        for (int64_t k = q0; k < q; ++k) {
          Li[k] = col[k - q0].first;
          Lx[k] = col[k - q0].second;
        }
      }
    }
  }
  return TACHO_OK;
}

int tacho_get_factor(tacho_num_t f, int64_t* Lp, int32_t* Li, double* Lx) {
  if (!f || !Lp || !Li || !Lx) return fail(TACHO_ERR_INVALID, "NULL argument");
  if (f->pending) {
    int rc = read_fail_flag(f, nullptr);
    if (rc != TACHO_OK) return rc;
  }
  // after an FP32 pivot breakdown the FP32 factor is not valid: the FP64
  // factor of the same values is the one the solves fall back to
  if (f->fp32_broken && f->fallback) f = f->fallback;
  return export_panels(f, f->L, f->precision == TACHO_LDLT || f->precision == TACHO_LU, Lp, Li, Lx);
}

int tacho_get_lu(tacho_num_t f, int64_t* Up, int32_t* Ui, double* Ux, int32_t* q) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  if (f->precision != TACHO_LU) return fail(TACHO_ERR_INVALID, "not an LU factorization");
  if (f->pending) {
    int rc = read_fail_flag(f, nullptr);
    if (rc != TACHO_OK) return rc;
  } else if (f->last_status != TACHO_OK) {
    return fail(f->last_status, "no valid factor in this handle");
  }
  const int64_t n = f->sym->S.n;
  if (q && n > 0) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(q, f->ld_q.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  }
  if (Up || Ui || Ux) {
    if (!Up || !Ui || !Ux) return fail(TACHO_ERR_INVALID, "Up, Ui and Ux go together");
    // U's columns keep the analysis order: no remapping
    return export_panels(f, f->lu_t, false, Up, Ui, Ux);
  }
  return TACHO_OK;
}

int tacho_get_ldlt(tacho_num_t f, double* d, double* e, int32_t* q) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  if (f->precision != TACHO_LDLT) return fail(TACHO_ERR_INVALID, "not an LDL^T factorization");
  if (f->pending) {
    int rc = read_fail_flag(f, nullptr);
    if (rc != TACHO_OK) return rc;
  } else if (f->last_status != TACHO_OK) {
    return fail(f->last_status, "no valid factor in this handle");
  }
  const int64_t n = f->sym->S.n;
  HIP_TRY(hipDeviceSynchronize());
  if (n > 0) {
    if (d) HIP_TRY(hipMemcpy(d, f->ld_d.p, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (e) HIP_TRY(hipMemcpy(e, f->ld_e.p, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (q) HIP_TRY(hipMemcpy(q, f->ld_q.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  }
  return TACHO_OK;
}

int tacho_last_times(tacho_num_t f, double* factor_ms, double* solve_ms) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  float a = 0, b = 0;
  if (factor_ms) {
    HIP_TRY(hipEventSynchronize(f->ev[1]));
    HIP_TRY(hipEventElapsedTime(&a, f->ev[0], f->ev[1]));
    *factor_ms = a;
  }
  if (solve_ms) {
    HIP_TRY(hipEventSynchronize(f->ev[3]));
    HIP_TRY(hipEventElapsedTime(&b, f->ev[2], f->ev[3]));
    *solve_ms = b;
  }
  return TACHO_OK;
}

int tacho_profile(tacho_num_t f, int enable) {
  if (!f) return fail(TACHO_ERR_INVALID, "NULL handle");
  if (enable) {
    HIP_TRY(f->prof.collect());
    f->prof.clear();
  }
  f->prof.on = enable != 0;
  return TACHO_OK;
}

int tacho_profile_read(tacho_num_t f, int kind, int64_t* launches, double* ms, double* flops,
                       double* bytes) {
  if (!f || kind < 0 || kind >= TACHO_PROFILE_KINDS) return fail(TACHO_ERR_INVALID, "bad kind");
  HIP_TRY(f->prof.collect());
  if (launches) *launches = f->prof.launches[kind];
  if (ms) *ms = f->prof.ms[kind];
  if (flops) *flops = f->prof.flops[kind];
  if (bytes) *bytes = f->prof.bytes[kind];
  return TACHO_OK;
}

const char* tacho_kernel_name(int kind) {
  static const char* names[TACHO_PROFILE_KINDS] = {
      "k_small", "k_assemble", "k_diag", "k_panel", "k_gemm",
      "k_gather", "k_fwd", "k_bwd", "k_permute", "k_residual", "k_front", "k_pinv"};
  return kind >= 0 && kind < TACHO_PROFILE_KINDS ? names[kind] : "unknown";
}

int tacho_free_symbolic(tacho_sym_t h) {
  delete h;
  return TACHO_OK;
}

int tacho_free_numeric(tacho_num_t f) {
  if (f && f->last_stream) (void)hipStreamSynchronize(f->last_stream);
  delete f;
  return TACHO_OK;
}

}  // extern "C"
