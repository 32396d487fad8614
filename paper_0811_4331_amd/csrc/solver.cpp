// Host drivers: MR smoother, coarse-grid correction, V-cycle, coarsest GCR,
// flexible GCR outer solve, BiCGStab comparator and the adaptive setup.
// Every arithmetic step runs in the kernels; the host only sequences launches
// on the context's stream and reads back residual norms.
//
// Paper passages: MR smoother with omega (Sec. 3, last paragraph); coarse-grid
// correction with the minimal-residual step alpha (Sec. 3, step-size
// equation); V(nu_pre, nu_post) cycle (Sec. 2) and the modified 3-level cycle
// with 4 next-coarser cycles between fine restriction and prolongation
// (Sec. 5); GCR(k) outer solver, flexible because the preconditioner is not
// stationary (Sec. 5); adaptive setup by relaxation of A v = 0 and block QR
// (Sec. 2).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"
#include "solver.h"

namespace wdmg {

// ---------------------------------------------------------------------------
// memory
void* dev_alloc(Ctx& c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (c.alloc.alloc) {
    p = c.alloc.alloc(bytes, c.alloc.user);
    if (!p) throw Error(WDMG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    if (reinterpret_cast<uintptr_t>(p) & 255)  // not an allocation: never hand it to a kernel
      throw Error(WDMG_ERR_OOM, "device allocation of " + std::to_string(bytes) +
                                    " bytes returned a misaligned pointer");
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(WDMG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  c.bufs.push_back(Buf{p, bytes});
  return p;
}

void dev_free(Ctx& c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c.bufs.size(); ++i) {
    if (c.bufs[i].p == p) {
      c.bufs.erase(c.bufs.begin() + i);
      break;
    }
  }
  if (c.alloc.free)
    c.alloc.free(p, c.alloc.user);
  else
    (void)hipFree(p);
}

void ensure_io(Ctx& c, size_t bytes) {
  if (bytes <= c.io_bytes) return;
  WDMG_HIP(hipStreamSynchronize(c.stream));
  dev_free(c, c.io_a);
  dev_free(c, c.io_b);
  c.io_a = dev_alloc(c, bytes);
  c.io_b = dev_alloc(c, bytes);
  c.io_bytes = bytes;
}

ProfScope::ProfScope(Ctx& ctx, int id, long long units) : c(ctx) {
  if (!c.prof_on || c.no_alloc) return;
  Ctx::ProfRec r{id, units, nullptr, nullptr};
  for (hipEvent_t* e : {&r.a, &r.b}) {
    if (!c.prof_pool.empty()) {
      *e = c.prof_pool.back();
      c.prof_pool.pop_back();
    } else {
      WDMG_HIP(hipEventCreate(e));
    }
  }
  WDMG_HIP(hipEventRecord(r.a, c.stream));
  c.prof_recs.push_back(r);
  idx = (int)c.prof_recs.size() - 1;
}

ProfScope::~ProfScope() {
  if (idx >= 0) (void)hipEventRecord(c.prof_recs[idx].b, c.stream);
}

void prof_collect(Ctx& c) {
  if (c.prof_recs.empty()) return;
  WDMG_HIP(hipStreamSynchronize(c.stream));
  for (auto& r : c.prof_recs) {
    float ms = 0.f;
    WDMG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    c.prof_launch[r.id] += 1;
    c.prof_units[r.id] += r.units;
    c.prof_ms[r.id] += ms;
    c.prof_pool.push_back(r.a);
    c.prof_pool.push_back(r.b);
  }
  c.prof_recs.clear();
}

double read_scalar(Ctx& c, int slot) {
  WDMG_HIP(hipMemcpyAsync(c.hsc, c.dsc + slot, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  WDMG_HIP(hipStreamSynchronize(c.stream));
  return c.hsc[0];
}

void check_flags(Ctx& c) {
  WDMG_HIP(hipMemcpyAsync(c.hsc, c.dsc + S_ERR, 2 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  WDMG_HIP(hipStreamSynchronize(c.stream));
  const double nan_flag = c.hsc[0], rank_flag = c.hsc[1];
  if (nan_flag != 0.0 || rank_flag != 0.0) {
    set_scalar(c, S_ERR, 0.0, 0.0);
    WDMG_HIP(hipStreamSynchronize(c.stream));
    if (rank_flag != 0.0) throw Error(WDMG_ERR_RANK_DEFICIENT, "candidate vectors are rank deficient on an aggregate");
    throw Error(WDMG_ERR_NAN, "NaN or Inf met in a reduction");
  }
}

// ---------------------------------------------------------------------------
// level helpers
template <typename R>
cx<R>* work(Level& L, int i);
template <>
cx<double>* work<double>(Level& L, int i) {
  return L.w64[i];
}
template <>
cx<float>* work<float>(Level& L, int i) {
  return L.w32[i];
}
template <typename R>
const cx<R>* vecs(const Level& L);
// The accessors refuse copies that wdmg_release_unused freed (before any launch).
template <>
const cx<double>* vecs<double>(const Level& L) {
  if (!L.V64) throw Error(WDMG_ERR_ARG, "FP64 prolongator released by wdmg_release_unused");
  return L.V64;
}
template <>
const cx<float>* vecs<float>(const Level& L) {
  if (!L.V32) throw Error(WDMG_ERR_ARG, "FP32 prolongator released by wdmg_release_unused");
  return L.V32;
}
template <typename R>
const cx<R>* stencil(const Level& L);
template <>
const cx<double>* stencil<double>(const Level& L) {
  if (!L.Dc64) throw Error(WDMG_ERR_ARG, "FP64 coarse blocks released by wdmg_release_unused");
  return L.Dc64;
}
template <>
const cx<float>* stencil<float>(const Level& L) {
  if (!L.Dc32) throw Error(WDMG_ERR_ARG, "FP32 coarse blocks released by wdmg_release_unused");
  return L.Dc32;
}

// Coarse levels of a V-cycle running in 16-bit storage (c.vc_half) apply
// their 16-bit coarse blocks to FP32 vectors.
template <typename R>
void apply_op(Ctx& c, int l, cx<R>* out, const cx<R>* in, int nrhs) {
  if (l == 0)
    dslash<R>(c, out, in, nrhs);
  else if constexpr (sizeof(R) == 4) {
    if (c.vc_half)
      coarse_apply_h(c, c.lev[l], c.vc_half, out, in, nrhs);
    else
      coarse_apply<R>(c, c.lev[l], stencil<R>(c.lev[l]), out, in, nrhs);
  } else {
    coarse_apply<R>(c, c.lev[l], stencil<R>(c.lev[l]), out, in, nrhs);
  }
}

template <typename R>
void restrict_to(Ctx& c, int l, const cx<R>* fine, cx<R>* crs, int nrhs) {
  if (l == 0)
    restrict0<R>(c, c.lev[0], vecs<R>(c.lev[0]), fine, crs, nrhs);
  else
    restrictC<R>(c, c.lev[l], vecs<R>(c.lev[l]), fine, crs, nrhs);
}

template <typename R>
void prolong_from(Ctx& c, int l, const cx<R>* crs, cx<R>* fine, int nrhs) {
  if (l == 0)
    prolong0<R>(c, c.lev[0], vecs<R>(c.lev[0]), crs, fine, nrhs);
  else
    prolongC<R>(c, c.lev[l], vecs<R>(c.lev[l]), crs, fine, nrhs);
}

// ---------------------------------------------------------------------------
// Work space.  Every level keeps kWork fields per right-hand side in each
// precision it runs in; the buffers grow to the largest batch seen.
template <typename R>
void ensure_work(Ctx& c, int l, int nrhs) {
  Level& L = c.lev[l];
  int& cap = sizeof(R) == 8 ? L.cap64 : L.cap32;
  if (nrhs <= cap) return;
  WDMG_HIP(hipStreamSynchronize(c.stream));
  for (int i = 0; i < kWork; ++i) {
    if (l == 0 && (i == 0 || i > 4)) continue;  // the fine level uses work fields 1..4 only
    if constexpr (sizeof(R) == 8) {
      dev_free(c, L.w64[i]);
      L.w64[i] = static_cast<cx<double>*>(dev_alloc(c, (size_t)nrhs * L.n * sizeof(cx<double>)));
    } else {
      dev_free(c, L.w32[i]);
      L.w32[i] = static_cast<cx<float>*>(dev_alloc(c, (size_t)nrhs * L.n * sizeof(cx<float>)));
    }
  }
  cap = nrhs;
}

void ensure_coarsest_basis(Ctx& c, int nrhs) {
  Level& L = c.lev[c.nlevels - 1];
  if (nrhs <= L.capB) return;
  WDMG_HIP(hipStreamSynchronize(c.stream));
  dev_free(c, L.basisZ);
  dev_free(c, L.basisW);
  dev_free(c, L.xT);
  const size_t sz = (size_t)c.mg.coarse_restart * nrhs * L.n * sizeof(cx<double>);
  L.basisZ = static_cast<cx<double>*>(dev_alloc(c, sz));
  L.basisW = static_cast<cx<double>*>(dev_alloc(c, sz));
  L.xT = static_cast<cx<double>*>(dev_alloc(c, (size_t)nrhs * L.n * sizeof(cx<double>)));
  dev_free(c, L.cpart);
  dev_free(c, L.cpart3);
  dev_free(c, L.chist);
  L.cpart = static_cast<double*>(dev_alloc(c, coarsest_gcr_partials(nrhs, c.mg.coarse_restart) * sizeof(double)));
  L.cpart3 = static_cast<double*>(dev_alloc(c, coarsest_gcr_partials3(nrhs) * sizeof(double)));
  L.chist = static_cast<double*>(dev_alloc(c, coarsest_gcr_history(nrhs, c.mg.coarse_restart) * sizeof(double)));
  L.capB = nrhs;
}

// Work space of a whole V-cycle solve with nrhs right-hand sides in precision prec.
// A V-cycle in 16-bit storage works on the 16-bit fields of level 0
// (ensure_work_h), so its FP32 work vectors start at level 1 (first = 1).
void ensure_mg_work(Ctx& c, int nrhs, int prec, int first) {
  for (int l = first; l < c.nlevels; ++l) {
    if (prec == WDMG_F32)
      ensure_work<float>(c, l, nrhs);
    else
      ensure_work<double>(c, l, nrhs);
  }
  // the coarsest solve runs in FP64 whatever the V-cycle precision
  ensure_work<double>(c, c.nlevels - 1, nrhs);
  ensure_coarsest_basis(c, nrhs);
  dots_buffer(c, nrhs);
}

// ---------------------------------------------------------------------------
// MR smoother (Sec. 3): p = A r; alpha = omega <p,r>/<p,p>; x += alpha r;
// r -= alpha p, with one step size per right-hand side.
// With b0, the steps start from x = 0 and residual b0 (the first step reads
// b0 and writes x and r); with last_x_only the last step updates x alone.
template <typename R>
void mr(Ctx& c, int l, cx<R>* x, cx<R>* r, cx<R>* p, int nrhs, int iters, double omega, const cx<R>* b0,
        bool last_x_only) {
  const size_t n = c.lev[l].n;
  for (int it = 0; it < iters; ++it) {
    const bool first = it == 0 && b0;
    const cx<R>* in = first ? b0 : r;
    if (l == 0) {
      dslash_mr<R>(c, p, in, nrhs, omega, S_BATCH);
    } else {
      apply_op<R>(c, l, p, in, nrhs);
      step_alpha_batch<R>(c, p, in, n, n, nrhs, omega, S_BATCH);
    }
    update2_batch<R>(c, x, in, r, p, n, n, nrhs, S_BATCH, first ? 1 : (last_x_only && it == iters - 1 ? 2 : 0));
  }
}

// ---------------------------------------------------------------------------
// Coarsest solve: GCR(restart) on D_c in FP64 to relative tolerance tol_c,
// for nrhs right-hand sides together (each with its own coefficients).
void coarsest_solve(Ctx& c, cx<double>* x, const cx<double>* b, int nrhs) {
  Level& L = c.lev[c.nlevels - 1];
  coarsest_gcr(c, L, x, b, nrhs, c.mg.coarse_tol, c.mg.coarse_restart, c.mg.coarse_maxit);
}

// ---------------------------------------------------------------------------
// V-cycle M_l (Sec. 2 / Sec. 3 / Sec. 5): x = M_l b from x = 0.
template <typename R>
void vcycle(Ctx& c, int l, cx<R>* x, const cx<R>* b, int nrhs);

// Coarse-grid solve of level lc >= 1 for the restricted residual rc: the
// FP64 GCR on the coarsest level, else the stationary iteration
// e <- e + M_lc (r_c - D_lc e) from e = 0 (Sec. 5).
template <typename R>
void coarse_solve_level(Ctx& c, int lc, cx<R>* rc, cx<R>* ec, int nrhs) {
  Level& C = c.lev[lc];
  const size_t nc = C.n * nrhs;
  if (lc == c.nlevels - 1) {
    if constexpr (sizeof(R) == 8) {
      coarsest_solve(c, ec, rc, nrhs);
    } else {
      convert<double, float>(c, C.w64[5], rc, nc);
      coarsest_solve(c, C.w64[6], C.w64[5], nrhs);
      convert<float, double>(c, ec, C.w64[6], nc);
    }
  } else {
    const int ncyc = c.mg.coarse_cycles > 0 ? c.mg.coarse_cycles : 1;
    cx<R>* t = work<R>(C, 7);
    cx<R>* xo = work<R>(C, 0);
    vcycle<R>(c, lc, xo, rc, nrhs);
    copy<R>(c, ec, xo, nc);
    for (int it = 1; it < ncyc; ++it) {
      apply_op<R>(c, lc, t, ec, nrhs);
      xmy<R>(c, rc, t, nc);
      vcycle<R>(c, lc, xo, t, nrhs);
      add<R>(c, ec, xo, nc);
    }
  }
}

template <typename R>
void coarse_correction(Ctx& c, int l, const cx<R>* res, cx<R>* y, int nrhs) {
  Level& C = c.lev[l + 1];
  cx<R>* rc = work<R>(C, 5);
  cx<R>* ec = work<R>(C, 6);
  restrict_to<R>(c, l, res, rc, nrhs);
  coarse_solve_level<R>(c, l + 1, rc, ec, nrhs);
  prolong_from<R>(c, l, ec, y, nrhs);
}

template <typename R>
void vcycle(Ctx& c, int l, cx<R>* x, const cx<R>* b, int nrhs) {
  Level& L = c.lev[l];
  const size_t n = L.n;
  cx<R>* res = work<R>(L, 1);
  cx<R>* p = work<R>(L, 2);
  cx<R>* y = work<R>(L, 3);
  cx<R>* dy = work<R>(L, 4);
  if (c.mg.nu_pre > 0) {
    mr<R>(c, l, x, res, p, nrhs, c.mg.nu_pre, c.mg.omega, b, false);
  } else {
    zero<R>(c, x, n * nrhs);
    copy<R>(c, res, b, n * nrhs);
  }
  coarse_correction<R>(c, l, res, y, nrhs);
  apply_op<R>(c, l, dy, y, nrhs);
  if (c.mg.use_alpha)
    step_alpha_batch<R>(c, dy, res, n, n, nrhs, 1.0, S_BATCH);  // Sec. 3 step-size equation
  else
    fill_pairs(c, S_BATCH, nrhs, 1.0, 0.0);
  update2_batch<R>(c, x, y, res, dy, n, n, nrhs, S_BATCH, c.mg.nu_post > 0 ? 0 : 2);
  mr<R>(c, l, x, res, p, nrhs, c.mg.nu_post, c.mg.omega, nullptr, true);
}

#define INST(R)                                                                \
  template void vcycle<R>(Ctx&, int, cx<R>*, const cx<R>*, int);              \
  template void apply_op<R>(Ctx&, int, cx<R>*, const cx<R>*, int);            \
  template void restrict_to<R>(Ctx&, int, const cx<R>*, cx<R>*, int);         \
  template void prolong_from<R>(Ctx&, int, const cx<R>*, cx<R>*, int);        \
  template void mr<R>(Ctx&, int, cx<R>*, cx<R>*, cx<R>*, int, int, double, const cx<R>*, bool); \
  template void ensure_work<R>(Ctx&, int, int);
INST(double)
INST(float)
#undef INST

// ---------------------------------------------------------------------------
// The fine level of the V-cycle in 16-bit storage: the fine fields, links and
// P in H with FP32 arithmetic; coarse levels in FP32 with 16-bit coarse
// blocks; the coarsest solve in FP64.
void ensure_work_h(Ctx& c, int nrhs) {
  Level& L = c.lev[0];
  if (nrhs <= L.caph) return;
  WDMG_HIP(hipStreamSynchronize(c.stream));
  for (HF& f : L.wh) {
    hf_free(c, f);
    f = hf_alloc(c, nrhs);
  }
  L.caph = nrhs;
}

// With b0, the steps start from x = 0 and residual *b0 (the first step reads
// b0 and writes x and r, no copy or zero fill); with last_x_only the last
// step updates x alone (a V-cycle does not read the residual after its
// post-smoothing).
template <typename H>
void mr_h(Ctx& c, HF x, HF r, HF p, int nrhs, int iters, double omega, const HF* b0, bool last_x_only) {
  for (int it = 0; it < iters; ++it) {
    const bool first = it == 0 && b0;
    dslash_h_mr<H>(c, p, first ? *b0 : r, nrhs, omega, S_BATCH);
    const int mode = first ? 1 : (last_x_only && it == iters - 1 ? 2 : 0);
    update2_half<H>(c, x, first ? *b0 : r, r, p, nrhs, S_BATCH, mode);
  }
}

template <typename H>
void vcycle_h(Ctx& c, HF x, HF b, int nrhs) {
  Level& L = c.lev[0];
  Level& C = c.lev[1];
  const void* V = v16(c, L, half_kind<H>());
  HF res = L.wh[0], p = L.wh[1], y = L.wh[2], dy = L.wh[3];
  if (c.mg.nu_pre > 0) {
    mr_h<H>(c, x, res, p, nrhs, c.mg.nu_pre, c.mg.omega, &b, false);
  } else {
    hf_zero<H>(c, x, nrhs);
    hf_copy(c, res, b, nrhs);
  }
  cx<float>* rc = C.w32[5];
  cx<float>* ec = C.w32[6];
  restrict0_h<H>(c, L, V, res, rc, nrhs);
  coarse_solve_level<float>(c, 1, rc, ec, nrhs);
  prolong0_h<H>(c, L, V, ec, y, nrhs);
  dslash_h<H>(c, dy, y, nrhs);
  if (c.mg.use_alpha)
    step_alpha_half<H>(c, dy, res, nrhs, 1.0, S_BATCH);  // Sec. 3 step-size equation
  else
    fill_pairs(c, S_BATCH, nrhs, 1.0, 0.0);
  update2_half<H>(c, x, y, res, dy, nrhs, S_BATCH, c.mg.nu_post > 0 ? 0 : 2);
  mr_h<H>(c, x, res, p, nrhs, c.mg.nu_post, c.mg.omega, nullptr, true);
}

template void mr_h<f16_t>(Ctx&, HF, HF, HF, int, int, double, const HF*, bool);
template void mr_h<bf16_t>(Ctx&, HF, HF, HF, int, int, double, const HF*, bool);
template void vcycle_h<f16_t>(Ctx&, HF, HF, int);
template void vcycle_h<bf16_t>(Ctx&, HF, HF, int);

// ---------------------------------------------------------------------------
// Outer flexible GCR(k) in FP64 (Sec. 5) for nrhs right-hand sides in
// lockstep, each with its own coefficients; a converged right-hand side is
// frozen (its steps are zero).  b (input) and x (initial guess, output) are
// nrhs internal fields.
int fgcr(Ctx& c, cx<double>* x, const cx<double>* b, int nrhs, const wdmg_solve_params& p, wdmg_solve_stats* st,
         const void* b_canon) {
  Level& L = c.lev[0];
  const size_t n = L.n;
  const size_t bs = n * nrhs;
  const int k = p.restart;
  const bool half = p.precond && (p.mg_prec == WDMG_F16 || p.mg_prec == WDMG_BF16);
  const bool f32 = p.precond && p.mg_prec == WDMG_F32;
  // With a reduced-precision V-cycle the outer basis z_j, w_j = D z_j is kept
  // in FP32 (z_j comes out of the V-cycle in FP32 or 16 bits anyway); x, r and
  // every restart's true residual stay FP64.
  const bool basis32 = f32 || half;
  // FP32 copies of r and z: the FP32 V-cycle's input, and the fixed output of
  // a graph-captured V-cycle
  ensure_outer(c, k, nrhs, f32 || (p.use_graph && basis32), basis32);
  // in place: b in the internal layout lives in the FP32 W basis (two slots'
  // worth) while that basis is idle, at the start and at the end of a cycle
  if (!b && (!basis32 || k < 2 || !b_canon))
    throw Error(WDMG_ERR_ARG, "an in-place solve needs an FP32 outer basis of at least two directions");
  cx<double>* bslot = b ? nullptr : reinterpret_cast<cx<double>*>(c.outer_W32);
  auto load_b = [&]() {
    if (bslot) fine_to_internal<double, double>(c, c.g0, static_cast<const cx<double>*>(b_canon), bslot, nrhs);
  };
  if (bslot) b = bslot;
  if (p.precond) ensure_mg_work(c, nrhs, f32 || half ? WDMG_F32 : WDMG_F64, half ? 1 : 0);
  if (half) ensure_work_h(c, nrhs);
  HalfScope hs(c, half ? p.mg_prec : 0);
  const bool graph = p.precond && p.use_graph;
  if (graph) {
    if (!c.cap_stream) WDMG_HIP(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
    if (!basis32 && nrhs > c.outer_zf_cap) {
      WDMG_HIP(hipStreamSynchronize(c.stream));
      dev_free(c, c.outer_zf);
      c.outer_zf = static_cast<cx<double>*>(dev_alloc(c, (size_t)nrhs * n * sizeof(cx<double>)));
      c.outer_zf_cap = nrhs;
    }
  }
  struct GraphHolder {
    hipStream_t s;
    hipGraphExec_t e = nullptr;
    ~GraphHolder() {
      if (e) {
        (void)hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(e);
      }
    }
  } gh{c.stream};
  hipGraphExec_t& gexec = gh.e;
  long long g_nd = 0, g_ndc[WDMG_MAX_LEVELS] = {0, 0, 0, 0};
  cx<double>* r = c.outer_r;
  const int G = 4;  // scalar block of the outer solve
  // preconditioner application z = M r (Sec. 2 V-cycle) in the chosen
  // precision; zdst is FP32 when basis32, else FP64
  auto apply_M = [&](void* zdst) {
    if (half) {
      Level& L0 = c.lev[0];
      if (p.mg_prec == WDMG_F16) {
        to_half<double, f16_t>(c, r, L0.wh[4], nrhs);
        vcycle_h<f16_t>(c, L0.wh[5], L0.wh[4], nrhs);
        from_half<f16_t, float>(c, L0.wh[5], static_cast<cx<float>*>(zdst), nrhs);
      } else {
        to_half<double, bf16_t>(c, r, L0.wh[4], nrhs);
        vcycle_h<bf16_t>(c, L0.wh[5], L0.wh[4], nrhs);
        from_half<bf16_t, float>(c, L0.wh[5], static_cast<cx<float>*>(zdst), nrhs);
      }
    } else if (f32) {
      convert<float, double>(c, c.outer_r32, r, bs);
      vcycle<float>(c, 0, static_cast<cx<float>*>(zdst), c.outer_r32, nrhs);
    } else {
      vcycle<double>(c, 0, static_cast<cx<double>*>(zdst), r, nrhs);
    }
  };
  // output of a graph-captured V-cycle (a fixed address), and its copy into a
  // basis slot
  void* zfix = basis32 ? static_cast<void*>(c.outer_z32) : static_cast<void*>(c.outer_zf);
  auto copy_z = [&](void* dst, const void* src) {
    if (basis32)
      copy<float>(c, static_cast<cx<float>*>(dst), static_cast<const cx<float>*>(src), bs);
    else
      copy<double>(c, static_cast<cx<double>*>(dst), static_cast<const cx<double>*>(src), bs);
  };
  // Reliable update: with an FP32 basis one cycle cannot bring the true
  // residual much below 1e-7 of its starting value, so a cycle also ends once
  // every active rhs has reduced its recursive residual by kReliable^2 in norm^2.
  constexpr double kReliable = 1e-5;
  double rstart2[kMaxRhs];
  set_scalar(c, S_ERR, 0.0, 0.0);
  load_b();
  norm2_b(c, b, n, nrhs, G, c.dring);
  WDMG_HIP(hipStreamSynchronize(c.stream));
  double bn2[kMaxRhs], tol2[kMaxRhs], act[kMaxRhs];
  int nact = 0;
  for (int q = 0; q < nrhs; ++q) {
    bn2[q] = c.hring[q];
    if (!std::isfinite(bn2[q])) throw Error(WDMG_ERR_NAN, "NaN or Inf in the right-hand side");
    tol2[q] = p.tol * p.tol * bn2[q];
    st[q].iters = st[q].restarts = st[q].converged = 0;
    st[q].true_res = 0.0;
  }
  // r = b - D x
  dslash<double>(c, r, x, nrhs);
  xmy_norm_b(c, b, r, n, nrhs, G);
  auto read_rn = [&](double* out) {
    WDMG_HIP(hipMemcpyAsync(c.hsc, c.dsc + gcr_base(G) + G_RN, nrhs * sizeof(double), hipMemcpyDeviceToHost,
                            c.stream));
    WDMG_HIP(hipStreamSynchronize(c.stream));
    for (int q = 0; q < nrhs; ++q) {
      out[q] = c.hsc[q];
      if (!std::isfinite(out[q])) throw Error(WDMG_ERR_NAN, "NaN in the outer solve");
    }
  };
  double rn2[kMaxRhs];
  read_rn(rn2);
  auto update_active = [&]() {
    nact = 0;
    for (int q = 0; q < nrhs; ++q) {
      const bool on = bn2[q] > 0.0 && rn2[q] > tol2[q] && st[q].iters < p.maxit;
      act[q] = on ? 1.0 : 0.0;
      nact += on;
    }
    set_active(c, G, act, nrhs);
  };
  int total = 0;
  while (true) {
    update_active();
    if (nact == 0) break;
    for (int q = 0; q < nrhs; ++q) rstart2[q] = rn2[q];
    int jn = 0;  // directions of this cycle (x is formed from them at its end)
    for (int j = 0; j < k && nact > 0; ++j) {
      void* z = basis32 ? static_cast<void*>(c.outer_Z32 + (size_t)j * bs) : static_cast<void*>(c.outer_Z + (size_t)j * bs);
      void* w = basis32 ? static_cast<void*>(c.outer_W32 + (size_t)j * bs) : static_cast<void*>(c.outer_W + (size_t)j * bs);
      if (p.precond) {
        if (!graph) {
          apply_M(z);
        } else if (!gexec) {
          // first application: eager; it also measures the coarsest iterations
          c.last_coarse_iters = 0;
          apply_M(zfix);
          copy_z(z, zfix);
          const int fixed = (3 * c.last_coarse_iters + 1) / 2 + 1;
          // capture the V-cycle on a side stream, then replay it on c.stream
          hipStream_t main_stream = c.stream;
          const bool prof = c.prof_on;
          c.prof_on = false;
          c.capturing = true;
          c.coarse_fixed_iters = fixed;
          c.stream = c.cap_stream;
          const long long nd1 = c.n_D;
          long long ndc1[WDMG_MAX_LEVELS];
          for (int l = 0; l < WDMG_MAX_LEVELS; ++l) ndc1[l] = c.n_Dc[l];
          hipGraph_t graph_def = nullptr;
          hipError_t e = hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeRelaxed);
          if (e == hipSuccess) {
            try {
              apply_M(zfix);
            } catch (...) {
              (void)hipStreamEndCapture(c.cap_stream, &graph_def);
              if (graph_def) (void)hipGraphDestroy(graph_def);
              c.stream = main_stream;
              c.capturing = false;
              c.prof_on = prof;
              throw;
            }
            e = hipStreamEndCapture(c.cap_stream, &graph_def);
          }
          c.stream = main_stream;
          c.capturing = false;
          c.prof_on = prof;
          if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph_def, nullptr, nullptr, 0);
          if (graph_def) (void)hipGraphDestroy(graph_def);
          WDMG_HIP(e);
          g_nd = c.n_D - nd1;
          for (int l = 0; l < WDMG_MAX_LEVELS; ++l) g_ndc[l] = c.n_Dc[l] - ndc1[l];
          // the capture itself executed nothing
          c.n_D = nd1;
          for (int l = 0; l < WDMG_MAX_LEVELS; ++l) c.n_Dc[l] = ndc1[l];
        } else {
          WDMG_HIP(hipGraphLaunch(gexec, c.stream));
          c.n_D += g_nd;
          for (int l = 0; l < WDMG_MAX_LEVELS; ++l) c.n_Dc[l] += g_ndc[l];
          copy_z(z, zfix);
        }
      } else if (basis32) {
        convert<float, double>(c, static_cast<cx<float>*>(z), r, bs);
      } else {
        copy<double>(c, static_cast<cx<double>*>(z), r, bs);
      }
      if (basis32) {
        cx<float>* w32 = static_cast<cx<float>*>(w);
        dslash<float>(c, w32, static_cast<cx<float>*>(z), nrhs);
        gcr_orth_b<float>(c, c.outer_W32, w32, r, n, nrhs, j, G);
        gcr_record(c, c.outer_hist, c.outer_av, nrhs, j, k, G);
        gcr_step_b<float>(c, w32, r, n, nrhs, G);
      } else {
        cx<double>* w64 = static_cast<cx<double>*>(w);
        dslash<double>(c, w64, static_cast<cx<double>*>(z), nrhs);
        gcr_orth_b<double>(c, c.outer_W, w64, r, n, nrhs, j, G);
        gcr_record(c, c.outer_hist, c.outer_av, nrhs, j, k, G);
        gcr_step_b<double>(c, w64, r, n, nrhs, G);
      }
      jn = j + 1;
      for (int q = 0; q < nrhs; ++q) st[q].iters += act[q] != 0.0;
      ++total;
      read_rn(rn2);
      bool changed = false, reliable = basis32;
      for (int q = 0; q < nrhs; ++q) {
        if (act[q] == 0.0) continue;
        if (rn2[q] <= tol2[q] || st[q].iters >= p.maxit) changed = true;
        if (rn2[q] > kReliable * kReliable * rstart2[q] && rn2[q] > tol2[q]) reliable = false;
      }
      if (reliable) break;  // recompute the true residual now
      if (changed) update_active();
    }
    // end of the cycle: x += sum_j y_j zt_j, then the true residual in FP64
    if (basis32)
      gcr_combine<float>(c, x, c.outer_Z32, c.outer_hist, c.outer_av, c.outer_y, n, nrhs, jn, k);
    else
      gcr_combine<double>(c, x, c.outer_Z, c.outer_hist, c.outer_av, c.outer_y, n, nrhs, jn, k);
    dslash<double>(c, r, x, nrhs);
    load_b();
    xmy_norm_b(c, b, r, n, nrhs, G);
    read_rn(rn2);
    bool again = false;
    for (int q = 0; q < nrhs; ++q) {
      if (bn2[q] > 0.0 && rn2[q] > tol2[q] && st[q].iters < p.maxit) {
        ++st[q].restarts;
        again = true;
      }
    }
    if (!again) break;
  }
  int rc = WDMG_OK;
  for (int q = 0; q < nrhs; ++q) {
    st[q].converged = bn2[q] == 0.0 || rn2[q] <= tol2[q];
    st[q].true_res = bn2[q] > 0.0 ? std::sqrt(rn2[q] / bn2[q]) : 0.0;
    if (!st[q].converged) rc = WDMG_NOT_CONVERGED;
  }
  (void)total;
  check_flags(c);
  return rc;
}

// ---------------------------------------------------------------------------
// BiCGStab (van der Vorst 1992), FP64, x = 0 start (Sec. 5 comparator).
// z = M r for one rhs: the V-cycle in the precision of pc (FP64 in and out).
static void precond_apply1(Ctx& c, const wdmg_solve_params& pc, const cx<double>* r, cx<double>* z) {
  const size_t n = c.lev[0].n;
  Level& L0 = c.lev[0];
  if (pc.mg_prec == WDMG_F16) {
    to_half<double, f16_t>(c, r, L0.wh[4], 1);
    vcycle_h<f16_t>(c, L0.wh[5], L0.wh[4], 1);
    from_half<f16_t, double>(c, L0.wh[5], z, 1);
  } else if (pc.mg_prec == WDMG_BF16) {
    to_half<double, bf16_t>(c, r, L0.wh[4], 1);
    vcycle_h<bf16_t>(c, L0.wh[5], L0.wh[4], 1);
    from_half<bf16_t, double>(c, L0.wh[5], z, 1);
  } else if (pc.mg_prec == WDMG_F32) {
    convert<float, double>(c, c.outer_r32, r, n);
    vcycle<float>(c, 0, c.outer_z32, c.outer_r32, 1);
    convert<double, float>(c, z, c.outer_z32, n);
  } else {
    vcycle<double>(c, 0, z, r, 1);
  }
}

int bicgstab(Ctx& c, cx<double>* x, const cx<double>* b, double tol, int maxit, wdmg_solve_stats& st,
             const wdmg_solve_params* pc) {
  const size_t n = c.lev[0].n;
  ensure_bicg(c);
  cx<double>* r = c.bicg[0];
  cx<double>* rhat = c.bicg[1];
  cx<double>* p = c.bicg[2];
  cx<double>* v = c.bicg[3];
  cx<double>* s = c.bicg[4];
  cx<double>* t = c.bicg[5];
  cx<double>* ph = c.bicg[6];  // M p
  cx<double>* sh = c.bicg[7];  // M s
  const bool half = pc && (pc->mg_prec == WDMG_F16 || pc->mg_prec == WDMG_BF16);
  if (pc) {
    const bool low = pc->mg_prec != WDMG_F64;
    ensure_outer(c, 1, 1, low, true);
    ensure_mg_work(c, 1, low ? WDMG_F32 : WDMG_F64, half ? 1 : 0);
    if (half) ensure_work_h(c, 1);
  }
  HalfScope hs(c, half ? pc->mg_prec : 0);
  set_scalar(c, S_ERR, 0.0, 0.0);
  norm2<double>(c, b, n, S_TMP + 4);
  const double bn2 = read_scalar(c, S_TMP + 4);
  if (!std::isfinite(bn2)) throw Error(WDMG_ERR_NAN, "NaN or Inf in the right-hand side");
  st.iters = 0;
  st.restarts = 0;
  st.converged = 0;
  zero<double>(c, x, n);
  if (bn2 == 0.0) {
    st.converged = 1;
    st.true_res = 0.0;
    return WDMG_OK;
  }
  const double tol2 = tol * tol * bn2;
  copy<double>(c, r, b, n);
  const int check_every = 8;
  double rn2 = bn2;
  while (st.iters < maxit) {
    copy<double>(c, rhat, r, n);
    dot<double>(c, rhat, r, n, S_BICG + 0);  // rho_new
    set_scalar(c, S_BICG + 6, 1.0, 0.0);     // omega
    bool first = true;
    int since = 0;
    bool breakdown = false;
    while (st.iters < maxit) {
      bicg_p(c, p, r, v, n, first);
      first = false;
      const cx<double>* pp = p;
      if (pc) {
        precond_apply1(c, *pc, p, ph);
        pp = ph;
      }
      dslash<double>(c, v, pp, 1);
      bicg_alpha(c, rhat, v, n);
      bicg_s(c, s, r, v, n);
      const cx<double>* ss = s;
      if (pc) {
        precond_apply1(c, *pc, s, sh);
        ss = sh;
      }
      dslash<double>(c, t, ss, 1);
      bicg_omega(c, t, s, n);
      bicg_xr(c, x, r, pp, s, ss, t, rhat, n);
      ++st.iters;
      if (++since >= check_every || st.iters >= maxit) {
        since = 0;
        WDMG_HIP(hipMemcpyAsync(c.hsc, c.dsc + S_BICG, 10 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
        WDMG_HIP(hipStreamSynchronize(c.stream));
        rn2 = c.hsc[8];
        if (!std::isfinite(rn2)) throw Error(WDMG_ERR_NAN, "NaN in BiCGStab");
        if (rn2 <= tol2) break;
        if (c.hsc[0] == 0.0 && c.hsc[1] == 0.0) {
          breakdown = true;
          break;
        }
      }
    }
    // true residual
    dslash<double>(c, r, x, 1);
    xmy_norm(c, b, r, n, S_RNORM);
    rn2 = read_scalar(c, S_RNORM);
    if (rn2 <= tol2) {
      st.converged = 1;
      break;
    }
    (void)breakdown;
    ++st.restarts;
  }
  st.true_res = std::sqrt(rn2 / bn2);
  check_flags(c);
  return st.converged ? WDMG_OK : WDMG_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// Adaptive setup (Sec. 2): relax the starting vectors on A v = 0, block QR,
// Galerkin coarse operator; recursively.
void free_hierarchy(Ctx& c) {
  WDMG_HIP(hipStreamSynchronize(c.stream));
  for (int l = 0; l < WDMG_MAX_LEVELS; ++l) {
    Level& L = c.lev[l];
    dev_free(c, L.V64);
    dev_free(c, L.V32);
    dev_free(c, L.Dc64);
    dev_free(c, L.Dc32);
    dev_free(c, L.V16);
    dev_free(c, L.Dc16);
    dev_free(c, L.Dc16s);
    dev_free(c, L.Nc64);
    dev_free(c, L.noff);
    for (int i = 0; i < kWork; ++i) {
      if (l > 0) {
        dev_free(c, L.w64[i]);
        dev_free(c, L.w32[i]);
      }
    }
    dev_free(c, L.basisZ);
    dev_free(c, L.basisW);
    dev_free(c, L.xT);
    dev_free(c, L.cpart);
    dev_free(c, L.cpart3);
    dev_free(c, L.chist);
    Level blank;
    if (l == 0) {
      // level 0 work vectors outlive the hierarchy (same geometry)
      for (int i = 0; i < kWork; ++i) {
        blank.w64[i] = L.w64[i];
        blank.w32[i] = L.w32[i];
      }
      blank.cap64 = L.cap64;
      blank.cap32 = L.cap32;
      for (int i = 0; i < 6; ++i) blank.wh[i] = L.wh[i];
      blank.caph = L.caph;
    }
    L = blank;
  }
  c.have_mg = false;
  c.released = false;
  c.nlevels = 0;
  init_level0(c);
}

void init_level0(Ctx& c) {
  Level& L = c.lev[0];
  L.l = 0;
  std::memcpy(L.dims, c.dims, sizeof(L.dims));
  L.g = c.g0;
  L.nsite = c.g0.vol;
  L.dof = 12;
  L.n = (size_t)c.g0.vpad * 12;
}

// Sec. 2 setup relaxation: setup_iters MR steps on A v = 0 for all Nv
// vectors at once (each its own step size), in precision R, in place on X.
// The batch is cut only when the work fields would exceed a 16 GB budget.
template <typename R>
static void relax_batch(Ctx& c, int l, cx<R>* V, int nv, int iters, double omega) {
  Level& F = c.lev[l];
  const size_t n = F.n;
  const size_t field = n * sizeof(cx<R>);
  size_t kb = ((size_t)16 << 30) / (2 * field);
  if (kb < 1) kb = 1;
  if (kb > (size_t)nv) kb = nv;
  if (kb > (size_t)kMaxRhs) kb = kMaxRhs;
  cx<R>* Rb = static_cast<cx<R>*>(dev_alloc(c, kb * field));
  cx<R>* Pb = static_cast<cx<R>*>(dev_alloc(c, kb * field));
  if (l == 0) dots_buffer(c, (int)kb);
  for (int k0 = 0; k0 < nv; k0 += (int)kb) {
    const int nb = (nv - k0) < (int)kb ? (nv - k0) : (int)kb;
    cx<R>* X = V + (size_t)k0 * n;
    // r = 0 - A x
    apply_op<R>(c, l, Rb, X, nb);
    neg<R>(c, Rb, (size_t)nb * n);
    for (int it = 0; it < iters; ++it) {
      if (l == 0) {
        dslash_mr<R>(c, Pb, Rb, nb, omega, S_BATCH);
      } else {
        apply_op<R>(c, l, Pb, Rb, nb);
        step_alpha_batch<R>(c, Pb, Rb, n, n, nb, omega, S_BATCH);
      }
      update2_batch<R>(c, X, Rb, Rb, Pb, n, n, nb, S_BATCH);
    }
  }
  WDMG_HIP(hipStreamSynchronize(c.stream));
  dev_free(c, Rb);
  dev_free(c, Pb);
}

// The same relaxation at level 0 with the candidates, residuals and A r in
// 16-bit storage (per-site scales, FP32 arithmetic; the dslash launch fuses
// the MR partial sums as in the 16-bit smoother).  The batch is cut when its
// three 16-bit fields would exceed a 16 GB budget.
template <typename H>
static void relax_batch_h(Ctx& c, cx<double>* V, int nv, int iters, double omega) {
  const size_t n = c.lev[0].n;
  const size_t per_rhs = (size_t)c.g0.vpad * (12 * 4 + 4) * 3;
  size_t kb = ((size_t)16 << 30) / per_rhs;
  if (kb < 1) kb = 1;
  if (kb > (size_t)nv) kb = nv;
  if (kb > (size_t)kMaxRhs) kb = kMaxRhs;
  HF X = hf_alloc(c, (int)kb), Rb = hf_alloc(c, (int)kb), Pb = hf_alloc(c, (int)kb);
  dots_buffer(c, (int)kb);
  for (int k0 = 0; k0 < nv; k0 += (int)kb) {
    const int nb = (nv - k0) < (int)kb ? (nv - k0) : (int)kb;
    to_half<double, H>(c, V + (size_t)k0 * n, X, nb);
    // r = 0 - A x
    dslash_h<H>(c, Rb, X, nb);
    hf_neg(c, Rb, nb);
    for (int it = 0; it < iters; ++it) {
      dslash_h_mr<H>(c, Pb, Rb, nb, omega, S_BATCH);
      update2_half<H>(c, X, Rb, Rb, Pb, nb, S_BATCH, 0);
    }
    from_half<H, double>(c, X, V + (size_t)k0 * n, nb);
  }
  WDMG_HIP(hipStreamSynchronize(c.stream));
  hf_free(c, X);
  hf_free(c, Rb);
  hf_free(c, Pb);
}

static void relax(Ctx& c, int l, const wdmg_level_params& lp, double omega) {
  Level& F = c.lev[l];
  if (lp.setup_prec == WDMG_F16 || lp.setup_prec == WDMG_BF16) {
    if (lp.setup_prec == WDMG_F16)
      relax_batch_h<f16_t>(c, F.V64, lp.nv, lp.setup_iters, omega);
    else
      relax_batch_h<bf16_t>(c, F.V64, lp.nv, lp.setup_iters, omega);
    return;
  }
  if (lp.setup_prec == WDMG_F32) {
    const size_t nn = (size_t)lp.nv * F.n;
    convert<float, double>(c, F.V32, F.V64, nn);
    relax_batch<float>(c, l, F.V32, lp.nv, lp.setup_iters, omega);
    convert<double, float>(c, F.V64, F.V32, nn);
  } else {
    relax_batch<double>(c, l, F.V64, lp.nv, lp.setup_iters, omega);
  }
}

// Sec. 2 adaptive augmentation of the candidates of level l (already relaxed
// in F.V64): for k = 1..nv-1 the two-level multigrid of the first k candidates
// (block QR in place, Galerkin D_c with 2k coarse dof, level l+1 solved as the
// coarsest) is applied `iters` times to candidate k as x <- x - M A x, in FP64.
// The QR of the first k columns leaves earlier, already orthonormal columns
// unchanged (Q is unique with diag(R) > 0), so it is redone in place each step.
// Work space of level l+1 and the coarsest basis are sized for the final nv.
static void adapt_candidates(Ctx& c, int l, int iters) {
  Level& F = c.lev[l];
  Level& C = c.lev[l + 1];
  const int nv = F.nv;
  const int saved_levels = c.nlevels;
  c.nlevels = l + 2;
  C.dof = 2 * nv;
  C.n = (size_t)C.nsite * C.dof;
  ensure_work<double>(c, l, 1);
  ensure_work<double>(c, l + 1, 1);
  ensure_coarsest_basis(c, 1);
  cx<double>* ax = static_cast<cx<double>*>(dev_alloc(c, F.n * sizeof(cx<double>)));
  cx<double>* mx = static_cast<cx<double>*>(dev_alloc(c, F.n * sizeof(cx<double>)));
  for (int k = 1; k < nv; ++k) {
    F.nv = k;
    if (l == 0)
      block_qr0(c, F, F.V64);
    else
      block_qrC(c, F, F.V64);
    C.dof = 2 * k;
    C.n = (size_t)C.nsite * C.dof;
    if (l == 0)
      coarse_build0(c, F, C);
    else
      coarse_buildC(c, F, C);
    cx<double>* x = F.V64 + (size_t)k * F.n;
    for (int it = 0; it < iters; ++it) {
      apply_op<double>(c, l, ax, x, 1);
      vcycle<double>(c, l, mx, ax, 1);
      xmy<double>(c, x, mx, F.n);  // mx = x - M A x
      copy<double>(c, x, mx, F.n);
    }
    check_flags(c);
  }
  WDMG_HIP(hipStreamSynchronize(c.stream));
  dev_free(c, ax);
  dev_free(c, mx);
  F.nv = nv;
  C.dof = 2 * nv;
  C.n = (size_t)C.nsite * C.dof;
  c.nlevels = saved_levels;
}

void mg_setup(Ctx& c, const wdmg_mg_params& p) {
  if (!c.have_gauge) throw Error(WDMG_ERR_NOT_SETUP, "set the gauge field before the multigrid setup");
  if (p.n_levels < 2 || p.n_levels > WDMG_MAX_LEVELS - 1)
    throw Error(WDMG_ERR_ARG, "n_levels must be 2 or 3");
  if (!(p.omega > 0.0 && p.omega < 2.0)) throw Error(WDMG_ERR_ARG, "omega must lie in (0, 2)");
  if (p.nu_pre < 0 || p.nu_post < 0 || p.coarse_maxit < 1 || p.coarse_restart < 1 || p.coarse_restart > 128 ||
      !(p.coarse_tol > 0.0))
    throw Error(WDMG_ERR_ARG, "bad cycle parameters");
  // validate geometry of every level before allocating
  int dims[4];
  std::memcpy(dims, c.dims, sizeof(dims));
  for (int l = 0; l < p.n_levels - 1; ++l) {
    const wdmg_level_params& lp = p.level[l];
    if (lp.nv < 1 || lp.nv > 32) throw Error(WDMG_ERR_ARG, "nv must be in 1..32");
    if (lp.setup_iters < 0) throw Error(WDMG_ERR_ARG, "setup_iters must be >= 0");
    if (lp.setup_prec < WDMG_F64 || lp.setup_prec > WDMG_BF16)
      throw Error(WDMG_ERR_ARG, "setup_prec must be WDMG_F64, WDMG_F32, WDMG_F16 or WDMG_BF16");
    if (l > 0 && lp.setup_prec != WDMG_F64 && lp.setup_prec != WDMG_F32)
      throw Error(WDMG_ERR_ARG, "16-bit setup relaxation exists for level 0 only");
    if (lp.adapt_iters < 0) throw Error(WDMG_ERR_ARG, "adapt_iters must be >= 0");
    if (!lp.vectors) throw Error(WDMG_ERR_ARG, "starting vectors are required for every level");
    int bvol = 1;
    for (int mu = 0; mu < 4; ++mu) {
      if (lp.block[mu] < 1 || dims[mu] % lp.block[mu] != 0)
        throw Error(WDMG_ERR_DIMS, "aggregate extents must divide the level's extents");
      bvol *= lp.block[mu];
      dims[mu] /= lp.block[mu];
    }
    const int dof = l == 0 ? 12 : 2 * p.level[l - 1].nv;
    if (bvol * dof / 2 < lp.nv) throw Error(WDMG_ERR_DIMS, "aggregate too small for nv vectors");
    if (p.normal) {
      for (int mu = 0; mu < 4; ++mu)
        if (lp.block[mu] < 2 || dims[mu] < 3)
          throw Error(WDMG_ERR_DIMS, "a normal-equation hierarchy needs aggregates of extent >= 2 and coarse "
                                     "extents >= 3");
    }
  }
  if (p.normal && p.n_levels != 2) throw Error(WDMG_ERR_ARG, "a normal-equation hierarchy has 2 levels");
  if (p.normal && p.level[0].adapt_iters > 0)
    throw Error(WDMG_ERR_ARG, "the adaptive augmentation runs the direct V-cycle: not with normal = 1");
  free_hierarchy(c);
  set_scalar(c, S_ERR, 0.0, 0.0);
  c.mg = p;
  c.nlevels = p.n_levels;
  c.setup_mass = c.mass;
  init_level0(c);
  for (int l = 0; l < p.n_levels - 1; ++l) {
    const wdmg_level_params& lp = p.level[l];
    Level& F = c.lev[l];
    Level& C = c.lev[l + 1];
    std::memcpy(F.block, lp.block, sizeof(F.block));
    F.nv = lp.nv;
    F.V64 = static_cast<cx<double>*>(dev_alloc(c, (size_t)lp.nv * F.n * sizeof(cx<double>)));
    F.V32 = static_cast<cx<float>*>(dev_alloc(c, (size_t)lp.nv * F.n * sizeof(cx<float>)));
    const cx<double>* src = static_cast<const cx<double>*>(lp.vectors);
    if (l == 0)
      fine_to_internal<double, double>(c, F.g, src, F.V64, lp.nv);
    else
      copy<double>(c, F.V64, src, (size_t)lp.nv * F.n);
    if (lp.setup_iters > 0) {
      if (p.normal)
        normal_relax(c, F, lp.nv, lp.setup_iters, p.omega);  // candidates of D^dagger D v = 0
      else
        relax(c, l, lp, p.omega);
    }
    // coarse level geometry
    C.l = l + 1;
    int one[4] = {1, 1, 1, 1};
    for (int mu = 0; mu < 4; ++mu) C.dims[mu] = F.dims[mu] / lp.block[mu];
    C.g = make_geom(C.dims, one);
    C.nsite = C.g.vol;
    C.dof = 2 * lp.nv;
    C.n = (size_t)C.nsite * C.dof;
    const size_t dcn = (size_t)C.nsite * 9 * C.dof * C.dof;
    C.Dc64 = static_cast<cx<double>*>(dev_alloc(c, dcn * sizeof(cx<double>)));
    C.Dc32 = static_cast<cx<float>*>(dev_alloc(c, dcn * sizeof(cx<float>)));
    if (lp.adapt_iters > 0 && lp.nv > 1) adapt_candidates(c, l, lp.adapt_iters);
    if (l == 0)
      block_qr0(c, F, F.V64);
    else
      block_qrC(c, F, F.V64);
    check_flags(c);
    convert<float, double>(c, F.V32, F.V64, (size_t)lp.nv * F.n);
    if (l == 0)
      coarse_build0(c, F, C);
    else
      coarse_buildC(c, F, C);
    convert<float, double>(c, C.Dc32, C.Dc64, dcn);
    if (p.normal) normal_build(c, F, C);
  }
  // coarse-level GCR blocks: every right-hand side active
  {
    double ones[kMaxRhs];
    for (int q = 0; q < kMaxRhs; ++q) ones[q] = 1.0;
    for (int l = 1; l < p.n_levels; ++l) set_active(c, l, ones, kMaxRhs);
  }
  WDMG_HIP(hipStreamSynchronize(c.stream));
  check_flags(c);
  c.have_mg = true;
}

void release_unused(Ctx& c, int kind) {
  if (!c.have_mg) throw Error(WDMG_ERR_NOT_SETUP, "no multigrid hierarchy set up");
  if (kind != WDMG_F16 && kind != WDMG_BF16) throw Error(WDMG_ERR_ARG, "mg_prec must be WDMG_F16 or WDMG_BF16");
  Level& L0 = c.lev[0];
  v16(c, L0, kind);
  for (int l = 1; l < c.nlevels - 1; ++l) ensure_dc16(c, c.lev[l], kind);
  WDMG_HIP(hipStreamSynchronize(c.stream));
  dev_free(c, L0.V64);
  dev_free(c, L0.V32);
  L0.V64 = nullptr;
  L0.V32 = nullptr;
  for (int l = 1; l < c.nlevels - 1; ++l) {
    Level& C = c.lev[l];
    dev_free(c, C.Dc64);
    dev_free(c, C.Dc32);
    C.Dc64 = nullptr;
    C.Dc32 = nullptr;
  }
  c.released = true;
}

void ensure_outer(Ctx& c, int k, int nrhs, bool need32, bool basis32) {
  const size_t n = (size_t)c.g0.vpad * 12;
  if (nrhs > c.outer_cap) {
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.outer_r);
    c.outer_r = static_cast<cx<double>*>(dev_alloc(c, (size_t)nrhs * n * sizeof(cx<double>)));
    c.outer_cap = nrhs;
  }
  if (!basis32 && (k > c.outer_k || nrhs > c.outer_capB)) {
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.outer_Z);
    dev_free(c, c.outer_W);
    const int kk = k > c.outer_k ? k : c.outer_k;
    const int cc = nrhs > c.outer_capB ? nrhs : c.outer_capB;
    c.outer_Z = static_cast<cx<double>*>(dev_alloc(c, (size_t)kk * cc * n * sizeof(cx<double>)));
    c.outer_W = static_cast<cx<double>*>(dev_alloc(c, (size_t)kk * cc * n * sizeof(cx<double>)));
    c.outer_k = kk;
    c.outer_capB = cc;
  }
  if (k > c.outer_histk || nrhs > c.outer_histcap) {
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.outer_hist);
    dev_free(c, c.outer_av);
    dev_free(c, c.outer_y);
    const int kk = k > c.outer_histk ? k : c.outer_histk;
    const int cc = nrhs > c.outer_histcap ? nrhs : c.outer_histcap;
    c.outer_hist = static_cast<cx<double>*>(dev_alloc(c, (size_t)cc * kk * kk * sizeof(cx<double>)));
    c.outer_av = static_cast<cx<double>*>(dev_alloc(c, (size_t)cc * kk * sizeof(cx<double>)));
    c.outer_y = static_cast<cx<double>*>(dev_alloc(c, (size_t)cc * kk * sizeof(cx<double>)));
    c.outer_histk = kk;
    c.outer_histcap = cc;
  }
  if (basis32 && (k > c.outer_k32 || nrhs > c.outer_capB32)) {
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.outer_Z32);
    dev_free(c, c.outer_W32);
    const int kk = k > c.outer_k32 ? k : c.outer_k32;
    const int cc = nrhs > c.outer_capB32 ? nrhs : c.outer_capB32;
    c.outer_Z32 = static_cast<cx<float>*>(dev_alloc(c, (size_t)kk * cc * n * sizeof(cx<float>)));
    c.outer_W32 = static_cast<cx<float>*>(dev_alloc(c, (size_t)kk * cc * n * sizeof(cx<float>)));
    c.outer_k32 = kk;
    c.outer_capB32 = cc;
  }
  if (need32 && nrhs > c.outer_cap32) {
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.outer_r32);
    dev_free(c, c.outer_z32);
    c.outer_r32 = static_cast<cx<float>*>(dev_alloc(c, (size_t)nrhs * n * sizeof(cx<float>)));
    c.outer_z32 = static_cast<cx<float>*>(dev_alloc(c, (size_t)nrhs * n * sizeof(cx<float>)));
    c.outer_cap32 = nrhs;
  }
}

void ensure_bicg(Ctx& c) {
  if (c.bicg[0]) return;
  const size_t n = (size_t)c.g0.vpad * 12;
  for (cx<double>*& f : c.bicg) f = static_cast<cx<double>*>(dev_alloc(c, n * sizeof(cx<double>)));
}

}  // namespace wdmg
