// extern "C" entry points of libwdmg (declared in include/wdmg.h).  Each call
// validates its arguments on the host, runs the drivers, and turns any
// wdmg::Error into a return code; no exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fine_field.h"
#include "internal.h"
#include "solver.h"

using namespace wdmg;

struct wdmg_ctx : Ctx {};

// ---------------------------------------------------------------------------
// Scratch of wdmg_apply_D_noalloc: the internal-layout input and output fields
// live in this file-scope device array instead of library allocations.  Its
// device address is taken once per device in wdmg_create (with that device
// current); host code uses only that address, never the array's name.
static constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static void* g_scratch[kMaxDevices] = {};
static hipError_t g_scratch_rc[kMaxDevices] = {};
static std::once_flag g_scratch_once[kMaxDevices];

namespace {

// Records the scratch address of the current device (once per device).
void init_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::call_once(g_scratch_once[dev], [dev]() {
    void* p = nullptr;
    g_scratch_rc[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g_scratch_rc[dev] == hipSuccess) g_scratch[dev] = p;
  });
}

template <class F>
int guarded(wdmg_ctx* c, F&& f) {
  if (!c) return WDMG_ERR_ARG;
  c->err.clear();
  try {
    return f();
  } catch (const Error& e) {
    c->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    c->err = "host allocation failed";
    return WDMG_ERR_OOM;
  } catch (const std::exception& e) {
    c->err = e.what();
    return WDMG_ERR_HIP;
  }
}

void need_gauge(Ctx& c) {
  if (!c.have_gauge) throw Error(WDMG_ERR_NOT_SETUP, "no gauge field set");
}
void need_mg(Ctx& c, int level, bool coarse) {
  if (!c.have_mg) throw Error(WDMG_ERR_NOT_SETUP, "no multigrid hierarchy set up");
  const int hi = coarse ? c.nlevels - 1 : c.nlevels - 2;
  const int lo = coarse ? 1 : 0;
  if (level < lo || level > hi) throw Error(WDMG_ERR_ARG, "level out of range");
}
void need_prec(int prec) {
  if (prec != WDMG_F64 && prec != WDMG_F32 && prec != WDMG_F16 && prec != WDMG_BF16)
    throw Error(WDMG_ERR_ARG, "unknown precision");
}
bool is_half(int prec) { return prec == WDMG_F16 || prec == WDMG_BF16; }

// 16-bit scratch fine fields for nrhs right-hand sides
void ensure_ioh(Ctx& c, int nrhs) {
  if (nrhs <= c.ioh_cap) return;
  WDMG_HIP(hipStreamSynchronize(c.stream));
  for (HF& f : c.ioh) {
    hf_free(c, f);
    f = hf_alloc(c, nrhs);
  }
  c.ioh_cap = nrhs;
}

template <typename H>
void apply_D_half(Ctx& c, void* out, const void* in, int nrhs) {
  ensure_ioh(c, nrhs);
  canon_to_half<H>(c, static_cast<const cx<float>*>(in), c.ioh[0], nrhs);
  dslash_h<H>(c, c.ioh[1], c.ioh[0], nrhs);
  half_to_canon<H>(c, c.ioh[1], static_cast<cx<float>*>(out), nrhs);
}

template <typename H>
void roundtrip_half(Ctx& c, void* out, const void* in, int nrhs) {
  ensure_ioh(c, nrhs);
  canon_to_half<H>(c, static_cast<const cx<float>*>(in), c.ioh[0], nrhs);
  half_to_canon<H>(c, c.ioh[0], static_cast<cx<float>*>(out), nrhs);
}

template <typename H>
void restrict_half(Ctx& c, void* cout, const void* fin, int nrhs) {
  ensure_ioh(c, nrhs);
  const void* V = v16(c, c.lev[0], half_kind<H>());
  canon_to_half<H>(c, static_cast<const cx<float>*>(fin), c.ioh[0], nrhs);
  restrict0_h<H>(c, c.lev[0], V, c.ioh[0], static_cast<cx<float>*>(cout), nrhs);
}

template <typename H>
void prolong_half(Ctx& c, void* fout, const void* cin, int nrhs) {
  ensure_ioh(c, nrhs);
  const void* V = v16(c, c.lev[0], half_kind<H>());
  prolong0_h<H>(c, c.lev[0], V, static_cast<const cx<float>*>(cin), c.ioh[0], nrhs);
  half_to_canon<H>(c, c.ioh[0], static_cast<cx<float>*>(fout), nrhs);
}

// MR on the fine level in 16-bit storage.  The starting residual b - D x is
// formed in FP32; x and r are then held in 16 bits for the iterations.
template <typename H>
void smooth_half0(Ctx& c, void* x, const void* b, int nrhs, int iters) {
  const size_t n = c.lev[0].n;
  ensure_io(c, 2 * n * nrhs * sizeof(cx<float>));
  ensure_ioh(c, nrhs);
  cx<float>* xi = static_cast<cx<float>*>(c.io_a);
  cx<float>* ri = xi + n * nrhs;
  cx<float>* bi = static_cast<cx<float>*>(c.io_b);
  fine_to_internal<float, float>(c, c.g0, static_cast<const cx<float>*>(x), xi, nrhs);
  fine_to_internal<float, float>(c, c.g0, static_cast<const cx<float>*>(b), bi, nrhs);
  dslash<float>(c, ri, xi, nrhs);
  xmy<float>(c, bi, ri, n * nrhs);
  to_half<float, H>(c, xi, c.ioh[0], nrhs);
  to_half<float, H>(c, ri, c.ioh[1], nrhs);
  const double omega = c.have_mg ? c.mg.omega : 0.8;
  mr_h<H>(c, c.ioh[0], c.ioh[1], c.ioh[2], nrhs, iters, omega);
  half_to_canon<H>(c, c.ioh[0], static_cast<cx<float>*>(x), nrhs);
}
void need_ptr(const void* p, const char* what) {
  if (!p) throw Error(WDMG_ERR_ARG, std::string("null pointer: ") + what);
}
void need_nrhs(int nrhs) {
  if (nrhs < 1 || nrhs > 65535) throw Error(WDMG_ERR_ARG, "nrhs must be in 1..65535");
}

// canonical fine layout <-> level-0 internal layout, in precision R
template <typename R>
void fine_in(Ctx& c, const void* canon, cx<R>* dst, int nrhs) {
  fine_to_internal<R, R>(c, c.g0, static_cast<const cx<R>*>(canon), dst, nrhs);
}
template <typename R>
void fine_out(Ctx& c, const cx<R>* src, void* canon, int nrhs) {
  fine_to_canonical<R, R>(c, c.g0, src, static_cast<cx<R>*>(canon), nrhs);
}

template <typename R>
void apply_D_impl(Ctx& c, void* out, const void* in, int nrhs) {
  const size_t n = (size_t)c.g0.vpad * 12;
  ensure_io(c, n * nrhs * sizeof(cx<R>));
  cx<R>* a = static_cast<cx<R>*>(c.io_a);
  cx<R>* b = static_cast<cx<R>*>(c.io_b);
  fine_in<R>(c, in, a, nrhs);
  dslash<R>(c, b, a, nrhs);
  fine_out<R>(c, b, out, nrhs);
}

template <typename R>
const cx<R>* dc_of(const Level& L) {
  const cx<R>* p;
  if constexpr (sizeof(R) == 8)
    p = L.Dc64;
  else
    p = L.Dc32;
  if (!p) throw Error(WDMG_ERR_ARG, "coarse blocks released by wdmg_release_unused");
  return p;
}

template <typename R>
void restrict_impl(Ctx& c, int level, void* cout, const void* fin, int nrhs) {
  cx<R>* co = static_cast<cx<R>*>(cout);
  if (level == 0) {
    const size_t n = c.lev[0].n;
    ensure_io(c, n * nrhs * sizeof(cx<R>));
    cx<R>* a = static_cast<cx<R>*>(c.io_a);
    fine_in<R>(c, fin, a, nrhs);
    restrict_to<R>(c, 0, a, co, nrhs);
  } else {
    restrict_to<R>(c, level, static_cast<const cx<R>*>(fin), co, nrhs);
  }
}

template <typename R>
void prolong_impl(Ctx& c, int level, void* fout, const void* cin, int nrhs) {
  const cx<R>* ci = static_cast<const cx<R>*>(cin);
  if (level == 0) {
    const size_t n = c.lev[0].n;
    ensure_io(c, n * nrhs * sizeof(cx<R>));
    cx<R>* a = static_cast<cx<R>*>(c.io_a);
    prolong_from<R>(c, 0, ci, a, nrhs);
    fine_out<R>(c, a, fout, nrhs);
  } else {
    prolong_from<R>(c, level, ci, static_cast<cx<R>*>(fout), nrhs);
  }
}

template <typename R>
void smooth_impl(Ctx& c, int level, void* x, const void* b, int nrhs, int iters) {
  Level& L = c.lev[level];
  const size_t n = L.n;
  const size_t ncan = level == 0 ? (size_t)c.g0.vol * 12 : n;  // canonical stride per rhs
  ensure_io(c, 2 * n * sizeof(cx<R>));
  cx<R>* xi = static_cast<cx<R>*>(c.io_a);
  cx<R>* ri = xi + n;
  cx<R>* p = static_cast<cx<R>*>(c.io_b);
  cx<R>* bi = p + n;
  const double omega = c.have_mg ? c.mg.omega : 0.8;
  for (int k = 0; k < nrhs; ++k) {
    if (level == 0) {
      fine_in<R>(c, static_cast<const cx<R>*>(x) + (size_t)k * ncan, xi, 1);
      fine_in<R>(c, static_cast<const cx<R>*>(b) + (size_t)k * ncan, bi, 1);
    } else {
      copy<R>(c, xi, static_cast<const cx<R>*>(x) + (size_t)k * n, n);
      copy<R>(c, bi, static_cast<const cx<R>*>(b) + (size_t)k * n, n);
    }
    apply_op<R>(c, level, ri, xi, 1);
    xmy<R>(c, bi, ri, n);
    mr<R>(c, level, xi, ri, p, 1, iters, omega);
    if (level == 0)
      fine_out<R>(c, xi, static_cast<cx<R>*>(x) + (size_t)k * ncan, 1);
    else
      copy<R>(c, static_cast<cx<R>*>(x) + (size_t)k * n, xi, n);
  }
}

// Internal x (and, unless the solve runs in place, b) for nrhs right-hand sides.
void ensure_solve_io(Ctx& c, int nrhs, bool need_b = true) {
  const size_t n = (size_t)c.g0.vpad * 12;
  if (nrhs > c.sol_cap) {
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.sol_x);
    c.sol_x = static_cast<cx<double>*>(dev_alloc(c, (size_t)nrhs * n * sizeof(cx<double>)));
    c.sol_cap = nrhs;
  }
  if (need_b && nrhs > c.sol_bcap) {
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.sol_b);
    c.sol_b = static_cast<cx<double>*>(dev_alloc(c, (size_t)nrhs * n * sizeof(cx<double>)));
    c.sol_bcap = nrhs;
  }
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

void wdmg_default_mg_params(wdmg_mg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n_levels = 2;
  for (int l = 0; l < WDMG_MAX_LEVELS - 1; ++l) {
    for (int mu = 0; mu < 4; ++mu) p->level[l].block[mu] = 4;
    p->level[l].nv = 20;
    p->level[l].setup_iters = 100;
    p->level[l].vectors = nullptr;
    p->level[l].setup_prec = WDMG_F64;
  }
  p->normal = 0;
  p->omega = 0.8;
  p->nu_pre = 2;
  p->nu_post = 2;
  p->coarse_cycles = 4;
  p->coarse_tol = 1e-1;
  p->coarse_maxit = 200;
  p->coarse_restart = 32;
  p->use_alpha = 1;
}

void wdmg_default_solve_params(wdmg_solve_params* p) {
  if (!p) return;
  p->tol = 1e-10;
  p->restart = 50;
  p->maxit = 1000;
  p->precond = 1;
  p->mg_prec = WDMG_F64;
  p->use_graph = 0;
  p->outer = 0;
  p->in_place = 0;
}

int wdmg_create(wdmg_ctx** out, const int dims[4], const wdmg_alloc* alloc, void* hip_stream) {
  if (!out || !dims) return WDMG_ERR_ARG;
  *out = nullptr;
  long long vol = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (dims[mu] < 2) return WDMG_ERR_DIMS;
    vol *= dims[mu];
  }
  if (vol * 12 > (1LL << 31)) return WDMG_ERR_DIMS;
  wdmg_ctx* c = new (std::nothrow) wdmg_ctx();
  if (!c) return WDMG_ERR_OOM;
  std::memcpy(c->dims, dims, sizeof(c->dims));
  std::memset(c->tune_dslash, -1, sizeof(c->tune_dslash));
  std::memset(c->tune_group, -1, sizeof(c->tune_group));
  for (int k = 0; k < WDMG_TUNE_COUNT; ++k) c->tune_force[k] = WDMG_TUNE_AUTO;
  int B[4];
  for (int mu = 0; mu < 4; ++mu) B[mu] = dims[mu] % 4 == 0 ? 4 : (dims[mu] % 2 == 0 ? 2 : 1);
  c->g0 = make_geom(dims, B);
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return WDMG_ERR_HIP;
  }
  init_scratch(c->device);
  if (alloc) {
    c->alloc = *alloc;
    if (!alloc->alloc || !alloc->free) {
      delete c;
      return WDMG_ERR_ARG;
    }
  }
  int rc = guarded(c, [&]() {
    c->dsc = static_cast<double*>(dev_alloc(*c, S_TOTAL * sizeof(double)));
    c->partials = static_cast<double*>(dev_alloc(*c, (size_t)8192 * 16 * sizeof(double)));

    WDMG_HIP(hipMemsetAsync(c->dsc, 0, S_TOTAL * sizeof(double), c->stream));

    WDMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->hsc), kHscSize * sizeof(double), hipHostMallocDefault));
    WDMG_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->hring), kRing * kMaxRhs * sizeof(double),
                           hipHostMallocMapped | hipHostMallocCoherent));
    WDMG_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->dring), c->hring, 0));
    for (int i = 0; i < kRing; ++i) WDMG_HIP(hipEventCreateWithFlags(&c->ring_ev[i], hipEventDisableTiming));
    init_level0(*c);
    WDMG_HIP(hipStreamSynchronize(c->stream));
    return WDMG_OK;
  });
  if (rc != WDMG_OK) {
    wdmg_destroy(c);
    return rc;
  }
  *out = c;
  return WDMG_OK;
}

void wdmg_destroy(wdmg_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  while (!c->bufs.empty()) {
    void* p = c->bufs.back().p;
    c->bufs.pop_back();
    if (c->alloc.free)
      c->alloc.free(p, c->alloc.user);
    else
      (void)hipFree(p);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->hsc) (void)hipHostFree(c->hsc);
  if (c->hring) (void)hipHostFree(c->hring);
  for (int i = 0; i < kRing; ++i)
    if (c->ring_ev[i]) (void)hipEventDestroy(c->ring_ev[i]);
  for (auto& r : c->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  delete c;
}

const char* wdmg_last_error(const wdmg_ctx* c) { return c ? c->err.c_str() : "null context"; }

int wdmg_set_gauge(wdmg_ctx* c, const void* U, int t_bc) {
  return guarded(c, [&]() {
    need_ptr(U, "U");
    if (t_bc != 1 && t_bc != -1) throw Error(WDMG_ERR_ARG, "t_bc must be +1 or -1");
    if (c->have_mg) free_hierarchy(*c);
    const size_t n = (size_t)c->g0.vpad * kLinkComp;
    if (!c->U64) {
      c->U64 = static_cast<cx<double>*>(dev_alloc(*c, n * sizeof(cx<double>)));
      c->U32 = static_cast<cx<float>*>(dev_alloc(*c, n * sizeof(cx<float>)));
    }
    set_scalar(*c, S_ERR + 2, 0.0, 0.0);
    c->u16_kind = 0;
    gauge_import(*c, static_cast<const cx<double>*>(U), t_bc);
    c->t_bc = t_bc;
    c->have_gauge = false;
    if (read_scalar(*c, S_ERR + 2) != 0.0) {
      set_scalar(*c, S_ERR + 2, 0.0, 0.0);
      throw Error(WDMG_ERR_ARG, "links must be SU(3): third row != conj(row0 x row1) to 1e-10");
    }
    c->have_gauge = true;
    return WDMG_OK;
  });
}

int wdmg_release_unused(wdmg_ctx* c, int mg_prec) {
  return guarded(c, [&]() {
    release_unused(*c, mg_prec);
    return WDMG_OK;
  });
}

int wdmg_set_mass(wdmg_ctx* c, double m) {
  return guarded(c, [&]() {
    if (!std::isfinite(m)) throw Error(WDMG_ERR_ARG, "mass must be finite");
    if (c->have_mg && c->released)
      throw Error(WDMG_ERR_ARG, "coarse blocks released by wdmg_release_unused: set up again to change the mass");
    c->mass = m;
    if (c->have_mg) {
      const double dm = m - c->setup_mass;
      for (int l = 1; l < c->nlevels; ++l) coarse_shift(*c, c->lev[l], dm);
      c->setup_mass = m;
      // (D^dagger D)_c is not a shift of itself: probe it again at the new mass
      if (c->lev[1].Nc64) normal_build(*c, c->lev[0], c->lev[1]);
    }
    return WDMG_OK;
  });
}

int wdmg_apply_D(wdmg_ctx* c, void* out, const void* in, int nrhs, int prec) {
  return guarded(c, [&]() {
    need_ptr(out, "out");
    need_ptr(in, "in");
    need_nrhs(nrhs);
    need_prec(prec);
    need_gauge(*c);
    if (out == in) throw Error(WDMG_ERR_ARG, "out must differ from in");
    if (prec == WDMG_F64)
      apply_D_impl<double>(*c, out, in, nrhs);
    else if (prec == WDMG_F32)
      apply_D_impl<float>(*c, out, in, nrhs);
    else if (prec == WDMG_F16)
      apply_D_half<f16_t>(*c, out, in, nrhs);
    else
      apply_D_half<bf16_t>(*c, out, in, nrhs);
    return WDMG_OK;
  });
}

int wdmg_apply_D_noalloc(wdmg_ctx* c, void* out, const void* in, int nrhs, int prec) {
  return guarded(c, [&]() {
    need_ptr(out, "out");
    need_ptr(in, "in");
    need_nrhs(nrhs);
    need_prec(prec);
    need_gauge(*c);
    if (out == in) throw Error(WDMG_ERR_ARG, "out must differ from in");
    if (prec != WDMG_F64 && prec != WDMG_F32)
      throw Error(WDMG_ERR_ARG, "wdmg_apply_D_noalloc takes WDMG_F64 or WDMG_F32");
    const int dev = c->device;
    if (dev < 0 || dev >= kMaxDevices || !g_scratch[dev])
      throw Error(WDMG_ERR_HIP, std::string("no scratch address on this device: hipGetSymbolAddress: ") +
                                    (dev >= 0 && dev < kMaxDevices ? hipGetErrorString(g_scratch_rc[dev]) : "bad device"));
    const size_t field = (size_t)c->g0.vpad * 12 * (prec == WDMG_F64 ? 16 : 8) * (size_t)nrhs;
    if (2 * field > kNoAllocScratchBytes)
      throw Error(WDMG_ERR_ARG, "wdmg_apply_D_noalloc: " + std::to_string(2 * field) +
                                    " bytes of scratch needed, the maximum is 64 MiB");
    // `field` is a multiple of 64 sites x 12 x 8 bytes, so b stays 256-byte aligned
    unsigned char* base = static_cast<unsigned char*>(g_scratch[dev]);
    c->no_alloc = true;
    struct Restore {
      Ctx& c;
      ~Restore() { c.no_alloc = false; }
    } restore{*c};
    if (prec == WDMG_F64) {
      cx<double>* a = reinterpret_cast<cx<double>*>(base);
      cx<double>* b = reinterpret_cast<cx<double>*>(base + field);
      fine_in<double>(*c, in, a, nrhs);
      dslash<double>(*c, b, a, nrhs);
      fine_out<double>(*c, b, out, nrhs);
    } else {
      cx<float>* a = reinterpret_cast<cx<float>*>(base);
      cx<float>* b = reinterpret_cast<cx<float>*>(base + field);
      fine_in<float>(*c, in, a, nrhs);
      dslash<float>(*c, b, a, nrhs);
      fine_out<float>(*c, b, out, nrhs);
    }
    return WDMG_OK;
  });
}

int wdmg_roundtrip(wdmg_ctx* c, void* out, const void* in, int nrhs, int prec) {
  return guarded(c, [&]() {
    need_ptr(out, "out");
    need_ptr(in, "in");
    need_nrhs(nrhs);
    need_prec(prec);
    if (out == in) throw Error(WDMG_ERR_ARG, "out must differ from in");
    const size_t n = (size_t)c->g0.vpad * 12;
    if (prec == WDMG_F64) {
      ensure_io(*c, n * nrhs * sizeof(cx<double>));
      fine_in<double>(*c, in, static_cast<cx<double>*>(c->io_a), nrhs);
      fine_out<double>(*c, static_cast<cx<double>*>(c->io_a), out, nrhs);
    } else if (prec == WDMG_F32) {
      ensure_io(*c, n * nrhs * sizeof(cx<float>));
      fine_in<float>(*c, in, static_cast<cx<float>*>(c->io_a), nrhs);
      fine_out<float>(*c, static_cast<cx<float>*>(c->io_a), out, nrhs);
    } else if (prec == WDMG_F16) {
      roundtrip_half<f16_t>(*c, out, in, nrhs);
    } else {
      roundtrip_half<bf16_t>(*c, out, in, nrhs);
    }
    return WDMG_OK;
  });
}

int wdmg_mg_setup(wdmg_ctx* c, const wdmg_mg_params* p) {
  return guarded(c, [&]() {
    need_ptr(p, "params");
    mg_setup(*c, *p);
    return WDMG_OK;
  });
}

int wdmg_get_prolongator(wdmg_ctx* c, int level, void* V_out) {
  return guarded(c, [&]() {
    need_ptr(V_out, "V_out");
    need_mg(*c, level, false);
    Level& L = c->lev[level];
    if (!L.V64) throw Error(WDMG_ERR_ARG, "prolongator released by wdmg_release_unused");
    if (level == 0)
      fine_to_canonical<double, double>(*c, c->g0, L.V64, static_cast<cx<double>*>(V_out), L.nv);
    else
      copy<double>(*c, static_cast<cx<double>*>(V_out), L.V64, (size_t)L.nv * L.n);
    return WDMG_OK;
  });
}

int wdmg_apply_Dc(wdmg_ctx* c, int level, void* out, const void* in, int nrhs, int prec) {
  return guarded(c, [&]() {
    need_ptr(out, "out");
    need_ptr(in, "in");
    need_nrhs(nrhs);
    need_prec(prec);
    need_mg(*c, level, true);
    if (out == in) throw Error(WDMG_ERR_ARG, "out must differ from in");
    Level& L = c->lev[level];
    if (prec == WDMG_F64)
      coarse_apply<double>(*c, L, dc_of<double>(L), static_cast<cx<double>*>(out),
                           static_cast<const cx<double>*>(in), nrhs);
    else if (prec == WDMG_F32)
      coarse_apply<float>(*c, L, dc_of<float>(L), static_cast<cx<float>*>(out), static_cast<const cx<float>*>(in),
                          nrhs);
    else
      coarse_apply_h(*c, L, prec, static_cast<cx<float>*>(out), static_cast<const cx<float>*>(in), nrhs);
    return WDMG_OK;
  });
}

int wdmg_apply_Nc(wdmg_ctx* c, int level, void* out, const void* in, int nrhs) {
  return guarded(c, [&]() {
    need_ptr(out, "out");
    need_ptr(in, "in");
    need_nrhs(nrhs);
    need_mg(*c, level, true);
    if (out == in) throw Error(WDMG_ERR_ARG, "out must differ from in");
    normal_apply_c(*c, c->lev[level], static_cast<cx<double>*>(out), static_cast<const cx<double>*>(in), nrhs);
    return WDMG_OK;
  });
}

int wdmg_restrict(wdmg_ctx* c, int level, void* c_out, const void* f_in, int nrhs, int prec) {
  return guarded(c, [&]() {
    need_ptr(c_out, "c_out");
    need_ptr(f_in, "f_in");
    need_nrhs(nrhs);
    need_prec(prec);
    need_mg(*c, level, false);
    if (is_half(prec) && level != 0) throw Error(WDMG_ERR_ARG, "16-bit transfers exist for level 0 only");
    if (prec == WDMG_F64)
      restrict_impl<double>(*c, level, c_out, f_in, nrhs);
    else if (prec == WDMG_F32)
      restrict_impl<float>(*c, level, c_out, f_in, nrhs);
    else if (prec == WDMG_F16)
      restrict_half<f16_t>(*c, c_out, f_in, nrhs);
    else
      restrict_half<bf16_t>(*c, c_out, f_in, nrhs);
    return WDMG_OK;
  });
}

int wdmg_prolong(wdmg_ctx* c, int level, void* f_out, const void* c_in, int nrhs, int prec) {
  return guarded(c, [&]() {
    need_ptr(f_out, "f_out");
    need_ptr(c_in, "c_in");
    need_nrhs(nrhs);
    need_prec(prec);
    need_mg(*c, level, false);
    if (is_half(prec) && level != 0) throw Error(WDMG_ERR_ARG, "16-bit transfers exist for level 0 only");
    if (prec == WDMG_F64)
      prolong_impl<double>(*c, level, f_out, c_in, nrhs);
    else if (prec == WDMG_F32)
      prolong_impl<float>(*c, level, f_out, c_in, nrhs);
    else if (prec == WDMG_F16)
      prolong_half<f16_t>(*c, f_out, c_in, nrhs);
    else
      prolong_half<bf16_t>(*c, f_out, c_in, nrhs);
    return WDMG_OK;
  });
}

int wdmg_smooth(wdmg_ctx* c, int level, void* x, const void* b, int nrhs, int iters, int prec) {
  return guarded(c, [&]() {
    need_ptr(x, "x");
    need_ptr(b, "b");
    need_nrhs(nrhs);
    need_prec(prec);
    need_gauge(*c);
    if (iters < 0) throw Error(WDMG_ERR_ARG, "iters must be >= 0");
    if (level != 0) need_mg(*c, level, true);
    if (prec == WDMG_F64) {
      smooth_impl<double>(*c, level, x, b, nrhs, iters);
    } else if (prec == WDMG_F32) {
      smooth_impl<float>(*c, level, x, b, nrhs, iters);
    } else if (level == 0) {
      if (prec == WDMG_F16)
        smooth_half0<f16_t>(*c, x, b, nrhs, iters);
      else
        smooth_half0<bf16_t>(*c, x, b, nrhs, iters);
    } else {
      HalfScope hs(*c, prec);
      smooth_impl<float>(*c, level, x, b, nrhs, iters);
    }
    return WDMG_OK;
  });
}

int wdmg_solve(wdmg_ctx* c, void* x, const void* b, int nrhs, const wdmg_solve_params* p, wdmg_solve_stats* stats) {
  return guarded(c, [&]() {
    need_ptr(x, "x");
    need_ptr(b, "b");
    need_ptr(p, "params");
    need_gauge(*c);
    if (nrhs < 1 || nrhs > kMaxRhs) throw Error(WDMG_ERR_ARG, "nrhs must be in 1..64 for a solve");
    if (!(p->tol > 0.0) || p->restart < 1 || p->restart > kMaxKrylov || p->maxit < 1)
      throw Error(WDMG_ERR_ARG, "bad solve parameters");
    if (p->precond) {
      if (!c->have_mg) throw Error(WDMG_ERR_NOT_SETUP, "no multigrid hierarchy set up");
      need_prec(p->mg_prec);
    }
    if (p->outer < 0 || p->outer > 3) throw Error(WDMG_ERR_ARG, "outer must be 0 (FGCR), 1 (BiCGStab), 2 (CGNR) or 3 (MG-CG)");
    if (p->outer == 2 || p->outer == 3) {
      // CG on the normal equations, plain or preconditioned by the normal-equation V-cycle
      ensure_solve_io(*c, 1);
      const size_t nc = (size_t)c->g0.vol * 12;
      int worst = WDMG_OK;
      for (int k = 0; k < nrhs; ++k) {
        wdmg_solve_stats st{};
        c->n_D = 0;
        for (int l = 0; l < WDMG_MAX_LEVELS; ++l) c->n_Dc[l] = 0;
        const double t0 = now();
        fine_in<double>(*c, static_cast<const cx<double>*>(b) + k * nc, c->sol_b, 1);
        const int rc = normal_solve(*c, c->sol_x, c->sol_b, p->tol, p->maxit, p->outer == 3, st);
        fine_out<double>(*c, c->sol_x, static_cast<cx<double>*>(x) + k * nc, 1);
        WDMG_HIP(hipStreamSynchronize(c->stream));
        st.seconds = now() - t0;
        st.n_D = c->n_D;
        for (int l = 0; l < WDMG_MAX_LEVELS; ++l) st.n_Dc[l] = c->n_Dc[l];
        if (stats) stats[k] = st;
        if (rc != WDMG_OK) worst = rc;
      }
      return worst;
    }
    if (p->outer == 1) {
      // MG-preconditioned BiCGStab, one right-hand side after another
      ensure_solve_io(*c, 1);
      const size_t nc = (size_t)c->g0.vol * 12;  // canonical stride per rhs
      int worst = WDMG_OK;
      for (int k = 0; k < nrhs; ++k) {
        wdmg_solve_stats st{};
        c->n_D = 0;
        for (int l = 0; l < WDMG_MAX_LEVELS; ++l) c->n_Dc[l] = 0;
        const double t0 = now();
        fine_in<double>(*c, static_cast<const cx<double>*>(b) + k * nc, c->sol_b, 1);
        const int rc = bicgstab(*c, c->sol_x, c->sol_b, p->tol, p->maxit, st, p->precond ? p : nullptr);
        fine_out<double>(*c, c->sol_x, static_cast<cx<double>*>(x) + k * nc, 1);
        WDMG_HIP(hipStreamSynchronize(c->stream));
        st.seconds = now() - t0;
        st.n_D = c->n_D;
        for (int l = 0; l < WDMG_MAX_LEVELS; ++l) st.n_Dc[l] = c->n_Dc[l];
        if (stats) stats[k] = st;
        if (rc != WDMG_OK) worst = rc;
      }
      return worst;
    }
    const bool in_place = p->in_place != 0;
    if (in_place && (!p->precond || p->mg_prec == WDMG_F64 || p->restart < 2 || p->use_graph))
      throw Error(WDMG_ERR_ARG, "in-place solves need FGCR with a V-cycle below FP64, restart >= 2 and no graph");
    if (!in_place && x == b) throw Error(WDMG_ERR_ARG, "x and b are the same buffer: set in_place");
    ensure_solve_io(*c, nrhs, !in_place);
    std::vector<wdmg_solve_stats> st(nrhs);
    c->n_D = 0;
    for (int l = 0; l < WDMG_MAX_LEVELS; ++l) c->n_Dc[l] = 0;

    const double t0 = now();
    int rc;
    if (in_place) {
      // x starts from zero; b is read from the caller's buffer whenever the
      // residual is recomputed, and x is written over it at the end
      zero<double>(*c, c->sol_x, (size_t)nrhs * c->g0.vpad * 12);
      rc = fgcr(*c, c->sol_x, nullptr, nrhs, *p, st.data(), b);
    } else {
      fine_in<double>(*c, b, c->sol_b, nrhs);
      fine_in<double>(*c, x, c->sol_x, nrhs);
      rc = fgcr(*c, c->sol_x, c->sol_b, nrhs, *p, st.data());
    }
    fine_out<double>(*c, c->sol_x, x, nrhs);
    WDMG_HIP(hipStreamSynchronize(c->stream));
    const double secs = now() - t0;
    for (int q = 0; q < nrhs; ++q) {
      // operator applications and wall time are shared by the batch: per rhs
      st[q].seconds = secs / nrhs;
      st[q].n_D = c->n_D / nrhs;
      for (int l = 0; l < WDMG_MAX_LEVELS; ++l) st[q].n_Dc[l] = c->n_Dc[l] / nrhs;
      if (stats) stats[q] = st[q];
    }
    return rc;
  });
}

int wdmg_solve_bicgstab(wdmg_ctx* c, void* x, const void* b, int nrhs, double tol, int maxit,
                        wdmg_solve_stats* stats) {
  return guarded(c, [&]() {
    need_ptr(x, "x");
    need_ptr(b, "b");
    need_nrhs(nrhs);
    need_gauge(*c);
    if (!(tol > 0.0) || maxit < 1) throw Error(WDMG_ERR_ARG, "bad solve parameters");
    ensure_solve_io(*c, 1);
    const size_t n = (size_t)c->g0.vol * 12;  // canonical stride per rhs
    int worst = WDMG_OK;
    for (int k = 0; k < nrhs; ++k) {
      wdmg_solve_stats st{};
      c->n_D = 0;
      const double t0 = now();
      fine_in<double>(*c, static_cast<const cx<double>*>(b) + k * n, c->sol_b, 1);
      const int rc = bicgstab(*c, c->sol_x, c->sol_b, tol, maxit, st);
      fine_out<double>(*c, c->sol_x, static_cast<cx<double>*>(x) + k * n, 1);
      WDMG_HIP(hipStreamSynchronize(c->stream));
      st.seconds = now() - t0;
      st.n_D = c->n_D;
      if (stats) stats[k] = st;
      if (rc != WDMG_OK) worst = rc;
    }
    return worst;
  });
}

int wdmg_set_tuning(wdmg_ctx* c, int key, int value) {
  return guarded(c, [&]() {
    if (key < 0 || key >= WDMG_TUNE_COUNT) throw Error(WDMG_ERR_ARG, "unknown tuning key");
    const int hi = key == WDMG_TUNE_DSLASH ? 9 : key == WDMG_TUNE_COARSE_APPLY ? 1 : kMaxRhs;
    const int lo = key == WDMG_TUNE_DSLASH_GROUP ? 1 : 0;
    if (value != WDMG_TUNE_AUTO && (value < lo || value > hi)) throw Error(WDMG_ERR_ARG, "bad tuning value");
    c->tune_force[key] = value;
    return WDMG_OK;
  });
}

int wdmg_set_tuning_for(wdmg_ctx* c, int key, int prec, int nrhs, int value) {
  return guarded(c, [&]() {
    if (key != WDMG_TUNE_DSLASH && key != WDMG_TUNE_DSLASH_GROUP)
      throw Error(WDMG_ERR_ARG, "only the Wilson form and rhs group are kept per precision and batch");
    need_prec(prec);
    need_nrhs(nrhs);
    const int hi = key == WDMG_TUNE_DSLASH ? 9 : kMaxRhs;
    const int lo = key == WDMG_TUNE_DSLASH_GROUP ? 1 : 0;
    if (value != WDMG_TUNE_AUTO && (value < lo || value > hi)) throw Error(WDMG_ERR_ARG, "bad tuning value");
    const int slot = nrhs < kMaxRhs ? nrhs : kMaxRhs;
    if (key == WDMG_TUNE_DSLASH)
      c->tune_dslash[prec][slot] = (signed char)value;
    else
      c->tune_group[prec][slot] = (signed char)value;
    return WDMG_OK;
  });
}

int wdmg_get_tuning(wdmg_ctx* c, int key, int prec, int nrhs, int* value) {
  return guarded(c, [&]() {
    need_ptr(value, "value");
    if (key < 0 || key >= WDMG_TUNE_COUNT) throw Error(WDMG_ERR_ARG, "unknown tuning key");
    need_prec(prec);
    need_nrhs(nrhs);
    const int slot = nrhs < kMaxRhs ? nrhs : kMaxRhs;
    *value = c->tune_force[key] >= 0                 ? c->tune_force[key]
             : key == WDMG_TUNE_DSLASH               ? (int)c->tune_dslash[prec][slot]
             : key == WDMG_TUNE_DSLASH_GROUP         ? (int)c->tune_group[prec][slot]
                                                     : WDMG_TUNE_AUTO;
    return WDMG_OK;
  });
}

int wdmg_profile(wdmg_ctx* c, int enable) {
  return guarded(c, [&]() {
    prof_collect(*c);
    if (enable) {
      for (int k = 0; k < WDMG_K_COUNT; ++k) {
        c->prof_launch[k] = 0;
        c->prof_units[k] = 0;
        c->prof_ms[k] = 0.0;
      }
    }
    c->prof_on = enable != 0;
    return WDMG_OK;
  });
}

int wdmg_profile_read(wdmg_ctx* c, int kernel, long long* launches, long long* units, double* ms) {
  return guarded(c, [&]() {
    if (kernel < 0 || kernel >= WDMG_K_COUNT) throw Error(WDMG_ERR_ARG, "unknown kernel id");
    prof_collect(*c);
    if (launches) *launches = c->prof_launch[kernel];
    if (units) *units = c->prof_units[kernel];
    if (ms) *ms = c->prof_ms[kernel];
    return WDMG_OK;
  });
}

}  // extern "C"
