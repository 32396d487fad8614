// Host-side internals of libwdmg: context, levels, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/wdmg.h"
#include "common.h"

namespace wdmg {

// Error carried from the host drivers to the ABI layer.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define WDMG_HIP(call)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::wdmg::Error(WDMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

Geom make_geom(const int L[4], const int B[4]);

// ---------------------------------------------------------------------------
// Device scalar area.  Solver coefficients live here and are consumed by
// kernels directly; the host reads back only residual norms.
constexpr int kMaxRhs = 64;     // right-hand sides solved together
constexpr int kMaxKrylov = 128;  // GCR restart length limit

enum ScalarSlot {
  S_ERR = 0,        // NaN / rank / SU(3) flags (as doubles)
  S_MR = 8,         // single MR / correction step: alpha (re, im)
  S_TMP = 16,       // misc: norms, dots
  S_BICG = 32,      // BiCGStab: rho, alpha, omega, beta, ... (complex)
  S_RNORM = 64,     // residual norm^2 per level (real)
  S_GCR = 128,      // unused (kept for layout stability)
  S_GCR_STRIDE = 512,
  S_BATCH = S_GCR + 4 * S_GCR_STRIDE,  // batched step sizes: 2 per rhs
  // Batched GCR state, one block per level (0..3) and one for the outer solve
  // (index 4): h [rhs][2*kMaxKrylov], nrm [rhs][kMaxKrylov], a [rhs][2],
  // rnorm^2 [rhs], active [rhs], target rnorm^2 [rhs].
  G_H = 0,
  G_NRM = G_H + kMaxRhs * 2 * kMaxKrylov,
  G_A = G_NRM + kMaxRhs * kMaxKrylov,
  G_RN = G_A + 2 * kMaxRhs,
  G_ACT = G_RN + kMaxRhs,
  G_TOL = G_ACT + kMaxRhs,
  G_STRIDE = G_TOL + kMaxRhs,
  S_G = S_BATCH + 2 * kMaxRhs,
  S_TOTAL = S_G + 5 * G_STRIDE
};
inline int gcr_base(int slot_level) { return S_G + slot_level * G_STRIDE; }

// ---------------------------------------------------------------------------
// 16-bit storage (half_field.h).  A fine field in 16-bit storage is a pair of
// arrays: values [rhs][vpad/64][12][64] of 4-byte complex and scales
// [rhs][vpad] of float.
typedef _Float16 f16_t;
typedef __bf16 bf16_t;
template <typename H>
constexpr int half_kind() {
  return std::is_same<H, f16_t>::value ? WDMG_F16 : WDMG_BF16;
}
struct HF {
  void* v = nullptr;   // values
  float* s = nullptr;  // per-site scales
};
inline HF hf_rhs(HF f, int rhs, int vpad) {
  HF r;
  r.v = static_cast<char*>(f.v) + (size_t)rhs * 12 * vpad * 4;
  r.s = f.s + (size_t)rhs * vpad;
  return r;
}

// ---------------------------------------------------------------------------
// Memory owned by a context.
struct Ctx;
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// One multigrid level.  Level 0 is the Wilson operator on the fine lattice
// (spinor fields stored [rhs][12][V] component-major over tile-major sites);
// level l >= 1 is a coarse stencil with fields [rhs][site][2 Nv].
struct Level {
  int l = 0;
  int dims[4] = {0, 0, 0, 0};
  Geom g;
  int nsite = 0;
  int dof = 0;          // complex dof per site: 12 at level 0, 2*Nv_{l-1} above
  size_t n = 0;         // complex elements per field = nsite * dof
  // transfer to level l+1
  int block[4] = {1, 1, 1, 1};
  int nv = 0;
  cx<double>* V64 = nullptr;   // orthonormal block columns, nv fields of this level
  cx<float>* V32 = nullptr;
  // coarse operator of this level (l >= 1): [site][9][col][row]
  cx<double>* Dc64 = nullptr;
  cx<float>* Dc32 = nullptr;
  // normal-equation coarse operator (D^dagger D)_c of this level (l >= 1) when
  // the hierarchy was set up for the normal equations: [site][33][col][row],
  // and its offset table (33 int4 offsets, then 81 ints: offset index by code)
  cx<double>* Nc64 = nullptr;
  void* noff = nullptr;
  // 16-bit copies, made on first use (kind WDMG_F16 / WDMG_BF16, 0: none):
  // prolongator columns (unscaled) and coarse blocks with one scale per block
  void* V16 = nullptr;
  int v16_kind = 0;
  void* Dc16 = nullptr;
  float* Dc16s = nullptr;
  int dc16_kind = 0;
  // 16-bit work fields of the fine level (V-cycle in 16-bit storage)
  HF wh[6];
  int caph = 0;
  // work vectors of the V-cycle at this level, each holding `cap` fields
  cx<double>* w64[8] = {};
  cx<float>* w32[8] = {};
  int cap64 = 0, cap32 = 0;
  int capB = 0;         // capacity (rhs) of the coarsest GCR basis
  // GCR basis of the coarsest solve (coarsest level only)
  cx<double>* basisZ = nullptr;
  cx<double>* basisW = nullptr;
  cx<double>* xT = nullptr;  // solution of a batched coarsest solve in the rhs-fast layout
  double* cpart = nullptr;   // partial sums of the coarsest GCR
  double* cpart3 = nullptr;
  double* chist = nullptr;   // per-rhs coefficient history of a batched coarsest GCR cycle
};

constexpr int kWork = 8;

constexpr int kRing = 8;
constexpr int kHscFlags = 128;   // offset of the active-flag staging area in Ctx::hsc
constexpr int kHscSize = 256;

struct Ctx {
  int dims[4];
  Geom g0;
  hipStream_t stream = nullptr;
  wdmg_alloc alloc{};
  bool own_alloc = true;
  std::string err;
  std::vector<Buf> bufs;

  double mass = 0.0;
  int t_bc = -1;
  bool have_gauge = false;
  cx<double>* U64 = nullptr;   // [4][9][V], t boundary sign folded in
  cx<float>* U32 = nullptr;
  void* U16 = nullptr;          // 16-bit links, made on first use
  int u16_kind = 0;             // WDMG_F16 / WDMG_BF16 (0: none)
  int vc_half = 0;              // 16-bit kind of the running V-cycle (0: none)
  // kernel variants: forced choice per tuning key (-1: autotune) and the
  // autotuner's choices per (precision, batch size)
  int tune_force[WDMG_TUNE_COUNT] = {-1};
  signed char tune_dslash[4][kMaxRhs + 1];
  signed char tune_group[4][kMaxRhs + 1];  // rhs group size of batched Wilson launches
  // HIP-graph capture of a V-cycle: while capturing, the coarsest GCR runs
  // exactly coarse_fixed_iters iterations with no host interaction
  bool capturing = false;
  // inside wdmg_apply_D_noalloc: no autotuning (its timing buffers) and no
  // event records; kernels take already-tuned or default forms
  bool no_alloc = false;
  int device = 0;               // HIP device current at wdmg_create
  int coarse_fixed_iters = 0;
  int last_coarse_iters = 0;    // most iterations of one coarsest solve since reset
  hipStream_t cap_stream = nullptr;
  cx<double>* outer_zf = nullptr;  // fixed output of a captured V-cycle
  int outer_zf_cap = 0;


  double* dsc = nullptr;        // device scalars (S_TOTAL doubles)
  double* partials = nullptr;   // reduction partials
  double* dots = nullptr;       // MR partial sums written by the fused Wilson operator
  size_t dots_cap = 0;          // its capacity in doubles

  double* hsc = nullptr;        // pinned host mirror of a few scalars
  double* hring = nullptr;      // pinned ring [kRing][kMaxRhs] for lagged residual checks (host view)
  double* dring = nullptr;      // the same ring as seen from the device
  hipEvent_t ring_ev[kRing] = {};

  // multigrid
  bool have_mg = false;
  bool released = false;  // wdmg_release_unused freed higher-precision copies of P / D_c
  wdmg_mg_params mg{};
  int nlevels = 0;
  Level lev[WDMG_MAX_LEVELS];
  double setup_mass = 0.0;

  // scratch fine / coarse fields for canonical <-> internal conversion
  void* io_a = nullptr;
  void* io_b = nullptr;
  size_t io_bytes = 0;
  HF ioh[3];                    // 16-bit scratch fine fields
  int ioh_cap = 0;

  // outer FGCR and BiCGStab work space (fine level, FP64)
  int outer_k = 0;
  cx<double>* outer_Z = nullptr;
  cx<double>* outer_W = nullptr;
  cx<double>* outer_r = nullptr;
  cx<float>* outer_r32 = nullptr;
  cx<float>* outer_z32 = nullptr;
  cx<double>* outer_hist = nullptr;  // [rhs][k][k] orthogonalisation coefficients of a cycle
  cx<double>* outer_av = nullptr;    // [rhs][k] step sizes of a cycle
  cx<double>* outer_y = nullptr;     // [rhs][k] combination coefficients
  int outer_histk = 0, outer_histcap = 0;
  cx<float>* outer_Z32 = nullptr;  // FP32 outer basis (reduced-precision V-cycle)
  cx<float>* outer_W32 = nullptr;
  int outer_k32 = 0, outer_capB32 = 0;
  cx<double>* bicg[8] = {};
  cx<double>* sol_x = nullptr;   // internal x, b of a solve
  cx<double>* sol_b = nullptr;
  int sol_cap = 0;    // rhs capacity of sol_x
  int sol_bcap = 0;   // rhs capacity of sol_b (in-place solves keep none)
  int outer_cap = 0;             // rhs capacity of outer_r
  int outer_capB = 0;            // rhs capacity of the FP64 outer basis
  int outer_cap32 = 0;

  // kernel timing (instrumentation)
  bool prof_on = false;
  struct ProfRec {
    int id;
    long long units;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> prof_pool;
  long long prof_launch[WDMG_K_COUNT] = {};
  long long prof_units[WDMG_K_COUNT] = {};
  double prof_ms[WDMG_K_COUNT] = {};

  // counters of the current solve
  long long n_D = 0;
  long long n_Dc[WDMG_MAX_LEVELS] = {0, 0, 0, 0};
};

// Records HIP events around one kernel launch when timing is enabled.
struct ProfScope {
  Ctx& c;
  int idx = -1;
  ProfScope(Ctx& ctx, int id, long long units);
  ~ProfScope();
};
void prof_collect(Ctx& c);

void* dev_alloc(Ctx& c, size_t bytes);
void dev_free(Ctx& c, void* p);
void ensure_io(Ctx& c, size_t bytes);

constexpr int kReduceThreads = 256;
constexpr int kMaxReduceBlocks = 1024;
constexpr int kPartialsPerBlock = 64;

// ---------------------------------------------------------------------------
// Layout conversion (layout.hip).
void gauge_import(Ctx& c, const cx<double>* canon, int t_bc);
template <typename Rio, typename R>
void fine_to_internal(Ctx& c, const Geom& g, const cx<Rio>* canon, cx<R>* out, int nrhs);
template <typename R, typename Rio>
void fine_to_canonical(Ctx& c, const Geom& g, const cx<R>* in, cx<Rio>* canon, int nrhs);
template <typename Rout, typename Rin>
void convert(Ctx& c, cx<Rout>* out, const cx<Rin>* in, size_t n);

// 16-bit storage (half.hip).  Links and prolongator columns are rounded
// from their FP32 copies.
const void* u16(Ctx& c, int kind);
const void* v16(Ctx& c, Level& L, int kind);
HF hf_alloc(Ctx& c, int nrhs);
void hf_free(Ctx& c, HF& f);
template <typename H>
void hf_zero(Ctx& c, HF f, int nrhs);
void hf_copy(Ctx& c, HF dst, HF src, int nrhs);
void hf_neg(Ctx& c, HF f, int nrhs);  // f = -f, exact
// internal R field [rhs][12 vpad] <-> 16-bit field
template <typename R, typename H>
void to_half(Ctx& c, const cx<R>* in, HF out, int nrhs);
template <typename H, typename R>
void from_half(Ctx& c, HF in, cx<R>* out, int nrhs);
// canonical complex64 <-> 16-bit field
template <typename H>
void canon_to_half(Ctx& c, const cx<float>* canon, HF out, int nrhs);
template <typename H>
void half_to_canon(Ctx& c, HF in, cx<float>* canon, int nrhs);
// Batched MR pieces on 16-bit fields: dsc[slot + 2q] = scale <a_q,b_q>/<a_q,a_q>;
// x_q += s_q u_q, r_q -= s_q v_q (u may be r).
template <typename H>
void step_alpha_half(Ctx& c, HF a, HF b, int nrhs, double scale, int slot);
template <typename H>
// x += s u ; r -= s v (mode 0); x = s u ; r = u - s v (mode 1, x not read);
// x += s u only (mode 2)
void update2_half(Ctx& c, HF x, HF u, HF r, HF v, int nrhs, int slot, int mode = 0);

// Wilson operator (dslash.hip): out = diag * in - 1/2 sum_mu hops.
template <typename R>
void dslash(Ctx& c, cx<R>* out, const cx<R>* in, int nrhs);
// The same on 16-bit fields and links, FP32 arithmetic.
template <typename H>
void dslash_h(Ctx& c, HF out, HF in, int nrhs);
// Fused MR step (Sec. 3): out = D in, and for every rhs q
// dsc[slot + 2q] = scale <out_q, in_q> / <out_q, out_q> (0 if the norm is 0),
// from partial sums the operator launch writes per wave.
template <typename R>
void dslash_mr(Ctx& c, cx<R>* out, const cx<R>* in, int nrhs, double scale, int slot);
template <typename H>
void dslash_h_mr(Ctx& c, HF out, HF in, int nrhs, double scale, int slot);
// The partial-sum buffer of the fused operator, grown to nrhs right-hand
// sides (never inside a graph capture).
double* dots_buffer(Ctx& c, int nrhs);
// dsc[slot + 2q] = scale (p0 + i p1) / p2 from nparts triples per rhs q
// (parts[(q * nparts + j) * 3 + k]), summed in a fixed order.
void step_alpha_fin(Ctx& c, const double* parts, int nparts, int nrhs, double scale, int slot);

// BLAS-1 and reductions (blas.hip).  Vectors are flat arrays of n complex.
template <typename R> void zero(Ctx& c, cx<R>* x, size_t n);
template <typename R> void copy(Ctx& c, cx<R>* y, const cx<R>* x, size_t n);
template <typename R> void neg(Ctx& c, cx<R>* x, size_t n);           // x = -x
template <typename R> void xmy(Ctx& c, const cx<R>* b, cx<R>* y, size_t n);  // y = b - y
template <typename R> void add(Ctx& c, cx<R>* y, const cx<R>* x, size_t n);  // y += x
// dsc[slot] = scale * <a, b> / <a, a>  (0 if <a,a> == 0); complex result.
template <typename R> void step_alpha(Ctx& c, const cx<R>* a, const cx<R>* b, size_t n, double scale, int slot);
// x += s u ; r -= s v with s = dsc[slot] (complex).
template <typename R> void update2(Ctx& c, cx<R>* x, const cx<R>* u, cx<R>* r, const cx<R>* v, size_t n, int slot);
// Batched over nb vectors (stride apart): dsc[slot + 2 q] = scale <a_q,b_q>/<a_q,a_q>;
// x_q += s_q u_q ; r_q -= s_q v_q.
template <typename R>
void step_alpha_batch(Ctx& c, const cx<R>* a, const cx<R>* b, size_t n, size_t stride, int nb, double scale,
                      int slot);
template <typename R>
void update2_batch(Ctx& c, cx<R>* x, const cx<R>* u, cx<R>* r, const cx<R>* v, size_t n, size_t stride, int nb,
                   int slot, int mode = 0);
// Batched GCR over nb right-hand sides.  Fields of one rhs are n long and
// consecutive (batch stride n); basis vector i of all rhs is W + i*nb*n.
// State in the block gcr_base(g): h, nrm, a, rnorm^2, active (see ScalarSlot).
// B is the storage type of the basis W, Z and of w, z (double or float);
// r and x are double and every sum is formed in double.
// Classical Gram-Schmidt of w against the j earlier directions W: h_i =
// <W_i, w> / nrm_i, w -= sum h_i W_i, nrm_j = |w|^2, step a = <w, r> / nrm_j.
template <typename B>
void gcr_orth_b(Ctx& c, const cx<B>* W, cx<B>* w, const cx<double>* r, size_t n, int nb, int j, int g);
// r -= a w per rhs (a = 0 for inactive rhs); rnorm^2 per rhs, also to host
// (device-visible pinned address, nb doubles) when given.
template <typename B>
void gcr_step_b(Ctx& c, const cx<B>* w, cx<double>* r, size_t n, int nb, int g, double* host = nullptr);
// Search directions are kept as the preconditioner returned them (zt_j) and
// combined once per cycle: gcr_record stores iteration j's h_i and a of every
// rhs (hist [rhs][k][k], av [rhs][k]); gcr_combine solves y_j = a_j -
// sum_{m>j} h_jm y_m and adds sum_{j < jn} y_j zt_j to x.
void gcr_record(Ctx& c, cx<double>* hist, cx<double>* av, int nb, int j, int k, int g);
template <typename B>
void gcr_combine(Ctx& c, cx<double>* x, const cx<B>* Z, const cx<double>* hist, const cx<double>* av, cx<double>* y,
                 size_t n, int nb, int jn, int k);
// rnorm^2 of nb fields into the block g (and host when given).
void norm2_b(Ctx& c, const cx<double>* a, size_t n, int nb, int g, double* host = nullptr);
// y = b - y per rhs, with rnorm^2 into block g.
void xmy_norm_b(Ctx& c, const cx<double>* b, cx<double>* y, size_t n, int nb, int g);
// sets active flags of block g from a host array (nb doubles, 1 or 0)
void set_active(Ctx& c, int g, const double* host_flags, int nb);
// dsc[slot] = ||a||^2
template <typename R> void norm2(Ctx& c, const cx<R>* a, size_t n, int slot);
// dsc[slot] = <a, b>
template <typename R> void dot(Ctx& c, const cx<R>* a, const cx<R>* b, size_t n, int slot);
// y = b - y (residual from an operator application); dsc[slot] = ||y||^2.
void xmy_norm(Ctx& c, const cx<double>* b, cx<double>* y, size_t n, int slot);
// BiCGStab kernels (FP64).
void bicg_p(Ctx& c, cx<double>* p, const cx<double>* r, const cx<double>* v, size_t n, bool first);
void bicg_alpha(Ctx& c, const cx<double>* rhat, const cx<double>* v, size_t n);
void bicg_s(Ctx& c, cx<double>* s, const cx<double>* r, const cx<double>* v, size_t n);
void bicg_omega(Ctx& c, const cx<double>* t, const cx<double>* s, size_t n);
// x += alpha p + omega sx; r = s - omega t (sx = s unpreconditioned)
void bicg_xr(Ctx& c, cx<double>* x, cx<double>* r, const cx<double>* p, const cx<double>* s, const cx<double>* sx,
             const cx<double>* t, const cx<double>* rhat, size_t n);
void set_scalar(Ctx& c, int slot, double re, double im);
// dsc[slot + 2 i] = re, dsc[slot + 2 i + 1] = im for i < count (count <= kMaxRhs)
void fill_pairs(Ctx& c, int slot, int count, double re, double im);

// Transfer (transfer.hip).
template <typename R>
void restrict0(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs);
template <typename R>
void prolong0(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs);
template <typename R>
void restrictC(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs);
template <typename R>
void prolongC(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs);
// Block orthonormalisation in FP64, in place; sets dsc[S_ERR+1] != 0 on rank loss.
void block_qr0(Ctx& c, const Level& f, cx<double>* V);
// level 0 with 16-bit fields and prolongator: coarse side in FP32
template <typename H>
void restrict0_h(Ctx& c, const Level& f, const void* V16, HF in, cx<float>* out, int nrhs);
template <typename H>
void prolong0_h(Ctx& c, const Level& f, const void* V16, const cx<float>* in, HF out, int nrhs);
void block_qrC(Ctx& c, const Level& f, cx<double>* V);

// Coarse operator (coarse.hip).
void coarse_build0(Ctx& c, const Level& f, Level& cl);
void coarse_buildC(Ctx& c, const Level& f, Level& cl);
// out = D_c in; when copy is given, copy = in as well (one pass).
template <typename R>
void coarse_apply(Ctx& c, const Level& cl, const cx<R>* Dc, cx<R>* out, const cx<R>* in, int nrhs,
                  cx<R>* copy = nullptr);
void coarse_shift(Ctx& c, Level& cl, double dm);
// The 16-bit blocks of kind (WDMG_F16 / WDMG_BF16) of coarse level cl, made
// from its FP64 blocks unless already current.
void ensure_dc16(Ctx& c, Level& cl, int kind);
// Frees what a V-cycle in 16-bit storage of kind does not read (after making
// the 16-bit copies it does): the FP64 and FP32 first prolongator and the FP64
// and FP32 blocks of every coarse level but the coarsest.
void release_unused(Ctx& c, int kind);
// The coarsest-level GCR(k) in FP64 for nrhs right-hand sides: x = 0, r = b,
// iterate until every ||r_q|| <= tol ||b_q|| (lagged test) or maxit.  One rhs:
// three launches per iteration on the canonical layout; a batch: four, on
// vectors kept rhs-fast for the whole solve.  Work space: L.basisW/Z (k slots),
// L.w64[1] (r), L.xT (batched x), L.cpart / L.cpart3 (partial sums, sized by
// the two functions below).
void coarsest_gcr(Ctx& c, Level& L, cx<double>* x, const cx<double>* b, int nrhs, double tol, int k, int maxit);
size_t coarsest_gcr_partials(int nrhs, int k);
size_t coarsest_gcr_partials3(int nrhs);
size_t coarsest_gcr_history(int nrhs, int k);
// out = D_c in with the blocks stored in 16-bit (one scale per block), FP32
// vectors; the 16-bit blocks are made from the FP64 ones on first use.
void coarse_apply_h(Ctx& c, Level& cl, int kind, cx<float>* out, const cx<float>* in, int nrhs,
                    cx<float>* copy = nullptr);

}  // namespace wdmg
