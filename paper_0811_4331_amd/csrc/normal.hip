// Multigrid on the normal equations (Sec. 3, first approach; Sec. 4 MG-CG):
// the operator A = D^dagger D = gamma5 D gamma5 D (Hermitian positive
// definite), its Galerkin coarse operator A_c = P^dagger A P, CG on the
// normal equations (CGNR) and flexible CG preconditioned by the two-level
// V-cycle on A (MG-CG).
//
// A couples fine sites up to two steps apart (0, +-mu, +-2mu, +-mu+-nu), so
// on aggregates of extent >= 2 A_c couples coarse sites whose offsets have
// every component in {-1, 0, 1} and at most two of them non-zero: 33 dense
// (2Nv x 2Nv) blocks per coarse site, stored [site][33][col][row].  The
// blocks are read off P^dagger A P applied to coloured probe vectors: coarse
// sites are coloured by xhat_mu mod K_mu (K_mu >= 3 dividing the extent), a
// probe is one coarse dof on every site of one colour, and every coarse site
// reaches at most one probed site, whose offset names the block; the 2Nv
// dofs of one colour are probed as one batch.  Coarse extents below 3 are
// refused (the +mu and -mu neighbours would coincide).
//
// The solvers here run one right-hand side at a time in FP64 and read their
// scalars back to the host every iteration: this path is the normal-equation
// alternative and the CG comparator, not the batched hot path.
#include <cmath>
#include <vector>

#include "fine_field.h"
#include "internal.h"
#include "solver.h"

namespace wdmg {

namespace {

constexpr int kNOff = 33;

// offsets in the order (number of non-zero components, then lexicographic in
// (dx, dy, dz, dt) with -1 < 0 < 1)
struct OffsetTable {
  int d[kNOff][4];
};

OffsetTable make_offsets() {
  OffsetTable t{};
  int k = 0;
  for (int nz = 0; nz <= 2; ++nz)
    for (int a = 0; a < 81; ++a) {
      int d[4], v = a, cnt = 0;
      for (int mu = 3; mu >= 0; --mu) {  // lexicographic in (dx, dy, dz, dt): dx most significant
        d[mu] = v % 3 - 1;
        v /= 3;
      }
      for (int mu = 0; mu < 4; ++mu) cnt += d[mu] != 0;
      if (cnt != nz) continue;
      for (int mu = 0; mu < 4; ++mu) t.d[k][mu] = d[mu];
      ++k;
    }
  return t;
}

__device__ __forceinline__ int wrap(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

__device__ __forceinline__ int coarse_site(const Geom& g, const int (&c)[4]) {
  return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

__device__ __forceinline__ void coarse_coords(const Geom& g, int s, int (&c)[4]) {
  c[0] = s % g.L[0];
  s /= g.L[0];
  c[1] = s % g.L[1];
  s /= g.L[1];
  c[2] = s % g.L[2];
  c[3] = s / g.L[2];
}

// gamma5 on fine fields in the internal layout: components 6..11 (spins 2, 3)
// change sign.
__global__ void k_gamma5(cx<double>* f, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)((i >> 6) % 12);
    if (k >= 6) f[i] = mk(-f[i].re, -f[i].im);
  }
}

// Probe batch of one colour: probe a (a = 0..n2-1) is dof a on every coarse
// site of colour kappa.  Layout [a][site][n2].
__global__ void k_probe_fill(Geom g, int n2, int4 K, int4 kappa, cx<double>* out) {
  const size_t total = (size_t)n2 * g.vol * n2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int dof = (int)(i % n2);
    const int s = (int)((i / n2) % g.vol);
    const int a = (int)(i / ((size_t)n2 * g.vol));
    int c[4];
    coarse_coords(g, s, c);
    const bool on = c[0] % K.x == kappa.x && c[1] % K.y == kappa.y && c[2] % K.z == kappa.z && c[3] % K.w == kappa.w;
    out[i] = mk(on && dof == a ? 1.0 : 0.0, 0.0);
  }
}

// Column a of the block of every coarse site reached by the probes of colour
// kappa: y[a][site][row] -> Nc[site][o][a][row], o the offset to the probed
// site (sites that reach none, or only through an offset outside the stencil,
// are skipped).  `code` maps an offset (d + 1 in base 3, x most significant)
// to its index or -1.
__global__ void k_probe_scatter(Geom g, int n2, int4 K, int4 kappa, const int* __restrict__ code,
                                const cx<double>* __restrict__ y, cx<double>* __restrict__ nc) {
  const size_t total = (size_t)n2 * g.vol * n2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(i % n2);
    const int s = (int)((i / n2) % g.vol);
    const int a = (int)(i / ((size_t)n2 * g.vol));
    int c[4];
    coarse_coords(g, s, c);
    const int Ks[4] = {K.x, K.y, K.z, K.w}, ks[4] = {kappa.x, kappa.y, kappa.z, kappa.w};
    int key = 0;
    bool reach = true;
    for (int mu = 0; mu < 4; ++mu) {
      int dmu = 9;
      for (int v = -1; v <= 1; ++v)
        if (wrap(c[mu] + v, g.L[mu]) % Ks[mu] == ks[mu]) dmu = v;
      reach = reach && dmu != 9;
      key = key * 3 + (dmu + 1);
    }
    if (!reach) continue;
    const int o = code[key];
    if (o < 0) continue;
    nc[(((size_t)s * kNOff + o) * n2 + a) * n2 + row] = y[i];
  }
}

// y(xhat) = sum_o B_o(xhat) c(xhat + d_o) for nrhs coarse fields [rhs][site][n2]:
// one thread per (rhs, site, row).
__global__ void k_apply33(Geom g, int n2, int nrhs, const int4* __restrict__ offs, const cx<double>* __restrict__ nc,
                          const cx<double>* __restrict__ in, cx<double>* __restrict__ out) {
  const size_t total = (size_t)nrhs * g.vol * n2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(i % n2);
    const int s = (int)((i / n2) % g.vol);
    const int q = (int)(i / ((size_t)n2 * g.vol));
    int c[4];
    coarse_coords(g, s, c);
    const cx<double>* src = in + (size_t)q * g.vol * n2;
    cx<double> acc = mk(0.0, 0.0);
    for (int o = 0; o < kNOff; ++o) {
      const int4 d = offs[o];
      const int nb[4] = {wrap(c[0] + d.x, g.L[0]), wrap(c[1] + d.y, g.L[1]), wrap(c[2] + d.z, g.L[2]),
                         wrap(c[3] + d.w, g.L[3])};
      const cx<double>* v = src + (size_t)coarse_site(g, nb) * n2;
      const cx<double>* blk = nc + ((size_t)s * kNOff + o) * n2 * n2 + row;
      for (int col = 0; col < n2; ++col) cmadd(acc, blk[(size_t)col * n2], v[col]);
    }
    out[i] = acc;
  }
}

__global__ void k_xpby(cx<double>* p, const cx<double>* z, cx<double> beta, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

__global__ void k_axpy2(cx<double>* x, const cx<double>* p, cx<double>* r, const cx<double>* q, cx<double> a,
                        size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    x[i] = x[i] + a * p[i];
    r[i] = r[i] - a * q[i];
  }
}

unsigned ew_grid(size_t n) {
  size_t b = (n + 255) / 256;
  return (unsigned)(b < 4096 ? b : 4096);
}

cx<double> read_pair(Ctx& c, int slot) {
  WDMG_HIP(hipMemcpyAsync(c.hsc, c.dsc + slot, 2 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  WDMG_HIP(hipStreamSynchronize(c.stream));
  return mk(c.hsc[0], c.hsc[1]);
}

cx<double> dotc(Ctx& c, const cx<double>* a, const cx<double>* b, size_t n) {
  dot<double>(c, a, b, n, S_TMP);
  return read_pair(c, S_TMP);
}

double nrm2(Ctx& c, const cx<double>* a, size_t n) {
  norm2<double>(c, a, n, S_TMP + 2);
  return read_scalar(c, S_TMP + 2);
}

cx<double> cdivh(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

void gamma5(Ctx& c, cx<double>* f, size_t n) {
  hipLaunchKernelGGL(k_gamma5, dim3(ew_grid(n)), dim3(256), 0, c.stream, f, n);
  WDMG_HIP(hipGetLastError());
}

}  // namespace

// Device memory owned by the normal-equation path of a context.
struct NormalWork {
  std::vector<void*> bufs;
  Ctx* c = nullptr;
  cx<double>* get(size_t n) {
    void* p = dev_alloc(*c, n * sizeof(cx<double>));
    bufs.push_back(p);
    return static_cast<cx<double>*>(p);
  }
  ~NormalWork() {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (void* p : bufs) dev_free(*c, p);
  }
};

// out = A in = gamma5 D gamma5 D in on nrhs internal fine fields; tmp holds nrhs fields.
void normal_apply0(Ctx& c, cx<double>* out, const cx<double>* in, cx<double>* tmp, int nrhs) {
  const size_t n = c.lev[0].n * nrhs;
  dslash<double>(c, tmp, in, nrhs);
  gamma5(c, tmp, n);
  dslash<double>(c, out, tmp, nrhs);
  gamma5(c, out, n);
}

// out = D^dagger in (one or more fields).
void apply_Ddag0(Ctx& c, cx<double>* out, const cx<double>* in, cx<double>* tmp, int nrhs) {
  const size_t n = c.lev[0].n * nrhs;
  copy<double>(c, tmp, in, n);
  gamma5(c, tmp, n);
  dslash<double>(c, out, tmp, nrhs);
  gamma5(c, out, n);
}

// Coarse extents >= 3 and fine aggregates of extent >= 2 in every direction.
void normal_check_geometry(const Level& f, const Level& cl) {
  for (int mu = 0; mu < 4; ++mu) {
    if (f.block[mu] < 2)
      throw Error(WDMG_ERR_DIMS, "a normal-equation hierarchy needs aggregates of extent >= 2");
    if (cl.dims[mu] < 3) throw Error(WDMG_ERR_DIMS, "a normal-equation hierarchy needs coarse extents >= 3");
  }
}

void normal_build(Ctx& c, Level& f, Level& cl) {
  normal_check_geometry(f, cl);
  const int n2 = cl.dof;
  const size_t ncn = (size_t)cl.nsite * kNOff * n2 * n2;
  if (!cl.Nc64) cl.Nc64 = static_cast<cx<double>*>(dev_alloc(c, ncn * sizeof(cx<double>)));
  zero<double>(c, cl.Nc64, ncn);
  // offset table and its base-3 code map, on the device
  const OffsetTable t = make_offsets();
  int codes[81];
  for (int i = 0; i < 81; ++i) codes[i] = -1;
  int4 offs[kNOff];
  for (int o = 0; o < kNOff; ++o) {
    int key = 0;
    for (int mu = 0; mu < 4; ++mu) key = key * 3 + (t.d[o][mu] + 1);
    codes[key] = o;
    offs[o] = make_int4(t.d[o][0], t.d[o][1], t.d[o][2], t.d[o][3]);
  }
  if (!cl.noff) {
    cl.noff = dev_alloc(c, sizeof(offs) + sizeof(codes));
    WDMG_HIP(hipMemcpyAsync(cl.noff, offs, sizeof(offs), hipMemcpyHostToDevice, c.stream));
    WDMG_HIP(hipMemcpyAsync(static_cast<char*>(cl.noff) + sizeof(offs), codes, sizeof(codes), hipMemcpyHostToDevice,
                            c.stream));
    WDMG_HIP(hipStreamSynchronize(c.stream));
  }
  const int* dcode = reinterpret_cast<const int*>(static_cast<char*>(cl.noff) + sizeof(offs));
  int K[4];
  for (int mu = 0; mu < 4; ++mu) {
    K[mu] = cl.dims[mu];
    for (int k = 3; k <= cl.dims[mu]; ++k)
      if (cl.dims[mu] % k == 0) {
        K[mu] = k;
        break;
      }
  }
  NormalWork w;
  w.c = &c;
  const size_t nf = f.n * n2, ncv = (size_t)cl.n * n2;
  cx<double>* probe = w.get(ncv);
  cx<double>* y = w.get(ncv);
  cx<double>* pf = w.get(nf);
  cx<double>* af = w.get(nf);
  cx<double>* tf = w.get(nf);
  const int4 Kv = make_int4(K[0], K[1], K[2], K[3]);
  for (int k0 = 0; k0 < K[0]; ++k0)
    for (int k1 = 0; k1 < K[1]; ++k1)
      for (int k2 = 0; k2 < K[2]; ++k2)
        for (int k3 = 0; k3 < K[3]; ++k3) {
          const int4 kap = make_int4(k0, k1, k2, k3);
          hipLaunchKernelGGL(k_probe_fill, dim3(ew_grid(ncv)), dim3(256), 0, c.stream, cl.g, n2, Kv, kap, probe);
          WDMG_HIP(hipGetLastError());
          prolong_from<double>(c, 0, probe, pf, n2);
          normal_apply0(c, af, pf, tf, n2);
          restrict_to<double>(c, 0, af, y, n2);
          hipLaunchKernelGGL(k_probe_scatter, dim3(ew_grid(ncv)), dim3(256), 0, c.stream, cl.g, n2, Kv, kap, dcode,
                             y, cl.Nc64);
          WDMG_HIP(hipGetLastError());
        }
  WDMG_HIP(hipStreamSynchronize(c.stream));
}

void normal_apply_c(Ctx& c, const Level& cl, cx<double>* out, const cx<double>* in, int nrhs) {
  if (!cl.Nc64) throw Error(WDMG_ERR_NOT_SETUP, "no normal-equation coarse operator (set normal in the setup)");
  const size_t n = (size_t)cl.n * nrhs;
  hipLaunchKernelGGL(k_apply33, dim3(ew_grid(n)), dim3(256), 0, c.stream, cl.g, cl.dof, nrhs,
                     static_cast<const int4*>(cl.noff), cl.Nc64, in, out);
  WDMG_HIP(hipGetLastError());
  c.n_Dc[cl.l] += nrhs;
}

// MR relaxation of the candidates on A v = 0 (FP64, one vector at a time),
// each normalised afterwards (the relaxation of the direct setup, on A).
void normal_relax(Ctx& c, Level& f, int nv, int iters, double omega) {
  NormalWork w;
  w.c = &c;
  const size_t n = f.n;
  cx<double>* r = w.get(n);
  cx<double>* p = w.get(n);
  cx<double>* t = w.get(n);
  for (int k = 0; k < nv; ++k) {
    cx<double>* x = f.V64 + (size_t)k * n;
    normal_apply0(c, r, x, t, 1);
    neg<double>(c, r, n);
    for (int it = 0; it < iters; ++it) {
      normal_apply0(c, p, r, t, 1);
      step_alpha<double>(c, p, r, n, omega, S_TMP + 8);
      update2<double>(c, x, r, r, p, n, S_TMP + 8);
    }
    const double nn = nrm2(c, x, n);
    if (!(nn > 0.0) || !std::isfinite(nn)) throw Error(WDMG_ERR_NAN, "a relaxed candidate vanished or is not finite");
    set_scalar(c, S_TMP + 10, 1.0 / std::sqrt(nn) - 1.0, 0.0);
    update2<double>(c, x, x, p, p, n, S_TMP + 10);  // x *= 1/|x| (p is scratch)
  }
}

namespace {

// Flexible CG on an HPD operator: the new direction is the preconditioned
// residual A-orthogonalised against the previous direction (Notay 2000).
// Stops when `done(x, rn2)` says so (rn2 = |r|^2), or after maxit.
// The four work vectors come from w, allocated on its first use and reused
// by later calls with the same w (every call on one w has the same n).
template <class Apply, class Precond, class Done>
int fcg(Ctx& c, size_t n, cx<double>* x, const cx<double>* rhs, Apply apply, Precond precond, Done done, int maxit,
        NormalWork& w) {
  while (w.bufs.size() < 4) w.get(n);
  cx<double>* r = static_cast<cx<double>*>(w.bufs[0]);
  cx<double>* z = static_cast<cx<double>*>(w.bufs[1]);
  cx<double>* p = static_cast<cx<double>*>(w.bufs[2]);
  cx<double>* q = static_cast<cx<double>*>(w.bufs[3]);
  copy<double>(c, r, rhs, n);
  zero<double>(c, x, n);
  int it = 0;
  cx<double> pq_prev = mk(0.0, 0.0);
  while (it < maxit) {
    precond(z, r);
    if (it == 0) {
      copy<double>(c, p, z, n);
    } else {
      const cx<double> qz = dotc(c, q, z, n);
      const cx<double> beta = cdivh(mk(-qz.re, -qz.im), pq_prev);
      hipLaunchKernelGGL(k_xpby, dim3(ew_grid(n)), dim3(256), 0, c.stream, p, z, beta, n);
      WDMG_HIP(hipGetLastError());
    }
    apply(q, p);
    const cx<double> pq = dotc(c, p, q, n);
    if (!(pq.re > 0.0) || !std::isfinite(pq.re)) break;  // exact solution or breakdown
    const cx<double> pr = dotc(c, p, r, n);
    const cx<double> a = cdivh(pr, pq);
    hipLaunchKernelGGL(k_axpy2, dim3(ew_grid(n)), dim3(256), 0, c.stream, x, p, r, q, a, n);
    WDMG_HIP(hipGetLastError());
    pq_prev = pq;
    ++it;
    if (done(x, nrm2(c, r, n))) break;
  }
  return it;
}

}  // namespace

// Work vectors of the two-level V-cycle on A, allocated once per solve.
struct NormalVc {
  cx<double>*res, *p, *t, *y, *dy, *rc, *ec;
  NormalWork cg;  // vectors of the coarse CG
  NormalVc(Ctx& c, NormalWork& w) {
    const size_t n = c.lev[0].n, nc = c.lev[1].n;
    res = w.get(n);
    p = w.get(n);
    t = w.get(n);
    y = w.get(n);
    dy = w.get(n);
    rc = w.get(nc);
    ec = w.get(nc);
    cg.c = &c;
  }
};

// Two-level V-cycle on A (Sec. 2 cycle, Sec. 3 smoother), x = M b from x = 0:
// MR(nu_pre) on A, P^dagger, coarse solve by CG on A_c to coarse_tol, P, the
// step size of Sec. 3 (or 1), MR(nu_post).
void normal_vcycle(Ctx& c, cx<double>* x, const cx<double>* b, NormalVc& v) {
  Level& L = c.lev[0];
  Level& C = c.lev[1];
  const size_t n = L.n, nc = C.n;
  zero<double>(c, x, n);
  copy<double>(c, v.res, b, n);
  auto smooth = [&](int iters) {
    for (int it = 0; it < iters; ++it) {
      normal_apply0(c, v.p, v.res, v.t, 1);
      step_alpha<double>(c, v.p, v.res, n, c.mg.omega, S_TMP + 8);
      update2<double>(c, x, v.res, v.res, v.p, n, S_TMP + 8);
    }
  };
  smooth(c.mg.nu_pre);
  restrict_to<double>(c, 0, v.res, v.rc, 1);
  const double rc2 = nrm2(c, v.rc, nc);
  fcg(
      c, nc, v.ec, v.rc, [&](cx<double>* o, const cx<double>* i) { normal_apply_c(c, C, o, i, 1); },
      [&](cx<double>* o, const cx<double>* i) { copy<double>(c, o, i, nc); },
      [&](const cx<double>*, double rn2) { return rn2 <= c.mg.coarse_tol * c.mg.coarse_tol * rc2; },
      c.mg.coarse_maxit, v.cg);
  prolong_from<double>(c, 0, v.ec, v.y, 1);
  normal_apply0(c, v.dy, v.y, v.t, 1);
  if (c.mg.use_alpha)
    step_alpha<double>(c, v.dy, v.res, n, 1.0, S_TMP + 8);
  else
    set_scalar(c, S_TMP + 8, 1.0, 0.0);
  update2<double>(c, x, v.y, v.res, v.dy, n, S_TMP + 8);
  smooth(c.mg.nu_post);
}

// CG on the normal equations (precond = false) or MG-CG (precond = true) for
// one right-hand side b (internal layout), x from 0.  Converged when the true
// residual ||b - D x|| / ||b|| <= tol, checked once the normal residual has
// fallen below 1e-2 tol ||b|| (||b - D x|| can exceed it by the conditioning).
int normal_solve(Ctx& c, cx<double>* x, const cx<double>* b, double tol, int maxit, bool precond,
                 wdmg_solve_stats& st) {
  if (precond && !(c.have_mg && c.lev[1].Nc64))
    throw Error(WDMG_ERR_NOT_SETUP, "MG-CG needs a normal-equation hierarchy (wdmg_mg_params.normal = 1)");
  const size_t n = c.lev[0].n;
  NormalWork w, wk;
  w.c = &c;
  wk.c = &c;
  cx<double>* rhs = w.get(n);
  cx<double>* t = w.get(n);
  cx<double>* dx = w.get(n);
  NormalVc* vc = precond ? new NormalVc(c, w) : nullptr;
  struct Del {
    NormalVc* v;
    ~Del() { delete v; }
  } del{vc};
  const double bn2 = nrm2(c, b, n);
  if (!std::isfinite(bn2)) throw Error(WDMG_ERR_NAN, "NaN or Inf in the right-hand side");
  st = wdmg_solve_stats{};
  zero<double>(c, x, n);
  if (bn2 == 0.0) {
    st.converged = 1;
    return WDMG_OK;
  }
  apply_Ddag0(c, rhs, b, t, 1);
  const double thr = 1e-4 * tol * tol * bn2;
  double tres = 1.0;
  auto true_res = [&](const cx<double>* xx) {
    dslash<double>(c, dx, xx, 1);
    xmy_norm(c, b, dx, n, S_TMP + 4);
    return std::sqrt(read_scalar(c, S_TMP + 4) / bn2);
  };
  const int it = fcg(
      c, n, x, rhs, [&](cx<double>* o, const cx<double>* i) { normal_apply0(c, o, i, t, 1); },
      [&](cx<double>* o, const cx<double>* i) {
        if (precond)
          normal_vcycle(c, o, i, *vc);
        else
          copy<double>(c, o, i, n);
      },
      [&](const cx<double>* xx, double rn2) {
        if (rn2 > thr) return false;
        tres = true_res(xx);
        return tres <= tol;
      },
      maxit, wk);
  st.iters = it;
  st.true_res = true_res(x);
  st.converged = st.true_res <= tol;
  return st.converged ? WDMG_OK : WDMG_NOT_CONVERGED;
}

}  // namespace wdmg
