// Wilson-Dirac operator on gfx950 (Sec. 1):
//   (D psi)(x) = (4 + m) psi(x)
//              - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
// in the chiral basis (gamma5 = diag(1,1,-1,-1)).  Each hop projects the
// neighbour spinor onto the two-dimensional image of (1 -+ gamma_mu), applies
// the SU(3) link to the two colour vectors of that half spinor, and expands
// back to four spins.  The antiperiodic time sign is folded into the stored
// links U_t(x) at t = Lt-1, so it reaches both hop directions.
//
// Layout: fields in 64-site blocks, links as their first two rows (see
// fine_field.h).  Three forms with the same result: one thread per (site,
// right-hand side); one wave per direction; the latter with its registers
// capped for a fourth wave per SIMD.  Workgroups are remapped so spatially
// adjacent tiles share an XCD's L2.
#include "half_field.h"
#include "internal.h"
#include "wilson_spin.h"

namespace wdmg {
namespace {

constexpr int kDslashThreads = 128;

// Field and link access of one precision.  FullIO: FP64 or FP32 fields and
// links.  HalfIO: 16-bit fields with per-site scales and 16-bit links,
// arithmetic in FP32.
template <typename R>
struct FullIO {
  using T = R;
  static constexpr bool kScaled = false;  // values are read as they are stored
  const cx<R>* in;
  cx<R>* out;
  const cx<R>* U;
  __device__ __forceinline__ void select_rhs(int rhs, int vpad) {
    in += (size_t)rhs * 12 * vpad;
    out += (size_t)rhs * 12 * vpad;
  }
  __device__ __forceinline__ void spinor(int s, cx<R> (&p)[12]) const {
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = in[fidx(s, k, 12)];
  }
  __device__ __forceinline__ void link(int mu, int s, bool neg, cx<R> (&u)[9]) const { load_link(U, mu, s, neg, u); }
  __device__ __forceinline__ void store(int s, const cx<R> (&v)[12]) const {
#pragma unroll
    for (int k = 0; k < 12; ++k) out[fidx(s, k, 12)] = v[k];
  }
  // right-hand side r of the selected chunk
  __device__ __forceinline__ void spinor_r(int r, int vpad, int s, cx<R> (&p)[12]) const {
    const cx<R>* b = in + (size_t)r * 12 * vpad;
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = b[fidx(s, k, 12)];
  }
  __device__ __forceinline__ void store_r(int r, int vpad, int s, const cx<R> (&v)[12]) const {
    cx<R>* b = out + (size_t)r * 12 * vpad;
#pragma unroll
    for (int k = 0; k < 12; ++k) b[fidx(s, k, 12)] = v[k];
  }
};

template <typename H>
struct HalfIO {
  using T = float;
  static constexpr bool kScaled = true;  // spinor_raw: stored values and the site scale apart
  const cxh<H>* in;
  const float* isc;
  cxh<H>* out;
  float* osc;
  const cxh<H>* U;
  __device__ __forceinline__ void select_rhs(int rhs, int vpad) {
    in += (size_t)rhs * 12 * vpad;
    out += (size_t)rhs * 12 * vpad;
    isc += (size_t)rhs * vpad;
    osc += (size_t)rhs * vpad;
  }
  __device__ __forceinline__ void spinor(int s, cx<float> (&p)[12]) const { load_site_h(in, isc, s, p); }
  // the stored values of site s (in [-1, 1]) and the scale they are multiplied by
  __device__ __forceinline__ void spinor_raw(int s, cx<float> (&p)[12], float& sc) const {
    sc = isc[s];
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = h2f(in[fidx(s, k, 12)]);
  }
  __device__ __forceinline__ void link(int mu, int s, bool neg, cx<float> (&u)[9]) const {
    load_link_h(U, mu, s, neg, u);
  }
  __device__ __forceinline__ void store(int s, const cx<float> (&v)[12]) const { store_site_h(out, osc, s, v); }
  __device__ __forceinline__ void spinor_r(int r, int vpad, int s, cx<float> (&p)[12]) const {
    load_site_h(in + (size_t)r * 12 * vpad, isc + (size_t)r * vpad, s, p);
  }
  __device__ __forceinline__ void spinor_r_raw(int r, int vpad, int s, cx<float> (&p)[12], float& sc) const {
    const cxh<H>* b = in + (size_t)r * 12 * vpad;
    sc = isc[(size_t)r * vpad + s];
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = h2f(b[fidx(s, k, 12)]);
  }
  __device__ __forceinline__ void store_r(int r, int vpad, int s, const cx<float> (&v)[12]) const {
    store_site_h(out + (size_t)r * 12 * vpad, osc + (size_t)r * vpad, s, v);
  }
};

template <int MU, int SIGN, class IO, typename R = typename IO::T>
__device__ __forceinline__ void hop(const IO& io, int nb, int link_site, bool neg, cx<R> (&acc)[12]) {
  cx<R> p[12];
  R sc = (R)1;
  if constexpr (IO::kScaled)
    io.spinor_raw(nb, p, sc);  // the scale is applied in the expansion
  else
    io.spinor(nb, p);
  cx<R> h[6];
  project<MU, SIGN>(p, h);
  cx<R> u[9];
  io.link(MU, link_site, neg, u);
  cx<R> uh[6];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cx<R> s = mk<R>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (SIGN > 0)
          cmadd(s, u[i * 3 + b], h[a * 3 + b]);   // U h
        else
          cmaddc(s, u[b * 3 + i], h[a * 3 + b]);  // U^+ h
      }
      uh[a * 3 + i] = s;
    }
  }
  if constexpr (IO::kScaled)
    expand_add_scaled<MU, SIGN>(uh, sc, acc);
  else
    expand_add<MU, SIGN>(uh, acc);
}

// One thread per site; blockIdx.y = right-hand side.  Padding sites
// (vol <= s < vpad) are written as zeros.
// Workgroup order for a batch of nrhs fields over nsb site blocks: the hardware
// sends workgroup b to XCD b % 8.  Each XCD takes a contiguous run of site
// blocks (spatial neighbours share its L2) and sweeps it once per group of rg
// right-hand sides, the rhs of a group back to back on each site block (its
// links come from HBM once per group).  Small groups keep more site blocks in
// flight (neighbour spinors stay in L2); large ones share links more.
__device__ __forceinline__ void batch_block(int nsb, int nrhs, int rg, int& sb, int& rhs) {
  const int b = blockIdx.x;
  if ((nsb & 7) || nrhs == 1) {
    if (nrhs == 1) {
      sb = xcd_block();
      rhs = 0;
    } else {
      sb = b % nsb;
      rhs = b / nsb;
    }
    return;
  }
  const int xcd = b & 7, local = b >> 3, nsb8 = nsb >> 3;
  if (rg < 1 || rg > nrhs) rg = nrhs;
  const int g = local / (nsb8 * rg);
  const int size = min(rg, nrhs - g * rg);
  const int off = local - g * nsb8 * rg;
  sb = xcd * nsb8 + off / size;
  rhs = g * rg + off % size;
}

// Tile-column box order (forms 6-8) for lattices cut into 4^4 tiles: XCD k
// takes box k of the xyz tile columns (the boxes of the t-marching form) and
// walks it layer by layer, t outermost within an rhs group: the blocks of
// one time layer of the box, then of the next, so the time neighbours of a
// layer are the blocks its XCD handled just before and just after.  `n`
// counts rhs (or rhs chunks of the register-blocked form) and rg the group.
struct BoxOrder {
  int on;
  int ncol, nT0, nT1, Lt;
  int box[3], nbox[3];
};

__device__ __forceinline__ void box_block(const BoxOrder& o, int n, int rg, int& sb, int& rhs) {
  const int b = blockIdx.x;
  const int xcd = b & 7, local = b >> 3;
  const int bs = o.box[0] * o.box[1] * o.box[2];
  if (rg < 1 || rg > n) rg = n;
  const int per = o.Lt * bs;  // blocks of one rhs in the box
  const int g = local / (per * rg);
  const int size = min(rg, n - g * rg);
  const int off = local - g * per * rg;
  const int t = off / (bs * size);
  const int rem = off % (bs * size);
  const int in = rem / size;
  rhs = g * rg + rem % size;
  const int bx = xcd % o.nbox[0], by = (xcd / o.nbox[0]) % o.nbox[1], bz = xcd / (o.nbox[0] * o.nbox[1]);
  const int tx = bx * o.box[0] + in % o.box[0];
  const int ty = by * o.box[1] + (in / o.box[0]) % o.box[1];
  const int tz = bz * o.box[2] + in / (o.box[0] * o.box[1]);
  const int col = tx + o.nT0 * (ty + o.nT1 * tz);
  sb = ((col + o.ncol * (t >> 2)) << 2) + (t & 3);
}

// MR step-size partial sums of one wave (Sec. 3 smoother): Re and Im of
// <out, in> and |out|^2 over the wave's sites, where `in` is the operator's
// input at the site itself (already loaded for the mass term).  Lanes of
// sites outside the lattice pass live = false.  Lane 0 writes the three sums
// to dots[(rhs * nparts + part) * 3 + k]; the fixed slot per wave keeps the
// result independent of scheduling.
template <typename R>
__device__ __forceinline__ void wave_dots(bool live, const cx<R> (&out)[12], const cx<R> (&in)[12], double* dots,
                                          size_t slot, R in_scale = (R)1) {
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  if (live) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double ore = out[k].re, oim = out[k].im, ire = in[k].re, iim = in[k].im;
      d0 += ore * ire + oim * iim;
      d1 += ore * iim - oim * ire;
      d2 += ore * ore + oim * oim;
    }
    d0 *= (double)in_scale;  // in = in_scale x the values passed (16-bit storage)
    d1 *= (double)in_scale;
  }
  d0 = wave_sum(d0);
  d1 = wave_sum(d1);
  d2 = wave_sum(d2);
  if ((threadIdx.x & 63) == 0) {
    dots[slot * 3 + 0] = d0;
    dots[slot * 3 + 1] = d1;
    dots[slot * 3 + 2] = d2;
  }
}

template <class IO, bool DOTS, typename R = typename IO::T>
__global__ __launch_bounds__(kDslashThreads) void k_dslash(Geom g, IO io, R diag, int tneg, int nsb, int nrhs,
                                                           int rg, double* dots) {
  int sb, rhs;
  batch_block(nsb, nrhs, rg, sb, rhs);
  const int s = sb * kDslashThreads + threadIdx.x;
  io.select_rhs(rhs, g.vpad);
  cx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<R>(0, 0);
  const bool live = s < g.vol;
  cx<R> p[12];
  R psc = (R)1;  // storage scale of p (16-bit fields read raw)
  if (live) {
    int c[4];
    coords_of(g, s, c);
    const bool tlast = tneg && c[3] == g.L[3] - 1, tfirst = tneg && c[3] == 0;
    {
      const int f = nbr_fwd(g, s, c, 0), b = nbr_bwd(g, s, c, 0);
      hop<0, +1>(io, f, s, false, acc);
      hop<0, -1>(io, b, b, false, acc);
    }
    {
      const int f = nbr_fwd(g, s, c, 1), b = nbr_bwd(g, s, c, 1);
      hop<1, +1>(io, f, s, false, acc);
      hop<1, -1>(io, b, b, false, acc);
    }
    {
      const int f = nbr_fwd(g, s, c, 2), b = nbr_bwd(g, s, c, 2);
      hop<2, +1>(io, f, s, false, acc);
      hop<2, -1>(io, b, b, false, acc);
    }
    {
      const int f = nbr_fwd(g, s, c, 3), b = nbr_bwd(g, s, c, 3);
      hop<3, +1>(io, f, s, tlast, acc);
      hop<3, -1>(io, b, b, tfirst, acc);
    }
    const R half = (R)0.5;
    if constexpr (IO::kScaled)
      io.spinor_raw(s, p, psc);
    else
      io.spinor(s, p);
    const R dg = diag * psc;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mk<R>(dg * p[k].re - half * acc[k].re, dg * p[k].im - half * acc[k].im);
  }
  if (s < g.vpad) io.store(s, acc);  // padding sites: zeros
  if constexpr (DOTS)
    wave_dots(live, acc, p, dots,
              (size_t)rhs * nsb * (kDslashThreads / 64) + (size_t)sb * (kDslashThreads / 64) + (threadIdx.x >> 6),
              psc);
}

// Direction-split form: a workgroup of four waves covers one 64-site block;
// wave mu computes the two hops along mu (forward and backward) for the 64
// sites, the partial sums meet in LDS, and wave 0 adds them in direction
// order, applies the mass term and stores.  Four times as many waves as the
// one-thread-per-site kernel, each with a quarter of the hops and of the
// registers, so loads of many more sites are in flight.
template <int MU, class IO, typename R>
__device__ __forceinline__ void hops_mu(const IO& io, const Geom& g, int s, const int (&c)[4], bool tneg,
                                        cx<R> (&acc)[12]) {
  const bool last = MU == 3 && tneg && c[3] == g.L[3] - 1, first = MU == 3 && tneg && c[3] == 0;
  const int f = nbr_fwd(g, s, c, MU), b = nbr_bwd(g, s, c, MU);
  hop<MU, +1>(io, f, s, last, acc);
  hop<MU, -1>(io, b, b, first, acc);
}

constexpr int kDs4Sites = 64;

// MINW: the fewest waves per SIMD the register allocation must allow (1: no
// limit).  FP64 needs 132 registers unconstrained (3 waves per SIMD); with
// MINW = 4 it fits in 128 with one spilled register.
template <class IO, bool DOTS, int MINW, typename R = typename IO::T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MINW))) void k_dslash4(Geom g, IO io, R diag,
                                                                                            int tneg, int nsb,
                                                                                            int nrhs, int rg,
                                                                                            double* dots,
                                                                                            BoxOrder bo) {
  __shared__ cx<R> part[3][12][kDs4Sites];
  int sb, rhs;
  if (bo.on)
    box_block(bo, nrhs, rg, sb, rhs);
  else
    batch_block(nsb, nrhs, rg, sb, rhs);
  const int lane = threadIdx.x & 63, mu = threadIdx.x >> 6;
  const int s = sb * kDs4Sites + lane;
  io.select_rhs(rhs, g.vpad);
  cx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<R>(0, 0);
  const bool live = s < g.vol;
  if (live) {
    int c[4];
    coords_of(g, s, c);
    switch (mu) {
      case 0: hops_mu<0>(io, g, s, c, tneg, acc); break;
      case 1: hops_mu<1>(io, g, s, c, tneg, acc); break;
      case 2: hops_mu<2>(io, g, s, c, tneg, acc); break;
      default: hops_mu<3>(io, g, s, c, tneg, acc); break;
    }
  }
  if (mu > 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) part[mu - 1][k][lane] = acc[k];
  }
  __syncthreads();
  // the grid covers vpad sites in whole 64-site blocks, so the test below is
  // uniform over the wave
  if (mu != 0 || s >= g.vpad) return;
  cx<R> p[12];
  R psc = (R)1;  // storage scale of p (16-bit fields read raw)
  if (live) {
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = acc[k] + part[0][k][lane] + part[1][k][lane] + part[2][k][lane];
    const R half = (R)0.5;
    if constexpr (IO::kScaled)
      io.spinor_raw(s, p, psc);
    else
      io.spinor(s, p);
    const R dg = diag * psc;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mk<R>(dg * p[k].re - half * acc[k].re, dg * p[k].im - half * acc[k].im);
  }
  io.store(s, acc);  // padding sites: zeros
  if constexpr (DOTS) wave_dots(live, acc, p, dots, (size_t)rhs * nsb + sb, psc);
}

// Register-blocked direction-split form for batches: the workgroup layout of
// k_dslash4 (wave mu computes the two hops along mu for 64 sites) with RB
// right-hand sides of one chunk per thread.  Each link is loaded (and its
// third row rebuilt) once and applied to the RB neighbour spinors, so a batch
// reads every link once per chunk instead of once per rhs, and each wave
// keeps RB independent spinor loads in flight.  The partial sums of the four
// directions meet in LDS one rhs at a time (two buffers, one barrier per rhs).
// The batch size must be a multiple of RB; chunks are ordered like the rhs
// of the other forms (batch_block with chunks in place of rhs).
template <int MU, int SIGN, int RB, class IO, typename R = typename IO::T>
__device__ __forceinline__ void hop_rb(const IO& io, int vpad, int nb, int link_site, bool neg,
                                       cx<R> (&acc)[RB][12]) {
  cx<R> u[9];
  io.link(MU, link_site, neg, u);
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    cx<R> p[12];
    R sc = (R)1;
    if constexpr (IO::kScaled)
      io.spinor_r_raw(r, vpad, nb, p, sc);
    else
      io.spinor_r(r, vpad, nb, p);
    cx<R> h[6];
    project<MU, SIGN>(p, h);
    cx<R> uh[6];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        cx<R> t = mk<R>(0, 0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          if (SIGN > 0)
            cmadd(t, u[i * 3 + b], h[a * 3 + b]);   // U h
          else
            cmaddc(t, u[b * 3 + i], h[a * 3 + b]);  // U^+ h
        }
        uh[a * 3 + i] = t;
      }
    }
    if constexpr (IO::kScaled)
      expand_add_scaled<MU, SIGN>(uh, sc, acc[r]);
    else
      expand_add<MU, SIGN>(uh, acc[r]);
  }
}

template <int MU, int RB, class IO, typename R>
__device__ __forceinline__ void hops_mu_rb(const IO& io, const Geom& g, int s, const int (&c)[4], bool tneg,
                                           cx<R> (&acc)[RB][12]) {
  const bool last = MU == 3 && tneg && c[3] == g.L[3] - 1, first = MU == 3 && tneg && c[3] == 0;
  const int f = nbr_fwd(g, s, c, MU), b = nbr_bwd(g, s, c, MU);
  hop_rb<MU, +1, RB>(io, g.vpad, f, s, last, acc);
  hop_rb<MU, -1, RB>(io, g.vpad, b, b, first, acc);
}

template <class IO, bool DOTS, int RB, typename R = typename IO::T>
__global__ __launch_bounds__(256) void k_dslash4_rb(Geom g, IO io, R diag, int tneg, int nsb, int nchunk, int rg,
                                                    double* dots, BoxOrder bo) {
  __shared__ cx<R> part[2][3][12][kDs4Sites];
  int sb, ch;
  if (bo.on)
    box_block(bo, nchunk, rg, sb, ch);
  else
    batch_block(nsb, nchunk, rg, sb, ch);
  const int lane = threadIdx.x & 63, mu = threadIdx.x >> 6;
  const int s = sb * kDs4Sites + lane;
  io.select_rhs(ch * RB, g.vpad);
  cx<R> acc[RB][12];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[r][k] = mk<R>(0, 0);
  const bool live = s < g.vol;
  if (live) {
    int c[4];
    coords_of(g, s, c);
    switch (mu) {
      case 0: hops_mu_rb<0, RB>(io, g, s, c, tneg, acc); break;
      case 1: hops_mu_rb<1, RB>(io, g, s, c, tneg, acc); break;
      case 2: hops_mu_rb<2, RB>(io, g, s, c, tneg, acc); break;
      default: hops_mu_rb<3, RB>(io, g, s, c, tneg, acc); break;
    }
  }
  const R half = (R)0.5;
  // the grid covers vpad sites in whole 64-site blocks: every lane's site is
  // below vpad, and the barrier below is reached by all four waves
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (mu > 0) {
#pragma unroll
      for (int k = 0; k < 12; ++k) part[r & 1][mu - 1][k][lane] = acc[r][k];
    }
    __syncthreads();
    if (mu == 0) {
      cx<R> p[12];
      R psc = (R)1;  // storage scale of p (16-bit fields read raw)
      if (live) {
#pragma unroll
        for (int k = 0; k < 12; ++k)
          acc[r][k] = acc[r][k] + part[r & 1][0][k][lane] + part[r & 1][1][k][lane] + part[r & 1][2][k][lane];
        if constexpr (IO::kScaled)
          io.spinor_r_raw(r, g.vpad, s, p, psc);
        else
          io.spinor_r(r, g.vpad, s, p);
        const R dg = diag * psc;
#pragma unroll
        for (int k = 0; k < 12; ++k)
          acc[r][k] = mk<R>(dg * p[k].re - half * acc[r][k].re, dg * p[k].im - half * acc[r][k].im);
      }
      io.store_r(r, g.vpad, s, acc[r]);  // padding sites: zeros
      if constexpr (DOTS) wave_dots(live, acc[r], p, dots, (size_t)(ch * RB + r) * nsb + sb, psc);
    }
  }
}

// t-marching form for lattices cut into 4^4 tiles: one wave per (xyz tile
// column, chunk of T time layers, rhs); lane = x + 4y + 16z of the 4x4x4 block
// of one layer (the field layout's 64-site block).  The wave walks its chunk
// layer by layer, so every spinor of the column is loaded once: psi(t+1) is
// loaded as the forward time neighbour and becomes the centre of the next
// step, and the backward time hop U_t(x-t)^+ (1+gamma_t) psi(x-t) is formed
// one step earlier from the centre and its own link.  Inside the block the
// x, y, z hops exchange half spinors between lanes (each lane sends
// (1-gamma_mu) psi to x-mu and U_mu^+ (1+gamma_mu) psi to x+mu, both from its
// own spinor and link); lanes on a tile face load the neighbouring tile's
// spinor (and link) instead.  Work items are grouped per XCD in boxes of
// adjacent tile columns, so neighbouring columns share an L2 while they walk
// the same layers (form 5), or per XCD in time slabs (form 9): XCD k takes
// every tile column of the k-th eighth of the time extent, so no x, y or z
// face of a column lies on another XCD and only the two slab ends read time
// neighbours from another XCD's layers; inside the slab the XCD runs the
// columns of a group of G right-hand sides back to back, rhs fastest, so the
// G waves of one column share its links in L2.
struct TmMap {
  int ncol;           // xyz tile columns
  int nch, T;         // chunks of T layers per column
  int nrhs;
  int box[3];         // tile columns per XCD box (0: no XCD boxes)
  int nbox[3];        // boxes per direction (product 8)
  int slab;           // 1: time slabs per XCD (nch a multiple of 8)
  int G;              // rhs group of the slab order (divides nrhs)
};

template <int SIGN, typename R>
__device__ __forceinline__ void link_mul(const cx<R> (&u)[9], const cx<R> (&h)[6], cx<R> (&uh)[6]) {
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cx<R> t = mk<R>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (SIGN > 0)
          cmadd(t, u[i * 3 + b], h[a * 3 + b]);   // U h
        else
          cmaddc(t, u[b * 3 + i], h[a * 3 + b]);  // U^+ h
      }
      uh[a * 3 + i] = t;
    }
  }
}

template <typename R>
__device__ __forceinline__ void shfl6(const cx<R> (&in)[6], cx<R> (&out)[6], int src) {
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = mk<R>(__shfl(in[k].re, src, 64), __shfl(in[k].im, src, 64));
}

// The x, y or z hops of one site with lane-exchanged half spinors.
template <int MU, class IO, typename R = typename IO::T>
__device__ __forceinline__ void tm_space_hops(const IO& io, const Geom& g, int s, const int (&c)[4], int lane,
                                              const cx<R> (&psi)[12], cx<R> (&acc)[12]) {
  constexpr int SL = MU == 0 ? 1 : (MU == 1 ? 4 : 16);
  const int lc = (lane / SL) & 3;
  cx<R> u[9];
  io.link(MU, s, false, u);
  // messages of this lane: (1-gamma) psi for x-mu, U^+ (1+gamma) psi for x+mu
  cx<R> mf[6], mb[6], t6[6];
  project<MU, +1>(psi, mf);
  project<MU, -1>(psi, t6);
  link_mul<-1>(u, t6, mb);
  // forward hop: (1-gamma) psi(x+mu) from lane + SL, or from the next tile
  cx<R> h[6];
  shfl6(mf, h, lane + SL);
  if (lc == 3) {
    cx<R> p[12];
    io.spinor(nbr_fwd(g, s, c, MU), p);
    project<MU, +1>(p, h);
  }
  cx<R> uh[6];
  link_mul<+1>(u, h, uh);
  expand_add<MU, +1>(uh, acc);
  // backward hop: U^+(x-mu) (1+gamma) psi(x-mu) from lane - SL, or computed
  // here from the previous tile's spinor and link
  shfl6(mb, uh, lane - SL);
  if (lc == 0) {
    const int b = nbr_bwd(g, s, c, MU);
    cx<R> p[12], ub[9];
    io.spinor(b, p);
    io.link(MU, b, false, ub);
    project<MU, -1>(p, t6);
    link_mul<-1>(ub, t6, uh);
  }
  expand_add<MU, -1>(uh, acc);
}

__device__ __forceinline__ void tm_work(const TmMap& m, int w, int& col, int& ch, int& rhs, const Geom& g) {
  int tx, ty, tz, local;
  if (m.slab) {
    const int xcd = w & 7;
    local = w >> 3;
    const int rin = local % m.G;
    int rest = local / m.G;
    col = rest % m.ncol;
    rest /= m.ncol;
    const int ngrp = m.nrhs / m.G;
    rhs = (rest % ngrp) * m.G + rin;
    ch = xcd * (m.nch >> 3) + rest / ngrp;
  } else if (m.box[0]) {
    const int xcd = w & 7;
    local = w >> 3;
    const int bs = m.box[0] * m.box[1] * m.box[2];
    const int in = local % bs;
    const int rest = local / bs;
    rhs = rest % m.nrhs;
    ch = rest / m.nrhs;
    const int bx = xcd % m.nbox[0], by = (xcd / m.nbox[0]) % m.nbox[1], bz = xcd / (m.nbox[0] * m.nbox[1]);
    tx = bx * m.box[0] + in % m.box[0];
    ty = by * m.box[1] + (in / m.box[0]) % m.box[1];
    tz = bz * m.box[2] + in / (m.box[0] * m.box[1]);
    col = tx + g.nT[0] * (ty + g.nT[1] * tz);
  } else {
    col = w % m.ncol;
    const int rest = w / m.ncol;
    rhs = rest % m.nrhs;
    ch = rest / m.nrhs;
  }
}

template <class IO, bool DOTS, typename R = typename IO::T>
__global__ __launch_bounds__(64) void k_dslash_tm(Geom g, IO io, R diag, int tneg, TmMap m, double* dots) {
  int col, ch, rhs;
  tm_work(m, blockIdx.x, col, ch, rhs, g);
  io.select_rhs(rhs, g.vpad);
  const int lane = threadIdx.x;
  const int ncol = m.ncol, Lt = g.L[3];
  auto site_at = [&](int t) { return ((col + ncol * (t >> 2)) << 8) + ((t & 3) << 6) + lane; };
  const int t0 = ch * m.T;
  int c[4];
  coords_of(g, site_at(t0), c);
  // backward time hop of the first layer, from layer t0 - 1
  cx<R> bt[6];
  {
    const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
    const int sp = site_at(tp);
    cx<R> p[12], u[9], h[6];
    io.spinor(sp, p);
    io.link(3, sp, tneg && tp == Lt - 1, u);
    project<3, -1>(p, h);
    link_mul<-1>(u, h, bt);
  }
  cx<R> psi[12];
  io.spinor(site_at(t0), psi);
  const R half = (R)0.5;
  for (int t = t0; t < t0 + m.T; ++t) {
    const int s = site_at(t);
    c[3] = t;
    const int tn = t == Lt - 1 ? 0 : t + 1;
    cx<R> nxt[12];
    io.spinor(site_at(tn), nxt);
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mk<R>(0, 0);
    tm_space_hops<0>(io, g, s, c, lane, psi, acc);
    tm_space_hops<1>(io, g, s, c, lane, psi, acc);
    tm_space_hops<2>(io, g, s, c, lane, psi, acc);
    {
      cx<R> u[9], h[6], uh[6];
      const bool neg = tneg && t == Lt - 1;
      io.link(3, s, neg, u);
      project<3, +1>(nxt, h);  // forward time hop
      link_mul<+1>(u, h, uh);
      expand_add<3, +1>(uh, acc);
      expand_add<3, -1>(bt, acc);  // backward time hop
      project<3, -1>(psi, h);      // the next layer's backward hop
      link_mul<-1>(u, h, bt);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[k] = mk<R>(diag * psi[k].re - half * acc[k].re, diag * psi[k].im - half * acc[k].im);
    io.store(s, acc);
    if constexpr (DOTS) wave_dots(true, acc, psi, dots, (size_t)rhs * (g.vpad / 64) + (s >> 6));
#pragma unroll
    for (int k = 0; k < 12; ++k) psi[k] = nxt[k];
  }
}

// Work map of the t-marching form: tile columns split into 8 boxes when the
// tile counts allow (one box per XCD), chunks of T layers.
inline TmMap tm_map(const Geom& g, int nrhs, int T) {
  TmMap m{};
  m.ncol = g.nT[0] * g.nT[1] * g.nT[2];
  m.T = T;
  m.nch = g.L[3] / T;
  m.nrhs = nrhs;
  const int nb[3][3] = {{2, 2, 2}, {1, 2, 4}, {1, 1, 8}};
  for (auto& split : nb) {
    // try the split and its permutations along x, y, z
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (auto& pm : perm) {
      bool ok = true;
      for (int d = 0; d < 3; ++d) ok = ok && g.nT[d] % split[pm[d]] == 0;
      if (!ok) continue;
      for (int d = 0; d < 3; ++d) {
        m.nbox[d] = split[pm[d]];
        m.box[d] = g.nT[d] / split[pm[d]];
      }
      return m;
    }
  }
  return m;
}

// Time-slab map (form 9): chunks of T layers, T the largest divisor of Lt / 8
// up to 8, so every XCD walks the same number of whole chunks; G = rg when it
// divides the batch, else 1.
inline TmMap tm_slab_map(const Geom& g, int nrhs, int rg) {
  TmMap m{};
  m.ncol = g.nT[0] * g.nT[1] * g.nT[2];
  const int nl = g.L[3] / 8;
  m.T = 1;
  for (int T = 1; T <= 8 && T <= nl; ++T)
    if (nl % T == 0) m.T = T;
  m.nch = g.L[3] / m.T;
  m.nrhs = nrhs;
  m.slab = 1;
  m.G = (rg >= 1 && nrhs % rg == 0) ? rg : 1;
  return m;
}

// Layers per chunk of the t-marching form: the rhs-group tuning value when it
// is 4, 8 or 16 and divides Lt, else 8 (or 4).
inline int tm_chunk(const Geom& g, int rg) {
  for (int T : {rg, 8, 4})
    if ((T == 4 || T == 8 || T == 16) && g.L[3] % T == 0) return T;
  return 4;
}

// Slots of MR partial sums per right-hand side written by a fused launch.
int dslash_parts(const Geom& g, int variant) {
  if (variant != 0) return g.vpad / kDs4Sites;  // forms 1-5: one slot per 64-site block
  return (g.vpad / kDslashThreads + (g.vpad % kDslashThreads != 0)) * (kDslashThreads / 64);
}

// Right-hand sides per thread of a form (forms 3 and 4 are register-blocked).
constexpr int rb_of(int variant) { return (variant == 3 || variant == 8) ? 2 : (variant == 4 ? 4 : 1); }

inline BoxOrder box_order(const Geom& g) {
  const TmMap m = tm_map(g, 1, 4);
  BoxOrder o{};
  o.on = m.box[0] != 0;
  o.ncol = m.ncol;
  o.nT0 = g.nT[0];
  o.nT1 = g.nT[1];
  o.Lt = g.L[3];
  for (int d = 0; d < 3; ++d) {
    o.box[d] = m.box[d];
    o.nbox[d] = m.nbox[d];
  }
  return o;
}

// Forms 3, 4 and 8 need a batch they divide; forms 5-9 need 4^4 tiles, 6-8
// tile columns that split into one box per XCD, and 9 a time extent that
// splits into 8 slabs.
inline bool form_fits(const Geom& g, int v, int nrhs) {
  const bool tiles = g.B[0] == 4 && g.B[1] == 4 && g.B[2] == 4 && g.B[3] == 4;
  if (v >= 5 && !tiles) return false;
  if (v == 9) return g.L[3] % 8 == 0;
  if (v >= 6 && !box_order(g).on) return false;
  return nrhs % rb_of(v) == 0;
}

template <class IO>
void run_dslash(Ctx& c, const IO& io, int nrhs, int variant, int rg, double* dots = nullptr) {
  const Geom& g = c.g0;
  const int tneg = c.t_bc < 0 ? 1 : 0;
  using R = typename IO::T;
  const R diag = (R)(4.0 + c.mass);
  BoxOrder bo{};
  if (variant >= 6) bo = box_order(g);  // forms 6-8: forms 1, 2, 3 in tile-column box order
  const int base = variant == 6 ? 1 : (variant == 7 ? 2 : (variant == 8 ? 3 : variant));
  if (base == 1 || base == 2) {
    const unsigned gx = g.vpad / kDs4Sites;
    const dim3 grid(gx * nrhs), block(256);
    if (base == 1) {
      if (dots)
        hipLaunchKernelGGL((k_dslash4<IO, true, 1>), grid, block, 0, c.stream, g, io, diag, tneg, (int)gx, nrhs, rg,
                           dots, bo);
      else
        hipLaunchKernelGGL((k_dslash4<IO, false, 1>), grid, block, 0, c.stream, g, io, diag, tneg, (int)gx, nrhs, rg,
                           dots, bo);
    } else {
      if (dots)
        hipLaunchKernelGGL((k_dslash4<IO, true, 4>), grid, block, 0, c.stream, g, io, diag, tneg, (int)gx, nrhs, rg,
                           dots, bo);
      else
        hipLaunchKernelGGL((k_dslash4<IO, false, 4>), grid, block, 0, c.stream, g, io, diag, tneg, (int)gx, nrhs, rg,
                           dots, bo);
    }
  } else if (base == 5 || base == 9) {
    const TmMap m = base == 5 ? tm_map(g, nrhs, tm_chunk(g, rg)) : tm_slab_map(g, nrhs, rg);
    const dim3 grid((unsigned)(m.ncol * m.nch * nrhs));
    if (dots)
      hipLaunchKernelGGL((k_dslash_tm<IO, true>), grid, dim3(64), 0, c.stream, g, io, diag, tneg, m, dots);
    else
      hipLaunchKernelGGL((k_dslash_tm<IO, false>), grid, dim3(64), 0, c.stream, g, io, diag, tneg, m, dots);
  } else if (base == 3 || base == 4) {
    const unsigned gx = g.vpad / kDs4Sites;
    if (base == 3) {
      const int nch = nrhs / 2, rgc = rg >= 2 ? rg / 2 : 1;
      if (dots)
        hipLaunchKernelGGL((k_dslash4_rb<IO, true, 2>), dim3(gx * nch), dim3(256), 0, c.stream, g, io, diag, tneg,
                           (int)gx, nch, rgc, dots, bo);
      else
        hipLaunchKernelGGL((k_dslash4_rb<IO, false, 2>), dim3(gx * nch), dim3(256), 0, c.stream, g, io, diag, tneg,
                           (int)gx, nch, rgc, dots, bo);
    } else {
      const int nch = nrhs / 4, rgc = rg >= 4 ? rg / 4 : 1;
      if (dots)
        hipLaunchKernelGGL((k_dslash4_rb<IO, true, 4>), dim3(gx * nch), dim3(256), 0, c.stream, g, io, diag, tneg,
                           (int)gx, nch, rgc, dots, bo);
      else
        hipLaunchKernelGGL((k_dslash4_rb<IO, false, 4>), dim3(gx * nch), dim3(256), 0, c.stream, g, io, diag, tneg,
                           (int)gx, nch, rgc, dots, bo);
    }
  } else {
    const unsigned gx = g.vpad / kDslashThreads + (g.vpad % kDslashThreads != 0);
    if (dots)
      hipLaunchKernelGGL((k_dslash<IO, true>), dim3(gx * nrhs), dim3(kDslashThreads), 0, c.stream, g, io, diag, tneg,
                         (int)gx, nrhs, rg, dots);
    else
      hipLaunchKernelGGL((k_dslash<IO, false>), dim3(gx * nrhs), dim3(kDslashThreads), 0, c.stream, g, io, diag, tneg,
                         (int)gx, nrhs, rg, dots);
  }
  WDMG_HIP(hipGetLastError());
}

// Autotuner: times the forms (HIP events, 3 launches each after one warm-up
// launch) on the caller's buffers -- the operator has no side effects besides
// writing `out` -- and returns the fastest (form 1 on ties).  The
// register-blocked forms 3 and 4 take part when the batch is a multiple of
// their 2 or 4 rhs per thread.
constexpr int kDslashForms = 10;

template <class IO>
float time_dslash(Ctx& c, const IO& io, int nrhs, int v, int rg, hipEvent_t (&ev)[2], int reps = 3) {
  run_dslash(c, io, nrhs, v, rg);
  WDMG_HIP(hipEventRecord(ev[0], c.stream));
  for (int i = 0; i < reps; ++i) run_dslash(c, io, nrhs, v, rg);
  WDMG_HIP(hipEventRecord(ev[1], c.stream));
  WDMG_HIP(hipEventSynchronize(ev[1]));
  float ms = 0.f;
  WDMG_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
  return ms / reps;
}

// Timing windows of the autotuner: launches shorter than 0.1 ms are timed in
// windows of at least 0.3 ms (up to 20 launches), best of three interleaved
// rounds, so a few microseconds of launch jitter cannot decide between forms
// that differ by 10%; longer launches keep one window of three.
struct TuneWindow {
  int reps = 3, rounds = 1;
};
inline TuneWindow tune_window(float ms_per_launch) {
  TuneWindow t;
  if (ms_per_launch > 0.f && ms_per_launch < 0.1f) {
    t.rounds = 3;
    t.reps = (int)(0.3f / ms_per_launch) + 1;
    if (t.reps < 3) t.reps = 3;
    if (t.reps > 20) t.reps = 20;
  }
  return t;
}

// Picks the form (rhs groups of the whole batch), then, for a batch, the rhs
// group size among 1, 2, 4, ... and nrhs with that form.  Forced values
// (wdmg_set_tuning) are kept and not timed.
template <class IO>
void tune_dslash(Ctx& c, const IO& io, int nrhs, int& form, int& rg) {
  hipEvent_t ev[2];
  for (auto& e : ev) WDMG_HIP(hipEventCreate(&e));
  TuneWindow tw;
  if (form < 0) {
    const int g = rg < 0 ? nrhs : rg;
    float ms[kDslashForms];
    for (int v = 0; v < kDslashForms; ++v) ms[v] = form_fits(c.g0, v, nrhs) ? time_dslash(c, io, nrhs, v, g, ev) : 1e30f;
    float est = ms[0];
    for (int v = 1; v < kDslashForms; ++v) est = ms[v] < est ? ms[v] : est;
    tw = tune_window(est);
    if (tw.rounds > 1) {
      for (int v = 0; v < kDslashForms; ++v) ms[v] = 1e30f;
      for (int r = 0; r < tw.rounds; ++r)
        for (int v = 0; v < kDslashForms; ++v) {
          if (!form_fits(c.g0, v, nrhs)) continue;
          const float t = time_dslash(c, io, nrhs, v, g, ev, tw.reps);
          if (t < ms[v]) ms[v] = t;
        }
    }
    form = 1;
    for (int v = 0; v < kDslashForms; ++v)
      if (ms[v] < ms[form]) form = v;
  }
  if (rg < 0) {
    rg = nrhs;
    if (nrhs > 1) {
      // candidates: the whole batch, then groups of 1, 2, 4, ...
      int cands[8], nc = 0;
      cands[nc++] = nrhs;
      for (int cand = 1; cand < nrhs && nc < 8; cand *= 2) cands[nc++] = cand;
      float ms[8];
      for (int i = 0; i < nc; ++i) ms[i] = time_dslash(c, io, nrhs, form, cands[i], ev);
      if (tw.rounds == 1) tw = tune_window(ms[0]);
      for (int r = 1; r < tw.rounds; ++r)
        for (int i = 0; i < nc; ++i) {
          const float t = time_dslash(c, io, nrhs, form, cands[i], ev, tw.reps);
          if (t < ms[i]) ms[i] = t;
        }
      float best = ms[0];
      for (int i = 1; i < nc; ++i)
        if (ms[i] < best) {
          best = ms[i];
          rg = cands[i];
        }
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
}

// Runs the operator in the tuned form; with `dots` the launch also writes the
// MR partial sums and the return value is the number of slots per rhs.
template <class IO>
int launch_dslash(Ctx& c, const IO& io, int nrhs, int prof_id, int prec_index, double* dots = nullptr) {
  const int key = nrhs < kMaxRhs ? nrhs : kMaxRhs;
  signed char& fslot = c.tune_dslash[prec_index][key];
  signed char& gslot = c.tune_group[prec_index][key];
  int v = c.tune_force[WDMG_TUNE_DSLASH] >= 0 ? c.tune_force[WDMG_TUNE_DSLASH] : fslot;
  if (v >= 0 && !form_fits(c.g0, v, nrhs)) v = 1;  // a forced register-blocked form on a batch it does not divide
  int rg = c.tune_force[WDMG_TUNE_DSLASH_GROUP] >= 0 ? c.tune_force[WDMG_TUNE_DSLASH_GROUP] : gslot;
  if ((v < 0 || rg < 0) && !c.capturing && !c.no_alloc) {
    tune_dslash(c, io, nrhs, v, rg);
    if (c.tune_force[WDMG_TUNE_DSLASH] < 0) fslot = (signed char)v;
    if (c.tune_force[WDMG_TUNE_DSLASH_GROUP] < 0) gslot = (signed char)rg;
  }
  if (v < 0) v = 1;
  if (rg < 0) rg = nrhs;
  ProfScope ps(c, prof_id, (long long)c.g0.vol * nrhs);
  run_dslash(c, io, nrhs, v, rg, dots);
  c.n_D += nrhs;
  return dslash_parts(c.g0, v);
}

}  // namespace

template <typename R>
void dslash(Ctx& c, cx<R>* out, const cx<R>* in, int nrhs) {
  FullIO<R> io;
  io.in = in;
  io.out = out;
  if constexpr (sizeof(R) == 8)
    io.U = c.U64;
  else
    io.U = c.U32;
  launch_dslash(c, io, nrhs, sizeof(R) == 8 ? WDMG_K_DSLASH_F64 : WDMG_K_DSLASH_F32,
                sizeof(R) == 8 ? WDMG_F64 : WDMG_F32);
}

template <typename H>
void dslash_h(Ctx& c, HF out, HF in, int nrhs) {
  HalfIO<H> io;
  io.in = static_cast<const cxh<H>*>(in.v);
  io.isc = in.s;
  io.out = static_cast<cxh<H>*>(out.v);
  io.osc = out.s;
  io.U = static_cast<const cxh<H>*>(u16(c, half_kind<H>()));
  launch_dslash(c, io, nrhs, half_kind<H>() == WDMG_F16 ? WDMG_K_DSLASH_F16 : WDMG_K_DSLASH_BF16, half_kind<H>());
}

double* dots_buffer(Ctx& c, int nrhs) {
  const size_t need = ((size_t)c.g0.vpad / 64 + 2) * 3 * (size_t)nrhs;
  if (need > c.dots_cap) {
    if (c.capturing) throw Error(WDMG_ERR_ARG, "MR partial-sum buffer too small inside a graph capture");
    WDMG_HIP(hipStreamSynchronize(c.stream));
    dev_free(c, c.dots);
    c.dots = static_cast<double*>(dev_alloc(c, need * sizeof(double)));
    c.dots_cap = need;
  }
  return c.dots;
}

template <typename R>
void dslash_mr(Ctx& c, cx<R>* out, const cx<R>* in, int nrhs, double scale, int slot) {
  FullIO<R> io;
  io.in = in;
  io.out = out;
  if constexpr (sizeof(R) == 8)
    io.U = c.U64;
  else
    io.U = c.U32;
  double* d = dots_buffer(c, nrhs);
  const int nparts = launch_dslash(c, io, nrhs, sizeof(R) == 8 ? WDMG_K_DSLASH_F64 : WDMG_K_DSLASH_F32,
                                   sizeof(R) == 8 ? WDMG_F64 : WDMG_F32, d);
  step_alpha_fin(c, d, nparts, nrhs, scale, slot);
}

template <typename H>
void dslash_h_mr(Ctx& c, HF out, HF in, int nrhs, double scale, int slot) {
  HalfIO<H> io;
  io.in = static_cast<const cxh<H>*>(in.v);
  io.isc = in.s;
  io.out = static_cast<cxh<H>*>(out.v);
  io.osc = out.s;
  io.U = static_cast<const cxh<H>*>(u16(c, half_kind<H>()));
  double* d = dots_buffer(c, nrhs);
  const int nparts = launch_dslash(c, io, nrhs, half_kind<H>() == WDMG_F16 ? WDMG_K_DSLASH_F16 : WDMG_K_DSLASH_BF16,
                                   half_kind<H>(), d);
  step_alpha_fin(c, d, nparts, nrhs, scale, slot);
}

template void dslash<double>(Ctx&, cx<double>*, const cx<double>*, int);
template void dslash<float>(Ctx&, cx<float>*, const cx<float>*, int);
template void dslash_h<f16_t>(Ctx&, HF, HF, int);
template void dslash_h<bf16_t>(Ctx&, HF, HF, int);
template void dslash_mr<double>(Ctx&, cx<double>*, const cx<double>*, int, double, int);
template void dslash_mr<float>(Ctx&, cx<float>*, const cx<float>*, int, double, int);
template void dslash_h_mr<f16_t>(Ctx&, HF, HF, int, double, int);
template void dslash_h_mr<bf16_t>(Ctx&, HF, HF, int, double, int);

}  // namespace wdmg
