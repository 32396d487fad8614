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
// fine_field.h).  One thread per (site, right-hand side); workgroups are
// remapped so spatially adjacent tiles share an XCD's L2.
#include "fine_field.h"
#include "internal.h"
#include "wilson_spin.h"

namespace wdmg {
namespace {

constexpr int kDslashThreads = 128;

template <int MU, int SIGN, typename R>
__device__ __forceinline__ void hop(const cx<R>* __restrict__ in, const cx<R>* __restrict__ U, int nb,
                                    int link_site, bool neg, cx<R> (&acc)[12]) {
  cx<R> p[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = in[fidx(nb, k, 12)];
  cx<R> h[6];
  project<MU, SIGN>(p, h);
  cx<R> u[9];
  load_link(U, MU, link_site, neg, u);
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
  expand_add<MU, SIGN>(uh, acc);
}

// One thread per site; blockIdx.y = right-hand side.  Padding sites
// (vol <= s < vpad) are written as zeros.
// Workgroup order for a batch of nrhs fields over nsb site blocks: the hardware
// sends workgroup b to XCD b % 8.  Each XCD takes a contiguous run of site
// blocks (spatial neighbours share its L2) and, within it, all right-hand
// sides of one site block back to back (its links are read once from HBM).
__device__ __forceinline__ void batch_block(int nsb, int nrhs, int& sb, int& rhs) {
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
  const int xcd = b & 7, local = b >> 3;
  sb = xcd * (nsb >> 3) + local / nrhs;
  rhs = local % nrhs;
}

template <typename R>
__global__ __launch_bounds__(kDslashThreads) void k_dslash(Geom g, cx<R>* __restrict__ out,
                                                          const cx<R>* __restrict__ in,
                                                          const cx<R>* __restrict__ U, R diag, int tneg, int nsb,
                                                          int nrhs) {
  int sb, rhs;
  batch_block(nsb, nrhs, sb, rhs);
  const int s = sb * kDslashThreads + threadIdx.x;
  const size_t off = (size_t)rhs * 12 * g.vpad;
  in += off;
  out += off;
  if (s >= g.vol) {
    if (s < g.vpad) {
#pragma unroll
      for (int k = 0; k < 12; ++k) out[fidx(s, k, 12)] = mk<R>(0, 0);
    }
    return;
  }
  int c[4];
  coords_of(g, s, c);
  cx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<R>(0, 0);
  const bool tlast = tneg && c[3] == g.L[3] - 1, tfirst = tneg && c[3] == 0;
  {
    const int f = nbr_fwd(g, s, c, 0), b = nbr_bwd(g, s, c, 0);
    hop<0, +1>(in, U, f, s, false, acc);
    hop<0, -1>(in, U, b, b, false, acc);
  }
  {
    const int f = nbr_fwd(g, s, c, 1), b = nbr_bwd(g, s, c, 1);
    hop<1, +1>(in, U, f, s, false, acc);
    hop<1, -1>(in, U, b, b, false, acc);
  }
  {
    const int f = nbr_fwd(g, s, c, 2), b = nbr_bwd(g, s, c, 2);
    hop<2, +1>(in, U, f, s, false, acc);
    hop<2, -1>(in, U, b, b, false, acc);
  }
  {
    const int f = nbr_fwd(g, s, c, 3), b = nbr_bwd(g, s, c, 3);
    hop<3, +1>(in, U, f, s, tlast, acc);
    hop<3, -1>(in, U, b, b, tfirst, acc);
  }
  const R half = (R)0.5;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const cx<R> p = in[fidx(s, k, 12)];
    out[fidx(s, k, 12)] = mk<R>(diag * p.re - half * acc[k].re, diag * p.im - half * acc[k].im);
  }
}

}  // namespace

template <typename R>
void dslash(Ctx& c, cx<R>* out, const cx<R>* in, int nrhs) {
  const Geom& g = c.g0;
  const cx<R>* U = nullptr;
  if constexpr (sizeof(R) == 8)
    U = c.U64;
  else
    U = c.U32;
  const unsigned gx = g.vpad / kDslashThreads + (g.vpad % kDslashThreads != 0);
  ProfScope ps(c, sizeof(R) == 8 ? WDMG_K_DSLASH_F64 : WDMG_K_DSLASH_F32, (long long)g.vol * nrhs);
  const int tneg = c.t_bc < 0 ? 1 : 0;
  hipLaunchKernelGGL((k_dslash<R>), dim3(gx * nrhs), dim3(kDslashThreads), 0, c.stream, g, out, in, U,
                     (R)(4.0 + c.mass), tneg, (int)gx, nrhs);
  WDMG_HIP(hipGetLastError());
  c.n_D += nrhs;
}

template void dslash<double>(Ctx&, cx<double>*, const cx<double>*, int);
template void dslash<float>(Ctx&, cx<float>*, const cx<float>*, int);

}  // namespace wdmg
