// Fine-lattice field layout and link storage.
//
// Sites are numbered tile-major (see Geom).  Fields are stored in blocks of
// 64 consecutive sites -- one wavefront -- with the components of a block
// contiguous: element (site s, component k) of an ncomp-component field sits
// at ((s / 64) * ncomp + k) * 64 + s % 64.  A wavefront's load of one
// component is one contiguous 64-element run, and all components a wavefront
// touches lie in one 12 * 64-element window, which keeps the number of
// distinct memory pages per hop small.  The site count is padded to a
// multiple of 64 (Geom::vpad); padding sites hold zeros.
//
// Links are SU(3) (Sec. 3: unitary connections).  Only their first two rows
// are stored (6 complex per link, 24 per site); the third row is rebuilt as
// the complex conjugate of the cross product of the first two.  The
// antiperiodic time sign is folded into the stored rows of U_t at t = Lt-1,
// so the rebuilt row takes the same sign explicitly.
#pragma once

#include "common.h"

namespace wdmg {

constexpr int kLinkComp = 24;  // stored complex numbers per site (4 links x 2 rows)

__host__ __device__ __forceinline__ size_t fidx(int s, int k, int ncomp) {
  return ((size_t)(s >> 6) * ncomp + k) * 64 + (s & 63);
}

// Third row of an SU(3) link from its first two: conj(row0 x row1), with
// the folded boundary sign when neg.
template <typename R>
__device__ __forceinline__ void recon_third_row(cx<R> (&u)[9], bool neg) {
  const cx<R> c0 = u[1] * u[5] - u[2] * u[4];
  const cx<R> c1 = u[2] * u[3] - u[0] * u[5];
  const cx<R> c2 = u[0] * u[4] - u[1] * u[3];
  const R sg = neg ? (R)-1 : (R)1;
  u[6] = mk<R>(sg * c0.re, -sg * c0.im);
  u[7] = mk<R>(sg * c1.re, -sg * c1.im);
  u[8] = mk<R>(sg * c2.re, -sg * c2.im);
}

template <typename R>
__device__ __forceinline__ void load_link(const cx<R>* __restrict__ U, int mu, int s, bool neg, cx<R> (&u)[9]) {
  const cx<R>* base = U + fidx(s, mu * 6, kLinkComp);
#pragma unroll
  for (int e = 0; e < 6; ++e) u[e] = base[e * 64];
  recon_third_row(u, neg);
}

// Workgroup index remapped so that consecutive tiles (spatial neighbours)
// run on the same XCD and share its L2: hardware dispatches workgroup b to
// XCD b % 8.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  if (nb & 7) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace wdmg
