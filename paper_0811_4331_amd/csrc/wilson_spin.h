// Spin structure of the Wilson hops in the chiral basis (Sec. 1 operator):
// the projectors (1 -+ gamma_mu) have rank two, so a hop acts on a half
// spinor (two spins x three colours) and expands back to four spins.
#pragma once

#include "common.h"

namespace wdmg {

// Half-spinor projection h = first two rows of (1 - sign*gamma_mu) psi, per colour.
template <int MU, int SIGN, typename R>
__device__ __forceinline__ void project(const cx<R> (&p)[12], cx<R> (&h)[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if (MU == 0) {  // gamma_1 : (g psi) = (-i p3, -i p2, i p1, i p0)
      h[c] = SIGN > 0 ? p0 + ti(p3) : p0 - ti(p3);
      h[3 + c] = SIGN > 0 ? p1 + ti(p2) : p1 - ti(p2);
    } else if (MU == 1) {  // gamma_2 : (-p3, p2, p1, -p0)
      h[c] = SIGN > 0 ? p0 + p3 : p0 - p3;
      h[3 + c] = SIGN > 0 ? p1 - p2 : p1 + p2;
    } else if (MU == 2) {  // gamma_3 : (-i p2, i p3, i p0, -i p1)
      h[c] = SIGN > 0 ? p0 + ti(p2) : p0 - ti(p2);
      h[3 + c] = SIGN > 0 ? p1 - ti(p3) : p1 + ti(p3);
    } else {  // gamma_4 : (p2, p3, p0, p1)
      h[c] = SIGN > 0 ? p0 - p2 : p0 + p2;
      h[3 + c] = SIGN > 0 ? p1 - p3 : p1 + p3;
    }
  }
}

// acc += full four-spin image of the (link-multiplied) half spinor.
template <int MU, int SIGN, typename R>
__device__ __forceinline__ void expand_add(const cx<R> (&h)[6], cx<R> (&acc)[12]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<R> h0 = h[c], h1 = h[3 + c];
    acc[c] = acc[c] + h0;
    acc[3 + c] = acc[3 + c] + h1;
    if (MU == 0) {  // (1 - g1): (h0, h1, -i h1, -i h0); (1 + g1): (h0, h1, i h1, i h0)
      acc[6 + c] = acc[6 + c] + (SIGN > 0 ? tmi(h1) : ti(h1));
      acc[9 + c] = acc[9 + c] + (SIGN > 0 ? tmi(h0) : ti(h0));
    } else if (MU == 1) {  // (h0, h1, -h1, h0) ; (h0, h1, h1, -h0)
      acc[6 + c] = SIGN > 0 ? acc[6 + c] - h1 : acc[6 + c] + h1;
      acc[9 + c] = SIGN > 0 ? acc[9 + c] + h0 : acc[9 + c] - h0;
    } else if (MU == 2) {  // (h0, h1, -i h0, i h1) ; (h0, h1, i h0, -i h1)
      acc[6 + c] = acc[6 + c] + (SIGN > 0 ? tmi(h0) : ti(h0));
      acc[9 + c] = acc[9 + c] + (SIGN > 0 ? ti(h1) : tmi(h1));
    } else {  // (h0, h1, -h0, -h1) ; (h0, h1, h0, h1)
      acc[6 + c] = SIGN > 0 ? acc[6 + c] - h0 : acc[6 + c] + h0;
      acc[9 + c] = SIGN > 0 ? acc[9 + c] - h1 : acc[9 + c] + h1;
    }
  }
}

// acc += sc * (full four-spin image of h): the expansion of a hop whose
// neighbour spinor was read without its 16-bit storage scale sc (the scale
// commutes with the projection and the link product, and every add of the
// expansion becomes one fused multiply-add).
template <int MU, int SIGN, typename R>
__device__ __forceinline__ void expand_add_scaled(const cx<R> (&h)[6], R sc, cx<R> (&acc)[12]) {
  const R ms = -sc;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<R> h0 = h[c], h1 = h[3 + c];
    acc[c] = mk<R>(fma(sc, h0.re, acc[c].re), fma(sc, h0.im, acc[c].im));
    acc[3 + c] = mk<R>(fma(sc, h1.re, acc[3 + c].re), fma(sc, h1.im, acc[3 + c].im));
    // the image's components 2 and 3 as (coefficient of h.re / h.im) pairs
    if (MU == 0) {  // (1 - g1): (-i h1, -i h0); (1 + g1): (i h1, i h0)
      if (SIGN > 0) {
        acc[6 + c] = mk<R>(fma(sc, h1.im, acc[6 + c].re), fma(ms, h1.re, acc[6 + c].im));
        acc[9 + c] = mk<R>(fma(sc, h0.im, acc[9 + c].re), fma(ms, h0.re, acc[9 + c].im));
      } else {
        acc[6 + c] = mk<R>(fma(ms, h1.im, acc[6 + c].re), fma(sc, h1.re, acc[6 + c].im));
        acc[9 + c] = mk<R>(fma(ms, h0.im, acc[9 + c].re), fma(sc, h0.re, acc[9 + c].im));
      }
    } else if (MU == 1) {  // (-h1, h0) ; (h1, -h0)
      const R s2 = SIGN > 0 ? ms : sc, s3 = SIGN > 0 ? sc : ms;
      acc[6 + c] = mk<R>(fma(s2, h1.re, acc[6 + c].re), fma(s2, h1.im, acc[6 + c].im));
      acc[9 + c] = mk<R>(fma(s3, h0.re, acc[9 + c].re), fma(s3, h0.im, acc[9 + c].im));
    } else if (MU == 2) {  // (-i h0, i h1) ; (i h0, -i h1)
      if (SIGN > 0) {
        acc[6 + c] = mk<R>(fma(sc, h0.im, acc[6 + c].re), fma(ms, h0.re, acc[6 + c].im));
        acc[9 + c] = mk<R>(fma(ms, h1.im, acc[9 + c].re), fma(sc, h1.re, acc[9 + c].im));
      } else {
        acc[6 + c] = mk<R>(fma(ms, h0.im, acc[6 + c].re), fma(sc, h0.re, acc[6 + c].im));
        acc[9 + c] = mk<R>(fma(sc, h1.im, acc[9 + c].re), fma(ms, h1.re, acc[9 + c].im));
      }
    } else {  // (-h0, -h1) ; (h0, h1)
      const R s23 = SIGN > 0 ? ms : sc;
      acc[6 + c] = mk<R>(fma(s23, h0.re, acc[6 + c].re), fma(s23, h0.im, acc[6 + c].im));
      acc[9 + c] = mk<R>(fma(s23, h1.re, acc[9 + c].re), fma(s23, h1.im, acc[9 + c].im));
    }
  }
}

}  // namespace wdmg
