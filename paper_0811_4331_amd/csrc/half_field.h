// 16-bit storage (FP16 or BF16) of fine fields, links, prolongator columns
// and coarse-operator blocks; arithmetic stays in FP32.
//
// Spinor fields: the 64-site block layout of fine_field.h with 4-byte
// complex elements, plus one FP32 scale per site (per right-hand side).  The
// scale of a site is the largest magnitude of its 24 real components; the
// stored values are those components times the FP32 reciprocal of the scale,
// rounded to nearest-even into the 16-bit format, so every stored value lies
// in [-1, 1].  A site whose scale is below the smallest normal FP32 number
// is stored as zero.  Reading multiplies by the scale.
//
// Links (|U_ab| <= 1) and prolongator columns (orthonormal, every entry of
// magnitude <= 1) are stored unscaled.  Coarse-operator blocks carry one
// FP32 scale per (2Nv x 2Nv) block, the largest magnitude of its real
// components.
#pragma once

#include <float.h>

#include "fine_field.h"

namespace wdmg {

typedef _Float16 f16_t;
typedef __bf16 bf16_t;

template <typename H>
struct __align__(4) cxh {
  H re, im;
};

template <typename H>
__device__ __forceinline__ cx<float> h2f(cxh<H> a) {
  return mk((float)a.re, (float)a.im);
}
template <typename H>
__device__ __forceinline__ cxh<H> f2h(float re, float im) {
  cxh<H> r;
  r.re = (H)re;
  r.im = (H)im;
  return r;
}

// Reciprocal used to quantise a site or block with largest magnitude m.
// Zero and subnormal m store zeros; NaN or Inf propagate into the values.
__device__ __forceinline__ float quant_scale(float m, float& inv) {
  if (m >= FLT_MIN && m <= FLT_MAX) {
    inv = 1.0f / m;
    return m;
  }
  if (m < FLT_MIN) {
    inv = 0.0f;
    return 0.0f;
  }
  inv = m;
  return m;
}

// One site of a 16-bit spinor field (values v, scales sc; sc indexed by site).
template <typename H>
__device__ __forceinline__ void load_site_h(const cxh<H>* __restrict__ v, const float* __restrict__ sc, int s,
                                            cx<float> (&a)[12]) {
  const float m = sc[s];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const cx<float> q = h2f(v[fidx(s, k, 12)]);
    a[k] = mk(m * q.re, m * q.im);
  }
}

// FP32 value -> 16 bits, where the value is the FP32 product x * inv: the
// empty asm statement pins the rounded FP32 product in a register, so the
// compiler cannot fuse multiply and conversion into one mixed-precision
// multiply (which would round the exact product once).
template <typename H>
__device__ __forceinline__ cxh<H> quantise(float re, float im, float inv) {
  float pr = re * inv, pi = im * inv;
  asm("" : "+v"(pr), "+v"(pi));
  return f2h<H>(pr, pi);
}

template <typename H>
__device__ __forceinline__ void store_site_h(cxh<H>* __restrict__ v, float* __restrict__ sc, int s,
                                             const cx<float> (&a)[12]) {
  float m = 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(a[k].re), fabsf(a[k].im)));
#pragma unroll
  for (int k = 0; k < 12; ++k)
    if (a[k].re != a[k].re || a[k].im != a[k].im) m = a[k].re + a[k].im;  // NaN wins
  float inv;
  sc[s] = quant_scale(m, inv);
#pragma unroll
  for (int k = 0; k < 12; ++k) v[fidx(s, k, 12)] = quantise<H>(a[k].re, a[k].im, inv);
}

// Links: first two rows, unscaled, same layout as fine_field.h.
template <typename H>
__device__ __forceinline__ void load_link_h(const cxh<H>* __restrict__ U, int mu, int s, bool neg,
                                            cx<float> (&u)[9]) {
  const cxh<H>* base = U + fidx(s, mu * 6, kLinkComp);
#pragma unroll
  for (int e = 0; e < 6; ++e) u[e] = h2f(base[e * 64]);
  recon_third_row(u, neg);
}

}  // namespace wdmg
