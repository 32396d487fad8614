// 16-bit storage of fine fields, links and prolongator columns: conversions
// and the buffers that hold them (layout and scaling rules in half_field.h).
#include "half_field.h"
#include "internal.h"

namespace wdmg {
namespace {

template <typename H>
__global__ void k_round_h(const cx<float>* __restrict__ in, cxh<H>* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = f2h<H>(in[i].re, in[i].im);
}

// -v for every stored value: flipping the sign bits of both halves is exact
// (the scales are unchanged).
__global__ void k_neg_h(uint32_t* __restrict__ v, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] ^= 0x80008000u;
}

template <typename H>
__global__ void k_zero_h(Geom g, cxh<H>* __restrict__ v, float* __restrict__ sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vpad) return;
  v += (size_t)r * 12 * g.vpad;
  sc += (size_t)r * g.vpad;
  sc[s] = 0.0f;
#pragma unroll
  for (int k = 0; k < 12; ++k) v[fidx(s, k, 12)] = f2h<H>(0.0f, 0.0f);
}

// internal field (FP64 or FP32, [rhs][12 vpad]) -> 16-bit field
template <typename R, typename H>
__global__ void k_to_half(Geom g, const cx<R>* __restrict__ in, cxh<H>* __restrict__ v, float* __restrict__ sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vpad) return;
  in += (size_t)r * 12 * g.vpad;
  v += (size_t)r * 12 * g.vpad;
  sc += (size_t)r * g.vpad;
  cx<float> a[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) a[k] = cvt<float>(in[fidx(s, k, 12)]);
  store_site_h(v, sc, s, a);
}

template <typename H, typename R>
__global__ void k_from_half(Geom g, const cxh<H>* __restrict__ v, const float* __restrict__ sc,
                            cx<R>* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vpad) return;
  out += (size_t)r * 12 * g.vpad;
  v += (size_t)r * 12 * g.vpad;
  sc += (size_t)r * g.vpad;
  cx<float> a[12];
  load_site_h(v, sc, s, a);
#pragma unroll
  for (int k = 0; k < 12; ++k) out[fidx(s, k, 12)] = cvt<R>(a[k]);
}

// canonical complex64 [rhs][T][Z][Y][X][4][3] -> 16-bit field (padding sites zero)
template <typename H>
__global__ void k_canon_to_half(Geom g, const cx<float>* __restrict__ canon, cxh<H>* __restrict__ v,
                                float* __restrict__ sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vpad) return;
  v += (size_t)r * 12 * g.vpad;
  sc += (size_t)r * g.vpad;
  cx<float> a[12];
  if (s < g.vol) {
    int c[4];
    coords_of(g, s, c);
    const size_t i = (size_t)c[0] + (size_t)g.L[0] * (c[1] + (size_t)g.L[1] * (c[2] + (size_t)g.L[2] * c[3]));
    const cx<float>* src = canon + ((size_t)r * g.vol + i) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = src[k];
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) a[k] = mk(0.0f, 0.0f);
  }
  store_site_h(v, sc, s, a);
}

template <typename H>
__global__ void k_half_to_canon(Geom g, const cxh<H>* __restrict__ v, const float* __restrict__ sc,
                                cx<float>* __restrict__ canon) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vol) return;
  v += (size_t)r * 12 * g.vpad;
  sc += (size_t)r * g.vpad;
  int c[4];
  coords_of(g, s, c);
  const size_t i = (size_t)c[0] + (size_t)g.L[0] * (c[1] + (size_t)g.L[1] * (c[2] + (size_t)g.L[2] * c[3]));
  cx<float> a[12];
  load_site_h(v, sc, s, a);
  cx<float>* dst = canon + ((size_t)r * g.vol + i) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = a[k];
}

template <typename H>
void round_to_half(Ctx& c, const cx<float>* in, void* out, size_t n) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_round_h<H>), dim3((unsigned)blocks), dim3(256), 0, c.stream, in, static_cast<cxh<H>*>(out),
                     n);
  WDMG_HIP(hipGetLastError());
}

void round_kind(Ctx& c, int kind, const cx<float>* in, void* out, size_t n) {
  if (kind == WDMG_F16)
    round_to_half<f16_t>(c, in, out, n);
  else
    round_to_half<bf16_t>(c, in, out, n);
}

dim3 site_grid(const Geom& g, int nrhs) { return dim3((g.vpad + 255) / 256, nrhs); }

}  // namespace

const void* u16(Ctx& c, int kind) {
  if (kind != WDMG_F16 && kind != WDMG_BF16) throw Error(WDMG_ERR_ARG, "not a 16-bit kind");
  if (c.u16_kind == kind) return c.U16;
  const size_t n = (size_t)c.g0.vpad * kLinkComp;
  if (!c.U16) c.U16 = dev_alloc(c, n * 4);
  round_kind(c, kind, c.U32, c.U16, n);
  c.u16_kind = kind;
  return c.U16;
}

const void* v16(Ctx& c, Level& L, int kind) {
  if (kind != WDMG_F16 && kind != WDMG_BF16) throw Error(WDMG_ERR_ARG, "not a 16-bit kind");
  if (L.v16_kind == kind) return L.V16;
  if (!L.V32) throw Error(WDMG_ERR_ARG, "FP32 prolongator released by wdmg_release_unused");
  const size_t n = (size_t)L.nv * L.n;
  if (!L.V16) L.V16 = dev_alloc(c, n * 4);
  round_kind(c, kind, L.V32, L.V16, n);
  L.v16_kind = kind;
  return L.V16;
}

HF hf_alloc(Ctx& c, int nrhs) {
  HF f;
  const size_t vp = c.g0.vpad;
  f.v = dev_alloc(c, (size_t)nrhs * 12 * vp * 4);
  f.s = static_cast<float*>(dev_alloc(c, (size_t)nrhs * vp * sizeof(float)));
  return f;
}

void hf_free(Ctx& c, HF& f) {
  dev_free(c, f.v);
  dev_free(c, f.s);
  f.v = nullptr;
  f.s = nullptr;
}

void hf_copy(Ctx& c, HF dst, HF src, int nrhs) {
  // values (4 bytes each) and scales copied unchanged, as pairs of floats
  const size_t vp = c.g0.vpad;
  copy<float>(c, static_cast<cx<float>*>(dst.v), static_cast<const cx<float>*>(src.v), (size_t)nrhs * 6 * vp);
  copy<float>(c, reinterpret_cast<cx<float>*>(dst.s), reinterpret_cast<const cx<float>*>(src.s),
              (size_t)nrhs * vp / 2);
}

void hf_neg(Ctx& c, HF f, int nrhs) {
  const size_t n = (size_t)nrhs * 12 * c.g0.vpad;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_neg_h, dim3((unsigned)blocks), dim3(256), 0, c.stream, static_cast<uint32_t*>(f.v), n);
  WDMG_HIP(hipGetLastError());
}

template <typename H>
void hf_zero(Ctx& c, HF f, int nrhs) {
  hipLaunchKernelGGL((k_zero_h<H>), site_grid(c.g0, nrhs), dim3(256), 0, c.stream, c.g0,
                     static_cast<cxh<H>*>(f.v), f.s);
  WDMG_HIP(hipGetLastError());
}

template <typename R, typename H>
void to_half(Ctx& c, const cx<R>* in, HF out, int nrhs) {
  hipLaunchKernelGGL((k_to_half<R, H>), site_grid(c.g0, nrhs), dim3(256), 0, c.stream, c.g0, in,
                     static_cast<cxh<H>*>(out.v), out.s);
  WDMG_HIP(hipGetLastError());
}

template <typename H, typename R>
void from_half(Ctx& c, HF in, cx<R>* out, int nrhs) {
  hipLaunchKernelGGL((k_from_half<H, R>), site_grid(c.g0, nrhs), dim3(256), 0, c.stream, c.g0,
                     static_cast<const cxh<H>*>(in.v), in.s, out);
  WDMG_HIP(hipGetLastError());
}

template <typename H>
void canon_to_half(Ctx& c, const cx<float>* canon, HF out, int nrhs) {
  hipLaunchKernelGGL((k_canon_to_half<H>), site_grid(c.g0, nrhs), dim3(256), 0, c.stream, c.g0, canon,
                     static_cast<cxh<H>*>(out.v), out.s);
  WDMG_HIP(hipGetLastError());
}

template <typename H>
void half_to_canon(Ctx& c, HF in, cx<float>* canon, int nrhs) {
  hipLaunchKernelGGL((k_half_to_canon<H>), dim3((c.g0.vol + 255) / 256, nrhs), dim3(256), 0, c.stream, c.g0,
                     static_cast<const cxh<H>*>(in.v), in.s, canon);
  WDMG_HIP(hipGetLastError());
}

#define INST(H)                                                       \
  template void hf_zero<H>(Ctx&, HF, int);                            \
  template void to_half<double, H>(Ctx&, const cx<double>*, HF, int); \
  template void to_half<float, H>(Ctx&, const cx<float>*, HF, int);   \
  template void from_half<H, double>(Ctx&, HF, cx<double>*, int);     \
  template void from_half<H, float>(Ctx&, HF, cx<float>*, int);       \
  template void canon_to_half<H>(Ctx&, const cx<float>*, HF, int);    \
  template void half_to_canon<H>(Ctx&, HF, cx<float>*, int);
INST(f16_t)
INST(bf16_t)
#undef INST

}  // namespace wdmg
