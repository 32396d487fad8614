// Layout and precision conversion between the canonical ABI layouts and the
// internal tile-major, component-major layouts.
#include "internal.h"

namespace wdmg {

Geom make_geom(const int L[4], const int B[4]) {
  Geom g{};
  int lb_sum = 0;
  for (int mu = 0; mu < 4; ++mu) {
    g.L[mu] = L[mu];
    g.B[mu] = B[mu];
    int lb = 0;
    while ((1 << lb) < B[mu]) ++lb;
    g.lb[mu] = lb;
    g.nT[mu] = L[mu] / B[mu];
    lb_sum += lb;
  }
  g.tvol = B[0] * B[1] * B[2] * B[3];
  g.ltvol = lb_sum;
  g.vol = L[0] * L[1] * L[2] * L[3];
  g.sl[0] = 1;
  g.st[0] = g.tvol;
  for (int mu = 1; mu < 4; ++mu) {
    g.sl[mu] = g.sl[mu - 1] * B[mu - 1];
    g.st[mu] = g.st[mu - 1] * g.nT[mu - 1];
  }
  return g;
}

namespace {

__global__ void k_gauge_import(Geom g, const cx<double>* __restrict__ canon, cx<double>* __restrict__ U64,
                               cx<float>* __restrict__ U32, double tsign) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.vol) return;
  int c[4];
  coords_of(g, s, c);
  const size_t i = (size_t)c[0] + (size_t)g.L[0] * (c[1] + (size_t)g.L[1] * (c[2] + (size_t)g.L[2] * c[3]));
  const cx<double>* src = canon + i * 36;
  for (int mu = 0; mu < 4; ++mu) {
    const double sg = (mu == 3 && c[3] == g.L[3] - 1) ? tsign : 1.0;
    for (int e = 0; e < 9; ++e) {
      cx<double> u = src[mu * 9 + e];
      u.re *= sg;
      u.im *= sg;
      const size_t o = (size_t)(mu * 9 + e) * g.vol + s;
      U64[o] = u;
      U32[o] = cvt<float>(u);
    }
  }
}

template <typename Rio, typename R>
__global__ void k_fine_in(Geom g, const cx<Rio>* __restrict__ canon, cx<R>* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vol) return;
  int c[4];
  coords_of(g, s, c);
  const size_t i = (size_t)c[0] + (size_t)g.L[0] * (c[1] + (size_t)g.L[1] * (c[2] + (size_t)g.L[2] * c[3]));
  const cx<Rio>* src = canon + ((size_t)r * g.vol + i) * 12;
  cx<R>* dst = out + (size_t)r * 12 * g.vol + s;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[(size_t)k * g.vol] = cvt<R>(src[k]);
}

template <typename R, typename Rio>
__global__ void k_fine_out(Geom g, const cx<R>* __restrict__ in, cx<Rio>* __restrict__ canon) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vol) return;
  int c[4];
  coords_of(g, s, c);
  const size_t i = (size_t)c[0] + (size_t)g.L[0] * (c[1] + (size_t)g.L[1] * (c[2] + (size_t)g.L[2] * c[3]));
  cx<Rio>* dst = canon + ((size_t)r * g.vol + i) * 12;
  const cx<R>* src = in + (size_t)r * 12 * g.vol + s;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = cvt<Rio>(src[(size_t)k * g.vol]);
}

template <typename Rout, typename Rin>
__global__ void k_convert(cx<Rout>* __restrict__ out, const cx<Rin>* __restrict__ in, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = cvt<Rout>(in[i]);
}

}  // namespace

void gauge_import(Ctx& c, const cx<double>* canon, int t_bc) {
  const Geom& g = c.g0;
  dim3 grid((g.vol + 255) / 256);
  hipLaunchKernelGGL(k_gauge_import, grid, dim3(256), 0, c.stream, g, canon, c.U64, c.U32, (double)t_bc);
  WDMG_HIP(hipGetLastError());
}

template <typename Rio, typename R>
void fine_to_internal(Ctx& c, const Geom& g, const cx<Rio>* canon, cx<R>* out, int nrhs) {
  dim3 grid((g.vol + 255) / 256, nrhs);
  hipLaunchKernelGGL((k_fine_in<Rio, R>), grid, dim3(256), 0, c.stream, g, canon, out);
  WDMG_HIP(hipGetLastError());
}

template <typename R, typename Rio>
void fine_to_canonical(Ctx& c, const Geom& g, const cx<R>* in, cx<Rio>* canon, int nrhs) {
  dim3 grid((g.vol + 255) / 256, nrhs);
  hipLaunchKernelGGL((k_fine_out<R, Rio>), grid, dim3(256), 0, c.stream, g, in, canon);
  WDMG_HIP(hipGetLastError());
}

template <typename Rout, typename Rin>
void convert(Ctx& c, cx<Rout>* out, const cx<Rin>* in, size_t n) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_convert<Rout, Rin>), dim3((unsigned)blocks), dim3(256), 0, c.stream, out, in, n);
  WDMG_HIP(hipGetLastError());
}

template void fine_to_internal<double, double>(Ctx&, const Geom&, const cx<double>*, cx<double>*, int);
template void fine_to_internal<float, float>(Ctx&, const Geom&, const cx<float>*, cx<float>*, int);
template void fine_to_internal<double, float>(Ctx&, const Geom&, const cx<double>*, cx<float>*, int);
template void fine_to_canonical<double, double>(Ctx&, const Geom&, const cx<double>*, cx<double>*, int);
template void fine_to_canonical<float, float>(Ctx&, const Geom&, const cx<float>*, cx<float>*, int);
template void fine_to_canonical<float, double>(Ctx&, const Geom&, const cx<float>*, cx<double>*, int);
template void convert<float, double>(Ctx&, cx<float>*, const cx<double>*, size_t);
template void convert<double, float>(Ctx&, cx<double>*, const cx<float>*, size_t);
template void convert<double, double>(Ctx&, cx<double>*, const cx<double>*, size_t);
template void convert<float, float>(Ctx&, cx<float>*, const cx<float>*, size_t);

}  // namespace wdmg
