// Layout and precision conversion between the canonical ABI layouts and the
// internal tile-major, component-major layouts.
#include "fine_field.h"
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
  g.vpad = (g.vol + 63) / 64 * 64;
  g.sl[0] = 1;
  g.st[0] = g.tvol;
  for (int mu = 1; mu < 4; ++mu) {
    g.sl[mu] = g.sl[mu - 1] * B[mu - 1];
    g.st[mu] = g.st[mu - 1] * g.nT[mu - 1];
  }
  return g;
}

namespace {

// Canonical links -> first two rows of every link (FP64 and FP32) with the
// antiperiodic sign folded into U_t at t = Lt-1.  Also checks that each link
// is SU(3) to 1e-10: its third row must equal conj(row0 x row1).
__global__ void k_gauge_import(Geom g, const cx<double>* __restrict__ canon, cx<double>* __restrict__ U64,
                               cx<float>* __restrict__ U32, double tsign, double* flag) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.vpad) return;
  if (s >= g.vol) {
    for (int k = 0; k < kLinkComp; ++k) {
      U64[fidx(s, k, kLinkComp)] = mk(0.0, 0.0);
      U32[fidx(s, k, kLinkComp)] = mk(0.0f, 0.0f);
    }
    return;
  }
  int c[4];
  coords_of(g, s, c);
  const size_t i = (size_t)c[0] + (size_t)g.L[0] * (c[1] + (size_t)g.L[1] * (c[2] + (size_t)g.L[2] * c[3]));
  const cx<double>* src = canon + i * 36;
  double dev = 0.0;
  for (int mu = 0; mu < 4; ++mu) {
    const cx<double>* u = src + mu * 9;
    const cx<double> r[3] = {u[1] * u[5] - u[2] * u[4], u[2] * u[3] - u[0] * u[5], u[0] * u[4] - u[1] * u[3]};
    for (int a = 0; a < 3; ++a) {
      dev = fmax(dev, fabs(u[6 + a].re - r[a].re));
      dev = fmax(dev, fabs(u[6 + a].im + r[a].im));
    }
    const double sg = (mu == 3 && c[3] == g.L[3] - 1) ? tsign : 1.0;
    for (int e = 0; e < 6; ++e) {
      const cx<double> v = mk(sg * u[e].re, sg * u[e].im);
      U64[fidx(s, mu * 6 + e, kLinkComp)] = v;
      U32[fidx(s, mu * 6 + e, kLinkComp)] = cvt<float>(v);
    }
  }
  if (!(dev <= 1e-10)) flag[0] = 1.0;
}

template <typename Rio, typename R>
__global__ void k_fine_in(Geom g, const cx<Rio>* __restrict__ canon, cx<R>* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vpad) return;
  cx<R>* dst = out + (size_t)r * 12 * g.vpad;
  if (s >= g.vol) {
#pragma unroll
    for (int k = 0; k < 12; ++k) dst[fidx(s, k, 12)] = mk<R>(0, 0);
    return;
  }
  int c[4];
  coords_of(g, s, c);
  const size_t i = (size_t)c[0] + (size_t)g.L[0] * (c[1] + (size_t)g.L[1] * (c[2] + (size_t)g.L[2] * c[3]));
  const cx<Rio>* src = canon + ((size_t)r * g.vol + i) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[fidx(s, k, 12)] = cvt<R>(src[k]);
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
  const cx<R>* src = in + (size_t)r * 12 * g.vpad;
#pragma unroll
  for (int k = 0; k < 12; ++k) dst[k] = cvt<Rio>(src[fidx(s, k, 12)]);
}

template <typename Rout, typename Rin>
__global__ void k_convert(cx<Rout>* __restrict__ out, const cx<Rin>* __restrict__ in, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = cvt<Rout>(in[i]);
}

}  // namespace

void gauge_import(Ctx& c, const cx<double>* canon, int t_bc) {
  const Geom& g = c.g0;
  dim3 grid((g.vpad + 255) / 256);
  hipLaunchKernelGGL(k_gauge_import, grid, dim3(256), 0, c.stream, g, canon, c.U64, c.U32, (double)t_bc,
                     c.dsc + S_ERR + 2);
  WDMG_HIP(hipGetLastError());
}

template <typename Rio, typename R>
void fine_to_internal(Ctx& c, const Geom& g, const cx<Rio>* canon, cx<R>* out, int nrhs) {
  dim3 grid((g.vpad + 255) / 256, nrhs);
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
