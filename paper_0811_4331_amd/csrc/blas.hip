// Vector kernels of the smoother and Krylov solvers: fused updates and
// reductions whose results stay in device memory.
//
// Reductions are single launches: each workgroup writes its partial sums,
// the last workgroup to finish (atomic ticket) adds the partials in a fixed
// order and applies a finalising formula (an MR step size, a GCR
// coefficient, ...) straight into the device scalar area.  The summation
// order depends only on the vector length, so results are bitwise
// reproducible run to run.
#include "half_field.h"
#include "internal.h"

namespace wdmg {
namespace {

constexpr int TPB = kReduceThreads;

inline unsigned reduce_blocks(size_t n) {
  size_t b = (n + (size_t)TPB * 4 - 1) / ((size_t)TPB * 4);
  if (b < 1) b = 1;
  if (b > (size_t)kMaxReduceBlocks) b = kMaxReduceBlocks;
  return (unsigned)b;
}

__device__ __forceinline__ bool bad(double x) { return !isfinite(x); }


// Reductions: each workgroup writes its partial sums; a second one-workgroup
// launch adds them in a fixed order and applies the finalising formula.  A
// vector small enough for one workgroup is reduced and finalised in a
// single launch.  (A last-workgroup ticket with device-scope fences was
// measured slower than the second launch once more than a few dozen
// workgroups take part.)
constexpr size_t kSingleBlockMax = 32768;
constexpr int TPB1 = 1024;

template <class Op>
__global__ __launch_bounds__(TPB) void k_reduce_part(Op op, size_t n, double* partials) {
  constexpr int K = Op::K;
  __shared__ double lds[K * (TPB / 64)];
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB) op.acc(i, v);
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) partials[blockIdx.x * K + k] = v[k];
  }
}

template <class Op>
__global__ __launch_bounds__(TPB) void k_reduce_fin(Op op, int nb, const double* partials) {
  constexpr int K = Op::K;
  __shared__ double lds[K * (TPB / 64)];
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += TPB) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += partials[b * K + k];
  }
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) op.fin(v);
}

template <class Op>
__global__ __launch_bounds__(TPB1) void k_reduce_one(Op op, size_t n) {
  constexpr int K = Op::K;
  __shared__ double lds[K * (TPB1 / 64)];
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (size_t i = threadIdx.x; i < n; i += TPB1) op.acc(i, v);
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) op.fin(v);
}

// Batched form: blockIdx.y selects one of several independent vectors.
template <class Op>
__global__ __launch_bounds__(TPB) void k_reduce_b_part(Op op, size_t n, double* partials) {
  constexpr int K = Op::K;
  __shared__ double lds[K * (TPB / 64)];
  const int y = blockIdx.y;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (size_t i = blockIdx.x * (size_t)TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * TPB) op.acc(i, y, v);
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) partials[((size_t)y * gridDim.x + blockIdx.x) * K + k] = v[k];
  }
}

template <class Op>
__global__ __launch_bounds__(TPB) void k_reduce_b_fin(Op op, int nb, const double* partials) {
  constexpr int K = Op::K;
  __shared__ double lds[K * (TPB / 64)];
  const int y = blockIdx.x;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += TPB) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += partials[((size_t)y * nb + b) * K + k];
  }
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) op.fin(v, y);
}

template <class Op>
void run_reduce(Ctx& c, const Op& op, size_t n) {
  if (n <= kSingleBlockMax) {
    hipLaunchKernelGGL((k_reduce_one<Op>), dim3(1), dim3(TPB1), 0, c.stream, op, n);
    WDMG_HIP(hipGetLastError());
    return;
  }
  const unsigned nb = reduce_blocks(n);
  hipLaunchKernelGGL((k_reduce_part<Op>), dim3(nb), dim3(TPB), 0, c.stream, op, n, c.partials);
  WDMG_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_reduce_fin<Op>), dim3(1), dim3(TPB), 0, c.stream, op, (int)nb, c.partials);
  WDMG_HIP(hipGetLastError());
}

// ---- ops ------------------------------------------------------------------
template <typename R>
struct StepAlphaOp {
  static constexpr int K = 3;
  const cx<R>* a;
  const cx<R>* b;
  double scale;
  double* dsc;
  int slot;
  __device__ void acc(size_t i, double* v) const {
    const cx<R> x = a[i], y = b[i];
    v[0] += (double)x.re * y.re + (double)x.im * y.im;
    v[1] += (double)x.re * y.im - (double)x.im * y.re;
    v[2] += (double)x.re * x.re + (double)x.im * x.im;
  }
  __device__ void fin(const double* v) const {
    double re = 0.0, im = 0.0;
    if (v[2] > 0.0) {
      re = scale * v[0] / v[2];
      im = scale * v[1] / v[2];
    }
    if (bad(v[0]) || bad(v[1]) || bad(v[2])) dsc[S_ERR] = 1.0;
    dsc[slot] = re;
    dsc[slot + 1] = im;
  }
};

template <typename R>
struct Norm2Op {
  static constexpr int K = 1;
  const cx<R>* a;
  double* dsc;
  int slot;
  __device__ void acc(size_t i, double* v) const {
    const cx<R> x = a[i];
    v[0] += (double)x.re * x.re + (double)x.im * x.im;
  }
  __device__ void fin(const double* v) const {
    if (bad(v[0])) dsc[S_ERR] = 1.0;
    dsc[slot] = v[0];
  }
};

template <typename R>
struct DotOp {
  static constexpr int K = 2;
  const cx<R>* a;
  const cx<R>* b;
  double* dsc;
  int slot;
  __device__ void acc(size_t i, double* v) const {
    const cx<R> x = a[i], y = b[i];
    v[0] += (double)x.re * y.re + (double)x.im * y.im;
    v[1] += (double)x.re * y.im - (double)x.im * y.re;
  }
  __device__ void fin(const double* v) const {
    dsc[slot] = v[0];
    dsc[slot + 1] = v[1];
  }
};

// Batched MR step sizes for nb vectors a_q, b_q (stride apart).
template <typename R>
struct StepAlphaBatchOp {
  static constexpr int K = 3;
  const cx<R>* a;
  const cx<R>* b;
  size_t stride;
  double scale;
  double* dsc;
  int slot;
  __device__ void acc(size_t i, int y, double* v) const {
    const cx<R> x = a[y * stride + i], z = b[y * stride + i];
    v[0] += (double)x.re * z.re + (double)x.im * z.im;
    v[1] += (double)x.re * z.im - (double)x.im * z.re;
    v[2] += (double)x.re * x.re + (double)x.im * x.im;
  }
  __device__ void fin(const double* v, int y) const {
    double re = 0.0, im = 0.0;
    if (v[2] > 0.0) {
      re = scale * v[0] / v[2];
      im = scale * v[1] / v[2];
    }
    if (bad(v[0]) || bad(v[1]) || bad(v[2])) dsc[S_ERR] = 1.0;
    dsc[slot + 2 * y] = re;
    dsc[slot + 2 * y + 1] = im;
  }
};

// Batched MR step sizes on 16-bit fields; i runs over sites.
template <typename H>
struct StepAlphaHalfOp {
  static constexpr int K = 3;
  const cxh<H>* a;
  const float* as;
  const cxh<H>* b;
  const float* bs;
  int vpad;
  double scale;
  double* dsc;
  int slot;
  __device__ void acc(size_t i, int y, double* v) const {
    const size_t vo = (size_t)y * 12 * vpad, so = (size_t)y * vpad;
    cx<float> x[12], z[12];
    load_site_h(a + vo, as + so, (int)i, x);
    load_site_h(b + vo, bs + so, (int)i, z);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      v[0] += (double)x[k].re * z[k].re + (double)x[k].im * z[k].im;
      v[1] += (double)x[k].re * z[k].im - (double)x[k].im * z[k].re;
      v[2] += (double)x[k].re * x[k].re + (double)x[k].im * x[k].im;
    }
  }
  __device__ void fin(const double* v, int y) const {
    double re = 0.0, im = 0.0;
    if (v[2] > 0.0) {
      re = scale * v[0] / v[2];
      im = scale * v[1] / v[2];
    }
    if (bad(v[0]) || bad(v[1]) || bad(v[2])) dsc[S_ERR] = 1.0;
    dsc[slot + 2 * y] = re;
    dsc[slot + 2 * y + 1] = im;
  }
};

struct XmyNormOp {
  static constexpr int K = 1;
  const cx<double>* b;
  cx<double>* y;
  double* dsc;
  int slot;
  __device__ void acc(size_t i, double* v) const {
    const cx<double> d = b[i] - y[i];
    y[i] = d;
    v[0] += d.re * d.re + d.im * d.im;
  }
  __device__ void fin(const double* v) const {
    if (bad(v[0])) dsc[S_ERR] = 1.0;
    dsc[slot] = v[0];
  }
};

// ---- BiCGStab (slots relative to S_BICG) ----------------------------------
enum { B_RHO_NEW = 0, B_RHO_OLD = 2, B_ALPHA = 4, B_OMEGA = 6, B_RNORM = 8 };

__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
  const double d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}

struct BicgAlphaOp {  // alpha = rho_new / <rhat, v>
  static constexpr int K = 2;
  const cx<double>* rhat;
  const cx<double>* v_;
  double* dsc;
  __device__ void acc(size_t i, double* v) const {
    const cx<double> x = rhat[i], y = v_[i];
    v[0] += x.re * y.re + x.im * y.im;
    v[1] += x.re * y.im - x.im * y.re;
  }
  __device__ void fin(const double* v) const {
    double* b = dsc + S_BICG;
    const cx<double> rn = mk(b[B_RHO_NEW], b[B_RHO_NEW + 1]);
    cx<double> a = mk(0.0, 0.0);
    if (v[0] != 0.0 || v[1] != 0.0) a = cdiv(rn, mk(v[0], v[1]));
    if (bad(a.re) || bad(a.im)) dsc[S_ERR] = 1.0;
    b[B_ALPHA] = a.re;
    b[B_ALPHA + 1] = a.im;
    b[B_RHO_OLD] = rn.re;
    b[B_RHO_OLD + 1] = rn.im;
  }
};

struct BicgOmegaOp {  // omega = <t, s> / <t, t>
  static constexpr int K = 3;
  const cx<double>* t;
  const cx<double>* s;
  double* dsc;
  __device__ void acc(size_t i, double* v) const {
    const cx<double> x = t[i], y = s[i];
    v[0] += x.re * y.re + x.im * y.im;
    v[1] += x.re * y.im - x.im * y.re;
    v[2] += x.re * x.re + x.im * x.im;
  }
  __device__ void fin(const double* v) const {
    double* b = dsc + S_BICG;
    b[B_OMEGA] = v[2] > 0.0 ? v[0] / v[2] : 0.0;
    b[B_OMEGA + 1] = v[2] > 0.0 ? v[1] / v[2] : 0.0;
    if (bad(v[0]) || bad(v[2])) dsc[S_ERR] = 1.0;
  }
};

// x += alpha p + omega sx ; r = s - omega t ; rho_new = <rhat, r>, ||r||^2
// (sx = s, or M s with a right preconditioner M, when p is M p too)
struct BicgXrOp {
  static constexpr int K = 3;
  cx<double>* x;
  cx<double>* r;
  const cx<double>* p;
  const cx<double>* s;
  const cx<double>* sx;
  const cx<double>* t;
  const cx<double>* rhat;
  double* dsc;
  __device__ void acc(size_t i, double* v) const {
    const double* b = dsc + S_BICG;
    const cx<double> al = mk(b[B_ALPHA], b[B_ALPHA + 1]), om = mk(b[B_OMEGA], b[B_OMEGA + 1]);
    const cx<double> si = s[i];
    x[i] = x[i] + al * p[i] + om * sx[i];
    const cx<double> ri = si - om * t[i];
    r[i] = ri;
    const cx<double> h = rhat[i];
    v[0] += h.re * ri.re + h.im * ri.im;
    v[1] += h.re * ri.im - h.im * ri.re;
    v[2] += ri.re * ri.re + ri.im * ri.im;
  }
  __device__ void fin(const double* v) const {
    double* b = dsc + S_BICG;
    b[B_RHO_NEW] = v[0];
    b[B_RHO_NEW + 1] = v[1];
    b[B_RNORM] = v[2];
    if (bad(v[2])) dsc[S_ERR] = 1.0;
  }
};

// ---- elementwise kernels ---------------------------------------------------
template <typename R>
__global__ void k_zero(cx<R>* x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = mk<R>(0, 0);
}

template <typename R>
__global__ void k_copy(cx<R>* __restrict__ y, const cx<R>* __restrict__ x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

template <typename R>
__global__ void k_neg(cx<R>* x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = mk<R>(-x[i].re, -x[i].im);
}

template <typename R>
__global__ void k_xmy(const cx<R>* __restrict__ b, cx<R>* __restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = b[i] - y[i];
}

template <typename R>
__global__ void k_add(cx<R>* __restrict__ y, const cx<R>* __restrict__ x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = y[i] + x[i];
}

// MODE 0: x += s u ; r -= s v.  MODE 1 (first MR step from x = 0 with
// residual u): x = s u ; r = u - s v.  MODE 2 (last MR step): x += s u only.
template <typename R, int MODE>
__global__ void k_update2_batch(cx<R>* x, const cx<R>* u, cx<R>* r, const cx<R>* v, size_t n, size_t stride,
                                const double* s) {
  const int y = blockIdx.y;
  const cx<R> a = mk<R>((R)s[2 * y], (R)s[2 * y + 1]);
  x += y * stride;
  u += y * stride;
  r += y * stride;
  v += y * stride;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const cx<R> ui = u[i];
    if constexpr (MODE == 1) {
      x[i] = a * ui;
      r[i] = ui - a * v[i];
    } else {
      x[i] = x[i] + a * ui;
      if constexpr (MODE == 0) r[i] = r[i] - a * v[i];
    }
  }
}

template <typename R>
__global__ void k_update2(cx<R>* x, const cx<R>* u, cx<R>* r, const cx<R>* v, size_t n, const double* s) {
  const cx<R> a = mk<R>((R)s[0], (R)s[1]);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const cx<R> ui = u[i], vi = v[i];
    x[i] = x[i] + a * ui;
    r[i] = r[i] - a * vi;
  }
}

// x += s u ; r -= s v on 16-bit fields (one thread per site and rhs); u may
// be the same field as r, so nothing here is declared non-aliasing.
// MODE 0: as written.  MODE 1 (first MR step of a cycle from x = 0 with
// residual u): x = s u and r = u - s v, x not read.  MODE 2 (last MR step,
// whose residual nobody reads): x += s u only.
template <typename H, int MODE>
__global__ void k_update2_half(Geom g, cxh<H>* xv, float* xs, const cxh<H>* uv, const float* us, cxh<H>* rv,
                               float* rs, const cxh<H>* vv, const float* vs, const double* sc) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (s >= g.vpad) return;
  const size_t vo = (size_t)y * 12 * g.vpad, so = (size_t)y * g.vpad;
  const cx<float> a = mk((float)sc[2 * y], (float)sc[2 * y + 1]);
  cx<float> x[12], u[12];
  load_site_h(uv + vo, us + so, s, u);
  if constexpr (MODE == 1) {
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = a * u[k];
  } else {
    load_site_h(xv + vo, xs + so, s, x);
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = x[k] + a * u[k];
  }
  store_site_h(xv + vo, xs + so, s, x);
  if constexpr (MODE != 2) {
    cx<float> r[12], v[12];
    if constexpr (MODE == 1) {
#pragma unroll
      for (int k = 0; k < 12; ++k) r[k] = u[k];
    } else {
      load_site_h(rv + vo, rs + so, s, r);
    }
    load_site_h(vv + vo, vs + so, s, v);
#pragma unroll
    for (int k = 0; k < 12; ++k) r[k] = r[k] - a * v[k];
    store_site_h(rv + vo, rs + so, s, r);
  }
}

__global__ void k_bicg_p(cx<double>* p, const cx<double>* r, const cx<double>* v, size_t n, const double* dsc,
                         int first) {
  const double* b = dsc + S_BICG;
  cx<double> beta = mk(0.0, 0.0), om = mk(b[B_OMEGA], b[B_OMEGA + 1]);
  if (!first) {
    const cx<double> rn = mk(b[B_RHO_NEW], b[B_RHO_NEW + 1]), ro = mk(b[B_RHO_OLD], b[B_RHO_OLD + 1]);
    const cx<double> al = mk(b[B_ALPHA], b[B_ALPHA + 1]);
    beta = cdiv(rn, ro) * cdiv(al, om);
  }
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    if (first)
      p[i] = r[i];
    else
      p[i] = r[i] + beta * (p[i] - om * v[i]);
  }
}

__global__ void k_bicg_s(cx<double>* s, const cx<double>* r, const cx<double>* v, size_t n, const double* dsc) {
  const double* b = dsc + S_BICG;
  const cx<double> al = mk(b[B_ALPHA], b[B_ALPHA + 1]);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s[i] = r[i] - al * v[i];
}

// GCR orthogonalisation: partial dot products <W_i, w> for up to 8 basis
// vectors per workgroup row (blockIdx.y), then one workgroup finalises all
// coefficients h_i = <W_i, w> / nrm_i.
constexpr int GCR_G = 8;
__global__ void k_fill_pairs(double* dsc, int slot, int count, double re, double im) {
  const int i = threadIdx.x;
  if (i < count) {
    dsc[slot + 2 * i] = re;
    dsc[slot + 2 * i + 1] = im;
  }
}

__global__ void k_set_scalar(double* dsc, int slot, double re, double im) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dsc[slot] = re;
    dsc[slot + 1] = im;
  }
}

inline unsigned ew_blocks(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

template <typename R>
void zero(Ctx& c, cx<R>* x, size_t n) {
  hipLaunchKernelGGL((k_zero<R>), dim3(ew_blocks(n)), dim3(256), 0, c.stream, x, n);
  WDMG_HIP(hipGetLastError());
}
template <typename R>
void copy(Ctx& c, cx<R>* y, const cx<R>* x, size_t n) {
  hipLaunchKernelGGL((k_copy<R>), dim3(ew_blocks(n)), dim3(256), 0, c.stream, y, x, n);
  WDMG_HIP(hipGetLastError());
}
template <typename R>
void neg(Ctx& c, cx<R>* x, size_t n) {
  hipLaunchKernelGGL((k_neg<R>), dim3(ew_blocks(n)), dim3(256), 0, c.stream, x, n);
  WDMG_HIP(hipGetLastError());
}
template <typename R>
void xmy(Ctx& c, const cx<R>* b, cx<R>* y, size_t n) {
  hipLaunchKernelGGL((k_xmy<R>), dim3(ew_blocks(n)), dim3(256), 0, c.stream, b, y, n);
  WDMG_HIP(hipGetLastError());
}
template <typename R>
void add(Ctx& c, cx<R>* y, const cx<R>* x, size_t n) {
  hipLaunchKernelGGL((k_add<R>), dim3(ew_blocks(n)), dim3(256), 0, c.stream, y, x, n);
  WDMG_HIP(hipGetLastError());
}
template <typename R>
void step_alpha(Ctx& c, const cx<R>* a, const cx<R>* b, size_t n, double scale, int slot) {
  run_reduce(c, StepAlphaOp<R>{a, b, scale, c.dsc, slot}, n);
}
template <typename R>
void update2(Ctx& c, cx<R>* x, const cx<R>* u, cx<R>* r, const cx<R>* v, size_t n, int slot) {
  hipLaunchKernelGGL((k_update2<R>), dim3(ew_blocks(n)), dim3(256), 0, c.stream, x, u, r, v, n, c.dsc + slot);
  WDMG_HIP(hipGetLastError());
}
template <typename R>
void norm2(Ctx& c, const cx<R>* a, size_t n, int slot) {
  run_reduce(c, Norm2Op<R>{a, c.dsc, slot}, n);
}
template <typename R>
void dot(Ctx& c, const cx<R>* a, const cx<R>* b, size_t n, int slot) {
  run_reduce(c, DotOp<R>{a, b, c.dsc, slot}, n);
}

// ---- batched GCR ------------------------------------------------------------
// B: storage type of the basis and of w (double, or float for a reduced-
// precision outer basis); sums are formed in double.
template <typename B>
__global__ __launch_bounds__(TPB) void k_gcr_dots_b(const cx<B>* __restrict__ W, const cx<B>* __restrict__ w,
                                                    size_t n, int nb, int j, int gx, int gy, double* partials) {
  __shared__ double lds[2 * GCR_G * (TPB / 64)];
  const int rhs = blockIdx.z;
  const int i0 = blockIdx.y * GCR_G;
  const int ni = min(GCR_G, j - i0);
  const cx<B>* wr = w + (size_t)rhs * n;
  double v[2 * GCR_G];
#pragma unroll
  for (int k = 0; k < 2 * GCR_G; ++k) v[k] = 0.0;
  for (size_t e = blockIdx.x * (size_t)TPB + threadIdx.x; e < n; e += (size_t)gridDim.x * TPB) {
    const cx<double> y = cvt<double>(wr[e]);
#pragma unroll
    for (int q = 0; q < GCR_G; ++q) {
      if (q < ni) {
        const cx<double> x = cvt<double>(W[((size_t)(i0 + q) * nb + rhs) * n + e]);
        v[2 * q] += x.re * y.re + x.im * y.im;
        v[2 * q + 1] += x.re * y.im - x.im * y.re;
      }
    }
  }
  block_sum<2 * GCR_G>(v, lds);
  if (threadIdx.x == 0) {
    const size_t myblk = ((size_t)rhs * gy + blockIdx.y) * gx + blockIdx.x;
#pragma unroll
    for (int k = 0; k < 2 * GCR_G; ++k) partials[myblk * 2 * GCR_G + k] = v[k];
  }
}

// One wave per coefficient: lanes add the workgroup partials in a strided
// order, then a fixed shuffle tree (deterministic).
__global__ __launch_bounds__(TPB) void k_gcr_dots_b_fin(int j, int gx, int gy, const double* partials, double* g) {
  const int rhs = blockIdx.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = TPB / 64;
  // blockIdx.y selects nw coefficients, one per wave
  for (int t = blockIdx.y * nw + wave; t < 2 * j; t += nw * gridDim.y) {
    const int i = t >> 1, part = t & 1;
    const int yy = i / GCR_G, q = i % GCR_G;
    double s = 0.0;
    for (int bx = lane; bx < gx; bx += 64) s += partials[(((size_t)rhs * gy + yy) * gx + bx) * 2 * GCR_G + 2 * q + part];
    s = wave_sum(s);
    if (lane == 0) {
      const double nrm = g[G_NRM + rhs * kMaxKrylov + i];
      g[G_H + rhs * 2 * kMaxKrylov + t] = nrm > 0.0 ? s / nrm : 0.0;
    }
  }
}

// w -= sum h_i W_i in double, stored as B; |w|^2 and <w, r> of the stored w.
// (The matching combination of the search directions z is deferred to the
// end of the cycle: see k_gcr_combine.)
template <typename B>
struct GcrAxpyCoefBOp {
  static constexpr int K = 3;
  const cx<B>* W;
  cx<B>* w;
  const cx<double>* r;
  double* g;
  double* dsc;
  size_t n;
  int nb, j;
  __device__ void acc(size_t e, int rhs, double* v) const {
    const size_t o = (size_t)rhs * n + e;
    cx<double> a = cvt<double>(w[o]);
    const double* h = g + G_H + rhs * 2 * kMaxKrylov;
    for (int i = 0; i < j; ++i) {
      const cx<double> hi = mk(h[2 * i], h[2 * i + 1]);
      a = a - hi * cvt<double>(W[((size_t)i * nb + rhs) * n + e]);
    }
    if (j > 0) {
      const cx<B> as = cvt<B>(a);
      w[o] = as;
      a = cvt<double>(as);
    }
    const cx<double> y = r[o];
    v[0] += a.re * a.re + a.im * a.im;
    v[1] += a.re * y.re + a.im * y.im;
    v[2] += a.re * y.im - a.im * y.re;
  }
  __device__ void fin(const double* v, int rhs) const {
    if (bad(v[0]) || bad(v[1]) || bad(v[2])) dsc[S_ERR] = 1.0;
    g[G_NRM + rhs * kMaxKrylov + j] = v[0];
    const bool on = g[G_ACT + rhs] != 0.0 && v[0] > 0.0;
    g[G_A + 2 * rhs] = on ? v[1] / v[0] : 0.0;
    g[G_A + 2 * rhs + 1] = on ? v[2] / v[0] : 0.0;
  }
};

// r -= a w per rhs, rnorm^2 per rhs.
template <typename B>
struct GcrUpdateBOp {
  static constexpr int K = 1;
  const cx<B>* w;
  cx<double>* r;
  double* g;
  double* dsc;
  double* host;
  size_t n;
  __device__ void acc(size_t e, int rhs, double* v) const {
    const size_t o = (size_t)rhs * n + e;
    const cx<double> s = mk(g[G_A + 2 * rhs], g[G_A + 2 * rhs + 1]);
    const cx<double> ri = r[o] - s * cvt<double>(w[o]);
    r[o] = ri;
    v[0] += ri.re * ri.re + ri.im * ri.im;
  }
  __device__ void fin(const double* v, int rhs) const {
    if (bad(v[0])) dsc[S_ERR] = 1.0;
    g[G_RN + rhs] = v[0];
    if (host) host[rhs] = v[0];
  }
};

// Records iteration j of every rhs: hist[q][i][j] = h_i (i < j), av[q][j] = a.
__global__ void k_gcr_record(const double* __restrict__ g, cx<double>* __restrict__ hist, cx<double>* __restrict__ av,
                             int nb, int j, int k) {
  const int q = blockIdx.x;
  if (q >= nb) return;
  for (int i = threadIdx.x; i < j; i += blockDim.x)
    hist[((size_t)q * k + i) * k + j] = mk(g[G_H + q * 2 * kMaxKrylov + 2 * i], g[G_H + q * 2 * kMaxKrylov + 2 * i + 1]);
  if (threadIdx.x == 0) av[(size_t)q * k + j] = mk(g[G_A + 2 * q], g[G_A + 2 * q + 1]);
}

// Coefficients of the unorthogonalised directions: with z_j = zt_j -
// sum_{i<j} h_ij z_i, sum_j a_j z_j = sum_j y_j zt_j where
// y_j = a_j - sum_{m>j} h_jm y_m (one thread per rhs).
__global__ void k_gcr_backsolve(const cx<double>* __restrict__ hist, const cx<double>* __restrict__ av,
                                cx<double>* __restrict__ y, int nb, int jn, int k) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nb) return;
  const cx<double>* hq = hist + (size_t)q * k * k;
  cx<double>* yq = y + (size_t)q * k;
  for (int jj = jn - 1; jj >= 0; --jj) {
    cx<double> t = av[(size_t)q * k + jj];
    for (int m = jj + 1; m < jn; ++m) t = t - hq[(size_t)jj * k + m] * yq[m];
    yq[jj] = t;
  }
}

// x += sum_{i < jn} y_i Zt_i per rhs.
template <typename B>
__global__ __launch_bounds__(256) void k_gcr_combine(cx<double>* __restrict__ x, const cx<B>* __restrict__ Z,
                                                     const cx<double>* __restrict__ y, size_t n, int nb, int jn,
                                                     int k) {
  const int q = blockIdx.y;
  __shared__ cx<double> ys[kMaxKrylov];
  for (int i = threadIdx.x; i < jn; i += blockDim.x) ys[i] = y[(size_t)q * k + i];
  __syncthreads();
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    cx<double> a = x[(size_t)q * n + e];
    for (int i = 0; i < jn; ++i) a = a + ys[i] * cvt<double>(Z[((size_t)i * nb + q) * n + e]);
    x[(size_t)q * n + e] = a;
  }
}

struct Norm2BOp {
  static constexpr int K = 1;
  const cx<double>* a;
  double* g;
  double* dsc;
  double* host;
  size_t n;
  __device__ void acc(size_t e, int rhs, double* v) const {
    const cx<double> x = a[(size_t)rhs * n + e];
    v[0] += x.re * x.re + x.im * x.im;
  }
  __device__ void fin(const double* v, int rhs) const {
    if (bad(v[0])) dsc[S_ERR] = 1.0;
    g[G_RN + rhs] = v[0];
    if (host) host[rhs] = v[0];
  }
};

struct XmyNormBOp {
  static constexpr int K = 1;
  const cx<double>* b;
  cx<double>* y;
  double* g;
  double* dsc;
  size_t n;
  __device__ void acc(size_t e, int rhs, double* v) const {
    const size_t o = (size_t)rhs * n + e;
    const cx<double> d = b[o] - y[o];
    y[o] = d;
    v[0] += d.re * d.re + d.im * d.im;
  }
  __device__ void fin(const double* v, int rhs) const {
    if (bad(v[0])) dsc[S_ERR] = 1.0;
    g[G_RN + rhs] = v[0];
  }
};

template <class Op>
__global__ __launch_bounds__(TPB1) void k_reduce_b_one(Op op, size_t n) {
  constexpr int K = Op::K;
  __shared__ double lds[K * (TPB1 / 64)];
  const int y = blockIdx.x;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (size_t i = threadIdx.x; i < n; i += TPB1) op.acc(i, y, v);
  block_sum<K>(v, lds);
  if (threadIdx.x == 0) op.fin(v, y);
}

template <class Op>
void run_reduce_b(Ctx& c, const Op& op, size_t n, int nb) {
  if (n <= kSingleBlockMax / 4) {
    // one workgroup per right-hand side, no second launch
    hipLaunchKernelGGL((k_reduce_b_one<Op>), dim3(nb), dim3(TPB1), 0, c.stream, op, n);
    WDMG_HIP(hipGetLastError());
    return;
  }
  unsigned nblk = reduce_blocks(n);
  if (nblk * nb > 8192) nblk = 8192 / nb;
  if (nblk < 1) nblk = 1;
  hipLaunchKernelGGL((k_reduce_b_part<Op>), dim3(nblk, nb), dim3(TPB), 0, c.stream, op, n, c.partials);
  WDMG_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_reduce_b_fin<Op>), dim3(nb), dim3(TPB), 0, c.stream, op, (int)nblk, c.partials);
  WDMG_HIP(hipGetLastError());
}

__global__ void k_set_active(double* g, const double* flags, int nb) {
  const int i = threadIdx.x;
  if (i < nb) g[G_ACT + i] = flags[i];
}

template <typename R>
void step_alpha_batch(Ctx& c, const cx<R>* a, const cx<R>* b, size_t n, size_t stride, int nb, double scale,
                      int slot) {
  unsigned nblk = reduce_blocks(n);
  if (nblk * nb > 8192) nblk = 8192 / nb;
  if (nblk < 1) nblk = 1;
  const StepAlphaBatchOp<R> op{a, b, stride, scale, c.dsc, slot};
  hipLaunchKernelGGL((k_reduce_b_part<StepAlphaBatchOp<R>>), dim3(nblk, nb), dim3(TPB), 0, c.stream, op, n,
                     c.partials);
  WDMG_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_reduce_b_fin<StepAlphaBatchOp<R>>), dim3(nb), dim3(TPB), 0, c.stream, op, (int)nblk,
                     c.partials);
  WDMG_HIP(hipGetLastError());
}
template <typename R>
void update2_batch(Ctx& c, cx<R>* x, const cx<R>* u, cx<R>* r, const cx<R>* v, size_t n, size_t stride, int nb,
                   int slot, int mode) {
  unsigned gx = ew_blocks(n);
  if (gx * nb > 8192) gx = (8192 + nb - 1) / nb;
  if (mode == 1)
    hipLaunchKernelGGL((k_update2_batch<R, 1>), dim3(gx, nb), dim3(256), 0, c.stream, x, u, r, v, n, stride,
                       c.dsc + slot);
  else if (mode == 2)
    hipLaunchKernelGGL((k_update2_batch<R, 2>), dim3(gx, nb), dim3(256), 0, c.stream, x, u, r, v, n, stride,
                       c.dsc + slot);
  else
    hipLaunchKernelGGL((k_update2_batch<R, 0>), dim3(gx, nb), dim3(256), 0, c.stream, x, u, r, v, n, stride,
                       c.dsc + slot);
  WDMG_HIP(hipGetLastError());
}

void step_alpha_fin(Ctx& c, const double* parts, int nparts, int nrhs, double scale, int slot) {
  const StepAlphaBatchOp<double> op{nullptr, nullptr, 0, scale, c.dsc, slot};
  hipLaunchKernelGGL((k_reduce_b_fin<StepAlphaBatchOp<double>>), dim3(nrhs), dim3(TPB), 0, c.stream, op, nparts,
                     parts);
  WDMG_HIP(hipGetLastError());
}

template <typename H>
void step_alpha_half(Ctx& c, HF a, HF b, int nrhs, double scale, int slot) {
  const size_t n = c.g0.vol;
  unsigned nblk = reduce_blocks(n);
  if (nblk * nrhs > 8192) nblk = 8192 / nrhs;
  if (nblk < 1) nblk = 1;
  const StepAlphaHalfOp<H> op{static_cast<const cxh<H>*>(a.v), a.s, static_cast<const cxh<H>*>(b.v), b.s,
                              c.g0.vpad, scale, c.dsc, slot};
  hipLaunchKernelGGL((k_reduce_b_part<StepAlphaHalfOp<H>>), dim3(nblk, nrhs), dim3(TPB), 0, c.stream, op, n,
                     c.partials);
  WDMG_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_reduce_b_fin<StepAlphaHalfOp<H>>), dim3(nrhs), dim3(TPB), 0, c.stream, op, (int)nblk,
                     c.partials);
  WDMG_HIP(hipGetLastError());
}

template <typename H>
void update2_half(Ctx& c, HF x, HF u, HF r, HF v, int nrhs, int slot, int mode) {
  const dim3 grid((c.g0.vpad + 255) / 256, nrhs);
  auto* xv = static_cast<cxh<H>*>(x.v);
  auto* uv = static_cast<const cxh<H>*>(u.v);
  auto* rv = static_cast<cxh<H>*>(r.v);
  auto* vv = static_cast<const cxh<H>*>(v.v);
  if (mode == 1)
    hipLaunchKernelGGL((k_update2_half<H, 1>), grid, dim3(256), 0, c.stream, c.g0, xv, x.s, uv, u.s, rv, r.s, vv, v.s,
                       c.dsc + slot);
  else if (mode == 2)
    hipLaunchKernelGGL((k_update2_half<H, 2>), grid, dim3(256), 0, c.stream, c.g0, xv, x.s, uv, u.s, rv, r.s, vv, v.s,
                       c.dsc + slot);
  else
    hipLaunchKernelGGL((k_update2_half<H, 0>), grid, dim3(256), 0, c.stream, c.g0, xv, x.s, uv, u.s, rv, r.s, vv, v.s,
                       c.dsc + slot);
  WDMG_HIP(hipGetLastError());
}

template void step_alpha_half<f16_t>(Ctx&, HF, HF, int, double, int);
template void step_alpha_half<bf16_t>(Ctx&, HF, HF, int, double, int);
template void update2_half<f16_t>(Ctx&, HF, HF, HF, HF, int, int, int);
template void update2_half<bf16_t>(Ctx&, HF, HF, HF, HF, int, int, int);

template <typename B>
void gcr_orth_b(Ctx& c, const cx<B>* W, cx<B>* w, const cx<double>* r, size_t n, int nb, int j, int gl) {
  double* g = c.dsc + gcr_base(gl);
  if (j > 0) {
    const int gy = (j + GCR_G - 1) / GCR_G;
    int gx = (int)reduce_blocks(n);
    if ((size_t)gx * gy * nb > 8192) gx = 8192 / (gy * nb);
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(k_gcr_dots_b<B>, dim3(gx, gy, nb), dim3(TPB), 0, c.stream, W, w, n, nb, j, gx, gy,
                       c.partials);
    WDMG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gcr_dots_b_fin, dim3(nb, (2 * j + TPB / 64 - 1) / (TPB / 64)), dim3(TPB), 0, c.stream, j, gx,
                       gy, c.partials, g);
    WDMG_HIP(hipGetLastError());
  }
  run_reduce_b(c, GcrAxpyCoefBOp<B>{W, w, r, g, c.dsc, n, nb, j}, n, nb);
}

template <typename B>
void gcr_step_b(Ctx& c, const cx<B>* w, cx<double>* r, size_t n, int nb, int gl, double* host) {
  run_reduce_b(c, GcrUpdateBOp<B>{w, r, c.dsc + gcr_base(gl), c.dsc, host, n}, n, nb);
}

void gcr_record(Ctx& c, cx<double>* hist, cx<double>* av, int nb, int j, int k, int gl) {
  hipLaunchKernelGGL(k_gcr_record, dim3(nb), dim3(64), 0, c.stream, c.dsc + gcr_base(gl), hist, av, nb, j, k);
  WDMG_HIP(hipGetLastError());
}

template <typename B>
void gcr_combine(Ctx& c, cx<double>* x, const cx<B>* Z, const cx<double>* hist, const cx<double>* av, cx<double>* y,
                 size_t n, int nb, int jn, int k) {
  if (jn == 0) return;
  hipLaunchKernelGGL(k_gcr_backsolve, dim3(1), dim3(kMaxRhs), 0, c.stream, hist, av, y, nb, jn, k);
  WDMG_HIP(hipGetLastError());
  unsigned gx = ew_blocks(n);
  if (gx * nb > 8192) gx = (8192 + nb - 1) / nb;
  hipLaunchKernelGGL(k_gcr_combine<B>, dim3(gx, nb), dim3(256), 0, c.stream, x, Z, y, n, nb, jn, k);
  WDMG_HIP(hipGetLastError());
}

template void gcr_orth_b<double>(Ctx&, const cx<double>*, cx<double>*, const cx<double>*, size_t, int, int, int);
template void gcr_orth_b<float>(Ctx&, const cx<float>*, cx<float>*, const cx<double>*, size_t, int, int, int);
template void gcr_step_b<double>(Ctx&, const cx<double>*, cx<double>*, size_t, int, int, double*);
template void gcr_step_b<float>(Ctx&, const cx<float>*, cx<double>*, size_t, int, int, double*);
template void gcr_combine<double>(Ctx&, cx<double>*, const cx<double>*, const cx<double>*, const cx<double>*,
                                  cx<double>*, size_t, int, int, int);
template void gcr_combine<float>(Ctx&, cx<double>*, const cx<float>*, const cx<double>*, const cx<double>*,
                                 cx<double>*, size_t, int, int, int);

void norm2_b(Ctx& c, const cx<double>* a, size_t n, int nb, int gl, double* host) {
  run_reduce_b(c, Norm2BOp{a, c.dsc + gcr_base(gl), c.dsc, host, n}, n, nb);
}

void xmy_norm_b(Ctx& c, const cx<double>* b, cx<double>* y, size_t n, int nb, int gl) {
  run_reduce_b(c, XmyNormBOp{b, y, c.dsc + gcr_base(gl), c.dsc, n}, n, nb);
}

void set_active(Ctx& c, int gl, const double* host_flags, int nb) {
  // staged through pinned memory so the copy is asynchronous and stream-ordered;
  // every reader of c.hsc synchronises the stream first, so the slot is free
  double* stage = c.hsc + kHscFlags;
  WDMG_HIP(hipStreamSynchronize(c.stream));
  for (int i = 0; i < nb; ++i) stage[i] = host_flags[i];
  WDMG_HIP(hipMemcpyAsync(c.dsc + gcr_base(gl) + G_ACT, stage, nb * sizeof(double), hipMemcpyHostToDevice,
                          c.stream));
}

void xmy_norm(Ctx& c, const cx<double>* b, cx<double>* y, size_t n, int slot) {
  run_reduce(c, XmyNormOp{b, y, c.dsc, slot}, n);
}

void bicg_p(Ctx& c, cx<double>* p, const cx<double>* r, const cx<double>* v, size_t n, bool first) {
  hipLaunchKernelGGL(k_bicg_p, dim3(ew_blocks(n)), dim3(256), 0, c.stream, p, r, v, n, c.dsc, first ? 1 : 0);
  WDMG_HIP(hipGetLastError());
}
void bicg_alpha(Ctx& c, const cx<double>* rhat, const cx<double>* v, size_t n) {
  run_reduce(c, BicgAlphaOp{rhat, v, c.dsc}, n);
}
void bicg_s(Ctx& c, cx<double>* s, const cx<double>* r, const cx<double>* v, size_t n) {
  hipLaunchKernelGGL(k_bicg_s, dim3(ew_blocks(n)), dim3(256), 0, c.stream, s, r, v, n, c.dsc);
  WDMG_HIP(hipGetLastError());
}
void bicg_omega(Ctx& c, const cx<double>* t, const cx<double>* s, size_t n) {
  run_reduce(c, BicgOmegaOp{t, s, c.dsc}, n);
}
void bicg_xr(Ctx& c, cx<double>* x, cx<double>* r, const cx<double>* p, const cx<double>* s, const cx<double>* sx,
             const cx<double>* t, const cx<double>* rhat, size_t n) {
  run_reduce(c, BicgXrOp{x, r, p, s, sx, t, rhat, c.dsc}, n);
}
void fill_pairs(Ctx& c, int slot, int count, double re, double im) {
  hipLaunchKernelGGL(k_fill_pairs, dim3(1), dim3(kMaxRhs), 0, c.stream, c.dsc, slot, count, re, im);
  WDMG_HIP(hipGetLastError());
}

void set_scalar(Ctx& c, int slot, double re, double im) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, c.stream, c.dsc, slot, re, im);
  WDMG_HIP(hipGetLastError());
}

#define INST(R)                                                                            \
  template void zero<R>(Ctx&, cx<R>*, size_t);                                             \
  template void copy<R>(Ctx&, cx<R>*, const cx<R>*, size_t);                               \
  template void neg<R>(Ctx&, cx<R>*, size_t);                                              \
  template void xmy<R>(Ctx&, const cx<R>*, cx<R>*, size_t);                                \
  template void add<R>(Ctx&, cx<R>*, const cx<R>*, size_t);                                \
  template void step_alpha<R>(Ctx&, const cx<R>*, const cx<R>*, size_t, double, int);      \
  template void update2<R>(Ctx&, cx<R>*, const cx<R>*, cx<R>*, const cx<R>*, size_t, int); \
  template void norm2<R>(Ctx&, const cx<R>*, size_t, int);                                 \
  template void dot<R>(Ctx&, const cx<R>*, const cx<R>*, size_t, int);                      \
  template void step_alpha_batch<R>(Ctx&, const cx<R>*, const cx<R>*, size_t, size_t, int, double, int); \
  template void update2_batch<R>(Ctx&, cx<R>*, const cx<R>*, cx<R>*, const cx<R>*, size_t, size_t, int, int, int);
INST(double)
INST(float)
#undef INST

}  // namespace wdmg
