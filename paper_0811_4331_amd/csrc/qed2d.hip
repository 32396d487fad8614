// The 2d U(1) Wilson-Dirac workload of Sec. 4 on gfx950 (FP64): the 2d form
// of the Sec. 1 operator, the adaptive setup of Sec. 2 with chirality-split
// block QR (Sec. 3), Galerkin coarse operators of D and of D^dagger D (Sec. 3,
// both approaches), V(nu_pre, nu_post) cycles with an exact coarsest solve,
// and the three solvers compared in Sec. 4 (MG-BiCGstab, MG-CG, CG).
//
// Design: every field of one level is a few hundred KB, so the work is bound
// by launch latency, not by HBM.  The solvers therefore keep every scalar on
// the device (a reduction kernel, one workgroup per right-hand side, computes
// its dot products and the coefficient that the next update kernel reads) and
// synchronise with the host once per outer iteration for the stopping test.
// The setup batches its right-hand sides: the Nv candidates relax together,
// and the Galerkin operator is read off 16 * 2Nv coloured probe vectors in
// one prolongation, one operator application and one restriction.  The
// coarsest operator is inverted once (Gauss-Jordan with partial pivoting) so
// that its solve is one dense matrix-vector product, one wavefront per row.
//
// Layouts: lexicographic sites s = t * Lx + x; a level-l field is
// [rhs][site][chirality][n_l]; the prolongator columns Q are [Nv][site][2][n_l];
// coarse-operator blocks are [offset][site][row][col].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/wdmg_2d.h"
#include "common.h"

using wdmg::cmadd;
using wdmg::cmaddc;
using wdmg::mk;
typedef wdmg::cx<double> C;

namespace {

struct Err {
  int code;
  std::string msg;
};

#define Q2_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) throw Err{WDMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Coarse offsets (d_x, d_t): the first five are the nearest-neighbour stencil
// of D_c, all nine the stencil of (D^dagger D)_c.
constexpr int kMaxOff = 9;
__constant__ int c_off[2][kMaxOff] = {{0, 1, -1, 0, 0, 1, -1, 1, -1}, {0, 0, 0, 1, -1, 1, 1, -1, -1}};

// Device scalar slots.
enum { S_RHO = 0, S_ALPHA, S_OMEGA, S_BETA, S_PQ, S_RR, S_FLAG, S_MR, S_TOTAL = S_MR + 64 };
// Workgroups of one reduction per rhs, and rhs of one reduction launch.
constexpr int kMaxDotGroups = 128, kMaxDotRhs = 64;

__device__ __forceinline__ C neg(C a) { return mk(-a.re, -a.im); }
__device__ __forceinline__ C cdiv(C a, C b) {
  const double d = b.re * b.re + b.im * b.im;
  return mk((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
__device__ __forceinline__ bool is_zero(C a) { return a.re == 0.0 && a.im == 0.0; }

inline unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// Fine operator: D (G5 = false) or gamma5 D gamma5 = D^dagger (G5 = true), one
// thread per site and rhs.  Spin projections of the 2d gamma matrices:
//   (1 - sigma_1) c = (h, -h),   h = c0 - c1;   (1 + sigma_1) c = (h, h),    h = c0 + c1;
//   (1 - sigma_2) c = (h, -i h), h = c0 + i c1; (1 + sigma_2) c = (h, i h),  h = c0 - i c1.
template <bool G5>
__global__ void __launch_bounds__(256) k_wilson(C* __restrict__ out, const C* __restrict__ in,
                                                const C* __restrict__ U, int lx, int lt, double diag,
                                                double tbc, int nrhs) {
  const int vol = lx * lt;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)vol * nrhs) return;
  const int r = (int)(gid / vol), s = (int)(gid - (size_t)r * vol);
  const int x = s % lx, t = s / lx;
  const C* f = in + (size_t)r * vol * 2;
  auto ld = [&](int site, C& c0, C& c1) {
    c0 = f[2 * site];
    c1 = f[2 * site + 1];
    if (G5) c1 = neg(c1);
  };
  C acc0 = mk(0.0, 0.0), acc1 = mk(0.0, 0.0), c0, c1;
  // +x
  {
    const int sn = t * lx + (x + 1 == lx ? 0 : x + 1);
    ld(sn, c0, c1);
    const C w = U[2 * s] * (c0 - c1);
    acc0 = acc0 + w;
    acc1 = acc1 - w;
  }
  // -x
  {
    const int sn = t * lx + (x == 0 ? lx - 1 : x - 1);
    ld(sn, c0, c1);
    C w = mk(0.0, 0.0);
    cmaddc(w, U[2 * sn], c0 + c1);
    acc0 = acc0 + w;
    acc1 = acc1 + w;
  }
  // +t
  {
    const bool wrap = t + 1 == lt;
    const int sn = (wrap ? 0 : t + 1) * lx + x;
    ld(sn, c0, c1);
    C w = U[2 * s + 1] * (c0 + wdmg::ti(c1));
    if (wrap) w = tbc * w;
    acc0 = acc0 + w;
    acc1 = acc1 + wdmg::tmi(w);
  }
  // -t
  {
    const bool wrap = t == 0;
    const int sn = (wrap ? lt - 1 : t - 1) * lx + x;
    ld(sn, c0, c1);
    C w = mk(0.0, 0.0);
    cmaddc(w, U[2 * sn + 1], c0 + wdmg::tmi(c1));
    if (wrap) w = tbc * w;
    acc0 = acc0 + w;
    acc1 = acc1 + wdmg::ti(w);
  }
  ld(s, c0, c1);
  C o0 = diag * c0 - 0.5 * acc0;
  C o1 = diag * c1 - 0.5 * acc1;
  if (G5) o1 = neg(o1);
  C* g = out + (size_t)r * vol * 2;
  g[2 * s] = o0;
  g[2 * s + 1] = o1;
}

// Coarse stencil: out(s)[i] = sum_o sum_j B[o][s][i][j] in(s + d_o)[j], one
// thread per (rhs, site, row).
__global__ void __launch_bounds__(256) k_stencil(C* __restrict__ out, const C* __restrict__ in,
                                                 const C* __restrict__ B, int lx, int lt, int N, int S,
                                                 int nrhs) {
  const int vol = lx * lt;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)nrhs * vol * N) return;
  const int i = (int)(gid % N);
  const int s = (int)((gid / N) % vol);
  const int r = (int)(gid / ((size_t)N * vol));
  const int x = s % lx, t = s / lx;
  C acc = mk(0.0, 0.0);
  for (int o = 0; o < S; ++o) {
    const int xn = (x + c_off[0][o] + lx) % lx, tn = (t + c_off[1][o] + lt) % lt;
    const C* b = B + (((size_t)o * vol + s) * N + i) * N;
    const C* v = in + ((size_t)r * vol + tn * lx + xn) * N;
    for (int j = 0; j < N; ++j) cmadd(acc, b[j], v[j]);
  }
  out[gid] = acc;
}

// The same stencil for N = 8, 16 or 32 dof per site: 64 / N rows of one
// site per wavefront, lane (row, j) multiplying B[o](s)[i][j] by in(s + d_o)[j],
// so that a wavefront reads 64 consecutive block entries per offset; the
// N lanes of a row are summed with cross-lane adds.
template <int N>
__global__ void __launch_bounds__(256) k_stencil_w(C* __restrict__ out, const C* __restrict__ in,
                                                   const C* __restrict__ B, int lx, int lt, int S, int nrhs) {
  static_assert(N >= 8 && N <= 64 && (N & (N - 1)) == 0, "N must be a power of two in 8..64");
  constexpr int R = 64 / N;  // rows per wavefront
  constexpr int W = N / R;   // wavefronts per site
  const int vol = lx * lt;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= (size_t)nrhs * vol * W) return;
  const int grp = (int)(wave % W);
  const size_t rest = wave / W;
  const int s = (int)(rest % vol), r = (int)(rest / vol);
  const int i = grp * R + lane / N, j = lane % N;
  const int x = s % lx, t = s / lx;
  C acc = mk(0.0, 0.0);
  for (int o = 0; o < S; ++o) {
    const int xn = (x + c_off[0][o] + lx) % lx, tn = (t + c_off[1][o] + lt) % lt;
    cmadd(acc, B[(((size_t)o * vol + s) * N + i) * N + j], in[((size_t)r * vol + tn * lx + xn) * N + j]);
  }
#pragma unroll
  for (int h = N / 2; h > 0; h >>= 1) {
    acc.re += __shfl_xor(acc.re, h, 64);
    acc.im += __shfl_xor(acc.im, h, 64);
  }
  if (j == 0) out[((size_t)r * vol + s) * N + i] = acc;
}

// Restriction P^dagger: out(sc, chi, k) = sum_{s in aggregate} sum_i conj(Q_k(s)_{chi,i}) in(s)_{chi,i}
// over g groups per site (g = 2 chiralities; g = 1 when the spin is blocked).
// With g5 (fine level only, where a site holds the two spins as its
// components chi * n + i) the restriction is P^dagger gamma5.
__global__ void __launch_bounds__(256) k_restrict(C* __restrict__ out, const C* __restrict__ in,
                                                  const C* __restrict__ Q, int lx, int lt, int bx, int bt,
                                                  int g, int n, int nv, int g5, int nrhs) {
  const int vol = lx * lt, lxc = lx / bx, volc = vol / (bx * bt);
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)nrhs * volc * g * nv) return;
  const int k = (int)(gid % nv);
  const int chi = (int)((gid / nv) % g);
  const int sc = (int)((gid / ((size_t)g * nv)) % volc);
  const int r = (int)(gid / ((size_t)g * nv * volc));
  const int xc = sc % lxc, tc = sc / lxc;
  C acc = mk(0.0, 0.0);
  for (int dt = 0; dt < bt; ++dt)
    for (int dx = 0; dx < bx; ++dx) {
      const int s = (tc * bt + dt) * lx + xc * bx + dx;
      const C* q = Q + (((size_t)k * vol + s) * g + chi) * n;
      const C* f = in + (((size_t)r * vol + s) * g + chi) * n;
      for (int i = 0; i < n; ++i) cmaddc(acc, q[i], (g5 && chi * n + i == 1) ? neg(f[i]) : f[i]);
    }
  out[gid] = acc;
}

// The same restriction with one lane per site of the aggregate (A = bx * bt
// lanes per output, A a power of two <= 64): lane a adds the n products of
// site a, and the A lanes of an output are summed with cross-lane adds.
template <int A>
__global__ void __launch_bounds__(256) k_restrict_w(C* __restrict__ out, const C* __restrict__ in,
                                                    const C* __restrict__ Q, int lx, int lt, int bx, int g, int n,
                                                    int nv, int g5, int nrhs) {
  const int bt = A / bx;
  const int vol = lx * lt, lxc = lx / bx, volc = vol / A;
  const size_t item = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / A;  // output index
  const int a = threadIdx.x % A;
  if (item >= (size_t)nrhs * volc * g * nv) return;
  const int k = (int)(item % nv);
  const int chi = (int)((item / nv) % g);
  const int sc = (int)((item / ((size_t)g * nv)) % volc);
  const int r = (int)(item / ((size_t)g * nv * volc));
  const int xc = sc % lxc, tc = sc / lxc;
  const int s = (tc * bt + a / bx) * lx + xc * bx + a % bx;
  const C* q = Q + (((size_t)k * vol + s) * g + chi) * n;
  const C* f = in + (((size_t)r * vol + s) * g + chi) * n;
  C acc = mk(0.0, 0.0);
  for (int i = 0; i < n; ++i) cmaddc(acc, q[i], (g5 && chi * n + i == 1) ? neg(f[i]) : f[i]);
#pragma unroll
  for (int h = A / 2; h > 0; h >>= 1) {
    acc.re += __shfl_xor(acc.re, h, 64);
    acc.im += __shfl_xor(acc.im, h, 64);
  }
  if (a == 0) out[item] = acc;
}

// Prolongation P: out(s)_{chi,i} = sum_k Q_k(s)_{chi,i} in(aggregate(s), chi, k).
__global__ void __launch_bounds__(256) k_prolong(C* __restrict__ out, const C* __restrict__ in,
                                                 const C* __restrict__ Q, int lx, int lt, int bx, int bt,
                                                 int g, int n, int nv, int nrhs) {
  const int vol = lx * lt, lxc = lx / bx, volc = vol / (bx * bt);
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)nrhs * vol * g * n) return;
  const int i = (int)(gid % n);
  const int chi = (int)((gid / n) % g);
  const int s = (int)((gid / ((size_t)g * n)) % vol);
  const int r = (int)(gid / ((size_t)g * n * vol));
  const int x = s % lx, t = s / lx;
  const int sc = (t / bt) * lxc + x / bx;
  C acc = mk(0.0, 0.0);
  const C* c = in + (((size_t)r * volc + sc) * g + chi) * nv;
  for (int k = 0; k < nv; ++k) cmadd(acc, Q[(((size_t)k * vol + s) * g + chi) * n + i], c[k]);
  out[gid] = acc;
}

// Block QR of the candidates (Sec. 2, P V_c = V with P^dagger P = I; Sec. 3,
// one block per aggregate and chirality): modified Gram-Schmidt applied twice
// per column, which yields the thin QR with a real positive diagonal of R.
// One thread per (aggregate, group); Q is overwritten in place.  A column
// whose remaining norm falls to 1e-12 of its original norm sets *status = 1.
__global__ void k_block_qr(C* __restrict__ Q, int lx, int lt, int bx, int bt, int g, int n, int nv,
                           int* __restrict__ status) {
  const int vol = lx * lt, lxc = lx / bx, volc = vol / (bx * bt);
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= volc * g) return;
  const int chi = gid % g, sc = gid / g;
  const int xc = sc % lxc, tc = sc / lxc;
  const int m = bx * bt * n;
  auto at = [&](int k, int e) -> C& {
    const int i = e % n, b = e / n;
    const int s = (tc * bt + b / bx) * lx + xc * bx + b % bx;
    return Q[(((size_t)k * vol + s) * g + chi) * n + i];
  };
  for (int k = 0; k < nv; ++k) {
    double orig = 0.0;
    for (int e = 0; e < m; ++e) {
      const C v = at(k, e);
      orig += v.re * v.re + v.im * v.im;
    }
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < k; ++j) {
        C d = mk(0.0, 0.0);
        for (int e = 0; e < m; ++e) cmaddc(d, at(j, e), at(k, e));
        for (int e = 0; e < m; ++e) {
          C& v = at(k, e);
          v = v - d * at(j, e);
        }
      }
    double nrm = 0.0;
    for (int e = 0; e < m; ++e) {
      const C v = at(k, e);
      nrm += v.re * v.re + v.im * v.im;
    }
    nrm = sqrt(nrm);
    if (!(nrm > 1e-12 * sqrt(orig))) {
      *status = 1;
      return;
    }
    const double inv = 1.0 / nrm;
    for (int e = 0; e < m; ++e) {
      C& v = at(k, e);
      v = inv * v;
    }
  }
}

// Coloured probe vectors of a coarse level with N dof per site: probe
// p = (kappa_t * K0 + kappa_x) * N + a is e_a on every site whose coordinates
// are congruent to kappa modulo (K0, K1), zero elsewhere.
__global__ void __launch_bounds__(256) k_probe_fill(C* __restrict__ c, int lxc, int ltc, int N, int K0, int K1) {
  const int volc = lxc * ltc;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)K0 * K1 * N * volc * N) return;
  const int j = (int)(gid % N);
  const int sc = (int)((gid / N) % volc);
  const int p = (int)(gid / ((size_t)N * volc));
  const int a = p % N, kap = p / N;
  const int xc = sc % lxc, tc = sc / lxc;
  const bool on = (xc % K0 == kap % K0) && (tc % K1 == kap / K0) && j == a;
  c[gid] = mk(on ? 1.0 : 0.0, 0.0);
}

// Galerkin blocks from the probe responses y_p = P^dagger A P c_p: with
// K >= 3 at most one site of a colour lies within one step of a coarse site,
// so B[o](s)[i][a] = y_p(s)[i] for the probe p of the colour of s + d_o.
__global__ void __launch_bounds__(256) k_probe_gather(C* __restrict__ B, const C* __restrict__ y, int lxc,
                                                      int ltc, int N, int S, int K0, int K1) {
  const int volc = lxc * ltc;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)S * volc * N * N) return;
  const int a = (int)(gid % N);
  const int i = (int)((gid / N) % N);
  const int sc = (int)((gid / ((size_t)N * N)) % volc);
  const int o = (int)(gid / ((size_t)N * N * volc));
  const int xc = sc % lxc, tc = sc / lxc;
  const int k0 = ((xc + c_off[0][o]) % K0 + K0) % K0;
  const int k1 = ((tc + c_off[1][o]) % K1 + K1) % K1;
  const int p = (k1 * K0 + k0) * N + a;
  B[gid] = y[((size_t)p * volc + sc) * N + i];
}

// Dense [M | I] (n x 2n, row-major) of the coarsest stencil, n = sites * N.
__global__ void __launch_bounds__(256) k_dense_aug(C* __restrict__ M, const C* __restrict__ B, int lxc, int ltc,
                                                   int N, int S) {
  const int volc = lxc * ltc, n = volc * N;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n * 2 * n) return;
  const int col = (int)(gid % (2 * n)), row = (int)(gid / (2 * n));
  if (col >= n) {
    M[gid] = mk(col - n == row ? 1.0 : 0.0, 0.0);
    return;
  }
  const int sr = row / N, i = row % N, scol = col / N, j = col % N;
  const int xr = sr % lxc, tr = sr / lxc;
  C acc = mk(0.0, 0.0);
  for (int o = 0; o < S; ++o) {
    const int sn = ((tr + c_off[1][o] + ltc) % ltc) * lxc + (xr + c_off[0][o] + lxc) % lxc;
    if (sn == scol) acc = acc + B[(((size_t)o * volc + sr) * N + i) * N + j];
  }
  M[gid] = acc;
}

// Gauss-Jordan step k, pivot part (one workgroup): the row with the largest
// |M[i][k]|, i >= k, is swapped into row k, which is scaled so that
// M[k][k] = 1; column k is saved for the elimination.  A zero pivot sets
// *status = 2.
__global__ void __launch_bounds__(1024) k_gj_pivot(C* __restrict__ M, C* __restrict__ col, int n, int k,
                                                   int* __restrict__ status) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x, bs = blockDim.x;
  const size_t ld = 2 * (size_t)n;
  double best = -1.0;
  int bi = k;
  for (int i = k + tid; i < n; i += bs) {
    const C v = M[i * ld + k];
    const double a = v.re * v.re + v.im * v.im;
    if (a > best) {
      best = a;
      bi = i;
    }
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int h = bs / 2; h > 0; h >>= 1) {
    if (tid < h && (sv[tid + h] > sv[tid] || (sv[tid + h] == sv[tid] && si[tid + h] < si[tid]))) {
      sv[tid] = sv[tid + h];
      si[tid] = si[tid + h];
    }
    __syncthreads();
  }
  const int p = si[0];
  if (!(sv[0] > 0.0)) {
    if (tid == 0) *status = 2;
    return;
  }
  if (p != k)
    for (size_t j = tid; j < ld; j += bs) {
      const C a = M[k * ld + j];
      M[k * ld + j] = M[p * ld + j];
      M[p * ld + j] = a;
    }
  __syncthreads();
  const C piv = M[k * ld + k];
  __syncthreads();
  const double d = piv.re * piv.re + piv.im * piv.im;
  const C inv = mk(piv.re / d, -piv.im / d);
  for (size_t j = tid; j < ld; j += bs) M[k * ld + j] = inv * M[k * ld + j];
  __syncthreads();
  for (int i = tid; i < n; i += bs) col[i] = M[i * ld + k];
}

// Gauss-Jordan step k, elimination: M[i][j] -= col[i] M[k][j] for i != k and
// j >= k (row k and the saved column are only read).
__global__ void __launch_bounds__(256) k_gj_elim(C* __restrict__ M, const C* __restrict__ col, int n, int k) {
  const size_t ld = 2 * (size_t)n, w = ld - k;
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (size_t)n * w) return;
  const int i = (int)(gid / w);
  const size_t j = k + gid % w;
  if (i == k) return;
  const C f = col[i];
  if (is_zero(f)) return;
  M[i * ld + j] = M[i * ld + j] - f * M[k * ld + j];
}

// Coarsest solve out = M^-1 in, the inverse being the right half of the
// reduced [I | M^-1]; one wavefront per (rhs, row).
__global__ void __launch_bounds__(256) k_dense_apply(C* __restrict__ out, const C* __restrict__ M,
                                                     const C* __restrict__ in, int n, int nrhs) {
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (wave >= (size_t)n * nrhs) return;
  const int row = (int)(wave % n), r = (int)(wave / n);
  const C* m = M + (size_t)row * 2 * n + n;
  const C* v = in + (size_t)r * n;
  C acc = mk(0.0, 0.0);
  for (int j = lane; j < n; j += 64) cmadd(acc, m[j], v[j]);
  const double re = wdmg::wave_sum(acc.re), im = wdmg::wave_sum(acc.im);
  if (lane == 0) out[(size_t)r * n + row] = mk(re, im);
}

// ---------------------------------------------------------------------------
// Reductions with the coefficient logic of the solvers, one workgroup per rhs.
enum {
  M_MR = 0,       // <p,p>, <p,r>:  coef[rhs] = omega <p,r> / <p,p>   (0 when <p,p> = 0)
  M_NORM,         // <r,r>:         rr
  M_RHO,          // <rhat,r>:      beta = (rho_new / rho)(alpha / omega), rho = rho_new
  M_BIC_ALPHA,    // <rhat,v>:      alpha = rho / <rhat,v>
  M_OMEGA,        // <t,s>, <t,t>:  omega = <t,s> / <t,t>  (0 when <t,t> = 0)
  M_FCG_BETA,     // <q,z>:         beta = -<q,z> / pq
  M_FCG_ALPHA     // <p,q>, <p,r>:  pq = <p,q>, alpha = <p,r> / pq
};

// The coefficient logic of the solvers, from the summed dot products.
template <int MODE>
__device__ void finish_dots(C d0, C d1, int rhs, C* sc, double omega) {
  if (MODE == M_MR) {
    sc[S_MR + rhs] = d0.re == 0.0 ? mk(0.0, 0.0) : (omega / d0.re) * d1;
  } else if (MODE == M_NORM) {
    sc[S_RR] = mk(d0.re, 0.0);
  } else if (MODE == M_RHO) {
    if (is_zero(d0)) {
      sc[S_FLAG] = mk(1.0, 0.0);
      return;
    }
    sc[S_BETA] = cdiv(d0, sc[S_RHO]) * cdiv(sc[S_ALPHA], sc[S_OMEGA]);
    sc[S_RHO] = d0;
  } else if (MODE == M_BIC_ALPHA) {
    if (sc[S_FLAG].re != 0.0) return;
    if (is_zero(d0)) {
      sc[S_FLAG] = mk(1.0, 0.0);
      return;
    }
    sc[S_ALPHA] = cdiv(sc[S_RHO], d0);
  } else if (MODE == M_OMEGA) {
    if (sc[S_FLAG].re != 0.0) return;
    sc[S_OMEGA] = d1.re == 0.0 ? mk(0.0, 0.0) : (1.0 / d1.re) * d0;
  } else if (MODE == M_FCG_BETA) {
    sc[S_BETA] = neg(cdiv(d0, sc[S_PQ]));
  } else if (MODE == M_FCG_ALPHA) {
    sc[S_PQ] = d0;
    sc[S_ALPHA] = cdiv(d1, d0);
  }
}

// One or two dot products per rhs over gridDim.x workgroups (grid y = rhs):
// each workgroup stores its partial sums [rhs][group][4]; the consumer (the
// next launch) adds them.  Kernel boundaries order the two, so no fence or
// atomic is needed inside the reduction.
template <int MODE>
__global__ void __launch_bounds__(256) k_dots(const C* __restrict__ a0, const C* __restrict__ b0,
                                              const C* __restrict__ a1, const C* __restrict__ b1, size_t n,
                                              double* __restrict__ part) {
  __shared__ double lds[4 * 4];
  constexpr bool two = MODE == M_MR || MODE == M_OMEGA || MODE == M_FCG_ALPHA;
  const int G = gridDim.x, g = blockIdx.x, rhs = blockIdx.y;
  const size_t off = (size_t)rhs * n;
  C d0 = mk(0.0, 0.0), d1 = mk(0.0, 0.0);
  for (size_t e = (size_t)g * blockDim.x + threadIdx.x; e < n; e += (size_t)G * blockDim.x) {
    cmaddc(d0, a0[off + e], b0[off + e]);
    if (two) cmaddc(d1, a1[off + e], b1[off + e]);
  }
  double v[4] = {d0.re, d0.im, d1.re, d1.im};
  wdmg::block_sum<4>(v, lds);
  if (threadIdx.x == 0) {
    double* p = part + ((size_t)rhs * G + g) * 4;
    for (int q = 0; q < 4; ++q) p[q] = v[q];
  }
}

// The partials of one rhs summed by one wavefront (lane k adds workgroups k
// and k + 64, G <= 128, then a fixed cross-lane tree).  Every lane of the
// wavefront must call it.
__device__ __forceinline__ void sum_partials(const double* __restrict__ part, int rhs, int G, double t[4]) {
  const int lane = threadIdx.x & 63;
  const double* p = part + (size_t)rhs * G * 4;
  for (int q = 0; q < 4; ++q) {
    t[q] = lane < G ? p[lane * 4 + q] : 0.0;
    if (lane + 64 < G) t[q] += p[(lane + 64) * 4 + q];
    t[q] = wdmg::wave_sum(t[q]);
  }
}

template <int MODE>
__global__ void __launch_bounds__(64) k_finish(const double* __restrict__ part, int G, C* __restrict__ sc,
                                               double omega) {
  double t[4];
  sum_partials(part, blockIdx.x, G, t);
  if (threadIdx.x == 0) finish_dots<MODE>(mk(t[0], t[1]), mk(t[2], t[3]), blockIdx.x, sc, omega);
}

// The MR step (and the minimal-residual step after a prolongation) in one
// launch: every wavefront sums the partials of <p,p> and <p,r> of its rhs,
// c = omega <p,r> / <p,p> (0 when <p,p> = 0), then x += c dx, r -= c dr.
// Needs n % 64 == 0, so that a wavefront never spans two right-hand sides.
__global__ void __launch_bounds__(256) k_update_mr(C* __restrict__ x, C* r, const C* dx, const C* __restrict__ dr,
                                                   const double* __restrict__ part, int G, double omega, size_t n,
                                                   int nrhs) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((gid & ~(size_t)63) >= n * nrhs) return;  // whole wavefronts
  const int rhs = (int)(gid / n);
  double t[4];
  sum_partials(part, rhs, G, t);
  const C c = t[0] == 0.0 ? mk(0.0, 0.0) : (omega / t[0]) * mk(t[2], t[3]);
  const C d = dx[gid];
  x[gid] = x[gid] + c * d;
  r[gid] = r[gid] - c * dr[gid];
}

// x += c dx; r -= c dr with c = coefficient slot `slot + rhs` (fields of n elements).
__global__ void __launch_bounds__(256) k_update(C* __restrict__ x, C* r, const C* dx, const C* __restrict__ dr,
                                                const C* __restrict__ sc, int slot, size_t n, int nrhs) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n * nrhs) return;
  const C c = sc[slot + gid / n];
  const C d = dx[gid];
  x[gid] = x[gid] + c * d;
  r[gid] = r[gid] - c * dr[gid];
}

__global__ void __launch_bounds__(256) k_neg(C* __restrict__ out, const C* __restrict__ in, size_t n) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < n) out[gid] = neg(in[gid]);
}

__global__ void __launch_bounds__(256) k_xmy(C* __restrict__ out, const C* __restrict__ a, const C* __restrict__ b,
                                             size_t n) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < n) out[gid] = a[gid] - b[gid];
}

__global__ void __launch_bounds__(256) k_add(C* __restrict__ y, const C* __restrict__ x, size_t n) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < n) y[gid] = y[gid] + x[gid];
}

__global__ void k_set(C* sc, int slot, double re) { sc[slot] = mk(re, 0.0); }

__global__ void k_bic_init(C* sc) {
  sc[S_RHO] = sc[S_ALPHA] = sc[S_OMEGA] = mk(1.0, 0.0);
  sc[S_FLAG] = mk(0.0, 0.0);
}

// p = r + beta (p - omega v)
__global__ void __launch_bounds__(256) k_bic_p(C* __restrict__ p, const C* __restrict__ r, const C* __restrict__ v,
                                               const C* __restrict__ sc, size_t n) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n || sc[S_FLAG].re != 0.0) return;
  p[gid] = r[gid] + sc[S_BETA] * (p[gid] - sc[S_OMEGA] * v[gid]);
}

// s = r - alpha v
__global__ void __launch_bounds__(256) k_bic_s(C* __restrict__ s, const C* __restrict__ r, const C* __restrict__ v,
                                               const C* __restrict__ sc, size_t n) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n || sc[S_FLAG].re != 0.0) return;
  s[gid] = r[gid] - sc[S_ALPHA] * v[gid];
}

// x += alpha ph + omega sh; r = s - omega t
__global__ void __launch_bounds__(256) k_bic_xr(C* __restrict__ x, C* __restrict__ r, const C* __restrict__ ph,
                                                const C* __restrict__ sh, const C* __restrict__ s,
                                                const C* __restrict__ t, const C* __restrict__ sc, size_t n) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n || sc[S_FLAG].re != 0.0) return;
  x[gid] = x[gid] + sc[S_ALPHA] * ph[gid] + sc[S_OMEGA] * sh[gid];
  r[gid] = s[gid] - sc[S_OMEGA] * t[gid];
}

// p = z (first) or z + beta p
__global__ void __launch_bounds__(256) k_fcg_p(C* __restrict__ p, const C* __restrict__ z, const C* __restrict__ sc,
                                               size_t n, int first) {
  const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  p[gid] = first ? z[gid] : z[gid] + sc[S_BETA] * p[gid];
}

}  // namespace

// ---------------------------------------------------------------------------
// Context.
struct Lev2 {
  int lx = 0, lt = 0, vol = 0;
  int g = 2, n = 1;                    // groups per site (2 chiralities, or 1: spin blocked), dof per group
  size_t nf = 0;                       // complex elements per field: vol * g * n
  int nv = 0;                          // candidates of the coarsening from this level
  C* Q = nullptr;                      // [nv][vol][g][n]
  C* B = nullptr;                      // stencil of this level (l >= 1)
  int S = 0;
  C *X = nullptr, *R = nullptr, *T = nullptr, *Y = nullptr, *Bv = nullptr;  // cycle work
  C *E = nullptr, *Rs = nullptr, *T2 = nullptr;  // repeated coarse cycles
};

struct wdmg_2d_ctx {
  int lx = 0, lt = 0;
  double m = 0.0;
  int t_bc = -1;
  bool have_gauge = false;
  hipStream_t stream = nullptr;
  wdmg_alloc alloc{};
  std::string err;
  std::vector<void*> bufs;       // lifetime of the context
  std::vector<void*> hier;       // lifetime of the hierarchy
  C* U = nullptr;
  C* sc = nullptr;               // device scalars
  C* hsc = nullptr;              // pinned host copy of the scalars
  int* status = nullptr;
  double* part = nullptr;        // reduction partials [rhs][group][4]
  C* tmp = nullptr;              // fine work for D^dagger D
  size_t tmp_fields = 0;
  std::vector<C*> sol;           // solver fields (fine, one rhs)
  // hierarchy
  std::vector<Lev2> lev;
  bool setup = false, normal = false;
  double omega = 0.8;
  int nu_pre = 2, nu_post = 2, use_alpha = 1, coarse_cycles = 1;
  int blocking = 0;              // 0 chirality kept; 1 spin blocked, R = P^dagger gamma5; 2 spin blocked, R = P^dagger
  C* Maug = nullptr;             // coarsest [M^-1 reduced | ...]: [nc][2 nc]
  C* gjcol = nullptr;
  int nc = 0;
  // counters
  long long wilson = 0;
  long long capp[WDMG_2D_MAX_LEVELS] = {0, 0, 0};
  double flops = 0.0;
};

namespace {
using Ctx = wdmg_2d_ctx;

void* dalloc(Ctx& c, size_t bytes, std::vector<void*>& owner) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (c.alloc.alloc) {
    p = c.alloc.alloc(bytes, c.alloc.user);
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255))
      throw Err{WDMG_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  } else if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Err{WDMG_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  owner.push_back(p);
  return p;
}

C* calloc_fields(Ctx& c, size_t elems, std::vector<void*>& owner) {
  return static_cast<C*>(dalloc(c, elems * sizeof(C), owner));
}

void release(Ctx& c, std::vector<void*>& owner) {
  for (void* p : owner) {
    if (c.alloc.free)
      c.alloc.free(p, c.alloc.user);
    else
      (void)hipFree(p);
  }
  owner.clear();
}

void drop_hierarchy(Ctx& c) {
  if (!c.hier.empty()) Q2_HIP(hipStreamSynchronize(c.stream));
  release(c, c.hier);
  c.lev.clear();
  c.setup = false;
  c.Maug = c.gjcol = nullptr;
  c.nc = 0;
}

void free_tmp(Ctx& c) {
  if (!c.tmp) return;
  Q2_HIP(hipStreamSynchronize(c.stream));
  for (size_t i = 0; i < c.bufs.size(); ++i)
    if (c.bufs[i] == c.tmp) {
      if (c.alloc.free)
        c.alloc.free(c.tmp, c.alloc.user);
      else
        (void)hipFree(c.tmp);
      c.bufs.erase(c.bufs.begin() + i);
      break;
    }
  c.tmp = nullptr;
  c.tmp_fields = 0;
}

C* ensure_tmp(Ctx& c, int nrhs) {
  const size_t need = (size_t)nrhs;
  if (c.tmp_fields < need) {
    free_tmp(c);
    c.tmp = calloc_fields(c, need * c.lx * c.lt * 2, c.bufs);
    c.tmp_fields = need;
  }
  return c.tmp;
}

// Work buffers of one setup, released when it ends (also when it fails).
struct SetupScratch {
  Ctx& c;
  std::vector<void*> bufs;
  explicit SetupScratch(Ctx& cc) : c(cc) {}
  ~SetupScratch() {
    (void)hipStreamSynchronize(c.stream);
    release(c, bufs);
  }
};

void launch_check() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Err{WDMG_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e)};
}

// D (dagger = false) or D^dagger on nrhs fine fields.
void wilson(Ctx& c, C* out, const C* in, int nrhs, bool dagger) {
  const size_t n = (size_t)c.lx * c.lt * nrhs;
  if (dagger)
    k_wilson<true><<<blocks_for(n, 256), 256, 0, c.stream>>>(out, in, c.U, c.lx, c.lt, 2.0 + c.m, c.t_bc, nrhs);
  else
    k_wilson<false><<<blocks_for(n, 256), 256, 0, c.stream>>>(out, in, c.U, c.lx, c.lt, 2.0 + c.m, c.t_bc, nrhs);
  launch_check();
  c.wilson += nrhs;
  c.flops += 8.0 * 18.0 * (double)n;
}

void normal0(Ctx& c, C* out, const C* in, int nrhs) {
  C* t = ensure_tmp(c, nrhs);
  wilson(c, t, in, nrhs, false);
  wilson(c, out, t, nrhs, true);
}

// out = A_l in.
void apply_level(Ctx& c, int l, C* out, const C* in, int nrhs) {
  if (l == 0) {
    if (c.normal)
      normal0(c, out, in, nrhs);
    else
      wilson(c, out, in, nrhs, false);
    return;
  }
  const Lev2& L = c.lev[l];
  const int N = L.g * L.n;
  const size_t tot = (size_t)nrhs * L.vol * N;
  const size_t lanes = tot * N;
  if (N == 8)
    k_stencil_w<8><<<blocks_for(lanes, 256), 256, 0, c.stream>>>(out, in, L.B, L.lx, L.lt, L.S, nrhs);
  else if (N == 16)
    k_stencil_w<16><<<blocks_for(lanes, 256), 256, 0, c.stream>>>(out, in, L.B, L.lx, L.lt, L.S, nrhs);
  else if (N == 32)
    k_stencil_w<32><<<blocks_for(lanes, 256), 256, 0, c.stream>>>(out, in, L.B, L.lx, L.lt, L.S, nrhs);
  else
    k_stencil<<<blocks_for(tot, 256), 256, 0, c.stream>>>(out, in, L.B, L.lx, L.lt, N, L.S, nrhs);
  launch_check();
  c.capp[l] += nrhs;
  c.flops += 8.0 * L.S * (double)L.vol * N * N * nrhs;
}

// P^dagger (or P^dagger gamma5 at the fine level of the spin-blocked control with blocking = 1)
void restrict_to(Ctx& c, int l, C* out, const C* in, int nrhs, const int blk[2]) {
  const Lev2& L = c.lev[l];
  const size_t tot = (size_t)nrhs * (L.vol / (blk[0] * blk[1])) * L.g * L.nv;
  const int A = blk[0] * blk[1];
  const int g5 = (l == 0 && c.blocking == 1) ? 1 : 0;
  if (A == 16)
    k_restrict_w<16><<<blocks_for(tot * 16, 256), 256, 0, c.stream>>>(out, in, L.Q, L.lx, L.lt, blk[0], L.g, L.n,
                                                                      L.nv, g5, nrhs);
  else if (A == 4)
    k_restrict_w<4><<<blocks_for(tot * 4, 256), 256, 0, c.stream>>>(out, in, L.Q, L.lx, L.lt, blk[0], L.g, L.n,
                                                                    L.nv, g5, nrhs);
  else
    k_restrict<<<blocks_for(tot, 256), 256, 0, c.stream>>>(out, in, L.Q, L.lx, L.lt, blk[0], blk[1], L.g, L.n,
                                                           L.nv, g5, nrhs);
  launch_check();
  c.flops += 8.0 * (double)L.vol * L.g * L.n * L.nv * nrhs;
}

void prolong_from(Ctx& c, int l, C* out, const C* in, int nrhs, const int blk[2]) {
  const Lev2& L = c.lev[l];
  const size_t tot = (size_t)nrhs * L.nf;
  k_prolong<<<blocks_for(tot, 256), 256, 0, c.stream>>>(out, in, L.Q, L.lx, L.lt, blk[0], blk[1], L.g, L.n, L.nv,
                                                        nrhs);
  launch_check();
  c.flops += 8.0 * (double)L.vol * L.g * L.n * L.nv * nrhs;
}

// about two elements per thread, at most kMaxDotGroups workgroups
int dot_groups(size_t n) { return (int)std::min<size_t>(kMaxDotGroups, std::max<size_t>(1, (n + 511) / 512)); }

// dot products and the coefficient logic of MODE, coefficients left in sc
template <int MODE>
void dots(Ctx& c, const C* a0, const C* b0, const C* a1, const C* b1, size_t n, int nrhs, double omega = 1.0) {
  const int G = dot_groups(n);
  k_dots<MODE><<<dim3(G, nrhs), 256, 0, c.stream>>>(a0, b0, a1, b1, n, c.part);
  k_finish<MODE><<<nrhs, 64, 0, c.stream>>>(c.part, G, c.sc, omega);
  launch_check();
}

// One MR step's coefficient and update: c = omega <p,r>/<p,p> per rhs, then
// x += c dx, r -= c dr (dx = r, dr = p for the smoother; the prolonged
// correction and its image for the minimal-residual step).
void mr_update(Ctx& c, C* x, C* r, const C* dx, const C* dr, const C* p, size_t n, int nrhs, double omega) {
  const int G = dot_groups(n);
  k_dots<M_MR><<<dim3(G, nrhs), 256, 0, c.stream>>>(p, p, p, r, n, c.part);
  if (n % 64 == 0) {
    k_update_mr<<<blocks_for(n * nrhs, 256), 256, 0, c.stream>>>(x, r, dx, dr, c.part, G, omega, n, nrhs);
  } else {
    k_finish<M_MR><<<nrhs, 64, 0, c.stream>>>(c.part, G, c.sc, omega);
    k_update<<<blocks_for(n * nrhs, 256), 256, 0, c.stream>>>(x, r, dx, dr, c.sc, S_MR, n, nrhs);
  }
  launch_check();
}

void update(Ctx& c, C* x, C* r, const C* dx, const C* dr, size_t n, int nrhs) {
  k_update<<<blocks_for(n * nrhs, 256), 256, 0, c.stream>>>(x, r, dx, dr, c.sc, S_MR, n, nrhs);
  launch_check();
}

void read_scalars(Ctx& c) {
  Q2_HIP(hipMemcpyAsync(c.hsc, c.sc, S_MR * sizeof(C), hipMemcpyDeviceToHost, c.stream));
  Q2_HIP(hipStreamSynchronize(c.stream));
}

double norm2(Ctx& c, const C* v, size_t n) {
  dots<M_NORM>(c, v, v, nullptr, nullptr, n, 1);
  read_scalars(c);
  return c.hsc[S_RR].re;
}

}  // namespace

namespace {

// aggregate extents (b_x, b_t) of coarsening l
void blk_pair(const Ctx& c, int l, int out[2]) {
  out[0] = c.lev[l].lx / c.lev[l + 1].lx;
  out[1] = c.lev[l].lt / c.lev[l + 1].lt;
}

// x = M r, V-cycle from x = 0 at level l (Sec. 2; Sec. 3 alpha step; Sec. 4 exact coarsest solve).
void vcycle(Ctx& c, int l, C* x, const C* r) {
  Lev2& L = c.lev[l];
  const int nl = (int)c.lev.size();
  int blk[2];
  blk_pair(c, l, blk);
  Q2_HIP(hipMemcpyAsync(L.R, r, L.nf * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
  Q2_HIP(hipMemsetAsync(x, 0, L.nf * sizeof(C), c.stream));
  auto mr_steps = [&](int k) {
    for (int i = 0; i < k; ++i) {
      apply_level(c, l, L.T, L.R, 1);
      mr_update(c, x, L.R, L.R, L.T, L.T, L.nf, 1, c.omega);
    }
  };
  mr_steps(c.nu_pre);
  Lev2& Cc = c.lev[l + 1];
  restrict_to(c, l, Cc.Bv, L.R, 1, blk);
  if (l + 1 == nl - 1) {
    k_dense_apply<<<blocks_for((size_t)c.nc * 64, 256), 256, 0, c.stream>>>(Cc.X, c.Maug, Cc.Bv, c.nc, 1);
    launch_check();
    c.capp[l + 1] += 1;
    c.flops += 8.0 * (double)c.nc * c.nc;
  } else if (c.coarse_cycles == 1) {
    vcycle(c, l + 1, Cc.X, Cc.Bv);
  } else {
    // e <- e + M_{l+1} (r_c - A_{l+1} e) from e = 0, coarse_cycles times
    Q2_HIP(hipMemsetAsync(Cc.E, 0, Cc.nf * sizeof(C), c.stream));
    for (int it = 0; it < c.coarse_cycles; ++it) {
      const C* res = Cc.Bv;
      if (it > 0) {
        apply_level(c, l + 1, Cc.T2, Cc.E, 1);
        k_xmy<<<blocks_for(Cc.nf, 256), 256, 0, c.stream>>>(Cc.Rs, Cc.Bv, Cc.T2, Cc.nf);
        launch_check();
        res = Cc.Rs;
      }
      vcycle(c, l + 1, Cc.X, res);
      k_add<<<blocks_for(Cc.nf, 256), 256, 0, c.stream>>>(Cc.E, Cc.X, Cc.nf);
      launch_check();
    }
    Q2_HIP(hipMemcpyAsync(Cc.X, Cc.E, Cc.nf * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
  }
  prolong_from(c, l, L.Y, Cc.X, 1, blk);
  apply_level(c, l, L.T, L.Y, 1);
  if (c.use_alpha)
    mr_update(c, x, L.R, L.Y, L.T, L.T, L.nf, 1, 1.0);
  else {
    k_set<<<1, 1, 0, c.stream>>>(c.sc, S_MR, 1.0);
    launch_check();
    update(c, x, L.R, L.Y, L.T, L.nf, 1);
  }
  mr_steps(c.nu_post);
}

void check_ready(const Ctx& c) {
  if (!c.have_gauge) throw Err{WDMG_ERR_NOT_SETUP, "no gauge field"};
}

int smallest_divisor_ge3(int e) {
  for (int k = 3; k <= e; ++k)
    if (e % k == 0) return k;
  return 0;
}

void mg_setup(Ctx& c, const wdmg_2d_mg_params& p) {
  check_ready(c);
  if (p.n_levels < 2 || p.n_levels > WDMG_2D_MAX_LEVELS) throw Err{WDMG_ERR_ARG, "n_levels must be 2 or 3"};
  if (p.block[0] < 1 || p.block[1] < 1) throw Err{WDMG_ERR_ARG, "block extents must be positive"};
  if (p.setup_iters < 0 || p.nu_pre < 0 || p.nu_post < 0 || !(p.omega > 0.0))
    throw Err{WDMG_ERR_ARG, "negative iteration count or non-positive omega"};
  if (p.coarse_cycles < 1 || p.coarse_cycles > 64) throw Err{WDMG_ERR_ARG, "coarse_cycles must be 1..64"};
  if (p.blocking < 0 || p.blocking > 2) throw Err{WDMG_ERR_ARG, "blocking must be 0, 1 or 2"};
  if (p.blocking && (p.n_levels != 2 || p.normal))
    throw Err{WDMG_ERR_ARG, "spin blocking is built for two-level hierarchies of D"};
  const int groups = p.blocking ? 1 : 2;
  {
    int lx = c.lx, lt = c.lt;
    for (int l = 0; l + 1 < p.n_levels; ++l) {
      if (p.nv[l] < 1 || p.nv[l] > 16) throw Err{WDMG_ERR_ARG, "nv must be 1..16"};
      if (!p.vectors[l]) throw Err{WDMG_ERR_ARG, "starting vectors required"};
      if (lx % p.block[0] || lt % p.block[1]) throw Err{WDMG_ERR_DIMS, "block extents must divide the level extents"};
      lx /= p.block[0];
      lt /= p.block[1];
      if (!smallest_divisor_ge3(lx) || !smallest_divisor_ge3(lt))
        throw Err{WDMG_ERR_DIMS, "coarse extents must be >= 3 (coloured probing)"};
      if (p.block[0] * p.block[1] * (l == 0 ? 2 / groups : p.nv[l - 1]) < p.nv[l])
        throw Err{WDMG_ERR_DIMS, "aggregate too small for nv candidates"};
    }
    const long long ncl = (long long)lx * lt * groups * p.nv[p.n_levels - 2];
    if (ncl > 4096) throw Err{WDMG_ERR_DIMS, "coarsest level above 4096 unknowns"};
  }
  drop_hierarchy(c);
  c.normal = p.normal != 0;
  c.omega = p.omega;
  c.nu_pre = p.nu_pre;
  c.nu_post = p.nu_post;
  c.use_alpha = p.use_alpha != 0;
  c.coarse_cycles = p.coarse_cycles;
  c.blocking = p.blocking;
  Lev2 L0;
  L0.lx = c.lx;
  L0.lt = c.lt;
  L0.vol = c.lx * c.lt;
  L0.g = groups;
  L0.n = 2 / groups;  // the two spins: two chirality groups of one, or one group of two
  L0.nf = (size_t)L0.vol * 2;
  c.lev.push_back(L0);
  const int blk[2] = {p.block[0], p.block[1]};
  SetupScratch scratch(c);
  for (int l = 0; l + 1 < p.n_levels; ++l) {
    const int nv = p.nv[l];
    {
      Lev2& L = c.lev[l];
      L.nv = nv;
      L.Q = calloc_fields(c, (size_t)nv * L.nf, c.hier);
      Q2_HIP(hipMemcpyAsync(L.Q, p.vectors[l], (size_t)nv * L.nf * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
      if (p.setup_iters > 0) {
        // relax A v = 0 (Sec. 2): r = -A v, then MR steps with one step size per vector
        C* R = calloc_fields(c, (size_t)nv * L.nf, scratch.bufs);
        C* T = calloc_fields(c, (size_t)nv * L.nf, scratch.bufs);
        apply_level(c, l, T, L.Q, nv);
        k_neg<<<blocks_for(nv * L.nf, 256), 256, 0, c.stream>>>(R, T, nv * L.nf);
        launch_check();
        for (int it = 0; it < p.setup_iters; ++it) {
          apply_level(c, l, T, R, nv);
          mr_update(c, L.Q, R, R, T, T, L.nf, nv, c.omega);
        }
      }
      Q2_HIP(hipMemsetAsync(c.status, 0, sizeof(int), c.stream));
      const int nagg = L.vol / (blk[0] * blk[1]) * L.g;
      k_block_qr<<<blocks_for(nagg, 64), 64, 0, c.stream>>>(L.Q, L.lx, L.lt, blk[0], blk[1], L.g, L.n, nv, c.status);
      launch_check();
      int st = 0;
      Q2_HIP(hipMemcpyAsync(&st, c.status, sizeof(int), hipMemcpyDeviceToHost, c.stream));
      Q2_HIP(hipStreamSynchronize(c.stream));
      if (st) throw Err{WDMG_ERR_RANK_DEFICIENT, "candidate vectors are rank deficient on an aggregate"};
    }
    Lev2 Cl;
    Cl.lx = c.lev[l].lx / blk[0];
    Cl.lt = c.lev[l].lt / blk[1];
    Cl.vol = Cl.lx * Cl.lt;
    Cl.g = groups;
    Cl.n = nv;
    Cl.nf = (size_t)Cl.vol * groups * nv;
    Cl.S = c.normal ? 9 : 5;
    const int N = groups * nv;
    Cl.B = calloc_fields(c, (size_t)Cl.S * Cl.vol * N * N, c.hier);
    c.lev.push_back(Cl);
    // Galerkin operator P^dagger A_l P by coloured probing
    {
      const Lev2& L = c.lev[l];
      const Lev2& Cc = c.lev[l + 1];
      const int K0 = smallest_divisor_ge3(Cc.lx), K1 = smallest_divisor_ge3(Cc.lt);
      const int np = K0 * K1 * N;
      C* probes = calloc_fields(c, (size_t)np * Cc.nf, scratch.bufs);
      C* fine = calloc_fields(c, (size_t)np * L.nf, scratch.bufs);
      C* fine2 = calloc_fields(c, (size_t)np * L.nf, scratch.bufs);
      k_probe_fill<<<blocks_for((size_t)np * Cc.nf, 256), 256, 0, c.stream>>>(probes, Cc.lx, Cc.lt, N, K0, K1);
      launch_check();
      prolong_from(c, l, fine, probes, np, blk);
      apply_level(c, l, fine2, fine, np);
      restrict_to(c, l, probes, fine2, np, blk);
      k_probe_gather<<<blocks_for((size_t)Cc.S * Cc.vol * N * N, 256), 256, 0, c.stream>>>(
          c.lev[l + 1].B, probes, Cc.lx, Cc.lt, N, Cc.S, K0, K1);
      launch_check();
    }
  }
  // the coarsest operator, inverted
  {
    const Lev2& Cc = c.lev.back();
    const int N = Cc.g * Cc.n;
    const int n = Cc.vol * N;
    c.nc = n;
    c.Maug = calloc_fields(c, (size_t)n * 2 * n, c.hier);
    c.gjcol = calloc_fields(c, (size_t)n, c.hier);
    k_dense_aug<<<blocks_for((size_t)n * 2 * n, 256), 256, 0, c.stream>>>(c.Maug, Cc.B, Cc.lx, Cc.lt, N, Cc.S);
    launch_check();
    Q2_HIP(hipMemsetAsync(c.status, 0, sizeof(int), c.stream));
    for (int k = 0; k < n; ++k) {
      k_gj_pivot<<<1, 1024, 0, c.stream>>>(c.Maug, c.gjcol, n, k, c.status);
      k_gj_elim<<<blocks_for((size_t)n * (2 * (size_t)n - k), 256), 256, 0, c.stream>>>(c.Maug, c.gjcol, n, k);
    }
    launch_check();
    int st = 0;
    Q2_HIP(hipMemcpyAsync(&st, c.status, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    Q2_HIP(hipStreamSynchronize(c.stream));
    if (st) throw Err{WDMG_ERR_NAN, "the coarsest operator is singular (zero pivot)"};
  }
  for (auto& L : c.lev) {
    L.X = calloc_fields(c, L.nf, c.hier);
    L.R = calloc_fields(c, L.nf, c.hier);
    L.T = calloc_fields(c, L.nf, c.hier);
    L.Y = calloc_fields(c, L.nf, c.hier);
    L.Bv = calloc_fields(c, L.nf, c.hier);
    L.E = calloc_fields(c, L.nf, c.hier);
    L.Rs = calloc_fields(c, L.nf, c.hier);
    L.T2 = calloc_fields(c, L.nf, c.hier);
  }
  if (c.tmp_fields > 1) free_tmp(c);  // the probes' D^dagger D work field
  ensure_tmp(c, 1);
  Q2_HIP(hipStreamSynchronize(c.stream));
  c.setup = true;
}

void need_setup(const Ctx& c) {
  if (!c.setup) throw Err{WDMG_ERR_NOT_SETUP, "no multigrid hierarchy"};
}

void check_level(const Ctx& c, int level, int lo, int hi) {
  if (level < lo || level > hi) throw Err{WDMG_ERR_ARG, "level out of range"};
}

C* solver_field(Ctx& c, int i) {
  while ((int)c.sol.size() <= i) c.sol.push_back(calloc_fields(c, (size_t)c.lx * c.lt * 2, c.bufs));
  return c.sol[i];
}

void bicgstab(Ctx& c, C* x, const C* b, double tol, int maxit, wdmg_2d_stats& st) {
  const size_t n = (size_t)c.lx * c.lt * 2;
  C *r = solver_field(c, 0), *rhat = solver_field(c, 1), *p = solver_field(c, 2), *v = solver_field(c, 3),
    *s = solver_field(c, 4), *t = solver_field(c, 5), *ph = solver_field(c, 6), *sh = solver_field(c, 7);
  Q2_HIP(hipMemsetAsync(x, 0, n * sizeof(C), c.stream));
  const double bn = std::sqrt(norm2(c, b, n));
  st.true_res = 1.0;
  if (!std::isfinite(bn)) throw Err{WDMG_ERR_NAN, "right-hand side holds NaN or Inf"};
  if (bn == 0.0) {
    st.converged = 1;
    st.true_res = 0.0;
    return;
  }
  Q2_HIP(hipMemcpyAsync(r, b, n * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
  while (st.iters < maxit) {
    Q2_HIP(hipMemcpyAsync(rhat, r, n * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
    Q2_HIP(hipMemsetAsync(v, 0, n * sizeof(C), c.stream));
    Q2_HIP(hipMemsetAsync(p, 0, n * sizeof(C), c.stream));
    k_bic_init<<<1, 1, 0, c.stream>>>(c.sc);
    launch_check();
    while (st.iters < maxit) {
      dots<M_RHO>(c, rhat, r, nullptr, nullptr, n, 1);
      k_bic_p<<<blocks_for(n, 256), 256, 0, c.stream>>>(p, r, v, c.sc, n);
      vcycle(c, 0, ph, p);
      wilson(c, v, ph, 1, false);
      dots<M_BIC_ALPHA>(c, rhat, v, nullptr, nullptr, n, 1);
      k_bic_s<<<blocks_for(n, 256), 256, 0, c.stream>>>(s, r, v, c.sc, n);
      vcycle(c, 0, sh, s);
      wilson(c, t, sh, 1, false);
      dots<M_OMEGA>(c, t, s, t, t, n, 1);
      k_bic_xr<<<blocks_for(n, 256), 256, 0, c.stream>>>(x, r, ph, sh, s, t, c.sc, n);
      launch_check();
      dots<M_NORM>(c, r, r, nullptr, nullptr, n, 1);
      read_scalars(c);
      if (c.hsc[S_FLAG].re != 0.0) break;  // breakdown: restart from the true residual
      if (!std::isfinite(c.hsc[S_RR].re)) throw Err{WDMG_ERR_NAN, "NaN or Inf in the BiCGstab residual"};
      st.iters += 1;
      const C om = c.hsc[S_OMEGA];
      if (std::sqrt(c.hsc[S_RR].re) <= tol * bn || (om.re == 0.0 && om.im == 0.0)) break;
    }
    wilson(c, t, x, 1, false);
    k_xmy<<<blocks_for(n, 256), 256, 0, c.stream>>>(r, b, t, n);
    launch_check();
    st.true_res = std::sqrt(norm2(c, r, n)) / bn;
    if (st.true_res <= tol) {
      st.converged = 1;
      return;
    }
  }
}

// Flexible CG on D^dagger D x = D^dagger b (Notay), with the V-cycle of the
// normal hierarchy (precond) or none; stopped on ||b - D x|| / ||b||.
void fcg_normal(Ctx& c, C* x, const C* b, double tol, int maxit, bool precond, wdmg_2d_stats& st) {
  const size_t n = (size_t)c.lx * c.lt * 2;
  C *r = solver_field(c, 0), *rhs = solver_field(c, 1), *p = solver_field(c, 2), *q = solver_field(c, 3),
    *z = solver_field(c, 4), *t = solver_field(c, 5);
  Q2_HIP(hipMemsetAsync(x, 0, n * sizeof(C), c.stream));
  const double bn = std::sqrt(norm2(c, b, n));
  st.true_res = 1.0;
  if (!std::isfinite(bn)) throw Err{WDMG_ERR_NAN, "right-hand side holds NaN or Inf"};
  if (bn == 0.0) {
    st.converged = 1;
    st.true_res = 0.0;
    return;
  }
  wilson(c, rhs, b, 1, true);
  const double rn = std::sqrt(norm2(c, rhs, n));
  const double tol2 = 1e-2 * tol * bn / std::max(rn, 1e-300);
  Q2_HIP(hipMemcpyAsync(r, rhs, n * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
  auto true_res = [&]() {
    wilson(c, t, x, 1, false);
    k_xmy<<<blocks_for(n, 256), 256, 0, c.stream>>>(t, b, t, n);
    launch_check();
    return std::sqrt(norm2(c, t, n)) / bn;
  };
  bool first = true;
  while (st.iters < maxit) {
    const C* zz = r;
    if (precond) {
      vcycle(c, 0, z, r);
      zz = z;
    }
    if (!first) dots<M_FCG_BETA>(c, q, zz, nullptr, nullptr, n, 1);
    k_fcg_p<<<blocks_for(n, 256), 256, 0, c.stream>>>(p, zz, c.sc, n, first ? 1 : 0);
    launch_check();
    first = false;
    normal0(c, q, p, 1);
    dots<M_FCG_ALPHA>(c, p, q, p, r, n, 1);
    k_update<<<blocks_for(n, 256), 256, 0, c.stream>>>(x, r, p, q, c.sc, S_ALPHA, n, 1);
    launch_check();
    st.iters += 1;
    const double rr = norm2(c, r, n);
    if (!std::isfinite(rr)) throw Err{WDMG_ERR_NAN, "NaN or Inf in the CG residual"};
    if (std::sqrt(rr) <= tol2 * rn) {
      st.true_res = true_res();
      if (st.true_res <= tol) {
        st.converged = 1;
        return;
      }
    }
  }
  st.true_res = true_res();
  st.converged = st.true_res <= tol;
}

template <class F>
int guard(wdmg_2d_ctx* h, F&& f) {
  if (!h) return WDMG_ERR_ARG;
  try {
    h->err.clear();
    return f(*h);
  } catch (const Err& e) {
    h->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return WDMG_ERR_OOM;
  } catch (...) {
    h->err = "unexpected error";
    return WDMG_ERR_HIP;
  }
}

}  // namespace

extern "C" {

int wdmg_2d_create(wdmg_2d_ctx** out, const int dims[2], const wdmg_alloc* alloc, void* hip_stream) {
  if (!out || !dims) return WDMG_ERR_ARG;
  *out = nullptr;
  if (dims[0] < 4 || dims[1] < 4 || (dims[0] & 1) || (dims[1] & 1)) return WDMG_ERR_DIMS;
  if (alloc && (!alloc->alloc || !alloc->free)) return WDMG_ERR_ARG;
  wdmg_2d_ctx* c = new (std::nothrow) wdmg_2d_ctx();
  if (!c) return WDMG_ERR_OOM;
  c->lx = dims[0];
  c->lt = dims[1];
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (alloc) c->alloc = *alloc;
  const int rc = guard(c, [](Ctx& cc) {
    cc.U = calloc_fields(cc, (size_t)cc.lx * cc.lt * 2, cc.bufs);
    cc.sc = calloc_fields(cc, S_TOTAL, cc.bufs);
    cc.status = static_cast<int*>(dalloc(cc, 256, cc.bufs));
    cc.part = static_cast<double*>(dalloc(cc, (size_t)kMaxDotRhs * kMaxDotGroups * 4 * sizeof(double), cc.bufs));

    Q2_HIP(hipHostMalloc(reinterpret_cast<void**>(&cc.hsc), S_TOTAL * sizeof(C), hipHostMallocDefault));
    Q2_HIP(hipMemsetAsync(cc.sc, 0, S_TOTAL * sizeof(C), cc.stream));
    return (int)WDMG_OK;
  });
  if (rc != WDMG_OK) {
    wdmg_2d_destroy(c);
    return rc;
  }
  *out = c;
  return WDMG_OK;
}

void wdmg_2d_destroy(wdmg_2d_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  release(*c, c->hier);
  release(*c, c->bufs);
  if (c->hsc) (void)hipHostFree(c->hsc);
  delete c;
}

const char* wdmg_2d_last_error(const wdmg_2d_ctx* c) { return c ? c->err.c_str() : "null context"; }

int wdmg_2d_set_gauge(wdmg_2d_ctx* h, const void* links, int t_bc) {
  return guard(h, [&](Ctx& c) {
    if (!links || (t_bc != 1 && t_bc != -1)) throw Err{WDMG_ERR_ARG, "links required, t_bc must be +1 or -1"};
    drop_hierarchy(c);
    Q2_HIP(hipMemcpyAsync(c.U, links, (size_t)c.lx * c.lt * 2 * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
    c.t_bc = t_bc;
    c.have_gauge = true;
    return (int)WDMG_OK;
  });
}

int wdmg_2d_set_mass(wdmg_2d_ctx* h, double m) {
  return guard(h, [&](Ctx& c) {
    if (!std::isfinite(m)) throw Err{WDMG_ERR_ARG, "mass must be finite"};
    drop_hierarchy(c);
    c.m = m;
    return (int)WDMG_OK;
  });
}

int wdmg_2d_apply_D(wdmg_2d_ctx* h, void* out, const void* in, int nrhs, int dagger) {
  return guard(h, [&](Ctx& c) {
    check_ready(c);
    if (!out || !in || nrhs < 1 || out == in) throw Err{WDMG_ERR_ARG, "bad buffers or nrhs"};
    wilson(c, static_cast<C*>(out), static_cast<const C*>(in), nrhs, dagger != 0);
    return (int)WDMG_OK;
  });
}

int wdmg_2d_mg_setup(wdmg_2d_ctx* h, const wdmg_2d_mg_params* p) {
  return guard(h, [&](Ctx& c) {
    if (!p) throw Err{WDMG_ERR_ARG, "params required"};
    try {
      mg_setup(c, *p);
    } catch (...) {
      drop_hierarchy(c);
      throw;
    }
    return (int)WDMG_OK;
  });
}

int wdmg_2d_get_prolongator(wdmg_2d_ctx* h, int level, void* q) {
  return guard(h, [&](Ctx& c) {
    need_setup(c);
    check_level(c, level, 0, (int)c.lev.size() - 2);
    if (!q) throw Err{WDMG_ERR_ARG, "q required"};
    const Lev2& L = c.lev[level];
    Q2_HIP(hipMemcpyAsync(q, L.Q, (size_t)L.nv * L.nf * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
    return (int)WDMG_OK;
  });
}

int wdmg_2d_apply_coarse(wdmg_2d_ctx* h, int level, void* out, const void* in, int nrhs) {
  return guard(h, [&](Ctx& c) {
    need_setup(c);
    check_level(c, level, 1, (int)c.lev.size() - 1);
    if (!out || !in || nrhs < 1 || out == in) throw Err{WDMG_ERR_ARG, "bad buffers or nrhs"};
    apply_level(c, level, static_cast<C*>(out), static_cast<const C*>(in), nrhs);
    return (int)WDMG_OK;
  });
}

int wdmg_2d_restrict(wdmg_2d_ctx* h, int level, void* out, const void* in, int nrhs) {
  return guard(h, [&](Ctx& c) {
    need_setup(c);
    check_level(c, level, 0, (int)c.lev.size() - 2);
    if (!out || !in || nrhs < 1) throw Err{WDMG_ERR_ARG, "bad buffers or nrhs"};
    int blk[2];
    blk_pair(c, level, blk);
    restrict_to(c, level, static_cast<C*>(out), static_cast<const C*>(in), nrhs, blk);
    return (int)WDMG_OK;
  });
}

int wdmg_2d_prolong(wdmg_2d_ctx* h, int level, void* out, const void* in, int nrhs) {
  return guard(h, [&](Ctx& c) {
    need_setup(c);
    check_level(c, level, 0, (int)c.lev.size() - 2);
    if (!out || !in || nrhs < 1) throw Err{WDMG_ERR_ARG, "bad buffers or nrhs"};
    int blk[2];
    blk_pair(c, level, blk);
    prolong_from(c, level, static_cast<C*>(out), static_cast<const C*>(in), nrhs, blk);
    return (int)WDMG_OK;
  });
}

int wdmg_2d_get_coarse_operator(wdmg_2d_ctx* h, int level, void* blocks) {
  return guard(h, [&](Ctx& c) {
    need_setup(c);
    check_level(c, level, 1, (int)c.lev.size() - 1);
    if (!blocks) throw Err{WDMG_ERR_ARG, "blocks required"};
    const Lev2& L = c.lev[level];
    const size_t N = (size_t)L.g * L.n;
    Q2_HIP(hipMemcpyAsync(blocks, L.B, (size_t)L.S * L.vol * N * N * sizeof(C), hipMemcpyDeviceToDevice, c.stream));
    return (int)WDMG_OK;
  });
}

int wdmg_2d_vcycle(wdmg_2d_ctx* h, void* x, const void* r) {
  return guard(h, [&](Ctx& c) {
    need_setup(c);
    if (!x || !r || x == r) throw Err{WDMG_ERR_ARG, "bad buffers"};
    vcycle(c, 0, static_cast<C*>(x), static_cast<const C*>(r));
    return (int)WDMG_OK;
  });
}

int wdmg_2d_solve(wdmg_2d_ctx* h, void* x, const void* b, int method, double tol, int maxit, wdmg_2d_stats* stats) {
  return guard(h, [&](Ctx& c) {
    check_ready(c);
    if (!x || !b || x == b || !(tol > 0.0) || maxit < 1) throw Err{WDMG_ERR_ARG, "bad buffers, tol or maxit"};
    if (method < 0 || method > 2) throw Err{WDMG_ERR_ARG, "method must be 0, 1 or 2"};
    if (method == 0 && (!c.setup || c.normal)) throw Err{WDMG_ERR_NOT_SETUP, "MG-BiCGstab needs the hierarchy of D"};
    if (method == 1 && (!c.setup || !c.normal))
      throw Err{WDMG_ERR_NOT_SETUP, "MG-CG needs the hierarchy of D^dagger D"};
    wdmg_2d_stats st{};
    c.wilson = 0;
    for (auto& a : c.capp) a = 0;
    c.flops = 0.0;
    Q2_HIP(hipStreamSynchronize(c.stream));
    const auto t0 = std::chrono::steady_clock::now();
    C* xx = static_cast<C*>(x);
    const C* bb = static_cast<const C*>(b);
    if (method == 0)
      bicgstab(c, xx, bb, tol, maxit, st);
    else
      fcg_normal(c, xx, bb, tol, maxit, method == 1, st);
    Q2_HIP(hipStreamSynchronize(c.stream));
    st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    st.wilson = c.wilson;
    for (int l = 0; l < WDMG_2D_MAX_LEVELS; ++l) st.coarse_applies[l] = c.capp[l];
    st.flops = c.flops;
    if (stats) *stats = st;
    return st.converged ? (int)WDMG_OK : (int)WDMG_NOT_CONVERGED;
  });
}

}  // extern "C"
