// Device-side building blocks shared by every kernel of libwdmg (gfx950).
//
// * cx<R>: complex number, 8- or 16-byte aligned so a wavefront's loads of
//   consecutive elements coalesce into full 64-lane transactions.
// * Geom: lattice geometry of one multigrid level.  The fine level is stored
//   tile-major: the lattice is cut into (Bx,By,Bz,Bt) tiles (the 4^4
//   aggregates of the multigrid, Sec. 3), tiles are numbered
//   lexicographically and sites inside a tile lexicographically, so an
//   aggregate's sites are one contiguous run of every field.  Coarse levels
//   use B = 1 (plain lexicographic order).
// * wave / block reductions with a fixed summation order (deterministic).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wdmg {

template <typename R>
struct __align__(2 * sizeof(R)) cx {
  R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) {
  cx<R> z;
  z.re = a;
  z.im = b;
  return z;
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return mk(s * a.re, s * a.im); }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// acc += a * b
template <typename R>
__host__ __device__ __forceinline__ void cmadd(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ void cmaddc(cx<R>& acc, cx<R> a, cx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
// i * a and -i * a
template <typename R>
__host__ __device__ __forceinline__ cx<R> ti(cx<R> a) { return mk(-a.im, a.re); }
template <typename R>
__host__ __device__ __forceinline__ cx<R> tmi(cx<R> a) { return mk(a.im, -a.re); }

template <typename Rout, typename Rin>
__host__ __device__ __forceinline__ cx<Rout> cvt(cx<Rin> a) {
  return mk((Rout)a.re, (Rout)a.im);
}

// ---------------------------------------------------------------------------
// Geometry.
struct Geom {
  int L[4];    // extents x, y, z, t
  int B[4];    // tile extents (1, 2 or 4)
  int lb[4];   // log2 B
  int nT[4];   // tiles per direction
  int sl[4];   // stride of a local coordinate inside a tile
  int st[4];   // stride (in sites) of a tile coordinate
  int vol;     // sites
  int vpad;    // sites rounded up to a multiple of 64 (fine-field blocks)
  int tvol;    // sites per tile
  int ltvol;   // log2 tvol
};

struct Coord {
  int c[4];   // global coordinates
};

__host__ __device__ __forceinline__ int site_of(const Geom& g, int x, int y, int z, int t) {
  const int c[4] = {x, y, z, t};
  int tile = 0, loc = 0;
#pragma unroll
  for (int mu = 3; mu >= 0; --mu) {
    const int tc = c[mu] >> g.lb[mu];
    const int lc = c[mu] & (g.B[mu] - 1);
    tile = tile * g.nT[mu] + tc;
    loc += lc * g.sl[mu];
  }
  return (tile << g.ltvol) + loc;
}

__host__ __device__ __forceinline__ void coords_of(const Geom& g, int s, int c[4]) {
  int tile = s >> g.ltvol;
  const int loc = s & (g.tvol - 1);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int tc = tile % g.nT[mu];
    tile /= g.nT[mu];
    const int lc = (loc >> (g.lb[0] * (mu > 0) + g.lb[1] * (mu > 1) + g.lb[2] * (mu > 2))) & (g.B[mu] - 1);
    c[mu] = (tc << g.lb[mu]) + lc;
  }
}

// Neighbour of site s (with coordinates c) one step forward / backward in mu,
// periodic.  No division: local step inside the tile, else tile step.
__host__ __device__ __forceinline__ int nbr_fwd(const Geom& g, int s, const int c[4], int mu) {
  const int lc = c[mu] & (g.B[mu] - 1);
  if (lc < g.B[mu] - 1) return s + g.sl[mu];
  s -= (g.B[mu] - 1) * g.sl[mu];
  const int tc = c[mu] >> g.lb[mu];
  return (tc < g.nT[mu] - 1) ? s + g.st[mu] : s - (g.nT[mu] - 1) * g.st[mu];
}

__host__ __device__ __forceinline__ int nbr_bwd(const Geom& g, int s, const int c[4], int mu) {
  const int lc = c[mu] & (g.B[mu] - 1);
  if (lc > 0) return s - g.sl[mu];
  s += (g.B[mu] - 1) * g.sl[mu];
  const int tc = c[mu] >> g.lb[mu];
  return (tc > 0) ? s - g.st[mu] : s + (g.nT[mu] - 1) * g.st[mu];
}

// ---------------------------------------------------------------------------
// Reductions (wave64).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sums K values over the block; the result is valid in thread 0.  `lds` must
// hold K * (blockDim.x / 64) doubles.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[wave * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += lds[w * K + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Load that bypasses the (non-coherent) per-CU vector L1, for data written by
// other workgroups of the same launch.
__device__ __forceinline__ double load_coherent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace wdmg
