// Restriction P^dagger, prolongation P and the FP64 block orthonormalisation
// that builds P (Sec. 2: P V_c = V, P^dagger P = I through a QR of the
// aggregated candidates; Sec. 3: geometric aggregates with chirality kept
// intact, so R = P^dagger).
//
// P is stored as its Nv orthonormal block columns laid out like Nv fields of
// the finer level; the column (xhat, chi, k) is field k restricted to the
// aggregate xhat and to the dofs of chirality chi.  A coarse field is
// [rhs][xhat][chi * Nv + k].
//
// Level 0 fields are [12][V] over tile-major sites; chirality chi owns the
// components 6 chi .. 6 chi + 5.  Level >= 1 fields are [site][dof] with the
// two chiralities as the two halves of dof.
#include "half_field.h"
#include "internal.h"

namespace wdmg {
namespace {

constexpr int KC = 8;  // coarse columns reduced per block-wide sum

// Sites of aggregate `agg` of a level with geometry g and aggregate block b.
struct AggMap {
  Geom g;
  int b[4];
  int nb[4];   // aggregates per direction
  int bvol;
  __device__ __forceinline__ int site(int agg, int l) const {
    int a[4], lc[4];
    int t = agg;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      a[mu] = t % nb[mu];
      t /= nb[mu];
    }
    int u = l;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      lc[mu] = u % b[mu];
      u /= b[mu];
    }
    return site_of(g, a[0] * b[0] + lc[0], a[1] * b[1] + lc[1], a[2] * b[2] + lc[2], a[3] * b[3] + lc[3]);
  }
  __device__ __forceinline__ int agg_of(int s) const {
    int c[4];
    coords_of(g, s, c);
    return (c[0] / b[0]) + nb[0] * ((c[1] / b[1]) + nb[1] * ((c[2] / b[2]) + nb[2] * (c[3] / b[3])));
  }
};

AggMap make_map(const Level& f) {
  AggMap m;
  m.g = f.g;
  m.bvol = 1;
  for (int mu = 0; mu < 4; ++mu) {
    m.b[mu] = f.block[mu];
    m.nb[mu] = f.dims[mu] / f.block[mu];
    m.bvol *= f.block[mu];
  }
  return m;
}

// Row accessors: row r of the (aggregate, chirality) block -> element offset.
struct Rows0 {  // level 0: r = m * bvol + l, m in 0..5 (component within chirality)
  AggMap map;
  int nrows() const { return map.bvol * 6; }
  __device__ __forceinline__ size_t off(int agg, int chi, int r) const {
    const int m = r / map.bvol, l = r - m * map.bvol;
    return fidx(map.site(agg, l), 6 * chi + m, 12);
  }
};
struct RowsC {  // level >= 1: r = d * bvol + l, d in 0..half-1
  AggMap map;
  int dof;
  int nrows() const { return map.bvol * (dof / 2); }
  __device__ __forceinline__ size_t off(int agg, int chi, int r) const {
    const int d = r / map.bvol, l = r - d * map.bvol;
    return (size_t)map.site(agg, l) * dof + chi * (dof / 2) + d;
  }
};

// Workgroup -> (aggregate, rhs) for a one-dimensional grid of nagg * nrhs
// workgroups.  The hardware sends workgroup b to XCD b % 8; the mapping gives
// every XCD a contiguous run of aggregates and runs all right-hand sides of
// an aggregate back to back there, so its P columns come from HBM once and
// are re-read from that XCD's L2.
__device__ __forceinline__ void agg_rhs_block(int nagg, int nrhs, int& agg, int& rhs) {
  const int b = blockIdx.x;
  if (nagg & 7) {
    agg = b % nagg;
    rhs = b / nagg;
    return;
  }
  const int xcd = b & 7, local = b >> 3;
  agg = xcd * (nagg >> 3) + local / nrhs;
  rhs = local % nrhs;
}

// ---- restriction: one workgroup per (aggregate, rhs, column range) ---------
// The nv columns of an aggregate are split into nsplit ranges of kper columns
// so that a single right-hand side still fills the chip; the ranges of one
// (aggregate, rhs) run back to back on one XCD and re-read the fine field
// from its L2.
template <typename R, class Rows>
__global__ __launch_bounds__(256) void k_restrict(Rows rows, int nrows, const cx<R>* __restrict__ Vv, size_t vstride,
                                                  const cx<R>* __restrict__ in, size_t fstride, cx<R>* __restrict__ out,
                                                  int nagg, int nv, int nsplit, int kper) {
  __shared__ double lds[4 * KC * 4];
  int agg, item;
  agg_rhs_block(nagg, gridDim.x / nagg, agg, item);
  const int rhs = item / nsplit, split = item % nsplit;
  const int kbeg = split * kper, kend = min(nv, kbeg + kper);
  in += (size_t)rhs * fstride;
  out += ((size_t)rhs * nagg + agg) * 2 * nv;
  for (int k0 = kbeg; k0 < kend; k0 += KC) {
    double v[4 * KC];
#pragma unroll
    for (int q = 0; q < 4 * KC; ++q) v[q] = 0.0;
    for (int chi = 0; chi < 2; ++chi) {
      for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
        const size_t o = rows.off(agg, chi, r);
        const cx<R> f = in[o];
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          if (k0 + q < kend) {
            const cx<R> w = Vv[(size_t)(k0 + q) * vstride + o];
            v[4 * q + 2 * chi] += (double)w.re * f.re + (double)w.im * f.im;
            v[4 * q + 2 * chi + 1] += (double)w.re * f.im - (double)w.im * f.re;
          }
        }
      }
    }
    block_sum<4 * KC>(v, lds);
    if (threadIdx.x == 0) {
      for (int q = 0; q < KC && k0 + q < kend; ++q) {
        out[k0 + q] = mk<R>((R)v[4 * q], (R)v[4 * q + 1]);
        out[nv + k0 + q] = mk<R>((R)v[4 * q + 2], (R)v[4 * q + 3]);
      }
    }
  }
}

constexpr int RB = 8;  // right-hand sides per workgroup in the batched prolongation

// ---- prolongation of a batch at level 0: V read once for RB rhs -----------
template <typename R>
__global__ __launch_bounds__(256) void k_prolong0_b(AggMap map, const cx<R>* __restrict__ Vv,
                                                    const cx<R>* __restrict__ in, cx<R>* __restrict__ out, int nagg,
                                                    int nv, int nrhs, int nsb) {
  int sb, grp;
  agg_rhs_block(nsb, gridDim.x / nsb, sb, grp);
  const int s = sb * blockDim.x + threadIdx.x;
  const int r0 = grp * RB;
  const int nr = min(RB, nrhs - r0);
  const size_t n = (size_t)12 * map.g.vpad;
  if (s >= map.g.vpad) return;
  const int agg = s < map.g.vol ? map.agg_of(s) : 0;
  for (int m = 0; m < 12; ++m) {
    cx<R> acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = mk<R>(0, 0);
    if (s < map.g.vol) {
      const int chi = m / 6;
      for (int k = 0; k < nv; ++k) {
        const cx<R> w = Vv[(size_t)k * n + fidx(s, m, 12)];
#pragma unroll
        for (int q = 0; q < RB; ++q)
          if (q < nr) cmadd(acc[q], w, in[((size_t)(r0 + q) * nagg + agg) * 2 * nv + chi * nv + k]);
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (q < nr) out[(size_t)(r0 + q) * n + fidx(s, m, 12)] = acc[q];
  }
}

// ---- prolongation: one thread per (row of a finer-level field) ------------
template <typename R>
__global__ __launch_bounds__(256) void k_prolong0(AggMap map, const cx<R>* __restrict__ Vv, const cx<R>* __restrict__ in,
                                                  cx<R>* __restrict__ out, int nagg, int nv) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  const size_t n = (size_t)12 * map.g.vpad;
  if (s >= map.g.vpad) return;
  cx<R>* o = out + (size_t)rhs * n;
  cx<R> acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = mk<R>(0, 0);
  if (s < map.g.vol) {
    const int agg = map.agg_of(s);
    const cx<R>* ec = in + ((size_t)rhs * nagg + agg) * 2 * nv;
    for (int k = 0; k < nv; ++k) {
      const cx<R> e0 = ec[k], e1 = ec[nv + k];
      const cx<R>* vk = Vv + (size_t)k * n;
#pragma unroll
      for (int m = 0; m < 6; ++m) cmadd(acc[m], vk[fidx(s, m, 12)], e0);
#pragma unroll
      for (int m = 6; m < 12; ++m) cmadd(acc[m], vk[fidx(s, m, 12)], e1);
    }
  }
#pragma unroll
  for (int m = 0; m < 12; ++m) o[fidx(s, m, 12)] = acc[m];
}

template <typename R>
__global__ __launch_bounds__(256) void k_prolongC(AggMap map, int dof, const cx<R>* __restrict__ Vv,
                                                  const cx<R>* __restrict__ in, cx<R>* __restrict__ out, int nagg,
                                                  int nv) {
  const size_t nsite = map.g.vol;
  const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (idx >= nsite * dof) return;
  const int s = (int)(idx / dof), e = (int)(idx % dof);
  const int chi = e >= dof / 2;
  const int agg = map.agg_of(s);
  const cx<R>* ec = in + ((size_t)rhs * nagg + agg) * 2 * nv + chi * nv;
  const size_t vstride = nsite * dof;
  cx<R> acc = mk<R>(0, 0);
  for (int k = 0; k < nv; ++k) cmadd(acc, Vv[(size_t)k * vstride + idx], ec[k]);
  out[(size_t)rhs * vstride + idx] = acc;
}

// ---- level 0 with 16-bit fine fields and prolongator columns ----------------
// Restriction: one workgroup per (aggregate, rhs) as above; values are read
// as scale(site) x stored value, P columns unscaled.
template <typename H>
__global__ __launch_bounds__(256) void k_restrict0_h(Rows0 rows, int nrows, const cxh<H>* __restrict__ Vv,
                                                     size_t vstride, const cxh<H>* __restrict__ in,
                                                     const float* __restrict__ isc, cx<float>* __restrict__ out,
                                                     int nagg, int nv, int vpad) {
  __shared__ double lds[4 * KC * 4];
  int agg, rhs;
  agg_rhs_block(nagg, gridDim.x / nagg, agg, rhs);
  in += (size_t)rhs * 12 * vpad;
  isc += (size_t)rhs * vpad;
  out += ((size_t)rhs * nagg + agg) * 2 * nv;
  const int bvol = rows.map.bvol;
  for (int k0 = 0; k0 < nv; k0 += KC) {
    double v[4 * KC];
#pragma unroll
    for (int q = 0; q < 4 * KC; ++q) v[q] = 0.0;
    for (int chi = 0; chi < 2; ++chi) {
      for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
        const int m = r / bvol, l = r - m * bvol;
        const int site = rows.map.site(agg, l);
        const size_t o = fidx(site, 6 * chi + m, 12);
        const float sc = isc[site];
        const cx<float> q16 = h2f(in[o]);
        const cx<float> f = mk(sc * q16.re, sc * q16.im);
#pragma unroll
        for (int q = 0; q < KC; ++q) {
          if (k0 + q < nv) {
            const cx<float> w = h2f(Vv[(size_t)(k0 + q) * vstride + o]);
            v[4 * q + 2 * chi] += (double)w.re * f.re + (double)w.im * f.im;
            v[4 * q + 2 * chi + 1] += (double)w.re * f.im - (double)w.im * f.re;
          }
        }
      }
    }
    block_sum<4 * KC>(v, lds);
    if (threadIdx.x == 0) {
      for (int q = 0; q < KC && k0 + q < nv; ++q) {
        out[k0 + q] = mk((float)v[4 * q], (float)v[4 * q + 1]);
        out[nv + k0 + q] = mk((float)v[4 * q + 2], (float)v[4 * q + 3]);
      }
    }
  }
}

// Prolongation into a 16-bit field: one thread per site and RBH right-hand
// sides (each site's 12 components are needed together for its scale).
constexpr int RBH = 4;
template <typename H>
__global__ __launch_bounds__(256) void k_prolong0_h(AggMap map, const cxh<H>* __restrict__ Vv,
                                                    const cx<float>* __restrict__ in, cxh<H>* __restrict__ out,
                                                    float* __restrict__ osc, int nagg, int nv, int nrhs, int nsb) {
  int sb, grp;
  agg_rhs_block(nsb, gridDim.x / nsb, sb, grp);
  const int s = sb * blockDim.x + threadIdx.x;
  const int r0 = grp * RBH;
  const int nr = min(RBH, nrhs - r0);
  const int vpad = map.g.vpad;
  const size_t n = (size_t)12 * vpad;
  if (s >= vpad) return;
  cx<float> acc[RBH][12];
#pragma unroll
  for (int q = 0; q < RBH; ++q)
#pragma unroll
    for (int m = 0; m < 12; ++m) acc[q][m] = mk(0.0f, 0.0f);
  if (s < map.g.vol) {
    const int agg = map.agg_of(s);
    for (int k = 0; k < nv; ++k) {
      cx<float> w[12];
#pragma unroll
      for (int m = 0; m < 12; ++m) w[m] = h2f(Vv[(size_t)k * n + fidx(s, m, 12)]);
#pragma unroll
      for (int q = 0; q < RBH; ++q) {
        if (q < nr) {
          const cx<float>* ec = in + ((size_t)(r0 + q) * nagg + agg) * 2 * nv;
          const cx<float> e0 = ec[k], e1 = ec[nv + k];
#pragma unroll
          for (int m = 0; m < 6; ++m) cmadd(acc[q][m], w[m], e0);
#pragma unroll
          for (int m = 6; m < 12; ++m) cmadd(acc[q][m], w[m], e1);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < RBH; ++q)
    if (q < nr) store_site_h(out + (size_t)(r0 + q) * n, osc + (size_t)(r0 + q) * vpad, s, acc[q]);
}

// ---- batched restriction on the matrix cores (FP32 arithmetic) ----------------
// For a batch of right-hand sides P^dagger is, per (aggregate, chirality), the
// complex GEMM out[k][q] = sum_row conj(V[row][k]) f[row][q]; it runs as the
// real GEMM with rows (k, re|im) and the contraction over (row, re|im):
//   A[(k,0)][(r,0)] = Re v, A[(k,0)][(r,1)] = Im v, A[(k,1)][(r,0)] = -Im v,
//   A[(k,1)][(r,1)] = Re v;  B[(r,0)][q] = Re f, B[(r,1)][q] = Im f.
// Workgroup = one aggregate and up to 32 right-hand sides; wave w handles
// chirality w / 2 and output row tile w % 2 (32 real rows, 2 Nv <= 64).
// Chunks of 64 rows (one spin-colour component on 64 aggregate sites) of V
// and of the fields are staged in LDS with coalesced loads, then fed to
// v_mfma_f32_32x32x2f32 (lanes as in the coarse-operator kernel).
// Operand loaders of the batched restriction: raw() issues the load, conv()
// turns its result into FP32 (kept apart so a load can be in flight while
// matrix-core work runs, and converted only when it is stored to LDS).
struct FieldF32 {  // plain FP32 fine fields [rhs][12 vpad]
  const cx<float>* f;
  int vpad;
  using Raw = cx<float>;
  __device__ __forceinline__ Raw raw(int q, int site, int comp) const {
    return f[(size_t)q * 12 * vpad + fidx(site, comp, 12)];
  }
  __device__ __forceinline__ static cx<float> conv(Raw r) { return r; }
};
template <typename H>
struct FieldH {  // 16-bit fine fields with per-site scales
  const cxh<H>* v;
  const float* sc;
  int vpad;
  struct Raw {
    cxh<H> x;
    float s;
  };
  __device__ __forceinline__ Raw raw(int q, int site, int comp) const {
    return {v[(size_t)q * 12 * vpad + fidx(site, comp, 12)], sc[(size_t)q * vpad + site]};
  }
  __device__ __forceinline__ static cx<float> conv(Raw r) {
    const cx<float> x = h2f(r.x);
    return mk(r.s * x.re, r.s * x.im);
  }
};
struct VF32 {
  const cx<float>* v;
  size_t stride;
  using Raw = cx<float>;
  __device__ __forceinline__ Raw raw(int k, size_t off) const { return v[(size_t)k * stride + off]; }
  __device__ __forceinline__ static cx<float> conv(Raw r) { return r; }
};
template <typename H>
struct VH {
  const cxh<H>* v;
  size_t stride;
  using Raw = cxh<H>;
  __device__ __forceinline__ Raw raw(int k, size_t off) const { return v[(size_t)k * stride + off]; }
  __device__ __forceinline__ static cx<float> conv(Raw r) { return h2f(r); }
};

typedef float floatx16_t __attribute__((ext_vector_type(16)));

template <class VL, class FL>
__global__ __launch_bounds__(256) void k_restrict0_mfma(AggMap map, VL V, FL F, cx<float>* __restrict__ out,
                                                        int nagg, int nv, int nrhs) {
  __shared__ cx<float> Vs[2][64][33];
  __shared__ cx<float> Fs[2][64][33];
  int agg, tile;
  agg_rhs_block(nagg, gridDim.x / nagg, agg, tile);
  const int q0 = tile * 32, nq = min(32, nrhs - q0);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int chi = w >> 1, rt = w & 1;
  const int i = rt * 32 + (l & 31), kidx = i >> 1, part = i & 1;
  const int q = l & 31;
  floatx16_t acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  const int per = map.bvol / 64;
  // Staging: for chunk c (component pair m, 64 sites from l0) thread t loads
  // site l0 + (t & 63), columns k = t / 64 + 4u and rhs q0 + t / 64 + 4u
  // (nv, nq <= 32: u < 8).  The loads of chunk c + 1 are issued before the
  // matrix-core work of chunk c and stored to LDS after it.
  const int ll = threadIdx.x & 63, grp = threadIdx.x >> 6;
  typename VL::Raw vr[2][8];
  typename FL::Raw fr[2][8];
  auto load = [&](int c) {
    const int m = c / per, l0 = (c % per) * 64;
    const int site = map.site(agg, l0 + ll);
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
      const size_t off = fidx(site, 6 * ch + m, 12);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (grp + 4 * u < nv) vr[ch][u] = V.raw(grp + 4 * u, off);
        if (grp + 4 * u < nq) fr[ch][u] = F.raw(q0 + grp + 4 * u, site, 6 * ch + m);
      }
    }
  };
  load(0);
  for (int c = 0; c < 6 * per; ++c) {
    __syncthreads();
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (grp + 4 * u < nv) Vs[ch][ll][grp + 4 * u] = VL::conv(vr[ch][u]);
        if (grp + 4 * u < nq) Fs[ch][ll][grp + 4 * u] = FL::conv(fr[ch][u]);
      }
    }
    __syncthreads();
    if (c + 1 < 6 * per) load(c + 1);
#pragma unroll 4
    for (int kk = 0; kk < 128; kk += 2) {
      const int kr = kk + (l >> 5), r = kr >> 1, pk = kr & 1;
      float a = 0.f, b = 0.f;
      if (kidx < nv) {
        const cx<float> v = Vs[chi][r][kidx];
        a = part == 0 ? (pk == 0 ? v.re : v.im) : (pk == 0 ? -v.im : v.re);
      }
      if (q < nq) {
        const cx<float> fv = Fs[chi][r][q];
        b = pk == 0 ? fv.re : fv.im;
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  }
  // D[i][q] in lane q + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4
  if (q < nq) {
    float* o = reinterpret_cast<float*>(out + ((size_t)(q0 + q) * nagg + agg) * 2 * nv + chi * nv);
#pragma unroll
    for (int reg = 0; reg < 16; ++reg) {
      const int ii = rt * 32 + 8 * (reg >> 2) + 4 * (l >> 5) + (reg & 3);
      if ((ii >> 1) < nv) o[ii] = acc[reg];
    }
  }
}

// ---- block orthonormalisation (FP64): CGS with a second pass --------------
// One workgroup per (aggregate, chirality); column j is orthogonalised
// against columns 0..j-1 twice, then normalised by its (real, positive) norm,
// which makes diag(R) real positive and Q unique.
template <class Rows>
__global__ __launch_bounds__(256) void k_block_qr(Rows rows, int nrows, cx<double>* Vv, size_t vstride, int nv,
                                                  double* dsc) {
  __shared__ double lds[2 * KC * 4];
  __shared__ double coef[2 * 64];
  __shared__ double scal;
  const int agg = blockIdx.x, chi = blockIdx.y;
  for (int j = 0; j < nv; ++j) {
    cx<double>* vj = Vv + (size_t)j * vstride;
    double n0[1] = {0.0};
    for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
      const cx<double> a = vj[rows.off(agg, chi, r)];
      n0[0] += a.re * a.re + a.im * a.im;
    }
    block_sum<1>(n0, lds);
    if (threadIdx.x == 0) scal = sqrt(n0[0]);
    __syncthreads();
    const double norm0 = scal;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int i0 = 0; i0 < j; i0 += KC) {
        double v[2 * KC];
#pragma unroll
        for (int q = 0; q < 2 * KC; ++q) v[q] = 0.0;
        for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
          const size_t o = rows.off(agg, chi, r);
          const cx<double> a = vj[o];
#pragma unroll
          for (int q = 0; q < KC; ++q) {
            if (i0 + q < j) {
              const cx<double> b = Vv[(size_t)(i0 + q) * vstride + o];
              v[2 * q] += b.re * a.re + b.im * a.im;
              v[2 * q + 1] += b.re * a.im - b.im * a.re;
            }
          }
        }
        block_sum<2 * KC>(v, lds);
        if (threadIdx.x == 0) {
          for (int q = 0; q < 2 * KC; ++q) coef[2 * i0 + q] = v[q];
        }
        __syncthreads();
      }
      for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
        const size_t o = rows.off(agg, chi, r);
        cx<double> a = vj[o];
        for (int i = 0; i < j; ++i) a = a - mk(coef[2 * i], coef[2 * i + 1]) * Vv[(size_t)i * vstride + o];
        vj[o] = a;
      }
      __syncthreads();
    }
    double n1[1] = {0.0};
    for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
      const cx<double> a = vj[rows.off(agg, chi, r)];
      n1[0] += a.re * a.re + a.im * a.im;
    }
    block_sum<1>(n1, lds);
    if (threadIdx.x == 0) {
      const double nr = sqrt(n1[0]);
      if (!(nr > 1e-12 * norm0)) dsc[S_ERR + 1] = 1.0;  // rank lost (or NaN)
      scal = nr > 0.0 ? 1.0 / nr : 0.0;
    }
    __syncthreads();
    const double inv = scal;
    for (int r = threadIdx.x; r < nrows; r += blockDim.x) {
      const size_t o = rows.off(agg, chi, r);
      const cx<double> a = vj[o];
      vj[o] = mk(a.re * inv, a.im * inv);
    }
    __syncthreads();
  }
}

inline int nagg_of(const Level& f) {
  int n = 1;
  for (int mu = 0; mu < 4; ++mu) n *= f.dims[mu] / f.block[mu];
  return n;
}

inline int tpb_for(int nrows) {
  int t = ((nrows + 63) / 64) * 64;
  return t > 256 ? 256 : t;
}

// Column ranges per (aggregate, rhs) of k_restrict: enough workgroups to
// fill the chip (about 2048), ranges of at least one column.
struct RestrictSplit {
  int nsplit, kper;
};
inline RestrictSplit restrict_split(int nagg, int nrhs, int nv) {
  const long long have = (long long)nagg * nrhs;
  int want = (int)((2048 + have - 1) / have);
  if (want > nv) want = nv;
  if (want < 1) want = 1;
  const int kper = (nv + want - 1) / want;
  return {(nv + kper - 1) / kper, kper};
}

}  // namespace

template <typename R>
void restrict0(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs) {
  if constexpr (sizeof(R) == 4) {
    const AggMap map = make_map(f);
    if (nrhs >= 2 && map.bvol % 64 == 0 && f.nv <= 32) {
      const int nagg = nagg_of(f);
      ProfScope ps(c, WDMG_K_RESTRICT_F32, (long long)f.nsite * nrhs);
      hipLaunchKernelGGL((k_restrict0_mfma<VF32, FieldF32>), dim3(nagg * ((nrhs + 31) / 32)), dim3(256), 0,
                         c.stream, map, VF32{V, f.n}, FieldF32{in, f.g.vpad}, out, nagg, f.nv, nrhs);
      WDMG_HIP(hipGetLastError());
      return;
    }
  }
  Rows0 rows{make_map(f)};
  const int nrows = rows.nrows();
  const int nagg = nagg_of(f);
  // (one workgroup per (aggregate, rhs): measured faster than reading V once
  // per rhs chunk, because the chunked form re-reads the fine fields per column)
  ProfScope ps(c, sizeof(R) == 8 ? WDMG_K_RESTRICT_F64 : WDMG_K_RESTRICT_F32, (long long)f.nsite * nrhs);
  const RestrictSplit sp = restrict_split(nagg, nrhs, f.nv);
  hipLaunchKernelGGL((k_restrict<R, Rows0>), dim3(nagg * nrhs * sp.nsplit), dim3(tpb_for(nrows)), 0, c.stream, rows,
                     nrows, V, f.n, in, f.n, out, nagg, f.nv, sp.nsplit, sp.kper);
  WDMG_HIP(hipGetLastError());
}

template <typename R>
void restrictC(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs) {
  RowsC rows{make_map(f), f.dof};
  const int nrows = rows.nrows();
  const int nagg = nagg_of(f);

  const RestrictSplit sp = restrict_split(nagg, nrhs, f.nv);
  hipLaunchKernelGGL((k_restrict<R, RowsC>), dim3(nagg * nrhs * sp.nsplit), dim3(tpb_for(nrows)), 0, c.stream, rows,
                     nrows, V, f.n, in, f.n, out, nagg, f.nv, sp.nsplit, sp.kper);
  WDMG_HIP(hipGetLastError());
}

template <typename R>
void prolong0(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs) {
  const AggMap map = make_map(f);
  if (nrhs > 1) {
    ProfScope ps(c, sizeof(R) == 8 ? WDMG_K_PROLONG_F64 : WDMG_K_PROLONG_F32, (long long)f.nsite * nrhs);
    const int nsb = (f.g.vpad + 255) / 256;
    hipLaunchKernelGGL((k_prolong0_b<R>), dim3(nsb * ((nrhs + RB - 1) / RB)), dim3(256), 0, c.stream, map, V, in,
                       out, nagg_of(f), f.nv, nrhs, nsb);
    WDMG_HIP(hipGetLastError());
    return;
  }
  ProfScope ps(c, sizeof(R) == 8 ? WDMG_K_PROLONG_F64 : WDMG_K_PROLONG_F32, (long long)f.nsite * nrhs);
  hipLaunchKernelGGL((k_prolong0<R>), dim3((f.g.vpad + 255) / 256, nrhs), dim3(256), 0, c.stream, map, V, in, out,
                     nagg_of(f), f.nv);
  WDMG_HIP(hipGetLastError());
}

template <typename R>
void prolongC(Ctx& c, const Level& f, const cx<R>* V, const cx<R>* in, cx<R>* out, int nrhs) {
  const AggMap map = make_map(f);
  hipLaunchKernelGGL((k_prolongC<R>), dim3((unsigned)((f.n + 255) / 256), nrhs), dim3(256), 0, c.stream, map, f.dof,
                     V, in, out, nagg_of(f), f.nv);
  WDMG_HIP(hipGetLastError());
}

template <typename H>
void restrict0_h(Ctx& c, const Level& f, const void* V16, HF in, cx<float>* out, int nrhs) {
  {
    const AggMap map = make_map(f);
    if (nrhs >= 2 && map.bvol % 64 == 0 && f.nv <= 32) {
      const int nagg = nagg_of(f);
      ProfScope ps(c, WDMG_K_RESTRICT_H, (long long)f.nsite * nrhs);
      hipLaunchKernelGGL((k_restrict0_mfma<VH<H>, FieldH<H>>), dim3(nagg * ((nrhs + 31) / 32)), dim3(256), 0,
                         c.stream, map, VH<H>{static_cast<const cxh<H>*>(V16), f.n},
                         FieldH<H>{static_cast<const cxh<H>*>(in.v), in.s, f.g.vpad}, out, nagg, f.nv, nrhs);
      WDMG_HIP(hipGetLastError());
      return;
    }
  }
  Rows0 rows{make_map(f)};
  const int nrows = rows.nrows();
  const int nagg = nagg_of(f);
  ProfScope ps(c, WDMG_K_RESTRICT_H, (long long)f.nsite * nrhs);
  hipLaunchKernelGGL((k_restrict0_h<H>), dim3(nagg * nrhs), dim3(tpb_for(nrows)), 0, c.stream, rows, nrows,
                     static_cast<const cxh<H>*>(V16), f.n, static_cast<const cxh<H>*>(in.v), in.s, out, nagg, f.nv,
                     f.g.vpad);
  WDMG_HIP(hipGetLastError());
}

template <typename H>
void prolong0_h(Ctx& c, const Level& f, const void* V16, const cx<float>* in, HF out, int nrhs) {
  const AggMap map = make_map(f);
  ProfScope ps(c, WDMG_K_PROLONG_H, (long long)f.nsite * nrhs);
  const int nsb = (f.g.vpad + 255) / 256;
  hipLaunchKernelGGL((k_prolong0_h<H>), dim3(nsb * ((nrhs + RBH - 1) / RBH)), dim3(256), 0, c.stream, map,
                     static_cast<const cxh<H>*>(V16), in, static_cast<cxh<H>*>(out.v), out.s, nagg_of(f), f.nv, nrhs,
                     nsb);
  WDMG_HIP(hipGetLastError());
}

template void restrict0_h<f16_t>(Ctx&, const Level&, const void*, HF, cx<float>*, int);
template void restrict0_h<bf16_t>(Ctx&, const Level&, const void*, HF, cx<float>*, int);
template void prolong0_h<f16_t>(Ctx&, const Level&, const void*, const cx<float>*, HF, int);
template void prolong0_h<bf16_t>(Ctx&, const Level&, const void*, const cx<float>*, HF, int);

void block_qr0(Ctx& c, const Level& f, cx<double>* V) {
  Rows0 rows{make_map(f)};
  const int nrows = rows.nrows();
  ProfScope ps(c, WDMG_K_BLOCK_QR, (long long)nagg_of(f) * 2);
  hipLaunchKernelGGL((k_block_qr<Rows0>), dim3(nagg_of(f), 2), dim3(tpb_for(nrows)), 0, c.stream, rows, nrows, V, f.n,
                     f.nv, c.dsc);
  WDMG_HIP(hipGetLastError());
}

void block_qrC(Ctx& c, const Level& f, cx<double>* V) {
  RowsC rows{make_map(f), f.dof};
  const int nrows = rows.nrows();
  hipLaunchKernelGGL((k_block_qr<RowsC>), dim3(nagg_of(f), 2), dim3(tpb_for(nrows)), 0, c.stream, rows, nrows, V, f.n,
                     f.nv, c.dsc);
  WDMG_HIP(hipGetLastError());
}

#define INST(R)                                                                                 \
  template void restrict0<R>(Ctx&, const Level&, const cx<R>*, const cx<R>*, cx<R>*, int);     \
  template void restrictC<R>(Ctx&, const Level&, const cx<R>*, const cx<R>*, cx<R>*, int);     \
  template void prolong0<R>(Ctx&, const Level&, const cx<R>*, const cx<R>*, cx<R>*, int);      \
  template void prolongC<R>(Ctx&, const Level&, const cx<R>*, const cx<R>*, cx<R>*, int);
INST(double)
INST(float)
#undef INST

}  // namespace wdmg
