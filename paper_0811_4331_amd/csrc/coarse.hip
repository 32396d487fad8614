// Galerkin coarse operator D_c = P^dagger D P (Sec. 2) as a nearest-neighbour
// stencil of dense complex (2Nv x 2Nv) blocks, and its application.
//
// Storage per coarse site: nine blocks, column-major ([col][row]), in the
// order d = 2 mu (Y_{+mu}, couples to xhat + mu), d = 2 mu + 1 (Y_{-mu},
// couples to xhat - mu), d = 8 (X, the site itself).
//
// Build: a fine-level coupling that leaves an aggregate through its +-mu face
// lands in Y_{+-mu}; every other coupling (the diagonal term and the hops
// that stay inside the aggregate) lands in X.  Each workgroup computes one
// block of one coarse site: it applies the fine hops to the chirality-split
// columns of P at a few sites at a time (staged in LDS) and contracts them
// with the conjugated columns, all in FP64.
#include <type_traits>

#include "half_field.h"
#include "internal.h"
#include "wilson_spin.h"

namespace wdmg {
namespace {

constexpr int kMfmaMinRhs = 2;  // batches of at least this many rhs use the matrix cores

struct AggGeom {
  Geom g;       // geometry of the finer level
  int b[4];     // aggregate extents
  int nb[4];    // aggregates per direction
  int bvol;
};

AggGeom make_agg(const Level& f) {
  AggGeom a;
  a.g = f.g;
  a.bvol = 1;
  for (int mu = 0; mu < 4; ++mu) {
    a.b[mu] = f.block[mu];
    a.nb[mu] = f.dims[mu] / f.block[mu];
    a.bvol *= f.block[mu];
  }
  return a;
}

// Global coordinates of local site `i` of the sites visited for block d of
// aggregate `agg`: the whole aggregate for d = 8, else its (mu, sign) face.
__device__ __forceinline__ void block_site(const AggGeom& a, int agg, int d, int i, int c[4]) {
  int base[4];
  int t = agg;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    base[mu] = (t % a.nb[mu]) * a.b[mu];
    t /= a.nb[mu];
  }
  const int fmu = d < 8 ? (d >> 1) : -1;
  int u = i;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    int lc;
    if (mu == fmu) {
      lc = (d & 1) ? 0 : a.b[mu] - 1;
    } else {
      lc = u % a.b[mu];
      u /= a.b[mu];
    }
    c[mu] = base[mu] + lc;
  }
}

__device__ __forceinline__ int nsites_of_block(const AggGeom& a, int d) {
  return d < 8 ? a.bvol / a.b[d >> 1] : a.bvol;
}

// Is the hop (mu, dir) from coordinates c inside the aggregate?
__device__ __forceinline__ bool inside(const AggGeom& a, const int c[4], int mu, int dir) {
  const int lc = c[mu] % a.b[mu];
  return dir > 0 ? (lc < a.b[mu] - 1) : (lc > 0);
}

// ---- level 0: Wilson hops ---------------------------------------------------
template <int MU, int SIGN>
__device__ __forceinline__ void wilson_hop_col(const cx<double>* __restrict__ U, const cx<double>* __restrict__ vk,
                                               int s, int nb, bool neg, int chi, cx<double> (&t)[12]) {
  cx<double> p[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const bool on = (k / 6) == chi;
    p[k] = on ? vk[fidx(nb, k, 12)] : mk(0.0, 0.0);
  }
  cx<double> h[6];
  project<MU, SIGN>(p, h);
  const int ls = SIGN > 0 ? s : nb;
  cx<double> u[9];
  load_link(U, MU, ls, neg, u);
  cx<double> uh[6];
#pragma unroll
  for (int aa = 0; aa < 2; ++aa) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cx<double> sacc = mk(0.0, 0.0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (SIGN > 0)
          cmadd(sacc, u[i * 3 + b], h[aa * 3 + b]);
        else
          cmaddc(sacc, u[b * 3 + i], h[aa * 3 + b]);
      }
      uh[aa * 3 + i] = sacc;
    }
  }
  expand_add<MU, SIGN>(uh, t);
}

__device__ void wilson_hop_dispatch(int mu, int dir, const cx<double>* U, const cx<double>* vk, int s, int nb,
                                    bool neg, int chi, cx<double> (&t)[12]) {
  switch (mu * 2 + (dir < 0)) {
    case 0: wilson_hop_col<0, +1>(U, vk, s, nb, neg, chi, t); break;
    case 1: wilson_hop_col<0, -1>(U, vk, s, nb, neg, chi, t); break;
    case 2: wilson_hop_col<1, +1>(U, vk, s, nb, neg, chi, t); break;
    case 3: wilson_hop_col<1, -1>(U, vk, s, nb, neg, chi, t); break;
    case 4: wilson_hop_col<2, +1>(U, vk, s, nb, neg, chi, t); break;
    case 5: wilson_hop_col<2, -1>(U, vk, s, nb, neg, chi, t); break;
    case 6: wilson_hop_col<3, +1>(U, vk, s, nb, neg, chi, t); break;
    default: wilson_hop_col<3, -1>(U, vk, s, nb, neg, chi, t); break;
  }
}

struct WilsonSide {
  const cx<double>* U;
  double diag;  // 4 + m
  int tneg;     // antiperiodic time: links at t = Lt-1 carry the sign
  static constexpr int kDof = 12;
  // Element offset of dof e at site s in a field of this level.
  __device__ __forceinline__ size_t off(size_t, int s, int e) const { return fidx(s, e, 12); }
  __device__ __forceinline__ bool neg(const Geom& g, const int c[4], int mu, int dir) const {
    return tneg && mu == 3 && c[3] == (dir > 0 ? g.L[3] - 1 : 0);
  }
  // T[q][e][cc] for columns col0 .. col0+ncc-1 at the chunk's sites.
  __device__ void columns(const AggGeom& a, int d, const int* sites, const int (*crd)[4], int ncs, int col0, int ncc,
                          int ldt, int nv, const cx<double>* Vv, size_t vstride, cx<double>* T) const {
    for (int w = threadIdx.x; w < ncs * ncc; w += blockDim.x) {
      const int q = w / ncc, cc = w % ncc;
      const int col = col0 + cc, chi = col / nv, k = col % nv;
      const cx<double>* vk = Vv + (size_t)k * vstride;
      const int s = sites[q];
      const int* c = crd[q];
      cx<double> t[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) t[e] = mk(0.0, 0.0);
      if (d < 8) {
        const int mu = d >> 1, dir = (d & 1) ? -1 : 1;
        const int nb = dir > 0 ? nbr_fwd(a.g, s, c, mu) : nbr_bwd(a.g, s, c, mu);
        wilson_hop_dispatch(mu, dir, U, vk, s, nb, neg(a.g, c, mu, dir), chi, t);
#pragma unroll
        for (int e = 0; e < 12; ++e) t[e] = (-0.5) * t[e];
      } else {
        for (int mu = 0; mu < 4; ++mu) {
          for (int dir = 1; dir >= -1; dir -= 2) {
            if (!inside(a, c, mu, dir)) continue;
            const int nb = dir > 0 ? nbr_fwd(a.g, s, c, mu) : nbr_bwd(a.g, s, c, mu);
            wilson_hop_dispatch(mu, dir, U, vk, s, nb, neg(a.g, c, mu, dir), chi, t);
          }
        }
#pragma unroll
        for (int e = 0; e < 12; ++e) {
          const bool on = (e / 6) == chi;
          const cx<double> f = on ? vk[fidx(s, e, 12)] : mk(0.0, 0.0);
          t[e] = mk(diag * f.re - 0.5 * t[e].re, diag * f.im - 0.5 * t[e].im);
        }
      }
#pragma unroll
      for (int e = 0; e < 12; ++e) T[((size_t)q * 12 + e) * ldt + cc] = t[e];
    }
  }
};

// ---- level >= 1: stencil hops ----------------------------------------------
struct StencilSide {
  const cx<double>* Dc;  // finer level's stencil [site][9][col][row]
  int dof;
  __device__ __forceinline__ size_t off(size_t, int s, int e) const { return (size_t)s * dof + e; }
  __device__ void columns(const AggGeom& a, int d, const int* sites, const int (*crd)[4], int ncs, int col0, int ncc,
                          int ldt, int nv, const cx<double>* Vv, size_t vstride, cx<double>* T) const {
    const int half = dof / 2;
    const size_t bsz = (size_t)dof * dof;
    for (int w = threadIdx.x; w < ncs * ncc * dof; w += blockDim.x) {
      const int e = w % dof;
      const int cc = (w / dof) % ncc;
      const int q = w / (dof * ncc);
      const int col = col0 + cc, chi = col / nv, k = col % nv;
      const cx<double>* vk = Vv + (size_t)k * vstride;
      const int s = sites[q];
      const int* c = crd[q];
      cx<double> acc = mk(0.0, 0.0);
      for (int dd = 0; dd < 9; ++dd) {
        int nb;
        if (d < 8) {
          if (dd != d) continue;
        } else if (dd < 8) {
          if (!inside(a, c, dd >> 1, (dd & 1) ? -1 : 1)) continue;
        }
        if (dd == 8)
          nb = s;
        else
          nb = (dd & 1) ? nbr_bwd(a.g, s, c, dd >> 1) : nbr_fwd(a.g, s, c, dd >> 1);
        const cx<double>* blk = Dc + ((size_t)s * 9 + dd) * bsz;
        const cx<double>* f = vk + (size_t)nb * dof + chi * half;
        for (int j = 0; j < half; ++j) cmadd(acc, blk[(size_t)(chi * half + j) * dof + e], f[j]);
      }
      T[((size_t)q * dof + e) * ldt + cc] = acc;
    }
  }
};

// ---- the build kernel ---------------------------------------------------------
template <class Side>
__global__ __launch_bounds__(256) void k_coarse_build(Side side, AggGeom a, const cx<double>* __restrict__ Vv,
                                                      size_t vstride, int nv, int dof, int cs, int cc_max,
                                                      cx<double>* __restrict__ Dc) {
  extern __shared__ cx<double> sm[];
  __shared__ int sites[8];
  __shared__ int crd[8][4];
  const int agg = blockIdx.x, d = blockIdx.y;
  const int n2 = 2 * nv, half = dof / 2;
  cx<double>* Vt = sm;                          // [cs][dof][nv]
  cx<double>* T = sm + (size_t)cs * dof * nv;   // [cs][dof][cc_max]
  const int nsites = nsites_of_block(a, d);
  cx<double>* out = Dc + ((size_t)agg * 9 + d) * n2 * n2;
  for (int col0 = 0; col0 < n2; col0 += cc_max) {
    const int ncc = min(cc_max, n2 - col0);
    const int nent = n2 * ncc;
    cx<double> acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = mk(0.0, 0.0);
    for (int i0 = 0; i0 < nsites; i0 += cs) {
      const int ncs = min(cs, nsites - i0);
      if (threadIdx.x < ncs) {
        int c[4];
        block_site(a, agg, d, i0 + threadIdx.x, c);
        sites[threadIdx.x] = site_of(a.g, c[0], c[1], c[2], c[3]);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) crd[threadIdx.x][mu] = c[mu];
      }
      __syncthreads();
      for (int w = threadIdx.x; w < ncs * dof * nv; w += blockDim.x) {
        const int k = w % nv, e = (w / nv) % dof, q = w / (nv * dof);
        Vt[w] = Vv[(size_t)k * vstride + side.off(a.g.vol, sites[q], e)];
      }
      side.columns(a, d, sites, crd, ncs, col0, ncc, cc_max, nv, Vv, vstride, T);
      __syncthreads();
#pragma unroll
      for (int slot = 0; slot < 16; ++slot) {
        const int ent = threadIdx.x + slot * 256;
        if (ent < nent) {
          const int row = ent % n2, cc = ent / n2;
          const int chi = row / nv, k = row % nv;
          cx<double> s = acc[slot];
          for (int q = 0; q < ncs; ++q) {
            for (int m = 0; m < half; ++m) {
              const int e = chi * half + m;
              cmaddc(s, Vt[((size_t)q * dof + e) * nv + k], T[((size_t)q * dof + e) * cc_max + cc]);
            }
          }
          acc[slot] = s;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int slot = 0; slot < 16; ++slot) {
      const int ent = threadIdx.x + slot * 256;
      if (ent < nent) {
        const int row = ent % n2, cc = ent / n2;
        out[(size_t)(col0 + cc) * n2 + row] = acc[slot];
      }
    }
  }
}

// ---- application ----------------------------------------------------------------
// One workgroup of nine waves per (coarse site, rhs); wave d applies block d
// (lane = row), and the nine partial rows are summed in a fixed order.
// acc += sum_j blk[j n2] v[j]: one row of a column-major block times a
// vector, in column order, with the loads of 8 columns issued together.
template <typename R>
__device__ __forceinline__ void block_row_madd(const cx<R>* __restrict__ blk, int n2, const cx<R>* v, cx<R>& acc) {
  int jj = 0;
  for (; jj + 8 <= n2; jj += 8) {
    cx<R> a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = blk[(size_t)(jj + u) * n2];
      b[u] = v[jj + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) cmadd(acc, a[u], b[u]);
  }
  for (; jj < n2; ++jj) cmadd(acc, blk[(size_t)jj * n2], v[jj]);
}

template <typename R>
__global__ __launch_bounds__(576) void k_coarse_apply(Geom g, int n2, const cx<R>* __restrict__ Dc,
                                                      const cx<R>* __restrict__ in, cx<R>* __restrict__ out,
                                                      cx<R>* __restrict__ copy) {
  __shared__ cx<R> part[9][64];
  const int s = blockIdx.x, rhs = blockIdx.y;
  const int d = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t nsite = g.vol;
  in += (size_t)rhs * nsite * n2;
  out += (size_t)rhs * nsite * n2;
  if (copy && d == 8 && lane < n2) copy[(size_t)rhs * nsite * n2 + (size_t)s * n2 + lane] = in[(size_t)s * n2 + lane];
  int nb = s;
  if (d < 8) {
    int c[4];
    coords_of(g, s, c);
    nb = (d & 1) ? nbr_bwd(g, s, c, d >> 1) : nbr_fwd(g, s, c, d >> 1);
  }
  cx<R> acc = mk<R>(0, 0);
  if (lane < n2) {
    block_row_madd(Dc + ((size_t)s * 9 + d) * n2 * n2 + lane, n2, in + (size_t)nb * n2, acc);
  }
  part[d][lane] = acc;
  __syncthreads();
  if (d == 0 && lane < n2) {
    cx<R> t = part[8][lane];
#pragma unroll
    for (int dd = 0; dd < 8; ++dd) t = t + part[dd][lane];
    out[(size_t)s * n2 + lane] = t;
  }
}

// ---- batched application on the matrix cores ---------------------------------
// For a block of right-hand sides the coarse operator at one site is a
// complex GEMM, y = [X | Y_{+x} | ... | Y_{-t}] [c(x); c(x+x); ...; c(x-t)],
// (2Nv x 9*2Nv) x (9*2Nv x nrhs).  It runs as the equivalent real GEMM with
// re/im-interleaved rows and columns: the complex entry a of row i, column j
// becomes the 2x2 block [[Re a, -Im a], [Im a, Re a]], and the right-hand
// sides enter as (Re, Im) row pairs.  The flop count equals the complex one.
// One workgroup per (site, rhs tile); wave t owns a tile of real rows; the
// right-hand-side operand of one direction is staged in LDS at a time.
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// real-row r, real-col k of the complex block stored column-major (col j, row i)
template <typename R>
__device__ __forceinline__ R real_entry(const cx<R>* __restrict__ blk, int n2, int r, int k) {
  const int i = r >> 1, j = k >> 1;
  if (i >= n2) return (R)0;
  const cx<R> a = blk[(size_t)j * n2 + i];
  const int pr = r & 1, pk = k & 1;
  return pr == 0 ? (pk == 0 ? a.re : -a.im) : (pk == 0 ? a.im : a.re);
}

// Operands are read straight from memory into the MFMA lane layout (no LDS
// staging): wave w owns real-row tile w % nrt and the directions
// d = w / nrt, w / nrt + ng, ... (ng direction groups), so the nine blocks of
// a site stream in parallel; the groups' partial products are added through
// LDS in group order.  The right-hand sides of a tile are the columns of the
// B operand.
//
// FP64: v_mfma_f64_16x16x4f64; tile = 16 real rows x 16 rhs.
// Operand lanes: A[i][k] at lane i + 16k, B[k][j] at lane j + 16k;
// result D[i][j] in lane j + 16 (i % 4), register i / 4.
__host__ __device__ inline int mfma64_row_tiles(int n2) { return (2 * n2 + 15) / 16; }
__host__ __device__ inline int mfma64_groups(int n2) {
  const int g = 16 / mfma64_row_tiles(n2);
  return g < 9 ? g : 9;
}
constexpr int kMfma64Lds = 4096;  // doubles of LDS for the group partials

// All right-hand sides of the batch (up to kMaxRhs = 4 tiles of 16) are
// done by one workgroup, so each operand chunk of A is loaded once and
// multiplied into every tile's accumulator.  NT >= ceil(nrhs / 16) tiles are
// held in registers; instantiating the smallest NT keeps the unused
// accumulators out of the register budget.
constexpr int kMaxTiles = kMaxRhs / 16;

// Coarse vector layouts: element (rhs q, site, row) of nrhs vectors.
struct RhsMajor {  // [rhs][site][row], the canonical coarse layout
  size_t fs;       // site count x rows
  __device__ __forceinline__ size_t at(int q, int site, int row, int n2) const {
    return (size_t)q * fs + (size_t)site * n2 + row;
  }
};
struct RhsFast {  // [site][row][rhs]: the rhs of one row are adjacent
  int nrhs;
  __device__ __forceinline__ size_t at(int q, int site, int row, int n2) const {
    return ((size_t)site * n2 + row) * nrhs + q;
  }
};

template <int NT, class Lay>
__device__ __forceinline__ void apply_site_mfma64(const Geom& g, int n2, int nrhs, int s,
                                                  const cx<double>* __restrict__ Dc, const cx<double>* in,
                                                  cx<double>* out, double* lds, Lay lay) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nrt = mfma64_row_tiles(n2), ng = mfma64_groups(n2);
  const int rt = w % nrt, grp = w / nrt;
  const int ntile = (nrhs + 15) / 16;
  const int kr = 2 * n2;
  const int r = rt * 16 + (l & 15), i = r >> 1, pr = r & 1;
  const bool rowok = i < n2;
  const int kl = l >> 4;
  int c[4];
  coords_of(g, s, c);
  doublex4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  // MFMA steps whose operands are loaded together (fewer when more tiles
  // hold accumulators, to stay within the register budget)
  constexpr int KC = NT == 1 ? 8 : 4;
  for (int d = grp; d < 9; d += ng) {
    const int nb = d == 8 ? s : ((d & 1) ? nbr_bwd(g, s, c, d >> 1) : nbr_fwd(g, s, c, d >> 1));
    const double* blk = reinterpret_cast<const double*>(Dc + ((size_t)s * 9 + d) * n2 * n2);
    for (int t0 = 0; 4 * t0 < kr; t0 += KC) {
      double av[KC];
#pragma unroll
      for (int t = 0; t < KC; ++t) {
        const int k = 4 * (t0 + t) + kl, j = k >> 1, pk = k & 1;
        av[t] = 0.0;
        if (k < kr && rowok) {
          const double a = blk[2 * ((size_t)j * n2 + i) + (pr ^ pk)];
          av[t] = (pr == 0 && pk == 1) ? -a : a;
        }
      }
#pragma unroll
      for (int tt = 0; tt < NT; ++tt) {
        if (tt >= ntile) break;
        const int q = tt * 16 + (l & 15);
        const bool qok = q < nrhs;
        double bv[KC];
#pragma unroll
        for (int t = 0; t < KC; ++t) {
          const int k = 4 * (t0 + t) + kl, j = k >> 1, pk = k & 1;
          bv[t] = (qok && k < kr) ? reinterpret_cast<const double*>(in + lay.at(q, nb, j, n2))[pk] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < KC; ++t)
          if (4 * (t0 + t) < kr) acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc[tt], 0, 0, 0);
      }
    }
  }
  // groups 1.. hand their partial tiles to group 0, one rhs tile at a time
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) {
    if (tt >= ntile) break;
    if (grp > 0 && grp < ng) {
      double* dst = lds + ((size_t)((grp - 1) * nrt + rt) * 64 + l) * 4;
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) dst[reg] = acc[tt][reg];
    }
    __syncthreads();
    if (grp == 0) {
      doublex4 a = acc[tt];
      for (int gg = 1; gg < ng; ++gg) {
        const double* src = lds + ((size_t)((gg - 1) * nrt + rt) * 64 + l) * 4;
#pragma unroll
        for (int reg = 0; reg < 4; ++reg) a[reg] += src[reg];
      }
      const int q = tt * 16 + (l & 15);
      if (q < nrhs) {
#pragma unroll
        for (int reg = 0; reg < 4; ++reg) {
          const int rr = rt * 16 + 4 * reg + (l >> 4);
          if ((rr >> 1) < n2) reinterpret_cast<double*>(out + lay.at(q, s, rr >> 1, n2))[rr & 1] = a[reg];
        }
      }
    }
    __syncthreads();
  }
}

// One right-hand side on the vector units: wave d (of nine) applies block d
// of site s with lane = row; the nine partial rows are added in order.
// Needs blockDim.x >= 576; ends with a block barrier.
__device__ __forceinline__ void apply_site_valu1(const Geom& g, int n2, int s, const cx<double>* __restrict__ Dc,
                                                 const cx<double>* in, cx<double>* out, double* lds) {
  const int d = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cx<double> acc = mk(0.0, 0.0);
  if (d < 9 && lane < n2) {
    int nb = s;
    if (d < 8) {
      int c[4];
      coords_of(g, s, c);
      nb = (d & 1) ? nbr_bwd(g, s, c, d >> 1) : nbr_fwd(g, s, c, d >> 1);
    }
    block_row_madd(Dc + ((size_t)s * 9 + d) * n2 * n2 + lane, n2, in + (size_t)nb * n2, acc);
  }
  if (d < 9) {
    lds[2 * (d * 64 + lane)] = acc.re;
    lds[2 * (d * 64 + lane) + 1] = acc.im;
  }
  __syncthreads();
  if (d == 0 && lane < n2) {
    cx<double> t = mk(lds[2 * (8 * 64 + lane)], lds[2 * (8 * 64 + lane) + 1]);
#pragma unroll
    for (int dd = 0; dd < 8; ++dd) t = t + mk(lds[2 * (dd * 64 + lane)], lds[2 * (dd * 64 + lane) + 1]);
    out[(size_t)s * n2 + lane] = t;
  }
  __syncthreads();
}

// copy = in on site s for the right-hand sides [q0, q0 + nq) (all threads of the block)
template <typename R>
__device__ __forceinline__ void copy_site(int n2, size_t fs, int s, int q0, int nq, const cx<R>* in, cx<R>* copy) {
  for (int w = threadIdx.x; w < nq * n2; w += blockDim.x) {
    const int q = q0 + w / n2, j = w % n2;
    copy[(size_t)q * fs + (size_t)s * n2 + j] = in[(size_t)q * fs + (size_t)s * n2 + j];
  }
}

template <int NT>
__global__ __launch_bounds__(1024) void k_coarse_apply_mfma64(Geom g, int n2, int nrhs,
                                                              const cx<double>* __restrict__ Dc,
                                                              const cx<double>* __restrict__ in,
                                                              cx<double>* __restrict__ out,
                                                              cx<double>* __restrict__ copy) {
  __shared__ double lds[kMfma64Lds];
  const int s = blockIdx.x;
  if (copy) copy_site(n2, (size_t)g.vol * n2, s, 0, nrhs, in, copy);
  apply_site_mfma64<NT>(g, n2, nrhs, s, Dc, in, out, lds, RhsMajor{(size_t)g.vol * n2});
}

// FP32: v_mfma_f32_32x32x2f32; tile = 32 real rows x 32 rhs.
// Operand lanes: A[i][k] at lane i + 32k, B[k][j] at lane j + 32k; result
// D[i][j] in lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.
__global__ __launch_bounds__(256) void k_coarse_apply_mfma32(Geom g, int n2, int nrhs,
                                                             const cx<float>* __restrict__ Dc,
                                                             const cx<float>* __restrict__ in,
                                                             cx<float>* __restrict__ out,
                                                             cx<float>* __restrict__ copy) {
  const int s = blockIdx.x, q0 = blockIdx.y * 32;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const size_t fs = (size_t)g.vol * n2;
  if (copy) copy_site(n2, fs, s, q0, min(32, nrhs - q0), in, copy);
  const int kr = 2 * n2;
  const int r = wave * 32 + (l & 31), i = r >> 1, pr = r & 1;
  const bool rowok = i < n2;
  const int q = q0 + (l & 31);
  const bool qok = q < nrhs;
  const int kl = l >> 5;
  int c[4];
  coords_of(g, s, c);
  floatx16 acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  constexpr int KC = 16;  // MFMA steps loaded together
  for (int d = 0; d < 9; ++d) {
    const int nb = d == 8 ? s : ((d & 1) ? nbr_bwd(g, s, c, d >> 1) : nbr_fwd(g, s, c, d >> 1));
    const float* blk = reinterpret_cast<const float*>(Dc + ((size_t)s * 9 + d) * n2 * n2);
    const float* v = reinterpret_cast<const float*>(in + (size_t)(qok ? q : 0) * fs + (size_t)nb * n2);
    for (int t0 = 0; 2 * t0 < kr; t0 += KC) {
      float av[KC], bv[KC];
#pragma unroll
      for (int t = 0; t < KC; ++t) {
        const int k = 2 * (t0 + t) + kl, j = k >> 1, pk = k & 1;
        av[t] = 0.f;
        bv[t] = 0.f;
        if (k < kr) {
          if (rowok) {
            const float a = blk[2 * ((size_t)j * n2 + i) + (pr ^ pk)];
            av[t] = (pr == 0 && pk == 1) ? -a : a;
          }
          if (qok) bv[t] = v[2 * j + pk];
        }
      }
#pragma unroll
      for (int t = 0; t < KC; ++t)
        if (2 * (t0 + t) < kr) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[t], bv[t], acc, 0, 0, 0);
    }
  }
  if (qok) {
    float* o = reinterpret_cast<float*>(out + (size_t)q * fs + (size_t)s * n2);
#pragma unroll
    for (int reg = 0; reg < 16; ++reg) {
      const int rr = wave * 32 + 8 * (reg >> 2) + 4 * (l >> 5) + (reg & 3);
      if ((rr >> 1) < n2) o[rr] = acc[reg];
    }
  }
}

// ---- 16-bit blocks ---------------------------------------------------------------
// One workgroup per block: scale = largest magnitude of the block's real
// components (after rounding to FP32), stored = fl16(fl32(value * fl32(1/scale))).
template <typename H>
__global__ __launch_bounds__(256) void k_dc_to_half(const cx<double>* __restrict__ Dc, cxh<H>* __restrict__ Dh,
                                                    float* __restrict__ scales, int nn) {
  __shared__ float red[4];
  const size_t b = blockIdx.x;
  const cx<double>* src = Dc + b * nn;
  float m = 0.0f;
  bool nan = false;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const cx<float> a = cvt<float>(src[i]);
    m = fmaxf(m, fmaxf(fabsf(a.re), fabsf(a.im)));
    nan = nan || a.re != a.re || a.im != a.im;
  }
  if (nan) m = __builtin_nanf("");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float o = __shfl_xor(m, off, 64);
    m = (o != o || m != m) ? __builtin_nanf("") : fmaxf(m, o);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  float mm = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mm = (red[w] != red[w] || mm != mm) ? __builtin_nanf("") : fmaxf(mm, red[w]);
  float inv;
  const float sc = quant_scale(mm, inv);
  if (threadIdx.x == 0) scales[b] = sc;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const cx<float> a = cvt<float>(src[i]);
    Dh[b * nn + i] = quantise<H>(a.re, a.im, inv);
  }
}

// One right-hand side on the vector units (as k_coarse_apply), 16-bit blocks.
template <typename H>
__global__ __launch_bounds__(576) void k_coarse_apply_h(Geom g, int n2, const cxh<H>* __restrict__ Dc,
                                                        const float* __restrict__ Dcs,
                                                        const cx<float>* __restrict__ in,
                                                        cx<float>* __restrict__ out, cx<float>* __restrict__ copy) {
  __shared__ cx<float> part[9][64];
  const int s = blockIdx.x, rhs = blockIdx.y;
  const int d = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t nsite = g.vol;
  in += (size_t)rhs * nsite * n2;
  out += (size_t)rhs * nsite * n2;
  if (copy && d == 8 && lane < n2) copy[(size_t)rhs * nsite * n2 + (size_t)s * n2 + lane] = in[(size_t)s * n2 + lane];
  int nb = s;
  if (d < 8) {
    int c[4];
    coords_of(g, s, c);
    nb = (d & 1) ? nbr_bwd(g, s, c, d >> 1) : nbr_fwd(g, s, c, d >> 1);
  }
  cx<float> acc = mk(0.0f, 0.0f);
  if (lane < n2) {
    const cxh<H>* blk = Dc + ((size_t)s * 9 + d) * n2 * n2 + lane;
    const cx<float>* v = in + (size_t)nb * n2;
    for (int j = 0; j < n2; ++j) cmadd(acc, h2f(blk[(size_t)j * n2]), v[j]);
    const float sc = Dcs[(size_t)s * 9 + d];
    acc = mk(sc * acc.re, sc * acc.im);
  }
  part[d][lane] = acc;
  __syncthreads();
  if (d == 0 && lane < n2) {
    cx<float> t = part[8][lane];
#pragma unroll
    for (int dd = 0; dd < 8; ++dd) t = t + part[dd][lane];
    out[(size_t)s * n2 + lane] = t;
  }
}

// A batch on the matrix cores with 16-bit operands (v_mfma_f32_32x32x8 f16 or
// bf16, FP32 accumulation).  Same real-GEMM form and tiling as the FP32
// kernel.  Per direction, each right-hand-side column of the staged operand
// is rounded to 16 bits: in FP16 after scaling it into [-1, 1] by its largest
// magnitude (the format's range is narrow), in BF16 as it is (BF16 has the
// range of FP32, so a scale would change no relative rounding error); the
// product of that direction is accumulated from zero and added to the result
// times the block scale (and the FP16 column scale).  Operand lanes: A[i][k] at lane
// i + 32 (k / 4), element k % 4; B[k][j] at lane j + 32 (k / 4), element
// k % 4; result as for the FP32 kernel.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));

template <typename H>
__device__ __forceinline__ floatx16 mfma_32x32x8(const float (&a)[4], const float (&b)[4], floatx16 acc);
template <>
__device__ __forceinline__ floatx16 mfma_32x32x8<f16_t>(const float (&a)[4], const float (&b)[4], floatx16 acc) {
  half4_t x, y;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    x[e] = (_Float16)a[e];
    y[e] = (_Float16)b[e];
  }
  return __builtin_amdgcn_mfma_f32_32x32x8f16(x, y, acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ floatx16 mfma_32x32x8<bf16_t>(const float (&a)[4], const float (&b)[4], floatx16 acc) {
  short4_t x, y;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    x[e] = __builtin_bit_cast(short, (__bf16)a[e]);
    y[e] = __builtin_bit_cast(short, (__bf16)b[e]);
  }
  return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(x, y, acc, 0, 0, 0);
}

// Per-thread staging of one direction (workgroup of 64 ceil(2 n2 / 32)
// threads, n2 <= 64): the block's 16-byte chunks, n2^2 / 4 <= 4 per thread,
// and the batch's rhs rows, 32 n2 <= 8 per thread.
constexpr int kH16Chunks = 4, kH16Rows = 8;
template <typename H, int CB = kH16Rows>  // CB: rhs rows staged per thread (>= 32 n2 / threads for the batch)
__global__ __launch_bounds__(256) void k_coarse_apply_mfma16(Geom g, int n2, int nrhs, const cxh<H>* __restrict__ Dc,
                                                             const float* __restrict__ Dcs,
                                                             const cx<float>* __restrict__ in,
                                                             cx<float>* __restrict__ out,
                                                             cx<float>* __restrict__ copy) {
  __shared__ float Bs[128][33];
  __shared__ float Bsc[32], Binv[32];
  extern __shared__ __align__(16) char dyn16[];
  cxh<H>* As16 = reinterpret_cast<cxh<H>*>(dyn16);
  const int s = blockIdx.x, q0 = blockIdx.y * 32;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const size_t nsite = g.vol, fs = nsite * n2;
  const int kr = 2 * n2;
  int c[4];
  coords_of(g, s, c);
  floatx16 acc;
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.f;
  // rhs columns beyond the batch stay zero for every direction
  const int nq = nrhs - q0 < 32 ? nrhs - q0 : 32;
  for (int w = threadIdx.x; w < (32 - nq) * kr; w += blockDim.x) Bs[w % kr][nq + w / kr] = 0.f;
  const int nthr = blockDim.x;
  const int nch = n2 * n2 / 4;  // 16-byte chunks of a block (n2 even)
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  u4v ra[kH16Chunks];
  f2v rb[CB];
  float fsc = 0.f;  // block scale of the fetched direction
  // Direction d + 1 is fetched into registers (every load issued before any
  // use) while the matrix cores work on direction d from LDS.
  auto fetch = [&](int d) {
    const int nb = d == 8 ? s : ((d & 1) ? nbr_bwd(g, s, c, d >> 1) : nbr_fwd(g, s, c, d >> 1));
    const u4v* blk = reinterpret_cast<const u4v*>(Dc + ((size_t)s * 9 + d) * n2 * n2);
#pragma unroll
    for (int u = 0; u < kH16Chunks; ++u) {
      const int e = threadIdx.x + u * nthr;
      if (e < nch) ra[u] = blk[e];
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const int w = threadIdx.x + u * nthr;
      if (w < nq * n2)
        rb[u] = *reinterpret_cast<const f2v*>(in + (size_t)(q0 + w / n2) * fs + (size_t)nb * n2 + w % n2);
    }
    fsc = Dcs[(size_t)s * 9 + d];
  };
  auto stage = [&](int d) {
#pragma unroll
    for (int u = 0; u < kH16Chunks; ++u) {
      const int e = threadIdx.x + u * nthr;
      if (e < nch) reinterpret_cast<u4v*>(As16)[e] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const int w = threadIdx.x + u * nthr;
      if (w < nq * n2) {
        const int q = w / n2, j = w % n2;
        Bs[2 * j][q] = rb[u].x;
        Bs[2 * j + 1][q] = rb[u].y;
        if (d == 8 && copy) copy[(size_t)(q0 + q) * fs + (size_t)s * n2 + j] = mk(rb[u].x, rb[u].y);
      }
    }
  };
  fetch(0);
  for (int d = 0; d < 9; ++d) {
    __syncthreads();  // every wave is done with the previous direction's operands
    stage(d);
    const float fd = fsc;
    if (d + 1 < 9) fetch(d + 1);
    __syncthreads();
    float binv = 1.0f, bsc = 1.0f;
    if constexpr (sizeof(H) == 2 && !std::is_same<H, bf16_t>::value) {
      if (threadIdx.x < 32) {
        float m = 0.0f;
        for (int k = 0; k < kr; ++k) m = fmaxf(m, fabsf(Bs[k][threadIdx.x]));
        float inv;
        Bsc[threadIdx.x] = quant_scale(m, inv);
        Binv[threadIdx.x] = inv;
      }
      __syncthreads();
      binv = Binv[l & 31];
      bsc = Bsc[l & 31];
    }
    const int r = wave * 32 + (l & 31), i = r >> 1, pr = r & 1;
    floatx16 t;
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = 0.f;
    for (int k0 = 0; k0 < kr; k0 += 8) {
      float a[4], b[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + 4 * (l >> 5) + e;
        a[e] = 0.f;
        b[e] = 0.f;
        if (k < kr) {
          b[e] = Bs[k][l & 31] * binv;
          if (i < n2) {
            const cx<float> z = h2f(As16[(size_t)(k >> 1) * n2 + i]);
            const int pk = k & 1;
            a[e] = pr == 0 ? (pk == 0 ? z.re : -z.im) : (pk == 0 ? z.im : z.re);
          }
        }
      }
      t = mfma_32x32x8<H>(a, b, t);
    }
    const float f = fd * bsc;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] += f * t[e];
  }
  const int q = q0 + (l & 31);
  if (q < nrhs) {
    float* o = reinterpret_cast<float*>(out + (size_t)q * fs + (size_t)s * n2);
#pragma unroll
    for (int reg = 0; reg < 16; ++reg) {
      const int r = wave * 32 + 8 * (reg >> 2) + 4 * (l >> 5) + (reg & 3);
      if ((r >> 1) < n2) o[r] = acc[reg];
    }
  }
}

// ---- coarsest-level GCR in three launches per iteration -------------------------
// GCR(k) on D_c in FP64 for a batch of right-hand sides, each with its own
// coefficients and stopping test (Sec. 2: the coarsest solve).  Iteration j:
//   K1  w_j = D_c r, z_j = r, and per workgroup partial sums of
//       c_i = <W_i, w_j>, d_i = <W_i, r> (i < j), <w_j, w_j>, <w_j, r>, <r, r>
//   K2  (one workgroup per rhs) the sums in a fixed order; h_i = c_i / |W_i|^2;
//       |w'|^2 = <w,w> - sum |c_i|^2 / |W_i|^2 and <w', r> = <w, r> - sum h_i^* d_i
//       for w' = w_j - sum h_i W_i (classical Gram-Schmidt, the W_i orthogonal);
//       a = <w', r> / |w'|^2; a right-hand side with |r| <= tol |b| is frozen
//   K3  w_j = w', z_j -= sum h_i Z_i, x += a z_j, r -= a w_j, and partial sums
//       of the exact |w_j|^2, which K2 of the next iteration stores as |W_j|^2.
// The stopping test is thus lagged by one iteration; the per-rhs active flags
// go to pinned host memory, where the host inspects them two iterations
// later, so it never waits for the GPU inside the solve.
constexpr int kCgcrG1 = 4096;  // workgroups of K1 (one coarse site each up to this many sites)
constexpr int kCgcrG3 = 64;   // chunks per rhs of K3

struct CgcrState {  // per-rhs device scalars of one solve (inside the level's scalar block)
  double* h;    // [rhs][2 kMaxKrylov]
  double* nrm;  // [rhs][kMaxKrylov]
  double* a;    // [rhs][2]
  double* rn;   // [rhs]
  double* act;  // [rhs]
  double* tol2; // [rhs]
};

// x = 0, r = b, tol2 = tol^2 |b|^2, active = |b| > 0 (one workgroup per rhs)
__global__ __launch_bounds__(256) void k_cgcr_init(const cx<double>* __restrict__ b, cx<double>* __restrict__ x,
                                                   cx<double>* __restrict__ r, size_t n, double tol, CgcrState S,
                                                   double* err) {
  __shared__ double red[4];
  const int q = blockIdx.x;
  const size_t o = (size_t)q * n;
  double v[1] = {0.0};
  for (size_t e = threadIdx.x; e < n; e += blockDim.x) {
    const cx<double> bv = b[o + e];
    x[o + e] = mk(0.0, 0.0);
    r[o + e] = bv;
    v[0] += bv.re * bv.re + bv.im * bv.im;
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) {
    if (!isfinite(v[0])) err[0] = 1.0;
    S.tol2[q] = tol * tol * v[0];
    S.act[q] = v[0] > 0.0 && isfinite(v[0]) ? 1.0 : 0.0;
    S.rn[q] = v[0];
  }
}

// K1 of a single rhs: grid-stride over sites, nine waves (one per block of
// the stencil), then the dot products of w_j with the basis and r.
__global__ __launch_bounds__(1024) void k_cgcr_apply(Geom g, int n2, int nrhs, int j, int vals,
                                                    const cx<double>* __restrict__ Dc, const cx<double>* r,
                                                    const cx<double>* Wb, cx<double>* w, cx<double>* z,
                                                    double* part) {
  extern __shared__ __align__(16) char dyn1[];
  double* acc = reinterpret_cast<double*>(dyn1);  // [nrhs][vals]
  __shared__ double lds[kMfma64Lds];
  const int q0 = 0, nq = nrhs;
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  const size_t fs = (size_t)g.vol * n2, bs = (size_t)nrhs * fs;
  for (int t = threadIdx.x; t < nq * vals; t += blockDim.x) acc[t] = 0.0;
  for (int s = blockIdx.x; s < g.vol; s += gridDim.x) {
    copy_site(n2, fs, s, q0, nq, r, z);
    // ends with a block barrier: w_j of site s is then complete
    apply_site_valu1(g, n2, s, Dc, r, w, lds);
    // Dot-product tasks (rhs qq, basis vector i < j) and (qq, the four
    // norms) spread over the waves; a task keeps its wave for every site of
    // the loop, so each accumulator has a single writer.
    const int per = j + 1;
    for (int t = wave; t < nq * per; t += nw) {
      const int qq = t / per, i = t % per;
      const size_t o = (size_t)(q0 + qq) * fs + (size_t)s * n2 + lane;
      cx<double> wv = mk(0.0, 0.0), rv = mk(0.0, 0.0);
      if (lane < n2) {
        wv = w[o];
        rv = r[o];
      }
      double* aq = acc + qq * vals;
      if (i < j) {
        cx<double> u = mk(0.0, 0.0);
        if (lane < n2) u = Wb[(size_t)i * bs + o];
        const double c_re = wave_sum(u.re * wv.re + u.im * wv.im);
        const double c_im = wave_sum(u.re * wv.im - u.im * wv.re);
        const double d_re = wave_sum(u.re * rv.re + u.im * rv.im);
        const double d_im = wave_sum(u.re * rv.im - u.im * rv.re);
        if (lane == 0) {
          aq[2 * i] += c_re;
          aq[2 * i + 1] += c_im;
          aq[2 * j + 2 * i] += d_re;
          aq[2 * j + 2 * i + 1] += d_im;
        }
      } else {
        const double ww = wave_sum(wv.re * wv.re + wv.im * wv.im);
        const double wr_re = wave_sum(wv.re * rv.re + wv.im * rv.im);
        const double wr_im = wave_sum(wv.re * rv.im - wv.im * rv.re);
        const double rr = wave_sum(rv.re * rv.re + rv.im * rv.im);
        if (lane == 0) {
          aq[4 * j] += ww;
          aq[4 * j + 1] += wr_re;
          aq[4 * j + 2] += wr_im;
          aq[4 * j + 3] += rr;
        }
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nq * vals; t += blockDim.x) {
    const int qq = t / vals, v = t % vals;
    part[((size_t)(q0 + qq) * gridDim.x + blockIdx.x) * vals + v] = acc[t];
  }
}

// K2: one workgroup per rhs.  vals = 4 j + 4 partial values per K1 workgroup;
// p3: K3's g3 partial |w_{j-1}|^2 per rhs (j > 0).
// hist (batched solves, else null): per rhs and iteration j, the h_i of
// iteration j at [2 i], a_j at [2 kmax]; stride 2 kmax + 4 doubles per j.
__global__ __launch_bounds__(1024) void k_cgcr_coef(int j, int vals, int g1, const double* __restrict__ part,
                                                   const double* __restrict__ p3, int g3, int kmax, CgcrState S,
                                                   double* host_act, double* err, double* hist) {
  extern __shared__ __align__(16) char dyn2[];
  double* tot = reinterpret_cast<double*>(dyn2);  // [vals + 1]
  const int q = blockIdx.x;
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
  for (int v = wave; v <= vals; v += nw) {
    double s = 0.0;
    if (v < vals) {
      for (int b = lane; b < g1; b += 64) s += part[((size_t)q * g1 + b) * vals + v];
    } else if (j > 0) {
      for (int b = lane; b < g3; b += 64) s += p3[(size_t)q * g3 + b];
    }
    s = wave_sum(s);
    if (lane == 0) tot[v] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* nrm = S.nrm + (size_t)q * kmax;
  double* h = S.h + (size_t)q * 2 * kmax;
  if (j > 0) nrm[j - 1] = tot[vals];
  double ww = tot[4 * j], wr_re = tot[4 * j + 1], wr_im = tot[4 * j + 2];
  const double rr = tot[4 * j + 3];
  for (int i = 0; i < j; ++i) {
    const double ni = nrm[i];
    const double cr = tot[2 * i], ci = tot[2 * i + 1];
    const double hr = ni > 0.0 ? cr / ni : 0.0, hi = ni > 0.0 ? ci / ni : 0.0;
    h[2 * i] = hr;
    h[2 * i + 1] = hi;
    if (hist) {
      hist[((size_t)q * kmax + j) * (2 * kmax + 4) + 2 * i] = hr;
      hist[((size_t)q * kmax + j) * (2 * kmax + 4) + 2 * i + 1] = hi;
    }
    ww -= hr * cr + hi * ci;  // |c_i|^2 / |W_i|^2
    const double dr = tot[2 * j + 2 * i], di = tot[2 * j + 2 * i + 1];
    wr_re -= hr * dr + hi * di;  // conj(h_i) d_i
    wr_im -= hr * di - hi * dr;
  }
  S.rn[q] = rr;
  if (!isfinite(rr) || !isfinite(ww)) err[0] = 1.0;
  const bool on = S.act[q] != 0.0 && rr > S.tol2[q];
  const bool ok = on && ww > 1e-28 * tot[4 * j];
  S.act[q] = on ? 1.0 : 0.0;
  S.a[2 * q] = ok ? wr_re / ww : 0.0;
  S.a[2 * q + 1] = ok ? wr_im / ww : 0.0;
  if (hist) {
    hist[((size_t)q * kmax + j) * (2 * kmax + 4) + 2 * kmax] = S.a[2 * q];
    hist[((size_t)q * kmax + j) * (2 * kmax + 4) + 2 * kmax + 1] = S.a[2 * q + 1];
  }
  if (host_act) host_act[q] = on ? 1.0 : 0.0;
}

// K3: blocks (kCgcrG3 chunks, rhs).
__global__ __launch_bounds__(256) void k_cgcr_update(size_t n, int nrhs, int j, int kmax, const cx<double>* Wb,
                                                     const cx<double>* Zb, cx<double>* w, cx<double>* z,
                                                     cx<double>* x, cx<double>* r, CgcrState S, double* p3) {
  __shared__ double red[4];
  __shared__ double hs[2 * kMaxKrylov];
  const int q = blockIdx.y;
  if (S.act[q] == 0.0) {
    if (threadIdx.x == 0) p3[(size_t)q * kCgcrG3 + blockIdx.x] = 0.0;
    return;
  }
  const double* h = S.h + (size_t)q * 2 * kmax;
  for (int t = threadIdx.x; t < 2 * j; t += blockDim.x) hs[t] = h[t];
  __syncthreads();
  const cx<double> a = mk(S.a[2 * q], S.a[2 * q + 1]);
  const size_t bs = (size_t)nrhs * n, o = (size_t)q * n;
  const size_t cs = (n + kCgcrG3 - 1) / kCgcrG3, e0 = blockIdx.x * cs, e1 = e0 + cs < n ? e0 + cs : n;
  double v[1] = {0.0};
  for (size_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    cx<double> wv = w[o + e], zv = z[o + e];
    for (int i = 0; i < j; ++i) {
      const cx<double> hi = mk(hs[2 * i], hs[2 * i + 1]);
      wv = wv - hi * Wb[(size_t)i * bs + o + e];
      zv = zv - hi * Zb[(size_t)i * bs + o + e];
    }
    w[o + e] = wv;
    z[o + e] = zv;
    x[o + e] = x[o + e] + a * zv;
    r[o + e] = r[o + e] - a * wv;
    v[0] += wv.re * wv.re + wv.im * wv.im;
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) p3[(size_t)q * kCgcrG3 + blockIdx.x] = v[0];
}

// ---- the same solve for a batch of rhs in the rhs-fast layout ---------------
// Vectors of the batch are stored [site][row][rhs] for the whole solve, so the
// matrix-core operand of one row and 16 rhs is one contiguous 256-byte run.
// Threads of a workgroup form a (rows x nrhs) grid, thread t handling rhs
// t % nrhs at positions (site, row) t / nrhs, t / nrhs + R, ... of the
// workgroup's chunk; sums over those positions meet in LDS, per rhs.
constexpr int kCgcrG3T = 1024;   // workgroups (chunks) of the rhs-fast update: four per CU
constexpr int kCgcrDotIG = 4;    // basis vectors per pass of the dot kernel

// Sums v over the threads of each rhs column; thread q < nrhs receives its total.
__device__ __forceinline__ double rhs_column_sum(double v, int nrhs, int rows, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  double sum = 0.0;
  if ((int)threadIdx.x < nrhs)
    for (int rr = 0; rr < rows; ++rr) sum += red[rr * nrhs + threadIdx.x];
  __syncthreads();
  return sum;
}

// The same for K values per thread at once (red holds K x 256 doubles): value
// k of rhs q is summed by thread k * nrhs + q (looping when K * nrhs > 256)
// and handed to put(k, q, sum).
template <int K, class Put>
__device__ __forceinline__ void rhs_column_sums(const double (&v)[K], int nrhs, int rows, double* red, Put put) {
#pragma unroll
  for (int k = 0; k < K; ++k) red[k * 256 + threadIdx.x] = v[k];
  __syncthreads();
  for (int u = threadIdx.x; u < K * nrhs; u += 256) {
    const int k = u / nrhs, q = u % nrhs;
    double sum = 0.0;
    for (int rr = 0; rr < rows; ++rr) sum += red[k * 256 + rr * nrhs + q];
    put(k, q, sum);
  }
  __syncthreads();
}

// r = b and x = 0 in the rhs-fast layout; partial |b_q|^2 per workgroup.
__global__ __launch_bounds__(256) void k_cgcrT_init(size_t npos, int nrhs, const cx<double>* __restrict__ b,
                                                    cx<double>* __restrict__ xT, cx<double>* __restrict__ rT,
                                                    double* p3) {
  __shared__ double red[256];
  const int rows = 256 / nrhs, q = threadIdx.x % nrhs, rho = threadIdx.x / nrhs;
  const size_t cs = (npos + gridDim.x - 1) / gridDim.x, p0 = blockIdx.x * cs, p1 = p0 + cs < npos ? p0 + cs : npos;
  double v = 0.0;
  if (rho < rows) {
    for (size_t p = p0 + rho; p < p1; p += rows) {
      const cx<double> bv = b[(size_t)q * npos + p];
      rT[p * nrhs + q] = bv;
      xT[p * nrhs + q] = mk(0.0, 0.0);
      v += bv.re * bv.re + bv.im * bv.im;
    }
  }
  const double sum = rhs_column_sum(v, nrhs, rows, red);
  if ((int)threadIdx.x < nrhs) p3[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = sum;
}

// tol2 = tol^2 |b|^2, active = |b| > 0, from the init partials.
// One wave per rhs sums the g partials.
__global__ __launch_bounds__(64) void k_cgcrT_init_fin(int nrhs, int g, const double* __restrict__ p3, double tol,
                                                       CgcrState S, double* err) {
  const int q = blockIdx.x;
  double v = 0.0;
  for (int b = threadIdx.x; b < g; b += 64) v += p3[(size_t)q * g + b];
  v = wave_sum(v);
  if (threadIdx.x != 0) return;
  if (!isfinite(v)) err[0] = 1.0;
  S.tol2[q] = tol * tol * v;
  S.act[q] = v > 0.0 && isfinite(v) ? 1.0 : 0.0;
  S.rn[q] = v;
}

// x (canonical) = xT.
__global__ __launch_bounds__(256) void k_cgcrT_out(size_t npos, int nrhs, const cx<double>* __restrict__ xT,
                                                   cx<double>* __restrict__ x) {
  const size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (e >= npos * nrhs) return;
  const size_t p = e / nrhs;
  const int q = (int)(e % nrhs);
  x[(size_t)q * npos + p] = xT[e];
}

// K1 (rhs-fast): w_j = D_c r and z_j = r at one site per workgroup.
template <int NT>
__global__ __launch_bounds__(1024) void k_cgcrT_apply(Geom g, int n2, int nrhs, const cx<double>* __restrict__ Dc,
                                                     const cx<double>* __restrict__ r, cx<double>* __restrict__ w,
                                                     cx<double>* __restrict__ z) {
  __shared__ double lds[kMfma64Lds];
  const int s = blockIdx.x;
  const size_t o = (size_t)s * n2 * nrhs;
  for (int e = threadIdx.x; e < n2 * nrhs; e += blockDim.x) z[o + e] = r[o + e];
  apply_site_mfma64<NT>(g, n2, nrhs, s, Dc, r, w, lds, RhsFast{nrhs});
}

// K1 (rhs-fast) with both operands staged through LDS: one workgroup per
// site, split into ng direction groups of nrt x ntile waves; wave (rt, tt) of
// group g owns real rows 16 rt.. and rhs 16 tt.. of w for the directions
// g, g + ng, ...  Each group fetches the block of its next direction and the
// neighbour's n2 x nrhs rows (contiguous in the rhs-fast layout) into
// registers with 16-byte loads while the matrix cores work on its current
// direction from LDS, so the product loop issues no global loads.  The
// groups' partial tiles are added through LDS at the end (one group: none).
// Block columns are padded to ldc = 8 (mod 16) complex so the two columns one
// MFMA operand fetch touches fall in disjoint bank halves.  Needs n2 % 8 == 0.
// Staging registers hold complex numbers as a clang vector of two doubles: an
// array of HIP's double2 class is not promoted to registers (it lands in
// scratch memory, whose stores wait for the loads and serialise the prefetch).
typedef double dbl2 __attribute__((ext_vector_type(2)));
constexpr int kStageA = 8;  // most complex of a block staged per thread (n2 <= 64)
constexpr int kStageB = 2;  // complex of the rhs rows staged per thread
__host__ __device__ inline int cgcr_ldc(int n2) {
  int l = n2;
  while ((l & 15) != 8) ++l;
  return l;
}
// LDS of one direction group's operands, and of the whole workgroup
__host__ __device__ inline size_t cgcr_group_bytes(int n2, int nrhs) {
  return ((size_t)n2 * cgcr_ldc(n2) + (size_t)n2 * nrhs) * 16;
}
__host__ __device__ inline size_t cgcr_lds_bytes(int n2, int nrhs, int ng) {
  const size_t waves = (size_t)mfma64_row_tiles(n2) * ((nrhs + 15) / 16);
  const size_t ops = ng * cgcr_group_bytes(n2, nrhs), part = (ng - 1) * waves * 64 * 4 * sizeof(double);
  return ops > part ? ops : part;
}
// (the smaller stagings keep to 80 registers so that two 12-wave workgroups
// share a compute unit)
template <int SA>  // complex of the block staged per thread (n2^2 <= SA x group threads)
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(SA <= 4 ? 6 : 4))) void k_cgcrT_apply_lds(
    Geom g, int n2, int nrhs, int ng, const cx<double>* __restrict__ Dc, const cx<double>* __restrict__ r,
    cx<double>* __restrict__ w, cx<double>* __restrict__ z) {
  extern __shared__ __align__(16) char dyn4[];
  const int ldc = cgcr_ldc(n2), nrt = mfma64_row_tiles(n2);
  const int wg = nrt * ((nrhs + 15) / 16);  // waves per group
  const int nthr = 64 * wg;                 // threads per group
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = wave / wg, wv = wave % wg, tid = threadIdx.x - grp * nthr;
  const int rt = wv % nrt, tt = wv / nrt;
  dbl2* al = reinterpret_cast<dbl2*>(dyn4 + grp * cgcr_group_bytes(n2, nrhs));  // [n2 cols][ldc]
  dbl2* bl = al + (size_t)n2 * ldc;                                              // [n2 rows][nrhs]
  const int s = blockIdx.x;
  const int nblk = n2 * n2, nb2 = n2 * nrhs;
  const size_t o = (size_t)s * nb2;
  for (int e = threadIdx.x; e < nb2; e += blockDim.x) z[o + e] = r[o + e];
  int c[4];
  coords_of(g, s, c);
  // staging slots: block element e = tid + u nthr (column-major) goes to
  // column e / n2, row e % n2; loads past the end re-read the last element
  dbl2 sa[SA], sb[kStageB];
  auto fetch = [&](int d) {
    const int nb = d == 8 ? s : ((d & 1) ? nbr_bwd(g, s, c, d >> 1) : nbr_fwd(g, s, c, d >> 1));
    const dbl2* blk = reinterpret_cast<const dbl2*>(Dc + ((size_t)s * 9 + d) * nblk);
    const dbl2* rows = reinterpret_cast<const dbl2*>(r + (size_t)nb * nb2);
#pragma unroll
    for (int u = 0; u < SA; ++u) sa[u] = blk[min(tid + u * nthr, nblk - 1)];
#pragma unroll
    for (int u = 0; u < kStageB; ++u) sb[u] = rows[min(tid + u * nthr, nb2 - 1)];
  };
  auto stage = [&]() {
#pragma unroll
    for (int u = 0; u < SA; ++u) {
      const int e = tid + u * nthr, col = e / n2;
      if (e < nblk) al[col * ldc + (e - col * n2)] = sa[u];
    }
#pragma unroll
    for (int u = 0; u < kStageB; ++u)
      if (tid + u * nthr < nb2) bl[tid + u * nthr] = sb[u];
  };
  // lane roles of the 16x16x4 product: A row rr, B column q, k = 4 t + kl
  const int rr = rt * 16 + (l & 15), kl = l >> 4;
  const int i = min(rr >> 1, n2 - 1), pr = rr & 1, pk = kl & 1, jl = kl >> 1;
  const int q = tt * 16 + (l & 15), qc = min(q, nrhs - 1);
  // real entry (rr, k) of the complex block: Re or Im of element (i, j), the
  // sign bit flipped for row pr = 0, column pk = 1 (-Im)
  const unsigned long long sgn = (pr == 0 && pk == 1) ? 0x8000000000000000ull : 0ull;
  const double* pa = reinterpret_cast<const double*>(al) + 2 * (jl * ldc + i) + (pr ^ pk);
  const double* pb = reinterpret_cast<const double*>(bl) + 2 * (jl * nrhs + qc) + pk;
  const int sa4 = 4 * ldc, sb4 = 4 * nrhs;  // doubles per step of t (j += 2)
  const int nk = n2 / 2;
  doublex4 acc = doublex4{0.0, 0.0, 0.0, 0.0};
  const int rounds = (9 + ng - 1) / ng;
  if (grp < 9) {
    fetch(grp);
    stage();
  }
  __syncthreads();
  for (int k = 0; k < rounds; ++k) {
    const int d = grp + k * ng, dn = d + ng;
    if (dn < 9) fetch(dn);
    if (d < 9) {
      for (int t = 0; t < nk; t += 4) {
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          av[u] = __longlong_as_double(__double_as_longlong(pa[(t + u) * sa4]) ^ sgn);
          bv[u] = pb[(t + u) * sb4];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
      }
    }
    if (k + 1 < rounds) {
      __syncthreads();  // every wave of the group is done with direction d
      if (dn < 9) stage();
      __syncthreads();
    }
  }
  if (ng > 1) {  // groups 1.. hand their tiles to group 0 (in group order)
    double* part = reinterpret_cast<double*>(dyn4);
    __syncthreads();
    if (grp > 0) {
      double* dst = part + ((size_t)((grp - 1) * wg + wv) * 64 + l) * 4;
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) dst[reg] = acc[reg];
    }
    __syncthreads();
    if (grp == 0) {
      for (int gg = 1; gg < ng; ++gg) {
        const double* src = part + ((size_t)((gg - 1) * wg + wv) * 64 + l) * 4;
#pragma unroll
        for (int reg = 0; reg < 4; ++reg) acc[reg] += src[reg];
      }
    }
  }
  if (grp == 0 && q < nrhs) {
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) {
      const int row = rt * 16 + 4 * reg + (l >> 4);
      if ((row >> 1) < n2) reinterpret_cast<double*>(w + ((size_t)s * n2 + (row >> 1)) * nrhs + q)[row & 1] = acc[reg];
    }
  }
}

// The staged K1 needs n2 % 8 == 0 and a group's block and waves within the
// staging registers.  Direction groups: one when the grid has several sites
// per compute unit (workgroups then overlap each other's loads), else the
// most of 3, 2 that fit 16 waves and the LDS limit.
constexpr int kCgcrStagedMinSites = 1024;
constexpr size_t kCgcrStagedLds = 128 * 1024;
inline int cgcr_staged_groups(int n2, int nrhs, long long nsite) {
  const int wg = mfma64_row_tiles(n2) * ((nrhs + 15) / 16);
  if (n2 % 8 != 0 || n2 > 64 || wg > 16 || n2 * n2 > kStageA * 64 * wg || n2 * nrhs > kStageB * 64 * wg ||
      cgcr_lds_bytes(n2, nrhs, 1) > kCgcrStagedLds)
    return 0;
  if (nsite < kCgcrStagedMinSites)
    for (int ng = 3; ng >= 2; --ng)
      if (ng * wg <= 16 && cgcr_lds_bytes(n2, nrhs, ng) <= kCgcrStagedLds) return ng;
  return 1;
}

// Dots (rhs-fast): partial c_i = <W_i, w>, d_i = <W_i, r> (i < j) and
// |w|^2, <w, r>, |r|^2 of one chunk of positions, stored in the value order of
// k_cgcr_coef.  Basis vectors are taken kCgcrDotIG per pass over the chunk.
__global__ __launch_bounds__(256) void k_cgcrT_dots(size_t npos, int nrhs, int j, int vals,
                                                    const cx<double>* __restrict__ Wb,
                                                    const cx<double>* __restrict__ w,
                                                    const cx<double>* __restrict__ r, double* part) {
  __shared__ double red[4 * kCgcrDotIG * 256];
  const int rows = 256 / nrhs, q = threadIdx.x % nrhs, rho = threadIdx.x / nrhs;
  const bool on = rho < rows;
  const size_t bs = npos * nrhs;
  const size_t cs = (npos + gridDim.x - 1) / gridDim.x, p0 = blockIdx.x * cs, p1 = p0 + cs < npos ? p0 + cs : npos;
  auto out = [&](int qq) { return part + ((size_t)qq * gridDim.x + blockIdx.x) * vals; };
  for (int i0 = 0; i0 == 0 || i0 < j; i0 += kCgcrDotIG) {
    const int ni = j - i0 < kCgcrDotIG ? j - i0 : kCgcrDotIG;
    double a[kCgcrDotIG][4] = {}, nv[4] = {};
    if (on) {
      for (size_t p = p0 + rho; p < p1; p += rows) {
        const size_t e = p * nrhs + q;
        const cx<double> wv = w[e], rv = r[e];
        if (i0 == 0) {
          nv[0] += wv.re * wv.re + wv.im * wv.im;
          nv[1] += wv.re * rv.re + wv.im * rv.im;
          nv[2] += wv.re * rv.im - wv.im * rv.re;
          nv[3] += rv.re * rv.re + rv.im * rv.im;
        }
#pragma unroll
        for (int u = 0; u < kCgcrDotIG; ++u) {
          if (u < ni) {
            const cx<double> bv = Wb[(size_t)(i0 + u) * bs + e];
            a[u][0] += bv.re * wv.re + bv.im * wv.im;
            a[u][1] += bv.re * wv.im - bv.im * wv.re;
            a[u][2] += bv.re * rv.re + bv.im * rv.im;
            a[u][3] += bv.re * rv.im - bv.im * rv.re;
          }
        }
      }
    }
    // value k = 4 u + c of this pass: c = 0, 1 -> c_i (re, im), 2, 3 -> d_i
    double flat[4 * kCgcrDotIG];
#pragma unroll
    for (int u = 0; u < kCgcrDotIG; ++u)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) flat[4 * u + cc] = a[u][cc];
    rhs_column_sums<4 * kCgcrDotIG>(flat, nrhs, rows, red, [&](int k, int qq, double sum) {
      const int u = k >> 2, cc = k & 3, i = i0 + u;
      if (u < ni) out(qq)[cc < 2 ? 2 * i + cc : 2 * j + 2 * i + (cc - 2)] = sum;
    });
    if (i0 == 0)
      rhs_column_sums<4>(nv, nrhs, rows, red, [&](int k, int qq, double sum) { out(qq)[4 * j + k] = sum; });
  }
}

// K3 (rhs-fast): w' = w - sum h_i W_i, z' = z - sum h_i Z_i, x += a z',
// r -= a w', partial |w'|^2 per rhs; frozen rhs are left unchanged.
// K3 (rhs-fast): w_j -= sum_i h_i W_i (kept, with |w_j|^2 for the next
// iteration) and r -= a w_j.  The search directions stay unorthogonalised
// (z_j = r_j as K1 copied it) and x is formed once per cycle by
// k_cgcrT_backsolve + k_cgcrT_combine from the recorded h and a.
__global__ __launch_bounds__(256) void k_cgcrT_update(size_t npos, int nrhs, int j, int kmax,
                                                      const cx<double>* __restrict__ Wb, cx<double>* __restrict__ w,
                                                      cx<double>* __restrict__ r, CgcrState S, double* p3) {
  __shared__ double red[256];
  const int rows = 256 / nrhs, q = threadIdx.x % nrhs, rho = threadIdx.x / nrhs;
  const bool on = rho < rows && S.act[q] != 0.0;
  const size_t bs = npos * nrhs;
  const size_t cs = (npos + gridDim.x - 1) / gridDim.x, p0 = blockIdx.x * cs, p1 = p0 + cs < npos ? p0 + cs : npos;
  double v = 0.0;
  if (on) {
    const double* h = S.h + (size_t)q * 2 * kmax;
    const cx<double> a = mk(S.a[2 * q], S.a[2 * q + 1]);
    for (size_t p = p0 + rho; p < p1; p += rows) {
      const size_t e = p * nrhs + q;
      cx<double> wv = w[e];
#pragma unroll 4
      for (int i = 0; i < j; ++i) wv = wv - mk(h[2 * i], h[2 * i + 1]) * Wb[(size_t)i * bs + e];
      w[e] = wv;
      r[e] = r[e] - a * wv;
      v += wv.re * wv.re + wv.im * wv.im;
    }
  }
  const double sum = rhs_column_sum(v, nrhs, rows, red);
  if ((int)threadIdx.x < nrhs) p3[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = sum;
}

// With orthogonalised directions z_m = z~_m - sum_{i<m} h_{m,i} z_i, the
// cycle's update sum_m a_m z_m equals sum_m y_m z~_m for
// y_m = a_m - sum_{i>m} y_i h_{i,m}, taken from the last direction down.
// One thread per rhs; y_m lands at [2 kmax + 2] of row m of the history.
__global__ __launch_bounds__(64) void k_cgcrT_backsolve(int nrhs, int J, int kmax, double* __restrict__ hist) {
  const int q = threadIdx.x;
  if (q >= nrhs) return;
  const size_t st = 2 * (size_t)kmax + 4;
  double* hq = hist + (size_t)q * kmax * st;
  for (int m = J - 1; m >= 0; --m) {
    cx<double> y = mk(hq[m * st + 2 * kmax], hq[m * st + 2 * kmax + 1]);
    for (int i = m + 1; i < J; ++i)
      y = y - mk(hq[i * st + 2 * kmax + 2], hq[i * st + 2 * kmax + 3]) * mk(hq[i * st + 2 * m], hq[i * st + 2 * m + 1]);
    hq[m * st + 2 * kmax + 2] = y.re;
    hq[m * st + 2 * kmax + 3] = y.im;
  }
}

// x += sum_{m<J} y_m z~_m (rhs-fast vectors, element e belongs to rhs e % nrhs).
__global__ __launch_bounds__(256) void k_cgcrT_combine(size_t npos, int nrhs, int J, int kmax,
                                                       const cx<double>* __restrict__ Zb,
                                                       const double* __restrict__ hist, cx<double>* __restrict__ x) {
  const size_t bs = npos * nrhs;
  const size_t st = 2 * (size_t)kmax + 4;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < bs; e += (size_t)gridDim.x * blockDim.x) {
    const double* yq = hist + (size_t)(e % nrhs) * kmax * st + 2 * kmax + 2;
    cx<double> xv = x[e];
    for (int m = 0; m < J; ++m) xv = xv + mk(yq[m * st], yq[m * st + 1]) * Zb[(size_t)m * bs + e];
    x[e] = xv;
  }
}

template <typename R>
__global__ void k_coarse_shift(cx<R>* Dc, int nsite, int n2, double dm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsite * n2) return;
  const int s = i / n2, r = i % n2;
  cx<R>* x = Dc + ((size_t)s * 9 + 8) * n2 * n2;
  x[(size_t)r * n2 + r].re += (R)dm;
}

template <class Side>
void launch_build(Ctx& c, const Side& side, const Level& f, Level& cl, int dof) {
  const AggGeom a = make_agg(f);
  const int n2 = 2 * f.nv;
  // LDS budget ~48 KiB: cs sites of V (dof x nv) and T (dof x cc) columns.
  int cc = n2;
  int cs = 4;
  auto bytes = [&](int cs_, int cc_) { return (size_t)cs_ * dof * (f.nv + cc_) * sizeof(cx<double>); };
  while (cs > 1 && (bytes(cs, cc) > 48 * 1024 || cs * cc > 256)) --cs;
  while (cc > 1 && (bytes(cs, cc) > 48 * 1024 || n2 * cc > 16 * 256)) cc = (cc + 1) / 2;
  const int nagg = cl.nsite;
  ProfScope ps(c, WDMG_K_DC_BUILD, nagg);
  hipLaunchKernelGGL((k_coarse_build<Side>), dim3(nagg, 9), dim3(256), bytes(cs, cc), c.stream, side, a, f.V64,
                     f.n, f.nv, dof, cs, cc, cl.Dc64);
  WDMG_HIP(hipGetLastError());
}

}  // namespace

void coarse_build0(Ctx& c, const Level& f, Level& cl) {
  WilsonSide side{c.U64, 4.0 + c.mass, c.t_bc < 0 ? 1 : 0};
  launch_build(c, side, f, cl, 12);
}

void coarse_buildC(Ctx& c, const Level& f, Level& cl) {
  StencilSide side{f.Dc64, f.dof};
  launch_build(c, side, f, cl, f.dof);
}

template <typename R>
void coarse_apply(Ctx& c, const Level& cl, const cx<R>* Dc, cx<R>* out, const cx<R>* in, int nrhs, cx<R>* copy) {
  const int n2 = cl.dof;
  if (nrhs >= kMfmaMinRhs && n2 <= 64) {
    // matrix-core path for a batch of right-hand sides
    if constexpr (sizeof(R) == 8) {
      ProfScope ps(c, WDMG_K_DC_MFMA_F64, (long long)cl.nsite * nrhs);
      const int waves = mfma64_row_tiles(n2) * mfma64_groups(n2);
      const dim3 grid(cl.nsite), block(64 * waves);
      switch ((nrhs + 15) / 16) {
        case 1: hipLaunchKernelGGL(k_coarse_apply_mfma64<1>, grid, block, 0, c.stream, cl.g, n2, nrhs, Dc, in, out, copy); break;
        case 2: hipLaunchKernelGGL(k_coarse_apply_mfma64<2>, grid, block, 0, c.stream, cl.g, n2, nrhs, Dc, in, out, copy); break;
        case 3: hipLaunchKernelGGL(k_coarse_apply_mfma64<3>, grid, block, 0, c.stream, cl.g, n2, nrhs, Dc, in, out, copy); break;
        default: hipLaunchKernelGGL(k_coarse_apply_mfma64<kMaxTiles>, grid, block, 0, c.stream, cl.g, n2, nrhs, Dc, in, out, copy); break;
      }
    } else {
      ProfScope ps(c, WDMG_K_DC_MFMA_F32, (long long)cl.nsite * nrhs);
      const int waves = (2 * n2 + 31) / 32;
      hipLaunchKernelGGL(k_coarse_apply_mfma32, dim3(cl.nsite, (nrhs + 31) / 32), dim3(64 * waves), 0, c.stream,
                         cl.g, n2, nrhs, Dc, in, out, copy);
    }
    WDMG_HIP(hipGetLastError());
    c.n_Dc[cl.l] += nrhs;
    return;
  }
  ProfScope ps(c, sizeof(R) == 8 ? WDMG_K_DC_F64 : WDMG_K_DC_F32, (long long)cl.nsite * nrhs);
  hipLaunchKernelGGL((k_coarse_apply<R>), dim3(cl.nsite, nrhs), dim3(576), 0, c.stream, cl.g, cl.dof, Dc, in, out,
                     copy);
  WDMG_HIP(hipGetLastError());
  c.n_Dc[cl.l] += nrhs;
}

void coarse_shift(Ctx& c, Level& cl, double dm) {
  if (!cl.Dc64 || !cl.Dc32) throw Error(WDMG_ERR_ARG, "coarse blocks released by wdmg_release_unused");
  const int n = cl.nsite * cl.dof;
  hipLaunchKernelGGL((k_coarse_shift<double>), dim3((n + 255) / 256), dim3(256), 0, c.stream, cl.Dc64, cl.nsite,
                     cl.dof, dm);
  WDMG_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_coarse_shift<float>), dim3((n + 255) / 256), dim3(256), 0, c.stream, cl.Dc32, cl.nsite,
                     cl.dof, dm);
  WDMG_HIP(hipGetLastError());
  cl.dc16_kind = 0;  // the 16-bit copy is remade from the shifted FP64 blocks on next use
}

void ensure_dc16(Ctx& c, Level& cl, int kind) {
  const int n2 = cl.dof;
  const size_t nblk = (size_t)cl.nsite * 9, nn = (size_t)n2 * n2;
  if (cl.dc16_kind != kind) {
    if (!cl.Dc64) throw Error(WDMG_ERR_ARG, "FP64 coarse blocks released by wdmg_release_unused");
    if (!cl.Dc16) {
      cl.Dc16 = dev_alloc(c, nblk * nn * 4);
      cl.Dc16s = static_cast<float*>(dev_alloc(c, nblk * sizeof(float)));
    }
    if (kind == WDMG_F16)
      hipLaunchKernelGGL((k_dc_to_half<f16_t>), dim3((unsigned)nblk), dim3(256), 0, c.stream, cl.Dc64,
                         static_cast<cxh<f16_t>*>(cl.Dc16), cl.Dc16s, (int)nn);
    else
      hipLaunchKernelGGL((k_dc_to_half<bf16_t>), dim3((unsigned)nblk), dim3(256), 0, c.stream, cl.Dc64,
                         static_cast<cxh<bf16_t>*>(cl.Dc16), cl.Dc16s, (int)nn);
    WDMG_HIP(hipGetLastError());
    cl.dc16_kind = kind;
  }
}

void coarse_apply_h(Ctx& c, Level& cl, int kind, cx<float>* out, const cx<float>* in, int nrhs, cx<float>* copy) {
  const int n2 = cl.dof;
  const size_t nn = (size_t)n2 * n2;
  ensure_dc16(c, cl, kind);
  if (nrhs >= kMfmaMinRhs && n2 <= 64) {
    ProfScope ps(c, WDMG_K_DC_MFMA_H, (long long)cl.nsite * nrhs);
    const int waves = (2 * n2 + 31) / 32;
    const size_t lds = nn * 4;
    // small batches stage at most two rhs rows per thread (fewer registers)
    const bool few = (nrhs < 32 ? nrhs : 32) * n2 <= 2 * 64 * waves;
    const dim3 grid(cl.nsite, (nrhs + 31) / 32), block(64 * waves);
    if (kind == WDMG_F16) {
      const auto* d16 = static_cast<const cxh<f16_t>*>(cl.Dc16);
      if (few)
        hipLaunchKernelGGL((k_coarse_apply_mfma16<f16_t, 2>), grid, block, lds, c.stream, cl.g, n2, nrhs, d16,
                           cl.Dc16s, in, out, copy);
      else
        hipLaunchKernelGGL((k_coarse_apply_mfma16<f16_t>), grid, block, lds, c.stream, cl.g, n2, nrhs, d16, cl.Dc16s,
                           in, out, copy);
    } else {
      const auto* d16 = static_cast<const cxh<bf16_t>*>(cl.Dc16);
      if (few)
        hipLaunchKernelGGL((k_coarse_apply_mfma16<bf16_t, 2>), grid, block, lds, c.stream, cl.g, n2, nrhs, d16,
                           cl.Dc16s, in, out, copy);
      else
        hipLaunchKernelGGL((k_coarse_apply_mfma16<bf16_t>), grid, block, lds, c.stream, cl.g, n2, nrhs, d16,
                           cl.Dc16s, in, out, copy);
    }
  } else {
    ProfScope ps(c, WDMG_K_DC_H, (long long)cl.nsite * nrhs);
    if (kind == WDMG_F16)
      hipLaunchKernelGGL((k_coarse_apply_h<f16_t>), dim3(cl.nsite, nrhs), dim3(576), 0, c.stream, cl.g, n2,
                         static_cast<const cxh<f16_t>*>(cl.Dc16), cl.Dc16s, in, out, copy);
    else
      hipLaunchKernelGGL((k_coarse_apply_h<bf16_t>), dim3(cl.nsite, nrhs), dim3(576), 0, c.stream, cl.g, n2,
                         static_cast<const cxh<bf16_t>*>(cl.Dc16), cl.Dc16s, in, out, copy);
  }
  WDMG_HIP(hipGetLastError());
  c.n_Dc[cl.l] += nrhs;
}

void coarsest_gcr(Ctx& c, Level& L, cx<double>* x, const cx<double>* b, int nrhs, double tol, int k, int maxit) {
  const int n2 = L.dof;
  const size_t n = L.n, bs = (size_t)nrhs * n;
  double* gb = c.dsc + gcr_base(L.l);
  CgcrState S{gb + G_H, gb + G_NRM, gb + G_A, gb + G_RN, gb + G_ACT, gb + G_TOL};
  const int g1 = L.nsite < kCgcrG1 ? L.nsite : kCgcrG1;
  const int waves = mfma64_row_tiles(n2) * mfma64_groups(n2);
  const int form = c.tune_force[WDMG_TUNE_COARSE_APPLY];
  const int sgroups = nrhs >= 2 && form != 0 ? cgcr_staged_groups(n2, nrhs, L.nsite) : 0;
  if (nrhs == 1 && (size_t)(4 * k + 4) * sizeof(double) > 96 * 1024)
    throw Error(WDMG_ERR_ARG, "coarse_restart too long (LDS)");
  static bool lds_attr = false;
  if (!lds_attr) {  // the single-rhs K1 keeps 4 j + 4 partial sums in LDS, the staged one a block
    WDMG_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cgcr_apply),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
    for (const void* f : {reinterpret_cast<const void*>(&k_cgcrT_apply_lds<2>),
                          reinterpret_cast<const void*>(&k_cgcrT_apply_lds<4>),
                          reinterpret_cast<const void*>(&k_cgcrT_apply_lds<kStageA>)})
      WDMG_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCgcrStagedLds));
    lds_attr = true;
  }
  // a batch keeps its vectors rhs-fast for the whole solve (x in L.xT)
  const bool fast = nrhs >= 2;
  const size_t npos = (size_t)L.nsite * n2;
  long long g1t = ((long long)npos * nrhs + 511) / 512;
  if (g1t > 1024) g1t = 1024;
  const int g1f = (int)g1t;
  cx<double>* r = L.w64[1];
  if (fast) {
    hipLaunchKernelGGL(k_cgcrT_init, dim3(kCgcrG3T), dim3(256), 0, c.stream, npos, nrhs, b, L.xT, r, L.cpart3);
    WDMG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cgcrT_init_fin, dim3(nrhs), dim3(64), 0, c.stream, nrhs, kCgcrG3T, L.cpart3, tol, S,
                       c.dsc + S_ERR);
  } else {
    hipLaunchKernelGGL(k_cgcr_init, dim3(nrhs), dim3(256), 0, c.stream, b, x, r, n, tol, S, c.dsc + S_ERR);
  }
  WDMG_HIP(hipGetLastError());
  // The active flags of iteration it land in pinned memory and are inspected
  // `lag` iterations later, so the stream never drains while the host waits.
  const int lag = 2;
  auto done_at = [&](int i) {
    WDMG_HIP(hipEventSynchronize(c.ring_ev[i % kRing]));
    const double* f = c.hring + (size_t)(i % kRing) * kMaxRhs;
    for (int q = 0; q < nrhs; ++q)
      if (f[q] != 0.0) return false;
    return true;
  };
  // batch: x += sum_m y_m z~_m over the J directions of the cycle just ended
  auto combine = [&](int J) {
    hipLaunchKernelGGL(k_cgcrT_backsolve, dim3(1), dim3(64), 0, c.stream, nrhs, J, k, L.chist);
    WDMG_HIP(hipGetLastError());
    const size_t nb = (npos * nrhs + 255) / 256;
    hipLaunchKernelGGL(k_cgcrT_combine, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, c.stream, npos, nrhs,
                       J, k, L.basisZ, L.chist, L.xT);
    WDMG_HIP(hipGetLastError());
  };
  const int fixed = c.capturing ? (c.coarse_fixed_iters < maxit ? c.coarse_fixed_iters : maxit) : 0;
  int it = 0;
  for (; it < (c.capturing ? fixed : maxit); ++it) {
    const int j = it % k;
    cx<double>* w = L.basisW + (size_t)j * bs;
    cx<double>* z = L.basisZ + (size_t)j * bs;
    const int vals = 4 * j + 4;
    if (fast) {
      {
        ProfScope ps(c, WDMG_K_COARSE_GCR, (long long)L.nsite * nrhs);
        const dim3 grid(L.nsite);
        if (sgroups) {
          const int nthr = 64 * mfma64_row_tiles(n2) * ((nrhs + 15) / 16);
          const size_t lb = cgcr_lds_bytes(n2, nrhs, sgroups);
          const dim3 block(nthr * sgroups);
          if (n2 * n2 <= 2 * nthr)
            hipLaunchKernelGGL(k_cgcrT_apply_lds<2>, grid, block, lb, c.stream, L.g, n2, nrhs, sgroups, L.Dc64, r, w,
                               z);
          else if (n2 * n2 <= 4 * nthr)
            hipLaunchKernelGGL(k_cgcrT_apply_lds<4>, grid, block, lb, c.stream, L.g, n2, nrhs, sgroups, L.Dc64, r, w,
                               z);
          else
            hipLaunchKernelGGL(k_cgcrT_apply_lds<kStageA>, grid, block, lb, c.stream, L.g, n2, nrhs, sgroups, L.Dc64,
                               r, w, z);
        } else {
          const dim3 block(64 * waves);
          switch ((nrhs + 15) / 16) {
            case 1: hipLaunchKernelGGL(k_cgcrT_apply<1>, grid, block, 0, c.stream, L.g, n2, nrhs, L.Dc64, r, w, z); break;
            case 2: hipLaunchKernelGGL(k_cgcrT_apply<2>, grid, block, 0, c.stream, L.g, n2, nrhs, L.Dc64, r, w, z); break;
            case 3: hipLaunchKernelGGL(k_cgcrT_apply<3>, grid, block, 0, c.stream, L.g, n2, nrhs, L.Dc64, r, w, z); break;
            default:
              hipLaunchKernelGGL(k_cgcrT_apply<kMaxTiles>, grid, block, 0, c.stream, L.g, n2, nrhs, L.Dc64, r, w, z);
              break;
          }
        }
        WDMG_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(k_cgcrT_dots, dim3(g1f), dim3(256), 0, c.stream, npos, nrhs, j, vals, L.basisW, w, r,
                         L.cpart);
      WDMG_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_cgcr_coef, dim3(nrhs), dim3(1024), (size_t)(vals + 1) * sizeof(double), c.stream, j, vals,
                         g1f, L.cpart, L.cpart3, kCgcrG3T, k, S,
                         c.capturing ? nullptr : c.dring + (size_t)(it % kRing) * kMaxRhs, c.dsc + S_ERR, L.chist);
      WDMG_HIP(hipGetLastError());
      if (!c.capturing) WDMG_HIP(hipEventRecord(c.ring_ev[it % kRing], c.stream));
      hipLaunchKernelGGL(k_cgcrT_update, dim3(kCgcrG3T), dim3(256), 0, c.stream, npos, nrhs, j, k, L.basisW, w, r, S,
                         L.cpart3);
      WDMG_HIP(hipGetLastError());
      if (j == k - 1) combine(k);
      c.n_Dc[L.l] += nrhs;
      if (!c.capturing && it >= lag && done_at(it - lag)) {
        ++it;
        break;
      }
      continue;
    }
    {
      ProfScope ps(c, WDMG_K_COARSE_GCR, (long long)L.nsite * nrhs);
      hipLaunchKernelGGL(k_cgcr_apply, dim3(g1), dim3(576), (size_t)vals * sizeof(double), c.stream, L.g, n2, nrhs,
                         j, vals, L.Dc64, r, L.basisW, w, z, L.cpart);
      WDMG_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_cgcr_coef, dim3(nrhs), dim3(1024), (size_t)(vals + 1) * sizeof(double), c.stream, j, vals,
                       g1, L.cpart, L.cpart3, kCgcrG3, k, S,
                       c.capturing ? nullptr : c.dring + (size_t)(it % kRing) * kMaxRhs, c.dsc + S_ERR, nullptr);
    WDMG_HIP(hipGetLastError());
    if (!c.capturing) WDMG_HIP(hipEventRecord(c.ring_ev[it % kRing], c.stream));
    hipLaunchKernelGGL(k_cgcr_update, dim3(kCgcrG3, nrhs), dim3(256), 0, c.stream, n, nrhs, j, k, L.basisW,
                       L.basisZ, w, z, x, r, S, L.cpart3);
    WDMG_HIP(hipGetLastError());
    c.n_Dc[L.l] += nrhs;
    if (!c.capturing && it >= lag && done_at(it - lag)) {
      ++it;
      break;
    }
  }
  if (fast) {
    if (it > 0 && (it - 1) % k != k - 1) combine((it - 1) % k + 1);
    hipLaunchKernelGGL(k_cgcrT_out, dim3((unsigned)((npos * nrhs + 255) / 256)), dim3(256), 0, c.stream, npos, nrhs,
                       L.xT, x);
    WDMG_HIP(hipGetLastError());
  }
  if (it > c.last_coarse_iters) c.last_coarse_iters = it;
}

size_t coarsest_gcr_partials(int nrhs, int k) {
  return (size_t)nrhs * kCgcrG1 * (4 * k + 4);
}
size_t coarsest_gcr_history(int nrhs, int k) { return (size_t)nrhs * k * (2 * (size_t)k + 4); }
size_t coarsest_gcr_partials3(int nrhs) { return (size_t)nrhs * (kCgcrG3T > kCgcrG3 ? kCgcrG3T : kCgcrG3); }

template void coarse_apply<double>(Ctx&, const Level&, const cx<double>*, cx<double>*, const cx<double>*, int,
                                   cx<double>*);
template void coarse_apply<float>(Ctx&, const Level&, const cx<float>*, cx<float>*, const cx<float>*, int,
                                  cx<float>*);

}  // namespace wdmg
