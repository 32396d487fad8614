/*
 * wdmg_2d.h -- C ABI of the 2d U(1) Wilson-Dirac workload of libwdmg: the
 * multigrid comparison of Sec. 4 of Clark et al., "The removal of critical
 * slowing down" (Lattice 2008): 3-level V(2,2) cycles on 4^2 blocks with an
 * exact coarsest solve, MG-BiCGstab (multigrid on D), MG-CG (multigrid on the
 * normal equations D^dagger D, Sec. 3) and CG on the normal equations.
 *
 * The rules of wdmg.h apply (caller-owned device buffers, one HIP stream,
 * WDMG_OK / WDMG_ERR_* / WDMG_NOT_CONVERGED return codes, no exception across
 * the ABI, the wdmg_alloc device-memory provider).  Everything is FP64
 * (complex128).
 *
 * Operator (the 2d form of the Sec. 1 operator):
 *   (D psi)(x) = (2 + m) psi(x)
 *                - 1/2 sum_{mu=0,1} [ (1 - gamma_mu) U_mu(x) psi(x + mu)
 *                                   + (1 + gamma_mu) conj(U_mu(x - mu)) psi(x - mu) ]
 * gamma_0 = sigma_1, gamma_1 = sigma_2, gamma5 = sigma_3 = diag(1, -1)
 * (chirality + is spin 0); mu = 0 is x (periodic), mu = 1 is t (a hop across
 * the t boundary carries t_bc = +1 or -1).
 *
 * Canonical layouts (x fastest, complex interleaved re/im):
 *   links        : [T][X][mu=2] complex128, U_mu(x) of modulus 1;
 *   fine field   : [nrhs][T][X][spin=2];
 *   level-l field: [nrhs][Tl][Xl][chirality=2][n_l], n_0 = 1, n_l = Nv_{l-1}
 *     (with spin blocking: [nrhs][Tl][Xl][1][n_l], n_0 = 2);
 *   prolongator of coarsening l: [Nv][Tl][Xl][g][n_l] (g = 2, or 1 with spin
 *     blocking), the block-orthonormal columns: column (aggregate, chi, k) is
 *     entry k restricted to the aggregate and group chi;
 *   coarse operator of level l >= 1: S blocks of (g n_l)^2 per site (S = 5 for D_c: offsets
 *     (0,0), (+1,0), (-1,0), (0,+1), (0,-1) in (x, t); S = 9 for the normal
 *     operator: those and (+1,+1), (-1,+1), (+1,-1), (-1,-1)),
 *     (A_c c)(xhat) = sum_o B_o(xhat) c(xhat + d_o), periodic coarse indexing.
 */
#ifndef WDMG_2D_H
#define WDMG_2D_H

#include "wdmg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wdmg_2d_ctx wdmg_2d_ctx;

#define WDMG_2D_MAX_LEVELS 3

typedef struct {
  int n_levels;            /* 2 or 3 (fine level included)                          */
  int block[2];            /* aggregate extents (b_x, b_t), the same at every
                              coarsening; paper 4 x 4 (Sec. 4)                       */
  int nv[WDMG_2D_MAX_LEVELS - 1];  /* near-null vectors per coarsening, 1..16; paper
                              3 for MG-BiCGstab, 8 for MG-CG (Sec. 4)                */
  int setup_iters;         /* MR steps relaxing A_l v = 0 from the starting vectors
                              (Sec. 2); 0 takes them as given                        */
  const void* vectors[WDMG_2D_MAX_LEVELS - 1];  /* device: nv[l] starting vectors in
                              the level-l layout ([nv][Tl][Xl][2][n_l]); required    */
  int normal;              /* 0: hierarchy of D (MG-BiCGstab); 1: hierarchy of
                              A = D^dagger D (Sec. 3 normal equations, MG-CG)         */
  double omega;            /* MR under-relaxation, paper 0.8 (Sec. 3)                */
  int nu_pre, nu_post;     /* V(nu_pre, nu_post), paper 2, 2 (Sec. 4)                */
  int use_alpha;           /* 1: minimal-residual step after each prolongation (Sec. 3) */
  int coarse_cycles;       /* cycles of an intermediate level per correction (three
                              levels): 1 is the V-cycle of Sec. 4; k > 1 runs
                              e <- e + M_1 (r_c - A_1 e) k times from e = 0, the
                              modified cycle of Sec. 5 (k = 4 there), 1..64          */
  int blocking;            /* 0: chirality kept intact (Sec. 3), the method.  The
                              negative control of the Sec. 3 footnote, two levels of D
                              only (else WDMG_ERR_ARG): both spins in one block per
                              aggregate (coarse dof per site Nv, level-1 fields
                              [Tl][Xl][1][Nv]), restricted with 1: P^dagger gamma5
                              (coarse operator P^dagger gamma5 D P, singular for the
                              free-field constant) or 2: P^dagger                   */
} wdmg_2d_mg_params;

typedef struct {
  int iters;               /* outer iterations                                       */
  int converged;           /* 1 when ||b - D x|| / ||b|| <= tol                       */
  double true_res;         /* ||b - D x|| / ||b||, recomputed in FP64 at the end      */
  long long wilson;        /* fine-level applications of D or D^dagger (Sec. 4 metric;
                              D^dagger D counts two), outer solver and cycles          */
  long long coarse_applies[WDMG_2D_MAX_LEVELS];  /* stencil applications per level
                              (index 0 unused); the coarsest counts its exact solves  */
  double flops;            /* 8 x complex multiply-adds of every operator, transfer
                              and coarsest-solve application (vector updates excluded) */
  double seconds;          /* wall time of the solve (stream synchronised)           */
} wdmg_2d_stats;

/* Lattice Lx x Lt (each even, >= 4).  alloc/hip_stream as for wdmg_create. */
int wdmg_2d_create(wdmg_2d_ctx** out, const int dims[2], const wdmg_alloc* alloc, void* hip_stream);
void wdmg_2d_destroy(wdmg_2d_ctx* ctx);
const char* wdmg_2d_last_error(const wdmg_2d_ctx* ctx);

/* Links (device, canonical layout, copied) and t boundary sign (+1 or -1).
 * Drops any hierarchy. */
int wdmg_2d_set_gauge(wdmg_2d_ctx* ctx, const void* links, int t_bc);
/* Bare mass m of the operator above.  Drops any hierarchy. */
int wdmg_2d_set_mass(wdmg_2d_ctx* ctx, double m);

/* out = D in (dagger = 0) or D^dagger in = gamma5 D gamma5 in (dagger = 1),
 * nrhs fine fields; out and in must not overlap. */
int wdmg_2d_apply_D(wdmg_2d_ctx* ctx, void* out, const void* in, int nrhs, int dagger);

/* Adaptive setup (Sec. 2) of the hierarchy of D or D^dagger D: per coarsening,
 * relaxation of the starting vectors, block QR per aggregate and chirality
 * (Sec. 3, chirality kept intact), Galerkin operator P^dagger A P (read off by
 * coloured probing, the colours repeating with the smallest divisor >= 3 of
 * each coarse extent: every coarse extent must be >= 3, else WDMG_ERR_DIMS;
 * the coarsest level may hold at most 4096 unknowns), and on the coarsest level the
 * explicit inverse of its operator (Gauss-Jordan with partial pivoting), which
 * makes the coarsest solve exact to rounding (Sec. 4).  Errors:
 * WDMG_ERR_RANK_DEFICIENT (candidates dependent on an aggregate),
 * WDMG_ERR_NAN (a zero pivot: the coarsest operator is singular). */
int wdmg_2d_mg_setup(wdmg_2d_ctx* ctx, const wdmg_2d_mg_params* params);

/* Prolongator columns of coarsening `level` (0-based) into `q` (device,
 * canonical layout above). */
int wdmg_2d_get_prolongator(wdmg_2d_ctx* ctx, int level, void* q);
/* out = A_l in for level l >= 1 (the stencil; level-l layout), nrhs fields. */
int wdmg_2d_apply_coarse(wdmg_2d_ctx* ctx, int level, void* out, const void* in, int nrhs);
/* Restriction P^dagger from level l to l + 1 and prolongation P from l + 1 to l
 * (Sec. 2, R = P^dagger), nrhs fields. */
int wdmg_2d_restrict(wdmg_2d_ctx* ctx, int level, void* out, const void* in, int nrhs);
int wdmg_2d_prolong(wdmg_2d_ctx* ctx, int level, void* out, const void* in, int nrhs);
/* Coarse-operator blocks of level l >= 1 into `blocks` (device,
 * [S][Tl][Xl][2 n_l][2 n_l], row index first); S as above. */
int wdmg_2d_get_coarse_operator(wdmg_2d_ctx* ctx, int level, void* blocks);
/* x = M r: one V(nu_pre, nu_post) cycle from x = 0 on the fine level (of D or of
 * D^dagger D, as set up); one fine field each. */
int wdmg_2d_vcycle(wdmg_2d_ctx* ctx, void* x, const void* r);

/* Solve D x = b for one fine field, from x = 0, until ||b - D x|| / ||b|| <= tol
 * or maxit outer iterations:
 *   method 0: MG-BiCGstab, BiCGstab with the V-cycle of the hierarchy of D as
 *             right preconditioner (Sec. 4); restarts from the true residual;
 *   method 1: MG-CG, flexible CG on D^dagger D x = D^dagger b with the V-cycle
 *             of the normal hierarchy (Sec. 3, Sec. 4);
 *   method 2: CG on D^dagger D x = D^dagger b (the CG of Sec. 4), no hierarchy.
 * The CG methods drive the normal residual to 1e-2 tol ||b|| and then check the
 * true residual.  x and b must not overlap.  stats may be NULL.  A b holding
 * NaN or Inf, or a residual turning NaN, ends the solve with WDMG_ERR_NAN. */
int wdmg_2d_solve(wdmg_2d_ctx* ctx, void* x, const void* b, int method, double tol, int maxit,
                  wdmg_2d_stats* stats);

#ifdef __cplusplus
}
#endif

#endif
