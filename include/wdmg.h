/*
 * wdmg.h -- C ABI of libwdmg, an adaptive-multigrid solver for the 4d SU(3)
 * Wilson-Dirac system D x = b on one AMD Instinct MI355X (gfx950).
 *
 * Method: M. A. Clark, J. Brannick, R. C. Brower, S. F. McCormick,
 * T. A. Manteuffel, J. C. Osborn, C. Rebbi, "The removal of critical slowing
 * down", Lattice 2008.  Section numbers below refer to that paper.
 *
 * General rules
 *  - Every pointer argument named "device" is a device (HBM) pointer owned by
 *    the caller; the library never frees it and never keeps it after the call
 *    returns (inputs are copied into library-owned layouts).
 *  - All work is enqueued on the HIP stream given to wdmg_create.  Calls that
 *    return values to the host (setup, solve) synchronise that stream.
 *  - Every call returns WDMG_OK (0) on success, a negative WDMG_ERR_* on
 *    failure (nothing enqueued after the failing step; wdmg_last_error gives
 *    a message), or WDMG_NOT_CONVERGED (> 0) when a solve stopped at its
 *    iteration cap with its statistics filled.  No C++ exception crosses the
 *    ABI.
 *  - Canonical layouts (x fastest, complex interleaved re/im):
 *      gauge field : [T][Z][Y][X][mu=4][3][3] complex128, U_mu(x)[a][b] takes
 *                    colour b at x+mu to colour a at x; mu = 0..3 = x,y,z,t.
 *      fine field  : [nrhs][T][Z][Y][X][spin=4][colour=3]
 *      coarse field at level l >= 1 : [nrhs][T][Z][Y][X][chirality=2][Nv]
 *    with the chiral gamma basis, gamma5 = diag(1,1,-1,-1): chirality + is
 *    spins {0,1}.  Element type: complex128 for WDMG_F64, complex64 for the
 *    other precisions (which run lower-precision kernels on FP32 I/O).
 */
#ifndef WDMG_H
#define WDMG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WDMG_OK = 0,
  WDMG_NOT_CONVERGED = 1,
  WDMG_ERR_ARG = -1,            /* null pointer, bad size, bad enum value   */
  WDMG_ERR_DIMS = -2,           /* lattice or block extents not compatible  */
  WDMG_ERR_OOM = -3,            /* device allocation failed                 */
  WDMG_ERR_HIP = -4,            /* a HIP runtime call failed                */
  WDMG_ERR_NOT_SETUP = -5,      /* gauge field or multigrid hierarchy missing */
  WDMG_ERR_NAN = -6,            /* NaN/Inf met in a reduction or the input  */
  WDMG_ERR_RANK_DEFICIENT = -7  /* candidate vectors dependent on an aggregate */
};

/* Precision of a kernel path.  WDMG_F16 and WDMG_BF16 store fields and
 * operators in 16 bits and compute in FP32:
 *  - a fine field keeps, per site, an FP32 scale s = the largest magnitude of
 *    its 24 real components and the values fl16(fl32(v * fl32(1/s))), each
 *    rounded to nearest-even (first to FP32, then to the 16-bit format); a
 *    site with s below the smallest normal FP32 number is stored as zero;
 *  - links and prolongator columns (entries of magnitude <= 1) are stored
 *    unscaled, rounded from FP64 to FP32 to 16 bits;
 *  - coarse-operator blocks keep one FP32 scale per (2Nv x 2Nv) block and
 *    coarse vectors stay in FP32. */
enum { WDMG_F64 = 0, WDMG_F32 = 1, WDMG_F16 = 2, WDMG_BF16 = 3 };

#define WDMG_MAX_LEVELS 4

typedef struct wdmg_ctx wdmg_ctx;

/* Device-memory provider.  alloc(bytes, user) returns device memory aligned
 * to 256 bytes, or NULL when it has none (the call then fails with
 * WDMG_ERR_OOM; a misaligned pointer is rejected the same way); free(ptr,
 * user) releases it.  Neither may unwind through the library (a callback
 * written in another language must catch its own errors).  Pass NULL to
 * wdmg_create for hipMalloc/hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} wdmg_alloc;

/* Per coarsening l (level l -> l+1) of the hierarchy (Sec. 2 setup, Sec. 3
 * blocking, Sec. 5 4d parameters). */
typedef struct {
  int block[4];          /* aggregate extents (bx,by,bz,bt); must divide the level's dims */
  int nv;                /* near-null vectors Nv (coarse dof per site = 2 Nv), 1..32 */
  int setup_iters;       /* MR relaxation steps on D v = 0 (0: take the vectors as given) */
  const void* vectors;   /* device: nv starting vectors, canonical complex128 layout of
                            level l ([nv][sites][dof]); required */
  int setup_prec;        /* arithmetic of the relaxation: WDMG_F64 or WDMG_F32, or at
                            level 0 also WDMG_F16 / WDMG_BF16 (vectors, residuals
                            and D r in 16-bit storage with per-site scales, FP32
                            arithmetic); the block orthonormalisation is FP64
                            either way                                              */
  int adapt_iters;       /* adaptive augmentation (Sec. 2): after the relaxation,
                            candidate k = 2..nv is refined by this many stationary
                            iterations x <- x - M A x of the two-level multigrid
                            built from candidates 1..k-1 (FP64, this level and its
                            coarse level, the coarse level solved as the coarsest);
                            0: relaxation only                                      */
} wdmg_level_params;

typedef struct {
  int n_levels;                  /* 2 or 3 (fine level included)                      */
  wdmg_level_params level[WDMG_MAX_LEVELS - 1];
  double omega;                  /* MR under-relaxation, paper value 0.8 (Sec. 3)     */
  int nu_pre, nu_post;           /* V(nu_pre, nu_post), paper value 2, 2 (Sec. 5)      */
  int coarse_cycles;             /* next-level cycles between the fine restriction and
                                    prolongation of a 3-level hierarchy; paper 4 (Sec. 5) */
  double coarse_tol;             /* relative tolerance of the coarsest GCR solve       */
  int coarse_maxit;              /* iteration cap of the coarsest solve                 */
  int coarse_restart;            /* restart length of the coarsest GCR                  */
  int use_alpha;                 /* 1: minimal-residual step after prolongation (Sec. 3) */
  int normal;                    /* 1: also set up multigrid on the normal equations
                                    (Sec. 3, first approach): the candidates are relaxed on
                                    D^dagger D v = 0, and besides D_c the Galerkin operator
                                    (D^dagger D)_c = P^dagger D^dagger D P is built (33 blocks
                                    per coarse site, wdmg_apply_Nc), for MG-CG solves.  Two
                                    levels, aggregates of extent >= 2 and coarse extents >= 3
                                    only (else WDMG_ERR_ARG / WDMG_ERR_DIMS); FP64.         */
} wdmg_mg_params;

typedef struct {
  double tol;            /* stop when the true ||b - D x|| / ||b|| <= tol (FP64)   */
  int restart;           /* FGCR restart length k (paper GCR(50), Sec. 5)          */
  int maxit;             /* cap on outer iterations                                */
  int precond;           /* 0: plain GCR, 1: multigrid V-cycle                      */
  int mg_prec;           /* precision of the V-cycle: WDMG_F64, WDMG_F32, or WDMG_F16 /
                            WDMG_BF16 (16-bit fine fields, links, P and intermediate
                            coarse operators; the coarsest solve stays FP64).  Below
                            FP64 the outer basis z_j, w_j = D z_j is stored and
                            applied in FP32 (sums in FP64; x, r and the true
                            residual of every restart stay FP64), and a cycle
                            restarts from the true residual once its recursive
                            residual has fallen by 1e-5.                          */
  int use_graph;         /* 1: the first V-cycle of a solve runs as usual; it is then
                            captured once in a HIP graph that later iterations replay.
                            Inside the graph the coarsest GCR runs a fixed number of
                            iterations, 1.5x (rounded up, plus one) the count the first
                            V-cycle needed, at most coarse_maxit; right-hand sides that
                            reach coarse_tol earlier are frozen on the device.      */
  int outer;             /* outer Krylov method: 0 flexible GCR(restart) (Sec. 5); 1
                            BiCGStab with the V-cycle as right preconditioner (the
                            MG-BiCGstab of Sec. 4), one rhs after another, from x = 0
                            (x on input is ignored), restarting from the true residual
                            after a breakdown; use_graph does not apply to it; 2 CG on
                            the normal equations D^dagger D x = D^dagger b (the CG of
                            Sec. 4 and 5; precond and mg_prec ignored); 3 MG-CG (Sec. 4):
                            flexible CG on the normal equations preconditioned by the
                            two-level V-cycle on D^dagger D of a normal-equation
                            hierarchy (wdmg_mg_params.normal; coarse solve by CG to
                            coarse_tol).  2 and 3 run in FP64, one rhs after another,
                            from x = 0, and stop on the true residual of D x = b.      */
  int in_place;          /* 1 (FGCR with a V-cycle below FP64, restart >= 2, no graph):
                            the solve starts from x = 0 (x on input is ignored) and
                            keeps no internal copy of b; b is read from the caller's
                            buffer whenever the true residual is recomputed, so it must
                            stay unchanged during the call, and x may be the same
                            buffer as b (the solution then replaces b at the end).  Saves
                            one FP64 field per rhs, for the largest batches.  0: x and b
                            must be different buffers.                              */
} wdmg_solve_params;

typedef struct {
  int iters;             /* outer iterations (BiCGStab: iterations, two D each)    */
  int restarts;
  int converged;
  double true_res;       /* ||b - D x|| / ||b|| recomputed in FP64 at exit          */
  long long n_D;         /* applications of the fine operator, all precisions      */
  long long n_Dc[WDMG_MAX_LEVELS]; /* applications of the coarse operator per level */
  double seconds;        /* wall time of the solve of this right-hand side         */
} wdmg_solve_stats;

/* Defaults equal to the paper's constants: omega 0.8, V(2,2), 4 coarse cycles,
 * GCR(50), tol 1e-10. */
void wdmg_default_mg_params(wdmg_mg_params* p);
void wdmg_default_solve_params(wdmg_solve_params* p);

/* Creates a context for a (Lx,Ly,Lz,Lt) lattice.  Extents >= 2.  hip_stream is
 * a hipStream_t (NULL: the null stream).  alloc may be NULL.  On failure *out
 * is NULL. */
int wdmg_create(wdmg_ctx** out, const int dims[4], const wdmg_alloc* alloc, void* hip_stream);

/* Frees every library-owned buffer; synchronises the stream first. */
void wdmg_destroy(wdmg_ctx* ctx);

/* Message of the last failure on ctx ("" if none).  Valid until the next call. */
const char* wdmg_last_error(const wdmg_ctx* ctx);

/* Sec. 1 / Sec. 3: the SU(3) links.  U: device, canonical complex128 gauge
 * layout.  t_bc = -1 (antiperiodic time) or +1 (periodic).  Copied into the
 * internal FP64 and FP32 layouts with the boundary sign folded in; the
 * caller may free U afterwards.  Invalidates a multigrid hierarchy. */
int wdmg_set_gauge(wdmg_ctx* ctx, const void* U, int t_bc);

/* Sec. 1: the mass m in D = Dslash + m.  After a multigrid setup the coarse
 * operators are shifted by (m_new - m_old) I, exact because P^dagger P = I. */
int wdmg_set_mass(wdmg_ctx* ctx, double m);

/* Sec. 1: out = D in for nrhs fine fields.  in, out: device, canonical fine
 * layout, out != in.  prec WDMG_F64 (complex128 I/O) or WDMG_F32, WDMG_F16,
 * WDMG_BF16 (complex64 I/O; the 16-bit paths store `in`, the links and the
 * result in 16 bits as described for WDMG_F16 and compute in FP32). */
int wdmg_apply_D(wdmg_ctx* ctx, void* out, const void* in, int nrhs, int prec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * out = D in as wdmg_apply_D, with the internal-layout input and output
 * fields in a 64 MiB device array that the library holds on every GPU it
 * runs on until the process ends.  prec WDMG_F64 or WDMG_F32 only; at most
 * 2 x 12 x padded sites x nrhs x (16 or 8) bytes <= 64 MiB (a 16^4 lattice
 * takes 2 FP64 or 5 FP32 right-hand sides), else WDMG_ERR_ARG before
 * anything is launched.  Makes no hipMalloc/hipFree or other allocating call:
 * the Wilson form is the one the autotuner already chose for (prec, nrhs) on
 * this context, else the default form, and the call is not timed by
 * wdmg_profile.  All calls on one GPU share its array (which keeps the last
 * call's contents; nothing in it needs to start at zero), so calls that
 * overlap on one GPU, from any context or stream, race. */
int wdmg_apply_D_noalloc(wdmg_ctx* ctx, void* out, const void* in, int nrhs, int prec);

/* Storage conversion of fine fields (the layout and precision conversion in
 * front of every fine-level kernel): out = in after conversion into the
 * internal fine-field storage of precision prec and back.  Canonical layout;
 * complex128 for WDMG_F64, complex64 otherwise; out != in. */
int wdmg_roundtrip(wdmg_ctx* ctx, void* out, const void* in, int nrhs, int prec);

/* Sec. 2 (adaptive setup, block QR with P V_c = V and P^dagger P = I),
 * Sec. 3 (geometric aggregates, chirality kept in the blocks, R = P^dagger),
 * Sec. 2 (Galerkin D_c = P^dagger D P).  For each coarsening the starting
 * vectors are relaxed with setup_iters MR steps on D v = 0 (each vector its
 * own step size), normalised, block-orthonormalised in FP64 per (aggregate,
 * chirality) and the coarse stencil is built.  Synchronises. */
int wdmg_mg_setup(wdmg_ctx* ctx, const wdmg_mg_params* params);

/* Memory for large batches (memory management, not an operation of the
 * paper): after wdmg_mg_setup, frees what a V-cycle in
 * 16-bit storage of mg_prec (WDMG_F16 or WDMG_BF16) does not read, after
 * making the 16-bit copies it does.  Freed are the FP64 and FP32 columns of
 * the first prolongator, and the FP64 and FP32 blocks of every coarse level
 * but the coarsest (whose FP64 GCR keeps them).  Until the next
 * wdmg_mg_setup, calls that would read a freed copy fail with WDMG_ERR_ARG
 * before launching anything: solves with a V-cycle in another precision,
 * wdmg_get_prolongator(0), wdmg_restrict / wdmg_prolong / wdmg_apply_Dc in
 * FP64 or FP32 where they need it, and wdmg_set_mass.  Synchronises.
 * Errors: WDMG_ERR_NOT_SETUP without a hierarchy, WDMG_ERR_ARG for another
 * precision. */
int wdmg_release_unused(wdmg_ctx* ctx, int mg_prec);

/* The orthonormalised columns of P from level l to l+1: device output,
 * canonical complex128 layout of level l, [nv][sites][dof]. */
int wdmg_get_prolongator(wdmg_ctx* ctx, int level, void* V_out);

/* Sec. 2: out = D_c in on coarse level l >= 1 (nrhs fields).  Canonical
 * coarse layout; prec WDMG_F64 (complex128) or WDMG_F32, WDMG_F16, WDMG_BF16
 * (complex64 vectors; the 16-bit kinds use 16-bit blocks with one scale per
 * block). */
int wdmg_apply_Dc(wdmg_ctx* ctx, int level, void* out, const void* in, int nrhs, int prec);

/* Sec. 3 (normal equations): out = (D^dagger D)_c in = P^dagger D^dagger D P in
 * on coarse level 1 of a hierarchy set up with wdmg_mg_params.normal = 1,
 * as the 33-block stencil the setup built.  Canonical coarse layout,
 * complex128; WDMG_ERR_NOT_SETUP without a normal-equation hierarchy. */
int wdmg_apply_Nc(wdmg_ctx* ctx, int level, void* out, const void* in, int nrhs);

/* Sec. 2 / Sec. 3: c_out = P^dagger f_in (restriction from level l to l+1)
 * and f_out = P c_in (prolongation from level l+1 to l).  Canonical layouts
 * of the two levels; precision as for wdmg_apply_D.  The 16-bit kinds
 * (level 0 only) store the fine field and P in 16 bits; the coarse side is
 * complex64. */
int wdmg_restrict(wdmg_ctx* ctx, int level, void* c_out, const void* f_in, int nrhs, int prec);
int wdmg_prolong(wdmg_ctx* ctx, int level, void* f_out, const void* c_in, int nrhs, int prec);

/* Sec. 3: iters under-relaxed MR steps (omega of the setup params, 0.8 if no
 * setup) on A x = b at level l, starting from the given x (updated in place).
 * Canonical layout of level l.  With a 16-bit kind, level 0 keeps x, r and
 * D r in 16-bit storage; coarse levels use the 16-bit coarse blocks. */
int wdmg_smooth(wdmg_ctx* ctx, int level, void* x, const void* b, int nrhs, int iters, int prec);

/* Sec. 5: solve D x = b for nrhs (1..64) right-hand sides with flexible
 * GCR(k), preconditioned by the multigrid V-cycle (params->precond = 1) or
 * not.  The right-hand sides are solved together: each keeps its own Krylov
 * coefficients, step sizes and stopping test (a converged one is frozen),
 * while every operator pass (D, V-cycle, D_c, P, P^dagger) is shared by the
 * batch.  x (device, canonical complex128) holds the initial guesses and
 * receives the solutions; b is not modified.  stats: host array of nrhs
 * entries or NULL; `seconds`, `n_D` and `n_Dc` report the batch's totals
 * divided by nrhs.  Synchronises. */
int wdmg_solve(wdmg_ctx* ctx, void* x, const void* b, int nrhs,
               const wdmg_solve_params* params, wdmg_solve_stats* stats);

/* Sec. 5 comparator: unpreconditioned BiCGStab in FP64 from x = 0 to the same
 * true-residual criterion.  Same layouts as wdmg_solve. */
int wdmg_solve_bicgstab(wdmg_ctx* ctx, void* x, const void* b, int nrhs, double tol,
                        int maxit, wdmg_solve_stats* stats);

/* ---- kernel variants and the autotuner ------------------------------------
 * Some kernels exist in more than one form with the same result (up to the
 * order of floating-point additions).  With value WDMG_TUNE_AUTO (the
 * default) the library times the forms on first use for each precision and
 * batch size (HIP events, a few launches each, on the context's stream) and
 * keeps the fastest for the context's lifetime; a fixed value forces a form.
 *   WDMG_TUNE_DSLASH: 0 one thread per site, 1 one wave per direction with
 *                     the four partial sums added in LDS, 2 form 1 with its
 *                     registers capped so that four waves fit per SIMD,
 *                     3 and 4 form 1 with 2 or 4 right-hand sides per
 *                     thread (each link loaded once for them, the
 *                     direction sums meeting in LDS one rhs at a time);
 *                     forms 3 and 4 apply to batches they divide (a forced
 *                     value runs form 1 on other batch sizes); 5 one wave per
 *                     4x4x4 tile column walking a chunk of time layers, each
 *                     spinor loaded once per chunk, the x, y, z hops exchanged
 *                     between lanes (lattices cut into 4^4 tiles only, else
 *                     form 1; the rhs-group value 4, 8 or 16 sets the chunk);
 *                     6, 7, 8 forms 1, 2, 3 with the workgroups of each XCD
 *                     walking a box of tile columns layer by layer (4^4
 *                     tiles and tile columns that split into 8 boxes only,
 *                     else form 1); 9 form 5 with XCD k taking the k-th
 *                     eighth of the time extent (every tile column of it)
 *                     and the rhs of a group running each column back to
 *                     back (4^4 tiles and Lt a multiple of 8 only, else
 *                     form 1; the rhs-group value sets the group).
 *   WDMG_TUNE_DSLASH_GROUP: right-hand sides per group (1..64) in the
 *                     workgroup order of a batched Wilson launch: each XCD
 *                     sweeps its lattice region once per group, with the
 *                     group's rhs of one site block back to back (a value
 *                     above the batch size means the whole batch).  Tuned
 *                     after the form.
 *   WDMG_TUNE_COARSE_APPLY: the batched coarsest-level operator (nrhs >= 2)
 *                     on the FP64 matrix cores; 0 waves split over
 *                     directions with operands read straight from memory,
 *                     1 operator block and neighbour rows staged through
 *                     LDS one direction at a time, the next one loading
 *                     during the products (needs 2Nv % 8 == 0 and at most
 *                     16 waves for 16 rhs x 16 rows tiles, else form 0).
 *                     AUTO means form 1 where it applies (not timed);
 *                     wdmg_get_tuning reports only a forced value. */
enum {
  WDMG_TUNE_AUTO = -1,
  WDMG_TUNE_DSLASH = 0,
  WDMG_TUNE_DSLASH_GROUP = 1,
  WDMG_TUNE_COARSE_APPLY = 2,
  WDMG_TUNE_COUNT
};
int wdmg_set_tuning(wdmg_ctx* ctx, int key, int value);
/* Sets the choice the autotuner keeps for key (WDMG_TUNE_DSLASH or
 * WDMG_TUNE_DSLASH_GROUP) at precision prec and batch size nrhs (sizes from
 * 64 up share one entry), as if it had timed the forms and picked `value`;
 * WDMG_TUNE_AUTO clears the entry, so the next launch times the forms again.
 * A value forced with wdmg_set_tuning takes precedence.  A form that does not
 * apply to the batch or lattice runs form 1, as with wdmg_set_tuning.
 * WDMG_ERR_ARG for another key, an unknown precision, nrhs < 1 or a value
 * out of range. */
int wdmg_set_tuning_for(wdmg_ctx* ctx, int key, int prec, int nrhs, int value);
/* Current choice for key (WDMG_TUNE_AUTO until tuned) for precision prec
 * and batch size nrhs. */
int wdmg_get_tuning(wdmg_ctx* ctx, int key, int prec, int nrhs, int* value);

/* ---- instrumentation (not part of the method) ----------------------------
 * Kernel timing with HIP events recorded on the context's stream around each
 * launch of the kernels below.  `units` counts the work items the kernel
 * processed: fine sites x rhs (D, P, P^dagger), coarse sites x rhs (D_c
 * apply, on the vector units for one rhs or on the matrix cores (MFMA) for a
 * batch), coarse sites (D_c build) or (aggregate, chirality) blocks (QR);
 * WDMG_K_COARSE_GCR is the operator launch of one coarsest-level GCR
 * iteration (D_c with the Gram-Schmidt partial sums; coarse sites x rhs). */
enum {
  WDMG_K_DSLASH_F64 = 0, WDMG_K_DSLASH_F32, WDMG_K_DC_F64, WDMG_K_DC_F32,
  WDMG_K_RESTRICT_F64, WDMG_K_RESTRICT_F32, WDMG_K_PROLONG_F64, WDMG_K_PROLONG_F32,
  WDMG_K_DC_BUILD, WDMG_K_BLOCK_QR, WDMG_K_DC_MFMA_F64, WDMG_K_DC_MFMA_F32,
  WDMG_K_DSLASH_F16, WDMG_K_DSLASH_BF16, WDMG_K_RESTRICT_H, WDMG_K_PROLONG_H, WDMG_K_DC_H, WDMG_K_DC_MFMA_H,
  WDMG_K_COARSE_GCR, WDMG_K_COUNT
};

/* enable = 1 starts recording (and clears earlier records), 0 stops. */
int wdmg_profile(wdmg_ctx* ctx, int enable);

/* Totals since the last wdmg_profile(ctx, 1) for one kernel id: launches,
 * work units and summed event time in milliseconds.  Synchronises. */
int wdmg_profile_read(wdmg_ctx* ctx, int kernel, long long* launches, long long* units, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* WDMG_H */
