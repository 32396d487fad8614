// Host drivers of libwdmg (solver.cpp).
#pragma once

#include "internal.h"

namespace wdmg {

double read_scalar(Ctx& c, int slot);
void check_flags(Ctx& c);

template <typename R>
void apply_op(Ctx& c, int l, cx<R>* out, const cx<R>* in, int nrhs);
template <typename R>
void restrict_to(Ctx& c, int l, const cx<R>* fine, cx<R>* crs, int nrhs);
template <typename R>
void prolong_from(Ctx& c, int l, const cx<R>* crs, cx<R>* fine, int nrhs);
template <typename R>
void mr(Ctx& c, int l, cx<R>* x, cx<R>* r, cx<R>* p, int nrhs, int iters, double omega, const cx<R>* b0 = nullptr,
        bool last_x_only = false);
template <typename R>
void vcycle(Ctx& c, int l, cx<R>* x, const cx<R>* b, int nrhs);
void coarsest_solve(Ctx& c, cx<double>* x, const cx<double>* b, int nrhs);
// 16-bit fine level (x, r, p and b are 16-bit fields of nrhs right-hand sides)
void ensure_work_h(Ctx& c, int nrhs);
template <typename H>
void mr_h(Ctx& c, HF x, HF r, HF p, int nrhs, int iters, double omega, const HF* b0 = nullptr,
          bool last_x_only = false);
template <typename H>
void vcycle_h(Ctx& c, HF x, HF b, int nrhs);

// Sets the 16-bit kind of the coarse operators (Ctx::vc_half) for a scope.
struct HalfScope {
  Ctx& c;
  int saved;
  HalfScope(Ctx& ctx, int kind) : c(ctx), saved(ctx.vc_half) { c.vc_half = kind; }
  ~HalfScope() { c.vc_half = saved; }
};
template <typename R>
void ensure_work(Ctx& c, int l, int nrhs);
void ensure_mg_work(Ctx& c, int nrhs, int prec, int first = 0);

// b_canon (with b == nullptr): the right-hand sides in the caller's canonical
// layout, converted into the idle FP32 W basis whenever the residual is
// recomputed (in-place solves keep no internal copy of b).
int fgcr(Ctx& c, cx<double>* x, const cx<double>* b, int nrhs, const wdmg_solve_params& p, wdmg_solve_stats* st,
         const void* b_canon = nullptr);
// BiCGStab from x = 0; with pc (precond set) the V-cycle of pc's precision is
// the right preconditioner.
int bicgstab(Ctx& c, cx<double>* x, const cx<double>* b, double tol, int maxit, wdmg_solve_stats& st,
             const wdmg_solve_params* pc = nullptr);

void mg_setup(Ctx& c, const wdmg_mg_params& p);

// Normal equations (normal.hip): A = D^dagger D on level 0, its Galerkin
// coarse operator on level 1, CGNR and MG-CG for one right-hand side.
void normal_apply0(Ctx& c, cx<double>* out, const cx<double>* in, cx<double>* tmp, int nrhs);
void normal_check_geometry(const Level& f, const Level& cl);
void normal_relax(Ctx& c, Level& f, int nv, int iters, double omega);
void normal_build(Ctx& c, Level& f, Level& cl);
void normal_apply_c(Ctx& c, const Level& cl, cx<double>* out, const cx<double>* in, int nrhs);
int normal_solve(Ctx& c, cx<double>* x, const cx<double>* b, double tol, int maxit, bool precond,
                 wdmg_solve_stats& st);
void free_hierarchy(Ctx& c);
void init_level0(Ctx& c);
void ensure_outer(Ctx& c, int k, int nrhs, bool need32, bool basis32);
void ensure_bicg(Ctx& c);

}  // namespace wdmg
