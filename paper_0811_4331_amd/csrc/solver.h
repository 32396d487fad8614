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
void mr(Ctx& c, int l, cx<R>* x, cx<R>* r, cx<R>* p, int nrhs, int iters, double omega);
template <typename R>
void vcycle(Ctx& c, int l, cx<R>* x, const cx<R>* b, int nrhs);
void coarsest_solve(Ctx& c, cx<double>* x, const cx<double>* b, int nrhs);
template <typename R>
void ensure_work(Ctx& c, int l, int nrhs);
void ensure_mg_work(Ctx& c, int nrhs, int prec);

int fgcr(Ctx& c, cx<double>* x, const cx<double>* b, int nrhs, const wdmg_solve_params& p, wdmg_solve_stats* st);
int bicgstab(Ctx& c, cx<double>* x, const cx<double>* b, double tol, int maxit, wdmg_solve_stats& st);

void mg_setup(Ctx& c, const wdmg_mg_params& p);
void free_hierarchy(Ctx& c);
void init_level0(Ctx& c);
void ensure_fine_work(Ctx& c);
void ensure_outer(Ctx& c, int k, int nrhs, bool need32);
void ensure_bicg(Ctx& c);

}  // namespace wdmg
