// Batches of interpolation problems: one forest over every (plan, right-hand
// side) system, solved in lockstep by the projected PCG driver, so each
// FMM stage, preconditioner apply and vector step is one launch over all
// systems still iterating.
#include <chrono>
#include <cstring>

#include "phs_internal.h"

namespace phs {

Batch::~Batch() {
  (void)hipDeviceSynchronize();
  for (auto &w : works) w.release();
}

void batch_create(Batch &b, const std::vector<Plan *> &plans, const std::vector<int> &nrhs,
                  hipStream_t s) {
  PHS_REQUIRE(!plans.empty() && plans.size() == nrhs.size(), PHS_ERR_INVALID_ARGUMENT,
              "batch needs at least one plan and one count per plan");
  const Plan *ev = nullptr;
  for (size_t i = 0; i < plans.size(); ++i) {
    PHS_REQUIRE(plans[i] && nrhs[i] >= 1, PHS_ERR_INVALID_ARGUMENT, "bad plan or rhs count");
    const Plan &p = *plans[i];
    if (p.core_log && !p.direct) {
      if (!ev) ev = &p;
      PHS_REQUIRE(p.p64 == ev->p64 && p.p32 == ev->p32, PHS_ERR_INVALID_ARGUMENT,
                  "even-order plans of a batch must share their expansion orders");
    }
  }
  b.plans = plans;
  b.nrhs = nrhs;
  int nsys = 0;
  for (int r : nrhs) nsys += r;
  b.works.resize(nsys);
  std::vector<Plan *> sp;
  std::vector<SysWork *> sw;
  for (size_t i = 0; i < plans.size(); ++i)
    for (int c = 0; c < nrhs[i]; ++c) {
      const int k = (int)b.sys_plan.size();
      alloc_syswork(b.works[k], *plans[i]);
      b.sys_plan.push_back((int)i);
      b.sys_col.push_back(c);
      sp.push_back(plans[i]);
      sw.push_back(&b.works[k]);
    }
  build_forest(b.F, sp, sw, s);
  PHS_HIP(hipStreamSynchronize(s));
}

phs_status batch_solve(Batch &b, const double *const *f, double *const *w,
                       double *const *beta, const phs_solve_opts *o, phs_solve_info *info,
                       hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const double rtol = (o && o->rtol > 0) ? o->rtol : 1e-8;
  const int maxit = (o && o->maxit > 0) ? o->maxit : 500;
  const int check_every = (o && o->check_every > 0) ? o->check_every : 1;
  const int prec = (o && o->precision >= 0) ? o->precision : b.plans[0]->precision;
  PHS_REQUIRE(prec == PHS_FP64 || prec == PHS_MIXED || prec == PHS_NEAR32,
              PHS_ERR_INVALID_ARGUMENT, "bad precision");
  for (size_t i = 0; i < b.plans.size(); ++i)
    PHS_REQUIRE(f[i] && w[i] && beta[i], PHS_ERR_INVALID_ARGUMENT, "null batch array");
  sync_forest_pc(b.F, s);  // preconditioners may have been (re)built
  std::vector<SolveJob> jobs(b.sys_plan.size());
  for (size_t k = 0; k < jobs.size(); ++k) {
    const int i = b.sys_plan[k], c = b.sys_col[k];
    const Plan &pl = *b.plans[i];
    jobs[k].sys = (int)k;
    jobs[k].f = f[i] + (int64_t)c * pl.n;
    jobs[k].w_out = w[i] + (int64_t)c * pl.n;
    jobs[k].beta_out = beta[i] + (int64_t)c * pl.S;
  }
  solve_forest(b.F, jobs, rtol, maxit, check_every, prec, s);
  const double t =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  phs_status st = PHS_OK;
  if (info)
    for (size_t i = 0; i < b.plans.size(); ++i) {
      std::memset(&info[i], 0, sizeof(info[i]));
      info[i].t_solve = t;
      info[i].t_plan = b.plans[i]->t_plan;
      info[i].t_precond = b.plans[i]->t_precond;
    }
  for (size_t k = 0; k < jobs.size(); ++k) {
    const int i = b.sys_plan[k];
    if (info) {
      info[i].iters += jobs[k].iters;
      info[i].outer_refinements += jobs[k].outer;
      info[i].rel_residual = std::max(info[i].rel_residual, jobs[k].rel);
      info[i].iters_fp32 += jobs[k].iters32;
      info[i].iters_fp64 += jobs[k].iters64;
      info[i].fp64_fallback += jobs[k].fallback ? 1 : 0;
    }
    if (jobs[k].status != PHS_OK && st == PHS_OK) st = jobs[k].status;
  }
  if (st == PHS_ERR_NOT_CONVERGED) set_error(st, "PCG did not reach rtol within maxit");
  if (st == PHS_ERR_BREAKDOWN) set_error(st, "PCG breakdown: non-positive curvature");
  return st;
}

}  // namespace phs
