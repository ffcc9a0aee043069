// Projected PCG over a forest of systems (paper eq. phs_linsys_solve with the
// preconditioner of Sec. 2.2), in lockstep: every GPU step of the method is
// one masked launch over all systems that take that step in the current
// round, so one plan alone and many plans in a batch run the same arithmetic
// per system.
//
// Per system (x0 = 0, b = sign_k Pi f), iterative refinement around PCG:
//   inner PCG on sign_k Pi M Pi with z = Pi U~ U~^T r for the correction dw,
//   stopped when the recursively updated residual ||r|| <= tol; then
//   w += dw and the true residual r = sign_k Pi (f - M64 w) with the FP64
//   matvec.  The solve ends when ||r|| <= rtol ||b||.
//   FP64: the inner operator is the FP64 one and the inner tolerance is
//          rtol ||b||, so usually one inner solve suffices; when the true
//          residual misses the target (FMM error against a rough, strongly
//          preconditioned direction) PCG restarts from it, and stops if a
//          restart no longer halves it.  If the FP64 operator at the matvec
//          order breaks down at once or its restarts stall, the system moves
//          to the FP64 operator at the plan's (higher) evaluation order for
//          the rest of the solve, residual and coefficients included.
//   MIXED / NEAR32: the inner operator is FP32 (far and near field, or near
//          field only).  An inner solve that breaks down at once, or an
//          outer step that does not halve the true residual, switches the
//          rest of the solve to the FP64 operator.
//   Then beta from R beta = Q^T (f - M64 w), and the FP64 relative residual.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "phs_internal.h"

namespace phs {

namespace {

// masks of the solve (slot 0 is all ones and never changed)
enum MaskSlot {
  MK_ALL = 0,
  MK_PCG = 1,
  MK_P64 = 2,
  MK_P32 = 3,
  MK_PN32 = 4,
  MK_CONT = 5,
  MK_START = 6,
  MK_RESID = 7,
  MK_FINISH = 8,
  MK_UPD = 9,
  MK_P64H = 10,  // PCG on the FP64 operator at the evaluation order
  MK_HI = 11     // residual / final matvecs at the evaluation order
};

// A system can move to the FP64 operator at the plan's evaluation order when
// that order is higher than the matvec order.
bool can_escalate(const Plan &pl) {
  if (pl.direct) return false;
  return pl.core_log ? pl.pe > pl.p64 : pl.qe > pl.q64;
}

using JobRun = SolveJob;

void set_mask(Forest &F, int slot, const std::vector<SolveJob *> &jr, bool (*pred)(const JobRun &),
              bool &any, hipStream_t s) {
  std::vector<int32_t> m(F.nsys, 0);
  any = false;
  for (const auto *r : jr)
    if (pred(*r)) {
      m[r->sys] = 1;
      any = true;
    }
  set_mask(F, slot, m, s);
}

void start_pcg(JobRun &r, const SolveParams &P) {
  const bool mixed = P.prec != PHS_FP64;
  const int p64 = r.hi ? PHS_FP64_EVAL : PHS_FP64;
  if (!mixed) {
    r.inner_prec = p64;
    r.inner_tol = r.tol_abs;
    r.maxit_inner = r.budget;
  } else {
    // FP32 far field: small steps (its error is relative to ||M||); FP32
    // near field only: the operator is accurate enough to go to rtol at once
    r.inner_prec = r.fp64_finish ? p64 : P.prec;
    r.inner_tol = r.fp64_finish ? r.tol_abs
                                : (P.prec == PHS_NEAR32 ? 0.5 * r.tol_abs
                                                        : std::max(r.tol_abs, 1e-4 * r.rn));
    // an FP32 inner solve gets at most 60 iterations: if it stalls, the outer
    // step sees no progress and the rest runs on the FP64 operator
    r.maxit_inner = r.fp64_finish ? r.budget : std::min(r.budget, 60);
  }
  r.it = 0;
  r.pcg_conv = r.pcg_break = false;
  r.have_q = false;
  r.state = J_START;
}

}  // namespace

void solve_begin(Forest &F, std::vector<SolveJob *> &jr, const SolveParams &P, hipStream_t s) {
  PHS_REQUIRE(F.nsys >= 1 && Forest::kMasks >= 12, PHS_ERR_INVALID_ARGUMENT, "empty forest");
  bool any = false;
  // ---- INIT: f in tree order, b = sign Pi f, ||b||, ||f||
  for (auto *r : jr) f_gather_user(F, r->sys, r->f, V_F, s);
  set_mask(F, MK_START, jr, [](const JobRun &r) { return r.state == J_INIT; }, any, s);
  f_scale_sign(F, F.mask[MK_START], V_R, V_F, s);
  f_project(F, F.mask[MK_START], V_R, s);
  f_dot(F, F.mask[MK_START], V_R, V_R, SC_DOT, s);
  f_dot(F, F.mask[MK_START], V_F, V_F, SC_DOT + 1, s);
  f_fill(F, F.mask[MK_START], V_W, 0.0, s);
  f_read_scalars(F, SC_DOT, 2, s);
  for (auto *rp : jr) {
    JobRun &r = *rp;
    const int sy = r.sys;
    r.bn = std::sqrt(F.hgsc[sy * 8 + 0]);
    r.fn = std::sqrt(F.hgsc[sy * 8 + 1]);
    r.tol_abs = P.rtol * r.bn;
    r.rn = r.bn;
    r.budget = P.maxit;
    r.fp64_finish = P.prec == PHS_FP64;
    if (r.bn <= 1e-13 * r.fn) {
      // data in span(B) to rounding level: the polynomial alone interpolates
      r.state = J_FINISH;
    } else {
      start_pcg(r, P);
    }
  }
}

bool solve_round(Forest &F, std::vector<SolveJob *> &jr, const SolveParams &P, hipStream_t s) {
  const bool mixed = P.prec != PHS_FP64;
  const int check_every = P.check_every;
  bool any = false;
  {
    bool live = false;
    for (auto *r : jr) live = live || r->state != J_DONE;
    if (!live) return false;

    // ---- START: dw = 0, z = precond(r), rho = r.z, p = z
    set_mask(F, MK_START, jr, [](const JobRun &r) { return r.state == J_START; }, any, s);
    if (any) {
      f_fill(F, F.mask[MK_START], V_DW, 0.0, s);
      f_precond_dot(F, F.mask[MK_START], V_R, V_Z, V_TMP, SC_RHO, s);
      f_copy(F, F.mask[MK_START], V_P, V_Z, s);
      for (auto *rp_ : jr) if (auto &r = *rp_; true)
        if (r.state == J_START) r.state = J_PCG;
    }

    // ---- PCG iteration
    set_mask(F, MK_PCG, jr, [](const JobRun &r) { return r.state == J_PCG; }, any, s);
    if (any) {
      bool a64 = false, a64h = false, a32 = false, an32 = false;
      set_mask(F, MK_P64, jr,
               [](const JobRun &r) { return r.state == J_PCG && r.inner_prec == PHS_FP64; }, a64,
               s);
      set_mask(F, MK_P64H, jr,
               [](const JobRun &r) { return r.state == J_PCG && r.inner_prec == PHS_FP64_EVAL; },
               a64h, s);
      set_mask(F, MK_P32, jr,
               [](const JobRun &r) { return r.state == J_PCG && r.inner_prec == PHS_MIXED; },
               a32, s);
      set_mask(F, MK_PN32, jr,
               [](const JobRun &r) { return r.state == J_PCG && r.inner_prec == PHS_NEAR32; },
               an32, s);
      // FP64 iterations checked every time run from graphs: (q = sign Pi M p,
      // p.q, the w / r update, r.r, their gather) and (z = precond(r), r.z,
      // the new p).  The kernels read the masks uploaded above.
      const bool graphs = check_every == 1 && !a32 && !an32;
      if (graphs) {
        f_run(F, (a64 ? 1 : 0) | (a64h ? 2 : 0), s, [&](hipStream_t cs) {
          if (a64) f_matvec(F, F.mask[MK_P64], V_P, V_Q, PHS_FP64, cs);
          if (a64h) f_matvec(F, F.mask[MK_P64H], V_P, V_Q, PHS_FP64_EVAL, cs);
          f_project_dot(F, F.mask[MK_PCG], V_Q, true, V_P, SC_PQ, cs);
          f_pcg_wr(F, F.mask[MK_PCG], cs);
          f_read_scalars_launch(F, 0, 4, cs);
        });
        PHS_HIP(hipStreamSynchronize(s));
      }
      // q = sign Pi M p
      if (!graphs) {
        if (a64) f_matvec(F, F.mask[MK_P64], V_P, V_Q, PHS_FP64, s);
        if (a64h) f_matvec(F, F.mask[MK_P64H], V_P, V_Q, PHS_FP64_EVAL, s);
        if (a32) f_matvec(F, F.mask[MK_P32], V_P, V_Q, PHS_MIXED, s);
        if (an32) f_matvec(F, F.mask[MK_PN32], V_P, V_Q, PHS_NEAR32, s);
        f_project_dot(F, F.mask[MK_PCG], V_Q, true, V_P, SC_PQ, s);
      }
      const int32_t *upd_mask = F.mask[MK_PCG];
      if (check_every == 1 && (a32 || an32)) {
        // curvature check before the update so a breakdown step of an inexact
        // (FP32) operator is never applied
        f_read_scalars(F, SC_PQ, 1, s);
        bool drop = false;
        for (auto *rp_ : jr) if (auto &r = *rp_; true)
          if (r.state == J_PCG && (r.inner_prec == PHS_MIXED || r.inner_prec == PHS_NEAR32) &&
              !(F.hgsc[r.sys * 8] > 0.0)) {
            r.pcg_break = true;
            r.state = J_PCG_END;
            drop = true;
          }
        if (drop) {
          set_mask(F, MK_UPD, jr, [](const JobRun &r) { return r.state == J_PCG; }, any, s);
          upd_mask = F.mask[MK_UPD];
        }
      }
      if (!graphs) f_pcg_wr(F, upd_mask, s);
      bool need_check = false;
      for (auto *rp_ : jr) if (auto &r = *rp_; true)
        if (r.state == J_PCG) {
          ++r.it;
          if (r.it % check_every == 0 || r.it == r.maxit_inner) need_check = true;
        }
      if (need_check && !graphs) f_read_scalars(F, 0, 4, s);
      for (auto *rp_ : jr) if (auto &r = *rp_; true) {
        if (r.state != J_PCG) continue;
        if (!(r.it % check_every == 0 || r.it == r.maxit_inner)) continue;
        const double *g = F.hgsc + r.sys * 8;
        if (!(g[SC_PQ] > 0.0)) {
          r.pcg_break = true;
          r.state = J_PCG_END;
        } else if (std::sqrt(g[SC_RR]) <= r.inner_tol) {
          r.pcg_conv = true;
          r.state = J_PCG_END;
        } else if (r.it >= r.maxit_inner) {
          r.state = J_PCG_END;
        }
      }
      // z = precond(r), rho_new = r.z, p = z + (rho_new / rho) p, rho = rho_new
      set_mask(F, MK_CONT, jr, [](const JobRun &r) { return r.state == J_PCG; }, any, s);
      if (any) {
        auto next_p = [&](hipStream_t cs) {
          f_precond_dot(F, F.mask[MK_CONT], V_R, V_Z, V_TMP, SC_RHO_NEW, cs);
          f_pcg_p(F, F.mask[MK_CONT], cs);
          f_sc_copy(F, F.mask[MK_CONT], SC_RHO, SC_RHO_NEW, cs);
        };
        if (graphs) f_run(F, 4, s, next_p);
        else next_p(s);
      }
    }

    // ---- end of an inner solve
    for (auto *rp_ : jr) if (auto &r = *rp_; true) {
      if (r.state != J_PCG_END) continue;
      r.iters += r.it;
      r.budget -= r.it;
      if (r.inner_prec == PHS_FP64 || r.inner_prec == PHS_FP64_EVAL) r.iters64 += r.it;
      else r.iters32 += r.it;
      if (r.pcg_break && r.it <= 1) {
        if (r.fp64_finish) {
          if (!r.hi && can_escalate(*F.plan[r.sys])) {
            // the FP64 operator at the matvec order is not definite enough
            // on this direction: continue at the evaluation order, from the
            // residual recomputed there
            r.hi = true;
            r.count_outer = false;
            r.state = J_RESID;
            continue;
          }
          r.status = PHS_ERR_BREAKDOWN;
          r.state = J_FINISH;
          continue;
        }
        r.fp64_finish = true;  // no usable FP32 step: restart this residual in FP64
        r.fallback = true;
        r.count_outer = false;
        r.state = J_RESID;
        continue;
      }
      r.count_outer = true;
      r.apply_dw = true;
      r.state = J_RESID;
    }
    // w += dw
    set_mask(F, MK_UPD, jr, [](const JobRun &r) { return r.apply_dw; }, any, s);
    if (any) f_axpby(F, F.mask[MK_UPD], V_W, V_DW, 1.0, 1.0, s);
    for (auto *rp_ : jr) if (auto &r = *rp_; true) r.apply_dw = false;

    // ---- FP64 residual of the refinement: r = sign Pi (f - M64 w)
    bool any_hi = false;
    set_mask(F, MK_HI, jr, [](const JobRun &r) { return r.state == J_RESID && r.hi; }, any_hi,
             s);
    set_mask(F, MK_UPD, jr, [](const JobRun &r) { return r.state == J_RESID && !r.hi; }, any,
             s);
    if (any) f_matvec(F, F.mask[MK_UPD], V_W, V_Q, PHS_FP64, s);
    if (any_hi) f_matvec(F, F.mask[MK_HI], V_W, V_Q, PHS_FP64_EVAL, s);
    set_mask(F, MK_RESID, jr, [](const JobRun &r) { return r.state == J_RESID; }, any, s);
    if (any) {
      f_axpby(F, F.mask[MK_RESID], V_Q, V_F, 1.0, -1.0, s);  // q = f - M w
      f_scale_sign(F, F.mask[MK_RESID], V_R, V_Q, s);
      f_project(F, F.mask[MK_RESID], V_R, s);
      f_dot(F, F.mask[MK_RESID], V_R, V_R, SC_DOT, s);
      f_read_scalars(F, SC_DOT, 1, s);
      for (auto *rp_ : jr) if (auto &r = *rp_; true) {
        if (r.state != J_RESID) continue;
        const double rn_new = std::sqrt(F.hgsc[r.sys * 8]);
        if (!std::isfinite(rn_new)) {
          r.status = PHS_ERR_BREAKDOWN;
          r.state = J_FINISH;
          r.have_q = true;
          continue;
        }
        bool stalled = false, worse = false;
        if (!r.count_outer) {
          // a residual recomputed without a correction (after a switch of
          // operator): it is the reference the next restart must halve
          r.rn = rn_new;
        } else {
          // refinement steps; in FP64 only the restarts count
          if (mixed || rn_new > r.tol_abs) ++r.outer;
          stalled = !(rn_new < 0.5 * r.rn);
          if (stalled && !r.fp64_finish) {
            r.fp64_finish = true;  // the FP32 operator stopped helping
            r.fallback = true;
            stalled = false;
          }
          // a final correction that raised the residual is taken back, so
          // the solve returns the best iterate of its restarts
          worse = stalled && rn_new > r.rn;
          if (!worse) r.rn = rn_new;
          if (stalled && r.fp64_finish && !r.hi && can_escalate(*F.plan[r.sys])) {
            // restarts at the matvec order stopped helping: take back a
            // correction that raised the residual, then go on at the
            // evaluation order from the residual recomputed there
            r.hi = true;
            r.undo_dw = worse;
            r.count_outer = false;
            continue;  // stays in J_RESID
          }
        }
        if (r.rn > r.tol_abs && r.budget > 0 && !stalled) {
          start_pcg(r, P);
        } else {
          if (r.rn > r.tol_abs && r.status == PHS_OK) r.status = PHS_ERR_NOT_CONVERGED;
          r.state = J_FINISH;
          r.have_q = !worse;  // q = f - M w of the final w
          r.undo_dw = worse;
        }
      }
    }
    // w -= dw where the last correction was taken back
    set_mask(F, MK_UPD, jr, [](const JobRun &r) { return r.undo_dw; }, any, s);
    if (any) f_axpby(F, F.mask[MK_UPD], V_W, V_DW, -1.0, 1.0, s);  // w = w - dw
    for (auto *rp_ : jr) if (auto &r = *rp_; true) r.undo_dw = false;

    // ---- beta from R beta = Q^T (f - M w), the FP64 residual, w to the caller
    set_mask(F, MK_UPD, jr,
             [](const JobRun &r) { return r.state == J_FINISH && !r.have_q && !r.hi; }, any, s);
    if (any) f_matvec(F, F.mask[MK_UPD], V_W, V_Q, PHS_FP64, s);
    set_mask(F, MK_HI, jr,
             [](const JobRun &r) { return r.state == J_FINISH && !r.have_q && r.hi; }, any_hi,
             s);
    if (any_hi) f_matvec(F, F.mask[MK_HI], V_W, V_Q, PHS_FP64_EVAL, s);
    set_mask(F, MK_UPD, jr, [](const JobRun &r) { return r.state == J_FINISH && !r.have_q; },
             any, s);
    if (any) f_axpby(F, F.mask[MK_UPD], V_Q, V_F, 1.0, -1.0, s);  // q = f - M w
    set_mask(F, MK_FINISH, jr, [](const JobRun &r) { return r.state == J_FINISH; }, any, s);
    if (any) {
      f_qt(F, F.mask[MK_FINISH], V_Q, SC_QTF, s);
      f_project(F, F.mask[MK_FINISH], V_Q, s);
      f_dot(F, F.mask[MK_FINISH], V_Q, V_Q, SC_DOT, s);
      // Q^T q (S <= 28 values) and ||Pi q||^2 per system
      std::vector<std::vector<double>> qtf(jr.size());
      for (int off = 0; off < F.maxS; off += 8) {
        const int cnt = std::min(8, F.maxS - off);
        f_read_scalars(F, SC_QTF + off, cnt, s);
        for (size_t i = 0; i < jr.size(); ++i) {
          if (jr[i]->state != J_FINISH) continue;
          for (int c = 0; c < cnt; ++c)
            qtf[i].push_back(F.hgsc[jr[i]->sys * 8 + c]);
        }
      }
      f_read_scalars(F, SC_DOT, 1, s);
      for (size_t i = 0; i < jr.size(); ++i) {
        JobRun &r = *jr[i];
        if (r.state != J_FINISH) continue;
        const Plan &pl = *F.plan[r.sys];
        const int S = pl.S;
        std::vector<double> bet(S);
        for (int a = S - 1; a >= 0; --a) {
          double acc = qtf[i][a];
          for (int k2 = a + 1; k2 < S; ++k2) acc -= pl.Rm[(size_t)a * S + k2] * bet[k2];
          bet[a] = acc / pl.Rm[(size_t)a * S + a];
        }
        r.beta_host = bet;
        r.rel = r.bn > 0 ? std::sqrt(F.hgsc[r.sys * 8]) / r.bn : 0.0;
        PHS_HIP(hipMemcpyAsync(r.beta_out, r.beta_host.data(), S * sizeof(double),
                               hipMemcpyHostToDevice, s));
        f_scatter_user(F, r.sys, V_W, r.w_out, s);
        r.state = J_DONE;
      }
      PHS_HIP(hipStreamSynchronize(s));
    }
  }
  return true;
}

void solve_forest(Forest &F, std::vector<SolveJob> &jobs, double rtol, int maxit,
                  int check_every, int prec, hipStream_t s) {
  const SolveParams P{rtol, maxit, check_every, prec};
  std::vector<SolveJob *> jr;
  for (auto &j : jobs) jr.push_back(&j);
  solve_begin(F, jr, P, s);
  while (solve_round(F, jr, P, s)) {
  }
}

}  // namespace phs
