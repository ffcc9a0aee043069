// C ABI of the PHS library: plan construction (normalisation, quadtree,
// polynomial block and thin QR), the kernel matvec, projected PCG with
// residual refinement, coefficient recovery and evaluation (paper Sec. 2,
// eq. phs_linsys_solve; Sec. 2.2 preconditioning).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <atomic>
#include <mutex>

#include "phs_internal.h"

namespace phs {

void fill_log_table(double *tab);
void fill_near_log_table(double *tab);

void log_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                      const double *targets, int64_t m, double *out, hipStream_t s);
void dist_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                       const double *targets, int64_t m, double *out, hipStream_t s);

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

void set_error(phs_status code, const std::string &msg) {
  (void)code;
  g_last_error = msg;
}

// ------------------------------------------------------------------ profiling
namespace {
struct ProfRec {
  int64_t launches = 0;
  double ms = 0.0;
};
struct Pending {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
int g_prof_level = 0;
std::map<std::string, ProfRec> g_prof;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;  // recycled events
thread_local std::vector<std::pair<std::string, hipEvent_t>> g_open;

hipEvent_t pool_get() {
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_pool.empty()) {
      hipEvent_t e = g_pool.back();
      g_pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_flush_locked() {
  for (auto &p : g_pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p.a, p.b);
    auto &r = g_prof[p.name];
    r.launches += 1;
    r.ms += ms;
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pending.clear();
}
}  // namespace

bool profiling_on() { return g_prof_on; }

namespace {
std::atomic<bool> g_graphs{false};
}
bool graphs_enabled() { return g_graphs.load(std::memory_order_relaxed); }

// level 2 times only the kernels the roofline figures use
bool prof_wants(const char *name) {
  if (g_prof_level != 2) return true;
  static const char *keep[] = {"leaf_eval",  "leaf_eval_near32", "leaf_eval_f32", "m2l",
                               "m2l_f32",    "vecchia_factor",   "vecchia_knn",   "precond_u",
                               "precond_ut", "direct",           "direct_f32"};
  for (const char *k : keep)
    if (std::strcmp(k, name) == 0) return true;
  return false;
}

void prof_begin(const char *name, hipStream_t s) {
  hipEvent_t a = pool_get();
  if (!a) return;
  (void)hipEventRecord(a, s);
  g_open.push_back({name, a});
}

void prof_end(hipStream_t s) {
  if (g_open.empty()) return;
  auto op = g_open.back();
  g_open.pop_back();
  hipEvent_t b = pool_get();
  if (!b) return;
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_pending.push_back({op.first, op.second, b});
  if (g_pending.size() > 4096) prof_flush_locked();
}

// ------------------------------------------------------------------ plan
Plan::~Plan() {
  delete self;
  self = nullptr;
  sw.release();
  dfree(order);
  dfree(inv_order);
  dfree(leafkey);
  dfree(x);
  dfree(y);
  dfree(ux);
  dfree(uy);
  dfree(xy2);
  dfree(logtab);
  dfree(neartab);
  dfree(Q);
  dfree(tree.leaf_start);
  free_log_tables(lt64);
  free_log_tables(lt32);
  free_cheb_tables(ct64);
  free_cheb_tables(ct32);
  free_log_tables(lte);
  free_cheb_tables(cte);
  dfree(red);
  dfree(scal);
  if (hscal) (void)hipHostFree(hscal);
  dfree(iscratch);
  vecchia_free(*this);
}

namespace {

inline hipStream_t S(void *s) { return (hipStream_t)s; }

// Host Cholesky of an S x S symmetric matrix (row-major, upper triangle
// valid); returns upper R with R^T R = G.  Returns false on a non-positive or
// negligible pivot.
bool host_chol_upper(const std::vector<double> &G, int n, std::vector<double> &Rm) {
  Rm.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = G[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= Rm[(size_t)k * n + j] * Rm[(size_t)k * n + j];
    if (!(s > 1e-24 * G[(size_t)j * n + j])) return false;
    const double rjj = std::sqrt(s);
    Rm[(size_t)j * n + j] = rjj;
    for (int i = j + 1; i < n; ++i) {
      double t = G[(size_t)j * n + i];
      for (int k = 0; k < j; ++k) t -= Rm[(size_t)k * n + j] * Rm[(size_t)k * n + i];
      Rm[(size_t)j * n + i] = t / rjj;
    }
  }
  return true;
}

std::vector<double> upper_inverse(const std::vector<double> &Rm, int n) {
  std::vector<double> X((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    X[(size_t)j * n + j] = 1.0 / Rm[(size_t)j * n + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += Rm[(size_t)i * n + k] * X[(size_t)k * n + j];
      X[(size_t)i * n + j] = -s / Rm[(size_t)i * n + i];
    }
  }
  return X;
}

std::vector<double> upper_mul(const std::vector<double> &A, const std::vector<double> &B,
                              int n) {
  std::vector<double> C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double s = 0.0;
      for (int k = i; k <= j; ++k) s += A[(size_t)i * n + k] * B[(size_t)k * n + j];
      C[(size_t)i * n + j] = s;
    }
  return C;
}

std::vector<double> gram_host(Plan &pl, hipStream_t s) {
  const int Sn = pl.S;
  const int npairs = Sn * (Sn + 1) / 2;
  gram(pl.Q, pl.n, Sn, pl.red, pl.scal, s);
  PHS_HIP(hipMemcpyAsync(pl.hscal, pl.scal, npairs * sizeof(double), hipMemcpyDeviceToHost, s));
  PHS_HIP(hipStreamSynchronize(s));
  std::vector<double> G((size_t)Sn * Sn, 0.0);
  int t = 0;
  for (int a = 0; a < Sn; ++a)
    for (int b = a; b < Sn; ++b) {
      G[(size_t)a * Sn + b] = pl.hscal[t];
      G[(size_t)b * Sn + a] = pl.hscal[t];
      ++t;
    }
  return G;
}

// CholeskyQR2 of the polynomial block B (n x S, held in pl.Q): Q = B R^{-1}.
void thin_qr(Plan &pl, hipStream_t s) {
  const int Sn = pl.S;
  double *Rinv_dev = pl.scal + 512;
  std::vector<double> R1, R2;
  std::vector<double> G = gram_host(pl, s);
  if (!host_chol_upper(G, Sn, R1))
    throw Error{PHS_ERR_UNISOLVENT, "polynomial block is rank deficient on these nodes"};
  std::vector<double> X = upper_inverse(R1, Sn);
  PHS_HIP(hipMemcpyAsync(Rinv_dev, X.data(), X.size() * 8, hipMemcpyHostToDevice, s));
  apply_rinv(pl.Q, pl.n, Sn, Rinv_dev, s);
  G = gram_host(pl, s);
  if (!host_chol_upper(G, Sn, R2))
    throw Error{PHS_ERR_UNISOLVENT, "polynomial block is numerically rank deficient"};
  X = upper_inverse(R2, Sn);
  PHS_HIP(hipMemcpyAsync(Rinv_dev, X.data(), X.size() * 8, hipMemcpyHostToDevice, s));
  apply_rinv(pl.Q, pl.n, Sn, Rinv_dev, s);
  PHS_HIP(hipStreamSynchronize(s));
  pl.Rm = upper_mul(R2, R1, Sn);
}

int order_for_tol(double tol, bool fp64) {
  // Terms of the scaled log expansions.  Measured FP64 matvec relative errors
  // on 2^20 uniform nodes: P=15 1e-9, P=23 8e-13, P=27 2e-14, P=31 1.5e-15.
  // The default tolerance 1e-12 takes P=27: the weights of the ill-conditioned
  // saddle system amplify the matvec error by ~1e5.
  if (!fp64) return 15;
  if (tol >= 1e-8) return 15;
  if (tol >= 1e-11) return 23;
  if (tol >= 1e-13) return 27;
  return 31;
}

void build_tree(Plan &pl, const double *xy, int leaf_size, hipStream_t s) {
  const int64_t n = pl.n;
  uint32_t *keys = dmalloc<uint32_t>(n), *ktmp = dmalloc<uint32_t>(n);
  int32_t *vals = dmalloc<int32_t>(n), *vtmp = dmalloc<int32_t>(n);
  int32_t *scr = dmalloc<int32_t>(radix_sort_scratch_ints(n));
  try {
    int L = (int)std::lround(std::log((double)n / leaf_size) / std::log(4.0));
    L = std::max(2, std::min(10, L));
    pl.tree.h = pl.hnorm;
    std::vector<int32_t> hstart;
    for (;;) {
      const int G = 1 << L;
      const int nleaf = G * G;
      leaf_keys(xy, n, pl.c[0], pl.c[1], pl.rho, pl.tree.h, L, keys, vals, s);
      radix_sort_u32(keys, vals, n, 2 * L, ktmp, vtmp, scr, s);
      dfree(pl.tree.leaf_start);
      pl.tree.leaf_start = nullptr;
      pl.tree.leaf_start = dmalloc<int32_t>(nleaf + 1);
      leaf_ranges(keys, n, nleaf, pl.tree.leaf_start, s);
      hstart.resize(nleaf + 1);
      PHS_HIP(hipMemcpyAsync(hstart.data(), pl.tree.leaf_start, (nleaf + 1) * 4,
                             hipMemcpyDeviceToHost, s));
      PHS_HIP(hipStreamSynchronize(s));
      int maxocc = 0;
      for (int c = 0; c < nleaf; ++c) maxocc = std::max(maxocc, hstart[c + 1] - hstart[c]);
      if (maxocc > 16 * leaf_size && L < 10) {
        ++L;
        continue;
      }
      pl.tree.L = L;
      pl.tree.G = G;
      break;
    }
    pl.order = vals;
    vals = nullptr;
    pl.inv_order = dmalloc<int32_t>(n);
    pl.leafkey = dmalloc<int32_t>(n);
    pl.x = dmalloc<double>(n);
    pl.y = dmalloc<double>(n);
    pl.ux = dmalloc<float>(n);
    pl.uy = dmalloc<float>(n);
    pl.xy2 = dmalloc<double2>(n);
    build_tree_points(xy, pl.order, keys, n, pl.c[0], pl.c[1], pl.rho, pl.tree.h, pl.tree.L,
                      pl.x, pl.y, pl.ux, pl.uy, pl.xy2, pl.leafkey, pl.inv_order, s);
    int32_t *flag = scr;
    PHS_HIP(hipMemsetAsync(flag, 0, 4, s));
    count_duplicates(pl.x, pl.y, pl.tree.leaf_start, pl.tree.G * pl.tree.G, flag, s);
    int32_t hflag = 0;
    PHS_HIP(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
    PHS_HIP(hipStreamSynchronize(s));
    dfree(keys);
    dfree(ktmp);
    dfree(vtmp);
    dfree(scr);
    keys = ktmp = nullptr;
    vtmp = scr = nullptr;
    if (hflag) throw Error{PHS_ERR_DUPLICATE_POINTS, "two nodes coincide"};
  } catch (...) {
    dfree(keys);
    dfree(ktmp);
    dfree(vals);
    dfree(vtmp);
    dfree(scr);
    throw;
  }
}

void plan_create(const double *xy, int64_t n, const phs_plan_opts *o, hipStream_t s,
                 Plan &pl) {
  const auto t0 = std::chrono::steady_clock::now();
  PHS_REQUIRE(xy && o, PHS_ERR_INVALID_ARGUMENT, "null argument");
  PHS_REQUIRE(o->k >= 1 && o->k <= 4, PHS_ERR_INVALID_ARGUMENT, "k must be 1..4");
  pl.k = o->k;
  pl.d = o->poly_degree < 0 ? min_degree(o->k) : o->poly_degree;
  PHS_REQUIRE(pl.d >= min_degree(o->k), PHS_ERR_INVALID_ARGUMENT,
              "polynomial degree below the minimum for this k");
  PHS_REQUIRE(pl.d <= 5, PHS_ERR_INVALID_ARGUMENT, "polynomial degree above 5");
  pl.S = n_monomials(pl.d);
  PHS_REQUIRE(n >= pl.S && n < (int64_t(1) << 30), PHS_ERR_INVALID_ARGUMENT,
              "n must be >= number of polynomial terms and < 2^30");
  PHS_REQUIRE(o->precision == PHS_FP64 || o->precision == PHS_MIXED ||
                  o->precision == PHS_NEAR32,
              PHS_ERR_INVALID_ARGUMENT, "bad precision");
  pl.n = n;
  pl.R = hadamard_rank(pl.k);
  pl.core_log = (pl.k % 2 == 0);
  pl.sign = definiteness_sign(pl.k);
  pl.precision = o->precision;
  pl.hnorm = domain_half_width(pl.k);
  pl.tree.h = pl.hnorm;
  PHS_REQUIRE(o->matvec == PHS_MATVEC_FMM || o->matvec == PHS_MATVEC_DIRECT,
              PHS_ERR_INVALID_ARGUMENT, "matvec must be PHS_MATVEC_FMM or PHS_MATVEC_DIRECT");
  pl.direct = o->matvec == PHS_MATVEC_DIRECT;
  const double tol = o->fmm_tol > 0 ? o->fmm_tol : 1e-12;
  if (pl.core_log) {
    pl.p64 = o->expansion_order > 0 ? o->expansion_order : order_for_tol(tol, true);
    pl.p32 = order_for_tol(tol, false);
    PHS_REQUIRE(pl.p64 >= 4 && pl.p64 <= 63, PHS_ERR_INVALID_ARGUMENT,
                "expansion order must be 4..63");
    pl.pe = std::max(pl.p64, 31);
  } else {
    // Chebyshev nodes per axis: 12 -> ~2e-12, 16 -> ~1e-14 core relative error.
    // The default is 16 at every size: the odd-order saddle systems are
    // ill-conditioned enough (kappa ~1e4 for k = 1, ~1e7 for k = 3 at a few
    // thousand clustered nodes) that a 2e-12 matvec error moves the weights
    // by 1e-8..1e-5, and from 2^17 nodes on the Vecchia factor of the
    // odd-order Matern covariance (entries ~1e17 at 1e6 nodes) turns it into
    // a loss of definiteness in PCG.  A looser fmm_tol (>= 1e-10) takes 12.
    pl.q64 = o->expansion_order > 0 ? o->expansion_order : (tol >= 1e-10 ? 12 : 16);
    pl.q32 = 8;
    PHS_REQUIRE(pl.q64 == 8 || pl.q64 == 10 || pl.q64 == 12 || pl.q64 == 14 || pl.q64 == 16,
                PHS_ERR_INVALID_ARGUMENT, "Chebyshev order must be 8, 10, 12, 14 or 16");
    pl.qe = 16;
  }
  // scratch used by the bounding box, reductions and scalars
  pl.red_cap = dot_blocks(n) * 32 + 4096;
  pl.red = dmalloc<double>(pl.red_cap);
  pl.scal = dmalloc<double>(1024);
  PHS_HIP(hipHostMalloc((void **)&pl.hscal, 1024 * sizeof(double), 0));

  // bounding box -> c, rho (exact operation order shared with the oracle)
  {
    const int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    minmax_xy(xy, n, pl.scal, pl.red, nb, s);
    PHS_HIP(hipMemcpyAsync(pl.hscal, pl.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    PHS_HIP(hipStreamSynchronize(s));
    const double mnx = pl.hscal[0], mny = pl.hscal[1], mxx = pl.hscal[2], mxy = pl.hscal[3];
    PHS_REQUIRE(std::isfinite(mnx) && std::isfinite(mny) && std::isfinite(mxx) &&
                    std::isfinite(mxy),
                PHS_ERR_INVALID_ARGUMENT, "non-finite coordinates");
    pl.c[0] = (mnx + mxx) * 0.5;
    pl.c[1] = (mny + mxy) * 0.5;
    const double ex = mxx - mnx, ey = mxy - mny;
    const double half = std::max(ex, ey) * 0.5;
    PHS_REQUIRE(half > 0.0, PHS_ERR_INVALID_ARGUMENT, "nodes have zero extent");
    pl.rho = pl.tree.h / half;  // the normalised nodes fill [-h_k, h_k]^2
  }
  int leaf_size = o->leaf_size > 0 ? o->leaf_size : (pl.core_log ? 40 : 64);
  build_tree(pl, xy, leaf_size, s);

  // polynomial block and thin QR
  pl.Q = dmalloc<double>((size_t)n * pl.S);
  poly_block_tree(pl.x, pl.y, n, pl.d, pl.Q, s);
  thin_qr(pl, s);

  // FMM tables and workspace (none for a plan that sums directly)
  size_t eb = 0;
  if (pl.direct) {
  } else if (pl.core_log) {
    build_log_tables(pl.lt64, pl.p64);
    build_log_tables(pl.lt32, pl.p32);
    if (pl.pe != pl.p64) build_log_tables(pl.lte, pl.pe);
    eb = std::max({log_expansion_bytes(pl.tree.L, pl.p64, pl.R, true),
                   log_expansion_bytes(pl.tree.L, pl.pe, pl.R, true),
                   log_expansion_bytes(pl.tree.L, pl.p32, pl.R, false)});
  } else {
    build_cheb_tables(pl.ct64, pl.q64);
    build_cheb_tables(pl.ct32, pl.q32);
    if (pl.qe != pl.q64) build_cheb_tables(pl.cte, pl.qe);
    eb = std::max({cheb_expansion_bytes(pl.tree.L, pl.q64, pl.R, true),
                   cheb_expansion_bytes(pl.tree.L, pl.qe, pl.R, true),
                   cheb_expansion_bytes(pl.tree.L, pl.q32, pl.R, false)});
  }
  pl.exp_bytes = eb;
  {
    std::vector<double> tab(256);
    fill_log_table(tab.data());
    pl.logtab = dmalloc<double>(256);
    PHS_HIP(hipMemcpy(pl.logtab, tab.data(), 256 * sizeof(double), hipMemcpyHostToDevice));
    std::vector<double> nt(kNearLogTab);
    fill_near_log_table(nt.data());
    pl.neartab = dmalloc<double>(kNearLogTab);
    PHS_HIP(hipMemcpy(pl.neartab, nt.data(), kNearLogTab * sizeof(double), hipMemcpyHostToDevice));
  }
  alloc_syswork(pl.sw, pl);
  pl.self = new Forest();
  build_forest(*pl.self, {&pl}, {&pl.sw}, s);
  PHS_HIP(hipStreamSynchronize(s));
  pool_mark_idle();
  pl.t_plan = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

void create_plan(const double *xy, int64_t n, const phs_plan_opts *o, hipStream_t s, Plan &pl) {
  plan_create(xy, n, o, s, pl);
}

void eval_plan(Plan &pl, const double *w, const double *beta, int nrhs, const double *targets,
               int64_t m, double *out, hipStream_t s) {
  for (int c = 0; c < nrhs; ++c) {
    f_gather_user(*pl.self, 0, w + (int64_t)c * pl.n, V_IN, s);
    const double *wt = pl.sw.v[V_IN];
    if (pl.direct) {
      direct_eval_targets(pl, wt, beta + (int64_t)c * pl.S, targets, m, out + (int64_t)c * m, s);
    } else if (pl.core_log) {
      log_expansions(pl, V_IN, s);
      log_eval_targets(pl, wt, beta + (int64_t)c * pl.S, targets, m, out + (int64_t)c * m, s);
    } else {
      dist_expansions(pl, V_IN, s);
      dist_eval_targets(pl, wt, beta + (int64_t)c * pl.S, targets, m, out + (int64_t)c * m, s);
    }
  }
}

namespace {

// One column at a time through the plan's own forest (one system), so a
// column's arithmetic is that of the same system in a batch.
phs_status solve_impl(Plan &pl, const double *f, int nrhs, const phs_solve_opts *o,
                      double *w_out, double *beta_out, phs_solve_info *info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = pl.n;
  const double rtol = (o && o->rtol > 0) ? o->rtol : 1e-8;
  const int maxit = (o && o->maxit > 0) ? o->maxit : 500;
  const int check_every = (o && o->check_every > 0) ? o->check_every : 1;
  const int prec = (o && o->precision >= 0) ? o->precision : pl.precision;
  PHS_REQUIRE(prec == PHS_FP64 || prec == PHS_MIXED || prec == PHS_NEAR32,
              PHS_ERR_INVALID_ARGUMENT, "bad precision");
  int total_iters = 0, total_outer = 0, it32 = 0, it64 = 0, falls = 0;
  double worst_rel = 0.0;
  phs_status st = PHS_OK;
  sync_forest_pc(*pl.self, s);
  for (int c = 0; c < nrhs; ++c) {
    std::vector<SolveJob> jobs(1);
    jobs[0].sys = 0;
    jobs[0].f = f + (int64_t)c * n;
    jobs[0].w_out = w_out + (int64_t)c * n;
    jobs[0].beta_out = beta_out + (int64_t)c * pl.S;
    solve_forest(*pl.self, jobs, rtol, maxit, check_every, prec, s);
    total_iters += jobs[0].iters;
    total_outer += jobs[0].outer;
    it32 += jobs[0].iters32;
    it64 += jobs[0].iters64;
    falls += jobs[0].fallback ? 1 : 0;
    worst_rel = std::max(worst_rel, jobs[0].rel);
    if (jobs[0].status != PHS_OK && st == PHS_OK) st = jobs[0].status;
    if (jobs[0].status == PHS_ERR_BREAKDOWN) st = PHS_ERR_BREAKDOWN;
  }
  PHS_HIP(hipStreamSynchronize(s));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->iters = total_iters;
    info->outer_refinements = total_outer;
    info->rel_residual = worst_rel;
    info->t_solve =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->iters_fp32 = it32;
    info->iters_fp64 = it64;
    info->fp64_fallback = falls;
    info->t_plan = pl.t_plan;
    info->t_precond = pl.t_precond;
  }
  if (st == PHS_ERR_NOT_CONVERGED) set_error(st, "PCG did not reach rtol within maxit");
  if (st == PHS_ERR_BREAKDOWN) set_error(st, "PCG breakdown: non-positive curvature");
  return st;
}

template <class F>
phs_status guarded(F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    set_error(e.code, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error(PHS_ERR_OUT_OF_MEMORY, "host allocation failed");
    return PHS_ERR_OUT_OF_MEMORY;
  } catch (...) {
    set_error(PHS_ERR_DEVICE, "unexpected internal error");
    return PHS_ERR_DEVICE;
  }
}

}  // namespace
}  // namespace phs

using namespace phs;

struct phs_plan_s {
  Plan pl;
};

extern "C" {

phs_status phs_plan(const double *xy, int64_t n, const phs_plan_opts *opts, void *stream,
                    phs_plan_t *out) {
  if (!out) {
    set_error(PHS_ERR_INVALID_ARGUMENT, "null output handle");
    return PHS_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  phs_plan_s *h = new (std::nothrow) phs_plan_s();
  if (!h) {
    set_error(PHS_ERR_OUT_OF_MEMORY, "host allocation failed");
    return PHS_ERR_OUT_OF_MEMORY;
  }
  phs_status st = guarded([&] {
    plan_create(xy, n, opts, S(stream), h->pl);
    return PHS_OK;
  });
  if (st != PHS_OK) {
    delete h;
    return st;
  }
  *out = h;
  return PHS_OK;
}

phs_status phs_matvec(phs_plan_t plan, const double *v, double *y, int32_t nrhs,
                      int32_t precision, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && v && y && nrhs >= 1, PHS_ERR_INVALID_ARGUMENT, "bad matvec arguments");
    PHS_REQUIRE(precision == PHS_FP64 || precision == PHS_MIXED || precision == PHS_NEAR32,
                PHS_ERR_INVALID_ARGUMENT, "bad precision");
    Plan &pl = plan->pl;
    hipStream_t s = S(stream);
    Forest &F = *pl.self;
    for (int c = 0; c < nrhs; ++c) {
      f_gather_user(F, 0, v + (int64_t)c * pl.n, V_IN, s);
      f_matvec(F, F.mask[0], V_IN, V_OUT, precision, s);
      f_scatter_user(F, 0, V_OUT, y + (int64_t)c * pl.n, s);
    }
    return PHS_OK;
  });
}

phs_status phs_precond_build(phs_plan_t plan, const phs_precond_opts *opts, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && opts, PHS_ERR_INVALID_ARGUMENT, "bad precond arguments");
    const auto t0 = std::chrono::steady_clock::now();
    vecchia_build(plan->pl, *opts, S(stream));
    refresh_forest(*plan->pl.self, S(stream));
    plan->pl.t_precond =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return PHS_OK;
  });
}

phs_status phs_solve(phs_plan_t plan, const double *f, int32_t nrhs, const phs_solve_opts *opts,
                     double *w, double *beta, phs_solve_info *info, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && f && w && beta && nrhs >= 1, PHS_ERR_INVALID_ARGUMENT,
                "bad solve arguments");
    return solve_impl(plan->pl, f, nrhs, opts, w, beta, info, S(stream));
  });
}

phs_status phs_eval(phs_plan_t plan, const double *w, const double *beta, int32_t nrhs,
                    const double *targets, int64_t m, double *out, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && w && beta && nrhs >= 1 && m >= 0, PHS_ERR_INVALID_ARGUMENT,
                "bad eval arguments");
    if (m == 0) return PHS_OK;
    PHS_REQUIRE(targets && out, PHS_ERR_INVALID_ARGUMENT, "null targets/out");
    eval_plan(plan->pl, w, beta, nrhs, targets, m, out, S(stream));
    return PHS_OK;
  });
}

phs_status phs_plan_info(phs_plan_t plan, double *center, double *scale, int32_t *Sout,
                         int32_t *Rout, int32_t *leaf_level, int32_t *order,
                         double *tree_half_width) {
  return guarded([&] {
    PHS_REQUIRE(plan, PHS_ERR_INVALID_ARGUMENT, "null plan");
    const Plan &pl = plan->pl;
    if (center) {
      center[0] = pl.c[0];
      center[1] = pl.c[1];
    }
    if (scale) *scale = pl.rho;
    if (Sout) *Sout = pl.S;
    if (Rout) *Rout = pl.R;
    if (leaf_level) *leaf_level = pl.tree.L;
    if (order) *order = pl.core_log ? pl.p64 : pl.q64;
    if (tree_half_width) *tree_half_width = pl.tree.h;
    return PHS_OK;
  });
}

phs_status phs_plan_tree(phs_plan_t plan, int32_t *order, int32_t *leaf, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && order && leaf, PHS_ERR_INVALID_ARGUMENT, "bad arguments");
    const Plan &pl = plan->pl;
    hipStream_t s = S(stream);
    PHS_HIP(hipMemcpyAsync(order, pl.order, pl.n * 4, hipMemcpyDeviceToDevice, s));
    PHS_HIP(hipMemcpyAsync(leaf, pl.leafkey, pl.n * 4, hipMemcpyDeviceToDevice, s));
    return PHS_OK;
  });
}

phs_status phs_precond_export(phs_plan_t plan, int32_t *rank, int32_t *nbr, double *coef,
                              double *diag, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && rank && nbr && coef && diag, PHS_ERR_INVALID_ARGUMENT,
                "bad export arguments");
    PHS_REQUIRE(plan->pl.has_pc, PHS_ERR_NOT_READY, "no preconditioner built");
    vecchia_export(plan->pl, rank, nbr, coef, diag, S(stream));
    return PHS_OK;
  });
}

phs_status phs_precond_apply(phs_plan_t plan, const double *r, double *z, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && r && z, PHS_ERR_INVALID_ARGUMENT, "bad apply arguments");
    Plan &pl = plan->pl;
    PHS_REQUIRE(pl.has_pc, PHS_ERR_NOT_READY, "no preconditioner built");
    hipStream_t s = S(stream);
    Forest &F = *pl.self;
    sync_forest_pc(F, s);
    f_gather_user(F, 0, r, V_IN, s);
    f_precond_apply(F, F.mask[0], V_IN, V_OUT, V_TMP, s);
    f_scatter_user(F, 0, V_OUT, z, s);
    return PHS_OK;
  });
}

struct phs_batch_s {
  Batch b;
};

phs_status phs_batch_create(const phs_plan_t *plans, int32_t nplans, const int32_t *nrhs,
                            void *stream, phs_batch_t *out) {
  if (!out) {
    set_error(PHS_ERR_INVALID_ARGUMENT, "null output handle");
    return PHS_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  phs_batch_s *h = new (std::nothrow) phs_batch_s();
  if (!h) {
    set_error(PHS_ERR_OUT_OF_MEMORY, "host allocation failed");
    return PHS_ERR_OUT_OF_MEMORY;
  }
  phs_status st = guarded([&] {
    PHS_REQUIRE(plans && nrhs && nplans >= 1, PHS_ERR_INVALID_ARGUMENT, "bad batch arguments");
    std::vector<Plan *> pv;
    std::vector<int> rv;
    for (int i = 0; i < nplans; ++i) {
      PHS_REQUIRE(plans[i], PHS_ERR_INVALID_ARGUMENT, "null plan in batch");
      pv.push_back(&plans[i]->pl);
      rv.push_back(nrhs[i]);
    }
    batch_create(h->b, pv, rv, S(stream));
    return PHS_OK;
  });
  if (st != PHS_OK) {
    delete h;
    return st;
  }
  *out = h;
  return PHS_OK;
}

phs_status phs_batch_solve(phs_batch_t batch, const double *const *f, double *const *w,
                           double *const *beta, const phs_solve_opts *opts,
                           phs_solve_info *info, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(batch && f && w && beta, PHS_ERR_INVALID_ARGUMENT, "bad batch solve arguments");
    return batch_solve(batch->b, f, w, beta, opts, info, S(stream));
  });
}

void phs_batch_destroy(phs_batch_t batch) {
  delete batch;
  pool_mark_idle();
}

struct phs_server_s {
  Server sv;
};

phs_status phs_server_create(const phs_server_opts *opts, void *stream, phs_server_t *out) {
  if (!out) {
    set_error(PHS_ERR_INVALID_ARGUMENT, "null output handle");
    return PHS_ERR_INVALID_ARGUMENT;
  }
  *out = nullptr;
  phs_server_s *h = new (std::nothrow) phs_server_s();
  if (!h) {
    set_error(PHS_ERR_OUT_OF_MEMORY, "host allocation failed");
    return PHS_ERR_OUT_OF_MEMORY;
  }
  phs_status st = guarded([&] {
    PHS_REQUIRE(opts, PHS_ERR_INVALID_ARGUMENT, "null server options");
    server_create(h->sv, *opts, S(stream));
    return PHS_OK;
  });
  if (st != PHS_OK) {
    delete h;
    return st;
  }
  *out = h;
  return PHS_OK;
}

phs_status phs_server_submit(phs_server_t srv, const phs_request *req, int64_t *id) {
  return guarded([&] {
    PHS_REQUIRE(srv && req && id, PHS_ERR_INVALID_ARGUMENT, "bad submit arguments");
    *id = server_submit(srv->sv, *req);
    return PHS_OK;
  });
}

phs_status phs_server_step(phs_server_t srv, int32_t *active, int32_t *queued) {
  return guarded([&] {
    PHS_REQUIRE(srv, PHS_ERR_INVALID_ARGUMENT, "null server");
    server_step(srv->sv);
    if (active) *active = (int32_t)srv->sv.active.size();
    if (queued) *queued = (int32_t)(srv->sv.queue.size() + srv->sv.building);
    return PHS_OK;
  });
}

phs_status phs_server_poll(phs_server_t srv, int64_t id, phs_request_info *info) {
  return guarded([&] {
    PHS_REQUIRE(srv && info, PHS_ERR_INVALID_ARGUMENT, "bad poll arguments");
    server_poll(srv->sv, id, *info);
    return PHS_OK;
  });
}

phs_status phs_server_memory(phs_server_t srv, int64_t *in_use, int64_t *peak) {
  return guarded([&] {
    PHS_REQUIRE(srv, PHS_ERR_INVALID_ARGUMENT, "null server");
    if (in_use) *in_use = srv->sv.in_use + srv->sv.reserved + srv->sv.forest_bytes;
    if (peak) *peak = srv->sv.peak;
    return PHS_OK;
  });
}

void phs_server_destroy(phs_server_t srv) {
  delete srv;
  pool_mark_idle();
}

void phs_plan_destroy(phs_plan_t plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  delete plan;
  pool_mark_idle();
}

const char *phs_last_error(void) { return g_last_error.c_str(); }

phs_status phs_tune_precond(phs_plan_t plan, const double *f, const phs_tune_opts *opts,
                            phs_tune_result *out, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(plan && f && out, PHS_ERR_INVALID_ARGUMENT, "bad tune arguments");
    phs_tune_opts o{};
    if (opts) o = *opts;
    *out = phs_tune_result{};
    tune_precond(plan->pl, f, o, *out, S(stream));
    return PHS_OK;
  });
}

phs_status phs_autotune_plan(const double *xy, int64_t n, int32_t k, int32_t poly_degree,
                             const phs_autotune_opts *opts, phs_plan_opts *best,
                             phs_autotune_result *out, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(xy && best && out && k >= 1 && k <= 4 && n >= 8 && n < (int64_t(1) << 30),
                PHS_ERR_INVALID_ARGUMENT, "bad autotune arguments");
    phs_autotune_opts o{};
    if (opts) o = *opts;
    autotune_plan(xy, n, k, poly_degree, o, *best, *out, S(stream));
    return PHS_OK;
  });
}

phs_status phs_direct_sum(int32_t k, const double *xy, int64_t n, const double *q,
                          const double *targets, int64_t m, double *out, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(k >= 1 && k <= 4, PHS_ERR_INVALID_ARGUMENT, "k must be 1..4");
    PHS_REQUIRE(n >= 1 && m >= 0 && n < (int64_t(1) << 31) && m < (int64_t(1) << 31),
                PHS_ERR_INVALID_ARGUMENT, "bad sizes");
    PHS_REQUIRE(xy && q && (m == 0 || (targets && out)), PHS_ERR_INVALID_ARGUMENT,
                "null argument");
    if (m == 0) return PHS_OK;
    hipStream_t s = S(stream);
    const int64_t need = direct_scratch_doubles(m, n);
    double *scr = need > 0 ? dmalloc<double>(need) : nullptr;
    try {
      direct_sum_plain(k, xy, n, q, targets, m, out, scr, need, s);
    } catch (...) {
      dfree(scr);
      throw;
    }
    dfree(scr);  // recycled only once the device is idle
    return PHS_OK;
  });
}

phs_status phs_direct_sum_noalloc(int32_t k, const double *xy, int64_t n, const double *q,
                                  const double *targets, int64_t m, double *out, void *stream) {
  return guarded([&] {
    PHS_REQUIRE(k >= 1 && k <= 4, PHS_ERR_INVALID_ARGUMENT, "k must be 1..4");
    PHS_REQUIRE(n >= 1 && m >= 0 && n < (int64_t(1) << 31) && m < (int64_t(1) << 31),
                PHS_ERR_INVALID_ARGUMENT, "bad sizes");
    PHS_REQUIRE(xy && q && (m == 0 || (targets && out)), PHS_ERR_INVALID_ARGUMENT,
                "null argument");
    if (m == 0) return PHS_OK;
    int64_t cap = 0;
    double *scr = direct_scratch(&cap);
    const int64_t need = direct_scratch_doubles(m, n);
    PHS_REQUIRE(need <= cap, PHS_ERR_INVALID_ARGUMENT,
                "direct sum needs " + std::to_string(need) +
                    " doubles of scratch, above the no-allocation maximum of " +
                    std::to_string(cap));
    direct_sum_plain(k, xy, n, q, targets, m, out, scr, cap, S(stream));
    return PHS_OK;
  });
}

phs_status phs_memory_stats(int64_t *allocations, int64_t *device_mallocs,
                            int64_t *bytes_in_use, int64_t *bytes_held) {
  pool_stats(allocations, device_mallocs, bytes_in_use, bytes_held);
  return PHS_OK;
}

void phs_set_graphs(int32_t on) { g_graphs.store(on != 0, std::memory_order_relaxed); }

void phs_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  g_prof_level = on;
}

int32_t phs_profile_read(char (*names)[48], int64_t *launches, double *total_ms,
                         int32_t cap) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_flush_locked();
  int32_t i = 0;
  for (auto &kv : g_prof) {
    if (i >= cap) break;
    if (names) {
      std::strncpy(names[i], kv.first.c_str(), 47);
      names[i][47] = 0;
    }
    if (launches) launches[i] = kv.second.launches;
    if (total_ms) total_ms[i] = kv.second.ms;
    ++i;
  }
  g_prof.clear();
  return i;
}

}  // extern "C"
