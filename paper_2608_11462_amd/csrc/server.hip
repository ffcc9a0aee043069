// Serving: a request loop with continuous batching over the lockstep PCG
// engine.  Requests wait in FIFO order until a slot and device memory are
// free; an admitted request's plan (tree, polynomial block, FMM tables,
// workspace) and Vecchia preconditioner are built by a worker thread on a
// stream of its own while the lockstep rounds of the active requests go on,
// and stay resident in HBM with its Krylov vectors until it finishes.  Each step runs one PCG round of
// every active request in shared launches; requests that finish are evaluated
// at their targets and release their memory, and the forest of active systems
// is rebuilt before the next round.  Requests much smaller than the largest
// active one get extra rounds of their own between full rounds (time sharing),
// so they are not held to the pace of the largest request.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "phs_internal.h"

namespace phs {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

// Estimate of the device memory of one request with the default plan options
// (leaf size 40/64, FP64 log orders 27 and 31, Chebyshev 16 and FP32 8), used
// to decide whether a waiting request may be admitted; once built, the
// request is charged what it really holds.  Counted:
// node arrays, polynomial block, FMM workspace of one system and its tables
// (with the four near-field partial sums per node of a log-kernel plan),
// ten Krylov vectors, the Vecchia factor and its transpose, and the peak of
// the temporaries of the preconditioner build.
int64_t request_bytes(int64_t n, int k, int m) {
  const bool log_k = (k % 2 == 0);
  const int leaf = log_k ? 40 : 64;
  int L = (int)std::lround(std::log((double)std::max<int64_t>(n, 1) / leaf) / std::log(4.0));
  L = std::max(2, std::min(10, L));
  const int64_t boxes = ((int64_t)1 << (2 * (L + 1))) - 16;  // levels 2..L, x3
  const int R = hadamard_rank(k);
  const int S = n_monomials(std::max(min_degree(k), 2));
  const int mm = m > 0 ? m : (k == 2 ? 30 : 50);
  int64_t exp;
  int64_t tables;
  if (log_k) {
    exp = 32LL * R * boxes / 3 * 16;
    tables = 3 * (32LL * 32 * 8 * 9 + 512);
  } else {
    exp = 256LL * R * boxes / 3 * 8;
    tables = 40LL * (256 * 256 * 8 + 64 * 64 * 4) + (4 << 20);
  }
  const int64_t nodes = n * (52 + 8LL * S + 10 * 8 + 4 + (log_k ? 32 : 0));
  const int64_t vecchia = n * (16 + 24LL * mm);
  const int64_t transient = n * (100 + 16LL * mm);
  return 2 * exp + tables + nodes + vecchia + transient + (int64_t)(1 << 22);
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(bmu);
    stop = true;
  }
  bcv.notify_all();
  if (builder.joinable()) builder.join();
  (void)hipDeviceSynchronize();
  delete F;
  for (Request *r : all) {
    delete r->plan;
    delete r;
  }
  if (bs) (void)hipStreamDestroy(bs);
}

namespace {

// The worker: builds the plan and preconditioner of each request handed to
// it, on its own stream, and hands it back with the device bytes the build
// left held (this thread's pool tally; the build's temporaries are returned
// by then).  A failed build leaves no plan and the error in the request.
void build_request(Server &sv, Request *r) {
  const phs_request &in = r->in;
  phs_plan_opts po{};
  po.k = in.k;
  po.poly_degree = in.poly_degree;
  po.precision = sv.opts.precision;
  const int64_t n0 = pool_thread_net();
  try {
    r->plan = new Plan();
    create_plan(in.xy, in.n, &po, sv.bs, *r->plan);
    vecchia_build(*r->plan, in.precond, sv.bs);
    PHS_HIP(hipStreamSynchronize(sv.bs));
    r->built_bytes = std::max<int64_t>(pool_thread_net() - n0, 0);
    r->built_status = PHS_OK;
  } catch (const Error &e) {
    (void)hipStreamSynchronize(sv.bs);
    delete r->plan;
    r->plan = nullptr;
    r->built_status = e.code;
  } catch (const std::bad_alloc &) {
    (void)hipStreamSynchronize(sv.bs);
    delete r->plan;
    r->plan = nullptr;
    r->built_status = PHS_ERR_OUT_OF_MEMORY;
  }
  pool_mark_idle();
}

void builder_loop(Server *sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->bmu);
      sv->bcv.wait(lk, [&] { return sv->stop || !sv->to_build.empty(); });
      if (sv->stop) return;
      // smallest request first: a small request is not held behind the build
      // of a large one
      auto it = std::min_element(sv->to_build.begin(), sv->to_build.end(),
                                 [](const Request *a, const Request *b) { return a->in.n < b->in.n; });
      r = *it;
      sv->to_build.erase(it);
    }
    build_request(*sv, r);
    {
      std::lock_guard<std::mutex> lk(sv->bmu);
      sv->built.push_back(r);
    }
    sv->bcv.notify_all();
  }
}

}  // namespace

void server_create(Server &sv, const phs_server_opts &o, hipStream_t s) {
  PHS_REQUIRE(o.precision == PHS_FP64 || o.precision == PHS_MIXED || o.precision == PHS_NEAR32,
              PHS_ERR_INVALID_ARGUMENT, "bad precision");
  PHS_REQUIRE(o.hbm_budget >= 0 && o.max_active >= 0 && o.maxit >= 0 && o.rtol >= 0,
              PHS_ERR_INVALID_ARGUMENT, "bad server options");
  sv.opts = o;
  sv.s = s;
  sv.P = SolveParams{o.rtol > 0 ? o.rtol : 1e-8, o.maxit > 0 ? o.maxit : 500, 1, o.precision};
  if (o.max_active <= 0) sv.opts.max_active = 64;
  if (o.hbm_budget > 0) {
    sv.budget = o.hbm_budget;
  } else {
    size_t fr = 0, tot = 0;
    PHS_HIP(hipMemGetInfo(&fr, &tot));
    sv.budget = (int64_t)(fr / 4 * 3);
  }
  sv.t0 = now_s();
  PHS_HIP(hipGetDevice(&sv.device));
  PHS_HIP(hipStreamCreateWithFlags(&sv.bs, hipStreamNonBlocking));
  sv.builder = std::thread(builder_loop, &sv);
}

int64_t server_submit(Server &sv, const phs_request &r) {
  PHS_REQUIRE(r.xy && r.f && r.w && r.beta && r.n >= 1 && r.m >= 0, PHS_ERR_INVALID_ARGUMENT,
              "bad request arrays");
  PHS_REQUIRE(r.m == 0 || (r.targets && r.values), PHS_ERR_INVALID_ARGUMENT,
              "request with targets needs targets and values arrays");
  PHS_REQUIRE(r.k >= 1 && r.k <= 4, PHS_ERR_INVALID_ARGUMENT, "k must be 1..4");
  Request *q = new Request();
  q->id = sv.next_id++;
  q->in = r;
  q->t_submit = now_s() - sv.t0;
  q->bytes = request_bytes(r.n, r.k, r.precond.m);
  sv.all.push_back(q);
  sv.queue.push_back(q);
  return q->id;
}

namespace {

void fail(Server &sv, Request *r, phs_status st) {
  r->state = PHS_REQ_FAILED;
  r->status = st;
  r->t_done = now_s() - sv.t0;
  delete r->plan;
  r->plan = nullptr;
}


}  // namespace

void server_step(Server &sv) {
  hipStream_t s = sv.s;
  // 1. requests whose builds finished join the active set (with nothing
  // active, wait for one rather than return empty-handed)
  std::vector<Request *> fresh;
  std::vector<Request *> got;
  {
    std::unique_lock<std::mutex> lk(sv.bmu);
    if (sv.active.empty() && sv.building > 0 && sv.built.empty())
      sv.bcv.wait(lk, [&] { return !sv.built.empty(); });
    got.swap(sv.built);
  }
  for (Request *r : got) {
    --sv.building;
    sv.reserved -= r->reserve;
    r->reserve = 0;
    if (!r->plan) {
      set_error(r->built_status, "request build failed");
      fail(sv, r, r->built_status);
      continue;
    }
    r->bytes = r->built_bytes;
    r->measured = true;
    // the shared forest grows with each member (descriptors and work tables,
    // well under 1/32 of a request's own memory): keep that much in hand
    if (sv.in_use + sv.reserved + sv.forest_bytes + r->bytes + r->bytes / 32 > sv.budget) {
      // its real footprint is larger than the estimate and does not fit now:
      // release it and let it wait at the head of the queue with its
      // measured size
      delete r->plan;
      r->plan = nullptr;
      r->state = PHS_REQ_QUEUED;
      pool_mark_idle();
      if (r->bytes > sv.budget) {
        set_error(PHS_ERR_OUT_OF_MEMORY, "request larger than the server's memory budget");
        fail(sv, r, PHS_ERR_OUT_OF_MEMORY);
        continue;
      }
      sv.queue.insert(sv.queue.begin(), r);
      continue;
    }
    r->state = PHS_REQ_ACTIVE;
    r->t_admit = now_s() - sv.t0;
    r->job = SolveJob();
    r->job.f = r->in.f;
    r->job.w_out = r->in.w;
    r->job.beta_out = r->in.beta;
    sv.in_use += r->bytes;
    sv.active.push_back(r);
    fresh.push_back(r);
    sv.changed = true;
  }
  // 2. waiting requests go to the builder, FIFO, by slot and memory budget
  // (their estimated bytes reserved); at most kBuilding handed over at a time
  constexpr int kBuilding = 8;
  while (!sv.queue.empty() && (int)sv.active.size() + sv.building < sv.opts.max_active &&
         sv.building < kBuilding) {
    Request *r = sv.queue.front();
    if (r->bytes > sv.budget) {
      sv.queue.erase(sv.queue.begin());
      set_error(PHS_ERR_OUT_OF_MEMORY, "request larger than the server's memory budget");
      fail(sv, r, PHS_ERR_OUT_OF_MEMORY);
      continue;
    }
    // a build reserves half again its estimate (its temporaries come and go
    // while it runs beside the steps), or what room is left if nothing else
    // is active or building
    const int64_t room = sv.budget - (sv.in_use + sv.reserved + sv.forest_bytes);
    if (r->bytes + r->bytes / 32 > room) break;
    if (r->bytes + r->bytes / 2 > room && (!sv.active.empty() || sv.building > 0)) break;
    sv.queue.erase(sv.queue.begin());
    r->reserve = std::min(r->bytes + r->bytes / 2, room);
    sv.reserved += r->reserve;
    ++sv.building;
    {
      std::lock_guard<std::mutex> lk(sv.bmu);
      sv.to_build.push_back(r);
    }
    sv.bcv.notify_all();
  }
  sv.peak = std::max(sv.peak, sv.in_use + sv.reserved + sv.forest_bytes);
  // 3. the forest of active systems (its descriptors and work tables are
  // charged to the server as measured)
  if (sv.changed) {
    delete sv.F;
    sv.F = nullptr;
    pool_mark_idle();
    const int64_t u0 = pool_thread_net();
    sv.forest_bytes = 0;
    if (!sv.active.empty()) {
      std::vector<Plan *> pl;
      std::vector<SysWork *> wk;
      for (size_t i = 0; i < sv.active.size(); ++i) {
        pl.push_back(sv.active[i]->plan);
        wk.push_back(&sv.active[i]->plan->sw);
        sv.active[i]->job.sys = (int)i;
      }
      sv.F = new Forest();
      build_forest(*sv.F, pl, wk, s);
      sv.forest_bytes = std::max<int64_t>(pool_thread_net() - u0, 0);
      sv.peak = std::max(sv.peak, sv.in_use + sv.reserved + sv.forest_bytes);
    }
    sv.changed = false;
  }
  if (sv.active.empty()) return;
  Forest &F = *sv.F;
  if (!fresh.empty()) {
    std::vector<SolveJob *> js;
    for (Request *r : fresh) js.push_back(&r->job);
    solve_begin(F, js, sv.P, s);
  }
  // 4. one lockstep round of every active request
  std::vector<SolveJob *> js;
  int64_t n_big = 0;
  for (Request *r : sv.active) {
    js.push_back(&r->job);
    n_big = std::max(n_big, r->in.n);
  }
  const double ta = now_s();
  solve_round(F, js, sv.P, s);
  const double t_full = now_s() - ta;
  // 5. time sharing: a round lasts as long as the largest request's
  // iteration, so requests at most a quarter of its size get extra rounds of
  // their own, for up to half the time of the full round
  std::vector<SolveJob *> small;
  for (Request *r : sv.active)
    if (r->in.n * 4 <= n_big && r->job.state != J_DONE) small.push_back(&r->job);
  double t_extra = 0.0;
  for (int rounds = 0; !small.empty() && t_extra < 0.5 * t_full && rounds < 32; ++rounds) {
    const double tb = now_s();
    if (!solve_round(F, small, sv.P, s)) break;
    t_extra += now_s() - tb;
    small.erase(std::remove_if(small.begin(), small.end(),
                               [](const SolveJob *j) { return j->state == J_DONE; }),
                small.end());
  }
  // 6. finished requests: evaluate, release
  std::vector<Request *> keep;
  for (Request *r : sv.active) {
    if (r->job.state != J_DONE) {
      keep.push_back(r);
      continue;
    }
    try {
      if (r->in.m > 0)
        eval_plan(*r->plan, r->in.w, r->in.beta, 1, r->in.targets, r->in.m, r->in.values, s);
      PHS_HIP(hipStreamSynchronize(s));
      r->status = r->job.status;
      r->state = PHS_REQ_DONE;
    } catch (const Error &e) {
      set_error(e.code, e.msg);
      r->status = e.code;
      r->state = PHS_REQ_FAILED;
    }
    r->t_done = now_s() - sv.t0;
    delete r->plan;
    r->plan = nullptr;
    sv.in_use -= r->bytes;
    sv.changed = true;
  }
  if (keep.size() != sv.active.size()) pool_mark_idle();
  sv.active = keep;
  if (sv.active.empty()) {
    delete sv.F;
    sv.F = nullptr;
    sv.forest_bytes = 0;
    sv.changed = false;
    pool_mark_idle();
  }
}

void server_poll(Server &sv, int64_t id, phs_request_info &info) {
  PHS_REQUIRE(id >= 1 && id < sv.next_id, PHS_ERR_INVALID_ARGUMENT, "unknown request id");
  const Request &r = *sv.all[id - 1];
  info.state = r.state;
  info.status = r.status;
  info.iters = r.job.iters;
  info.rel_residual = r.job.rel;
  info.t_submit = r.t_submit;
  info.t_admit = r.t_admit;
  info.t_done = r.t_done;
  info.bytes = r.bytes;
}

}  // namespace phs
