// Internal declarations of the PHS library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <thread>
#include <mutex>
#include <condition_variable>
#include <deque>
#include <functional>
#include <vector>

#include "../../include/phs.h"

namespace phs {

// ------------------------------------------------------------------ errors
struct Error {
  phs_status code;
  std::string msg;
};

void set_error(phs_status code, const std::string &msg);

#define PHS_HIP(call)                                                         \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::phs::Error{e_ == hipErrorOutOfMemory ? PHS_ERR_OUT_OF_MEMORY    \
                                                   : PHS_ERR_DEVICE,          \
                         std::string(#call) + ": " + hipGetErrorString(e_)};  \
  } while (0)

#define PHS_REQUIRE(cond, code, msg)                                          \
  do {                                                                        \
    if (!(cond)) throw ::phs::Error{(code), (msg)};                           \
  } while (0)

// ------------------------------------------------------------------ profiling
// Kernel launches go through launch(); when profiling is on each launch is
// bracketed by events on its stream and the elapsed time is charged to name.
bool profiling_on();
bool prof_wants(const char *name);
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);

struct ProfScope {
  hipStream_t s;
  bool on;
  ProfScope(const char *name, hipStream_t st) : s(st), on(profiling_on() && prof_wants(name)) {
    if (on) prof_begin(name, s);
  }
  ~ProfScope() {
    if (on) prof_end(s);
  }
};

// Work-table warm-up: while a WarmTables object lives on this thread,
// PHS_LAUNCH enqueues nothing, so running the FMM drivers over a forest only
// builds the work tables they look up (done once when the forest is built,
// so the per-call entry points never allocate).
bool launches_suppressed();
struct WarmTables {
  WarmTables();
  ~WarmTables();
};

#define PHS_LAUNCH(name, stream, ...)                                         \
  do {                                                                        \
    if (!::phs::launches_suppressed()) {                                      \
      ::phs::ProfScope ps_(name, stream);                                     \
      __VA_ARGS__;                                                            \
      PHS_HIP(hipGetLastError());                                             \
    }                                                                         \
  } while (0)

// Table of the near-field logarithm: 2^kNearLogBits centred subintervals of
// the mantissa, each (1/c, -log(1/c)); kNearLogTab doubles in all.  Eight
// bits (4 KB, degree-5 polynomial) measured faster than nine (8 KB, degree 4:
// more LDS bank conflicts) and seven (2 KB, degree 6: one more FMA a pair).
constexpr int kNearLogBits = 8;
constexpr int kNearLogTab = 2 << kNearLogBits;

// ------------------------------------------------------------------ address spaces
// Kernels reach most arrays through per-system descriptors, i.e. as generic
// pointers read from memory.  Read-only inputs are viewed through the
// constant address space (a wave-uniform address then becomes a scalar load)
// and outputs through the global one (global rather than flat stores).
template <class T>
using cptr = const __attribute__((address_space(4))) T *;
template <class T>
using gptr = __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ cptr<T> ro(const T *p) {
  return (cptr<T>)(p);
}
template <class T>
__device__ __forceinline__ gptr<T> rw(T *p) {
  return (gptr<T>)(p);
}
// A wave-uniform read-only pointer the compiler cannot treat as loop
// invariant: loads through it stay where they are written.  A fully unrolled
// loop over a constant table (shift matrices, series coefficients) would
// otherwise have every entry hoisted into registers ahead of the loop.
template <class T>
__device__ __forceinline__ cptr<T> in_place(cptr<T> p) {
  asm volatile("" : "+s"(p));
  return p;
}

// ------------------------------------------------------------------ memory
// Device memory comes from a caching pool: a freed block is parked on the
// freeing thread's pending list and becomes reusable only at pool_mark_idle,
// which synchronises the device first, so a block is never handed out while
// work that used it may still run.  Plans built and destroyed over and over
// (one per solve) then cost no hipMalloc/hipFree in steady state.
void *pool_alloc(size_t bytes);
void pool_free(void *p);
void pool_mark_idle();  // synchronises the device, then recycles pending blocks
void pool_trim();       // returns every idle cached block to HIP
// blocks handed out by pool_alloc so far, hipMalloc calls so far, device
// bytes handed out and not yet recycled, device bytes the pool owns (in use
// and cached)
void pool_stats(int64_t *allocs, int64_t *device_mallocs, int64_t *bytes_in_use,
                int64_t *bytes_held);
// bytes the calling thread has taken from the pool minus the bytes it has
// released (a block counts as released when freed, before it is recycled)
int64_t pool_thread_net();

template <class T>
T *dmalloc(size_t count) {
  if (count == 0) count = 1;
  return static_cast<T *>(pool_alloc(count * sizeof(T)));
}

inline void dfree(void *p) { pool_free(p); }

// ------------------------------------------------------------------ sizes
inline int64_t boxes_at(int l) { return int64_t(1) << (2 * l); }

// Lanes per output of the log M2M / L2L kernels on level l: the coarse levels,
// whose few threads each run a long chain of dependent loads, split every
// sum over a quad of lanes.
// lanes per output coefficient of the generic M2M / L2L kernels: the coarse
// levels have few boxes, so each output is spread over more lanes (shorter
// chains of dependent loads per lane)
__host__ __device__ inline int shift_split(int l) { return l <= 3 ? 16 : l <= 5 ? 4 : 1; }

// Number of core-kernel densities (Hadamard rank) for order k.
inline int hadamard_rank(int k) {
  switch (k) {
    case 1: return 1;
    case 2: return 4;
    case 3: return 4;
    case 4: return 9;
    default: return 0;
  }
}

inline int min_degree(int k) { return (k % 2 == 1) ? (k + 1) / 2 - 1 : k / 2; }
inline int n_monomials(int d) { return (d + 1) * (d + 2) / 2; }
inline double domain_half_width(int k) {
  if (k == 2) return 0.25;
  if (k % 2 == 1) return 0.5;
  return 1.0;
}
// sign of Q_perp^T M Q_perp: +1 positive definite, -1 negative definite
inline int definiteness_sign(int k) { return (k % 4 == 2 || k % 4 == 3) ? 1 : -1; }

// Internal matvec precision: FP64 at the plan's evaluation order (the
// tighter FP64 expansion order that serves phs_eval), which a solve moves to
// when the FP64 operator at the matvec order loses definiteness or stalls.
constexpr int PHS_FP64_EVAL = 3;

// ------------------------------------------------------------------ tree
struct Tree {
  int L = 2;        // leaf level; grid side G = 2^L
  int G = 4;
  double h = 0.25;  // domain [-h, h]^2 in normalised coordinates
  int32_t *leaf_start = nullptr;  // G*G + 1, tree order ranges per leaf
};

// ------------------------------------------------------------------ FMM config
struct LogTables {  // translation tables for one expansion order P
  int P = 0;
  double *Ht64 = nullptr;   // (P+1)^2 real, k-major: Ht[k*(P+1)+l]
  float *Ht32 = nullptr;
  double2 *M2M64 = nullptr; // 4 x (P+1)^2, [c][l][k]
  double2 *L2L64 = nullptr; // 4 x (P+1)^2, [c][j][k]
  float2 *M2M32 = nullptr;
  float2 *L2L32 = nullptr;
  double *Off64 = nullptr;  // 49 x 16 per M2L offset: D^-1, D^-4, D^-q (q=0..3), log|D|
  // shifts in factored form M2M[c] = U_c Rm U_c^-1, L2L[c] = U_c^-1 Rl U_c with
  // U_c = diag(u_c^l), u_c the unit phase of child c's centre offset
  double *Rm64 = nullptr;   // (P+1)^2 real, [l][k]
  double *Rl64 = nullptr;   // (P+1)^2 real, [j][k]
  double2 *Ph64 = nullptr;  // 4 x 32: u_c^k
  void *block = nullptr;    // one device allocation holding all of the above
};

struct ChebTables {  // Chebyshev interpolation tables for Q nodes per axis
  int Q = 0;
  double *nodes64 = nullptr;  // Q
  double *S2c64 = nullptr;    // 2 x Q x Q : child node -> parent basis value
  double *K64 = nullptr;      // 40 x Q^2 x Q^2 : M2L at unit half-width
  float *nodes32 = nullptr;
  float *S2c32 = nullptr;
  float *K32 = nullptr;
};

// ------------------------------------------------------------------ systems
// A "system" is one right-hand side being solved on one plan: it owns the
// PCG vectors, the FMM expansion slabs and the reduction scratch, and shares
// the plan's tree, polynomial block and preconditioner.  Every per-iteration
// kernel runs over a set of systems (a forest: one plan alone, or many plans
// in a batch) through a table of (system, block) work items, so a system's
// arithmetic is the same whatever else runs in the launch.
constexpr int kSysVecs = 10;
constexpr int kSysScal = 128;
enum VecSlot { V_F = 0, V_R, V_W, V_Z, V_P, V_Q, V_TMP, V_DW, V_IN, V_OUT };
// device scalar slots: [0] rho_new [1] rho [2] p.q [3] r.r [4] generic dot
// [8..8+S) projection coefficients, [40..40+S) Q^T (f - M w)
enum ScalSlot { SC_RHO_NEW = 0, SC_RHO = 1, SC_PQ = 2, SC_RR = 3, SC_DOT = 4, SC_PROJ = 8,
                SC_QTF = 40 };

struct SysDev {
  const double *x, *y;
  const float *ux, *uy;
  const double2 *xy2;
  const int32_t *leaf_start;
  const int32_t *order;
  const double *Q;
  const int32_t *nbr;
  const double *coef, *dinv;
  const int32_t *tstart, *tidx;
  const double *tcoef;
  void *mp, *loc;
  double *v[kSysVecs];
  double *red;
  double *sc;
  float *t32;
  double *npart;
  int64_t n;
  double h;
  int32_t S, L, k, R, sign, nbdot, m, has_pc;
};

struct BlkRef {
  int32_t sys, blk;
};

struct SysWork {  // device workspace of one system
  void *mp = nullptr, *loc = nullptr;
  double *v[kSysVecs] = {};
  double *red = nullptr;
  double *sc = nullptr;
  double *dpart = nullptr;  // chunk partial sums of the direct matvec (direct plans)
  int64_t dpart_cap = 0;    // doubles
  float *t32 = nullptr;     // FP32 copy of the densities of an FP32 near field (FMM plans)
  // near-field sums of a node received from the four leaves that take its
  // leaf's pairs symmetrically (log-kernel FMM plans): 4 n doubles
  double *npart = nullptr;
  void release();
};

// ------------------------------------------------------------------ plan
struct Plan {
  int64_t n = 0;
  int k = 2, d = 1, S = 3, R = 4;
  int precision = PHS_FP64;
  int sign = 1;
  bool core_log = true;
  bool direct = false;  // M applied by all-pairs summation instead of the FMM
  double c[2] = {0, 0};
  double rho = 1;
  double hnorm = 0.25;  // half-width of the normalised domain (tree.h >= hnorm)
  Tree tree;
  int p64 = 31, p32 = 15;  // log expansion order (terms beyond the constant)
  int q64 = 16, q32 = 10;  // Chebyshev nodes per axis (distance kernel)
  // FP64 orders of the expansions that serve target evaluation (>= the
  // matvec orders; evaluation runs once per solve, so it takes the tighter one)
  int pe = 31, qe = 16;

  // tree-order node data
  int32_t *order = nullptr;    // tree position -> caller index
  int32_t *inv_order = nullptr;// caller index -> tree position
  int32_t *leafkey = nullptr;
  double *x = nullptr, *y = nullptr;   // normalised coordinates
  float *ux = nullptr, *uy = nullptr;  // FP32 offsets from the leaf centre
  double2 *xy2 = nullptr;              // packed (x, y), source records of the near field
  double *logtab = nullptr;            // 256-entry table of the 1-ulp logarithm (Matern)
  double *neartab = nullptr;           // table of the near-field logarithm (kNearLogTab)

  // polynomial block
  double *Q = nullptr;  // n x S column-major, tree order, orthonormal columns
  std::vector<double> Rm;  // S x S upper triangular (row-major), B = Q R

  // FMM workspace of one system, in bytes (FP64 at the largest order in use)
  size_t exp_bytes = 0;
  LogTables lt64, lt32;  // tables for p64 (FP64) and p32 (FP32)
  ChebTables ct64, ct32;
  LogTables lte;         // tables for pe when pe != p64
  ChebTables cte;        // tables for qe when qe != q64

  // the plan's own system (matvec, solve one column at a time, evaluation)
  SysWork sw;
  struct Forest *self = nullptr;
  double *red = nullptr;    // reduction partials (plan-time reductions)
  int red_cap = 0;
  double *scal = nullptr;   // device scalars
  double *hscal = nullptr;  // pinned host mirror
  int32_t *iscratch = nullptr;  // sort scratch etc. (plan time)

  // preconditioner
  bool has_pc = false;
  int m = 0;
  double nu = 1, alpha = 0.35;
  int pc_nugget_nodes = 0;      // nodes whose block needed a diagonal nugget
  double t_plan = 0, t_precond = 0;  // host seconds of phs_plan / the last precond build
  int32_t *pc_rank = nullptr;   // tree position -> rank
  // after the build: column-major m x n, entry s of node p at s*n + p
  int32_t *pc_nbr = nullptr;    // tree positions, -1 padded
  double *pc_coef = nullptr;    // -lambda / c
  double *pc_dinv = nullptr;    // n      (1 / c)
  int32_t *pc_tstart = nullptr; // n + 1  transpose CSR
  int32_t *pc_tidx = nullptr;   // n*m
  double *pc_tcoef = nullptr;   // n*m

  ~Plan();
};

// ------------------------------------------------------------------ forest
struct Tab {
  BlkRef *d = nullptr;
  int64_t count = 0;
  int64_t off = 0;  // first entry in the forest's table block
};

struct Forest {
  std::vector<Plan *> plan;   // plan of each system
  std::vector<SysWork *> work;
  std::vector<SysDev> hsys;
  SysDev *dsys = nullptr;
  int nsys = 0;
  int maxS = 1;
  int maxL_log = 0, maxL_dist = 0;
  // masks: device int32[nsys] each, host pinned mirrors
  static constexpr int kMasks = 12;
  int32_t *mask[kMasks] = {};   // slices of mask_block
  int32_t *mask_block = nullptr;
  int32_t *hmask[kMasks] = {};   // pinned staging of the last upload
  hipEvent_t mask_ev[kMasks] = {};
  bool mask_pending[kMasks] = {};
  double *hgsc = nullptr;  // packed scalar readback (nsys x 8), pinned, written by the GPU
  void *hpin = nullptr;                    // one pinned block: host masks + hgsc
  // every work table of the forest, concatenated on the host while the forest
  // is built and uploaded in one copy into tab_block at its end (the host
  // copy is the source of that copy and is kept with the forest)
  std::vector<BlkRef> htab;
  BlkRef *tab_block = nullptr;
  Tab vec, dot, pc;                     // element blocks, dot blocks, 8-row blocks
  std::vector<std::pair<uint64_t, Tab>> cache;  // FMM tables keyed by (kind, K, P, level)
  bool any_direct = false;  // some system's plan applies M by direct summation
  bool frozen = false;  // every table is built: a lookup miss is an internal error
  // Launch sequences of the PCG iteration replayed from HIP graphs.  The
  // kernels take only the forest's fixed descriptors, tables, masks and slot
  // numbers as arguments and read masks and scalars from device memory, so a
  // graph stays valid for the forest's lifetime; it is captured (on a stream
  // of the forest's own, as the caller's may be the null stream) the second
  // time its sequence runs.
  static constexpr int kGraphs = 8;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph[kGraphs] = {};
  int graph_runs[kGraphs] = {};
  ~Forest();
};

// Run fn (launches only: no allocation, copy, memset or synchronisation) on
// stream s, from the forest's graph number key once that is captured; eager
// while graphs are switched off, while profiling (its events would be
// captured), or while launches are suppressed.
void f_run(Forest &F, int key, hipStream_t s, const std::function<void(hipStream_t)> &fn);
// PCG iterations through HIP graphs (off by default; phs_set_graphs)
bool graphs_enabled();

// build a forest over systems (plan[i], work[i]); uploads descriptors and the
// element/dot/preconditioner tables.  refresh_forest re-reads the plans'
// preconditioner pointers after phs_precond_build.
void build_forest(Forest &F, const std::vector<Plan *> &plans,
                  const std::vector<SysWork *> &work, hipStream_t s);
void refresh_forest(Forest &F, hipStream_t s);
// refresh_forest if any system's descriptor no longer matches its plan's
// preconditioner (a factor built or rebuilt since the forest last looked)
void sync_forest_pc(Forest &F, hipStream_t s);
void alloc_syswork(SysWork &w, const Plan &pl);
Tab forest_tab(Forest &F, uint64_t key, hipStream_t s);
// Workgroups sharing the output rows of one FP64 Chebyshev M2L tile (the
// split shortens each workgroup's sequence of dependent steps; measured faster
// at every tree size from 3e3 to 1e6 nodes)
__host__ __device__ constexpr int cheb_m2l_max_split(int QQ) {
  return QQ >= 256 ? 4 : (QQ >= 128 ? 2 : 1);
}
// log-kernel P2M packs this many leaves per wavefront (lane = coefficient)
__host__ __device__ inline int p2m_leaves_per_wave(int P) {
  const int g = 64 / (P + 1);
  return g >= 4 ? 4 : (g >= 2 ? 2 : 1);
}
int m2l_chunk(int P);
uint64_t tab_key(int kind, int K, int P, int level);
SysDev make_sysdev(const Plan &pl, const SysWork &w);

// set device mask i to m (nsys flags); uploads only when it changes, and
// never rewrites the pinned staging buffer while its last copy is in flight
void set_mask(Forest &F, int i, const std::vector<int32_t> &m, hipStream_t s);
// gather cnt scalars from slot off of every system into F.hgsc (pinned); the
// values are the host's after the stream synchronises.  f_read_scalars
// synchronises itself.
void f_read_scalars_launch(Forest &F, int off, int cnt, hipStream_t s);

// forest vector operations (systems with mask[sys] != 0)
void f_fill(Forest &F, const int32_t *mask, int slot, double a, hipStream_t s);
void f_copy(Forest &F, const int32_t *mask, int dst, int src, hipStream_t s);
void f_axpby(Forest &F, const int32_t *mask, int y, int x, double a, double b, hipStream_t s);
void f_scale_sign(Forest &F, const int32_t *mask, int dst, int src, hipStream_t s);
void f_dot(Forest &F, const int32_t *mask, int a, int b, int out, hipStream_t s);
void f_project(Forest &F, const int32_t *mask, int slot, hipStream_t s);
// v[slot] = g Pi v[slot] (g = sign_k if sign, else 1) and sc[out] = v[w].v[slot]
void f_project_dot(Forest &F, const int32_t *mask, int slot, bool sign, int w, int out,
                   hipStream_t s);
void f_qt(Forest &F, const int32_t *mask, int slot, int out, hipStream_t s);
void f_pcg_wr(Forest &F, const int32_t *mask, hipStream_t s);
void f_pcg_p(Forest &F, const int32_t *mask, hipStream_t s);
void f_sc_copy(Forest &F, const int32_t *mask, int dst, int src, hipStream_t s);
void f_read_scalars(Forest &F, int off, int cnt, hipStream_t s);  // -> F.hgsc[sys*8+i]
// z = Pi U~ U~^T r (f_precond) or U~ U~^T r (f_precond_apply)
void f_precond(Forest &F, const int32_t *mask, int r, int z, int tmp, hipStream_t s);
// f_precond, then sc[out] = r.z
void f_precond_dot(Forest &F, const int32_t *mask, int r, int z, int tmp, int out,
                   hipStream_t s);
void f_precond_apply(Forest &F, const int32_t *mask, int r, int z, int tmp, hipStream_t s);
void f_gather_user(Forest &F, int sys, const double *src_user, int slot, hipStream_t s);
void f_scatter_user(Forest &F, int sys, int slot, double *dst_user, hipStream_t s);
// y[out] = M v[in] for every masked system, in tree order
void f_matvec(Forest &F, const int32_t *mask, int in, int out, int precision, hipStream_t s);
// adds the symmetric near-field partial sums of the log-kernel systems to v[out]
void f_near_combine(Forest &F, const int32_t *mask, int out, hipStream_t s);

// one right-hand side of one system: inputs in caller order, results, and
// the state of its solve between rounds
enum JobState { J_INIT, J_START, J_PCG, J_PCG_END, J_RESID, J_FINISH, J_DONE };
struct SolveJob {
  int sys = 0;
  const double *f = nullptr;
  double *w_out = nullptr;
  double *beta_out = nullptr;
  int iters = 0, outer = 0;
  double rel = 0.0;
  phs_status status = PHS_OK;
  std::vector<double> beta_host;
  // solve state
  JobState state = J_INIT;
  double bn = 0, fn = 0, tol_abs = 0, rn = 0;
  int it = 0, maxit_inner = 0, inner_prec = PHS_FP64;
  double inner_tol = 0;
  bool pcg_conv = false, pcg_break = false;
  int budget = 0;
  bool fp64_finish = false, count_outer = false, apply_dw = false, have_q = false;
  bool undo_dw = false;  // the last correction raised the residual: take it back
  int iters32 = 0, iters64 = 0;  // inner iterations on the reduced / FP64 operator
  bool fallback = false;         // a reduced-precision solve moved to the FP64 operator
  bool hi = false;               // the FP64 operator is taken at the evaluation order
};
struct SolveParams {
  double rtol;
  int maxit, check_every, prec;
};
// solve_begin: first step for jobs in state J_INIT (all must be systems of F);
// solve_round: one lockstep round of every job not yet J_DONE; false when
// none is left.  Jobs may join between rounds through solve_begin.
void solve_begin(Forest &F, std::vector<SolveJob *> &jobs, const SolveParams &P, hipStream_t s);
bool solve_round(Forest &F, std::vector<SolveJob *> &jobs, const SolveParams &P, hipStream_t s);
void solve_forest(Forest &F, std::vector<SolveJob> &jobs, double rtol, int maxit,
                  int check_every, int prec, hipStream_t s);

// ------------------------------------------------------------------ plans
void create_plan(const double *xy, int64_t n, const phs_plan_opts *o, hipStream_t s, Plan &pl);
void eval_plan(Plan &pl, const double *w, const double *beta, int nrhs, const double *targets,
               int64_t m, double *out, hipStream_t s);

// ------------------------------------------------------------------ batch
struct Batch {
  std::vector<Plan *> plans;
  std::vector<int> nrhs;
  std::vector<SysWork> works;  // one per system
  std::vector<int> sys_plan, sys_col;
  Forest F;
  ~Batch();
};
void batch_create(Batch &b, const std::vector<Plan *> &plans, const std::vector<int> &nrhs,
                  hipStream_t s);
phs_status batch_solve(Batch &b, const double *const *f, double *const *w,
                       double *const *beta, const phs_solve_opts *o, phs_solve_info *info,
                       hipStream_t s);

// ------------------------------------------------------------------ serving
struct Request {
  int64_t id = 0;
  phs_request in;
  int state = PHS_REQ_QUEUED;
  phs_status status = PHS_OK;
  Plan *plan = nullptr;
  SolveJob job;
  int64_t bytes = 0;      // estimate while queued, measured once built
  int64_t reserve = 0;    // bytes reserved while its build runs
  // the build thread's results, read by the scheduling thread once the build
  // is handed back (poll reads the fields above only)
  int64_t built_bytes = 0;
  phs_status built_status = PHS_OK;
  bool measured = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Server {
  phs_server_opts opts{};
  SolveParams P{1e-8, 500, 1, PHS_FP64};
  hipStream_t s = nullptr;
  int64_t budget = 0, in_use = 0, peak = 0;
  int64_t forest_bytes = 0;  // descriptors and work tables of the shared forest
  int64_t next_id = 1;
  std::vector<Request *> queue;    // FIFO
  std::vector<Request *> active;
  std::vector<Request *> all;      // every request ever submitted (owned)
  Forest *F = nullptr;
  bool changed = false;
  double t0 = 0;
  // Plans and preconditioners of admitted requests are built by a worker
  // thread on a stream of its own while the lockstep rounds go on; a request
  // handed to it reserves its estimated bytes until its build is collected.
  std::thread builder;
  std::mutex bmu;
  std::condition_variable bcv;
  std::deque<Request *> to_build;
  std::vector<Request *> built;
  int building = 0;        // handed to the worker, not yet collected
  int64_t reserved = 0;    // estimated bytes of those
  bool stop = false;
  int device = 0;
  hipStream_t bs = nullptr;
  ~Server();
};
void server_create(Server &sv, const phs_server_opts &o, hipStream_t s);
int64_t server_submit(Server &sv, const phs_request &r);
void server_step(Server &sv);
void server_poll(Server &sv, int64_t id, phs_request_info &info);
// device bytes a request of n nodes, order k and conditioning-set size m holds
int64_t request_bytes(int64_t n, int k, int m);

// ------------------------------------------------------------------ launchers
// tree.hip
void minmax_xy(const double *xy, int64_t n, double *out4, double *partials,
               int nblocks, hipStream_t s);
void leaf_keys(const double *xy, int64_t n, double cx, double cy, double rho,
               double h, int L, uint32_t *keys, int32_t *idx, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of key.
// With `in_tmp` given, a result left in (keys_tmp, vals_tmp) by an odd number
// of passes stays there and *in_tmp is set; otherwise it is copied back.
// Temporary buffers: keys_tmp, vals_tmp (n each), hist (256*nblocks + scan ws).
size_t radix_sort_scratch_ints(int64_t n);
void radix_sort_u32(uint32_t *keys, int32_t *vals, int64_t n, int bits,
                    uint32_t *keys_tmp, int32_t *vals_tmp, int32_t *scratch,
                    hipStream_t s, bool *in_tmp = nullptr);
void radix_sort_u64(uint64_t *keys, int32_t *vals, int64_t n, int bits,
                    uint64_t *keys_tmp, int32_t *vals_tmp, int32_t *scratch,
                    hipStream_t s);
void leaf_ranges(const uint32_t *sorted_keys, int64_t n, int nleaves,
                 int32_t *leaf_start, hipStream_t s);
void build_tree_points(const double *xy, const int32_t *order,
                       const uint32_t *keys_sorted, int64_t n, double cx,
                       double cy, double rho, double h, int L, double *x,
                       double *y, float *ux, float *uy, double2 *xy2, int32_t *leafkey,
                       int32_t *inv_order, hipStream_t s);
void count_duplicates(const double *x, const double *y,
                      const int32_t *leaf_start, int nleaves, int32_t *flag,
                      hipStream_t s);

// vec.hip
void poly_block_tree(const double *x, const double *y, int64_t n, int d,
                     double *B, hipStream_t s);
// Grid size of the forest's reductions (depends only on n).
int dot_blocks(int64_t n);
// Gram matrix out[a*S + b] = B_a . B_b (a <= b) of the S tree-ordered columns of
// B, by deterministic two-stage reductions; partials holds the block sums.
void gram(const double *B, int64_t n, int S, double *partials, double *out,
          hipStream_t s);
void apply_rinv(double *B, int64_t n, int S, const double *Rinv_dev,
                hipStream_t s);

// fmm_log.hip
void build_log_tables(LogTables &t, int P);
void free_log_tables(LogTables &t);
size_t log_expansion_bytes(int L, int P, int ndens, bool fp64);
// even-k systems of the forest: y[out] = M v[in]
void log_matvec(Forest &F, const int32_t *mask, int in, int out, int precision,
                hipStream_t s);
// expansions at the evaluation order of system `sys` of the plan's own forest
void log_expansions(Plan &pl, int in, hipStream_t s);

// fmm_dist.hip
void build_cheb_tables(ChebTables &t, int Q);
void free_cheb_tables(ChebTables &t);
size_t cheb_expansion_bytes(int L, int Q, int ndens, bool fp64);
void dist_matvec(Forest &F, const int32_t *mask, int in, int out, int precision,
                 hipStream_t s);
void dist_expansions(Plan &pl, int in, hipStream_t s);

void log_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                      const double *targets, int64_t m, double *out, hipStream_t s);
void dist_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                       const double *targets, int64_t m, double *out, hipStream_t s);

// direct.hip: all-pairs kernel sums out_i = sum_j q_j phi(|t_i - x_j|), t_i
// taken as (t - c) rho; split over source chunks whose partial sums go to
// `scratch` (nch x nt doubles, none when one chunk suffices) and are added in
// chunk order; beta (may be null): adds the polynomial part of degree d.
struct DirectSplit {
  int64_t ntiles = 1;  // target tiles of 256
  int nch = 1;         // source chunks
  int64_t chunk = 0;   // sources per chunk (a multiple of 256)
};
// cap >= 0: at most cap doubles of partials (fewer chunks if needed)
DirectSplit direct_split(int64_t nt, int64_t ns, int64_t cap);
int64_t direct_scratch_doubles(int64_t nt, int64_t ns);  // uncapped split
// fit_scratch: take the split that fits scratch_cap; otherwise the uncapped
// split, which must fit (INVALID_ARGUMENT if not)
void direct_sum(int k, bool fp64, const double *src, const double *q, int64_t ns,
                const double *tg, int64_t nt, double tcx, double tcy, double trho,
                const double *beta, int d, double *out, double *scratch, int64_t scratch_cap,
                const double *neartab, const int32_t *mask, int sys, hipStream_t s,
                bool fit_scratch);
void direct_matvec(Forest &F, const int32_t *mask, int in, int out, int precision,
                   hipStream_t s);
void direct_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                         const double *targets, int64_t m, double *out, hipStream_t s);
// plan-free FP64 direct sum in the caller's coordinates (no normalisation)
void direct_sum_plain(int k, const double *xy, int64_t n, const double *q, const double *targets,
                      int64_t m, double *out, double *part, int64_t cap, hipStream_t s);
// this device's static scratch of the no-allocation entry point (device
// address, from hipGetSymbolAddress) and its size in doubles
double *direct_scratch(int64_t *cap);
void fill_near_log_table(double *tab);

// tune.hip
void tune_precond(Plan &pl, const double *f, const phs_tune_opts &o, phs_tune_result &res,
                  hipStream_t s);
void autotune_plan(const double *xy, int64_t n, int k, int degree, const phs_autotune_opts &o,
                   phs_plan_opts &best, phs_autotune_result &res, hipStream_t s);

// vecchia.hip
void vecchia_build(Plan &pl, const phs_precond_opts &o, hipStream_t s);
void vecchia_free(Plan &pl);
void vecchia_export(Plan &pl, int32_t *rank, int32_t *nbr, double *coef, double *diag,
                    hipStream_t s);


}  // namespace phs
