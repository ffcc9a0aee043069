// All-pairs (direct) evaluation of the PHS kernel sums
//   out_i = sum_j q_j phi(|t_i - x_j|),  phi(r) = r^k (k odd), r^k log r (k even)
// (eq. phs_fun, the kernel part of eq. phs_interp; with t = x it is the matvec
// M q).  This is the exact matvec of the "hybrid" solver (Sec. 3.3: the same
// preconditioned CG with M applied exactly instead of by the FMM), used
// below the size where the FMM pays, and a plan-free direct sum.
//
// Layout of a launch: the targets are cut into tiles of 256 (one thread per
// target) and the sources into nch contiguous chunks, one workgroup per
// (tile, chunk).  A workgroup stages its chunk's sources through LDS, 256 at a
// time, and every lane reads the same source entry (an LDS broadcast).  With
// one chunk the workgroup writes the scaled sum; otherwise each chunk writes
// its partial sum to a scratch row (nch x nt doubles) and a second kernel adds
// the rows in chunk order, so the result does not depend on scheduling.  The
// chunk count is chosen so a launch has about kDirectBlocks workgroups.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "fmm_common.h"

namespace phs {

namespace {

constexpr int kDirBlock = 256;
constexpr int64_t kDirectBlocks = 2048;  // workgroups a launch aims for
constexpr int kDirMaxChunks = 64;

// Even k in FP64: phi from r^2 with the near-field logarithm (table in LDS).
// FP32: phi_r2f (hardware log2 / sqrt) with FP32 accumulation.
template <int K, class T>
__global__ __launch_bounds__(kDirBlock) void k_direct(
    const double *__restrict__ src, const double *__restrict__ q, int64_t ns,
    const double *__restrict__ tg, int64_t nt, double tcx, double tcy, double trho,
    int64_t ntiles, int64_t chunk, double *__restrict__ dst, int final_scale,
    const double *__restrict__ neartab, const int32_t *__restrict__ mask, int sys) {
  constexpr bool fp64 = std::is_same<T, double>::value;
  constexpr bool table = fp64 && (K % 2 == 0);
  __shared__ double stab[table ? kNearLogTab : 2];
  __shared__ T sx[kDirBlock], sy[kDirBlock], sq[kDirBlock];
  if (mask && !mask[sys]) return;
  const int64_t tile = blockIdx.x % ntiles, ch = blockIdx.x / ntiles;
  const int64_t i = tile * kDirBlock + threadIdx.x;
  if constexpr (table)
    for (int e = threadIdx.x; e < kNearLogTab; e += kDirBlock) stab[e] = neartab[e];
  T xi = T(0), yi = T(0);
  if (i < nt) {
    xi = (T)((tg[2 * i] - tcx) * trho);
    yi = (T)((tg[2 * i + 1] - tcy) * trho);
  }
  T acc = T(0);
  const int64_t j0 = ch * chunk, j1 = std::min(ns, j0 + chunk);
  for (int64_t jb = j0; jb < j1; jb += kDirBlock) {
    __syncthreads();
    const int64_t j = jb + threadIdx.x;
    if (j < j1) {
      sx[threadIdx.x] = (T)src[2 * j];
      sy[threadIdx.x] = (T)src[2 * j + 1];
      sq[threadIdx.x] = (T)q[j];
    }
    __syncthreads();
    const int cnt = (int)std::min<int64_t>(kDirBlock, j1 - jb);
#pragma unroll 8
    for (int s = 0; s < cnt; ++s) {
      const T dx = xi - sx[s], dy = yi - sy[s];
      if constexpr (fp64) {
        const double r2 = fma(dy, dy, dx * dx);
        double ph;
        if constexpr (K == 1) ph = sqrt(r2);
        else if constexpr (K == 3) ph = r2 * sqrt(r2);
        else {
          ph = r2 * near_log(r2, stab);
          if constexpr (K == 4) ph *= r2;
        }
        acc = fma(ph, sq[s], acc);
      } else {
        const float r2 = fmaf(dy, dy, dx * dx);
        acc = fmaf(phi_r2f<K>(r2), sq[s], acc);
      }
    }
  }
  if (i >= nt) return;
  double scale;
  if constexpr (fp64) scale = near_scale<K>();
  else scale = (double)phi_scale_f<K>();
  if (final_scale) dst[i] = scale * (double)acc;
  else dst[ch * nt + i] = (double)acc;
}

// out_i = scale * sum_c part[c][i] (chunk order) + P(t_i) beta (beta may be
// null); P the monomials of total degree <= d, ordered by degree and then by
// descending power of the first coordinate.
__global__ void k_direct_reduce(const double *__restrict__ part, int nch, int64_t nt,
                                double scale, double *__restrict__ out,
                                const double *__restrict__ tg, double tcx, double tcy,
                                double trho, const double *__restrict__ beta, int d,
                                int add_to_out, const int32_t *__restrict__ mask, int sys) {
  if (mask && !mask[sys]) return;
  const int64_t i = blockIdx.x * (int64_t)kDirBlock + threadIdx.x;
  if (i >= nt) return;
  double s = 0.0;
  if (add_to_out) {
    s = out[i];
  } else {
    for (int c = 0; c < nch; ++c) s += part[c * nt + i];
    s *= scale;
  }
  if (beta) {
    const double xi = (tg[2 * i] - tcx) * trho, yi = (tg[2 * i + 1] - tcy) * trho;
    double px[8], py[8];
    px[0] = py[0] = 1.0;
    for (int a = 1; a <= d; ++a) {
      px[a] = px[a - 1] * xi;
      py[a] = py[a - 1] * yi;
    }
    double poly = 0.0;
    int col = 0;
    for (int td = 0; td <= d; ++td)
      for (int a = td; a >= 0; --a) poly += beta[col++] * px[a] * py[td - a];
    s = poly + s;
  }
  out[i] = s;
}

template <class T>
void launch_direct(int k, const double *src, const double *q, int64_t ns, const double *tg,
                   int64_t nt, double tcx, double tcy, double trho, const DirectSplit &sp,
                   double *dst, bool final_scale, const double *neartab, const int32_t *mask,
                   int sys, hipStream_t s) {
  const unsigned nb = (unsigned)(sp.ntiles * sp.nch);
  const char *name = std::is_same<T, double>::value ? "direct" : "direct_f32";
#define PHS_DIRECT(K)                                                                        \
  PHS_LAUNCH(name, s,                                                                        \
             k_direct<K, T><<<nb, kDirBlock, 0, s>>>(src, q, ns, tg, nt, tcx, tcy, trho,     \
                                                     sp.ntiles, sp.chunk, dst,               \
                                                     final_scale ? 1 : 0, neartab, mask, sys))
  switch (k) {
    case 1: PHS_DIRECT(1); break;
    case 2: PHS_DIRECT(2); break;
    case 3: PHS_DIRECT(3); break;
    default: PHS_DIRECT(4); break;
  }
#undef PHS_DIRECT
}

double direct_scale(int k, bool fp64) {
  if (k % 2) return 1.0;
  return fp64 ? 0.5 : (double)0.34657359027997264f;
}

}  // namespace

DirectSplit direct_split(int64_t nt, int64_t ns, int64_t cap) {
  DirectSplit sp;
  sp.ntiles = std::max<int64_t>(1, (nt + kDirBlock - 1) / kDirBlock);
  const int64_t stiles = std::max<int64_t>(1, (ns + kDirBlock - 1) / kDirBlock);
  int64_t nch = (kDirectBlocks + sp.ntiles - 1) / sp.ntiles;
  nch = std::max<int64_t>(1, std::min<int64_t>({nch, (int64_t)kDirMaxChunks, stiles}));
  if (cap >= 0 && nch > 1 && nch * nt > cap) nch = std::max<int64_t>(1, cap / std::max<int64_t>(nt, 1));
  sp.chunk = (stiles + nch - 1) / nch * kDirBlock;
  sp.nch = (int)((ns + sp.chunk - 1) / sp.chunk);
  if (sp.nch < 1) sp.nch = 1;
  return sp;
}

void direct_sum(int k, bool fp64, const double *src, const double *q, int64_t ns,
                const double *tg, int64_t nt, double tcx, double tcy, double trho,
                const double *beta, int d, double *out, double *scratch, int64_t scratch_cap,
                const double *neartab, const int32_t *mask, int sys, hipStream_t s,
                bool fit_scratch) {
  if (nt == 0) return;
  const DirectSplit sp = direct_split(nt, ns, fit_scratch ? scratch_cap : -1);
  const bool single = sp.nch == 1;
  PHS_REQUIRE(single || (int64_t)sp.nch * nt <= scratch_cap, PHS_ERR_INVALID_ARGUMENT,
              "direct sum needs more scratch than provided");
  double *dst = single ? out : scratch;
  if (fp64)
    launch_direct<double>(k, src, q, ns, tg, nt, tcx, tcy, trho, sp, dst, single, neartab, mask,
                          sys, s);
  else
    launch_direct<float>(k, src, q, ns, tg, nt, tcx, tcy, trho, sp, dst, single, neartab, mask,
                         sys, s);
  if (!single || beta) {
    const unsigned nb = (unsigned)((nt + kDirBlock - 1) / kDirBlock);
    PHS_LAUNCH("direct_reduce", s,
               k_direct_reduce<<<nb, kDirBlock, 0, s>>>(scratch, sp.nch, nt, direct_scale(k, fp64),
                                                        out, tg, tcx, tcy, trho, beta, d,
                                                        single ? 1 : 0, mask, sys));
  }
}

int64_t direct_scratch_doubles(int64_t nt, int64_t ns) {
  const DirectSplit sp = direct_split(nt, ns, -1);
  return sp.nch == 1 ? 0 : (int64_t)sp.nch * nt;
}

// Forest matvec of the systems whose plan applies M directly: one launch
// (plus the chunk reduction) per system, each checking its mask.
void direct_matvec(Forest &F, const int32_t *mask, int in, int out, int precision,
                   hipStream_t s) {
  for (int i = 0; i < F.nsys; ++i) {
    const Plan &pl = *F.plan[i];
    if (!pl.direct) continue;
    const SysDev &d = F.hsys[i];
    const SysWork &w = *F.work[i];
    const double *xy = (const double *)pl.xy2;
    const bool fp64 = precision == PHS_FP64 || precision == PHS_FP64_EVAL;
    direct_sum(pl.k, fp64, xy, d.v[in], pl.n, xy, pl.n, 0.0, 0.0, 1.0,
               nullptr, 0, d.v[out], w.dpart, w.dpart_cap, pl.neartab, mask, i, s, false);
  }
}

// Evaluation of a direct plan at user-coordinate targets: the exact kernel sum
// over the nodes plus the polynomial part.  The chunk partials go to the
// plan's own partial buffer (no allocation), with fewer chunks when there are
// many targets.
void direct_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                         const double *targets, int64_t m, double *out, hipStream_t s) {
  direct_sum(pl.k, true, (const double *)pl.xy2, w_tree, pl.n, targets, m, pl.c[0], pl.c[1],
             pl.rho, beta, pl.d, out, pl.sw.dpart, pl.sw.dpart_cap, pl.neartab, nullptr, 0, s,
             true);
}

// ------------------------------------------------------------------ plan-free
// The near-field logarithm table of the plan-free direct sums: one copy per
// device, filled on the first call on that device (no heap allocation: the
// host staging is static too).
namespace {
constexpr int kMaxDevices = 64;
__device__ __align__(256) double g_direct_tab[kNearLogTab];
std::mutex g_direct_mu;
double *g_direct_tab_ptr[kMaxDevices] = {};  // per device
double g_direct_tab_host[kNearLogTab];

int current_device() {
  int dev = 0;
  PHS_HIP(hipGetDevice(&dev));
  PHS_REQUIRE(dev >= 0 && dev < kMaxDevices, PHS_ERR_DEVICE, "device ordinal out of range");
  return dev;
}

const double *direct_table() {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_direct_mu);
  if (!g_direct_tab_ptr[dev]) {
    double *p = nullptr;
    PHS_HIP(hipGetSymbolAddress((void **)&p, HIP_SYMBOL(g_direct_tab)));
    fill_near_log_table(g_direct_tab_host);
    PHS_HIP(hipMemcpy(p, g_direct_tab_host, sizeof(g_direct_tab_host), hipMemcpyHostToDevice));
    g_direct_tab_ptr[dev] = p;
  }
  return g_direct_tab_ptr[dev];
}
}  // namespace

void direct_sum_plain(int k, const double *xy, int64_t n, const double *q, const double *targets,
                      int64_t m, double *out, double *part, int64_t cap, hipStream_t s) {
  const double *tab = direct_table();
  direct_sum(k, true, xy, q, n, targets, m, 0.0, 0.0, 1.0, nullptr, 0, out, part, cap, tab,
             nullptr, 0, s, false);
}

// ------------------------------------------------------------------ no allocation
// Device scratch of phs_direct_sum_noalloc: the chunk partials live in this
// file-scope array instead of pool memory, for callers that cannot allocate.
// Each GPU holds its own copy (8 MiB) until the process ends.  In host code
// its name is only a stand-in: the device address comes from
// hipGetSymbolAddress, taken once per device (with that device current) and
// kept in g_scratch_ptr; kernels and copies get that pointer.  The split of a
// direct sum never needs more than (kDirectBlocks + tiles) * 256 <= 2^20
// partials, so every size fits; the check below still guards it.  All calls
// on one GPU share the array: calls that overlap on one GPU (other streams,
// other threads) race on it.  Nothing in it needs to start at zero (every
// partial is written before it is read).
constexpr int64_t kScratchDoubles = int64_t(1) << 20;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

double *direct_scratch(int64_t *cap) {
  const int dev = current_device();
  std::lock_guard<std::mutex> lk(g_direct_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    PHS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PHS_REQUIRE(p != nullptr, PHS_ERR_DEVICE, "no device address for the direct-sum scratch");
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *cap = kScratchDoubles;
  return g_scratch_ptr[dev];
}

}  // namespace phs
