// Systems and forests: the per-iteration vector kernels of projected PCG
// (eq. phs_linsys_solve and the projector of Sec. 2) and the Vecchia
// preconditioner apply (Sec. 2.2, Fig. vecchia_chol), written once over a set
// of systems.  A launch walks a table of (system, block) items; every system
// reads its own descriptor, so the arithmetic of one system does not depend on
// which other systems share the launch.  Reductions are two-stage with a block
// count that depends only on the system's n, so results are bitwise
// reproducible and identical alone or in a batch.
#include <algorithm>
#include <cstring>

#include "fmm_common.h"
#include "phs_internal.h"

namespace phs {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
  __syncthreads();
  return t;  // valid in thread 0
}

// ------------------------------------------------------------------ elementwise
__global__ void kf_fill(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                        const int32_t *__restrict__ mask, int slot, double a) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  if (i < d.n) d.v[slot][i] = a;
}

// the densities of an FP32 near field, converted once per matvec instead of
// once per pair
__global__ void kf_near_t32(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                            const int32_t *__restrict__ mask, int slot) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  if (!d.t32) return;  // direct-summation systems
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  if (i < d.n) d.t32[i] = (float)d.v[slot][i];
}

// Adds the partial-sum slots of the symmetric FP64 near field of the log-kernel
// leaf pass (times the 1/2 of phi = (1/2) r^k log r^2) to its output.
__global__ void kf_near_combine(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                                const int32_t *__restrict__ mask, int out) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  if (!d.npart) return;  // not a log-kernel FMM system
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  if (i >= d.n) return;
  const cptr<double> p = ro((const double *)d.npart);
  const double s = (p[i] + p[d.n + i]) + (p[2 * d.n + i] + p[3 * d.n + i]);
  d.v[out][i] += 0.5 * s;
}

__global__ void kf_copy(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                        const int32_t *__restrict__ mask, int dst, int src) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  if (i < d.n) d.v[dst][i] = d.v[src][i];
}

// y = a x + b y
__global__ void kf_axpby(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                         const int32_t *__restrict__ mask, int y, int x, double a, double b) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  if (i < d.n) d.v[y][i] = a * d.v[x][i] + b * d.v[y][i];
}

// dst = sign_k * src
__global__ void kf_scale_sign(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                              const int32_t *__restrict__ mask, int dst, int src) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  if (i < d.n) d.v[dst][i] = (double)d.sign * d.v[src][i];
}

// v -= Q c, c = sc[SC_PROJ ..]
__global__ void kf_sub_Qc(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                          const int32_t *__restrict__ mask, int slot) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  if (i >= d.n) return;
  const cptr<double> Q = ro(d.Q);
  double s = 0.0;
  for (int j = 0; j < d.S; ++j) s += Q[(int64_t)j * d.n + i] * d.sc[SC_PROJ + j];
  rw(d.v[slot])[i] -= s;
}

// p = z + (rho_new / rho) p
__global__ void kf_pcg_p(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                         const int32_t *__restrict__ mask) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  const double beta = d.sc[SC_RHO_NEW] / d.sc[SC_RHO];
  if (i < d.n) d.v[V_P][i] = d.v[V_Z][i] + beta * d.v[V_P][i];
}

// ------------------------------------------------------------------ reductions
// Partial sums over the system's nbdot blocks (grid stride nbdot * 256).
// mode 0: one dot v[a].v[b]; mode 1: S dots Q_t.v[b].
template <int ND>
__global__ void kf_dot(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                       const int32_t *__restrict__ mask, int mode, int a, int b) {
  __shared__ double sh[kBlock / 64];
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = mode == 0 ? 1 : d.S;
  const int nb = d.nbdot;
  const cptr<double> vb = ro(d.v[b]), va = ro(d.v[a]), Q = ro(d.Q);
  double acc[ND];
#pragma unroll
  for (int t = 0; t < ND; ++t) acc[t] = 0.0;
  // four strided elements per step, loaded before they are summed (each
  // partial still adds its elements in index order)
  const int64_t st = (int64_t)nb * kBlock;
  int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  for (; i + 3 * st < d.n; i += 4 * st) {
    double bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) bv[u] = vb[i + u * st];
    if (mode == 0) {
      double av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = va[i + u * st];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[0] += av[u] * bv[u];
    } else {
#pragma unroll
      for (int t = 0; t < ND; ++t)
        if (t < nd) {
          double qv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) qv[u] = Q[(int64_t)t * d.n + i + u * st];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[t] += qv[u] * bv[u];
        }
    }
  }
  for (; i < d.n; i += st) {
    const double bi = vb[i];
    if (mode == 0) {
      acc[0] += va[i] * bi;
    } else {
#pragma unroll
      for (int t = 0; t < ND; ++t)
        if (t < nd) acc[t] += Q[(int64_t)t * d.n + i] * bi;
    }
  }
  for (int t = 0; t < ND; ++t) {
    if (t >= nd) break;
    const double s = block_sum(acc[t], sh);
    if (threadIdx.x == 0) d.red[t * nb + br.blk] = s;
  }
}

// One block per system: sc[out + t] = sum of the partials of dot t, which sit
// at slot base + t of the partial buffer.
__global__ void kf_dot_final(const SysDev *__restrict__ sys, const int32_t *__restrict__ mask,
                             int mode, int out, int base = 0) {
  __shared__ double sh[kBlock / 64];
  const int sy = blockIdx.x;
  if (!mask[sy]) return;
  const SysDev &d = sys[sy];
  const int nd = mode == 0 ? 1 : d.S;
  const int nb = d.nbdot;
  for (int t = 0; t < nd; ++t) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) v += d.red[(base + t) * nb + b];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) d.sc[out + t] = s;
  }
}

// dw += alpha p, r -= alpha q, alpha = rho / (p.q); partial sums of r.r
__global__ void kf_pcg_wr(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                          const int32_t *__restrict__ mask) {
  __shared__ double sh[kBlock / 64];
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nb = d.nbdot;
  const double alpha = d.sc[SC_RHO] / d.sc[SC_PQ];
  const gptr<double> w = rw(d.v[V_DW]), r = rw(d.v[V_R]);
  const cptr<double> p = ro(d.v[V_P]), q = ro(d.v[V_Q]);
  double acc = 0.0;
  const int64_t st = (int64_t)nb * kBlock;
  int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  for (; i + 3 * st < d.n; i += 4 * st) {  // four elements' loads in flight together
    double pv[4], qv[4], rv[4], wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      pv[u] = p[i + u * st];
      qv[u] = q[i + u * st];
      rv[u] = r[i + u * st];
      wv[u] = w[i + u * st];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      w[i + u * st] = wv[u] + alpha * pv[u];
      const double ri = rv[u] - alpha * qv[u];
      r[i + u * st] = ri;
      acc += ri * ri;
    }
  }
  for (; i < d.n; i += st) {
    w[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) d.red[br.blk] = s;
}

// Slot of the partial buffer for dots taken while slots 0.. hold another
// reduction's partials (S <= 21 projection dots).
constexpr int kDotSlot = 31;

// v = g (v - Q c), c = Q^T v from the partials of kf_dot (mode 1) at slots
// 0..S-1, g = sign_k if use_sign else 1, with the partial sums of w.v at slot
// kDotSlot (finished by kf_dot_final): the projection, the sign and the next
// dot product in one pass.  Each block finishes c itself in the order of
// kf_dot_final, and the arithmetic and summation order are those of kf_sub_Qc,
// kf_scale_sign and kf_dot, so the results are bitwise theirs.
__global__ void kf_sub_Qc_dot(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                              const int32_t *__restrict__ mask, int slot, int use_sign, int w) {
  __shared__ double sh[kBlock / 64];
  __shared__ double cq[kDotSlot];
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nb = d.nbdot;
  for (int t = 0; t < d.S; ++t) {
    double c = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) c += d.red[t * nb + b];
    const double cs = block_sum(c, sh);
    if (threadIdx.x == 0) cq[t] = cs;
  }
  __syncthreads();
  const cptr<double> Q = ro(d.Q), ww = ro(d.v[w]);
  const gptr<double> v = rw(d.v[slot]);
  const double g = use_sign ? (double)d.sign : 1.0;
  double acc = 0.0;
  const int64_t st = (int64_t)nb * kBlock;
  int64_t i = (int64_t)br.blk * kBlock + threadIdx.x;
  for (; i + 3 * st < d.n; i += 4 * st) {  // four elements' loads in flight together
    double sq[4] = {0.0, 0.0, 0.0, 0.0}, vv[4], wv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      vv[u] = v[i + u * st];
      wv[u] = ww[i + u * st];
    }
    for (int j = 0; j < d.S; ++j) {
      double qv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) qv[u] = Q[(int64_t)j * d.n + i + u * st];
#pragma unroll
      for (int u = 0; u < 4; ++u) sq[u] += qv[u] * cq[j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double vi = vv[u] - sq[u];
      if (use_sign) vi = g * vi;
      v[i + u * st] = vi;
      acc += wv[u] * vi;
    }
  }
  for (; i < d.n; i += st) {
    double sq = 0.0;
    for (int j = 0; j < d.S; ++j) sq += Q[(int64_t)j * d.n + i] * cq[j];
    double vi = v[i] - sq;
    if (use_sign) vi = g * vi;
    v[i] = vi;
    acc += ww[i] * vi;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) d.red[kDotSlot * nb + br.blk] = s;
}

__global__ void kf_sc_copy(const SysDev *__restrict__ sys, const int32_t *__restrict__ mask,
                           int nsys, int dst, int src) {
  const int sy = blockIdx.x * blockDim.x + threadIdx.x;
  if (sy >= nsys || !mask[sy]) return;
  sys[sy].sc[dst] = sys[sy].sc[src];
}

__global__ void kf_read_sc(const SysDev *__restrict__ sys, int nsys, int off, int cnt,
                           double *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nsys * cnt) return;
  const int sy = t / cnt, i = t % cnt;
  out[sy * 8 + i] = sys[sy].sc[off + i];
}

// ------------------------------------------------------------------ preconditioner
// yv = U~^T r: row j holds 1/c_j at j and -lambda/c_j at sigma(j).  A group of
// 32 lanes takes eight consecutive rows (a work item is 64 rows: eight groups
// per block), reading each row's node-major entries coalesced and summing
// them with a fixed butterfly.  Systems without a factor copy r.
constexpr int kPcRows = 8;  // rows per 32-lane group

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, CTRL, ROWS, 0xF, false);
}

// Sum over each 32-lane half of the wavefront by DPP row operations (no LDS):
// pairs, quads, half rows, rows, then row 0 (2) into row 1 (3).  The sum is
// valid in lanes 16..31 of each half.
__device__ __forceinline__ double half_sum(double v) {
  v += dpp_f64<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);       // row_half_mirror
  v += dpp_f64<0x140>(v);       // row_mirror
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  return v;
}

// yv = U^T r over the forward factor in column-major (ELL) layout: one lane
// per row, the m entries of row j at s*n + j, so a wavefront's loads of one
// slot are contiguous; 64 rows per block (8 * kPcRows).
__global__ __launch_bounds__(256) void kf_apply_ut(const SysDev *__restrict__ sys,
                                                   const BlkRef *__restrict__ tab, int64_t ntab,
                                                   const int32_t *__restrict__ mask, int rs,
                                                   int ys) {
  // four 64-row blocks per workgroup, one per wavefront (wave-uniform index)
  const int64_t item = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * 4 +
                       __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (item >= ntab) return;
  const BlkRef br = tab[item];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t j = (int64_t)br.blk * 64 + (threadIdx.x & 63);
  if (j >= d.n) return;
  const cptr<double> rr = ro(d.v[rs]);
  const gptr<double> yv = rw(d.v[ys]);
  if (!d.has_pc) {
    yv[j] = rr[j];
    return;
  }
  const int m = d.m;
  const int64_t n = d.n;
  const cptr<int32_t> nbr = ro(d.nbr);
  const cptr<double> coef = ro(d.coef), dinv = ro(d.dinv);
  double acc = dinv[j] * rr[j];
  // slots in batches of sixteen, the last one padded: the indices and
  // coefficients first, then the sixteen gathers (all in flight together),
  // then the sums in slot order
  for (int sl = 0; sl < m; sl += 16) {
    int q[16];
    double c[16], v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const bool in = sl + u < m;
      q[u] = in ? nbr[(sl + u) * n + j] : -1;
      c[u] = in ? coef[(sl + u) * n + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = rr[q[u] >= 0 ? q[u] : j];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (q[u] >= 0) acc = fma(c[u], v[u], acc);
  }
  yv[j] = acc;
}

// z = U~ yv: row gather of the transposed factor (CSR by row), kApplyLanes
// lanes per row (rows average m entries), 64 rows per block.
constexpr int kApplyLanes = 16;

template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
  v += dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);  // quad_perm [2,3,0,1]
  if constexpr (LPR >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
  if constexpr (LPR >= 16) v += dpp_f64<0x140>(v);  // row_mirror
  if constexpr (LPR >= 32) v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  return v;
}

__global__ __launch_bounds__(256) void kf_apply_u(const SysDev *__restrict__ sys,
                                                  const BlkRef *__restrict__ tab,
                                                  const int32_t *__restrict__ mask, int ys,
                                                  int zs) {
  constexpr int LPR = kApplyLanes, RPG = LPR / 4;  // rows per lane group
  const BlkRef br = tab[xcd_remap(blockIdx.x, gridDim.x)];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int64_t i0 = ((int64_t)br.blk * (256 / LPR) + threadIdx.x / LPR) * RPG;
  const int g = threadIdx.x % LPR;
  const int wl = LPR == 32 ? 31 : 0;  // lane holding the group's sum
  const cptr<double> yy = ro(d.v[ys]);
  const gptr<double> z = rw(d.v[zs]);
  if (!d.has_pc) {
    for (int i = 0; i < RPG; ++i)
      if (g == 0 && i0 + i < d.n) z[i0 + i] = yy[i0 + i];
    return;
  }
  const cptr<int32_t> tstart = ro(d.tstart), tidx = ro(d.tidx);
  const cptr<double> tcoef = ro(d.tcoef), dinv = ro(d.dinv);
  // the group's RPG rows advance together, so each lane keeps RPG
  // independent gathers in flight (each row's sum keeps its order)
  int b[RPG], e[RPG];
  int len = 0;
#pragma unroll
  for (int k = 0; k < RPG; ++k) {
    const bool in = i0 + k < d.n;
    b[k] = in ? tstart[i0 + k] : 0;
    e[k] = in ? tstart[i0 + k + 1] : 0;
    len = max(len, e[k] - b[k]);
  }
  double acc[RPG], dg[RPG];
#pragma unroll
  for (int k = 0; k < RPG; ++k) {
    acc[k] = 0.0;
    // the diagonal term, loaded before the gathers (it does not depend on them)
    dg[k] = i0 + k < d.n ? dinv[i0 + k] * yy[i0 + k] : 0.0;
  }
  // two entries of each of the RPG rows per step: 2 x RPG independent
  // gathers in flight per lane, each row still summed in entry order
  for (int o = g; o < len; o += 2 * LPR) {
    int ti[2][RPG];
    double tc[2][RPG], yv[2][RPG];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < RPG; ++k) {
        const int idx = b[k] + o + h * LPR;
        const bool in = idx < e[k];
        ti[h][k] = in ? tidx[idx] : -1;
        tc[h][k] = in ? tcoef[idx] : 0.0;
      }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < RPG; ++k) yv[h][k] = ti[h][k] >= 0 ? yy[ti[h][k]] : 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < RPG; ++k)
        if (ti[h][k] >= 0) acc[k] += tc[h][k] * yv[h][k];
  }
#pragma unroll
  for (int k = 0; k < RPG; ++k) {
    const int64_t i = i0 + k;
    const double sum = group_sum<LPR>(acc[k]);
    if (i < d.n && g == wl) z[i] = dg[k] + sum;
  }
}

__global__ void k_gather_one(const double *__restrict__ src, const int32_t *__restrict__ order,
                             int64_t n, double *__restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) dst[i] = src[order[i]];
}

__global__ void k_scatter_one(const double *__restrict__ src, const int32_t *__restrict__ order,
                              int64_t n, double *__restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) dst[order[i]] = src[i];
}

// The host copy stays alive with the forest, so the copy needs no wait.
// A work table joins the forest's host table block (at a 256-byte boundary);
// its device address is set when build_forest uploads the block.
Tab upload_tab(Forest &F, std::vector<BlkRef> &&h, hipStream_t s) {
  (void)s;
  Tab t;
  t.count = (int64_t)h.size();
  t.off = (int64_t)((F.htab.size() + 31) & ~(size_t)31);
  F.htab.resize((size_t)t.off);
  F.htab.insert(F.htab.end(), h.begin(), h.end());
  return t;
}

}  // namespace

namespace {
thread_local int t_warm = 0;
}

bool launches_suppressed() { return t_warm > 0; }
WarmTables::WarmTables() { ++t_warm; }
WarmTables::~WarmTables() { --t_warm; }

void SysWork::release() {
  dfree(mp);
  dfree(loc);
  for (auto &p : v) dfree(p);
  dfree(red);
  dfree(sc);
  dfree(dpart);
  dfree(t32);
  t32 = nullptr;
  dfree(npart);
  npart = nullptr;
  mp = loc = nullptr;
  for (auto &p : v) p = nullptr;
  red = sc = nullptr;
  dpart = nullptr;
  dpart_cap = 0;
}

void alloc_syswork(SysWork &w, const Plan &pl) {
  try {
    w.mp = dmalloc<char>(pl.exp_bytes);
    w.loc = dmalloc<char>(pl.exp_bytes);
    for (auto &p : w.v) p = dmalloc<double>(pl.n);
    w.red = dmalloc<double>((size_t)dot_blocks(pl.n) * 32);
    w.sc = dmalloc<double>(kSysScal);
    if (pl.direct) {
      w.dpart_cap = direct_scratch_doubles(pl.n, pl.n);
      if (w.dpart_cap > 0) w.dpart = dmalloc<double>(w.dpart_cap);
    } else {
      w.t32 = dmalloc<float>(std::max<int64_t>(pl.n, 1));
      if (pl.core_log) w.npart = dmalloc<double>(4 * std::max<int64_t>(pl.n, 1));
    }
  } catch (...) {
    w.release();
    throw;
  }
}

SysDev make_sysdev(const Plan &pl, const SysWork &w) {
  SysDev d;
  std::memset(&d, 0, sizeof(d));
  d.x = pl.x;
  d.y = pl.y;
  d.ux = pl.ux;
  d.uy = pl.uy;
  d.xy2 = pl.xy2;
  d.leaf_start = pl.tree.leaf_start;
  d.order = pl.order;
  d.Q = pl.Q;
  d.nbr = pl.pc_nbr;
  d.coef = pl.pc_coef;
  d.dinv = pl.pc_dinv;
  d.tstart = pl.pc_tstart;
  d.tidx = pl.pc_tidx;
  d.tcoef = pl.pc_tcoef;
  d.mp = w.mp;
  d.loc = w.loc;
  for (int i = 0; i < kSysVecs; ++i) d.v[i] = w.v[i];
  d.red = w.red;
  d.sc = w.sc;
  d.t32 = w.t32;
  d.npart = w.npart;
  d.n = pl.n;
  d.h = pl.tree.h;
  d.S = pl.S;
  d.L = pl.tree.L;
  d.k = pl.k;
  d.R = pl.R;
  d.sign = pl.sign;
  d.nbdot = dot_blocks(pl.n);
  d.m = pl.m;
  d.has_pc = pl.has_pc ? 1 : 0;
  return d;
}

Forest::~Forest() {
  bool graphs = false;
  for (auto &g : graph) graphs = graphs || g;
  if (graphs) {
    (void)hipDeviceSynchronize();  // no replay may still be running
    for (auto &g : graph)
      if (g) (void)hipGraphExecDestroy(g);
  }
  if (cap) (void)hipStreamDestroy(cap);
  dfree(dsys);
  for (int i = 0; i < kMasks; ++i) {
    if (mask_ev[i]) {
      (void)hipEventSynchronize(mask_ev[i]);
      (void)hipEventDestroy(mask_ev[i]);
    }
    mask[i] = nullptr;
  }
  dfree(mask_block);
  mask_block = nullptr;
  if (hpin) (void)hipHostFree(hpin);
  dfree(tab_block);
}

void build_forest(Forest &F, const std::vector<Plan *> &plans, const std::vector<SysWork *> &work,
                  hipStream_t s) {
  F.plan = plans;
  F.work = work;
  F.nsys = (int)plans.size();
  F.hsys.resize(F.nsys);
  F.maxS = 1;
  F.maxL_log = F.maxL_dist = 0;
  std::vector<BlkRef> hv, hd, hp;
  for (int i = 0; i < F.nsys; ++i) {
    const Plan &pl = *plans[i];
    F.hsys[i] = make_sysdev(pl, *work[i]);
    F.maxS = std::max(F.maxS, pl.S);
    if (pl.S >= kDotSlot)  // the projection's partials must not reach kDotSlot
      throw Error{PHS_ERR_INVALID_ARGUMENT, "polynomial space too large for the PCG reductions"};
    if (pl.direct) F.any_direct = true;
    else if (pl.core_log) F.maxL_log = std::max(F.maxL_log, pl.tree.L);
    else F.maxL_dist = std::max(F.maxL_dist, pl.tree.L);
    const int64_t nv = (pl.n + kBlock - 1) / kBlock;
    for (int64_t b = 0; b < nv; ++b) hv.push_back({i, (int32_t)b});
    for (int b = 0; b < dot_blocks(pl.n); ++b) hd.push_back({i, b});
    const int64_t np = (pl.n + 8 * kPcRows - 1) / (8 * kPcRows);
    for (int64_t b = 0; b < np; ++b) hp.push_back({i, (int32_t)b});
  }
  F.dsys = dmalloc<SysDev>(F.nsys);
  PHS_HIP(hipMemcpyAsync(F.dsys, F.hsys.data(), F.nsys * sizeof(SysDev), hipMemcpyHostToDevice,
                         s));
  {
    const size_t mb = ((size_t)F.nsys * sizeof(int32_t) + 63) / 64 * 64;
    PHS_HIP(hipHostMalloc(&F.hpin, mb * Forest::kMasks + (size_t)F.nsys * 8 * sizeof(double), 0));
    for (int i = 0; i < Forest::kMasks; ++i)
      F.hmask[i] = (int32_t *)((char *)F.hpin + mb * i);
    F.hgsc = (double *)((char *)F.hpin + mb * Forest::kMasks);
  }
  {
    // all masks in one device block laid out like the pinned staging, one copy
    const size_t mw = ((size_t)F.nsys * sizeof(int32_t) + 63) / 64 * 16;  // ints per mask
    F.mask_block = dmalloc<int32_t>(mw * Forest::kMasks);
    for (int i = 0; i < Forest::kMasks; ++i) {
      F.mask[i] = F.mask_block + mw * i;
      for (int j = 0; j < F.nsys; ++j) F.hmask[i][j] = 1;
    }
    PHS_HIP(hipMemcpyAsync(F.mask_block, F.hmask[0], mw * Forest::kMasks * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    for (int i = 0; i < Forest::kMasks; ++i) {
      PHS_HIP(hipEventCreateWithFlags(&F.mask_ev[i], hipEventDisableTiming));
      PHS_HIP(hipEventRecord(F.mask_ev[i], s));
      F.mask_pending[i] = true;
    }
  }
  F.vec = upload_tab(F, std::move(hv), s);
  F.dot = upload_tab(F, std::move(hd), s);
  F.pc = upload_tab(F, std::move(hp), s);
  // Every FMM work table a later call can look up: the matvec in each
  // precision and, on a plan's own forest, the expansions of the evaluation.
  // The drivers run with their launches suppressed, so this only builds and
  // uploads tables; afterwards a lookup miss is an error, never an allocation.
  {
    WarmTables warm;
    for (int prec : {(int)PHS_FP64, (int)PHS_MIXED, (int)PHS_NEAR32, PHS_FP64_EVAL})
      f_matvec(F, F.mask[0], V_IN, V_OUT, prec, s);
    for (Plan *pl : plans) {
      if (pl->self != &F || pl->direct) continue;
      if (pl->core_log) log_expansions(*pl, V_IN, s);
      else dist_expansions(*pl, V_IN, s);
    }
  }
  // all tables in one allocation and one copy
  F.tab_block = dmalloc<BlkRef>(std::max<size_t>(F.htab.size(), 1));
  if (!F.htab.empty())
    PHS_HIP(hipMemcpyAsync(F.tab_block, F.htab.data(), F.htab.size() * sizeof(BlkRef),
                           hipMemcpyHostToDevice, s));
  for (Tab *t : {&F.vec, &F.dot, &F.pc}) t->d = F.tab_block + t->off;
  for (auto &kv : F.cache) kv.second.d = F.tab_block + kv.second.off;
  F.frozen = true;
}

void refresh_forest(Forest &F, hipStream_t s) {
  for (int i = 0; i < F.nsys; ++i) F.hsys[i] = make_sysdev(*F.plan[i], *F.work[i]);
  PHS_HIP(hipMemcpyAsync(F.dsys, F.hsys.data(), F.nsys * sizeof(SysDev), hipMemcpyHostToDevice,
                         s));
  PHS_HIP(hipStreamSynchronize(s));
}

void sync_forest_pc(Forest &F, hipStream_t s) {
  for (int i = 0; i < F.nsys; ++i) {
    const Plan &pl = *F.plan[i];
    const SysDev &d = F.hsys[i];
    if (d.has_pc != (pl.has_pc ? 1 : 0) || d.m != pl.m || d.nbr != pl.pc_nbr ||
        d.coef != pl.pc_coef || d.dinv != pl.pc_dinv || d.tstart != pl.pc_tstart ||
        d.tidx != pl.pc_tidx || d.tcoef != pl.pc_tcoef) {
      refresh_forest(F, s);
      return;
    }
  }
}

uint64_t tab_key(int kind, int K, int P, int level) {
  return ((uint64_t)kind << 40) | ((uint64_t)K << 32) | ((uint64_t)P << 8) | (uint64_t)level;
}

void set_mask(Forest &F, int i, const std::vector<int32_t> &m, hipStream_t s) {
  if (std::equal(m.begin(), m.end(), F.hmask[i])) return;
  if (F.mask_pending[i]) PHS_HIP(hipEventSynchronize(F.mask_ev[i]));
  std::copy(m.begin(), m.end(), F.hmask[i]);
  PHS_HIP(hipMemcpyAsync(F.mask[i], F.hmask[i], F.nsys * sizeof(int32_t), hipMemcpyHostToDevice,
                         s));
  PHS_HIP(hipEventRecord(F.mask_ev[i], s));
  F.mask_pending[i] = true;
}

// ------------------------------------------------------------------ launchers
#define F_GRID(tab) (unsigned)(tab).count

void f_fill(Forest &F, const int32_t *mask, int slot, double a, hipStream_t s) {
  PHS_LAUNCH("fill", s, kf_fill<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask, slot, a));
}

void f_copy(Forest &F, const int32_t *mask, int dst, int src, hipStream_t s) {
  PHS_LAUNCH("copy", s, kf_copy<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask, dst, src));
}

void f_axpby(Forest &F, const int32_t *mask, int y, int x, double a, double b, hipStream_t s) {
  PHS_LAUNCH("axpby", s,
             kf_axpby<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask, y, x, a, b));
}

void f_scale_sign(Forest &F, const int32_t *mask, int dst, int src, hipStream_t s) {
  PHS_LAUNCH("scale_sign", s,
             kf_scale_sign<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask, dst, src));
}

static void dot_partials(Forest &F, const int32_t *mask, int mode, int a, int b,
                         hipStream_t s) {
  const int nd = mode == 0 ? 1 : F.maxS;
  if (nd <= 1)
    PHS_LAUNCH("dot", s, kf_dot<1><<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask, mode, a, b));
  else if (nd <= 8)
    PHS_LAUNCH("dot", s, kf_dot<8><<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask, mode, a, b));
  else
    PHS_LAUNCH("dot", s, kf_dot<32><<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask, mode, a, b));
}

static void dot_launch(Forest &F, const int32_t *mask, int mode, int a, int b, int out,
                       hipStream_t s) {
  const int nd = mode == 0 ? 1 : F.maxS;
  if (nd <= 1)
    PHS_LAUNCH("dot", s, kf_dot<1><<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask, mode, a, b));
  else if (nd <= 8)
    PHS_LAUNCH("dot", s, kf_dot<8><<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask, mode, a, b));
  else
    PHS_LAUNCH("dot", s, kf_dot<32><<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask, mode, a, b));
  PHS_LAUNCH("dot_final", s,
             kf_dot_final<<<(unsigned)F.nsys, kBlock, 0, s>>>(F.dsys, mask, mode, out));
}

void f_dot(Forest &F, const int32_t *mask, int a, int b, int out, hipStream_t s) {
  dot_launch(F, mask, 0, a, b, out, s);
}

void f_qt(Forest &F, const int32_t *mask, int slot, int out, hipStream_t s) {
  dot_launch(F, mask, 1, 0, slot, out, s);
}

void f_project(Forest &F, const int32_t *mask, int slot, hipStream_t s) {
  dot_launch(F, mask, 1, 0, slot, SC_PROJ, s);
  PHS_LAUNCH("project", s,
             kf_sub_Qc<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask, slot));
}

void f_project_dot(Forest &F, const int32_t *mask, int slot, bool sign, int w, int out,
                   hipStream_t s) {
  dot_partials(F, mask, 1, 0, slot, s);  // Q^T v, finished inside kf_sub_Qc_dot
  PHS_LAUNCH("project_dot", s,
             kf_sub_Qc_dot<<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask, slot,
                                                            sign ? 1 : 0, w));
  PHS_LAUNCH("dot_final", s,
             kf_dot_final<<<(unsigned)F.nsys, kBlock, 0, s>>>(F.dsys, mask, 0, out, kDotSlot));
}

void f_pcg_wr(Forest &F, const int32_t *mask, hipStream_t s) {
  PHS_LAUNCH("pcg_wr", s, kf_pcg_wr<<<F_GRID(F.dot), kBlock, 0, s>>>(F.dsys, F.dot.d, mask));
  PHS_LAUNCH("dot_final", s,
             kf_dot_final<<<(unsigned)F.nsys, kBlock, 0, s>>>(F.dsys, mask, 0, SC_RR));
}

void f_pcg_p(Forest &F, const int32_t *mask, hipStream_t s) {
  PHS_LAUNCH("pcg_p", s, kf_pcg_p<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask));
}

void f_sc_copy(Forest &F, const int32_t *mask, int dst, int src, hipStream_t s) {
  PHS_LAUNCH("sc_copy", s,
             kf_sc_copy<<<(F.nsys + 63) / 64, 64, 0, s>>>(F.dsys, mask, F.nsys, dst, src));
}

// The gather writes straight into the pinned host block (device-accessible),
// so the readback needs no copy: the kernel's completion and the stream
// synchronisation make the values visible to the host.
void f_read_scalars_launch(Forest &F, int off, int cnt, hipStream_t s) {
  const int tot = F.nsys * cnt;
  PHS_LAUNCH("read_sc", s,
             kf_read_sc<<<(tot + 255) / 256, 256, 0, s>>>(F.dsys, F.nsys, off, cnt, F.hgsc));
}

void f_read_scalars(Forest &F, int off, int cnt, hipStream_t s) {
  f_read_scalars_launch(F, off, cnt, s);
  PHS_HIP(hipStreamSynchronize(s));
}

void f_run(Forest &F, int key, hipStream_t s, const std::function<void(hipStream_t)> &fn) {
  PHS_REQUIRE(key >= 0 && key < Forest::kGraphs, PHS_ERR_INVALID_ARGUMENT, "graph key");
  if (!graphs_enabled() || profiling_on() || launches_suppressed()) {
    fn(s);
    return;
  }
  if (!F.graph[key]) {
    if (++F.graph_runs[key] < 2) {  // a sequence that runs once is not worth a capture
      fn(s);
      return;
    }
    if (!F.cap) PHS_HIP(hipStreamCreateWithFlags(&F.cap, hipStreamNonBlocking));
    PHS_HIP(hipStreamBeginCapture(F.cap, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      fn(F.cap);
    } catch (...) {
      (void)hipStreamEndCapture(F.cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    PHS_HIP(hipStreamEndCapture(F.cap, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    PHS_HIP(e);
    F.graph[key] = ex;
  }
  PHS_HIP(hipGraphLaunch(F.graph[key], s));
}

void f_precond_apply(Forest &F, const int32_t *mask, int r, int z, int tmp, hipStream_t s) {
  PHS_LAUNCH("precond_ut", s,
             kf_apply_ut<<<(unsigned)((F.pc.count + 3) / 4), 256, 0, s>>>(F.dsys, F.pc.d,
                                                                        F.pc.count, mask, r,
                                                                        tmp));
  PHS_LAUNCH("precond_u", s,
             kf_apply_u<<<F_GRID(F.pc), 256, 0, s>>>(F.dsys, F.pc.d, mask, tmp, z));
}

void f_precond(Forest &F, const int32_t *mask, int r, int z, int tmp, hipStream_t s) {
  f_precond_apply(F, mask, r, z, tmp, s);
  f_project(F, mask, z, s);
}

void f_precond_dot(Forest &F, const int32_t *mask, int r, int z, int tmp, int out,
                   hipStream_t s) {
  f_precond_apply(F, mask, r, z, tmp, s);
  f_project_dot(F, mask, z, false, r, out, s);
}

void f_gather_user(Forest &F, int sys, const double *src_user, int slot, hipStream_t s) {
  const SysDev &d = F.hsys[sys];
  PHS_LAUNCH("gather", s,
             k_gather_one<<<(unsigned)((d.n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
                 src_user, d.order, d.n, d.v[slot]));
}

void f_scatter_user(Forest &F, int sys, int slot, double *dst_user, hipStream_t s) {
  const SysDev &d = F.hsys[sys];
  PHS_LAUNCH("scatter", s,
             k_scatter_one<<<(unsigned)((d.n + kBlock - 1) / kBlock), kBlock, 0, s>>>(
                 d.v[slot], d.order, d.n, dst_user));
}

void f_near_combine(Forest &F, const int32_t *mask, int out, hipStream_t s) {
  PHS_LAUNCH("near_combine", s,
             kf_near_combine<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask, out));
}

void f_matvec(Forest &F, const int32_t *mask, int in, int out, int precision, hipStream_t s) {
  if ((precision == PHS_MIXED || precision == PHS_NEAR32) && F.maxL_log + F.maxL_dist > 0)
    PHS_LAUNCH("near_t32", s,
               kf_near_t32<<<F_GRID(F.vec), kBlock, 0, s>>>(F.dsys, F.vec.d, mask, in));
  if (F.maxL_log > 0) log_matvec(F, mask, in, out, precision, s);
  if (F.maxL_dist > 0) dist_matvec(F, mask, in, out, precision, s);
  if (F.any_direct) direct_matvec(F, mask, in, out, precision, s);
}

// Work-item tables of the FMM kernels, one per (kind, K, P, level), all built
// by the warm-up pass of build_forest and kept for the forest's lifetime.
Tab build_fmm_tab(Forest &F, int kind, int K, int P, int level, hipStream_t s);

Tab forest_tab(Forest &F, uint64_t key, hipStream_t s) {
  for (auto &kv : F.cache)
    if (kv.first == key) return kv.second;
  PHS_REQUIRE(!F.frozen, PHS_ERR_DEVICE,
              "internal error: an FMM work table was not built with its forest");
  const int kind = (int)(key >> 40), K = (int)((key >> 32) & 0xff),
            P = (int)((key >> 8) & 0xffffff), level = (int)(key & 0xff);
  F.cache.push_back({key, build_fmm_tab(F, kind, K, P, level, s)});
  return F.cache.back().second;
}

// kinds (low 4 bits): 1 leaf (k == K), 2 P2M groups of 4 x P leaves (k == K),
// 3 log M2M level, 4 log L2L level, 5 log M2L, 10 log M2L on the matrix
// cores (strips of 16 boxes x densities), 13 log M2M by row segments of 16
// parents x densities, 14 log L2L by row segments of 32 parents x densities;
// Chebyshev (P = Q, odd-k
// systems whose Q for the launch equals P): 6 leaf (k == K), 7 M2M level,
// 8 L2L level, 9 M2L.  Bits 4.. of a Chebyshev kind select which Q of the
// plan applies: 0 the FP64 matvec order, 1 the FP32 one, 2 the evaluation one.
int m2l_chunk(int P);

Tab build_fmm_tab(Forest &F, int kind, int K, int P, int level, hipStream_t s) {
  std::vector<BlkRef> h;
  const int tier = kind >> 4, base = kind & 15;
  // FP64 Chebyshev M2L (matrix cores): workgroups per tile
  const int rs = (base == 9 && tier != 1) ? cheb_m2l_max_split(P * P) : 1;
  for (int i = 0; i < F.nsys; ++i) {
    const Plan &pl = *F.plan[i];
    if (pl.direct) continue;  // no FMM
    const int L = pl.tree.L, R = pl.R;
    const bool log_k = pl.core_log;
    const int qsel = tier == 0 ? pl.q64 : (tier == 1 ? pl.q32 : pl.qe);
    const bool cheb = !log_k && qsel == P;
    switch (base) {
      case 1:
        if (pl.k == K)
          for (int64_t b = 0; b < boxes_at(L); ++b) h.push_back({i, (int32_t)b});
        break;
      case 2:  // P = leaves per wavefront; four wavefronts per item
        if (pl.k == K)
          for (int64_t b = 0; b < boxes_at(L) / (4 * P); ++b) h.push_back({i, (int32_t)b});
        break;
      case 3:  // M2M into level `level` from level+1
        if (log_k && L > level) {
          const int64_t tot = boxes_at(level) * R * (P + 1) * shift_split(level);
          for (int64_t b = 0; b < (tot + 255) / 256; ++b) h.push_back({i, (int32_t)b});
        }
        break;
      case 4:  // L2L into level `level` from level-1
        if (log_k && L >= level) {
          const int64_t tot = boxes_at(level) * R * (P + 1) * shift_split(level);
          for (int64_t b = 0; b < (tot + 255) / 256; ++b) h.push_back({i, (int32_t)b});
        }
        break;
      case 5:
        if (log_k) {
          int64_t tot = 0;
          for (int l = 2; l <= L; ++l) tot += boxes_at(l);
          const int64_t ntiles = (tot + 255) / 256;
          const int lch = m2l_chunk(P);
          const int64_t nch = (P + 1 + lch - 1) / lch;
          for (int64_t b = 0; b < ntiles * nch * R; ++b) h.push_back({i, (int32_t)b});
        }
        break;
      case 10:  // log M2L on the matrix cores: (strip of 16 boxes, density)
        if (log_k) {
          int64_t strips = 0;
          for (int l = 2; l <= L; ++l) {
            const int64_t half = (int64_t)1 << (l - 1);
            strips += 4 * half * ((half + 15) / 16);
          }
          for (int64_t b = 0; b < strips * R; ++b) h.push_back({i, (int32_t)b});
        }
        break;
      case 13:  // log M2M into level `level` (>= 4) by row segments of 16 parents
        if (log_k && L > level)
          for (int64_t b = 0; b < boxes_at(level) / 16 * R; ++b) h.push_back({i, (int32_t)b});
        break;
      case 14:  // log L2L into level `level` (>= 7) by row segments of 32 parents
        if (log_k && L >= level)
          for (int64_t b = 0; b < boxes_at(level - 1) / 32 * R; ++b) h.push_back({i, (int32_t)b});
        break;
      case 6:
        if (cheb && pl.k == K)
          for (int64_t b = 0; b < boxes_at(L); ++b) h.push_back({i, (int32_t)b});
        break;
      case 7:
        if (cheb && L > level)
          for (int64_t b = 0; b < boxes_at(level) * R; ++b) h.push_back({i, (int32_t)b});
        break;
      case 8:
        if (cheb && L >= level)
          for (int64_t b = 0; b < boxes_at(level) * R; ++b) h.push_back({i, (int32_t)b});
        break;
      case 9:
        if (cheb) {
          int64_t tiles = 0;
          for (int l = 2; l <= L; ++l) tiles += (boxes_at(l) * R + 63) / 64;
          // FP64 tiers: rs workgroups per tile (FP32: one)
          for (int64_t b = 0; b < tiles * rs; ++b) h.push_back({i, (int32_t)b});
        }
        break;
      default:
        throw Error{PHS_ERR_INVALID_ARGUMENT, "unknown table kind"};
    }
  }
  return upload_tab(F, std::move(h), s);
}

}  // namespace phs
