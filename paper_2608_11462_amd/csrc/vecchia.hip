// Vecchia / Matern sparse inverse-Cholesky preconditioner (paper Sec. 2.2:
// eqs. conditionals and vecchia_sumform, Fig. vecchia_chol; conditioning-set
// sizes and random ordering of Sec. 3).
//
//  1. ordering: rank order = nodes sorted by (splitmix64(seed ^ i), i), i the
//     caller index (stable LSD radix sort);
//  2. conditioning sets: sigma(j) = the min(m, rank_j) predecessors with the
//     smallest (d^2, rank), d^2 = dx*dx + dy*dy rounded exactly as written
//     (no contraction) — found by ring search in uniform grids built over the
//     rank prefixes [0, 2^t), so the predecessors of a node of rank in
//     [2^(t-1), 2^t) fill at least half of the grid it searches;
//  3. factor: per node, Cholesky of the (|sigma|+1)^2 Matern block with the
//     node last; its last row gives L^{-1} k and the conditional standard
//     deviation c, then lambda = L^{-T} (L^{-1} k); column j of U~ holds 1/c on
//     the diagonal and -lambda/c at sigma(j);
//  4. apply: z = U~ (U~^T r) as two gathers, the second through a transposed
//     copy whose rows are sorted by column, so sums are in a fixed order.
#include <cmath>

#include "fmm_common.h"

namespace phs {

namespace {

constexpr int kMaxM = 63;  // the augmented block (|sigma| + 1) fits one wavefront

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_rank_keys(int64_t n, uint64_t seed, uint64_t *keys, int32_t *vals) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = splitmix64(seed ^ (uint64_t)i);
  vals[i] = (int32_t)i;
}

__global__ void k_rank_maps(const int32_t *perm, const int32_t *inv_order, int64_t n,
                            const double *x, const double *y, int32_t *rank_tree,
                            int32_t *pos_of_rank, double *xr, double *yr) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int p = inv_order[perm[t]];
  pos_of_rank[t] = p;
  rank_tree[p] = (int32_t)t;
  xr[t] = x[p];
  yr[t] = y[p];
}

__device__ __forceinline__ int grid_cell(double v, double h, int g) {
#pragma clang fp contract(off)
  double u = (v + h) * ((double)g / (2.0 * h));
  int q = (int)floor(u);
  return q < 0 ? 0 : (q >= g ? g - 1 : q);
}

// entry e of the concatenated rank prefixes -> (level << 20 | cell, rank)
__global__ void k_grid_keys(const double *xr, const double *yr, int T,
                            const int64_t *lvl_off, const int32_t *gbits, double h,
                            int64_t total, uint32_t *keys, int32_t *vals) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  int t = 0;
  while (t < T && e >= lvl_off[t + 1]) ++t;
  const int r = (int)(e - lvl_off[t]);
  const int g = 1 << gbits[t];
  const int cx = grid_cell(xr[r], h, g), cy = grid_cell(yr[r], h, g);
  keys[e] = ((uint32_t)t << 20) | (uint32_t)(cy * g + cx);
  vals[e] = r;
}

// coordinates of the grid entries in their sorted (cell) order
__global__ void k_grid_coords(const int32_t *sorted_rank, const double *xr, const double *yr,
                              int64_t total, double2 *gxy) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= total) return;
  const int r = sorted_rank[q];
  gxy[q] = make_double2(xr[r], yr[r]);
}

__global__ void k_cell_start(const uint32_t *keys, int64_t total, int T, const int32_t *gbits,
                             const int64_t *cell_off, int64_t ncells_total, int32_t *start) {
  int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= ncells_total) return;
  int t = 0;
  while (t < T && q >= cell_off[t + 1]) ++t;
  const uint32_t c = (uint32_t)(q - cell_off[t]);
  const uint32_t key = ((uint32_t)t << 20) | c;
  int64_t lo = 0, hi = total;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  start[q] = (int32_t)lo;
}

__device__ __forceinline__ bool lessp(double da, int ra, double db, int rb) {
  return da < db || (da == db && ra < rb);
}

// Query order of the KNN: the ranks grouped by the grid level their search
// uses (lv = bit length of the rank, at most T), in tree order within a level,
// so a wavefront's queries share one grid and search neighbouring cells (rank
// order is random in space).  Keys per tree position p: lv(rank(p)), value
// rank(p); a stable sort by key gives the order.
__global__ void k_qkeys(const int32_t *__restrict__ rank, int64_t n, int T, uint32_t *keys,
                        int32_t *vals) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int t = rank[p];
  int lv = 64 - __clzll((unsigned long long)t);
  if (lv > T) lv = T;
  keys[p] = (uint32_t)lv;
  vals[p] = t;
}

// Squared distance with each product rounded, then the sum: no fused
// multiply-add, so d^2 is symmetric in (dx, dy) and identical to the CPU
// reference.
__device__ __forceinline__ double sq_dist(double ax, double ay, double qx, double qy) {
#pragma clang fp contract(off)
  const double dx = ax - qx;
  const double dy = ay - qy;
  return dx * dx + dy * dy;
}

// Lane exchanges within a 16-lane group (one DPP row): xor 1, 2, 8 and the
// mirrors of 4, 8 and 16 lanes by DPP, xor 4 by a swizzle.
constexpr int kX1 = 0xB1, kX2 = 0x4E, kX4 = -1, kX8 = 0x128;
constexpr int kM4 = 0x1B, kM8 = 0x141, kM16 = 0x140;

template <int C>
__device__ __forceinline__ int xchg_i(int v) {
  if constexpr (C == kX4) return __builtin_amdgcn_ds_swizzle(v, 0x101F);  // and 31, xor 4
  else return __builtin_amdgcn_update_dpp(0, v, C, 0xF, 0xF, false);
}
template <int C>
__device__ __forceinline__ double xchg_d(double v) {
  return __hiloint2double(xchg_i<C>(__double2hiint(v)), xchg_i<C>(__double2loint(v)));
}

// Compare-exchange of the key (d, r) with the partner lane's: this lane keeps
// the smaller key if keep_min, else the larger.  Keys are unique but for the
// empty key (+inf, INT_MAX), whose copies are interchangeable.
template <int C>
__device__ __forceinline__ void cmp_xchg(double &d, int &r, bool keep_min) {
  const double pd = xchg_d<C>(d);
  const int pr = xchg_i<C>(r);
  const bool pless = lessp(pd, pr, d, r);
  if (keep_min == pless) {
    d = pd;
    r = pr;
  }
}

// Ascending sort of one key per lane over a 16-lane group: bitonic merges of
// 2, 4, 8, 16 keys, each a flip (lane against its mirror in the block) and
// half-cleaners.
__device__ __forceinline__ void sort16(double &d, int &r, int li) {
  cmp_xchg<kX1>(d, r, !(li & 1));
  cmp_xchg<kM4>(d, r, !(li & 2));
  cmp_xchg<kX1>(d, r, !(li & 1));
  cmp_xchg<kM8>(d, r, !(li & 4));
  cmp_xchg<kX2>(d, r, !(li & 2));
  cmp_xchg<kX1>(d, r, !(li & 1));
  cmp_xchg<kM16>(d, r, !(li & 8));
  cmp_xchg<kX4>(d, r, !(li & 4));
  cmp_xchg<kX2>(d, r, !(li & 2));
  cmp_xchg<kX1>(d, r, !(li & 1));
}

// The 16E smallest of a sorted list (entry e*16 + li in Ld[e], Lr[e]) and 16
// sorted keys (one per lane): the list against the keys reversed and padded
// with empty keys below them, the smaller of each pair, is a bitonic sequence
// of the 16E smallest; half-cleaners sort it.
template <int E>
__device__ __forceinline__ void merge16(double (&Ld)[E], int (&Lr)[E], double d, int r, int li) {
  const double md = xchg_d<kM16>(d);
  const int mr = xchg_i<kM16>(r);
  if (lessp(md, mr, Ld[E - 1], Lr[E - 1])) {
    Ld[E - 1] = md;
    Lr[E - 1] = mr;
  }
#pragma unroll
  for (int D = E / 2; D >= 1; D /= 2)  // distances 16 D, within a lane
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (!(e & D) && lessp(Ld[e + D], Lr[e + D], Ld[e], Lr[e])) {
        const double td = Ld[e];
        const int tr = Lr[e];
        Ld[e] = Ld[e + D];
        Lr[e] = Lr[e + D];
        Ld[e + D] = td;
        Lr[e + D] = tr;
      }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    cmp_xchg<kX8>(Ld[e], Lr[e], !(li & 8));
    cmp_xchg<kX4>(Ld[e], Lr[e], !(li & 4));
    cmp_xchg<kX2>(Ld[e], Lr[e], !(li & 2));
    cmp_xchg<kX1>(Ld[e], Lr[e], !(li & 1));
  }
}

// Ordered nearest predecessors: sigma(j) = the K = min(m, rank) predecessors
// with the smallest (d^2, rank).  A group of 16 lanes takes one query (four
// per wavefront, in the order above) and keeps its list sorted across its
// lanes, 16E entries (16E >= m).  Rings of cells around the query's cell are
// searched outwards: the group's lanes take 16 cells of a ring at a time
// (cells that cannot hold a key below the K-th kept one are skipped once the
// list holds K), a prefix sum over the cells' entry counts numbers their
// entries, and the entries go in chunks of 16, one per lane.  A chunk with a
// predecessor below the K-th kept key (any predecessor while the list holds
// fewer than K) is sorted and merged into the list.  The search stops when
// the ring just searched bounds every unsearched cell beyond the K-th key.
// The comparisons are exact, so the lists are those of the definition,
// whatever the order the cells are visited in.
template <int E>
__global__ __launch_bounds__(256) void k_knn(const double *xr, const double *yr, int64_t n,
                                             int m, int T, double h, const int32_t *gbits,
                                             const int64_t *cell_off, const int32_t *cell_start,
                                             const int32_t *sorted_rank,
                                             const double2 *__restrict__ gxy,
                                             const int32_t *pos_of_rank,
                                             const int32_t *__restrict__ qord, int32_t *nbr,
                                             int32_t *cnt_out) {
  // per lane: start and exclusive entry prefix of the cell it took
  __shared__ int s_b[256], s_x[256];
  const int lane = threadIdx.x & 63, li = lane & 15;
  const int gl = lane & 48;            // the group's first lane in the wavefront
  const int gt = threadIdx.x & ~15;    // ... and its first thread in the block
  const int64_t qi = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const bool live = qi < n;
  int64_t t = 0;
  int K = 0, p = 0, g = 1, cqx = 0, cqy = 0, maxR = 0;
  double cw = 1.0, qx = 0.0, qy = 0.0;
  const int32_t *cs = cell_start;
  if (live) {
    t = qord[qi];
    K = (int)(t < m ? t : m);
    p = pos_of_rank[t];
    int lv = 64 - __clzll((unsigned long long)t);  // smallest lv with 2^lv >= t+1
    if (lv > T) lv = T;
    g = 1 << gbits[lv];
    cw = 2.0 * h / g;
    qx = xr[t];
    qy = yr[t];
    cqx = grid_cell(qx, h, g);
    cqy = grid_cell(qy, h, g);
    cs = cell_start + cell_off[lv];
    maxR = max(max(cqx, g - 1 - cqx), max(cqy, g - 1 - cqy));
  }
  double Ld[E];
  int Lr[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    Ld[e] = INFINITY;
    Lr[e] = 0x7fffffff;
  }
  int seen = 0;  // predecessors offered to the list (the group's count)
  double wd2 = INFINITY;  // the K-th kept key once seen >= K
  int wrk = 0x7fffffff;
  bool done = !live || K == 0;
  for (int R = 0;; ++R) {
    if (!done) {
      const int ncells = R == 0 ? 1 : 8 * R;
      for (int cb = 0; cb < ncells; cb += 16) {
        // the ring's cells: the row below (2R+1), the row above (2R+1), then
        // the two side columns in between
        const int ci = cb + li;
        int cx = cqx, cy = cqy;
        if (R > 0) {
          if (ci < 2 * R + 1) {
            cx = cqx - R + ci;
            cy = cqy - R;
          } else if (ci < 4 * R + 2) {
            cx = cqx - R + (ci - 2 * R - 1);
            cy = cqy + R;
          } else {
            const int sidx = ci - 4 * R - 2;
            cy = cqy - R + 1 + (sidx >> 1);
            cx = (sidx & 1) ? cqx + R : cqx - R;
          }
        }
        bool cv = ci < ncells && cx >= 0 && cx < g && cy >= 0 && cy < g;
        if (cv && seen >= K) {
          // skip a cell that cannot hold a point closer than the K-th kept
          // one (strictly; a tie at equal d^2 could still win on rank)
          const double lo_x = -h + cx * cw, lo_y = -h + cy * cw;
          const double ex = fmax(fmax(lo_x - qx, qx - (lo_x + cw)), 0.0);
          const double ey = fmax(fmax(lo_y - qy, qy - (lo_y + cw)), 0.0);
          cv = (ex * ex + ey * ey) * (1.0 - 1e-12) <= wd2;
        }
        int b = 0, cnt = 0;
        if (cv) {
          const int c = cy * g + cx;
          b = cs[c];
          cnt = cs[c + 1] - b;
        }
        // inclusive prefix sum of the counts over the group's 16 lanes
        int inc = cnt;
        inc += __builtin_amdgcn_update_dpp(0, inc, 0x111, 0xF, 0xF, false);  // row_shr:1
        inc += __builtin_amdgcn_update_dpp(0, inc, 0x112, 0xF, 0xF, false);  // row_shr:2
        inc += __builtin_amdgcn_update_dpp(0, inc, 0x114, 0xF, 0xF, false);  // row_shr:4
        inc += __builtin_amdgcn_update_dpp(0, inc, 0x118, 0xF, 0xF, false);  // row_shr:8
        const int total = __shfl(inc, gl + 15);
        s_b[threadIdx.x] = b;
        s_x[threadIdx.x] = inc - cnt;
        __builtin_amdgcn_wave_barrier();
        for (int j0 = 0; j0 < total; j0 += 16) {
          const int j = j0 + li;
          // the cell of entry j: the last of the group's cells whose
          // exclusive prefix is at most j (empty cells share their successor's)
          int c = 0;
#pragma unroll
          for (int st = 8; st >= 1; st >>= 1)
            if (s_x[gt + c + st] <= j) c += st;
          double d2 = INFINITY;
          int r = 0x7fffffff;
          bool valid = false;
          if (j < total) {
            const int q = s_b[gt + c] + (j - s_x[gt + c]);
            const int rq = sorted_rank[q];
            if (rq < t) {
              const double2 cxy = gxy[q];
              d2 = sq_dist(cxy.x, cxy.y, qx, qy);
              r = rq;
              valid = true;
            }
          }
          const bool better = valid && (seen < K || lessp(d2, r, wd2, wrk));
          const unsigned gv = (unsigned)(__ballot(valid) >> gl) & 0xFFFFu;
          const unsigned gb = (unsigned)(__ballot(better) >> gl) & 0xFFFFu;
          if (gb) {
            sort16(d2, r, li);
            merge16<E>(Ld, Lr, d2, r, li);
          }
          seen += __popc(gv);
          if (gb && seen >= K) {
            const int kr = (K - 1) >> 4, kl = (K - 1) & 15;
            double wv = Ld[0];
            int wr = Lr[0];
#pragma unroll
            for (int e = 1; e < E; ++e)
              if (e == kr) {
                wv = Ld[e];
                wr = Lr[e];
              }
            wd2 = __shfl(wv, gl + kl);
            wrk = __shfl(wr, gl + kl);
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      if (R >= maxR) {
        done = true;
      } else if (seen >= K && R >= 1) {
        const double bound = (double)R * cw;
        if (wd2 < bound * bound * (1.0 - 1e-12)) done = true;
      }
    }
    if (__ballot(!done) == 0) break;
  }
  if (!live) return;
  const int cnt = seen < K ? seen : K;
  if (li == 0) cnt_out[p] = cnt;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int s = e * 16 + li;
    if (s < m) nbr[(int64_t)s * n + p] = s < cnt ? pos_of_rank[Lr[e]] : -1;
  }
}

// ---------------------------------------------------------------- Matern
constexpr double kEuler = 0.57721566490153286061;

__device__ void bessel_k01(double x, double &K0, double &K1) {
  if (x <= 2.0) {
    // power series of I0, I1 and the logarithmic forms of K0, K1
    const double q = 0.25 * x * x;
    double t0 = 1.0, t1 = 1.0, I0 = 0.0, I1s = 0.0, S0 = 0.0, S1 = 0.0, H = 0.0;
    for (int k = 0; k < 40; ++k) {
      if (k > 0) {
        t0 *= q / ((double)k * k);
        t1 *= q / ((double)k * (k + 1));
        H += 1.0 / k;
      }
      I0 += t0;
      I1s += t1;
      S0 += H * t0;
      S1 += (-2.0 * kEuler + 2.0 * H + 1.0 / (k + 1)) * t1;
      if (k > 2 && t0 < 1e-18 * I0) break;
    }
    const double lg = log(0.5 * x);
    K0 = -(lg + kEuler) * I0 + S0;
    K1 = 1.0 / x + lg * (0.5 * x) * I1s - 0.25 * x * S1;
  } else {
    // trapezoid rule on K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt, with
    // e^{-x} factored out and a step shrinking like x^{-1/2}
    const double hh = fmin(0.25, 0.6 / sqrt(x));
    double s0 = 0.5, s1 = 0.5;
    for (int i = 1; i < 400; ++i) {
      const double tt = i * hh;
      const double c = cosh(tt);
      const double a = x * (c - 1.0);
      const double e = exp(-a);
      s0 += e;
      s1 += e * c;
      if (a > 42.0) break;
    }
    const double f = hh * exp(-x);
    K0 = s0 * f;
    K1 = s1 * f;
  }
}

// Power-series coefficients for q = x^2/4 <= 1 (x <= 2), kSerTerms each:
// c[0][k] = 1/(k!)^2,                     I0(x) = sum c0 q^k
// c[1][k] = H_k/(k!)^2,                   K0 = -(log(x/2)+gamma) I0 + sum c1 q^k
// c[2][k] = 1/(k!(k+1)!),                 I1(x) = (x/2) sum c2 q^k
// c[3][k] = (2H_k + 1/(k+1) - 2 gamma)/(k!(k+1)!),
//                                         x K1 = 1 + 2q log(x/2) I1s - q sum c3 q^k
// (H_k the harmonic numbers; the logarithmic series of K0 and K1).  They are
// compile-time constants kept in constant memory: the factor kernel reads them
// with scalar loads where it uses them (held in registers for the whole
// kernel, the 70 coefficients of the four truncations would take 140 VGPRs).
constexpr int kSerTerms = 16;
struct SerCoef {
  double c[4][kSerTerms];
};
constexpr SerCoef make_ser_coef() {
  SerCoef t{};
  double fk = 1.0, H = 0.0;  // k!, H_k
  for (int k = 0; k < kSerTerms; ++k) {
    if (k > 0) {
      fk *= k;
      H += 1.0 / k;
    }
    const double fk1 = fk * (k + 1);
    t.c[0][k] = 1.0 / (fk * fk);
    t.c[1][k] = H / (fk * fk);
    t.c[2][k] = 1.0 / (fk * fk1);
    t.c[3][k] = (2.0 * H + 1.0 / (k + 1) - 2.0 * kEuler) / (fk * fk1);
  }
  return t;
}
__constant__ SerCoef kSerTab = make_ser_coef();
typedef const __attribute__((address_space(4))) double *SerPtr;

// a pointer to the coefficients that the compiler cannot treat as loop
// invariant, so their loads stay where they are used
__device__ __forceinline__ SerPtr ser_coef() {
  SerPtr p = (SerPtr)&kSerTab.c[0][0];
  asm volatile("" : "+s"(p));
  return p;
}

// sum_{k < NT} c[S][k] q^k
template <int S, int NT>
__device__ __forceinline__ double horner_c(SerPtr c, double q) {
  double v = c[S * kSerTerms + NT - 1];
#pragma unroll
  for (int k = NT - 2; k >= 0; --k) v = fma(v, q, c[S * kSerTerms + k]);
  return v;
}

// Even orders nu2 in {2, 4} on q = x^2/4 <= 1 from NT series terms, with
// lg = log(x/2).
template <int NT>
__device__ __forceinline__ double matern_series(int nu2, double q, double lg) {
  const SerPtr c = ser_coef();
  const double xk1 = 1.0 + 2.0 * q * lg * horner_c<2, NT>(c, q) - q * horner_c<3, NT>(c, q);
  if (nu2 == 2) return xk1;
  const double k0 = -(lg + kEuler) * horner_c<0, NT>(c, q) + horner_c<1, NT>(c, q);
  return 2.0 * q * k0 + xk1;
}

// normalised Matern correlation for the factor kernel: division-free series
// and the table-driven logarithm for x <= 2, the trapezoid rule beyond.
// logtab is the near_log table (the log enters only through terms scaled by
// q = x^2/4, so its absolute error of ~3e-16 leaves the value at rounding level).
__device__ double matern_fast(int nu2, double x, const double *__restrict__ logtab) {
  if (x == 0.0) return 1.0;
  if (nu2 == 1) return exp(-x);
  if (nu2 == 3) return (1.0 + x) * exp(-x);
  if (nu2 == 5) return (1.0 + x + x * x * (1.0 / 3.0)) * exp(-x);
  if (x > 2.0) {
    double K0, K1;
    bessel_k01(x, K0, K1);
    return nu2 == 2 ? x * K1 : 0.5 * x * x * K0 + x * K1;
  }
  return matern_series<kSerTerms>(nu2, 0.25 * x * x, near_log(0.5 * x, logtab));
}

// The same from x2 = x^2, the form the factor kernel needs: for the K_1 and
// K_2 forms on x <= 2 no square root is taken (q = x^2/4 and
// log(x/2) = log(q)/2), and the series stops once q^k/(k!)^2 < 1e-17.
// The odd orders and x > 2 go through an out-of-line call (the Bessel and
// exponential paths would raise the register count of the whole factor
// kernel); the even-order series path is inlined into the caller.
__device__ __noinline__ double matern_far(int nu2, double x2, const double *__restrict__ logtab) {
  return matern_fast(nu2, sqrt(x2), logtab);
}

__device__ __forceinline__ double matern_fast2(int nu2, double x2,
                                               const double *__restrict__ logtab) {
  if (x2 == 0.0) return 1.0;
  if ((nu2 & 1) || x2 > 4.0) return matern_far(nu2, x2, logtab);
  const double q = 0.25 * x2;
  const double lg = 0.5 * near_log(q, logtab);
  if (q < 1e-4) return matern_series<4>(nu2, q, lg);
  if (q < 1e-2) return matern_series<6>(nu2, q, lg);
  if (q < 0.1) return matern_series<9>(nu2, q, lg);
  return matern_series<kSerTerms>(nu2, q, lg);
}

// value v of lane g*MM + i (i uniform across the wavefront), g the block
// this lane belongs to: a backward permute through the LDS crossbar for
// several blocks per wavefront, two readlanes for one
template <int G, int MM>
__device__ __forceinline__ double block_bcast(double v, int i, int g) {
  if constexpr (G == 1) {
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
    return __hiloint2double(hi, lo);
  } else {
    const int addr = (g * MM + i) * 4;
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    return __hiloint2double(hi, lo);
  }
}

// Factor of the Vecchia conditionals (eq. conditionals, Fig. vecchia_chol):
// for node j with conditioning set sigma(j) (K <= m points), the Cholesky
// factor L of the Matern block of sigma(j) u {j} (node last) has last row
// (L_s^{-1} k, c), and lambda = L_s^{-T} (L_s^{-1} k).
//
// A wavefront factors G = 64/MM nodes, MM the padded block size.  Each block
// is padded to MM rows with identity rows in front (their entries of k and
// lambda are zero), so every node has the same shape.  The block's lanes
// first build its lower triangle in LDS, packed by rows (row a starts at
// a(a+1)/2): rows p and MM-1-p together hold MM+1 entries, which lanes p and
// p + MM/2 share.  Then lane (g, r) keeps row r of block g in registers and
// runs a fully unrolled left-looking Cholesky: at step c it forms
// A[r][c] - sum_k L[r][k] L[c][k] with row c read from LDS (the same address
// across the block's lanes), takes the pivot from lane c, and scales by its
// reciprocal square root.  Lane r keeps 1/L[r][r].  A block that is not
// numerically positive definite is refactored with a diagonal nugget (1e-12,
// then x100), and the nodes that needed one, or still fail, are counted.  The
// packed triangles (about 9.5 KB per wavefront at MM = 32) and a cap of 168
// VGPRs let three wavefronts share a SIMD; at MM = 64 the row alone takes 128
// VGPRs, so two share one (a tighter cap spills the row to scratch).
template <int MM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MM <= 32 ? 3 : 2)))
void k_factor(const double *x, const double *y, int64_t n, int m, const int32_t *nbr,
              const int32_t *cnt, int nu2, double alpha, double *coef, double *dinv,
              int32_t *nfail, const double *logtab) {
  constexpr int G = 64 / MM;
  constexpr int T = MM * (MM + 1) / 2;
  constexpr int H = MM / 2, NI = H + 1;  // row pairs; entries per lane
  __shared__ double Lm[G][T];
  __shared__ double2 pxy[G][MM];
  const int lane = threadIdx.x, g = lane / MM, r = lane % MM;
  const int64_t p = xcd_remap(blockIdx.x, gridDim.x) * G + g;
  const bool valid = p < n;
  const int K = valid ? cnt[p] : 0;
  const int pad = MM - 1 - K;
  // coordinates: padding rows, then sigma(j), then the node
  {
    double cx = 0.0, cy = 0.0;
    if (valid && r >= pad && r < MM - 1) {
      const int q = nbr[(int64_t)(r - pad) * n + p];
      cx = x[q];
      cy = y[q];
    } else if (valid && r == MM - 1) {
      cx = x[p];
      cy = y[p];
    }
    pxy[g][r] = make_double2(cx, cy);
  }
  const double a2 = alpha * alpha;
  const int rb = r * (r + 1) / 2;           // row r in the packed triangle
  const int pr = r % H, j0 = (r / H) * NI;  // row pair (pr, MM-1-pr); first item
  double nug = 0.0;                         // this block's nugget
  double myinv = 0.0;                       // 1 / L[r][r]
  bool ok = false;
  for (int attempt = 0; attempt < 4; ++attempt) {
    __syncthreads();
    // items j of the row pair: (pr, j) for j <= pr, else (MM-1-pr, j-pr-1)
#pragma unroll 1
    for (int t = 0; t < NI; ++t) {
      const int j = j0 + t;
      if (j > MM) continue;
      const bool lo = j <= pr;
      const int a = lo ? pr : MM - 1 - pr, b = lo ? j : j - pr - 1;
      double v;
      if (a == b) {
        v = a < pad ? 1.0 : 1.0 + nug;
      } else if (b < pad) {
        v = 0.0;
      } else {
        const double2 qa = pxy[g][a], qb = pxy[g][b];
        const double dx = qa.x - qb.x, dy = qa.y - qb.y;
        v = matern_fast2(nu2, a2 * (dx * dx + dy * dy), logtab);
      }
      Lm[g][a * (a + 1) / 2 + b] = v;
    }
    __syncthreads();
    // Left-looking Cholesky, one column per step.  The block's lanes sit in one
    // wavefront, whose LDS accesses execute in program order, so row c written
    // at earlier steps is visible without a barrier.
    double Lr[MM];
#pragma unroll
    for (int c = 0; c < MM; ++c) Lr[c] = Lm[g][rb + c];  // c > r: never read validly
    bool badl = false;
    // the row index, opaque to the compiler: the per-column lane masks
    // (r >= c, r == c) are then formed where they are used instead of being
    // hoisted out of the retry loop as 2 x MM scalar register pairs, which
    // spilled to vector-register lanes (a read-lane at every use)
    int rq = r;
    asm volatile("" : "+v"(rq));
    // fully unrolled at every MM, so Lr stays in registers (at MM = 64 the
    // default heuristics unroll it only in part and index Lr in scratch)
#pragma clang loop unroll(full)
    for (int c = 0; c < MM; ++c) {
      // two partial sums; row c is read in chunks of eight, so no more than
      // eight of its entries are held in registers at once
      double s2[2] = {0.0, 0.0};
#pragma unroll
      for (int k0 = 0; k0 < c; k0 += 8) {
#pragma unroll
        for (int k = k0; k < k0 + 8 && k < c; ++k)
          s2[k & 1] = fma(Lr[k], Lm[g][c * (c + 1) / 2 + k], s2[k & 1]);
        __builtin_amdgcn_sched_barrier(0);
      }
      const double sacc = Lr[c] - (s2[0] + s2[1]);
      double pc = block_bcast<G, MM>(sacc, c, g);
      badl = badl || !(pc > 0.0);
      pc = pc > 0.0 ? pc : 1.0;
      // 1/sqrt(pc): hardware estimate and one Newton step
      double inv = __builtin_amdgcn_rsq(pc);
      inv = fma(inv, fma(-0.5 * pc * inv, inv, 0.5), inv);
      // L[r][c] for the lanes r >= c (lane c: sacc is the pivot, so this is
      // its square root).  Lanes r < c compute values of the upper triangle
      // that no valid result reads: lane r's own entries depend only on its
      // columns k <= r, and its results at columns c > r are discarded.
      Lr[c] = sacc * inv;
      if (rq >= c) Lm[g][rb + c] = Lr[c];
      myinv = rq == c ? inv : myinv;
    }
    ok = !badl;
    if (__all(ok)) break;
    if (!ok) {
      if (attempt == 0 && r == 0) atomicAdd(&nfail[0], 1);
      nug = attempt == 0 ? 1e-12 : nug * 100.0;
    }
  }
  if (!ok && r == 0 && valid) atomicAdd(&nfail[1], 1);
  // lambda = L_s^{-T} l, l = the node's row without its diagonal, column by
  // column from the last: lambda_i = u_i / L_ii (formed on lane i, whose u is
  // final by then), then u_r -= L[i][r] lambda_i on the lanes r < i.  Lane r
  // holds u_r and ends with lambda_r = u_r / L_rr.
  double u = r < MM - 1 ? Lm[g][(MM - 1) * MM / 2 + r] : 0.0;
#pragma unroll
  for (int i = MM - 2; i >= 0; --i) {
    const double li = block_bcast<G, MM>(u * myinv, i, g);
    const double lir = r < i ? Lm[g][i * (i + 1) / 2 + r] : 0.0;  // in bounds for all r
    u = fma(-lir, li, u);
  }
  const double v = u * myinv;
  const double inv_c = block_bcast<G, MM>(myinv, MM - 1, g);
  if (!valid || !ok) return;
  // lane r < MM-1 holds lambda of row r = pad + a; padding coefficients are 0
  if (r >= pad && r < MM - 1) coef[(int64_t)(r - pad) * n + p] = -v * inv_c;
  for (int a = K + r; a < m; a += MM) coef[(int64_t)a * n + p] = 0.0;
  if (r == 0) dinv[p] = inv_c;
}

// ---------------------------------------------------------------- transpose
// Entries of the factor (stored slot-major: slot s of node j at s*n + j),
// keyed by the row q = nbr[j][s], with the node-major index j*m + s as value.
// The sort is stable and sees the entries slot-major, so each row lists its
// entries by slot, then by column: a fixed order (each (q, j) pair occurs
// once), in which the transposed apply also measured faster than in plain
// column order (0.158 against 0.200 ms at n = 2^20, m = 30).
__global__ void k_tkeys(const int32_t *nbr, int64_t n, int m, uint32_t *keys, int32_t *vals) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int q = nbr[e];
  const int64_t s = e / n, j = e - s * n;
  keys[e] = q < 0 ? (uint32_t)n : (uint32_t)q;
  vals[e] = (int32_t)(j * m + s);
}

__global__ void k_tfill(const int32_t *vals, int64_t nnz, int64_t n, int m, const double *coef,
                        int32_t *tidx, double *tcoef) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= nnz) return;
  const int64_t v = vals[p];
  const int64_t j = v / m, s = v - j * m;
  tidx[p] = (int32_t)j;
  tcoef[p] = coef[s * n + j];
}

// export in caller order (factor stored column-major, entry s of node p at s*n + p)
__global__ void k_export(int64_t n, int m, const int32_t *order, const int32_t *rank_tree,
                         const int32_t *nbr, const double *coef, const double *dinv,
                         int32_t *rank_u, int32_t *nbr_u, double *coef_u, double *diag_u) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int u = order[p];
  rank_u[u] = rank_tree[p];
  diag_u[u] = dinv[p];
  for (int s = 0; s < m; ++s) {
    const int q = nbr[(int64_t)s * n + p];
    nbr_u[(int64_t)u * m + s] = q >= 0 ? order[q] : -1;
    coef_u[(int64_t)u * m + s] = coef[(int64_t)s * n + p];
  }
}

int nu_code(double nu) {
  const double v[5] = {0.5, 1.0, 1.5, 2.0, 2.5};
  for (int i = 0; i < 5; ++i)
    if (std::fabs(nu - v[i]) < 1e-12) return i + 1;
  return 0;
}

}  // namespace

void scan_exclusive(int32_t *data, int64_t count, int32_t *ws, hipStream_t s);
int64_t scan_ws_ints(int64_t count);

void vecchia_free(Plan &pl) {
  dfree(pl.pc_rank);
  dfree(pl.pc_nbr);
  dfree(pl.pc_coef);
  dfree(pl.pc_dinv);
  dfree(pl.pc_tstart);
  dfree(pl.pc_tidx);
  dfree(pl.pc_tcoef);
  pl.pc_rank = pl.pc_nbr = pl.pc_tstart = pl.pc_tidx = nullptr;
  pl.pc_coef = pl.pc_dinv = pl.pc_tcoef = nullptr;
  pl.has_pc = false;
}

void vecchia_build(Plan &pl, const phs_precond_opts &o, hipStream_t s) {
  const int64_t n = pl.n;
  const int m = o.m > 0 ? o.m : (pl.k == 2 ? 30 : 50);
  PHS_REQUIRE(m >= 1 && m <= kMaxM, PHS_ERR_INVALID_ARGUMENT,
              "conditioning-set size must be 1..63");
  const double nu = o.nu > 0 ? o.nu : 0.5 * pl.k;
  const int nu2 = nu_code(nu);
  PHS_REQUIRE(nu2 > 0, PHS_ERR_INVALID_ARGUMENT, "nu must be one of 0.5, 1, 1.5, 2, 2.5");
  double alpha;
  if (o.range > 0) {
    PHS_REQUIRE(o.range_units == PHS_RANGE_NORMALIZED || o.range_units == PHS_RANGE_USER,
                PHS_ERR_INVALID_ARGUMENT, "bad range units");
    alpha = o.range_units == PHS_RANGE_USER ? 1.0 / (o.range * pl.rho) : 1.0 / o.range;
  } else {
    // TPS: the paper's tuned 0.35 on [-1/4, 1/4]^2; k = 4: 2 on [-1, 1]^2;
    // k = 3 (nu = 3/2): 3, which keeps the factor's dynamic range small enough
    // for FP64 PCG to reach 1e-8 up to 1e6 nodes (0.35 stalls near 1e-6 there)
    alpha = pl.k == 4 ? 2.0 : (pl.k == 3 ? 3.0 : 0.35);
  }
  // The new factor is built into `nf` and replaces the plan's only once it
  // is complete: a failed rebuild leaves the previous factor (or none) in
  // place, so no descriptor ever points at freed memory.
  struct {
    int32_t *rank = nullptr, *nbr = nullptr, *tstart = nullptr, *tidx = nullptr;
    double *coef = nullptr, *dinv = nullptr, *tcoef = nullptr;
  } nf;
  const double h = pl.tree.h;
  const int B = 256;
  // 1. ordering
  uint64_t *k64 = dmalloc<uint64_t>(n), *k64t = dmalloc<uint64_t>(n);
  int32_t *perm = dmalloc<int32_t>(n), *vt = dmalloc<int32_t>(std::max<int64_t>(n, 1));
  int T = 0;
  while (((int64_t)1 << T) < n) ++T;
  std::vector<int64_t> lvl_off(T + 2), cell_off(T + 2);
  std::vector<int32_t> gb(T + 1);
  lvl_off[0] = 0;
  cell_off[0] = 0;
  for (int t = 0; t <= T; ++t) {
    const int64_t sz = std::min<int64_t>((int64_t)1 << t, n);
    lvl_off[t + 1] = lvl_off[t] + sz;
    gb[t] = std::min(10, std::max(0, (t - 2) / 2));
    cell_off[t + 1] = cell_off[t] + ((int64_t)1 << (2 * gb[t])) + 1;
  }
  const int64_t total = lvl_off[T + 1];
  const int64_t ncells = cell_off[T + 1];
  int32_t *scr = dmalloc<int32_t>(radix_sort_scratch_ints(std::max(total, n)));
  uint32_t *gk = dmalloc<uint32_t>(total), *gkt = dmalloc<uint32_t>(total);
  int32_t *gv = dmalloc<int32_t>(total), *gvt = dmalloc<int32_t>(total);
  int32_t *cstart = dmalloc<int32_t>(ncells);
  int64_t *d_lvl = dmalloc<int64_t>(T + 2), *d_coff = dmalloc<int64_t>(T + 2);
  int32_t *d_gb = dmalloc<int32_t>(T + 1);
  double *xr = dmalloc<double>(n), *yr = dmalloc<double>(n);
  int32_t *pos_of_rank = dmalloc<int32_t>(n), *cnt = dmalloc<int32_t>(n);
  int32_t *nfail = dmalloc<int32_t>(2);
  int32_t *qord = nullptr;
  try {
    PHS_LAUNCH("vecchia_rank_keys", s,
               k_rank_keys<<<(n + B - 1) / B, B, 0, s>>>(n, o.seed, k64, perm));
    radix_sort_u64(k64, perm, n, 64, k64t, vt, scr, s);
    nf.rank = dmalloc<int32_t>(n);
    PHS_LAUNCH("vecchia_rank_maps", s,
               k_rank_maps<<<(n + B - 1) / B, B, 0, s>>>(perm, pl.inv_order, n, pl.x, pl.y,
                                                        nf.rank, pos_of_rank, xr, yr));
    // 2. rank-prefix grids
    PHS_HIP(hipMemcpyAsync(d_lvl, lvl_off.data(), (T + 2) * 8, hipMemcpyHostToDevice, s));
    PHS_HIP(hipMemcpyAsync(d_coff, cell_off.data(), (T + 2) * 8, hipMemcpyHostToDevice, s));
    PHS_HIP(hipMemcpyAsync(d_gb, gb.data(), (T + 1) * 4, hipMemcpyHostToDevice, s));
    PHS_LAUNCH("vecchia_grid_keys", s,
               k_grid_keys<<<(total + B - 1) / B, B, 0, s>>>(xr, yr, T, d_lvl, d_gb, h, total,
                                                            gk, gv));
    radix_sort_u32(gk, gv, total, 25, gkt, gvt, scr, s);
    double2 *gxy = dmalloc<double2>(total);
    PHS_LAUNCH("vecchia_grid_coords", s,
               k_grid_coords<<<(total + B - 1) / B, B, 0, s>>>(gv, xr, yr, total, gxy));
    PHS_LAUNCH("vecchia_cell_start", s,
               k_cell_start<<<(ncells + B - 1) / B, B, 0, s>>>(gk, total, T, d_gb, d_coff,
                                                              ncells, cstart));
    // 3. ordered nearest predecessors, queries by grid level then tree position
    qord = dmalloc<int32_t>(n);
    {
      uint32_t *qk = reinterpret_cast<uint32_t *>(k64), *qkt = reinterpret_cast<uint32_t *>(k64t);
      PHS_LAUNCH("vecchia_qkeys", s,
                 k_qkeys<<<(n + B - 1) / B, B, 0, s>>>(nf.rank, n, T, qk, qord));
      int qbits = 1;
      while ((1 << qbits) <= T) ++qbits;
      radix_sort_u32(qk, qord, n, qbits, qkt, vt, scr, s);  // sorted ranks in qord
    }
    nf.nbr = dmalloc<int32_t>((size_t)n * m);
    PHS_LAUNCH("vecchia_knn", s,
               (m <= 16 ? k_knn<1> : m <= 32 ? k_knn<2> : k_knn<4>)<<<(n + 15) / 16, 256, 0, s>>>(
                   xr, yr, n, m, T, h, d_gb, d_coff, cstart, gv, gxy, pos_of_rank, qord, nf.nbr,
                   cnt));
    dfree(gxy);
    // 4. factor
    nf.coef = dmalloc<double>((size_t)n * m);
    nf.dinv = dmalloc<double>(n);
    PHS_HIP(hipMemsetAsync(nfail, 0, 8, s));
    if (m <= 15)
      PHS_LAUNCH("vecchia_factor", s,
                 k_factor<16><<<(n + 3) / 4, 64, 0, s>>>(pl.x, pl.y, n, m, nf.nbr, cnt, nu2,
                                                         alpha, nf.coef, nf.dinv, nfail,
                                                         pl.neartab));
    else if (m <= 31)
      PHS_LAUNCH("vecchia_factor", s,
                 k_factor<32><<<(n + 1) / 2, 64, 0, s>>>(pl.x, pl.y, n, m, nf.nbr, cnt, nu2,
                                                         alpha, nf.coef, nf.dinv, nfail,
                                                         pl.neartab));
    else
      PHS_LAUNCH("vecchia_factor", s,
                 k_factor<64><<<n, 64, 0, s>>>(pl.x, pl.y, n, m, nf.nbr, cnt, nu2, alpha,
                                              nf.coef, nf.dinv, nfail, pl.neartab));
    // 5. transpose: stable radix sort of the entries by row
    {
      const int64_t N = n * m;
      uint32_t *tk = dmalloc<uint32_t>(N), *tkt = dmalloc<uint32_t>(N);
      int32_t *tv = dmalloc<int32_t>(N), *tvt = dmalloc<int32_t>(N);
      int32_t *tscr = dmalloc<int32_t>(radix_sort_scratch_ints(N));
      int bits = 1;
      while (((int64_t)1 << bits) <= n) ++bits;
      PHS_LAUNCH("vecchia_tkeys", s,
                 k_tkeys<<<(N + B - 1) / B, B, 0, s>>>(nf.nbr, n, m, tk, tv));
      bool in_tmp = false;
      radix_sort_u32(tk, tv, N, bits, tkt, tvt, tscr, s, &in_tmp);
      const uint32_t *sk = in_tmp ? tkt : tk;  // sorted keys and values
      const int32_t *sv = in_tmp ? tvt : tv;
      try {
        nf.tstart = dmalloc<int32_t>(n + 1);
        leaf_ranges(sk, N, (int)n, nf.tstart, s);
        int32_t nnz = 0;
        PHS_HIP(hipMemcpyAsync(&nnz, nf.tstart + n, 4, hipMemcpyDeviceToHost, s));
        PHS_HIP(hipStreamSynchronize(s));
        nf.tidx = dmalloc<int32_t>(std::max(nnz, 1));
        nf.tcoef = dmalloc<double>(std::max(nnz, 1));
        if (nnz > 0)
          PHS_LAUNCH("vecchia_tfill", s,
                     k_tfill<<<(nnz + B - 1) / B, B, 0, s>>>(sv, nnz, n, m, nf.coef, nf.tidx,
                                                            nf.tcoef));
      } catch (...) {
        for (void *q : {(void *)tk, (void *)tkt, (void *)tv, (void *)tvt, (void *)tscr}) dfree(q);
        throw;
      }
      for (void *q : {(void *)tk, (void *)tkt, (void *)tv, (void *)tvt, (void *)tscr}) dfree(q);
    }
    int32_t hfail[2] = {0, 0};
    PHS_HIP(hipMemcpyAsync(hfail, nfail, 8, hipMemcpyDeviceToHost, s));
    PHS_HIP(hipStreamSynchronize(s));
    PHS_REQUIRE(hfail[1] == 0, PHS_ERR_INVALID_ARGUMENT,
                "Matern block not positive definite even with a diagonal nugget");
    // commit: the previous factor is released (its blocks are recycled only
    // once the device is idle) and the plan takes the new one
    vecchia_free(pl);
    pl.pc_rank = nf.rank;
    pl.pc_nbr = nf.nbr;
    pl.pc_coef = nf.coef;
    pl.pc_dinv = nf.dinv;
    pl.pc_tstart = nf.tstart;
    pl.pc_tidx = nf.tidx;
    pl.pc_tcoef = nf.tcoef;
    pl.m = m;
    pl.nu = nu;
    pl.alpha = alpha;
    pl.pc_nugget_nodes = hfail[0];
    pl.has_pc = true;
  } catch (...) {
    for (void *q : {(void *)nf.rank, (void *)nf.nbr, (void *)nf.coef, (void *)nf.dinv,
                    (void *)nf.tstart, (void *)nf.tidx, (void *)nf.tcoef})
      dfree(q);
    for (void *q : {(void *)k64, (void *)k64t, (void *)perm, (void *)vt, (void *)scr, (void *)gk,
                    (void *)gkt, (void *)gv, (void *)gvt, (void *)cstart, (void *)d_lvl,
                    (void *)d_coff, (void *)d_gb, (void *)xr, (void *)yr, (void *)pos_of_rank,
                    (void *)cnt, (void *)nfail, (void *)qord})
      dfree(q);
    throw;
  }
  for (void *q : {(void *)k64, (void *)k64t, (void *)perm, (void *)vt, (void *)scr, (void *)gk,
                  (void *)gkt, (void *)gv, (void *)gvt, (void *)cstart, (void *)d_lvl,
                  (void *)d_coff, (void *)d_gb, (void *)xr, (void *)yr, (void *)pos_of_rank,
                  (void *)cnt, (void *)nfail, (void *)qord})
    dfree(q);
  pool_mark_idle();
}

void vecchia_export(Plan &pl, int32_t *rank, int32_t *nbr, double *coef, double *diag,
                    hipStream_t s) {
  const int64_t n = pl.n;
  PHS_LAUNCH("precond_export", s,
             k_export<<<(n + 255) / 256, 256, 0, s>>>(n, pl.m, pl.order, pl.pc_rank,
                                                      pl.pc_nbr, pl.pc_coef, pl.pc_dinv, rank,
                                                      nbr, coef, diag));
}

}  // namespace phs
