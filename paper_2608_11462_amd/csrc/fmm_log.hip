// Log-kernel fast multipole method on the uniform quadtree (paper Sec. 2.1:
// eqs. outgoing and incoming, steps 2-6 of the FMM description), applied to
// the R densities of the Hadamard reduction (eq. matvec_hadamard).
//
// Expansions are scaled by the box width w_l so every coefficient is O(1):
//   outgoing about centre c:  Phi(z) = A_0 log(z - c) + sum_{k>=1} A_k ((z-c)/w)^{-k},
//                             A_0 = sum q,  A_k = -sum q ((y-c)/w)^k / k
//   incoming about centre c:  Phi(z) = sum_k B_k ((z-c)/w)^k      (real part taken)
// With these scalings the outgoing->outgoing and incoming->incoming shifts are
// the same four matrices on every level, and the outgoing->incoming operator
// for a source/target centre offset D (in box widths) is
//   B_l = sum_k H[l][k] D^{-(k+l)} A_k  (+ A_0 (log w + log|D|) for l = 0),
// H[0][k] = 1, H[l][0] = (-1)^{l+1}/l, H[l][k] = (-1)^l binom(k+l-1, l),
// one real matrix shared by all 40 offsets and all levels.
//
// Layout: level l holds (P+1) x nd x 4^l complex coefficients, box index
// fastest (coalesced across neighbouring boxes), levels 2..L concatenated.
#include <climits>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "fmm_common.h"

namespace phs {

namespace {

template <class T>
using V2 = typename Vec2<T>::type;

__host__ __device__ inline int64_t level_base(int l, int P, int nd) {
  // complex elements before level l (levels start at 2)
  return (int64_t)(P + 1) * nd * (((int64_t)1 << (2 * l)) - 16) / 3;
}

// ------------------------------------------------------------------ P2M
// Work item: 4 gpw leaves of one system, gpw = 64/(P+1) leaves per wavefront
// (lane = coefficient), four wavefronts per block.  The points of the wave's
// leaves pass in chunks of ch per leaf.  For each point one lane stores in LDS
// its powers z^0..z^3 and z^0, z^4, ..., z^{4(A-1)}, A = P/4 + 1, and its
// density terms v_r t; the lane of coefficient k then forms z^k as
// z^{4 floor(k/4)} z^{k mod 4}, one complex product per point.
constexpr int kP2MPadPw = 8;   // pair slots between two leaves' power tables
constexpr int kP2MPadQ = 16;   // scalars between two leaves' density terms
constexpr int kP2MLdsBlock = 32768;

template <class T>
__host__ __device__ inline int p2m_wave_bytes(int P, int R, int gpw, int ch) {
  const int ns = 4 + (P >> 2) + 1;
  const int b = gpw * ((ch * ns + kP2MPadPw) * 2 + ch * R + kP2MPadQ) * (int)sizeof(T);
  return (b + 15) & ~15;
}

// Points per leaf and chunk: the largest of 64/gpw, 32/gpw, ... whose tables
// for four wavefronts fit in kP2MLdsBlock bytes.
template <class T>
int p2m_chunk(int P, int R, int gpw) {
  int ch = 64 / gpw;
  while (ch > 4 && 4 * p2m_wave_bytes<T>(P, R, gpw, ch) > kP2MLdsBlock) ch >>= 1;
  return ch;
}

template <class T, int K>
__global__ __launch_bounds__(256) void kf_p2m(const SysDev *__restrict__ sys,
                                              const BlkRef *__restrict__ tab,
                                              const int32_t *__restrict__ mask, int P, int in,
                                              int ch) {
  constexpr int R = Rank<K>::R;
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int L = d.L;
  const int G = 1 << L;
  const int nleaf = G * G;
  const int P1 = P + 1;
  const int gpw = p2m_leaves_per_wave(P);
  const int sub = lane / P1, kk = lane % P1;
  const double h = d.h;
  const cptr<double> x = ro(d.x);
  const cptr<double> y = ro(d.y);
  const cptr<float> ux = ro(d.ux);
  const cptr<float> uy = ro(d.uy);
  const cptr<double> t = ro(d.v[in]);
  const cptr<int32_t> lstart = ro(d.leaf_start);
  const gptr<V2<T>> A = rw((V2<T> *)d.mp + level_base(L, P, R));
  const double w = 2.0 * h / G, invw = G / (2.0 * h);
  const bool active = sub < gpw;
  const int leaf0 = (br.blk * 4 + wave) * gpw;
  const int leaf = leaf0 + (active ? sub : 0);
  // the wave's leaves (uniform ranges) and the longest of them
  int bg[4] = {0, 0, 0, 0}, eg[4] = {0, 0, 0, 0};
  int maxcnt = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g)
    if (g < gpw) {
      bg[g] = lstart[leaf0 + g];
      eg[g] = lstart[leaf0 + g + 1];
      maxcnt = max(maxcnt, eg[g] - bg[g]);
    }
  const int b = active ? bg[sub] : 0, e = active ? eg[sub] : 0;
  T are[R], aim[R];
#pragma unroll
  for (int r = 0; r < R; ++r) are[r] = aim[r] = T(0);
  extern __shared__ __align__(16) unsigned char p2m_lds[];
  const int na = (P >> 2) + 1, ns = 4 + na;
  const int pw_leaf = ch * ns + kP2MPadPw, q_leaf = ch * R + kP2MPadQ;
  unsigned char *wb = p2m_lds + wave * p2m_wave_bytes<T>(P, R, gpw, ch);
  V2<T> *const spw = (V2<T> *)wb;
  T *const sq = (T *)(wb + (size_t)gpw * pw_leaf * sizeof(V2<T>));
  const V2<T> *const pa = spw + sub * pw_leaf + 4 + (kk >> 2);
  const V2<T> *const pb = spw + sub * pw_leaf + (kk & 3);
  const T *const qs = sq + sub * q_leaf;
  const C2<T> one = {T(1), T(0)};
  for (int off = 0; off < maxcnt; off += ch) {
    if (lane < gpw * ch) {
      const int g = lane / ch, jl = lane - g * ch;
      const int j = bg[g] + off + jl;
      if (j < eg[g]) {
        const int lf = leaf0 + g;
        const double xj = x[j], yj = y[j];
        // the powers are formed in FP64 and rounded once to T when stored
        C2<double> z;
        if constexpr (std::is_same<T, float>::value) {
          z = {(double)(ux[j] * (float)invw), (double)(uy[j] * (float)invw)};
        } else {
          const double cxg = -h + (lf % G + 0.5) * w, cyg = -h + (lf / G + 0.5) * w;
          z = {(xj - cxg) * invw, (yj - cyg) * invw};
        }
        V2<T> *const pp = spw + g * pw_leaf + jl * ns;
        const auto put = [&](int slot, C2<double> c) { st2<T>(pp + slot, {(T)c.re, (T)c.im}); };
        const C2<double> z2 = cmul(z, z), z4 = cmul(z2, z2);
        st2<T>(pp + 0, one);
        put(1, z);
        put(2, z2);
        put(3, cmul(z2, z));
        C2<double> za = {1.0, 0.0};
        st2<T>(pp + 4, one);
        for (int a = 1; a < na; ++a) {
          za = cmul(za, z4);
          put(4 + a, za);
        }
        T v[R];
        vfac<K, T>(xj, yj, v);
        const T tj = (T)t[j];
        T *const qq = sq + g * q_leaf + jl * R;
#pragma unroll
        for (int r = 0; r < R; ++r) qq[r] = v[r] * tj;
      }
    }
    // a wavefront's LDS accesses complete in program order
    __builtin_amdgcn_wave_barrier();
    const int cnt = active ? min(ch, e - b - off) : 0;
    for (int jj = 0; jj < cnt; ++jj) {
      const C2<T> zk = cmul(ld2<T>(pa + jj * ns), ld2<T>(pb + jj * ns));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const T q = qs[jj * R + r];
        are[r] += q * zk.re;
        aim[r] += q * zk.im;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (!active) return;
  const T sc = kk == 0 ? T(1) : T(-1) / T(kk);
#pragma unroll
  for (int r = 0; r < R; ++r)
    st2<T>(&A[((int64_t)kk * R + r) * nleaf + leaf], {are[r] * sc, aim[r] * sc});
}

// ------------------------------------------------------------------ M2M
// Work item: 256 lanes over (parent box, density, coefficient) triples of one
// level; on coarse levels four lanes per triple, lane c summing child c's
// contribution, added over the quad, and on the coarsest sixteen, lane 4q + c
// summing child c's terms k = q mod 4, added over the row.
template <class T>
__global__ void kf_m2m(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                       const int32_t *__restrict__ mask, int lp, int P,
                       const V2<T> *__restrict__ m2m) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R;
  const int Gp = 1 << lp, Gc = 2 * Gp;
  const int64_t nbp = (int64_t)Gp * Gp, nbc = 4 * nbp;
  const int split = shift_split(lp);
  const int64_t tid = (int64_t)br.blk * 256 + threadIdx.x;
  if (tid >= nbp * nd * (P + 1) * split) return;  // whole lane groups
  const cptr<V2<T>> Ac = ro((const V2<T> *)d.mp + level_base(lp + 1, P, nd));
  const gptr<V2<T>> Ap = rw((V2<T> *)d.mp + level_base(lp, P, nd));
  const int sub = (int)(tid & (split - 1));
  const int64_t o = tid / split;
  const int c0 = split >= 4 ? (sub & 3) : 0, c1 = split >= 4 ? c0 + 1 : 4;
  const int ks = split == 16 ? 4 : 1, kq = split == 16 ? (sub >> 2) : 0;  // terms k = kq mod ks
  const int box = (int)(o % nbp);
  const int64_t rest = o / nbp;
  const int r = (int)(rest % nd), lc = (int)(rest / nd);
  const int ix = box % Gp, iy = box / Gp;
  C2<T> acc = {T(0), T(0)};
  for (int c = c0; c < c1; ++c) {
    const int child = (2 * iy + (c >> 1)) * Gc + 2 * ix + (c & 1);
    const V2<T> *row = m2m + ((int64_t)c * (P + 1) + lc) * (P + 1);
    // four terms' loads in flight at a time, summed in k order
    int k = kq;
    for (; k + 3 * ks <= lc; k += 4 * ks) {
      C2<T> mv[4], av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        mv[u] = ld2<T>(row + k + u * ks);
        av[u] = ld2<T>(&Ac[((int64_t)(k + u * ks) * nd + r) * nbc + child]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = cadd(acc, cmul(mv[u], av[u]));
    }
    for (; k <= lc; k += ks)
      acc = cadd(acc, cmul(ld2<T>(row + k), ld2<T>(&Ac[((int64_t)k * nd + r) * nbc + child])));
  }
  if (split == 16) {
    acc.re = row_sum16(acc.re);
    acc.im = row_sum16(acc.im);
    if (sub != 0) return;
  } else if (split == 4) {
    acc.re = quad_sum(acc.re);
    acc.im = quad_sum(acc.im);
    if (sub != 0) return;
  }
  st2<T>(&Ap[((int64_t)lc * nd + r) * nbp + box], acc);
}

// ------------------------------------------------------------------ M2L
// Work item: (tile of 256 boxes over levels 2..L, density, chunk of LCH
// output coefficients) of one system, chunk fastest.  Boxes are enumerated by
// parity class so a wavefront shares one interaction-list pattern.  The table
// index is remapped so that consecutive items run on one XCD.
template <class T, int LCH>
__global__ __launch_bounds__(256) void kf_m2l(const SysDev *__restrict__ sys,
                                              const BlkRef *__restrict__ tab,
                                              const int32_t *__restrict__ mask, int P,
                                              const T *__restrict__ Ht, int nchunks) {
  const BlkRef br = tab[xcd_remap(blockIdx.x, gridDim.x)];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R, L = d.L;
  const double h = d.h;
  const cptr<V2<T>> A = ro((const V2<T> *)d.mp);
  const gptr<V2<T>> B = rw((V2<T> *)d.loc);
  const int64_t lb = br.blk;
  const int l0 = (int)(lb % nchunks) * LCH;
  const int r = (int)((lb / nchunks) % nd);
  const int64_t tile = lb / ((int64_t)nchunks * nd);
  int64_t t = tile * 256 + threadIdx.x;
  int l = 2;
  int64_t off = 0, base = 0;
  while (l <= L && t >= off + ((int64_t)1 << (2 * l))) {
    off += (int64_t)1 << (2 * l);
    base += (int64_t)(P + 1) * nd * ((int64_t)1 << (2 * l));
    ++l;
  }
  if (l > L) return;
  const int G = 1 << l;
  const int64_t nb = (int64_t)G * G;
  const int64_t ti = t - off;
  // boxes by strips of two rows: within a strip the four parity classes, each
  // a run of G/2 boxes with one interaction-list pattern
  const int half = G / 2;
  const int aa = (int)(ti % half);
  const int64_t rest = ti / half;
  const int cls = (int)(rest & 3);
  const int brow = (int)(rest >> 2);
  const int ix = 2 * aa + (cls & 1);
  const int iy = 2 * brow + (cls >> 1);
  const cptr<V2<T>> Al = A + base;
  const gptr<V2<T>> Bl = B + base;
  const T logw = (T)log(2.0 * h / G);
  C2<T> acc[LCH];
#pragma unroll
  for (int c = 0; c < LCH; ++c) acc[c] = {T(0), T(0)};
  const int pxp = ix >> 1, pyp = iy >> 1;
  for (int oy = -3; oy <= 3; ++oy) {
    const int jy = iy + oy;
    if (jy < 0 || jy >= G || abs((jy >> 1) - pyp) > 1) continue;
    for (int ox = -3; ox <= 3; ++ox) {
      if (abs(ox) <= 1 && abs(oy) <= 1) continue;
      const int jx = ix + ox;
      if (jx < 0 || jx >= G || abs((jx >> 1) - pxp) > 1) continue;
      const int64_t src = (int64_t)jy * G + jx;
      const T Dx = T(-ox), Dy = T(-oy);
      const T dd = Dx * Dx + Dy * Dy;
      const C2<T> Dinv = {Dx / dd, -Dy / dd};
      C2<T> Y[LCH];
#pragma unroll
      for (int c = 0; c < LCH; ++c) Y[c] = {T(0), T(0)};
      C2<T> dk = {T(1), T(0)};
      // coefficients k = k0..k0+3 are loaded one group ahead of their use, so
      // four loads are in flight while the previous group is multiplied
      const cptr<V2<T>> ap = Al + (int64_t)r * nb + src;
      const int64_t ks = (int64_t)nd * nb;
      C2<T> nx[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) nx[i] = i <= P ? ld2<T>(&ap[i * ks]) : C2<T>{T(0), T(0)};
      const T a0 = nx[0].re;
      for (int k0 = 0; k0 <= P; k0 += 4) {
        C2<T> cu[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) cu[i] = nx[i];
        if (k0 + 4 <= P) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            nx[i] = k0 + 4 + i <= P ? ld2<T>(&ap[(k0 + 4 + i) * ks]) : C2<T>{T(0), T(0)};
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int k = k0 + i;
          if (k > P) break;
          const C2<T> xk = cmul(cu[i], dk);
          const T *hrow = Ht + k * (P + 1) + l0;
#pragma unroll
          for (int c = 0; c < LCH; ++c) {
            Y[c].re += hrow[c] * xk.re;
            Y[c].im += hrow[c] * xk.im;
          }
          dk = cmul(dk, Dinv);
        }
      }
      C2<T> e = cpow_small(Dinv, l0);
#pragma unroll
      for (int c = 0; c < LCH; ++c) {
        acc[c] = cadd(acc[c], cmul(e, Y[c]));
        e = cmul(e, Dinv);
      }
      if (l0 == 0) acc[0].re += a0 * (logw + T(0.5) * (T)log((double)dd));
    }
  }
  const int64_t tgt = (int64_t)iy * G + ix;
#pragma unroll
  for (int c = 0; c < LCH; ++c)
    if (l0 + c <= P) st2<T>(&Bl[((int64_t)(l0 + c) * nd + r) * nb + tgt], acc[c]);
}

// ------------------------------------------------------------------ M2M / L2L, deep levels
// With the child centre offset delta_c = rho u_c (|u_c| = 1, rho = sqrt(2)/4
// in parent widths, the same for all four children), the shifts factor as
// M2M[c][l][k] = u_c^l Rm[l][k] u_c^-k and L2L[c][j][k] = u_c^-j Rl[j][k] u_c^k
// with real triangular Rm, Rl shared by the four children.  On the deep
// levels a block stages one row segment of coefficients in LDS once, where
// the per-coefficient kernels re-read each one from the cache dozens of times.

// Upward, parent level lp with at least 16 boxes per row: a block takes 16
// consecutive parents of one row and one density; their 64 children's
// coefficients are staged prescaled by u_c^-k, and thread (parent, lg) forms
// B_l = sum_c u_c^l sum_{k<=l} Rm[l][k] x_{c,k} for l = lg and lg + 16.
template <int P>
__global__ __launch_bounds__(256) void kf_m2m_seg(const SysDev *__restrict__ sys,
                                                 const BlkRef *__restrict__ tab,
                                                 const int32_t *__restrict__ mask, int lp,
                                                 const double *__restrict__ Rm,
                                                 const double2 *__restrict__ Ph) {
  constexpr int P1 = P + 1;
  __shared__ double2 sx[64 * P1];  // [k][child of the segment]
  __shared__ double srm[P1 * P1];
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R;
  const int Gp = 1 << lp, Gc = 2 * Gp;
  const int nseg = Gp / 16;
  const int r = (int)(br.blk % nd);
  const int64_t sg = br.blk / nd;
  const int py = (int)(sg / nseg), px0 = (int)(sg % nseg) * 16;
  const int64_t nbp = (int64_t)Gp * Gp, nbc = 4 * nbp;
  const cptr<double2> Ac = ro((const double2 *)d.mp + level_base(lp + 1, P, nd));
  const gptr<double2> Ap = rw((double2 *)d.mp + level_base(lp, P, nd));
  for (int e = threadIdx.x; e < 64 * P1; e += 256) {
    const int k = e >> 6, ch = e & 63;
    const int ccx = 2 * px0 + (ch & 31), ccy = 2 * py + (ch >> 5);
    const int c = (ccy & 1) * 2 + (ccx & 1);
    const C2<double> a = ld2<double>(&Ac[((int64_t)k * nd + r) * nbc + (int64_t)ccy * Gc + ccx]);
    const C2<double> uk = ld2<double>(&Ph[c * 32 + k]);
    sx[e] = make_double2(a.re * uk.re + a.im * uk.im, a.im * uk.re - a.re * uk.im);
  }
  for (int e = threadIdx.x; e < P1 * P1; e += 256) srm[e] = Rm[e];
  __syncthreads();
  const int pl = threadIdx.x & 15, lg = threadIdx.x >> 4;
  const int64_t parent = (int64_t)py * Gp + px0 + pl;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int l = lg + 16 * h;
    if (l > P) break;
    C2<double> acc = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int ch = (c >> 1) * 32 + 2 * pl + (c & 1);
      C2<double> y = {0.0, 0.0};
      for (int k = 0; k <= l; ++k) {
        const double m = srm[l * P1 + k];
        const double2 xv = sx[k * 64 + ch];
        y.re = fma(m, xv.x, y.re);
        y.im = fma(m, xv.y, y.im);
      }
      acc = cadd(acc, cmul(ld2<double>(&Ph[c * 32 + l]), y));
    }
    st2<double>(&Ap[((int64_t)l * nd + r) * nbp + parent], acc);
  }
}

// Downward, child level lc >= 7 (at least 64 parents per row: enough blocks
// for these long per-thread sums; used from level 7): a block takes 32
// consecutive parents of one row and one density, stages their incoming
// coefficients, and two threads per child (output orders j of either parity)
// form u_c^-j sum_{k>=j} Rl[j][k] u_c^k B_k, added to the child's expansion.
template <int P>
__global__ __launch_bounds__(256) void kf_l2l_seg(const SysDev *__restrict__ sys,
                                                 const BlkRef *__restrict__ tab,
                                                 const int32_t *__restrict__ mask, int lc,
                                                 const double *__restrict__ Rl,
                                                 const double2 *__restrict__ Ph) {
  constexpr int P1 = P + 1, NJ = P1 / 2;
  __shared__ double2 sb[32 * P1];  // [k][parent of the segment]
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R;
  const int Gc = 1 << lc, Gp = Gc / 2;
  const int nseg = Gp / 32;
  const int r = (int)(br.blk % nd);
  const int64_t sg = br.blk / nd;
  const int py = (int)(sg / nseg), px0 = (int)(sg % nseg) * 32;
  const int64_t nbc = (int64_t)Gc * Gc, nbp = nbc / 4;
  const cptr<double2> Bp = ro((const double2 *)d.loc + level_base(lc - 1, P, nd));
  const gptr<double2> Bc = rw((double2 *)d.loc + level_base(lc, P, nd));
  for (int e = threadIdx.x; e < 32 * P1; e += 256) {
    const int k = e >> 5, q = e & 31;
    const C2<double> bv = ld2<double>(&Bp[((int64_t)k * nd + r) * nbp + (int64_t)py * Gp + px0 + q]);
    sb[e] = make_double2(bv.re, bv.im);
  }
  __syncthreads();
  // par (the parity of the output orders j) is uniform across each wavefront;
  // saying so makes the Rl loads scalar and the j <= k tests branch-free
  const int ci = threadIdx.x & 127, par = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);
  const int cx = 2 * px0 + (ci & 63), cy = 2 * py + (ci >> 6);
  const int c = (cy & 1) * 2 + (cx & 1);
  const int q = (ci & 63) >> 1;
  const cptr<double> rl = ro(Rl);
  const C2<double> u = ld2<double>(&Ph[c * 32 + 1]);
  C2<double> uk = {1.0, 0.0};
  C2<double> y[NJ];
#pragma unroll
  for (int i = 0; i < NJ; ++i) y[i] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k <= P; ++k) {
    const double2 bv = sb[k * 32 + q];
    const C2<double> b = cmul(C2<double>{bv.x, bv.y}, uk);
    uk = cmul(uk, u);
    const cptr<double> rk = in_place(rl);  // column k of Rl, loaded here
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
      const int j = 2 * i + par;
      if (j <= k) {
        const double m = rk[j * P1 + k];
        y[i].re = fma(m, b.re, y[i].re);
        y[i].im = fma(m, b.im, y[i].im);
      }
    }
  }
  const int64_t child = (int64_t)cy * Gc + cx;
  const C2<double> u2 = cmul(u, u);
  C2<double> uj = par ? u : C2<double>{1.0, 0.0};
#pragma unroll
  for (int i = 0; i < NJ; ++i) {
    const int j = 2 * i + par;
    const C2<double> o = {y[i].re * uj.re + y[i].im * uj.im, y[i].im * uj.re - y[i].re * uj.im};
    const gptr<double2> dst = &Bc[((int64_t)j * nd + r) * nbc + child];
    st2<double>(dst, cadd(ld2<double>(dst), o));
    uj = cmul(uj, u2);
  }
}

// ------------------------------------------------------------------ M2L, matrix cores
// The FP64 outgoing->incoming translation as a product with the one real
// matrix H, on the matrix cores.  Work item: one wavefront = (strip of 16
// boxes of one parity class that are neighbours in x on one level, density
// r).  The interaction offset D is the same for the whole strip, so per
// offset, with lane = column c (box) + 16 q:
//   X[k][c] = D^{-k} A_k(source of c)     prescale, k = 4 s + q
//   Y = H X                               v_mfma_f64_16x16x4f64, two 16-row
//                                         tiles of l, NKS steps of 4 in k
//   B[l][c] += D^{-l} Y[l][c]             postscale, l = 16 t + q + 4 j
// plus A_0 (log w + log|D|) into B_0.  H (zero padded to 32 x 4 NKS) stays in
// the A-operand registers for the whole item.  Lane layout of the 16x16x4
// FP64 product (row m, column n, inner index k): A[m][k] at lane m + 16 k,
// B[k][n] at lane n + 16 k, result D[m][n] at lane n + 16 (m mod 4) in
// register m / 4.  Columns whose source box lies outside the grid, and
// columns past the end of a short strip, get X = 0.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// Capped at 168 VGPRs (three wavefronts per SIMD instead of two at 204): the
// grid is only a few wavefronts per SIMD, and the offsets' gathers wait on
// memory, so occupancy hides more than the few spilled registers cost.
template <int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3)))
void kf_m2l_mfma(const SysDev *__restrict__ sys,
                                                  const BlkRef *__restrict__ tab,
                                                  const int32_t *__restrict__ mask,
                                                  const double *__restrict__ Ht,
                                                  const double *__restrict__ Off) {
  constexpr int NKS = (P + 4) / 4;
  const BlkRef br = tab[xcd_remap(blockIdx.x, gridDim.x)];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R, L = d.L;
  const double h = d.h;
  const int lane = threadIdx.x;
  const int c = lane & 15, q = lane >> 4;
  const int r = (int)(br.blk % nd);
  int64_t strip = br.blk / nd;
  int l = 2;
  int64_t base = 0;
  int G = 4, half = 2, nsr = 1;
  for (;;) {
    G = 1 << l;
    half = G >> 1;
    nsr = (half + 15) >> 4;
    const int64_t S = 4LL * half * nsr;
    if (strip < S) break;
    strip -= S;
    base += (int64_t)(P + 1) * nd * G * G;
    if (++l > L) return;
  }
  const int sr = (int)(strip % nsr);
  const int64_t rest = strip / nsr;
  const int cls = (int)(rest & 3), brow = (int)(rest >> 2);
  const int aa = sr * 16 + c;
  const bool colok = aa < half;
  const int px = cls & 1, py = cls >> 1;
  const int ix = 2 * aa + px, iy = 2 * brow + py;
  const int64_t nb = (int64_t)G * G;
  const int64_t kstride = (int64_t)nd * nb;
  const cptr<double2> Al = ro((const double2 *)d.mp + base + (int64_t)r * nb);
  const gptr<double2> Bl = rw((double2 *)d.loc + base);
  const double logw = log(2.0 * h / G);
  double hA[2][NKS];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int st = 0; st < NKS; ++st) {
      const int lr = 16 * t + c, kk = 4 * st + q;
      hA[t][st] = (lr <= P && kk <= P) ? Ht[kk * (P + 1) + lr] : 0.0;
    }
  C2<double> acc[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[t][j] = {0.0, 0.0};
  const cptr<double> offt = ro(Off);
  for (int oy = -3; oy <= 3; ++oy) {
    const int jy = iy + oy;
    if (jy < 0 || jy >= G || abs((jy >> 1) - brow) > 1) continue;
    for (int ox = -3; ox <= 3; ++ox) {
      if (abs(ox) <= 1 && abs(oy) <= 1) continue;
      if (abs((px + ox) >> 1) > 1) continue;  // source parent not adjacent
      const int jx = ix + ox;
      const bool ok = colok && jx >= 0 && jx < G;
      const int64_t src = (int64_t)jy * G + (ok ? jx : 0);
      // D^-1, D^-4, D^-q and log|D| of this offset (uniform: scalar loads)
      const cptr<double> ot = offt + 16 * (7 * (oy + 3) + (ox + 3));
      const C2<double> D4 = {ot[2], ot[3]};
      C2<double> pw[8];  // pw[m] = D^-(4 m + q)
      pw[0] = {q == 0 ? ot[4] : q == 1 ? ot[6] : q == 2 ? ot[8] : ot[10],
               q == 0 ? ot[5] : q == 1 ? ot[7] : q == 2 ? ot[9] : ot[11]};
#pragma unroll
      for (int mm = 1; mm < 8; ++mm) pw[mm] = cmul(pw[mm - 1], D4);
      double xr[NKS], xim[NKS];
      double a0 = 0.0;
#pragma unroll
      for (int st = 0; st < NKS; ++st) {
        const int kk = 4 * st + q;
        C2<double> a = {0.0, 0.0};
        if (ok && (4 * st + 3 <= P || kk <= P)) a = ld2<double>(&Al[kk * kstride + src]);
        if (st == 0) a0 = a.re;
        const C2<double> x = cmul(a, pw[st]);
        xr[st] = x.re;
        xim[st] = x.im;
      }
      dbl4 yr0 = {0.0, 0.0, 0.0, 0.0}, yr1 = yr0, yi0 = yr0, yi1 = yr0;
#pragma unroll
      for (int st = 0; st < NKS; ++st) {
        yr0 = __builtin_amdgcn_mfma_f64_16x16x4f64(hA[0][st], xr[st], yr0, 0, 0, 0);
        yi0 = __builtin_amdgcn_mfma_f64_16x16x4f64(hA[0][st], xim[st], yi0, 0, 0, 0);
        yr1 = __builtin_amdgcn_mfma_f64_16x16x4f64(hA[1][st], xr[st], yr1, 0, 0, 0);
        yi1 = __builtin_amdgcn_mfma_f64_16x16x4f64(hA[1][st], xim[st], yi1, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[0][j] = cadd(acc[0][j], cmul(pw[j], C2<double>{yr0[j], yi0[j]}));
        acc[1][j] = cadd(acc[1][j], cmul(pw[4 + j], C2<double>{yr1[j], yi1[j]}));
      }
      if (q == 0) acc[0][0].re += a0 * (logw + ot[12]);
    }
  }
  if (!colok) return;
  const int64_t tgt = (int64_t)iy * G + ix;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int lr = 16 * t + q + 4 * j;
      if (lr <= P) st2<double>(&Bl[((int64_t)lr * nd + r) * nb + tgt], acc[t][j]);
    }
}

// ------------------------------------------------------------------ L2L
// Work item: 256 lanes over (child box, density, coefficient) triples of one
// level; on coarse levels four or sixteen lanes per triple over every fourth
// or sixteenth parent coefficient, added over the quad or the row.
template <class T>
__global__ void kf_l2l(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                       const int32_t *__restrict__ mask, int lc, int P,
                       const V2<T> *__restrict__ l2l) {
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R;
  const int Gc = 1 << lc, Gp = Gc / 2;
  const int64_t nbc = (int64_t)Gc * Gc, nbp = nbc / 4;
  const int split = shift_split(lc);
  const int64_t tid = (int64_t)br.blk * 256 + threadIdx.x;
  if (tid >= nbc * nd * (P + 1) * split) return;  // whole lane groups
  const gptr<V2<T>> Bp = rw((V2<T> *)d.loc + level_base(lc - 1, P, nd));
  const gptr<V2<T>> Bc = rw((V2<T> *)d.loc + level_base(lc, P, nd));
  const int64_t o = tid / split;
  const int sq = (int)(tid & (split - 1));
  const int box = (int)(o % nbc);
  const int64_t rest = o / nbc;
  const int r = (int)(rest % nd), j = (int)(rest / nd);
  const int ix = box % Gc, iy = box / Gc;
  const int c = (iy & 1) * 2 + (ix & 1);
  const int parent = (iy >> 1) * Gp + (ix >> 1);
  const V2<T> *row = l2l + ((int64_t)c * (P + 1) + j) * (P + 1);
  C2<T> acc = {T(0), T(0)};
  // four terms' loads in flight at a time, summed in k order
  int k = j + sq;
  for (; k + 3 * split <= P; k += 4 * split) {
    C2<T> mv[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      mv[u] = ld2<T>(row + k + u * split);
      bv[u] = ld2<T>(&Bp[((int64_t)(k + u * split) * nd + r) * nbp + parent]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = cadd(acc, cmul(mv[u], bv[u]));
  }
  for (; k <= P; k += split)
    acc = cadd(acc, cmul(ld2<T>(row + k), ld2<T>(&Bp[((int64_t)k * nd + r) * nbp + parent])));
  if (split == 16) {
    acc.re = row_sum16(acc.re);
    acc.im = row_sum16(acc.im);
    if (sq != 0) return;
  } else if (split == 4) {
    acc.re = quad_sum(acc.re);
    acc.im = quad_sum(acc.im);
    if (sq != 0) return;
  }
  const gptr<V2<T>> dst = &Bc[((int64_t)j * nd + r) * nbc + box];
  st2<T>(dst, cadd(ld2<T>(dst), acc));
}

// ------------------------------------------------------- symmetric near field
// The near field of two neighbouring leaves A and B needs phi(|x_i - x_j|) for
// every i in A and j in B twice: in the sum of each target of A over B's
// densities, and in the sum of each target of B over A's.  The wavefront of A
// forms each such phi once for the neighbours that follow A in the grid's
// row-major order (E, and NW, N, NE in the row above): lane i adds phi t_j to
// its own sum, and the sum over i of phi t_i, the contribution of A to source
// j, is reduced across the lanes and stored in one of four partial-sum slots
// of j, chosen by the direction from j's leaf to A.  Every slot has a single
// writer, so the results do not depend on the order in which wavefronts run;
// a combine pass adds the slots to the leaf pass's output.

constexpr int kDppRor8 = 0x128;        // row_ror:8 (lane l ^ 8 within a row)
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror (lane l ^ 7 within 8)
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]

template <int C>
__device__ __forceinline__ double dpp_f64(double v) {
  // every lane's source lane is valid for these controls, so no old value
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), C, 0xf, 0xf, false);
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), C, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// One halving step of a reduce-scatter across lane bit B: lanes whose bit B is
// clear return lo plus the partner's lo, the others hi plus the partner's hi,
// the partner differing in bit B (at B = 2 also in bits 1 and 0).  Bits 5 and
// 4 use the lane-swap instructions, which exchange the upper half of one
// register's lanes (or odd rows) with the lower half (even rows) of another,
// so the two registers then hold both addends without selects.
template <int B>
__device__ __forceinline__ double lane_halve(double lo, double hi, int lane) {
  if constexpr (B == 5 || B == 4) {
    const unsigned lh = (unsigned)__double2hiint(lo), ll = (unsigned)__double2loint(lo);
    const unsigned hh = (unsigned)__double2hiint(hi), hl = (unsigned)__double2loint(hi);
    const auto sh = B == 5 ? __builtin_amdgcn_permlane32_swap(lh, hh, false, false)
                           : __builtin_amdgcn_permlane16_swap(lh, hh, false, false);
    const auto sl = B == 5 ? __builtin_amdgcn_permlane32_swap(ll, hl, false, false)
                           : __builtin_amdgcn_permlane16_swap(ll, hl, false, false);
    return __hiloint2double((int)sh[0], (int)sl[0]) + __hiloint2double((int)sh[1], (int)sl[1]);
  } else {
    constexpr int C = B == 3 ? kDppRor8 : B == 2 ? kDppHalfMirror : B == 1 ? kDppXor2 : kDppXor1;
    const bool up = (lane >> B) & 1;
    return (up ? hi : lo) + dpp_f64<C>(up ? lo : hi);
  }
}

// one full summing step across lane bit B <= 2 (B = 2: the partner l ^ 7)
template <int B>
__device__ __forceinline__ double lane_fold(double v) {
  constexpr int C = B == 2 ? kDppHalfMirror : B == 1 ? kDppXor2 : kDppXor1;
  return v + dpp_f64<C>(v);
}

// Sums of eight per-lane values over each aligned group of 2^LW lanes
// (LW = 3..6): three halving steps over the group's top lane bits, then full
// steps over the rest.  Lane l returns the group total of value
// (l >> (LW - 3)) & 7; the partner masks of the steps are linearly
// independent, so each total covers every lane of the group once.
template <int LW>
__device__ __forceinline__ double lane_sum8(const double (&T)[8], int lane) {
  double a[4], b[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = lane_halve<LW - 1>(T[k], T[k + 4], lane);
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] = lane_halve<LW - 2>(a[k], a[k + 2], lane);
  double c = lane_halve<LW - 3>(b[0], b[1], lane);
  if constexpr (LW >= 6) c = lane_fold<2>(c);
  if constexpr (LW >= 5) c = lane_fold<1>(c);
  if constexpr (LW >= 4) c = lane_fold<0>(c);
  return c;
}

// Where the symmetric sums of a source range go.  Slot d of a node in leaf B
// holds the sum from the leaf A that takes the pair (A, B): d = 3 for A the
// west neighbour of B, d = 0, 1, 2 for A in the row below at column offset
// d - 1.  Seen from A at column ix, a source j of the row above lies in column
// ix - 1, ix or ix + 1, i.e. slot 2, 1 or 0: dir(j) = dbase - (j >= bnd1) -
// (j >= bnd2) with dbase = 2 and bnd1, bnd2 the first nodes of columns ix and
// ix + 1 there; the E leaf has dbase = 3 and no bounds.
struct SymDst {
  double *part;
  int64_t n;
  int dbase, bnd1, bnd2;
  bool accum;  // add to the slots (a later pass over the same target leaf)
};

// One batch of up to eight sources of a symmetric range for the W = 2^LW
// lanes of a group: cnt (per group) sources from j.  Adds the target sums to
// acc and stores the source sums.  Two halves of four sources: their loads,
// then their table reads, then their arithmetic.  FULL (eight sources,
// wave-uniform): the coordinates and densities are read from one base address
// at constant offsets (wide scalar loads, one wait); otherwise each index is
// clamped to jmax and a padding source gets density 0 (the padded last batch
// and the lane-group form, whose loads are per lane).
template <int K, int LW, bool FULL, class PXY, class PT, class PTAB>
__device__ __forceinline__ void sym_batch(double xi, double yi, double ti, PXY xy2, PT t, int j,
                                          int cnt, int jmax, PTAB tab, int lane,
                                          const SymDst &o, double &acc) {
  double T[8];
  const int k = (lane >> (LW - 3)) & 7;
  const int jk = j + k;
  const bool wr = (lane & ((1 << (LW - 3)) - 1)) == 0 && k < cnt;
  const gptr<double> dst =
      rw(o.part + (int64_t)(o.dbase - (jk >= o.bnd1) - (jk >= o.bnd2)) * o.n + jk);
  const double prev = (o.accum && wr) ? *dst : 0.0;
  const auto pxy = xy2 + 2 * j;
  const auto pt = t + j;
#pragma unroll
  for (int h = 0; h < 8; h += 4) {
    double sx[4], sy[4], tj[4], r2[4], ic[4], lc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if constexpr (FULL) {
        sx[i] = pxy[2 * (h + i)];
        sy[i] = pxy[2 * (h + i) + 1];
        tj[i] = pt[h + i];
      } else {
        const int jj = j + h + i < jmax ? j + h + i : jmax;
        sx[i] = xy2[2 * jj];
        sy[i] = xy2[2 * jj + 1];
        const double tv = t[jj];
        tj[i] = h + i < cnt ? tv : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double dx = xi - sx[i], dy = yi - sy[i];
      r2[i] = fma(dy, dy, dx * dx);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(r2[i]) >> 32);
      const double2 e = *reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(tab) +
                                                           near_log_offset(hi));
      ic[i] = e.x;
      lc[i] = e.y;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double ph = r2[i] * near_log_core(r2[i], ic[i], lc[i]);
      if constexpr (K == 4) ph *= r2[i];
      acc = fma(ph, tj[i], acc);
      T[h + i] = ph * ti;
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the halves apart (registers)
  }
  const double v = lane_sum8<LW>(T, lane);
  if (wr) *dst = prev + v;
}

// Symmetric range [js, je) for all 64 lanes (one target per lane).  Full
// batches of eight sources run as a pipeline: the next batch's coordinates
// and densities (wave-uniform, wide scalar loads from one base address) are
// requested once the current batch's last table reads have been waited for,
// so the scalar loads are in flight during that batch's remaining logarithms,
// its cross-lane reduction and its store.  (Scalar loads return out of order
// and share their completion counter with the LDS reads, so a scalar load
// issued before a table read would be waited for with it.)  After a batch's
// reduction the eight lanes holding source k's sum all hold it; lane
// 8k + m keeps the sum of batch m of each group of eight batches, and a group
// is stored at once: 64 consecutive sources, one store per lane.  The last
// batch is padded.
template <int K, class PXY, class PT, class PTAB>
__device__ __forceinline__ double near_sym64(double xi, double yi, double ti, PXY xy2, PT t,
                                             int js, int je, PTAB tab, int lane,
                                             const SymDst &o) {
  double acc = 0.0;
  const int nfull = (je - js) >> 3;
  int j = js;
  if (nfull > 0) {
    double sx[8], sy[8], tj[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      sx[i] = xy2[2 * (j + i)];
      sy[i] = xy2[2 * (j + i) + 1];
      tj[i] = t[j + i];
    }
    const int k = lane >> 3, m = lane & 7;
    double held = 0.0;
    for (int bi = 0; bi < nfull; ++bi, j += 8) {
      double T[8], r2[8], ic[8], lc[8];
#pragma unroll
      for (int h = 0; h < 8; h += 4) {
#pragma unroll
        for (int i = h; i < h + 4; ++i) {
          const double dx = xi - sx[i], dy = yi - sy[i];
          r2[i] = fma(dy, dy, dx * dx);
        }
#pragma unroll
        for (int i = h; i < h + 4; ++i) {
          const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(r2[i]) >> 32);
          const double2 e = *reinterpret_cast<const double2 *>(
              reinterpret_cast<const char *>(tab) + near_log_offset(hi));
          ic[i] = e.x;
          lc[i] = e.y;
        }
      }
      // the logarithms' first step consumes every table entry: all LDS reads
      // of this batch have completed past this point
      double rr[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) rr[i] = fma(__builtin_amdgcn_frexp_mant(r2[i]), ic[i], -1.0);
      __builtin_amdgcn_sched_barrier(0);
      double ntj[8], nsx[8], nsy[8];
      const int jn = bi + 1 < nfull ? j + 8 : j;  // the last batch reloads its own
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        nsx[i] = xy2[2 * (jn + i)];
        nsy[i] = xy2[2 * (jn + i) + 1];
        ntj[i] = t[jn + i];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        double ph = r2[i] * near_log_rest(r2[i], rr[i], lc[i]);
        if constexpr (K == 4) ph *= r2[i];
        acc = fma(ph, tj[i], acc);
        T[i] = ph * ti;
      }
      const double v = lane_sum8<6>(T, lane);
      const int bm = bi & 7;
      held = m == bm ? v : held;
      if (bm == 7 || bi + 1 == nfull) {
        // batches j - 8 bm .. j of this group: lane (k, m) stores batch m's source k
        const int jk = j - 8 * bm + 8 * m + k;
        if (m <= bm) {
          const gptr<double> dst =
              rw(o.part + (int64_t)(o.dbase - (jk >= o.bnd1) - (jk >= o.bnd2)) * o.n + jk);
          *dst = (o.accum ? *dst : 0.0) + held;
        }
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        sx[i] = nsx[i];
        sy[i] = nsy[i];
        tj[i] = ntj[i];
      }
    }
  }
  if (j < je) sym_batch<K, 6, false>(xi, yi, ti, xy2, t, j, je - j, je - 1, tab, lane, o, acc);
  return acc;
}

// Symmetric range [js, je) for 64/W groups of W = 2^LW lanes on the same
// targets: group g takes the sub-range [js + len g / ng, js + len (g+1) / ng)
// in batches of eight (the batch count is that of the longest sub-range, so
// every group runs the same steps; a group past its end has no valid source).
template <int K, int LW, class PXY, class PT, class PTAB>
__device__ __forceinline__ double near_sym_split(double xi, double yi, double ti, PXY xy2, PT t,
                                                 int js, int je, PTAB tab, int lane,
                                                 const SymDst &o) {
  constexpr int ng = 64 >> LW;
  const int g = lane >> LW, len = je - js;
  const int gs = js + len * g / ng, ge = js + len * (g + 1) / ng;
  const int nb = ((len + ng - 1) / ng + 7) / 8;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) {
    const int j = gs + 8 * b;
    const int cnt = ge - j;
    sym_batch<K, LW, false>(xi, yi, ti, xy2, t, j, cnt < 0 ? 0 : (cnt > 8 ? 8 : cnt), je - 1, tab,
                            lane, o, acc);
  }
  return acc;
}

// FP32 forms of the lane exchanges and of the symmetric batch (the FP32 near
// field of the mixed and near32 matvecs): a 32-bit value moves in one swap or
// DPP operation.
template <int C>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), C, 0xf, 0xf, false));
}
template <int B>
__device__ __forceinline__ float lane_halve_f(float lo, float hi, int lane) {
  if constexpr (B == 5 || B == 4) {
    const auto sw = B == 5 ? __builtin_amdgcn_permlane32_swap((unsigned)__float_as_int(lo),
                                                               (unsigned)__float_as_int(hi),
                                                               false, false)
                           : __builtin_amdgcn_permlane16_swap((unsigned)__float_as_int(lo),
                                                               (unsigned)__float_as_int(hi),
                                                               false, false);
    return __int_as_float((int)sw[0]) + __int_as_float((int)sw[1]);
  } else {
    constexpr int C = B == 3 ? kDppRor8 : B == 2 ? kDppHalfMirror : B == 1 ? kDppXor2 : kDppXor1;
    const bool up = (lane >> B) & 1;
    return (up ? hi : lo) + dpp_f32<C>(up ? lo : hi);
  }
}
template <int B>
__device__ __forceinline__ float lane_fold_f(float v) {
  constexpr int C = B == 2 ? kDppHalfMirror : B == 1 ? kDppXor2 : kDppXor1;
  return v + dpp_f32<C>(v);
}
template <int LW>
__device__ __forceinline__ float lane_sum8_f(const float (&T)[8], int lane) {
  float a[4], b[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = lane_halve_f<LW - 1>(T[k], T[k + 4], lane);
#pragma unroll
  for (int k = 0; k < 2; ++k) b[k] = lane_halve_f<LW - 2>(a[k], a[k + 2], lane);
  float c = lane_halve_f<LW - 3>(b[0], b[1], lane);
  if constexpr (LW >= 6) c = lane_fold_f<2>(c);
  if constexpr (LW >= 5) c = lane_fold_f<1>(c);
  if constexpr (LW >= 4) c = lane_fold_f<0>(c);
  return c;
}

// One FP32 batch of up to eight sources of one neighbouring leaf (coordinates
// relative to its centre, the target moved into that frame) for the W = 2^LW
// lanes of a group.  phi is formed from log2, so the source sums are stored
// times ln 2 (the combine pass applies the 1/2 of phi = (1/2) r^k log r^2).
template <int K, int LW, bool FULL, class PF>
__device__ __forceinline__ void sym_batch_f(float xc, float yc, float ti, PF ux, PF uy, PF tf,
                                            int j, int cnt, int jmax, int lane,
                                            const SymDst &o, float &acc) {
  float T[8];
  const int k = (lane >> (LW - 3)) & 7;
  const int jk = j + k;
  const bool wr = (lane & ((1 << (LW - 3)) - 1)) == 0 && k < cnt;
  const gptr<double> dst = rw(o.part + (int64_t)o.dbase * o.n + jk);
  const double prev = (o.accum && wr) ? *dst : 0.0;
  float sx[8], sy[8], tj[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if constexpr (FULL) {
      sx[i] = ux[j + i];
      sy[i] = uy[j + i];
      tj[i] = tf[j + i];
    } else {
      const int jj = j + i < jmax ? j + i : jmax;
      sx[i] = ux[jj];
      sy[i] = uy[jj];
      const float tv = tf[jj];
      tj[i] = i < cnt ? tv : 0.0f;
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float dx = xc - sx[i], dy = yc - sy[i];
    const float ph = phi_r2f<K>(dx * dx + dy * dy);
    acc += ph * tj[i];
    T[i] = ph * ti;
  }
  const float v = lane_sum8_f<LW>(T, lane);
  if (wr) *dst = prev + 0.69314718055994530942 * (double)v;
}

// The FP32 symmetric sums of one neighbouring leaf [js, je) into slot dbase:
// all 64 lanes on one target each (batches of eight, the last padded), or
// 64/W groups of W = 2^LW lanes on the same targets over 1/(64/W) of the
// sources each.
template <int K, int LW, class PF>
__device__ __forceinline__ float near_sym_f(float xc, float yc, float ti, PF ux, PF uy, PF tf,
                                            int js, int je, int lane, const SymDst &o) {
  float acc = 0.0f;
  if constexpr (LW == 6) {
    int j = js;
    for (; j + 8 <= je; j += 8)
      sym_batch_f<K, 6, true>(xc, yc, ti, ux, uy, tf, j, 8, j + 7, lane, o, acc);
    if (j < je) sym_batch_f<K, 6, false>(xc, yc, ti, ux, uy, tf, j, je - j, je - 1, lane, o, acc);
  } else {
    constexpr int ng = 64 >> LW;
    const int g = lane >> LW, len = je - js;
    const int gs = js + len * g / ng, ge = js + len * (g + 1) / ng;
    const int nb = ((len + ng - 1) / ng + 7) / 8;
    for (int b = 0; b < nb; ++b) {
      const int j = gs + 8 * b;
      const int cnt = ge - j;
      sym_batch_f<K, LW, false>(xc, yc, ti, ux, uy, tf, j, cnt < 0 ? 0 : (cnt > 8 ? 8 : cnt),
                                je - 1, lane, o, acc);
    }
  }
  return acc;
}

// ------------------------------------------------------------------ leaf
// One wavefront per leaf: each lane one target node.  Far field by Horner on
// the leaf's incoming expansions (L2P) combined with U_r; near field by
// direct phi over the 3x3 neighbouring leaves (step 2: direct evaluation).
// Held to 96 VGPRs, five wavefronts per SIMD, at k = 2 (the FP64 form
// otherwise takes 121: four): at n = 2^20 the FP64 leaf pass took 0.441
// against 0.454 ms, with a few lane-group set-up values spilled; six were no
// faster.  k = 4 (one more multiply a pair) is held to 80 VGPRs, six
// wavefronts: 0.62 against 0.64 ms.
template <class T, class TN, int K>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(K == 4 ? 6 : 5))) void kf_leaf_eval(const SysDev *__restrict__ sys,
                                                   const BlkRef *__restrict__ tab,
                                                   const int32_t *__restrict__ mask, int P,
                                                   int in, int out,
                                                   const double *__restrict__ logtab) {
  constexpr int R = Rank<K>::R;
  __shared__ double ltab[kNearLogTab];
  const BlkRef br = tab[xcd_remap(blockIdx.x, gridDim.x)];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int L = d.L;
  const double h = d.h;
  const int G = 1 << L;
  const int nleaf = G * G;
  const int leaf = br.blk;
  const int lane = threadIdx.x;
  const cptr<double> x = ro(d.x);
  const cptr<double> y = ro(d.y);
  const cptr<float> ux = ro(d.ux);
  const cptr<float> uy = ro(d.uy);
  const cptr<double> t = ro(d.v[in]);
  const cptr<double> xy2 = ro((const double *)d.xy2);
  const cptr<int32_t> start = ro(d.leaf_start);
  const cptr<V2<T>> Bleaf = ro((const V2<T> *)d.loc + level_base(L, P, R));
  const gptr<double> ytree = rw(d.v[out]);
  if constexpr (std::is_same<TN, double>::value && K % 2 == 0) {
    for (int i = lane; i < kNearLogTab; i += 64) ltab[i] = logtab[i];
    __syncthreads();
  }
  const int b = start[leaf], e = start[leaf + 1];
  if (b == e) return;
  const int ix = leaf % G, iy = leaf / G;
  const double w = 2.0 * h / G, invw = G / (2.0 * h);
  const double cx = -h + (ix + 0.5) * w, cy = -h + (iy + 0.5) * w;
  const int r0 = iy > 0 ? iy - 1 : 0, r1 = iy + 1 < G ? iy + 1 : G - 1;
  const int c0 = ix > 0 ? ix - 1 : 0, c1 = ix + 1 < G ? ix + 1 : G - 1;
  // FP64 near field: the own leaf directly, the E neighbour and the row above
  // symmetrically (the W neighbour and the row below deliver their pairs
  // through this leaf's partial-sum slots; a slot whose writer leaf is absent
  // or empty is cleared here)
  // (the FP32 near fields, of the mixed and near32 matvecs, take the same
  // pairs symmetrically, leaf by leaf in each leaf's own frame)
  constexpr bool kSym = std::is_same<TN, double>::value;
  int eE = e, us = 0, ue = 0, ub1 = 0, ub2 = 0, zmask = 0;
  if constexpr (kSym) {
    if (ix + 1 < G) eE = start[leaf + 2];
    if (iy + 1 < G) {
      const int rb = (iy + 1) * G;
      us = start[rb + c0];
      ue = start[rb + c1 + 1];
      ub1 = start[rb + ix];
      ub2 = start[rb + ix + 1];
    }
  }
  if (!(ix > 0 && start[leaf - 1] < b)) zmask |= 8;
#pragma unroll
  for (int dd = 0; dd < 3; ++dd) {
    const int col = ix + dd - 1;
    const bool has = iy > 0 && col >= 0 && col < G &&
                     start[(iy - 1) * G + col] < start[(iy - 1) * G + col + 1];
    if (!has) zmask |= 1 << dd;
  }
  for (int i0 = b; i0 < e; i0 += 64) {
    // a later pass over this leaf adds to the source sums the first one stored
    // (possibly from other lanes): the barrier orders those accesses
    if (i0 > b) __syncthreads();
    // A pass with at most 32 targets left (the tail of a leaf of more than 64
    // nodes, or a small leaf) runs G = 64/W groups of W lanes on the same W
    // targets, each group over 1/G of every source range, and sums the groups'
    // partial sums: the lanes a plain pass would leave idle share the work.
    const int rem = e - i0;
    const int W = rem <= 8 ? 8 : rem <= 16 ? 16 : rem <= 32 ? 32 : 64;
    const int gi = lane / W, li = lane % W;
    const int i = i0 + li;
    const bool act = li < rem;
    const int ii = act ? i : b;
    const double xi = x[ii], yi = y[ii];
    // far field
    T far = T(0);
    {
      C2<T> z;
      if constexpr (std::is_same<T, float>::value)
        z = {ux[ii] * (float)invw, uy[ii] * (float)invw};
      else
        z = {(xi - cx) * invw, (yi - cy) * invw};
      T u[R];
      ufac<K, T>(xi, yi, u);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C2<T> acc = ld2<T>(&Bleaf[((int64_t)P * R + r) * nleaf + leaf]);
        for (int k = P - 1; k >= 0; --k) {
          C2<T> bk = ld2<T>(&Bleaf[((int64_t)k * R + r) * nleaf + leaf]);
          acc = cadd(cmul(acc, z), bk);
        }
        far += u[r] * acc.re;
      }
    }
    // near field
    TN nearv = TN(0);
    if constexpr (kSym) {
      // the lane index, opaque to the compiler: the lane-group forms' per-lane
      // set-up (group sub-ranges of each range, for each group width) is then
      // computed where it is used instead of being hoisted out of the pass
      // loop and held in registers through the whole kernel
      int ln = lane;
      asm volatile("" : "+v"(ln));
      const double ti = act ? t[i] : 0.0;
      const SymDst oE{d.npart, d.n, 3, INT_MAX, INT_MAX, i0 > b};
      const SymDst oU{d.npart, d.n, 2, ub1, ub2, i0 > b};
      if (W == 64) {
        nearv = near_range8<K>(xi, yi, xy2, t, b, e, ltab);
        if (eE > e) nearv += near_sym64<K>(xi, yi, ti, xy2, t, e, eE, ltab, ln, oE);
        if (ue > us) nearv += near_sym64<K>(xi, yi, ti, xy2, t, us, ue, ltab, ln, oU);
      } else {
        const int ng = 64 / W;
        const int len = e - b;
        nearv = near_range<K>(xi, yi, xy2, t, b + len * gi / ng, b + len * (gi + 1) / ng, ltab);
        if (W == 32) {
          if (eE > e) nearv += near_sym_split<K, 5>(xi, yi, ti, xy2, t, e, eE, ltab, ln, oE);
          if (ue > us) nearv += near_sym_split<K, 5>(xi, yi, ti, xy2, t, us, ue, ltab, ln, oU);
        } else if (W == 16) {
          if (eE > e) nearv += near_sym_split<K, 4>(xi, yi, ti, xy2, t, e, eE, ltab, ln, oE);
          if (ue > us) nearv += near_sym_split<K, 4>(xi, yi, ti, xy2, t, us, ue, ltab, ln, oU);
        } else {
          if (eE > e) nearv += near_sym_split<K, 3>(xi, yi, ti, xy2, t, e, eE, ltab, ln, oE);
          if (ue > us) nearv += near_sym_split<K, 3>(xi, yi, ti, xy2, t, us, ue, ltab, ln, oU);
        }
        for (int o = W; o < 64; o <<= 1) nearv += __shfl_xor(nearv, o);
      }
      nearv *= near_scale<K>();
    } else {
      // coordinates relative to each point's own leaf centre: the target is
      // moved into the frame of each neighbouring leaf once, so a pair costs
      // one subtraction per axis; densities from the FP32 copy.  The own leaf
      // one-sided, the E leaf and the three leaves of the row above
      // symmetrically, one leaf (one frame) at a time.
      int ln = lane;
      asm volatile("" : "+v"(ln));
      const float uxi = ux[ii], uyi = uy[ii];
      const cptr<float> tf = ro((const float *)d.t32);
      const float ti = act ? tf[i] : 0.0f;
      const int ng = 64 / W;
      if (W == 64) {
        nearv = near_range_f32<K>(uxi, uyi, ux, uy, tf, b, e);
      } else {
        const int len = e - b;
        for (int j = b + len * gi / ng; j < b + len * (gi + 1) / ng; ++j) {
          const float dx = uxi - ux[j], dy = uyi - uy[j];
          nearv += phi_r2f<K>(dx * dx + dy * dy) * tf[j];
        }
      }
      const auto fwd = [&](int row, int col, int dir) {
        const int js = start[row * G + col], je = start[row * G + col + 1];
        if (je <= js) return;
        const float uyc = uyi + (float)((iy - row) * w);
        const float uxc = uxi + (float)((ix - col) * w);
        const SymDst o{d.npart, d.n, dir, INT_MAX, INT_MAX, i0 > b};
        if (W == 64)
          nearv += near_sym_f<K, 6>(uxc, uyc, ti, ux, uy, tf, js, je, ln, o);
        else if (W == 32)
          nearv += near_sym_f<K, 5>(uxc, uyc, ti, ux, uy, tf, js, je, ln, o);
        else if (W == 16)
          nearv += near_sym_f<K, 4>(uxc, uyc, ti, ux, uy, tf, js, je, ln, o);
        else
          nearv += near_sym_f<K, 3>(uxc, uyc, ti, ux, uy, tf, js, je, ln, o);
      };
      if (ix + 1 < G) fwd(iy, ix + 1, 3);
      if (iy + 1 < G)
        for (int col = c0; col <= c1; ++col) fwd(iy + 1, col, ix - col + 1);
      for (int o = W; o < 64; o <<= 1) nearv += __shfl_xor(nearv, o);
      nearv *= phi_scale_f<K>();
    }
    if (act && gi == 0) {
      ytree[i] = (double)far + (double)nearv;
#pragma unroll
      for (int dd = 0; dd < 4; ++dd)
        if ((zmask >> dd) & 1) d.npart[(int64_t)dd * d.n + i] = 0.0;
    }
  }
}

// ------------------------------------------------------------------ targets
// Evaluation of the interpolant at arbitrary targets (eq. phs_interp): inside
// the tree domain by L2P + direct phi over the 3x3 neighbouring leaves;
// outside it by descending the tree and evaluating outgoing expansions of
// boxes far enough from the target (|z - c| >= 1.8 w), direct sums at leaves.
template <int K>
__global__ void k_eval_targets(const double *__restrict__ tg, int64_t m, double cxn,
                               double cyn, double rho, const double *__restrict__ x,
                               const double *__restrict__ y, const double *__restrict__ wt,
                               const int32_t *__restrict__ start, int L, double h, int P,
                               const double2 *__restrict__ Aall,
                               const double2 *__restrict__ Bleaf,
                               const double *__restrict__ beta, int d,
                               double *__restrict__ out, const double2 *__restrict__ xy2,
                               const double *__restrict__ logtab) {
  constexpr int R = Rank<K>::R;
  const int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (it >= m) return;
  const double xi = (tg[2 * it] - cxn) * rho, yi = (tg[2 * it + 1] - cyn) * rho;
  // polynomial part
  double poly = 0.0;
  {
    double px[8], py[8];
    px[0] = py[0] = 1.0;
    for (int q = 1; q <= d; ++q) {
      px[q] = px[q - 1] * xi;
      py[q] = py[q - 1] * yi;
    }
    int col = 0;
    for (int tdeg = 0; tdeg <= d; ++tdeg)
      for (int a = tdeg; a >= 0; --a) poly += beta[col++] * px[a] * py[tdeg - a];
  }
  double u[R];
  ufac<K, double>(xi, yi, u);
  const int G = 1 << L;
  const int nleaf = G * G;
  double far = 0.0, nearv = 0.0;
  const bool inside = fabs(xi) <= h && fabs(yi) <= h;
  if (inside) {
    const double scale = G / (2.0 * h);
    int ix = (int)floor((xi + h) * scale), iy = (int)floor((yi + h) * scale);
    ix = ix < 0 ? 0 : (ix >= G ? G - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= G ? G - 1 : iy);
    const int leaf = iy * G + ix;
    const double w = 2.0 * h / G;
    const double cx = -h + (ix + 0.5) * w, cy = -h + (iy + 0.5) * w;
    const C2<double> z = {(xi - cx) * scale, (yi - cy) * scale};
    for (int r = 0; r < R; ++r) {
      C2<double> acc = ld2<double>(&Bleaf[((int64_t)P * R + r) * nleaf + leaf]);
      for (int k = P - 1; k >= 0; --k)
        acc = cadd(cmul(acc, z), ld2<double>(&Bleaf[((int64_t)k * R + r) * nleaf + leaf]));
      far += u[r] * acc.re;
    }
    const int r0 = iy > 0 ? iy - 1 : 0, r1 = iy + 1 < G ? iy + 1 : G - 1;
    const int c0 = ix > 0 ? ix - 1 : 0, c1 = ix + 1 < G ? ix + 1 : G - 1;
    for (int row = r0; row <= r1; ++row) {
      const int js = start[row * G + c0], je = start[row * G + c1 + 1];
      nearv += near_scale<K>() * near_range<K>(xi, yi, (const double *)xy2, wt, js, je, logtab);
    }
  } else {
    // explicit-stack descent from level 2
    int stk_l[64];
    int stk_b[64];
    int sp = 0;
    for (int b0 = 0; b0 < 16; ++b0) {
      stk_l[sp] = 2;
      stk_b[sp] = b0;
      ++sp;
    }
    while (sp > 0) {
      --sp;
      const int l = stk_l[sp], box = stk_b[sp];
      const int Gl = 1 << l;
      const double wl = 2.0 * h / Gl;
      const int bx = box % Gl, by = box / Gl;
      const double ccx = -h + (bx + 0.5) * wl, ccy = -h + (by + 0.5) * wl;
      const double ddx = xi - ccx, ddy = yi - ccy;
      const double dist2 = ddx * ddx + ddy * ddy;
      if (dist2 >= (1.8 * wl) * (1.8 * wl)) {
        const int64_t nbl = (int64_t)Gl * Gl;
        const double2 *Al = Aall + level_base(l, P, R);
        const C2<double> wz = {ddx / wl, ddy / wl};
        const double den = wz.re * wz.re + wz.im * wz.im;
        const C2<double> uinv = {wz.re / den, -wz.im / den};
        const double lw = log(wl) + 0.5 * log(den);
        for (int r = 0; r < R; ++r) {
          C2<double> acc = ld2<double>(&Al[((int64_t)P * R + r) * nbl + box]);
          for (int k = P - 1; k >= 1; --k)
            acc = cadd(cmul(acc, uinv), ld2<double>(&Al[((int64_t)k * R + r) * nbl + box]));
          acc = cmul(acc, uinv);
          const double a0 = ld2<double>(&Al[(int64_t)r * nbl + box]).re;
          far += u[r] * (a0 * lw + acc.re);
        }
      } else if (l == L) {
        const int js = start[box], je = start[box + 1];
        nearv += near_scale<K>() * near_range<K>(xi, yi, (const double *)xy2, wt, js, je, logtab);
      } else {
        for (int c = 0; c < 4; ++c) {
          stk_l[sp] = l + 1;
          stk_b[sp] = (2 * by + (c >> 1)) * (2 * Gl) + 2 * bx + (c & 1);
          ++sp;
        }
      }
    }
  }
  out[it] = poly + far + nearv;
}

// ------------------------------------------------------------------ host
double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Timing label of a per-level launch: "m2m_5", "l2l_7", ...
const char *level_name(const char *base, int l) {
  static const char *m2m[] = {"m2m_0", "m2m_1", "m2m_2", "m2m_3", "m2m_4", "m2m_5", "m2m_6",
                              "m2m_7", "m2m_8", "m2m_9", "m2m_10", "m2m_11"};
  static const char *l2l[] = {"l2l_0", "l2l_1", "l2l_2", "l2l_3", "l2l_4", "l2l_5", "l2l_6",
                              "l2l_7", "l2l_8", "l2l_9", "l2l_10", "l2l_11"};
  const int i = l < 0 ? 0 : (l > 11 ? 11 : l);
  return base[0] == 'm' ? m2m[i] : l2l[i];
}

// Upward pass, M2L and downward pass at order P with the tables of that order,
// for the even-k systems of the forest.  `m2l_name` labels the M2L launch in
// the per-kernel timing.
template <class T>
void far_field(Forest &F, const int32_t *mask, int in, int P, const LogTables &lt,
               const char *m2l_name, hipStream_t s) {
  const bool fp64 = std::is_same<T, double>::value;
  const V2<T> *M2M = fp64 ? (const V2<T> *)lt.M2M64 : (const V2<T> *)lt.M2M32;
  const V2<T> *L2L = fp64 ? (const V2<T> *)lt.L2L64 : (const V2<T> *)lt.L2L32;
  const T *Ht = fp64 ? (const T *)lt.Ht64 : (const T *)lt.Ht32;
  const int maxL = F.maxL_log;
  // P2M at the leaves, per order k (the Hadamard factors differ)
  {
    const int gpw = p2m_leaves_per_wave(P);
    const Tab t2 = forest_tab(F, tab_key(2, 2, gpw, 0), s);
    if (t2.count) {
      const int ch = p2m_chunk<T>(P, Rank<2>::R, gpw);
      PHS_LAUNCH("p2m", s,
                 kf_p2m<T, 2><<<(unsigned)t2.count, 256,
                                4 * p2m_wave_bytes<T>(P, Rank<2>::R, gpw, ch), s>>>(
                     F.dsys, t2.d, mask, P, in, ch));
    }
    const Tab t4 = forest_tab(F, tab_key(2, 4, gpw, 0), s);
    if (t4.count) {
      const int ch = p2m_chunk<T>(P, Rank<4>::R, gpw);
      PHS_LAUNCH("p2m", s,
                 kf_p2m<T, 4><<<(unsigned)t4.count, 256,
                                4 * p2m_wave_bytes<T>(P, Rank<4>::R, gpw, ch), s>>>(
                     F.dsys, t4.d, mask, P, in, ch));
    }
  }
  // upward pass
  // FP64 with the standard orders: row segments through LDS on the deep levels
  const bool seg = fp64 && (P == 15 || P == 23 || P == 27 || P == 31);
  for (int lp = maxL - 1; lp >= 2; --lp) {
    if (seg && lp >= 4) {
      const Tab tb = forest_tab(F, tab_key(13, 0, P, lp), s);
      if (tb.count) {
        const unsigned nb = (unsigned)tb.count;
        const double *Rm = lt.Rm64;
        const double2 *Ph = lt.Ph64;
        const char *nm = level_name("m2m", lp);
        switch (P) {
          case 15: PHS_LAUNCH(nm, s, kf_m2m_seg<15><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lp, Rm, Ph)); break;
          case 23: PHS_LAUNCH(nm, s, kf_m2m_seg<23><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lp, Rm, Ph)); break;
          case 27: PHS_LAUNCH(nm, s, kf_m2m_seg<27><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lp, Rm, Ph)); break;
          default: PHS_LAUNCH(nm, s, kf_m2m_seg<31><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lp, Rm, Ph)); break;
        }
      }
      continue;
    }
    const Tab tb = forest_tab(F, tab_key(3, 0, P, lp), s);
    if (tb.count)
      PHS_LAUNCH(level_name("m2m", lp), s, kf_m2m<T><<<(unsigned)tb.count, 256, 0, s>>>(F.dsys, tb.d, mask, lp, P, M2M));
  }
  // outgoing -> incoming on every level: FP64 with the standard orders on
  // the matrix cores, otherwise on the vector units
  if (fp64 && (P == 15 || P == 23 || P == 27 || P == 31)) {
    const Tab tb = forest_tab(F, tab_key(10, 0, P, 0), s);
    if (tb.count) {
      const unsigned nblk = (unsigned)tb.count;
      const double *H = lt.Ht64, *O = lt.Off64;
      switch (P) {
        case 15:
          PHS_LAUNCH(m2l_name, s, kf_m2l_mfma<15><<<nblk, 64, 0, s>>>(F.dsys, tb.d, mask, H, O));
          break;
        case 23:
          PHS_LAUNCH(m2l_name, s, kf_m2l_mfma<23><<<nblk, 64, 0, s>>>(F.dsys, tb.d, mask, H, O));
          break;
        case 27:
          PHS_LAUNCH(m2l_name, s, kf_m2l_mfma<27><<<nblk, 64, 0, s>>>(F.dsys, tb.d, mask, H, O));
          break;
        default:
          PHS_LAUNCH(m2l_name, s, kf_m2l_mfma<31><<<nblk, 64, 0, s>>>(F.dsys, tb.d, mask, H, O));
          break;
      }
    }
  } else {
    const Tab tb = forest_tab(F, tab_key(5, 0, P, 0), s);
    const int lch = m2l_chunk(P);
    const int nchunks = (P + 1 + lch - 1) / lch;
    if (tb.count) {
      const unsigned nblk = (unsigned)tb.count;
      switch (lch) {
        case 16:
          PHS_LAUNCH(m2l_name, s, kf_m2l<T, 16><<<nblk, 256, 0, s>>>(F.dsys, tb.d, mask, P, Ht, nchunks));
          break;
        case 14:
          PHS_LAUNCH(m2l_name, s, kf_m2l<T, 14><<<nblk, 256, 0, s>>>(F.dsys, tb.d, mask, P, Ht, nchunks));
          break;
        case 12:
          PHS_LAUNCH(m2l_name, s, kf_m2l<T, 12><<<nblk, 256, 0, s>>>(F.dsys, tb.d, mask, P, Ht, nchunks));
          break;
        default:
          PHS_LAUNCH(m2l_name, s, kf_m2l<T, 8><<<nblk, 256, 0, s>>>(F.dsys, tb.d, mask, P, Ht, nchunks));
          break;
      }
    }
  }
  // downward pass
  for (int lc = 3; lc <= maxL; ++lc) {
    if (seg && lc >= 7) {
      const Tab tb = forest_tab(F, tab_key(14, 0, P, lc), s);
      if (tb.count) {
        const unsigned nb = (unsigned)tb.count;
        const double *Rl = lt.Rl64;
        const double2 *Ph = lt.Ph64;
        const char *nm = level_name("l2l", lc);
        switch (P) {
          case 15: PHS_LAUNCH(nm, s, kf_l2l_seg<15><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lc, Rl, Ph)); break;
          case 23: PHS_LAUNCH(nm, s, kf_l2l_seg<23><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lc, Rl, Ph)); break;
          case 27: PHS_LAUNCH(nm, s, kf_l2l_seg<27><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lc, Rl, Ph)); break;
          default: PHS_LAUNCH(nm, s, kf_l2l_seg<31><<<nb, 256, 0, s>>>(F.dsys, tb.d, mask, lc, Rl, Ph)); break;
        }
      }
      continue;
    }
    const Tab tb = forest_tab(F, tab_key(4, 0, P, lc), s);
    if (tb.count)
      PHS_LAUNCH(level_name("l2l", lc), s, kf_l2l<T><<<(unsigned)tb.count, 256, 0, s>>>(F.dsys, tb.d, mask, lc, P, L2L));
  }
}

template <class T, class TN>
void leaf_pass(Forest &F, const int32_t *mask, int in, int out, int P, const double *logtab,
               hipStream_t s) {
  const char *name = std::is_same<T, float>::value    ? "leaf_eval_f32"
                     : std::is_same<TN, float>::value ? "leaf_eval_near32"
                                                      : "leaf_eval";
  const Tab t2 = forest_tab(F, tab_key(1, 2, 0, 0), s);
  if (t2.count)
    PHS_LAUNCH(name, s,
               kf_leaf_eval<T, TN, 2><<<(unsigned)t2.count, 64, 0, s>>>(F.dsys, t2.d, mask, P,
                                                                      in, out, logtab));
  const Tab t4 = forest_tab(F, tab_key(1, 4, 0, 0), s);
  if (t4.count)
    PHS_LAUNCH(name, s,
               kf_leaf_eval<T, TN, 4><<<(unsigned)t4.count, 64, 0, s>>>(F.dsys, t4.d, mask, P,
                                                                      in, out, logtab));
  if (t2.count + t4.count > 0) f_near_combine(F, mask, out, s);
}

const Plan &log_ref(const Forest &F) {
  for (const Plan *p : F.plan)
    if (p->core_log && !p->direct) return *p;
  throw Error{PHS_ERR_INVALID_ARGUMENT, "forest has no even-order system"};
}

}  // namespace

// Host tables gathered into one device allocation and one copy: each part is
// copied into the staging buffer when added (on a 256-byte boundary), and its
// device address is set on upload.
struct TableStage {
  std::vector<std::pair<void **, size_t>> dst;
  std::vector<unsigned char> host;
  void add(void **d, const void *src, size_t bytes) {
    const size_t off = (host.size() + 255) & ~(size_t)255;
    host.resize(off + bytes);
    std::memcpy(host.data() + off, src, bytes);
    dst.push_back({d, off});
  }
  void *upload() {
    unsigned char *dev = dmalloc<unsigned char>(host.size());
    try {
      PHS_HIP(hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice));
    } catch (...) {
      dfree(dev);
      throw;
    }
    for (const auto &p : dst) *p.first = dev + p.second;
    return dev;
  }
};

void build_log_tables(LogTables &t, int P) {
  free_log_tables(t);
  TableStage stage;
  t.P = P;
  const int P1 = P + 1;
  // k-major: H[k*P1 + l]; 64 zero entries of padding so a chunk of LCH
  // coefficients that runs past P reads zeros, not past the allocation.
  std::vector<double> H((size_t)P1 * P1 + 64, 0.0);
  for (int l = 0; l <= P; ++l)
    for (int k = 0; k <= P; ++k) {
      double v;
      if (l == 0) v = (k == 0) ? 0.0 : 1.0;
      else if (k == 0) v = ((l % 2) ? 1.0 : -1.0) / l;
      else v = ((l % 2) ? -1.0 : 1.0) * binom(k + l - 1, l);
      H[(size_t)k * P1 + l] = v;
    }
  std::vector<double2> M2M((size_t)4 * P1 * P1), L2L((size_t)4 * P1 * P1);
  for (int c = 0; c < 4; ++c) {
    const double dre = (c & 1) ? 0.25 : -0.25, dim = (c & 2) ? 0.25 : -0.25;
    std::vector<double> pre(2 * P1 + 1), pim(2 * P1 + 1);  // delta^e
    pre[0] = 1.0;
    pim[0] = 0.0;
    for (int e = 1; e <= 2 * P1; ++e) {
      pre[e] = pre[e - 1] * dre - pim[e - 1] * dim;
      pim[e] = pre[e - 1] * dim + pim[e - 1] * dre;
    }
    for (int l = 0; l <= P; ++l)
      for (int k = 0; k <= P; ++k) {
        double re = 0.0, im = 0.0;
        if (l == 0) {
          if (k == 0) re = 1.0;
        } else if (k == 0) {
          re = -pre[l] / l;
          im = -pim[l] / l;
        } else if (k <= l) {
          const double f = binom(l - 1, k - 1) * std::ldexp(1.0, -k);
          re = f * pre[l - k];
          im = f * pim[l - k];
        }
        M2M[((size_t)c * P1 + l) * P1 + k] = make_double2(re, im);
      }
    for (int j = 0; j <= P; ++j)
      for (int k = 0; k <= P; ++k) {
        double re = 0.0, im = 0.0;
        if (k >= j) {
          const double f = binom(k, j) * std::ldexp(1.0, -j);
          re = f * pre[k - j];
          im = f * pim[k - j];
        }
        L2L[((size_t)c * P1 + j) * P1 + k] = make_double2(re, im);
      }
  }
  // per M2L offset o = 7 (oy + 3) + (ox + 3), D = -(ox, oy) in box widths:
  // D^-1, D^-4, D^-q for q = 0..3, log|D| (entries 0..12 of 16)
  std::vector<double> Off(49 * 16, 0.0);
  for (int o = 0; o < 49; ++o) {
    const int oy = o / 7 - 3, ox = o % 7 - 3;
    if (ox == 0 && oy == 0) continue;
    const double Dx = -ox, Dy = -oy, dd = Dx * Dx + Dy * Dy;
    const double ir = Dx / dd, ii = -Dy / dd;
    double pr = 1.0, pi = 0.0;
    for (int e = 0; e < 4; ++e) {
      Off[o * 16 + 4 + 2 * e] = pr;
      Off[o * 16 + 5 + 2 * e] = pi;
      const double nr = pr * ir - pi * ii, ni = pr * ii + pi * ir;
      pr = nr;
      pi = ni;
    }
    Off[o * 16 + 0] = ir;
    Off[o * 16 + 1] = ii;
    Off[o * 16 + 2] = pr;  // D^-4
    Off[o * 16 + 3] = pi;
    Off[o * 16 + 12] = 0.5 * std::log(dd);
  }
  // factored shifts: rho = sqrt(2)/4 (child centre offset in parent widths),
  // u_c = delta_c / rho
  {
    const double rho = std::sqrt(2.0) / 4.0;
    std::vector<double> Rm((size_t)P1 * P1, 0.0), Rl((size_t)P1 * P1, 0.0);
    std::vector<double> rp(2 * P1 + 1);
    rp[0] = 1.0;
    for (int e = 1; e <= 2 * P1; ++e) rp[e] = rp[e - 1] * rho;
    for (int l = 0; l <= P; ++l)
      for (int k = 0; k <= P; ++k) {
        double v = 0.0;
        if (l == 0) v = (k == 0) ? 1.0 : 0.0;
        else if (k == 0) v = -rp[l] / l;
        else if (k <= l) v = binom(l - 1, k - 1) * std::ldexp(1.0, -k) * rp[l - k];
        Rm[(size_t)l * P1 + k] = v;
      }
    for (int j = 0; j <= P; ++j)
      for (int k = 0; k <= P; ++k)
        Rl[(size_t)j * P1 + k] = k >= j ? binom(k, j) * std::ldexp(1.0, -j) * rp[k - j] : 0.0;
    std::vector<double2> Ph(4 * 32);
    for (int c = 0; c < 4; ++c) {
      const double ur = ((c & 1) ? 0.25 : -0.25) / rho, ui = ((c & 2) ? 0.25 : -0.25) / rho;
      double pr = 1.0, pi = 0.0;
      for (int k = 0; k < 32; ++k) {
        Ph[c * 32 + k] = make_double2(pr, pi);
        const double nr = pr * ur - pi * ui, ni = pr * ui + pi * ur;
        pr = nr;
        pi = ni;
      }
    }
    stage.add((void **)&t.Rm64, Rm.data(), Rm.size() * 8);
    stage.add((void **)&t.Rl64, Rl.data(), Rl.size() * 8);
    stage.add((void **)&t.Ph64, Ph.data(), Ph.size() * 16);
  }
  std::vector<float> Hf(H.begin(), H.end());
  std::vector<float2> M2Mf(M2M.size()), L2Lf(L2L.size());
  for (size_t i = 0; i < M2M.size(); ++i) {
    M2Mf[i] = make_float2((float)M2M[i].x, (float)M2M[i].y);
    L2Lf[i] = make_float2((float)L2L[i].x, (float)L2L[i].y);
  }
  stage.add((void **)&t.Off64, Off.data(), Off.size() * 8);
  stage.add((void **)&t.Ht64, H.data(), H.size() * 8);
  stage.add((void **)&t.Ht32, Hf.data(), Hf.size() * 4);
  stage.add((void **)&t.M2M64, M2M.data(), M2M.size() * 16);
  stage.add((void **)&t.L2L64, L2L.data(), L2L.size() * 16);
  stage.add((void **)&t.M2M32, M2Mf.data(), M2Mf.size() * 8);
  stage.add((void **)&t.L2L32, L2Lf.data(), L2Lf.size() * 8);
  t.block = stage.upload();
}

void free_log_tables(LogTables &t) {
  dfree(t.block);
  t = LogTables();
}

void fill_log_table(double *tab) {
  for (int j = 0; j < 128; ++j) {
    tab[j] = 1.0 / (1.0 + j / 128.0);
    tab[128 + j] = std::log1p(j / 128.0);
  }
}

void fill_near_log_table(double *tab) {
  const int nent = 1 << kNearLogBits;
  for (int j = 0; j < nent; ++j) {
    const double invc = 1.0 / (0.5 * (1.0 + (j + 0.5) / nent));
    tab[2 * j] = invc;
    tab[2 * j + 1] = (double)(-std::log((long double)invc));
  }
}

size_t log_expansion_bytes(int L, int P, int nd, bool fp64) {
  return (size_t)level_base(L + 1, P, nd) * (fp64 ? 16 : 8);
}

int m2l_chunk(int P) {
  // widest of 16/14/12 dividing P+1, else 8 (the last chunk then stores only
  // its first coefficients)
  return ((P + 1) % 16 == 0) ? 16 : ((P + 1) % 14 == 0) ? 14 : ((P + 1) % 12 == 0) ? 12 : 8;
}

void log_matvec(Forest &F, const int32_t *mask, int in, int out, int precision,
                hipStream_t s) {
  const Plan &ref = log_ref(F);
  if (precision == PHS_MIXED) {
    far_field<float>(F, mask, in, ref.p32, ref.lt32, "m2l_f32", s);
    leaf_pass<float, float>(F, mask, in, out, ref.p32, ref.neartab, s);
  } else if (precision == PHS_FP64_EVAL) {
    far_field<double>(F, mask, in, ref.pe, ref.pe == ref.p64 ? ref.lt64 : ref.lte, "m2l_eval",
                      s);
    leaf_pass<double, double>(F, mask, in, out, ref.pe, ref.neartab, s);
  } else {
    far_field<double>(F, mask, in, ref.p64, ref.lt64, "m2l", s);
    if (precision == PHS_NEAR32)
      leaf_pass<double, float>(F, mask, in, out, ref.p64, ref.neartab, s);
    else
      leaf_pass<double, double>(F, mask, in, out, ref.p64, ref.neartab, s);
  }
}

void log_expansions(Plan &pl, int in, hipStream_t s) {
  Forest &F = *pl.self;
  far_field<double>(F, F.mask[0], in, pl.pe, pl.pe == pl.p64 ? pl.lt64 : pl.lte, "m2l_eval", s);
}

void log_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                      const double *targets, int64_t m, double *out, hipStream_t s) {
  const int P = pl.pe, L = pl.tree.L;
  const double2 *A = (const double2 *)pl.sw.mp;
  const double2 *BL = (const double2 *)pl.sw.loc + level_base(L, P, pl.R);
  const int64_t nb = (m + 127) / 128;
  if (pl.k == 2)
    PHS_LAUNCH("eval_targets", s,
               k_eval_targets<2><<<nb, 128, 0, s>>>(targets, m, pl.c[0], pl.c[1], pl.rho,
                                                    pl.x, pl.y, w_tree, pl.tree.leaf_start,
                                                    L, pl.tree.h, P, A, BL, beta, pl.d,
                                                    out, pl.xy2, pl.neartab));
  else
    PHS_LAUNCH("eval_targets", s,
               k_eval_targets<4><<<nb, 128, 0, s>>>(targets, m, pl.c[0], pl.c[1], pl.rho,
                                                    pl.x, pl.y, w_tree, pl.tree.leaf_start,
                                                    L, pl.tree.h, P, A, BL, beta, pl.d,
                                                    out, pl.xy2, pl.neartab));
}

}  // namespace phs
