// Distance-kernel FMM, core kernel |x - y|, used for odd k (paper eq.
// matvec_hadamard with M = [r^(k-1)] o [r]; the paper names this core sum but
// gives no expansion for it).
//
// The kernel is not harmonic, so instead of complex multipole series this unit
// uses tensor Chebyshev interpolation on every box (a kernel-independent FMM):
// a box of half-width w/2 carries Q x Q "equivalent densities" W at the
// Chebyshev nodes xbar_a = cos((2a+1) pi / (2Q)) of its scaled square, and the
// far field at the nodes of a target box is G_m = sum_s K(x_m, y_n) W_s[n].
//   P2M  W[a][b]   = sum_j q_j S_a(y1_j) S_b(y2_j)       (S_a Lagrange basis)
//   M2M  W_parent  = sum_children T_cx W_child T_cy^T,   T_s[a][a'] = S_a((xbar_a' + s)/2)
//   M2L  G_target  = (w/2) sum_s K_D W_s, K_D[m][n] = |2D + xbar_m - xbar_n| at unit
//        half-width (|x - y| is homogeneous of degree 1, so one set of 40
//        matrices serves every level)
//   L2L  G_child  += T_cx^T G_parent T_cy
//   L2P  f(x)      = sum_ab S_a(x1) S_b(x2) G[a][b]
// The near field (3x3 leaves) is direct phi(r) as in the log-kernel unit.
//
// Layout: per level, expansions [box][density][node] (node index a*Q + b).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "fmm_common.h"

namespace phs {

namespace {

template <class T>
using V2 = typename Vec2<T>::type;

constexpr int kNoff = 40;

__host__ __device__ inline int64_t cheb_level_base(int l, int QQ, int nd) {
  return (int64_t)QQ * nd * (((int64_t)1 << (2 * l)) - 16) / 3;
}

// Lagrange basis at the Q Chebyshev nodes evaluated at x (|x| <= 1):
// S_a(x) = (1 + 2 sum_{k>=1} T_k(x) T_k(xbar_a)) / Q.  Tk: table T_k(xbar_a), [k][a].
// IN_PLACE reads column a of the table where it is used; without it the
// compiler may load all Q^2 entries into registers once (which pays where the
// basis is evaluated once per point, not where the kernel holds much else).
template <class T, int Q, bool IN_PLACE = false>
__device__ __forceinline__ void cheb_basis(T x, const T *__restrict__ Tk, T *S) {
  T tk[Q];
  tk[0] = T(1);
  if (Q > 1) tk[1] = x;
#pragma unroll
  for (int k = 2; k < Q; ++k) tk[k] = T(2) * x * tk[k - 1] - tk[k - 2];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int col = a;
    if constexpr (IN_PLACE) asm volatile("" : "+s"(col));
    T s = T(0);
#pragma unroll
    for (int k = 1; k < Q; ++k) s += tk[k] * Tk[k * Q + col];
    S[a] = (T(1) + T(2) * s) * (T(1) / T(Q));
  }
}

// The bases at two points x1, x2 (the two coordinates of one target) in one
// pass over the table, each column read once where it is used.
template <class T, int Q>
__device__ __forceinline__ void cheb_basis2(T x1, T x2, const T *__restrict__ Tk, T *S1, T *S2) {
  T t1[Q], t2[Q];
  t1[0] = T(1);
  t2[0] = T(1);
  if (Q > 1) {
    t1[1] = x1;
    t2[1] = x2;
  }
#pragma unroll
  for (int k = 2; k < Q; ++k) {
    t1[k] = T(2) * x1 * t1[k - 1] - t1[k - 2];
    t2[k] = T(2) * x2 * t2[k - 1] - t2[k - 2];
  }
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    int col = a;
    asm volatile("" : "+s"(col));
    T s1 = T(0), s2 = T(0);
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const T tv = Tk[k * Q + col];
      s1 += t1[k] * tv;
      s2 += t2[k] * tv;
    }
    S1[a] = (T(1) + T(2) * s1) * (T(1) / T(Q));
    S2[a] = (T(1) + T(2) * s2) * (T(1) / T(Q));
  }
}

// ---------------------------------------------------------------- P2M
// Work item: one leaf of one system.
template <class T, int K, int Q>
__global__ __launch_bounds__(64) void kf_cheb_p2m(const SysDev *__restrict__ sys,
                                                  const BlkRef *__restrict__ tab,
                                                  const int32_t *__restrict__ mask, int in,
                                                  const T *__restrict__ Tk) {
  constexpr int R = Rank<K>::R;
  constexpr int QQ = Q * Q;
  constexpr int EPL = (QQ + 63) / 64;  // entries per lane
  __shared__ T s1[64][Q], s2[64][Q], qd[64][R];
  __shared__ T tk[Q * Q];
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int L = d.L;
  const double h = d.h;
  const cptr<double> x = ro(d.x);
  const cptr<double> y = ro(d.y);
  const cptr<float> ux = ro(d.ux);
  const cptr<float> uy = ro(d.uy);
  const cptr<double> t = ro(d.v[in]);
  const cptr<int32_t> start = ro(d.leaf_start);
  const gptr<T> W = rw((T *)d.mp + cheb_level_base(L, QQ, R));
  const int lane = threadIdx.x;
  const int G = 1 << L;
  const int leaf = br.blk;
  for (int i = lane; i < Q * Q; i += 64) tk[i] = Tk[i];
  const int b = start[leaf], e = start[leaf + 1];
  const double w = 2.0 * h / G;
  const double inv_half = 2.0 / w;
  const int ix = leaf % G, iy = leaf / G;
  const double cx = -h + (ix + 0.5) * w, cy = -h + (iy + 0.5) * w;
  T acc[EPL][R];
#pragma unroll
  for (int i = 0; i < EPL; ++i)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[i][r] = T(0);
  __syncthreads();
  for (int c0 = b; c0 < e; c0 += 64) {
    const int np = min(64, e - c0);
    if (lane < np) {
      const int j = c0 + lane;
      T u1, u2;
      if constexpr (std::is_same<T, float>::value) {
        u1 = ux[j] * (float)inv_half;
        u2 = uy[j] * (float)inv_half;
      } else {
        u1 = (x[j] - cx) * inv_half;
        u2 = (y[j] - cy) * inv_half;
      }
      T S[Q];
      cheb_basis<T, Q, true>(u1, tk, S);
#pragma unroll
      for (int a = 0; a < Q; ++a) s1[lane][a] = S[a];
      cheb_basis<T, Q, true>(u2, tk, S);
#pragma unroll
      for (int a = 0; a < Q; ++a) s2[lane][a] = S[a];
      T v[R];
      vfac<K, T>(x[j], y[j], v);
#pragma unroll
      for (int r = 0; r < R; ++r) qd[lane][r] = v[r] * (T)t[j];
    }
    __syncthreads();
    for (int p = 0; p < np; ++p) {
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        const int en = lane + 64 * i;
        if (en < QQ) {
          const T sab = s1[p][en / Q] * s2[p][en % Q];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[i][r] += qd[p][r] * sab;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    const int en = lane + 64 * i;
    if (en < QQ)
#pragma unroll
      for (int r = 0; r < R; ++r) W[((int64_t)leaf * R + r) * QQ + en] = acc[i][r];
  }
}

// ---------------------------------------------------------------- M2M / L2L
// Block per (box, density), QQ threads.  Tpm: [2][Q][Q] with Tpm[s][a][a'] =
// S_a((xbar_a' + (2s-1))/2).
template <class T, int Q>
__global__ void kf_cheb_m2m(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                            const int32_t *__restrict__ mask, int lp,
                            const T *__restrict__ Tpm) {
  constexpr int QQ = Q * Q;
  __shared__ T tm[2 * QQ], wc[QQ], yy[QQ];
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R;
  const cptr<T> Wc = ro((const T *)d.mp + cheb_level_base(lp + 1, QQ, nd));
  const gptr<T> Wp = rw((T *)d.mp + cheb_level_base(lp, QQ, nd));
  const int tid = threadIdx.x;
  const int Gp = 1 << lp, Gc = 2 * Gp;
  const int box = br.blk / nd, r = br.blk % nd;
  const int bx = box % Gp, by = box / Gp;
  for (int i = tid; i < 2 * QQ; i += blockDim.x) tm[i] = Tpm[i];
  const int a = tid / Q, bb = tid % Q;
  T acc = T(0);
  for (int c = 0; c < 4; ++c) {
    const int cxx = c & 1, cyy = c >> 1;
    const int child = (2 * by + cyy) * Gc + 2 * bx + cxx;
    __syncthreads();
    if (tid < QQ) wc[tid] = Wc[((int64_t)child * nd + r) * QQ + tid];
    __syncthreads();
    // Y[a'][b] = sum_b' W[a'][b'] T_cy[b][b']
    if (tid < QQ) {
      T s = T(0);
      const T *ty = tm + cyy * QQ + bb * Q;
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) s += wc[a * Q + q2] * ty[q2];
      yy[tid] = s;
    }
    __syncthreads();
    if (tid < QQ) {
      const T *tx = tm + cxx * QQ + a * Q;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) acc += tx[q1] * yy[q1 * Q + bb];
    }
  }
  if (tid < QQ) Wp[((int64_t)box * nd + r) * QQ + tid] = acc;
}

template <class T, int Q>
__global__ void kf_cheb_l2l(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                            const int32_t *__restrict__ mask, int lc,
                            const T *__restrict__ Tpm) {
  constexpr int QQ = Q * Q;
  __shared__ T tm[2 * QQ], gp[QQ], yy[QQ];
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int nd = d.R;
  const gptr<T> Gp = rw((T *)d.loc + cheb_level_base(lc - 1, QQ, nd));
  const gptr<T> Gc = rw((T *)d.loc + cheb_level_base(lc, QQ, nd));
  const int tid = threadIdx.x;
  const int G = 1 << lc;
  const int box = br.blk / nd, r = br.blk % nd;
  const int bx = box % G, by = box / G;
  const int cxx = bx & 1, cyy = by & 1;
  const int parent = (by >> 1) * (G / 2) + (bx >> 1);
  for (int i = tid; i < 2 * QQ; i += blockDim.x) tm[i] = Tpm[i];
  if (tid < QQ) gp[tid] = Gp[((int64_t)parent * nd + r) * QQ + tid];
  __syncthreads();
  const int a = tid / Q, bb = tid % Q;
  // Y[a'][b] = sum_b' G[a'][b'] T_cy[b'][b]
  if (tid < QQ) {
    T s = T(0);
#pragma unroll
    for (int q2 = 0; q2 < Q; ++q2) s += gp[a * Q + q2] * tm[cyy * QQ + q2 * Q + bb];
    yy[tid] = s;
  }
  __syncthreads();
  if (tid < QQ) {
    T s = T(0);
#pragma unroll
    for (int q1 = 0; q1 < Q; ++q1) s += tm[cxx * QQ + q1 * Q + a] * yy[q1 * Q + bb];
    const gptr<T> dst = &Gc[((int64_t)box * nd + r) * QQ + tid];
    *dst += s;
  }
}

// ---------------------------------------------------------------- M2L
// Tiled GEMM: a block owns all QQ rows of a tile of 64 (box, density)
// columns of one level and accumulates sum_D K_D W_{src(D)} over the 40
// offsets in a fixed order.  Boxes are enumerated by parity class so a tile
// mostly shares one interaction-list pattern.
constexpr int kCols = 64, kKc = 16;

template <class T, int QQ>
__global__ __launch_bounds__(256) void kf_cheb_m2l(const SysDev *__restrict__ sys,
                                                   const BlkRef *__restrict__ tab,
                                                   const int32_t *__restrict__ mask,
                                                   const T *__restrict__ Kd) {
  constexpr int RPT = (QQ + 15) / 16;  // rows per thread
  constexpr int AST = kKc + 1;         // padded row stride of the A tile
  __shared__ T As[QQ * AST];
  __shared__ T Bs[kKc * kCols];
  __shared__ int src_box[kCols];
  __shared__ int any_valid;
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const cptr<T> Wall = ro((const T *)d.mp);
  const gptr<T> Gall = rw((T *)d.loc);
  const int L = d.L, nd = d.R;
  const double h = d.h;
  const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
  // locate level and tile
  int64_t tcol = (int64_t)br.blk * kCols;
  int l = 2;
  int64_t off = 0, base = 0;
  while (l <= L) {
    const int64_t cols_l = ((int64_t)1 << (2 * l)) * nd;
    const int64_t tiles_l = (cols_l + kCols - 1) / kCols;
    if (tcol < off + tiles_l * kCols) break;
    off += tiles_l * kCols;
    base += cols_l * QQ;
    ++l;
  }
  if (l > L) return;
  const int G = 1 << l;
  const int64_t nb = (int64_t)G * G;
  const int64_t col0 = tcol - off;
  const cptr<T> Wl = Wall + base;
  const gptr<T> Gl = Gall + base;
  const T half_w = (T)(h / G);  // (w/2)
  // my columns: c = tx + 16 j
  T acc[RPT][4];
#pragma unroll
  for (int i = 0; i < RPT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
  // target box for column index (parity-class order)
  auto tgt_of = [&](int64_t cidx, int &ix, int &iy, int &r) -> bool {
    if (cidx >= nb * nd) return false;
    const int64_t bi = cidx / nd;
    r = (int)(cidx % nd);
    const int64_t quarter = nb / 4;
    const int cls = (int)(bi / quarter);
    const int64_t rem = bi % quarter;
    const int hf = G / 2;
    ix = 2 * (int)(rem % hf) + (cls & 1);
    iy = 2 * (int)(rem / hf) + (cls >> 1);
    return true;
  };
  int oi = 0;
  for (int oy = -3; oy <= 3; ++oy)
    for (int ox = -3; ox <= 3; ++ox) {
      if (abs(ox) <= 1 && abs(oy) <= 1) continue;
      const int d_idx = oi++;
      __syncthreads();
      if (tid == 0) any_valid = 0;
      __syncthreads();
      if (tid < kCols) {
        int ix, iy, r;
        int sb = -1;
        if (tgt_of(col0 + tid, ix, iy, r)) {
          const int jx = ix + ox, jy = iy + oy;
          if (jx >= 0 && jy >= 0 && jx < G && jy < G && abs((jx >> 1) - (ix >> 1)) <= 1 &&
              abs((jy >> 1) - (iy >> 1)) <= 1)
            sb = (jy * G + jx) * nd + r;
        }
        src_box[tid] = sb;
        if (sb >= 0) any_valid = 1;
      }
      __syncthreads();
      if (!any_valid) continue;
      const T *KD = Kd + (int64_t)d_idx * QQ * QQ;
      for (int k0 = 0; k0 < QQ; k0 += kKc) {
        // A tile: KD[m][k0..k0+kKc)
        for (int e = tid; e < QQ * kKc; e += 256) {
          const int m = e / kKc, kk = e % kKc;
          As[m * AST + kk] = (k0 + kk < QQ) ? KD[(int64_t)m * QQ + k0 + kk] : T(0);
        }
        // B tile: W[src][k0..k0+kKc) per column
        for (int e = tid; e < kKc * kCols; e += 256) {
          const int c = e / kKc, kk = e % kKc;
          const int sb = src_box[c];
          Bs[kk * kCols + c] = (sb >= 0 && k0 + kk < QQ) ? Wl[(int64_t)sb * QQ + k0 + kk] : T(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < kKc; ++kk) {
          T bv[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[j] = Bs[kk * kCols + tx + 16 * j];
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const int m = ty + 16 * i;
            if (m < QQ) {
              const T av = As[m * AST + kk];
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[i][j] += av * bv[j];
            }
          }
        }
        __syncthreads();
      }
    }
  // store
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int ix, iy, r;
    if (!tgt_of(col0 + tx + 16 * j, ix, iy, r)) continue;
    const int64_t tb = ((int64_t)(iy * G + ix) * nd + r) * QQ;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int m = ty + 16 * i;
      if (m < QQ) Gl[tb + m] = half_w * acc[i][j];
    }
  }
}

// FP64 M2L on the matrix cores: the tiles of kf_cheb_m2l (output rows by 64
// columns, the contraction staged through LDS in chunks of 16), with the
// products by v_mfma_f64_16x16x4f64.  Lane layout of the product (row m,
// column n, inner index k): A[m][k] at lane m + 16 k, B[k][n] at lane
// n + 16 k, result D[m][n] at lane n + 16 (m mod 4) in register m / 4.
//
// Row split: the QQ output rows of a tile are shared by
// cheb_m2l_max_split(QQ) workgroups, each taking a contiguous block of 16-row
// tiles (work item = tile * split + part), one tile per wavefront at QQ = 256.
// Pipelining: the source boxes of all 40 offsets are found first, the
// (offset, contraction chunk) steps then run as one flat sequence, and each
// thread loads the next step's operands into registers while the matrix cores
// work on the current step.  A tile was bound by the latency of its 40 x QQ/16
// dependent load-then-compute steps (a launch took ~4.6 ms whatever the tree
// size); every output row is still summed by one workgroup, offset by offset
// and chunk by chunk in the original order.
typedef double cdbl4 __attribute__((ext_vector_type(4)));

constexpr int kOffsets = 40;  // M2L offsets: the 7 x 7 square minus the 3 x 3 near field

template <int QQ>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void kf_cheb_m2l_mfma(const SysDev *__restrict__ sys, const BlkRef *__restrict__ tab,
                      const int32_t *__restrict__ mask, const double *__restrict__ Kd) {
  constexpr int RS = cheb_m2l_max_split(QQ);
  constexpr int MT_ALL = (QQ + 15) / 16;      // 16-row tiles (rows past QQ are zero)
  constexpr int MT = (MT_ALL + RS - 1) / RS;  // row tiles of one part
  constexpr int TPW = (MT + 3) / 4;           // row tiles per wavefront
  constexpr int KS = (QQ + kKc - 1) / kKc;    // contraction chunks per offset
  constexpr int APT = MT * 16 * kKc / 256;    // A operands a thread stages per step
  constexpr int BPT = kKc * kCols / 256;      // B operands a thread stages per step
  static_assert(MT * 16 * kKc % 256 == 0 && kKc * kCols % 256 == 0, "staging split");
  constexpr int AST = kKc + 1, BST = kCols + 1;  // padded strides
  __shared__ double As[MT * 16 * AST];
  __shared__ double Bs[kKc * BST];
  __shared__ int sbox[kOffsets * kCols];
  __shared__ int vlist[kOffsets];
  __shared__ int nvalid;
  const BlkRef br = tab[blockIdx.x];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const cptr<double> Wall = ro((const double *)d.mp);
  const gptr<double> Gall = rw((double *)d.loc);
  const int L = d.L, nd = d.R;
  const double h = d.h;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int lm = lane & 15, lk = lane >> 4;
  // this part's row tiles: rt0 .. rt0 + MT (those below MT_ALL)
  const int rt0 = (br.blk % RS) * MT;
  // locate level and tile
  int64_t tcol = (int64_t)(br.blk / RS) * kCols;
  int l = 2;
  int64_t off = 0, base = 0;
  while (l <= L) {
    const int64_t cols_l = ((int64_t)1 << (2 * l)) * nd;
    const int64_t tiles_l = (cols_l + kCols - 1) / kCols;
    if (tcol < off + tiles_l * kCols) break;
    off += tiles_l * kCols;
    base += cols_l * QQ;
    ++l;
  }
  if (l > L) return;
  const int G = 1 << l;
  const int64_t nb = (int64_t)G * G;
  const int64_t col0 = tcol - off;
  const cptr<double> Wl = Wall + base;
  const gptr<double> Gl = Gall + base;
  const double half_w = h / G;  // (w/2)
  // target box of a column index (parity-class order)
  auto tgt_of = [&](int64_t cidx, int &ix, int &iy, int &r) -> bool {
    if (cidx >= nb * nd) return false;
    const int64_t bi = cidx / nd;
    r = (int)(cidx % nd);
    const int64_t quarter = nb / 4;
    const int cls = (int)(bi / quarter);
    const int64_t rem = bi % quarter;
    const int hf = G / 2;
    ix = 2 * (int)(rem % hf) + (cls & 1);
    iy = 2 * (int)(rem / hf) + (cls >> 1);
    return true;
  };
  // source box of each column under each offset (-1: none)
  for (int e = tid; e < kOffsets * kCols; e += 256) {
    const int di = e / kCols, c = e % kCols;
    // offset di of the (oy, ox) row-major order over [-3, 3]^2 without the
    // 3 x 3 near field: rows oy = -3, -2 and 2, 3 hold 7 offsets, rows -1..1
    // hold 4 (ox = -3, -2, 2, 3)
    int oy, ox;
    if (di < 14) {
      oy = -3 + di / 7;
      ox = -3 + di % 7;
    } else if (di < 26) {
      oy = -1 + (di - 14) / 4;
      const int j = (di - 14) % 4;
      ox = j < 2 ? j - 3 : j;
    } else {
      oy = 2 + (di - 26) / 7;
      ox = -3 + (di - 26) % 7;
    }
    int sb = -1;
    int ix, iy, r;
    if (tgt_of(col0 + c, ix, iy, r)) {
      const int jx = ix + ox, jy = iy + oy;
      if (jx >= 0 && jy >= 0 && jx < G && jy < G && abs((jx >> 1) - (ix >> 1)) <= 1 &&
          abs((jy >> 1) - (iy >> 1)) <= 1)
        sb = (jy * G + jx) * nd + r;
    }
    sbox[e] = sb;
  }
  __syncthreads();
  if (tid == 0) {
    int nv = 0;
    for (int di = 0; di < kOffsets; ++di) {
      bool any = false;
      for (int c = 0; c < kCols && !any; ++c) any = sbox[di * kCols + c] >= 0;
      if (any) vlist[nv++] = di;
    }
    nvalid = nv;
  }
  __syncthreads();
  const int steps = nvalid * KS;
  double ra[APT], rb[BPT];
  auto stage = [&](int st) {  // this thread's operands of step st into registers
    const int di = vlist[st / KS], k0 = (st % KS) * kKc;
    const double *KD = Kd + (int64_t)di * QQ * QQ;
#pragma unroll
    for (int u = 0; u < APT; ++u) {
      const int e = tid + 256 * u;
      const int m = 16 * rt0 + e / kKc, kk = e % kKc;
      ra[u] = (m < QQ && k0 + kk < QQ) ? KD[(int64_t)m * QQ + k0 + kk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int e = tid + 256 * u;
      const int c = e / kKc, kk = e % kKc;
      const int sb = sbox[di * kCols + c];
      rb[u] = (sb >= 0 && k0 + kk < QQ) ? Wl[(int64_t)sb * QQ + k0 + kk] : 0.0;
    }
  };
  cdbl4 acc[TPW][4];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[t][ct] = cdbl4{0.0, 0.0, 0.0, 0.0};
  if (steps > 0) stage(0);
  for (int st = 0; st < steps; ++st) {
    __syncthreads();  // the previous step's reads of As / Bs are done
#pragma unroll
    for (int u = 0; u < APT; ++u) {
      const int e = tid + 256 * u;
      As[(e / kKc) * AST + e % kKc] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      const int e = tid + 256 * u;
      Bs[(e % kKc) * BST + e / kKc] = rb[u];
    }
    __syncthreads();
    if (st + 1 < steps) stage(st + 1);  // in flight during the products
#pragma unroll
    for (int q = 0; q < kKc / 4; ++q) {
      double b[4];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) b[ct] = Bs[(4 * q + lk) * BST + 16 * ct + lm];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int rt = wave + 4 * t;
        if (rt < MT && rt0 + rt < MT_ALL) {  // uniform across the wavefront
          const double a = As[(16 * rt + lm) * AST + 4 * q + lk];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct)
            acc[t][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[ct], acc[t][ct], 0, 0, 0);
        }
      }
    }
  }
  // store: D[m][n] of tile (t, ct) at lane n + 16 (m mod 4), register m / 4
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    int ix, iy, r;
    if (!tgt_of(col0 + 16 * ct + lm, ix, iy, r)) continue;
    const int64_t tb = ((int64_t)(iy * G + ix) * nd + r) * QQ;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int rt = wave + 4 * t;
      if (rt >= MT || rt0 + rt >= MT_ALL) continue;
#pragma unroll
      for (int reg = 0; reg < 4; ++reg) {
        const int m = 16 * (rt0 + rt) + 4 * reg + lk;
        if (m < QQ) Gl[tb + m] = half_w * acc[t][ct][reg];
      }
    }
  }
}

// ---------------------------------------------------------------- leaf
template <class T, class TN, int K, int Q>
__global__ __launch_bounds__(64) void kf_cheb_leaf_eval(const SysDev *__restrict__ sys,
                                                        const BlkRef *__restrict__ tab,
                                                        const int32_t *__restrict__ mask,
                                                        int in, int out,
                                                        const T *__restrict__ Tk,
                                                        const double *__restrict__ logtab) {
  constexpr int R = Rank<K>::R;
  constexpr int QQ = Q * Q;
  __shared__ T tk[QQ];
  __shared__ T s1s[Q * 64];  // basis S1 of each lane's target, [a][lane]
  const BlkRef br = tab[xcd_remap(blockIdx.x, gridDim.x)];
  if (!mask[br.sys]) return;
  const SysDev &d = sys[br.sys];
  const int L = d.L;
  const double h = d.h;
  const cptr<double> x = ro(d.x);
  const cptr<double> y = ro(d.y);
  const cptr<float> ux = ro(d.ux);
  const cptr<float> uy = ro(d.uy);
  const cptr<double> t = ro(d.v[in]);
  const cptr<int32_t> start = ro(d.leaf_start);
  const cptr<double> xy2 = ro((const double *)d.xy2);
  const cptr<T> Gleaf = ro((const T *)d.loc + cheb_level_base(L, QQ, R));
  const gptr<double> ytree = rw(d.v[out]);
  const int G = 1 << L;
  const int leaf = br.blk;
  const int lane = threadIdx.x;
  for (int i = lane; i < QQ; i += 64) tk[i] = Tk[i];
  __syncthreads();
  const int b = start[leaf], e = start[leaf + 1];
  if (b == e) return;
  const int ix = leaf % G, iy = leaf / G;
  const double w = 2.0 * h / G, inv_half = 2.0 / w;
  const double cx = -h + (ix + 0.5) * w, cy = -h + (iy + 0.5) * w;
  const int r0 = iy > 0 ? iy - 1 : 0, r1 = iy + 1 < G ? iy + 1 : G - 1;
  const int c0 = ix > 0 ? ix - 1 : 0, c1 = ix + 1 < G ? ix + 1 : G - 1;
  const cptr<T> Gl = Gleaf + (int64_t)leaf * R * QQ;
  for (int i0 = b; i0 < e; i0 += 64) {
    // a pass with at most 32 targets left runs 64/W groups of W lanes on the
    // same targets, each over its share of every source range, and sums the
    // groups' partial sums (the lanes a plain pass would leave idle share the
    // near field)
    const int rem = e - i0;
    const int W = rem <= 8 ? 8 : rem <= 16 ? 16 : rem <= 32 ? 32 : 64;
    const int ng = 64 / W, gi = lane / W, li = lane % W;
    const int i = i0 + li;
    const bool act = li < rem;
    const int ii = act ? i : b;
    const double xi = x[ii], yi = y[ii];
    T far = T(0);
    {
      T u1, u2;
      if constexpr (std::is_same<T, float>::value) {
        u1 = ux[ii] * (float)inv_half;
        u2 = uy[ii] * (float)inv_half;
      } else {
        u1 = (xi - cx) * inv_half;
        u2 = (yi - cy) * inv_half;
      }
      T S1[Q], S2[Q];
      cheb_basis2<T, Q>(u1, u2, tk, S1, S2);
#pragma unroll
      for (int a = 0; a < Q; ++a) s1s[a * 64 + lane] = S1[a];
      T u[R];
      ufac<K, T>(xi, yi, u);
      // sum_a S1[a] sum_b S2[b] g_r[a][b]: the loop over rows a stays rolled,
      // so each row's Q coefficients are loaded in its iteration (unrolled,
      // all R Q^2 of them were hoisted and spilled), and S1 comes from LDS
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const cptr<T> g = Gl + r * QQ;
        T s = T(0);
#pragma unroll 1
        for (int a = 0; a < Q; ++a) {
          const cptr<T> ga = g + a * Q;
          T sa = T(0);
#pragma unroll
          for (int bb = 0; bb < Q; ++bb) sa += S2[bb] * ga[bb];
          s += s1s[a * 64 + lane] * sa;
        }
        far += u[r] * s;
      }
    }
    TN nearv = TN(0);
    if constexpr (std::is_same<TN, double>::value) {
      for (int row = r0; row <= r1; ++row) {
        const int js = start[row * G + c0], je = start[row * G + c1 + 1];
        const int len = je - js;
        nearv += near_range<K>(xi, yi, xy2, t, js + len * gi / ng, js + len * (gi + 1) / ng,
                               logtab);
      }
      for (int o = W; o < 64; o <<= 1) nearv += __shfl_xor(nearv, o);
      nearv *= near_scale<K>();
    } else {
      // coordinates relative to each point's own leaf centre: the target is
      // moved into the frame of each neighbouring leaf once, so a pair costs
      // one subtraction per axis; densities from the FP32 copy
      const float uxi = ux[ii], uyi = uy[ii];
      const cptr<float> tf = ro((const float *)d.t32);
      for (int row = r0; row <= r1; ++row) {
        const float uyc = uyi + (float)((iy - row) * w);
        for (int col = c0; col <= c1; ++col) {
          const float uxc = uxi + (float)((ix - col) * w);
          const int js = start[row * G + col], je = start[row * G + col + 1];
          if (W == 64) {
            nearv += near_range_f32<K>(uxc, uyc, ux, uy, tf, js, je);
          } else {
            const int len = je - js;
            for (int j = js + len * gi / ng; j < js + len * (gi + 1) / ng; ++j) {
              const float dx = uxc - ux[j], dy = uyc - uy[j];
              nearv += phi_r2f<K>(dx * dx + dy * dy) * tf[j];
            }
          }
        }
      }
      for (int o = W; o < 64; o <<= 1) nearv += __shfl_xor(nearv, o);
      nearv *= phi_scale_f<K>();
    }
    if (act && gi == 0) ytree[i] = (double)far + (double)nearv;
  }
}

// ---------------------------------------------------------------- targets
template <int K, int Q>
__global__ void k_cheb_eval_targets(const double *__restrict__ tg, int64_t m, double cxn,
                                    double cyn, double rho, const double *__restrict__ x,
                                    const double *__restrict__ y,
                                    const double *__restrict__ wt,
                                    const int32_t *__restrict__ start, int L, double h,
                                    const double *__restrict__ Tk,
                                    const double *__restrict__ nodes,
                                    const double *__restrict__ Wall,
                                    const double *__restrict__ Gleaf,
                                    const double *__restrict__ beta, int d,
                                    double *__restrict__ out,
                                    const double2 *__restrict__ xy2,
                                    const double *__restrict__ logtab) {
  constexpr int R = Rank<K>::R;
  constexpr int QQ = Q * Q;
  const int64_t it = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (it >= m) return;
  const double xi = (tg[2 * it] - cxn) * rho, yi = (tg[2 * it + 1] - cyn) * rho;
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
    double S1[Q], S2[Q];
    cheb_basis<double, Q>((xi - cx) * (2.0 / w), Tk, S1);
    cheb_basis<double, Q>((yi - cy) * (2.0 / w), Tk, S2);
    for (int r = 0; r < R; ++r) {
      const double *g = Gleaf + ((int64_t)leaf * R + r) * QQ;
      double s = 0.0;
      for (int a = 0; a < Q; ++a) {
        double sa = 0.0;
        for (int bb = 0; bb < Q; ++bb) sa += S2[bb] * g[a * Q + bb];
        s += S1[a] * sa;
      }
      far += u[r] * s;
    }
    const int r0 = iy > 0 ? iy - 1 : 0, r1 = iy + 1 < G ? iy + 1 : G - 1;
    const int c0 = ix > 0 ? ix - 1 : 0, c1 = ix + 1 < G ? ix + 1 : G - 1;
    for (int row = r0; row <= r1; ++row) {
      const int js = start[row * G + c0], je = start[row * G + c1 + 1];
      nearv += near_scale<K>() * near_range<K>(xi, yi, (const double *)xy2, wt, js, je, logtab);
    }
  } else {
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
      if (ddx * ddx + ddy * ddy >= (2.5 * wl) * (2.5 * wl)) {
        // far: equivalent densities at the box's Chebyshev nodes
        const double *Wl = Wall + cheb_level_base(l, QQ, R);
        for (int a = 0; a < Q; ++a)
          for (int bb = 0; bb < Q; ++bb) {
            const double px = ccx + 0.5 * wl * nodes[a], py = ccy + 0.5 * wl * nodes[bb];
            const double dx = xi - px, dy = yi - py;
            const double kv = sqrt(dx * dx + dy * dy);
            for (int r = 0; r < R; ++r)
              far += u[r] * kv * Wl[((int64_t)box * R + r) * QQ + a * Q + bb];
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

// ---------------------------------------------------------------- host
// tier: which Q of each plan the launch uses (0 FP64 matvec, 1 FP32 matvec,
// 2 evaluation); only the odd-k systems whose Q for that tier equals Q take part.
template <class T, int Q>
void far_field_q(Forest &F, const int32_t *mask, int in, const ChebTables &ct, int tier,
                 hipStream_t s) {
  constexpr int QQ = Q * Q;
  const bool fp64 = std::is_same<T, double>::value;
  const T *Tk = fp64 ? (const T *)ct.nodes64 + Q : (const T *)ct.nodes32 + Q;
  const T *Tpm = fp64 ? (const T *)ct.S2c64 : (const T *)ct.S2c32;
  const T *Kd = fp64 ? (const T *)ct.K64 : (const T *)ct.K32;
  const int maxL = F.maxL_dist;
  {
    const Tab t1 = forest_tab(F, tab_key(6 + 16 * tier, 1, Q, 0), s);
    if (t1.count)
      PHS_LAUNCH("cheb_p2m", s, kf_cheb_p2m<T, 1, Q><<<(unsigned)t1.count, 64, 0, s>>>(
                                    F.dsys, t1.d, mask, in, Tk));
    const Tab t3 = forest_tab(F, tab_key(6 + 16 * tier, 3, Q, 0), s);
    if (t3.count)
      PHS_LAUNCH("cheb_p2m", s, kf_cheb_p2m<T, 3, Q><<<(unsigned)t3.count, 64, 0, s>>>(
                                    F.dsys, t3.d, mask, in, Tk));
  }
  const int thr = QQ <= 64 ? 64 : (QQ <= 128 ? 128 : 256);
  for (int lp = maxL - 1; lp >= 2; --lp) {
    const Tab tb = forest_tab(F, tab_key(7 + 16 * tier, 0, Q, lp), s);
    if (tb.count)
      PHS_LAUNCH("cheb_m2m", s, kf_cheb_m2m<T, Q><<<(unsigned)tb.count, thr, 0, s>>>(
                                    F.dsys, tb.d, mask, lp, Tpm));
  }
  {
    const Tab tb = forest_tab(F, tab_key(9 + 16 * tier, 0, Q, 0), s);
    if (tb.count)
    {
      if constexpr (std::is_same<T, double>::value)
        PHS_LAUNCH("cheb_m2l", s, kf_cheb_m2l_mfma<QQ><<<(unsigned)tb.count, 256, 0, s>>>(
                                      F.dsys, tb.d, mask, Kd));
      else
        PHS_LAUNCH("cheb_m2l", s, kf_cheb_m2l<T, QQ><<<(unsigned)tb.count, 256, 0, s>>>(
                                      F.dsys, tb.d, mask, Kd));
    }
  }
  for (int lc = 3; lc <= maxL; ++lc) {
    const Tab tb = forest_tab(F, tab_key(8 + 16 * tier, 0, Q, lc), s);
    if (tb.count)
      PHS_LAUNCH("cheb_l2l", s, kf_cheb_l2l<T, Q><<<(unsigned)tb.count, thr, 0, s>>>(
                                    F.dsys, tb.d, mask, lc, Tpm));
  }
}

template <class T, class TN, int Q>
void leaf_q(Forest &F, const int32_t *mask, int in, int out, const ChebTables &ct,
            const double *logtab, int tier, hipStream_t s) {
  const bool fp64 = std::is_same<T, double>::value;
  const T *Tk = fp64 ? (const T *)ct.nodes64 + Q : (const T *)ct.nodes32 + Q;
  const Tab t1 = forest_tab(F, tab_key(6 + 16 * tier, 1, Q, 0), s);
  if (t1.count)
    PHS_LAUNCH("cheb_leaf_eval", s, kf_cheb_leaf_eval<T, TN, 1, Q><<<(unsigned)t1.count, 64, 0, s>>>(
                                        F.dsys, t1.d, mask, in, out, Tk, logtab));
  const Tab t3 = forest_tab(F, tab_key(6 + 16 * tier, 3, Q, 0), s);
  if (t3.count)
    PHS_LAUNCH("cheb_leaf_eval", s, kf_cheb_leaf_eval<T, TN, 3, Q><<<(unsigned)t3.count, 64, 0, s>>>(
                                        F.dsys, t3.d, mask, in, out, Tk, logtab));
}

// One far-field pass (and, with `leaf`, the leaf pass) at Q nodes per axis;
// `ct` holds the tables of that Q.
template <class T, class TN>
void run_q(Forest &F, const int32_t *mask, int in, int out, bool leaf, int Q,
           const ChebTables &ct, const double *logtab, int tier, hipStream_t s) {
  switch (Q) {
    case 8:
      far_field_q<T, 8>(F, mask, in, ct, tier, s);
      if (leaf) leaf_q<T, TN, 8>(F, mask, in, out, ct, logtab, tier, s);
      break;
    case 10:
      far_field_q<T, 10>(F, mask, in, ct, tier, s);
      if (leaf) leaf_q<T, TN, 10>(F, mask, in, out, ct, logtab, tier, s);
      break;
    case 12:
      far_field_q<T, 12>(F, mask, in, ct, tier, s);
      if (leaf) leaf_q<T, TN, 12>(F, mask, in, out, ct, logtab, tier, s);
      break;
    case 14:
      far_field_q<T, 14>(F, mask, in, ct, tier, s);
      if (leaf) leaf_q<T, TN, 14>(F, mask, in, out, ct, logtab, tier, s);
      break;
    case 16:
      far_field_q<T, 16>(F, mask, in, ct, tier, s);
      if (leaf) leaf_q<T, TN, 16>(F, mask, in, out, ct, logtab, tier, s);
      break;
    default:
      throw Error{PHS_ERR_INVALID_ARGUMENT, "Chebyshev order must be 8, 10, 12, 14 or 16"};
  }
}

template <int Q>
void eval_q(Plan &pl, const double *w_tree, const double *beta, const double *targets,
            int64_t m, double *out, hipStream_t s) {
  constexpr int QQ = Q * Q;
  const int L = pl.tree.L;
  const ChebTables &ct = pl.qe == pl.q64 ? pl.ct64 : pl.cte;
  const double *Tk = ct.nodes64 + Q;
  const double *W = (const double *)pl.sw.mp;
  const double *GL = (const double *)pl.sw.loc + cheb_level_base(L, QQ, pl.R);
  const int64_t nb = (m + 127) / 128;
  if (pl.k == 1)
    PHS_LAUNCH("eval_targets", s, k_cheb_eval_targets<1, Q><<<nb, 128, 0, s>>>(
        targets, m, pl.c[0], pl.c[1], pl.rho, pl.x, pl.y, w_tree, pl.tree.leaf_start, L,
        pl.tree.h, Tk, ct.nodes64, W, GL, beta, pl.d, out, pl.xy2, pl.neartab));
  else
    PHS_LAUNCH("eval_targets", s, k_cheb_eval_targets<3, Q><<<nb, 128, 0, s>>>(
        targets, m, pl.c[0], pl.c[1], pl.rho, pl.x, pl.y, w_tree, pl.tree.leaf_start, L,
        pl.tree.h, Tk, ct.nodes64, W, GL, beta, pl.d, out, pl.xy2, pl.neartab));
}

std::vector<double> cheb_nodes(int Q) {
  std::vector<double> xm(Q);
  for (int a = 0; a < Q; ++a) xm[a] = std::cos((2 * a + 1) * M_PI / (2.0 * Q));
  return xm;
}

double basis_host(int Q, const std::vector<double> &xm, int a, double x) {
  double s = 1.0;
  double tkm = 1.0, tk = x;
  for (int k = 1; k < Q; ++k) {
    s += 2.0 * tk * std::cos(k * std::acos(xm[a]));
    const double nx = 2.0 * x * tk - tkm;
    tkm = tk;
    tk = nx;
  }
  return s / Q;
}

template <class T>
T *upload(const std::vector<double> &v) {
  std::vector<T> c(v.begin(), v.end());
  T *d = dmalloc<T>(c.size());
  PHS_HIP(hipMemcpy(d, c.data(), c.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

}  // namespace

void build_cheb_tables(ChebTables &t, int Q) {
  free_cheb_tables(t);
  t.Q = Q;
  const int QQ = Q * Q;
  const std::vector<double> xm = cheb_nodes(Q);
  // nodes followed by T_k(xbar_a) [k][a]
  std::vector<double> nt(Q + QQ);
  for (int a = 0; a < Q; ++a) nt[a] = xm[a];
  for (int k = 0; k < Q; ++k)
    for (int a = 0; a < Q; ++a) nt[Q + k * Q + a] = std::cos(k * std::acos(xm[a]));
  // Tpm[s][a][a'] = S_a((xbar_a' + (2s - 1))/2)
  std::vector<double> tpm(2 * QQ);
  for (int sgn = 0; sgn < 2; ++sgn)
    for (int a = 0; a < Q; ++a)
      for (int ap = 0; ap < Q; ++ap)
        tpm[sgn * QQ + a * Q + ap] = basis_host(Q, xm, a, (xm[ap] + (2 * sgn - 1)) * 0.5);
  // K_D at unit half-width, offsets in the M2L loop order (D = -o)
  std::vector<double> K((size_t)kNoff * QQ * QQ);
  int oi = 0;
  for (int oy = -3; oy <= 3; ++oy)
    for (int ox = -3; ox <= 3; ++ox) {
      if (std::abs(ox) <= 1 && std::abs(oy) <= 1) continue;
      const double Dx = -ox, Dy = -oy;
      for (int m = 0; m < QQ; ++m)
        for (int nn = 0; nn < QQ; ++nn) {
          const double dx = 2.0 * Dx + xm[m / Q] - xm[nn / Q];
          const double dy = 2.0 * Dy + xm[m % Q] - xm[nn % Q];
          K[((size_t)oi * QQ + m) * QQ + nn] = std::sqrt(dx * dx + dy * dy);
        }
      ++oi;
    }
  t.nodes64 = upload<double>(nt);
  t.nodes32 = upload<float>(nt);
  t.S2c64 = upload<double>(tpm);
  t.S2c32 = upload<float>(tpm);
  t.K64 = upload<double>(K);
  t.K32 = upload<float>(K);
}

void free_cheb_tables(ChebTables &t) {
  dfree(t.nodes64);
  dfree(t.nodes32);
  dfree(t.S2c64);
  dfree(t.S2c32);
  dfree(t.K64);
  dfree(t.K32);
  t = ChebTables();
}

size_t cheb_expansion_bytes(int L, int Q, int nd, bool fp64) {
  return (size_t)cheb_level_base(L + 1, Q * Q, nd) * (fp64 ? 8 : 4);
}

// One pass per distinct Chebyshev order among the odd-k systems (plans of
// different sizes may use different orders).
void dist_matvec(Forest &F, const int32_t *mask, int in, int out, int precision,
                 hipStream_t s) {
  const int tier = precision == PHS_MIXED ? 1 : (precision == PHS_FP64_EVAL ? 2 : 0);
  std::vector<int> done;
  for (const Plan *p : F.plan) {
    if (p->core_log || p->direct) continue;
    const int Q = tier == 1 ? p->q32 : (tier == 2 ? p->qe : p->q64);
    if (std::find(done.begin(), done.end(), Q) != done.end()) continue;
    done.push_back(Q);
    if (precision == PHS_MIXED)
      run_q<float, float>(F, mask, in, out, true, Q, p->ct32, p->neartab, tier, s);
    else if (precision == PHS_FP64_EVAL)
      run_q<double, double>(F, mask, in, out, true, Q, p->qe == p->q64 ? p->ct64 : p->cte,
                            p->neartab, tier, s);
    else if (precision == PHS_NEAR32)
      run_q<double, float>(F, mask, in, out, true, Q, p->ct64, p->neartab, tier, s);
    else
      run_q<double, double>(F, mask, in, out, true, Q, p->ct64, p->neartab, tier, s);
  }
}

void dist_expansions(Plan &pl, int in, hipStream_t s) {
  Forest &F = *pl.self;
  run_q<double, double>(F, F.mask[0], in, 0, false, pl.qe, pl.qe == pl.q64 ? pl.ct64 : pl.cte,
                        pl.neartab, 2, s);
}

void dist_eval_targets(Plan &pl, const double *w_tree, const double *beta,
                       const double *targets, int64_t m, double *out, hipStream_t s) {
  switch (pl.qe) {
    case 8: eval_q<8>(pl, w_tree, beta, targets, m, out, s); break;
    case 10: eval_q<10>(pl, w_tree, beta, targets, m, out, s); break;
    case 12: eval_q<12>(pl, w_tree, beta, targets, m, out, s); break;
    case 14: eval_q<14>(pl, w_tree, beta, targets, m, out, s); break;
    case 16: eval_q<16>(pl, w_tree, beta, targets, m, out, s); break;
    default: throw Error{PHS_ERR_INVALID_ARGUMENT, "bad Chebyshev order"};
  }
}

}  // namespace phs
