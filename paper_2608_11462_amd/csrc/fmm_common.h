// Device helpers shared by the FMM translation units: the PHS basis phi
// (eq. phs_fun), the separable factors of the even-power distance matrix
// (eq. norm_sep and the rank-(q+1)^2 factorisations behind eq.
// matvec_hadamard), and small complex arithmetic.
#pragma once

#include "phs_internal.h"

namespace phs {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  xcd_remap gives XCD x the contiguous logical range
// [x*q + min(x, r), ...) of the nb workgroups (q = nb / 8, r = nb % 8), so
// neighbouring boxes share one XCD's L2.  A bijection on [0, nb).
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7;
  const int64_t x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

template <class T>
struct C2 {
  T re, im;
};

template <class T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) {
  return {a.re + b.re, a.im + b.im};
}

template <class T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <class T>
__device__ __forceinline__ C2<T> ld2(const typename Vec2<T>::type *p) {
  typename Vec2<T>::type v = *p;
  return {v.x, v.y};
}
template <class T>
__device__ __forceinline__ void st2(typename Vec2<T>::type *p, C2<T> c) {
  typename Vec2<T>::type v;
  v.x = c.re;
  v.y = c.im;
  *p = v;
}
// the same through the constant / global address spaces (component loads and
// stores of one aligned pair, merged into one 8- or 16-byte access)
template <class T>
__device__ __forceinline__ C2<T> ld2(cptr<typename Vec2<T>::type> p) {
  const cptr<T> q = (cptr<T>)p;
  return {q[0], q[1]};
}
template <class T>
__device__ __forceinline__ C2<T> ld2(gptr<typename Vec2<T>::type> p) {
  const gptr<T> q = (gptr<T>)p;
  return {q[0], q[1]};
}
template <class T>
__device__ __forceinline__ void st2(gptr<typename Vec2<T>::type> p, C2<T> c) {
  const gptr<T> q = (gptr<T>)p;
  q[0] = c.re;
  q[1] = c.im;
}

// z^e for 0 <= e < 64 by binary powering.
template <class T>
__device__ __forceinline__ C2<T> cpow_small(C2<T> z, int e) {
  C2<T> r = {T(1), T(0)};
  C2<T> b = z;
#pragma unroll
  for (int bit = 0; bit < 6; ++bit) {
    if ((e >> bit) & 1) r = cmul(r, b);
    b = cmul(b, b);
  }
  return r;
}

// Sum over each group of four consecutive lanes (DPP quad permutations), the
// result in all four lanes.  The whole quad must be active.
template <class T>
__device__ __forceinline__ T quad_sum(T v) {
  v += __builtin_amdgcn_update_dpp(T(0), v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  v += __builtin_amdgcn_update_dpp(T(0), v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  return v;
}

// Sum over each group of sixteen consecutive lanes (one DPP row: quad
// permutations, then the half-row and row mirrors), the result in all
// sixteen lanes.  The whole row must be active.
template <class T>
__device__ __forceinline__ T row_sum16(T v) {
  v = quad_sum(v);
  v += __builtin_amdgcn_update_dpp(T(0), v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  v += __builtin_amdgcn_update_dpp(T(0), v, 0x140, 0xF, 0xF, false);  // row_mirror
  return v;
}

// Number of core densities for order K.
template <int K> struct Rank;
template <> struct Rank<1> { static constexpr int R = 1; };
template <> struct Rank<2> { static constexpr int R = 4; };
template <> struct Rank<3> { static constexpr int R = 4; };
template <> struct Rank<4> { static constexpr int R = 9; };

// Target-side factors U_r(x) and source-side factors V_r(y) with
// |x - y|^{2q} = sum_r U_r(x) V_r(y), q = floor(K/2).
template <int K, class T>
__device__ __forceinline__ void ufac(double x, double y, T *u) {
  if constexpr (K == 1) {
    u[0] = T(1);
  } else if constexpr (K == 2 || K == 3) {
    double a = x * x + y * y;
    u[0] = T(a);
    u[1] = T(1);
    u[2] = T(-2.0 * x);
    u[3] = T(-2.0 * y);
  } else {
    double a = x * x + y * y;
    u[0] = T(a * a);
    u[1] = T(1);
    u[2] = T(-4.0 * a * x);
    u[3] = T(-4.0 * a * y);
    u[4] = T(-4.0 * x);
    u[5] = T(-4.0 * y);
    u[6] = T(x * x);
    u[7] = T(y * y);
    u[8] = T(x * y);
  }
}

template <int K, class T>
__device__ __forceinline__ void vfac(double x, double y, T *v) {
  if constexpr (K == 1) {
    v[0] = T(1);
  } else if constexpr (K == 2 || K == 3) {
    double b = x * x + y * y;
    v[0] = T(1);
    v[1] = T(b);
    v[2] = T(x);
    v[3] = T(y);
  } else {
    double b = x * x + y * y;
    v[0] = T(1);
    v[1] = T(b * b);
    v[2] = T(x);
    v[3] = T(y);
    v[4] = T(b * x);
    v[5] = T(b * y);
    v[6] = T(6.0 * x * x + 2.0 * y * y);
    v[7] = T(2.0 * x * x + 6.0 * y * y);
    v[8] = T(8.0 * x * y);
  }
}

// phi(r) from r^2, with phi(0) = 0.
template <int K>
__device__ __forceinline__ double phi_r2(double r2) {
  if (r2 == 0.0) return 0.0;
  if constexpr (K == 1) return sqrt(r2);
  else if constexpr (K == 2) return 0.5 * r2 * log(r2);
  else if constexpr (K == 3) return r2 * sqrt(r2);
  else return 0.5 * r2 * r2 * log(r2);
}

// phi(r) from r^2 in FP32 without the constant factor: r^2 log2(r^2) (k=2),
// r^4 log2(r^2) (k=4), r (k=1), r^3 (k=3); multiply the sum by
// phi_scale_f<K>() (0.5 ln 2 for even k).  r = 0 gives 0 (clamped r^2 for
// even k).
template <int K>
__device__ __forceinline__ float phi_r2f(float r2) {
  if constexpr (K == 1) return __fsqrt_rn(r2);
  else if constexpr (K == 3) return r2 * __fsqrt_rn(r2);
  else {
    r2 = fmaxf(r2, 1e-30f);
    const float v = r2 * __log2f(r2);
    return K == 4 ? v * r2 : v;
  }
}

template <int K>
__device__ __forceinline__ float phi_scale_f() {
  return (K % 2 == 0) ? 0.34657359027997264f : 1.0f;  // 0.5 * ln 2
}

// sum_j phi(r) t_j (FP32, without phi_scale_f) over the sources js..je-1 of one
// leaf: coordinates relative to that leaf's centre, the target (xc, yc)
// already moved into the same frame.  The source values are wave-uniform, so
// they arrive by scalar loads, which complete out of order: a wait for one
// load is a wait for all.  Batches of eight therefore run one behind their
// loads: wait for the current batch, form its coordinate differences, issue
// the next batch's loads (the last batch re-reads itself, so no branch
// surrounds them), then evaluate phi while they land.  The scheduling
// barriers keep the compiler from moving the loads above the wait.  Terms are
// added in source order.
template <int K, class PF>
__device__ __forceinline__ float near_range_f32(float xc, float yc, PF ux, PF uy, PF tf, int js,
                                                int je) {
  float acc = 0.0f;
  const int nb = (je - js) / 8;  // full batches
  int j = js;
  if (nb > 0) {
    float cx[8], cy[8], ct[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      cx[i] = ux[j + i];
      cy[i] = uy[j + i];
      ct[i] = tf[j + i];
    }
    for (int b = 0; b < nb; ++b, j += 8) {
      float dx[8], dy[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        dx[i] = xc - cx[i];
        dy[i] = yc - cy[i];
      }
      __builtin_amdgcn_sched_barrier(0);
      const int jn = b + 1 < nb ? j + 8 : j;
      float nx[8], ny[8], nt[8];
      const PF px = ux + jn, py = uy + jn, pt = tf + jn;  // one base, constant offsets
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        nx[i] = px[i];
        ny[i] = py[i];
        nt[i] = pt[i];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < 8; ++i) acc += phi_r2f<K>(dx[i] * dx[i] + dy[i] * dy[i]) * ct[i];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        cx[i] = nx[i];
        cy[i] = ny[i];
        ct[i] = nt[i];
      }
    }
  }
  for (; j < je; ++j) {
    const float dx = xc - ux[j], dy = yc - uy[j];
    acc += phi_r2f<K>(dx * dx + dy * dy) * tf[j];
  }
  return acc;
}

// ---------------------------------------------------------------- near field
// Natural logarithm of a positive normal double by table-driven range
// reduction (Tang's method): x = m 2^e, m in [1, 2), c_j = 1 + j/128 from the
// top seven mantissa bits, r = (m - c_j) * (1/c_j) (m - c_j is exact), and
// log x = e ln2 + log c_j + log1p(r) with a degree-7 series for |r| < 1/128.
// tab: 1/c_j for j < 128, then log c_j.  Error: about one ulp of |log x|.
constexpr double kLn2Hi = 6.93147180369123816490e-01;  // 0x1.62e42fefa3800p-1
constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln2 - kLn2Hi

template <class PT>
__device__ __forceinline__ double tang_log(double x, PT tab) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t hi = (uint32_t)(b >> 32), lo = (uint32_t)b;
  const int e = (int)(hi >> 20) - 1023;
  const double m = __hiloint2double((int)((hi & 0x000FFFFFu) | 0x3FF00000u), (int)lo);
  const int j = (int)((hi >> 13) & 127u);
  const double c = fma((double)j, 0.0078125, 1.0);
  const double r = (m - c) * tab[j];
  double p = 1.0 / 7.0;
  p = fma(p, r, -1.0 / 6.0);
  p = fma(p, r, 1.0 / 5.0);
  p = fma(p, r, -0.25);
  p = fma(p, r, 1.0 / 3.0);
  p = fma(p, r, -0.5);
  const double l1p = fma(r * r, p, r);
  const double ed = (double)e;
  return fma(ed, kLn2Hi, tab[128 + j]) + fma(ed, kLn2Lo, l1p);
}

// Host: fill the 256-entry table used by tang_log.
void fill_log_table(double *tab);

// log x for the near field, where phi = r^k log r enters sums of O(1) terms and
// an absolute error of a few 1e-16 suffices: x = 2^e m with m in [1/2, 1)
// (frexp), c = (1 + (j + 1/2)/256)/2 the centre of the subinterval of m given
// by the top eight fraction bits j, r = m (1/c) - 1 in one fused multiply-add
// (|r| <= 2^-9), log1p(r) by its degree-5 Taylor polynomial (remainder
// < |r|^6/6 < 1e-17), log x = e ln2 - log(1/c) + log1p(r), where the table
// holds the rounded 1/c and minus the logarithm of that rounded value, so the
// rounding of 1/c cancels.  Absolute error about 1e-16.  tab: the pairs
// (1/c, -log(1/c)) for j = 0..255, interleaved, so a lookup is one 16-byte
// read (in LDS that halves the reads, and the bank conflicts, against two
// separate halves).  x = 0 gives a finite value (m = 0, e = 0), so x log x
// and x^2 log x are exactly 0 there.
__device__ __forceinline__ double near_log_core(double x, double invc, double logc) {
  const double m = __builtin_amdgcn_frexp_mant(x);
  const int e = __builtin_amdgcn_frexp_exp(x);
  const double r = fma(m, invc, -1.0);
  // log1p(r) = sum_k (-1)^(k+1) r^k / k to the degree whose remainder
  // |r|^(d+1)/(d+1) with |r| <= 2^-(bits+1) is below 2e-16 (bits 8: degree 5)
  constexpr int deg = kNearLogBits >= 9 ? 4 : kNearLogBits >= 8 ? 5 : kNearLogBits >= 6 ? 7 : 10;
  double p = (deg % 2 ? 1.0 : -1.0) / deg;
#pragma unroll
  for (int k = deg - 1; k >= 1; --k) p = fma(p, r, (k % 2 ? 1.0 : -1.0) / k);
  return fma((double)e, 0.69314718055994530942, fma(p, r, logc));
}
// near_log_core after its first step, r = frexp_mant(x) * invc - 1, was
// taken by the caller (the same operations in the same order)
__device__ __forceinline__ double near_log_rest(double x, double r, double logc) {
  const int e = __builtin_amdgcn_frexp_exp(x);
  constexpr int deg = kNearLogBits >= 9 ? 4 : kNearLogBits >= 8 ? 5 : kNearLogBits >= 6 ? 7 : 10;
  double p = (deg % 2 ? 1.0 : -1.0) / deg;
#pragma unroll
  for (int k = deg - 1; k >= 1; --k) p = fma(p, r, (k % 2 ? 1.0 : -1.0) / k);
  return fma((double)e, 0.69314718055994530942, fma(p, r, logc));
}
// byte offset of the table entry of a value whose high word is hi
__device__ __forceinline__ uint32_t near_log_offset(uint32_t hi) {
  return (hi >> (16 - kNearLogBits)) & ((((uint32_t)1 << kNearLogBits) - 1) << 4);
}
template <class PT>
__device__ __forceinline__ double near_log(double x, PT tab) {
  const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(x) >> 32);
  const int j = (int)(near_log_offset(hi) >> 4);
  return near_log_core(x, tab[2 * j], tab[2 * j + 1]);
}
// Host: fill the table of near_log (kNearLogTab doubles).
void fill_near_log_table(double *tab);

// sum_j phi(|x_i - y_j|) t_j over a contiguous source range, FP64.  xy2
// points to the interleaved source coordinates (x0, y0, x1, y1, ...); tab is
// the near_log table.  For even k the r = 0 term is exactly 0, as near_log(0)
// is finite.  Returns the sum without the factor 1/2 of
// phi = r^k log r = (1/2) r^k log r^2 for even k.
template <int K, class PXY, class PT, class PTAB>
__device__ __forceinline__ double near_range(double xi, double yi, PXY xy2, PT t, int js,
                                             int je, PTAB tab) {
  double acc = 0.0;
#pragma unroll 4
  for (int j = js; j < je; ++j) {
    const double sx = xy2[2 * j], sy = xy2[2 * j + 1];
    const double dx = xi - sx, dy = yi - sy;
    double r2 = fma(dy, dy, dx * dx);
    if constexpr (K == 1) {
      acc = fma(sqrt(r2), t[j], acc);
    } else if constexpr (K == 3) {
      acc = fma(r2 * sqrt(r2), t[j], acc);
    } else {
      double ph = r2 * near_log(r2, tab);
      if constexpr (K == 4) ph *= r2;
      acc = fma(ph, t[j], acc);
    }
  }
  return acc;
}

// near_range in batches of eight sources, pipelined: the eight sources'
// coordinates and densities are wave-uniform (wide scalar loads from one base
// address); the next batch's are requested once this batch's eight table
// reads have been waited for, so they are in flight during its logarithms.
// (Scalar and LDS loads share one completion counter and scalar loads return
// out of order: a scalar load issued before a table read would be waited for
// with it.)  Even k only; the sums are bitwise those of near_range (same
// operations in the same order).
template <int K, class PXY, class PT, class PTAB>
__device__ __forceinline__ double near_range8(double xi, double yi, PXY xy2, PT t, int js, int je,
                                              PTAB tab) {
  static_assert(K % 2 == 0, "even k");
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
    for (int bi = 0; bi < nfull; ++bi, j += 8) {
      double r2[8], ic[8], lc[8], rr[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const double dx = xi - sx[i], dy = yi - sy[i];
        r2[i] = fma(dy, dy, dx * dx);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(r2[i]) >> 32);
        // entry j (the top fraction bits) starts at byte 16 j: one shift, one mask
        const double2 e = *reinterpret_cast<const double2 *>(
            reinterpret_cast<const char *>(tab) + near_log_offset(hi));
        ic[i] = e.x;
        lc[i] = e.y;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) rr[i] = fma(__builtin_amdgcn_frexp_mant(r2[i]), ic[i], -1.0);
      __builtin_amdgcn_sched_barrier(0);
      double nsx[8], nsy[8], ntj[8];
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
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        sx[i] = nsx[i];
        sy[i] = nsy[i];
        tj[i] = ntj[i];
      }
    }
  }
  if (j < je) {
    // the last (je - js) mod 8 sources as one padded batch: loads clamped to
    // the range, padding with density 0 (each adds an exact zero)
    const int cnt = je - j;
    double r2[8], tj[8], ic[8], lc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int jj = i < cnt ? j + i : je - 1;
      const double dx = xi - xy2[2 * jj], dy = yi - xy2[2 * jj + 1];
      r2[i] = fma(dy, dy, dx * dx);
      const double tv = t[jj];
      tj[i] = i < cnt ? tv : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(r2[i]) >> 32);
      const double2 e = *reinterpret_cast<const double2 *>(
          reinterpret_cast<const char *>(tab) + near_log_offset(hi));
      ic[i] = e.x;
      lc[i] = e.y;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      double ph = r2[i] * near_log_core(r2[i], ic[i], lc[i]);
      if constexpr (K == 4) ph *= r2[i];
      acc = fma(ph, tj[i], acc);
    }
  }
  return acc;
}

template <int K>
__device__ __forceinline__ double near_scale() {
  return (K % 2 == 0) ? 0.5 : 1.0;
}

}  // namespace phs
