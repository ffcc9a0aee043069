// Device helpers shared by the FMM translation units: the PHS basis phi
// (eq. phs_fun), the separable factors of the even-power distance matrix
// (eq. norm_sep and the rank-(q+1)^2 factorisations behind eq.
// matvec_hadamard), and small complex arithmetic.
#pragma once

#include "phs_internal.h"

namespace phs {

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

template <int K>
__device__ __forceinline__ float phi_r2f(float r2) {
  // 0.5 * ln 2: log(r^2)/2 = log2(r^2) * ln2 / 2
  constexpr float kHalfLn2 = 0.34657359027997264f;
  if (r2 == 0.0f) return 0.0f;
  if constexpr (K == 1) return __fsqrt_rn(r2);
  else if constexpr (K == 2) return kHalfLn2 * r2 * __log2f(r2);
  else if constexpr (K == 3) return r2 * __fsqrt_rn(r2);
  else return kHalfLn2 * r2 * r2 * __log2f(r2);
}

}  // namespace phs
