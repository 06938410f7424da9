// angular.h -- the angular functions of the S_{n,k} sums (Sec. II.D) at a unit
// bond vector u = r_ij / r_ij, for the float32 kernels.
//
// S_{n,k} sums g_n(r_ij) b_k / r_ij^l; since b_k is homogeneous of degree l,
// b_k / r^l is b_k evaluated at u.  For l <= 4 the polynomials are the 24
// listed with eq. (S_nk), with r^2 = 1 substituted (they agree with the
// printed ones on the unit sphere).  For l = 5, 6 they are the real solid
// harmonics P_l^{(m)}(z) {Re, Im}(x + i y)^m (P_l^{(m)} the m-th derivative of
// the Legendre polynomial), ordered m = 0, then (cos, sin) for m = 1..l.
//
// The gradient callbacks receive the gradient of the polynomial as a
// function of (x, y, z); because only its component tangent to the sphere
// matters, the kernels project sum_k w_k grad b_k once per bond:
//   d(b_k(u))/d r_ij = (I - u u^T) grad b_k(u) / r_ij.
#pragma once
#include <hip/hip_runtime.h>

#include "nep_internal.h"

namespace nep {

constexpr int num_poly(int L) { return (L + 1) * (L + 1) - 1; }

// Degree l of polynomial k: k runs over [l^2 - 1, (l+1)^2 - 2].
__host__ __device__ constexpr int degree_of(int k) {
  int l = 1;
  while ((l + 1) * (l + 1) - 2 < k) ++l;
  return l;
}

struct Poly8 {
  double c[8];
};

constexpr double cfact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Coefficients of d^m/dz^m P_l(z) = sum_t c[t] z^t, from
// P_l(z) = 2^-l sum_j (-1)^j (2l-2j)! / (j! (l-j)! (l-2j)!) z^(l-2j).
constexpr Poly8 legendre_dm(int l, int m) {
  double base[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double two_l = 1.0;
  for (int i = 0; i < l; ++i) two_l *= 2.0;
  for (int j = 0; 2 * j <= l; ++j) {
    double sgn = (j % 2) ? -1.0 : 1.0;
    base[l - 2 * j] = sgn * cfact(2 * l - 2 * j) / (cfact(j) * cfact(l - j) * cfact(l - 2 * j)) / two_l;
  }
  Poly8 p{{0, 0, 0, 0, 0, 0, 0, 0}};
  for (int t = 0; t + m <= l; ++t) p.c[t] = base[t + m] * cfact(t + m) / cfact(t);
  return p;
}

template <int l, int m, class Fn>
__device__ __forceinline__ void high_terms(float z, const float* Cm, const float* Sm, Fn& fn) {
  if constexpr (m <= l) {
    constexpr Poly8 p = legendre_dm(l, m);
    float Q = 0.f, dQ = 0.f;
#pragma unroll
    for (int t = l - m; t >= 0; --t) {
      dQ = dQ * z + Q;
      Q = Q * z + (float)p.c[t];
    }
    constexpr int k0 = l * l - 1;
    if constexpr (m == 0) {
      fn(k0, Q, 0.f, 0.f, dQ);
    } else {
      const float mf = (float)m;
      fn(k0 + 2 * m - 1, Q * Cm[m], Q * mf * Cm[m - 1], -Q * mf * Sm[m - 1], dQ * Cm[m]);
      fn(k0 + 2 * m, Q * Sm[m], Q * mf * Sm[m - 1], Q * mf * Cm[m - 1], dQ * Sm[m]);
    }
    high_terms<l, m + 1>(z, Cm, Sm, fn);
  }
}

// fn(k, b_k, db/dx, db/dy, db/dz) for k = 0 .. num_poly(L) - 1.
template <int L, class Fn>
__device__ __forceinline__ void angular_terms(float x, float y, float z, Fn&& fn) {
  const float x2 = x * x, y2 = y * y, z2 = z * z;
  const float xy = x * y, xz = x * z, yz = y * z;
  fn(0, z, 0.f, 0.f, 1.f);
  fn(1, x, 1.f, 0.f, 0.f);
  fn(2, y, 0.f, 1.f, 0.f);
  if constexpr (L >= 2) {
    fn(3, 3.f * z2 - 1.f, 0.f, 0.f, 6.f * z);
    fn(4, xz, z, 0.f, x);
    fn(5, yz, 0.f, z, y);
    fn(6, x2 - y2, 2.f * x, -2.f * y, 0.f);
    fn(7, 2.f * xy, 2.f * y, 2.f * x, 0.f);
  }
  if constexpr (L >= 3) {
    const float a5 = 5.f * z2 - 1.f, dxy = x2 - y2;
    fn(8, (5.f * z2 - 3.f) * z, 0.f, 0.f, 15.f * z2 - 3.f);
    fn(9, a5 * x, a5, 0.f, 10.f * xz);
    fn(10, a5 * y, 0.f, a5, 10.f * yz);
    fn(11, dxy * z, 2.f * xz, -2.f * yz, dxy);
    fn(12, 2.f * xy * z, 2.f * yz, 2.f * xz, 2.f * xy);
    fn(13, (x2 - 3.f * y2) * x, 3.f * dxy, -6.f * xy, 0.f);
    fn(14, (3.f * x2 - y2) * y, 6.f * xy, 3.f * dxy, 0.f);
  }
  if constexpr (L >= 4) {
    const float a7 = 7.f * z2 - 3.f, b7 = 7.f * z2 - 1.f, dxy = x2 - y2;
    const float c3 = x2 - 3.f * y2, s3 = 3.f * x2 - y2;
    fn(15, (35.f * z2 - 30.f) * z2 + 3.f, 0.f, 0.f, (140.f * z2 - 60.f) * z);
    fn(16, a7 * xz, a7 * z, 0.f, (21.f * z2 - 3.f) * x);
    fn(17, a7 * yz, 0.f, a7 * z, (21.f * z2 - 3.f) * y);
    fn(18, b7 * dxy, 2.f * x * b7, -2.f * y * b7, 14.f * z * dxy);
    fn(19, b7 * 2.f * xy, 2.f * y * b7, 2.f * x * b7, 28.f * xy * z);
    fn(20, c3 * xz, 3.f * dxy * z, -6.f * xy * z, c3 * x);
    fn(21, s3 * yz, 6.f * xy * z, 3.f * dxy * z, s3 * y);
    fn(22, dxy * dxy - 4.f * x2 * y2, 4.f * x * c3, -4.f * y * s3, 0.f);
    fn(23, 4.f * dxy * xy, 4.f * y * s3, 4.f * x * c3, 0.f);
  }
  if constexpr (L >= 5) {
    float Cm[kMaxL + 1], Sm[kMaxL + 1];
    Cm[0] = 1.f;
    Sm[0] = 0.f;
#pragma unroll
    for (int m = 0; m < L; ++m) {
      Cm[m + 1] = x * Cm[m] - y * Sm[m];
      Sm[m + 1] = x * Sm[m] + y * Cm[m];
    }
    high_terms<5, 0>(z, Cm, Sm, fn);
    if constexpr (L >= 6) high_terms<6, 0>(z, Cm, Sm, fn);
  }
}

// Value-only variant: fn(k, b_k).
template <int L, class Fn>
__device__ __forceinline__ void angular_values(float x, float y, float z, Fn&& fn) {
  angular_terms<L>(x, y, z, [&](int k, float b, float, float, float)
                                __attribute__((always_inline)) { fn(k, b); });
}

}  // namespace nep
