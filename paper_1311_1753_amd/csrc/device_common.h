// Device helpers shared by the likelihood and normalisation-grid kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hf {

// ------------------------------------------------------------------ math
template <typename T> struct Mth;
template <> struct Mth<float> {
  static __device__ __forceinline__ float ex(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
  static __device__ __forceinline__ float ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_sqrtf(x); }
  static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ __forceinline__ float erfcx(float x) { return erfcxf(x); }
};
template <> struct Mth<double> {
  static __device__ __forceinline__ double ex(double x) { return ::exp(x); }
  static __device__ __forceinline__ double ln(double x) { return ::log(x); }
  static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
  static __device__ __forceinline__ double sqrt(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double rsqrt(double x) { return 1.0 / ::sqrt(x); }
  static __device__ __forceinline__ double erfcx(double x) { return ::erfcx(x); }
};

// Constant table accessor: double and float views of the same constants.
struct CS {
  const double* __restrict__ d;
  const float* __restrict__ f;
  template <typename T> __device__ __forceinline__ T get(int i) const;
};
template <> __device__ __forceinline__ double CS::get<double>(int i) const { return d[i]; }
template <> __device__ __forceinline__ float CS::get<float>(int i) const { return f[i]; }

template <typename T> struct Col;
template <> struct Col<double> { typedef double S; };
template <> struct Col<float> { typedef float S; };

// Small per-thread arrays indexed by wave-uniform values.  The compiler keeps
// a private array in VGPRs (indexed moves) only while it is a plain array of
// at most 128 bytes, so larger ones are split into two plain arrays.
template <typename T, int N, bool SPLIT = (N * sizeof(T) > 128)> struct RegArr;
template <typename T, int N> struct RegArr<T, N, false> {
  T a[N];
  __device__ __forceinline__ T get(int i) const { return a[i]; }
  __device__ __forceinline__ void set(int i, T v) { a[i] = v; }
};
template <typename T, int N> struct RegArr<T, N, true> {
  static constexpr int kA = 128 / sizeof(T);
  T a[kA];
  T b[N - kA];
  __device__ __forceinline__ T get(int i) const { return i < kA ? a[i] : b[i - kA]; }
  __device__ __forceinline__ void set(int i, T v) {
    if (i < kA) a[i] = v; else b[i - kA] = v;
  }
};

// ------------------------------------------------------------------ Dalitz pieces
template <typename T> struct Cx { T re, im; };
template <typename T> __device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// sqrt(B_J^2) * BW(sAB) for one resonance; `d` = m0^2 - sAB formed in double.
template <typename T>
__device__ __forceinline__ Cx<T> res_line(const CS& cs, int rb, int J, T sAB, T d) {
  const T thrP = cs.get<T>(rb + kResThrP), thrM = cs.get<T>(rb + kResThrM);
  const T inv_s = Mth<T>::rcp(sAB);
  T q2 = (sAB - thrP) * (sAB - thrM) * (T(0.25) * inv_s);
  q2 = q2 > T(0) ? q2 : T(0);
  const T q = Mth<T>::sqrt(q2);
  const T z = cs.get<T>(rb + kResR2) * q2;
  T B2 = T(1), qp = q;
  if (J == 1) {
    B2 = cs.get<T>(rb + kResBnum) * Mth<T>::rcp(T(1) + z);
    qp = q * q2;
  } else if (J == 2) {
    B2 = cs.get<T>(rb + kResBnum) * Mth<T>::rcp(z * z + T(3) * z + T(9));
    qp = q * q2 * q2;
  }
  const T mg = cs.get<T>(rb + kResKw) * qp * B2 * Mth<T>::rsqrt(sAB);  // m0 Gamma(s)
  const T den = Mth<T>::rcp(d * d + mg * mg);
  const T sb = J == 0 ? T(1) : Mth<T>::sqrt(B2);
  return {sb * d * den, sb * mg * den};
}

// Zemach spin factor; `diff` = sAC - sBC formed in double.
template <typename T>
__device__ __forceinline__ T zemach(const CS& cs, int rb, int J, T sAB, T diff) {
  if (J == 0) return T(1);
  const T inv_s = Mth<T>::rcp(sAB);
  const T z1 = diff + cs.get<T>(rb + kResZc1) * inv_s;
  if (J == 1) return z1;
  const T ta = sAB - cs.get<T>(rb + kResZtaC) + cs.get<T>(rb + kResZtaD) * inv_s;
  const T tb = sAB - cs.get<T>(rb + kResZtbC) + cs.get<T>(rb + kResZtbD) * inv_s;
  return z1 * z1 - ta * tb * T(1.0 / 3.0);
}

// Amplitudes A_k(s12, s13) (and, for TDDP, Abar_k = A_k(s13, s12)) of all
// resonances at one point; s12/s13/s23 in double.
template <typename T, bool TD>
__device__ __forceinline__ void dalitz_amps(const CS& cs, int c0, int R, double s12, double s13, double s23,
                                            Cx<T>* A, Cx<T>* Ab) {
  const int rbase = c0 + dz_res_base(R, TD);
#pragma unroll
  for (int k = 0; k < kMaxRes; ++k) {
    if (k < R) {
      const int rb = rbase + k * kResStride;
      const int ch = (int)cs.d[rb + kResCh];
      const int J = (int)cs.d[rb + kResJ];
      const double m02 = cs.d[rb + kResM02];
      // (sAB, sAC, sBC) for A; the swapped point for Abar
      double ab, ac, bc;
      if (ch == 23) { ab = s23; ac = s12; bc = s13; }
      else if (ch == 12) { ab = s12; ac = s13; bc = s23; }
      else { ab = s13; ac = s12; bc = s23; }
      const T sAB = (T)ab;
      const Cx<T> L = res_line<T>(cs, rb, J, sAB, (T)(m02 - ab));
      const T Z = zemach<T>(cs, rb, J, sAB, (T)(ac - bc));
      A[k] = {L.re * Z, L.im * Z};
      if (TD) {
        double ab2, ac2, bc2;
        if (ch == 23) { ab2 = s23; ac2 = s13; bc2 = s12; }
        else if (ch == 12) { ab2 = s13; ac2 = s12; bc2 = s23; }
        else { ab2 = s12; ac2 = s13; bc2 = s23; }
        Cx<T> L2 = L;
        const T sAB2 = (T)ab2;
        if (ch != 23) L2 = res_line<T>(cs, rb, J, sAB2, (T)(m02 - ab2));
        const T Z2 = zemach<T>(cs, rb, J, sAB2, (T)(ac2 - bc2));
        Ab[k] = {L2.re * Z2, L2.im * Z2};
      }
    }
  }
}

// Gaussian-resolution convolution of e^{-G t}, written without branches:
//   w = (G s^2 - t)/(sqrt2 s), g = e^{-t^2/(2 s^2)}
//   w > 0 : E = g erfcx(w) / 2
//   w <= 0: E = e^{G^2 s^2/2 - G t} - g erfcx(-w) / 2      (erfc(w) = 2 - erfc(-w))
//   dE/dG = (G s^2 - t) E - s g / sqrt(2 pi)
template <typename T>
__device__ __forceinline__ void econv(T t, T s, T G, T g, T& E, T& dE) {
  const T a = G * s * s - t;
  const T w = a * Mth<T>::rcp(s) * T(0.70710678118654752);
  const T ex = Mth<T>::erfcx(w > T(0) ? w : -w);
  const T half = T(0.5) * g * ex;
  if (w > T(0)) {
    E = half;
  } else {
    E = Mth<T>::ex(T(0.5) * G * G * s * s - G * t) - half;
  }
  dE = a * E - s * g * T(0.39894228040143268);
}

}  // namespace hf
