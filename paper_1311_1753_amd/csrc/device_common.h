// Device helpers shared by the likelihood and normalisation-grid kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "faddeeva_coef.h"
#include "internal.h"

namespace hf {

// Grid point t_k = lo + (k + 1/2) h of a numerical convolution, evaluated
// as written (no fused multiply-add), so that the residual-range decisions
// take the definition's double arithmetic.
__device__ __forceinline__ double conv_grid_point(double lo, double h, int k) {
#pragma clang fp contract(off)
  return lo + ((double)k + 0.5) * h;
}

// ------------------------------------------------------------------ math
template <typename T> struct Mth;
template <> struct Mth<float> {
  static __device__ __forceinline__ float ex(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
  static __device__ __forceinline__ float ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
  // m + ln(x) with one rounding less
  static __device__ __forceinline__ float ln_add(float x, float m) {
    return __builtin_fmaf(__builtin_amdgcn_logf(x), 0.693147180559945309f, m);
  }
  static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
  static __device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ __forceinline__ float lg2(float x) { return __builtin_amdgcn_logf(x); }
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_sqrtf(x); }
  static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
  static __device__ __forceinline__ float erfcx(float x) { return erfcxf(x); }
};
template <> struct Mth<double> {
  static __device__ __forceinline__ double ex(double x) { return ::exp(x); }
  static __device__ __forceinline__ double ln(double x) { return ::log(x); }
  static __device__ __forceinline__ double ln_add(double x, double m) { return m + ::log(x); }
  static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
  static __device__ __forceinline__ double ex2(double x) { return ::exp2(x); }
  static __device__ __forceinline__ double lg2(double x) { return ::log2(x); }
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

// Loop unrolled at compile time: f(std::integral_constant<int, 0>{}), ...,
// f(std::integral_constant<int, N - 1>{}).  Used where the index selects one
// of several register arrays, so that the selection is resolved before the
// arrays are placed.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------------------------ Dalitz pieces
// Per-event amplitudes: (re, im) pairs of the NR resonance places,
// written at wave-uniform runtime indices.  Each event's array is a separate
// plain array, picked by a compile-time event number, so that each is kept in
// registers on its own (a two-dimensional array indexed by a runtime
// resonance number would be placed in scratch memory).
template <typename T, int NR = kMaxRes> using AmpArr = T[2 * NR];
template <int e, class A>
__device__ __forceinline__ A& pick(A& x0, A& x1) {
  if constexpr (e == 0) return x0;
  else return x1;
}

template <typename T> struct Cx { T re, im; };
template <typename T> __device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// Kinematic quantities of one daughter pair at one point; they depend only on
// the pair's masses, so resonances in the same pair share them.  sAB, sAC,
// sBC are double; differences of invariants are formed in double.
template <typename T> struct Chan {
  double sABd;
  T inv_s, rs, q2, q, z1, z2;
};

template <typename T>
__device__ __forceinline__ Chan<T> chan_eval(const CS& cs, int cb, double sAB, double sAC, double sBC) {
  Chan<T> c;
  c.sABd = sAB;
  const T s = (T)sAB;
  c.inv_s = Mth<T>::rcp(s);
  c.rs = Mth<T>::rsqrt(s);
  T q2 = (s - cs.get<T>(cb + kChThrP)) * (s - cs.get<T>(cb + kChThrM)) * (T(0.25) * c.inv_s);
  c.q2 = q2 > T(0) ? q2 : T(0);
  c.q = Mth<T>::sqrt(c.q2);
  // Zemach factors: Z_1 = s_AC - s_BC + (M^2 - m_C^2)(m_B^2 - m_A^2)/s_AB,
  // Z_2 = Z_1^2 - (s_AB - 2M^2 - 2m_C^2 + (M^2-m_C^2)^2/s_AB)(s_AB - 2m_A^2 - 2m_B^2 + (m_A^2-m_B^2)^2/s_AB)/3
  c.z1 = (T)(sAC - sBC) + cs.get<T>(cb + kChZc1) * c.inv_s;
  const T ta = s - cs.get<T>(cb + kChZtaC) + cs.get<T>(cb + kChZtaD) * c.inv_s;
  const T tb = s - cs.get<T>(cb + kChZtbC) + cs.get<T>(cb + kChZtbD) * c.inv_s;
  c.z2 = c.z1 * c.z1 - ta * tb * T(1.0 / 3.0);
  return c;
}

// Zemach factor for the swapped point of a pi pi channel (s_AC <-> s_BC).
template <typename T>
__device__ __forceinline__ Chan<T> chan_swap_ac_bc(const CS& cs, int cb, const Chan<T>& c, double sAC, double sBC) {
  Chan<T> d = c;
  d.z1 = (T)(sBC - sAC) + cs.get<T>(cb + kChZc1) * c.inv_s;
  const T s = (T)c.sABd;
  const T ta = s - cs.get<T>(cb + kChZtaC) + cs.get<T>(cb + kChZtaD) * c.inv_s;
  const T tb = s - cs.get<T>(cb + kChZtbC) + cs.get<T>(cb + kChZtbD) * c.inv_s;
  d.z2 = d.z1 * d.z1 - ta * tb * T(1.0 / 3.0);
  return d;
}

// Resonance amplitude B_J(q) Z_J BW(s_AB) with the mass-dependent width
// m0 Gamma(s) = Kw q^{2J+1} B_J^2 / sqrt(s) and BW = 1/(m0^2 - s - i m0 Gamma).
// With the Blatt-Weisskopf factor B_J = B0 / sqrt(P_J(r^2 q^2)) (P_0 = 1,
// P_1 = 1 + z, P_2 = z^2 + 3z + 9, B0 = sqrt(P_J(r^2 q0^2))), everything but
// m0^2, Kw B0^2 and B0 depends only on the pair and the spin, so it is formed
// once per (pair, spin) group:
//   g  = q^{2J+1} / (P_J sqrt(s))     m0 Gamma(s) = (Kw B0^2) g
//   zf = Z_J / sqrt(P_J)              B_J Z_J = B0 zf
template <typename T> struct GroupQ { T g, zf; };

template <typename T, int J>
__device__ __forceinline__ GroupQ<T> group_q(T r2, const Chan<T>& c) {
  if (J == 0) return {c.q * c.rs, T(1)};
  const T z = r2 * c.q2;
  const T rp = Mth<T>::rsqrt(J == 1 ? T(1) + z : Mth<T>::fma(z, z + T(3), T(9)));
  const T qp = J == 1 ? c.q * c.q2 : c.q * c.q2 * c.q2;
  return {qp * (rp * rp) * c.rs, (J == 1 ? c.z1 : c.z2) * rp};
}

// One resonance: m0^2 - s is formed in double.
template <typename T>
__device__ __forceinline__ Cx<T> res_amp(const CS& cs, int rb, const GroupQ<T>& gq, double sABd) {
  const T d = (T)(cs.d[rb + kResM02] - sABd);
  const T mg = cs.get<T>(rb + kResKwB) * gq.g;  // m0 Gamma(s)
  const T den = Mth<T>::rcp(Mth<T>::fma(d, d, mg * mg));
  const T f = cs.get<T>(rb + kResSqB) * gq.zf * den;
  return {f * d, f * mg};
}

// Amplitudes of the resonances [k0, k1) of one (pair, spin) group, for E <= 2
// events at once, all with the pair quantities c[e] (and, for TD, cb[e] at
// the swapped point), into event e's array (a0, a1) at 2k, 2k + 1 (re, im)
// and the conjugate amplitudes into b0, b1.  The bounds are wave-uniform, so
// the writes are indexed register moves; each resonance's constants are read
// once for the E events.
template <typename T, int J, bool TD, int E, int NR>
__device__ __forceinline__ void res_group(const CS& cs, int rbase, T r2, int k0, int k1, const Chan<T> (&c)[E],
                                          const Chan<T> (&cb)[E], AmpArr<T, NR>& a0, AmpArr<T, NR>& a1,
                                          AmpArr<T, NR>& b0, AmpArr<T, NR>& b1) {
  if (k0 >= k1) return;
  GroupQ<T> gq[E], gb[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    gq[e] = group_q<T, J>(r2, c[e]);
    if (TD) gb[e] = group_q<T, J>(r2, cb[e]);
  }
  for (int k = k0; k < k1; ++k) {
    const int rb = rbase + k * kResStride;
    static_for<E>([&](auto ei) {
      constexpr int e = decltype(ei)::value;
      const Cx<T> v = res_amp<T>(cs, rb, gq[e], c[e].sABd);
      pick<e>(a0, a1)[2 * k] = v.re;
      pick<e>(a0, a1)[2 * k + 1] = v.im;
      if (TD) {
        const Cx<T> w = res_amp<T>(cs, rb, gb[e], cb[e].sABd);
        pick<e>(b0, b1)[2 * k] = w.re;
        pick<e>(b0, b1)[2 * k + 1] = w.im;
      }
    });
  }
}

// Amplitudes A_k(s12, s13) (and, for TDDP, Abar_k = A_k(s13, s12)) of all
// resonances of node `nd` at E <= 2 points into a0, a1 (b0, b1) as (re, im)
// pairs; s12/s13/s23 in double (b0, b1 are not touched without TD).  Pair quantities are
// evaluated once per pair (and, for the conjugate amplitudes, once per
// swapped pair); when m2 == m3 (SYM) the swapped 12 pair equals the 13 pair
// and vice versa.  The resonances are stored grouped by (pair, spin), so each
// group is one loop with the pair and spin fixed at compile time.  Absent
// resonance places (k >= R) get zero amplitudes.
template <typename T, bool TD, int E, int NR = kMaxRes>
__device__ __forceinline__ void dalitz_amps(const CS& cs, const KNode& nd, const double (&s12)[E],
                                            const double (&s13)[E], const double (&s23)[E], AmpArr<T, NR>& a0,
                                            AmpArr<T, NR>& a1, AmpArr<T, NR>& b0, AmpArr<T, NR>& b1) {
  const int R = nd.aux;
  const int chb = nd.c0 + dz_ch_base(R, TD), rbase = nd.c0 + dz_res_base(R, TD);
  // pair (A, B; C): 12 = (1, 2; 3), 13 = (1, 3; 2), 23 = (2, 3; 1)
  Chan<T> c12[E], c13[E], c23[E], b12[E], b13[E], b23[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    c12[e] = chan_eval<T>(cs, chb, s12[e], s13[e], s23[e]);
    c13[e] = chan_eval<T>(cs, chb + kChStride, s13[e], s12[e], s23[e]);
    c23[e] = chan_eval<T>(cs, chb + 2 * kChStride, s23[e], s12[e], s13[e]);
    b12[e] = c13[e];
    b13[e] = c12[e];
    b23[e] = c23[e];
  }
  if (TD) {
    // equal pair constants (m2 == m3) give bitwise equal pair quantities
    bool sym = true;
#pragma unroll
    for (int i = 0; i < kChStride; ++i) sym = sym && cs.d[chb + i] == cs.d[chb + kChStride + i];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!sym) {
        b12[e] = chan_eval<T>(cs, chb, s13[e], s12[e], s23[e]);
        b13[e] = chan_eval<T>(cs, chb + kChStride, s12[e], s13[e], s23[e]);
      }
      b23[e] = chan_swap_ac_bc<T>(cs, chb + 2 * kChStride, c23[e], s12[e], s13[e]);
    }
  }
  const int32_t* g = nd.res_end;
  const T r2 = cs.get<T>(nd.c0 + kDzR2);
  res_group<T, 0, TD, E, NR>(cs, rbase, r2, 0, g[0], c12, b12, a0, a1, b0, b1);
  res_group<T, 1, TD, E, NR>(cs, rbase, r2, g[0], g[1], c12, b12, a0, a1, b0, b1);
  res_group<T, 2, TD, E, NR>(cs, rbase, r2, g[1], g[2], c12, b12, a0, a1, b0, b1);
  res_group<T, 0, TD, E, NR>(cs, rbase, r2, g[2], g[3], c13, b13, a0, a1, b0, b1);
  res_group<T, 1, TD, E, NR>(cs, rbase, r2, g[3], g[4], c13, b13, a0, a1, b0, b1);
  res_group<T, 2, TD, E, NR>(cs, rbase, r2, g[4], g[5], c13, b13, a0, a1, b0, b1);
  res_group<T, 0, TD, E, NR>(cs, rbase, r2, g[5], g[6], c23, b23, a0, a1, b0, b1);
  res_group<T, 1, TD, E, NR>(cs, rbase, r2, g[6], g[7], c23, b23, a0, a1, b0, b1);
  res_group<T, 2, TD, E, NR>(cs, rbase, r2, g[7], g[8], c23, b23, a0, a1, b0, b1);
  for (int k = R; k < NR; ++k) {
    static_for<E>([&](auto ei) {
      constexpr int e = decltype(ei)::value;
      pick<e>(a0, a1)[2 * k] = pick<e>(a0, a1)[2 * k + 1] = T(0);
      if (TD) pick<e>(b0, b1)[2 * k] = pick<e>(b0, b1)[2 * k + 1] = T(0);
    });
  }
}

// The conjugate-pair amplitudes of one event one resonance at a time, with
// no per-event arrays: f(k, A_k, Abar_k) for every resonance k in place
// order (Abar_k = A_k(s13, s12), the same pair quantities as dalitz_amps).
// The double kernels of the full model take this form: sixteen places of
// double amplitudes do not fit the registers, and arrays indexed at run
// time would go to scratch memory.
template <typename T, int J, class F>
__device__ __forceinline__ void res_group_stream(const CS& cs, int rbase, T r2, int k0, int k1, const Chan<T>& c,
                                                 const Chan<T>& cb, const F& f) {
  if (k0 >= k1) return;
  const GroupQ<T> gq = group_q<T, J>(r2, c), gb = group_q<T, J>(r2, cb);
  for (int k = k0; k < k1; ++k) {
    const int rb = rbase + k * kResStride;
    f(k, res_amp<T>(cs, rb, gq, c.sABd), res_amp<T>(cs, rb, gb, cb.sABd));
  }
}

template <typename T, class F>
__device__ __forceinline__ void dalitz_stream(const CS& cs, const KNode& nd, double s12, double s13, double s23,
                                              const F& f) {
  const int R = nd.aux;
  const int chb = nd.c0 + dz_ch_base(R, true), rbase = nd.c0 + dz_res_base(R, true);
  const Chan<T> c12 = chan_eval<T>(cs, chb, s12, s13, s23);
  const Chan<T> c13 = chan_eval<T>(cs, chb + kChStride, s13, s12, s23);
  const Chan<T> c23 = chan_eval<T>(cs, chb + 2 * kChStride, s23, s12, s13);
  bool sym = true;
#pragma unroll
  for (int i = 0; i < kChStride; ++i) sym = sym && cs.d[chb + i] == cs.d[chb + kChStride + i];
  const Chan<T> b12 = sym ? c13 : chan_eval<T>(cs, chb, s13, s12, s23);
  const Chan<T> b13 = sym ? c12 : chan_eval<T>(cs, chb + kChStride, s12, s13, s23);
  const Chan<T> b23 = chan_swap_ac_bc<T>(cs, chb + 2 * kChStride, c23, s12, s13);
  const int32_t* g = nd.res_end;
  const T r2 = cs.get<T>(nd.c0 + kDzR2);
  res_group_stream<T, 0>(cs, rbase, r2, 0, g[0], c12, b12, f);
  res_group_stream<T, 1>(cs, rbase, r2, g[0], g[1], c12, b12, f);
  res_group_stream<T, 2>(cs, rbase, r2, g[1], g[2], c12, b12, f);
  res_group_stream<T, 0>(cs, rbase, r2, g[2], g[3], c13, b13, f);
  res_group_stream<T, 1>(cs, rbase, r2, g[3], g[4], c13, b13, f);
  res_group_stream<T, 2>(cs, rbase, r2, g[4], g[5], c13, b13, f);
  res_group_stream<T, 0>(cs, rbase, r2, g[5], g[6], c23, b23, f);
  res_group_stream<T, 1>(cs, rbase, r2, g[6], g[7], c23, b23, f);
  res_group_stream<T, 2>(cs, rbase, r2, g[7], g[8], c23, b23, f);
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

// Faddeeva function w(z) = exp(-z^2) erfc(-i z) for Im z >= 0 by Weideman's
// rational series in Z = (L + i z)/(L - i z) (coefficients and reference in
// faddeeva_coef.h; about 1e-14 relative in the upper half plane).
__device__ __forceinline__ Cx<double> faddeeva_uhp(Cx<double> z) {
  const double L = kFaddeevaL;
  // i z = (-Im z, Re z); den = L - i z, num = L + i z
  const double dre = L + z.im, dim = -z.re;
  const double nre = L - z.im, nim = z.re;
  const double r = 1.0 / (dre * dre + dim * dim);
  const Cx<double> rd = {dre * r, -dim * r};  // 1 / (L - i z)
  const Cx<double> Z = cmul(Cx<double>{nre, nim}, rd);
  Cx<double> p = {kFaddeevaA[0], 0.0};
#pragma unroll
  for (int n = 1; n < kFaddeevaN; ++n) {
    const Cx<double> q = cmul(p, Z);
    p = {q.re + kFaddeevaA[n], q.im};
  }
  const Cx<double> rd2 = cmul(rd, rd);
  const Cx<double> t = cmul(p, rd2);
  const double c = 0.56418958354775628;  // 1/sqrt(pi)
  return {2.0 * t.re + c * rd.re, 2.0 * t.im + c * rd.im};
}

// Gaussian-resolution convolution of e^{-z t} with complex z = G - i W
// (G > 0): its real part convolves e^{-G t} cos(W t), its imaginary part
// e^{-G t} sin(W t).  With xi = (z s^2 - t)/(sqrt2 s) and g = e^{-t^2/(2 s^2)}:
//   Re xi > 0 : E = g w(i xi) / 2
//   otherwise : E = e^{z^2 s^2/2 - z t} - g w(-i xi) / 2   (erfc(v) = 2 - erfc(-v))
//   dE/dz = (z s^2 - t) E - s g / sqrt(2 pi)
// The Faddeeva argument is in the upper half plane on both branches.
__device__ __forceinline__ void econv_c(double t, double s, double G, double W, double g, Cx<double>& E,
                                        Cx<double>& dE) {
  const double k = 0.70710678118654752 / s;
  const Cx<double> a = {G * s * s - t, -W * s * s};  // z s^2 - t
  const Cx<double> xi = {a.re * k, a.im * k};
  const bool pos = xi.re > 0.0;
  // i xi = (-Im xi, Re xi), -i xi = (Im xi, -Re xi)
  const Cx<double> arg = pos ? Cx<double>{-xi.im, xi.re} : Cx<double>{xi.im, -xi.re};
  const Cx<double> wv = faddeeva_uhp(arg);
  E = {0.5 * g * wv.re, 0.5 * g * wv.im};
  if (!pos) {
    // exponent z^2 s^2/2 - z t = (G^2 - W^2) s^2/2 - G t + i (W t - G W s^2)
    const double er = 0.5 * (G * G - W * W) * s * s - G * t, ei = W * t - G * W * s * s;
    const double m = ::exp(er);
    double sn, cn;
    ::sincos(ei, &sn, &cn);
    E = {m * cn - E.re, m * sn - E.im};
  }
  const Cx<double> aE = cmul(a, E);
  dE = {aE.re - s * g * 0.39894228040143268, aE.im};
}

}  // namespace hf
