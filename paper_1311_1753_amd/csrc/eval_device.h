// Per-event likelihood kernels for gfx950 (CDNA4, wave64).
//
// Work split.  The events of a dataset form chunks of 256 consecutive events
// (one per thread of a 256-thread block; every column load is a fully
// coalesced 256-lane access).  The chunks are divided into n_rows contiguous,
// equal (+-1 chunk) ranges, one per block: n_rows is fixed per dataset (a few
// rows per compute unit), so the launch is a single balanced wave of blocks
// and each block reduces its accumulators once.  Per event a kernel evaluates
// the PDF (forward pass in log space), the derivatives d ln P / d theta of
// every gradient slot (reverse pass), and accumulates -ln P and the slot
// derivatives per thread in double.  The block then sums its threads in a
// fixed order (LDS, DPP lane exchanges, fixed lanes) and writes one row of
// partials; partials are stored column-major, [column][row].  A second kernel
// sums the rows of each fit in a fixed order.  A row depends only on its event
// range and the constant table, never on the grid or on other fits of the
// same launch, so a fit gives bit-identical results alone and batched.
//
// Precision: T = double (FP64 path) or float (FP32-eval path).  In the float
// path events are stored as float offsets from a per-column double
// reference; location differences (x - a, x - mu, m0^2 - s) are formed from
// the stored offset and a double constant (in double, or as a float hi + lo
// pair), then rounded once.
#pragma once

#include <algorithm>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "dp_inside.h"
#include "internal.h"
#include "kernels.h"

namespace hf {


// ------------------------------------------------------------------ leaves
// Each leaf returns ln P (ln of the unnormalised density when hoisted) and
// writes its local derivatives d ln P / d(slot) into dl[0..n_slot).

template <typename T>
__device__ __forceinline__ T leaf_exp(const CS& cs, int c0, bool hoisted, double x, T* dl) {
  const T u = (T)(x + cs.d[c0 + 0]);
  T lv = cs.get<T>(c0 + 1) * u;
  dl[0] = u;
  if (!hoisted) {
    lv = (lv - cs.get<T>(c0 + 2)) - cs.get<T>(c0 + 3);
    dl[0] = u - cs.get<T>(c0 + 4);
  }
  return lv;
}

template <typename T>
__device__ __forceinline__ T leaf_gauss(const CS& cs, int c0, bool hoisted, double x, T* dl) {
  const T isg = cs.get<T>(c0 + 1);
  const T z = (T)(x + cs.d[c0 + 0]) * isg;
  T lv = T(-0.5) * z * z;
  dl[0] = z * isg;
  dl[1] = z * z * isg;
  if (!hoisted) {
    lv = (lv - cs.get<T>(c0 + 2)) - cs.get<T>(c0 + 3);
    dl[0] -= cs.get<T>(c0 + 4);
    dl[1] -= cs.get<T>(c0 + 5);
  }
  return lv;
}

template <typename T>
__device__ __forceinline__ T leaf_poly(const CS& cs, int c0, int deg, bool hoisted, double x, T* dl) {
  const T u = (T)(x + cs.d[c0 + 0]);
  T p = T(0);
  for (int k = deg; k >= 1; --k) p = (p + cs.get<T>(c0 + k)) * u;
  p += T(1);
  const T ip = Mth<T>::rcp(p);
  T lv = p > T(0) ? Mth<T>::ln(p) : T(-INFINITY);
  T uk = u;
  for (int k = 1; k <= deg; ++k) {
    T v = uk * ip;
    if (!hoisted) v -= cs.get<T>(c0 + deg + 2 + k);
    dl[k - 1] = v;
    uk *= u;
  }
  if (!hoisted) lv = (lv - cs.get<T>(c0 + deg + 1)) - cs.get<T>(c0 + deg + 2);
  return lv;
}

// DALITZ: ln |1 + sum c_k A_k|^2 for E events at once (lv[e]); the slot
// derivatives d/d(Re c_k), d/d(Im c_k) of all E events go to emit(slot,
// values[E]) (stored by the tree interpreter, accumulated directly by the
// single-leaf kernels).  The sums run over all kMaxRes resonance places:
// absent ones have zero amplitude and coefficient, and emit zero derivatives
// for slots 2R .. 2 kMaxRes - 1, which the caller drops or adds harmlessly.
template <typename T, int E, class Emit>
__device__ __forceinline__ void leaf_dalitz(const CS& cs, const KNode& nd, bool hoisted, const double (&x12)[E],
                                            const double (&x13)[E], T (&lv)[E], const Emit& emit) {
  const int c0 = nd.c0, R = nd.aux;
  double s12[E], s13[E], s23[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    s12[e] = x12[e] + cs.d[c0 + kDzRef12];
    s13[e] = x13[e] + cs.d[c0 + kDzRef13];
    s23[e] = cs.d[c0 + kDzSsum] - s12[e] - s13[e];
  }
  static_assert(E == 1 || E == 2, "one or two events per step");
  AmpArr<T> a0, a1;
  dalitz_amps<T, false, E>(cs, nd, s12, s13, s23, a0, a1, a0, a1);
  const int cb = c0 + dz_coef_base(R, false);
  Cx<T> S[E];
  T inv[E];
  static_for<E>([&](auto ei) {
    constexpr int e = decltype(ei)::value;
    const AmpArr<T>& ae = pick<e>(a0, a1);
    S[e] = {T(1), T(0)};
#pragma unroll
    for (int k = 0; k < kMaxRes; ++k) {
      const Cx<T> t = cmul(Cx<T>{cs.get<T>(cb + 2 * k), cs.get<T>(cb + 2 * k + 1)}, Cx<T>{ae[2 * k], ae[2 * k + 1]});
      S[e].re += t.re;
      S[e].im += t.im;
    }
    const T a2 = S[e].re * S[e].re + S[e].im * S[e].im;
    inv[e] = T(2) * Mth<T>::rcp(a2);
    lv[e] = a2 > T(0) ? Mth<T>::ln(a2) : T(-INFINITY);
    if (!hoisted) lv[e] = (lv[e] - cs.get<T>(c0 + kDzLnHi)) - cs.get<T>(c0 + kDzLnLo);
  });
#pragma unroll
  for (int k = 0; k < kMaxRes; ++k) {
    T d_re[E], d_im[E];
    static_for<E>([&](auto ei) {
      constexpr int e = decltype(ei)::value;
      const AmpArr<T>& ae = pick<e>(a0, a1);
      // conj(S) A_k
      const T re = S[e].re * ae[2 * k] + S[e].im * ae[2 * k + 1];
      const T im = S[e].re * ae[2 * k + 1] - S[e].im * ae[2 * k];
      d_re[e] = re * inv[e];
      d_im[e] = -im * inv[e];
      if (!hoisted && k < R) {
        d_re[e] -= cs.get<T>(c0 + kDzDln + 2 * k);
        d_im[e] -= cs.get<T>(c0 + kDzDln + 2 * k + 1);
      }
    });
    emit(2 * k, d_re);
    emit(2 * k + 1, d_im);
  }
}

// One resonance of the full model at one point, its pair and spin known
// only at run time (wave-uniform): the amplitude A, 1 / (m0^2 - s - i m0
// Gamma(s)) = D and the width factor g of m0 Gamma(s) = (Kw B0^2) g, from
// which the mass and width derivatives follow (dA = A [D (-d(m0^2) + i g
// d(Kw B0^2)) + d ln B0]).
template <typename T>
__device__ __forceinline__ void res_amp_rt(const CS& cs, const KNode& nd, int k, int pair, int J, double s12,
                                           double s13, double s23, Cx<T>& A, Cx<T>& D, T& g) {
  const int R = nd.aux;
  const int cb = nd.c0 + dz_ch_base(R, true) + pair * kChStride;
  const double sAB = pair == 0 ? s12 : (pair == 1 ? s13 : s23);
  const double sAC = pair == 0 ? s13 : s12;
  const double sBC = pair == 2 ? s13 : s23;
  const Chan<T> c = chan_eval<T>(cs, cb, sAB, sAC, sBC);
  const T r2 = cs.get<T>(nd.c0 + kDzR2);
  const GroupQ<T> gq = J == 0 ? group_q<T, 0>(r2, c) : (J == 1 ? group_q<T, 1>(r2, c) : group_q<T, 2>(r2, c));
  const int rb = nd.c0 + dz_res_base(R, true) + k * kResStride;
  const T d = (T)(cs.d[rb + kResM02] - sAB);
  const T mg = cs.get<T>(rb + kResKwB) * gq.g;
  const T den = Mth<T>::rcp(Mth<T>::fma(d, d, mg * mg));
  const T f = cs.get<T>(rb + kResSqB) * gq.zf * den;
  A = {f * d, f * mg};
  D = {d * den, mg * den};
  g = gq.g;
}

// Tail receiver of the plain kernels (they emit every slot through emit).
struct NoTail {
  template <class J, class V> __device__ __forceinline__ void operator()(J, const V&) const {}
};

// TDDP: ln [a_c C + a_0 Cz + a_s S + b_s Sz] for E events at once, with
// b_s = -Im(conj(A) Abar) and Cz + i Sz the resolution-convolved
// e^{-t/tau} e^{i x t/tau} (without x: Cz = E(t; 1/tau), Sz = 0); slot
// derivatives (coefficients, then tau, y and, with x, x) go to emit(slot,
// values[E]), the coefficients' first over all NR places as for DALITZ,
// then tau, y (, x) to slots 2R, 2R + 1 (, 2R + 2) after any zero emitted
// there.
// FULL (the mixing fit's model, E = 1): Abar carries q/p, the trigonometric
// terms are always formed (W = 0 without x), and the slots after the
// coefficients go to tail(integral_constant<j>, values) with j = 0 tau,
// 1 y, 2 x, 3 |q/p|, 4 arg q/p, 5 + 2f and 6 + 2f the mass and width of
// floating resonance f (only those the node has are emitted).
// NORM (full model, in double): one cell of the normalisation grid instead
// of an event; the time factors are their integrals over the real line,
// lv receives |A|^2 and tail 0, 1, 2 receive |Abar'|^2, a_s, b_s (their
// sums give the normalisation and its tau, y, x derivatives); emit and the
// q/p and shape tails receive derivatives of the time-integrated rate
// itself (not divided by it).
template <typename T, int E, bool HX, int NR = kMaxRes, bool FULL = false, bool NORM = false, class Emit,
          class Tail = NoTail>
__device__ __forceinline__ void leaf_tddp(const CS& cs, const KNode& nd, bool hoisted, const double (&x12)[E],
                                          const double (&x13)[E], const double (&xt)[E], const double (&xs)[E],
                                          T (&lv)[E], const Emit& emit, const Tail& tail = Tail{}) {
  const int c0 = nd.c0, R = nd.aux;
  constexpr bool hx = HX || FULL;  // trigonometric terms (x free: the plain node has 2R + 3 slots)
  static_assert(!FULL || E == 1, "the full model takes one event per step");
  static_assert(!NORM || FULL, "grid cells of the full model only");
  // the full model in double takes its amplitudes one at a time, twice
  // (sums, then derivatives), instead of holding them in arrays
  constexpr bool STREAM = FULL && std::is_same<T, double>::value;
  double s12[E], s13[E], s23[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    s12[e] = x12[e] + cs.d[c0 + kDzRef12];
    s13[e] = x13[e] + cs.d[c0 + kDzRef13];
    s23[e] = cs.d[c0 + kDzSsum] - s12[e] - s13[e];
  }
  static_assert(E == 1 || E == 2, "one or two events per step");
  AmpArr<T, NR> a0, a1, b0, b1;
  if constexpr (!STREAM) dalitz_amps<T, true, E, NR>(cs, nd, s12, s13, s23, a0, a1, b0, b1);
  const int cb = c0 + dz_coef_base(R, true);
  const int tb = c0 + dz_time_base(R, NR);
  const int fb = c0 + dz_full_base(R);
  // q/p multiplies the conjugate amplitudes (1 outside the full model)
  Cx<T> qp = {T(1), T(0)};
  if constexpr (FULL) {
    qp = {cs.get<T>(fb + kFqRe), cs.get<T>(fb + kFqIm)};
    if constexpr (!STREAM) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const Cx<T> w = cmul(qp, Cx<T>{b0[2 * k], b0[2 * k + 1]});
        b0[2 * k] = w.re;
        b0[2 * k + 1] = w.im;
      }
    }
  }
  Cx<T> S[E], Sb[E];
  T cc[E], cb_[E], St[E], Sz[E], iR[E], dtau[E], dy[E], dx[E], dqm[E], dqa[E], nBv[E], asv[E], bsv[E];
  static_for<E>([&](auto ei) {
    constexpr int e = decltype(ei)::value;
    const AmpArr<T, NR>& ae = pick<e>(a0, a1);
    const AmpArr<T, NR>& be = pick<e>(b0, b1);
    S[e] = {T(1), T(0)};
    Sb[e] = qp;
    if constexpr (STREAM) {
      dalitz_stream<T>(cs, nd, s12[e], s13[e], s23[e], [&](int k, Cx<T> A, Cx<T> Ab) {
        const Cx<T> c = {cs.get<T>(cb + 2 * k), cs.get<T>(cb + 2 * k + 1)};
        const Cx<T> t = cmul(c, A);
        const Cx<T> u = cmul(c, cmul(qp, Ab));
        S[e].re += t.re; S[e].im += t.im;
        Sb[e].re += u.re; Sb[e].im += u.im;
      });
    } else {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const Cx<T> c = {cs.get<T>(cb + 2 * k), cs.get<T>(cb + 2 * k + 1)};
        const Cx<T> t = cmul(c, Cx<T>{ae[2 * k], ae[2 * k + 1]});
        const Cx<T> u = cmul(c, Cx<T>{be[2 * k], be[2 * k + 1]});
        S[e].re += t.re; S[e].im += t.im;
        Sb[e].re += u.re; Sb[e].im += u.im;
      }
    }
    const T nA = S[e].re * S[e].re + S[e].im * S[e].im;
    const T nB = Sb[e].re * Sb[e].re + Sb[e].im * Sb[e].im;
    const T as = -(S[e].re * Sb[e].re + S[e].im * Sb[e].im);  // -Re(conj(A) Abar)
    const T bs = -(S[e].re * Sb[e].im - S[e].im * Sb[e].re);  // -Im(conj(A) Abar)
    if constexpr (NORM) {
      const double kc = cs.d[fb + kFkc], kz = cs.d[fb + kFkz];
      cc[e] = (T)(kc + kz);
      cb_[e] = (T)(kc - kz);
      St[e] = (T)cs.d[fb + kFks];
      Sz[e] = (T)cs.d[fb + kFkzs];
      iR[e] = T(1);
      lv[e] = nA;
      nBv[e] = nB;
      asv[e] = as;
      bsv[e] = bs;
      dqm[e] = (cb_[e] * nB + as * St[e] + bs * Sz[e]) * cs.get<T>(fb + kFiq);
      dqa[e] = as * Sz[e] - bs * St[e];
    } else {
    // Decay-time factors, formed in double: C - E(1/tau), S and the tau / y
    // derivative combinations are small differences of nearly equal terms
    // (|y| << 1), and rounding them in float would bias every event the
    // same way.
    const double t = xt[e], s = xs[e];
    const double g = ::exp(-0.5 * t * t / (s * s));
    double Em, dEm, Ep, dEp;
    econv<double>(t, s, cs.d[tb + kTdGm], g, Em, dEm);
    econv<double>(t, s, cs.d[tb + kTdGp], g, Ep, dEp);
    // trigonometric pair Cz, Sz and their tau and x derivatives
    double Cz, Szd = 0.0, Cz_tau, Sz_tau = 0.0, Cz_x = 0.0, Sz_x = 0.0;
    if (hx) {
      Cx<double> Ez, dEz;
      econv_c(t, s, cs.d[tb + kTdG], cs.d[tb + kTdW], g, Ez, dEz);
      Cz = Ez.re;
      Szd = Ez.im;
      // z = G - i W: dz/dtau = dG/dtau - i dW/dtau, dz/dx = -i dW/dx
      const double gt = cs.d[tb + kTdDGTau], wt = cs.d[tb + kTdDWTau], wx = cs.d[tb + kTdDWX];
      Cz_tau = dEz.re * gt + dEz.im * wt;
      Sz_tau = dEz.im * gt - dEz.re * wt;
      Cz_x = dEz.im * wx;
      Sz_x = -dEz.re * wx;
    } else {
      double dE0;
      econv<double>(t, s, cs.d[tb + kTdG], g, Cz, dE0);
      Cz_tau = dE0 * cs.d[tb + kTdDGTau];
    }
    const double Cd = 0.5 * (Em + Ep);
    const double Tm = dEm * cs.d[tb + kTdDGmTau], Tp = dEp * cs.d[tb + kTdDGpTau];
    const double T1 = 0.5 * (Tm + Tp);
    const double Ym = dEm * cs.d[tb + kTdDGmY], Yp = dEp * cs.d[tb + kTdDGpY];
    cc[e] = (T)(Cd + Cz);          // d R / d(|A|^2 / 2)
    cb_[e] = (T)(Cd - Cz);         // d R / d(|Abar|^2 / 2)
    St[e] = (T)(0.5 * (Em - Ep));  // S(t)
    Sz[e] = (T)Szd;
    const T tA = (T)(T1 + Cz_tau), tB = (T)(T1 - Cz_tau), tS = (T)(0.5 * (Tm - Tp)), tZ = (T)Sz_tau;
    const T yAB = (T)(0.5 * (Ym + Yp)), yS = (T)(0.5 * (Ym - Yp));
    // rate = a_c C + a_0 Cz + a_s S + b_s Sz
    //      = |A|^2 (C + Cz)/2 + |Abar|^2 (C - Cz)/2 + a_s S + b_s Sz
    T Rv = T(0.5) * nA * cc[e] + T(0.5) * nB * cb_[e] + as * St[e];
    T rt = T(0.5) * nA * tA + T(0.5) * nB * tB + as * tS;
    if (hx) {
      Rv += bs * Sz[e];
      rt += bs * tZ;
    }
    iR[e] = Mth<T>::rcp(Rv);
    lv[e] = Rv > T(0) ? Mth<T>::ln(Rv) : T(-INFINITY);
    dtau[e] = rt * iR[e];
    dy[e] = (T(0.5) * (nA + nB) * yAB + as * yS) * iR[e];
    dx[e] = hx ? (T(0.5) * (nA - nB) * (T)Cz_x + bs * (T)Sz_x) * iR[e] : T(0);
    if constexpr (FULL) {
      // q/p = |q/p| e^{i phi} scales Abar: |Abar|^2 goes as |q/p|^2, a_s and
      // b_s as |q/p|; the phase turns (a_s, b_s)
      dqm[e] = (cb_[e] * nB + as * St[e] + bs * Sz[e]) * cs.get<T>(fb + kFiq) * iR[e];
      dqa[e] = (as * Sz[e] - bs * St[e]) * iR[e];
    }
    if (!hoisted) {
      dtau[e] -= cs.get<T>(c0 + kDzDln + 2 * R);
      dy[e] -= cs.get<T>(c0 + kDzDln + 2 * R + 1);
      dx[e] -= cs.get<T>(c0 + kDzDln + 2 * R + 2);
      lv[e] = (lv[e] - cs.get<T>(c0 + kDzLnHi)) - cs.get<T>(c0 + kDzLnLo);
    }
    }
  });
  // coefficient k's two slot derivatives at event e from A_k = (ar, ai) and
  // the conjugate-side amplitude (br, bi) (with q/p): re part dA = A_k,
  // dAb = Ab_k; im part dA = i A_k, dAb = i Ab_k
  const auto coef_d = [&](int e, int k, T ar, T ai, T br, T bi, T& dre, T& dim) {
    const T pA_re = S[e].re * ar + S[e].im * ai;    // Re(conj(S) A_k)
    const T pA_im = S[e].re * ai - S[e].im * ar;    // Im(conj(S) A_k)
    const T pB_re = Sb[e].re * br + Sb[e].im * bi;
    const T pB_im = Sb[e].re * bi - Sb[e].im * br;
    const T x1_re = ar * Sb[e].re + ai * Sb[e].im;  // Re(conj(A_k) Sb)
    const T x1_im = ar * Sb[e].im - ai * Sb[e].re;  // Im(conj(A_k) Sb)
    const T x2_re = S[e].re * br + S[e].im * bi;    // Re(conj(S) Ab_k)
    const T x2_im = S[e].re * bi - S[e].im * br;    // Im(conj(S) Ab_k)
    T dR_re = cc[e] * pA_re + cb_[e] * pB_re - (x1_re + x2_re) * St[e];
    T dR_im = -cc[e] * pA_im - cb_[e] * pB_im - (x1_im - x2_im) * St[e];
    if (hx) {
      dR_re -= (x1_im + x2_im) * Sz[e];
      dR_im += (x1_re - x2_re) * Sz[e];
    }
    dre = dR_re * iR[e];
    dim = dR_im * iR[e];
    if (!hoisted && k < R) {
      dre -= cs.get<T>(c0 + kDzDln + 2 * k);
      dim -= cs.get<T>(c0 + kDzDln + 2 * k + 1);
    }
  };
  if constexpr (STREAM) {
    dalitz_stream<T>(cs, nd, s12[0], s13[0], s23[0], [&](int k, Cx<T> A, Cx<T> Ab) {
      const Cx<T> B = cmul(qp, Ab);
      T d_re[E], d_im[E];
      coef_d(0, k, A.re, A.im, B.re, B.im, d_re[0], d_im[0]);
      emit(2 * k, d_re);
      emit(2 * k + 1, d_im);
    });
  } else {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      T d_re[E], d_im[E];
      static_for<E>([&](auto ei) {
        constexpr int e = decltype(ei)::value;
        const AmpArr<T, NR>& ae = pick<e>(a0, a1);
        const AmpArr<T, NR>& be = pick<e>(b0, b1);
        coef_d(e, k, ae[2 * k], ae[2 * k + 1], be[2 * k], be[2 * k + 1], d_re[e], d_im[e]);
      });
      emit(2 * k, d_re);
      emit(2 * k + 1, d_im);
    }
  }
  if constexpr (!FULL) {
    emit(2 * R, dtau);
    emit(2 * R + 1, dy);
    if (hx) emit(2 * R + 2, dx);
  } else if constexpr (NORM) {
    tail(std::integral_constant<int, 0>{}, nBv);
    tail(std::integral_constant<int, 1>{}, asv);
    tail(std::integral_constant<int, 2>{}, bsv);
  } else {
    tail(std::integral_constant<int, 0>{}, dtau);
    tail(std::integral_constant<int, 1>{}, dy);
    if (cs.d[fb + kFhx] != 0.0) tail(std::integral_constant<int, 2>{}, dx);
  }
  if constexpr (FULL) {
    if (cs.d[fb + kFhq] != 0.0) {
      tail(std::integral_constant<int, 3>{}, dqm);
      tail(std::integral_constant<int, 4>{}, dqa);
    }
    // floating masses and widths: the rate moves along dA = c_k A_k F and
    // dAbar' = (q/p) c_k Abar_k Fbar (F, Fbar the amplitudes' relative
    // derivatives at the point and at the swapped point), so
    // dR = Re(alpha c_k A_k F) + Re(beta (q/p) c_k Abar_k Fbar) with the
    // adjoints alpha = d R / dA, beta = d R / dAbar' (as complex
    // derivatives of a real function: dR = Re(alpha dA + beta dAbar'))
    const int nf = (int)cs.d[fb + kFnf];
    const Cx<T> cS = {S[0].re, -S[0].im}, cSb = {Sb[0].re, -Sb[0].im};
    const Cx<T> al = {cc[0] * cS.re - St[0] * cSb.re + Sz[0] * cSb.im,
                      cc[0] * cS.im - St[0] * cSb.im - Sz[0] * cSb.re};
    const Cx<T> be = {cb_[0] * cSb.re - St[0] * cS.re - Sz[0] * cS.im,
                      cb_[0] * cSb.im - St[0] * cS.im + Sz[0] * cS.re};
    static_for<kMaxFloat>([&](auto fi) {
      constexpr int f = decltype(fi)::value;
      if (f < nf) {
        const int lb = fb + kFlBase + f * kFlStride;
        const int k = (int)cs.d[lb + kFlRes], pair = (int)cs.d[lb + kFlPair], J = (int)cs.d[lb + kFlJ];
        Cx<T> A, D, Ab, Db;
        T g, gb;
        res_amp_rt<T>(cs, nd, k, pair, J, s12[0], s13[0], s23[0], A, D, g);
        res_amp_rt<T>(cs, nd, k, pair, J, s13[0], s12[0], s23[0], Ab, Db, gb);
        const Cx<T> ck = {cs.get<T>(cb + 2 * k), cs.get<T>(cb + 2 * k + 1)};
        const Cx<T> w = cmul(al, cmul(ck, A));
        const Cx<T> wb = cmul(be, cmul(qp, cmul(ck, Ab)));
        const T dm2 = cs.get<T>(lb + kFlDm2), dkm = cs.get<T>(lb + kFlDkwM), dlb = cs.get<T>(lb + kFlDlbM),
                dkg = cs.get<T>(lb + kFlDkwG);
        // F_m = D (-dm2 + i g dkm) + dlb, F_g = D (i g dkg)
        const Cx<T> Fm = {-D.re * dm2 - D.im * g * dkm + dlb, -D.im * dm2 + D.re * g * dkm};
        const Cx<T> Fbm = {-Db.re * dm2 - Db.im * gb * dkm + dlb, -Db.im * dm2 + Db.re * gb * dkm};
        const Cx<T> Fg = {-D.im * g * dkg, D.re * g * dkg};
        const Cx<T> Fbg = {-Db.im * gb * dkg, Db.re * gb * dkg};
        const T dm[1] = {(cmul(w, Fm).re + cmul(wb, Fbm).re) * iR[0]};
        const T dg[1] = {(cmul(w, Fg).re + cmul(wb, Fbg).re) * iR[0]};
        tail(std::integral_constant<int, 5 + 2 * f>{}, dm);
        tail(std::integral_constant<int, 6 + 2 * f>{}, dg);
      }
    });
  }
}

// ------------------------------------------------------------------ cross-lane sums
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave (all lanes active): pair and quad
// exchanges, then rotations by 4 and 8 inside each 16-lane row, so lanes 0,
// 16, 32 and 48 hold their row sums; those four are added in a fixed order.
// The result is wave-uniform.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x124>(v);  // row_ror:4
  v += dpp_d<0x128>(v);  // row_ror:8
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Row store for few columns: the threads' accumulators go through LDS; wave
// w sums columns w, w + 4, ... over the four waves (fixed order) and its 64
// lanes.  `out` points at this row of column 0; columns are `stride` apart.
template <int NC>
__device__ __forceinline__ void row_store_lds(const double* acc, double* __restrict__ out, int stride) {
  __shared__ double sh[NC][kBlock];
#pragma unroll
  for (int j = 0; j < NC; ++j) sh[j][threadIdx.x] = acc[j];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = wave; j < NC; j += kBlock / 64) {
    const double v = ((sh[j][lane] + sh[j][lane + 64]) + sh[j][lane + 128]) + sh[j][lane + 192];
    const double s = wave_sum(v);
    if (lane == 0) out[(int64_t)j * stride] = s;
  }
  __syncthreads();  // sh is reused by the next row of a grid-stride block
}

// Row store for many columns (amplitude and tree kernels): a lane sum per
// wave and column, then the four waves in a fixed order.
template <int NC>
__device__ __forceinline__ void row_store_waves(const double* acc, int nc, double* __restrict__ out, int stride) {
  __shared__ double red[kBlock / 64][NC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if (j < nc) {
      const double s = wave_sum(acc[j]);
      if (lane == 0) red[wave][j] = s;
    }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < nc) out[(int64_t)t * stride] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
  __syncthreads();
}

// Per-thread double accumulators kept in LDS ([column][thread]) for the
// amplitude and tree kernels, whose per-event state already fills the VGPRs:
// each thread adds only to its own slots (ds_add_f64, program order, so the
// sums are deterministic), and the block reduction reads them in place.
template <int NC> struct LdsAcc {
  double (*a)[kBlock];
  __device__ __forceinline__ void zero(int nc) const {
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (j < nc) a[j][threadIdx.x] = 0.0;
  }
  __device__ __forceinline__ void add(int j, double v) const {
    __hip_atomic_fetch_add(&a[j][threadIdx.x], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// Row store of LDS accumulators: wave w sums columns w, w + 4, ... over the
// four waves (fixed order) and its 64 lanes.
template <int NC>
__device__ __forceinline__ void row_store_acc(const LdsAcc<NC>& acc, int nc, double* __restrict__ out, int stride) {
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = wave; j < nc; j += kBlock / 64) {
    const double v = ((acc.a[j][lane] + acc.a[j][lane + 64]) + acc.a[j][lane + 128]) + acc.a[j][lane + 192];
    const double s = wave_sum(v);
    if (lane == 0) out[(int64_t)j * stride] = s;
  }
  __syncthreads();  // the accumulators are reused by the next row of a grid-stride block
}

// Per-event output (the terms launches of nll_terms): every row holds one
// chunk, so after the row loop a thread's accumulators are the terms of its
// one event (zeros past the end of the dataset).  Thread t of the row
// starting at `out` writes column j to out[j * stride + t]; nothing is summed.
template <int NC>
__device__ __forceinline__ void thread_store(const double* acc, int nc, double* __restrict__ out, int64_t stride) {
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if (j < nc) out[(int64_t)j * stride + threadIdx.x] = acc[j];
}

template <int NC>
__device__ __forceinline__ void thread_store_acc(const LdsAcc<NC>& acc, int nc, double* __restrict__ out,
                                                 int64_t stride) {
#pragma unroll
  for (int j = 0; j < NC; ++j)
    if (j < nc) out[(int64_t)j * stride + threadIdx.x] = acc.a[j][threadIdx.x];
}

// Where a row's results go: the block sums into the row's place of the
// [column][row] partials (stride = rows), or, in a terms launch (TM), each
// thread's own terms into [column][event] (stride = rows x 256).
template <bool TM>
__device__ __forceinline__ int64_t out_stride(int n_rows) {
  return TM ? (int64_t)n_rows * kBlock : (int64_t)n_rows;
}

// Chunk range [c0, c1) of row r when the dataset's chunks are split into
// n_rows equal parts.
__device__ __forceinline__ void row_chunks(int64_t n_events, int n_rows, int r, int64_t& c0, int64_t& c1) {
  const int64_t nch = (n_events + kBlock - 1) / kBlock;
  c0 = (int64_t)r * nch / n_rows;
  c1 = (int64_t)(r + 1) * nch / n_rows;
}

// ------------------------------------------------------------------ row loops
// Single-column evaluators (mixtures, single EXP / GAUSS leaves): groups of
// U chunks, the loads of the next group in flight while the current one is
// evaluated.  An evaluator adds its NLL term to `nl` and its NA gradient
// accumulators to `ga` (type T over one group); the group sums go into the
// per-thread double accumulators: acc[0] += kNllScale * (group sum of nl),
// acc[1 + j] += group sum of ga[j].  Only the last
// chunk of a dataset can be partial, so all groups but the last are
// unchecked.
template <typename T, int U, class Ev>
__device__ __forceinline__ void light_row(const Ev& ev, const typename Col<T>::S* __restrict__ xp, int64_t n,
                                          int64_t c0, int64_t c1, double* acc) {
  typedef typename Col<T>::S Sx;
  constexpr int NA = Ev::NA;
  const int64_t t = threadIdx.x;
  const int64_t full = n / kBlock;                 // chunks with 256 events
  const int64_t cfe = c1 < full ? c1 : full;
  const int64_t ng = cfe > c0 ? (cfe - c0) / U : 0;
  int64_t c = c0;
  Sx nx[U];
  if (ng > 0) {
#pragma unroll
    for (int k = 0; k < U; ++k) nx[k] = xp[(c + k) * kBlock + t];
  }
  for (int64_t gi = 0; gi < ng; ++gi) {
    Sx cur[U];
#pragma unroll
    for (int k = 0; k < U; ++k) cur[k] = nx[k];
    if (gi + 1 < ng) {
#pragma unroll
      for (int k = 0; k < U; ++k) nx[k] = xp[(c + U + k) * kBlock + t];
    }
    T nl = T(0), ga[NA + 1];
#pragma unroll
    for (int j = 0; j < NA; ++j) ga[j] = T(0);
#pragma unroll
    for (int k = 0; k < U; ++k) ev((T)cur[k], nl, ga);
    acc[0] = __builtin_fma((double)nl, Ev::kNllScale, acc[0]);
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[1 + j] += (double)ga[j];
    c += U;
  }
  if (c < c1) {  // at most U chunks left, the last one possibly partial
    Sx cur[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t i = (c + k) * kBlock + t;
      cur[k] = (c + k < c1 && i < n) ? xp[i] : Sx(0);
    }
    T nl = T(0), ga[NA + 1];
#pragma unroll
    for (int j = 0; j < NA; ++j) ga[j] = T(0);
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t i = (c + k) * kBlock + t;
      if (c + k < c1 && i < n) ev((T)cur[k], nl, ga);
    }
    acc[0] = __builtin_fma((double)nl, Ev::kNllScale, acc[0]);
#pragma unroll
    for (int j = 0; j < NA; ++j) acc[1 + j] += (double)ga[j];
  }
}

// Multi-column evaluators (amplitude leaves, trees): one event per chunk and
// thread, the next event's columns in flight; the evaluator adds straight
// into the (LDS) double accumulators.
template <typename T, int NCOL, class Ev, class Acc>
__device__ __forceinline__ void heavy_row(const Ev& ev, const KProgram& P, const typename Col<T>::S* const* cp,
                                          int ncols, int64_t n, int64_t c0, int64_t c1, const Acc& acc) {
  typedef typename Col<T>::S Sx;
  const int64_t t = threadIdx.x;
  Sx cur[NCOL];
  {
    const int64_t i = c0 * kBlock + t;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) cur[c] = (c < ncols && c0 < c1 && i < n) ? cp[c][i] : Sx(0);
  }
#pragma unroll 1
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int64_t i = ch * kBlock + t;
    double xe[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) xe[c] = (double)cur[c];
    if (ch + 1 < c1) {
      const int64_t i1 = i + kBlock;
#pragma unroll
      for (int c = 0; c < NCOL; ++c)
        if (c < ncols) cur[c] = i1 < n ? cp[c][i1] : Sx(0);
    }
    if (i < n) ev(P, xe, i, acc);
  }
}

// ------------------------------------------------------------------ mixtures
// Root ADD of K single-column EXP / GAUSS leaves (the signal-plus-background
// shape), fully static: MASK bit j set means child j is a GAUSS.  With e_j =
// exp(lv_j - m) (m the largest child log-density), s = sum f_j e_j and q_j =
// e_j / s, the per-event terms are ln P = m + ln s and
//   d ln P / d f_j      = q_j - q_{K-1}                 (j < K-1)
//   d ln P / d(GAUSS j) = f_j q_j (z / sigma - dlnN), f_j q_j (z^2 / sigma - dlnN')
//   d ln P / d(EXP j)   = f_j q_j (x - a - dlnN).
// The kernel accumulates per child sum q_j, sum q_j z (EXP: sum q_j x) and
// sum q_j z^2; the host combines them with the constants.
template <typename T> struct Split;
template <> struct Split<double> {
  double v;
  __device__ __forceinline__ void set(double x) { v = x; }
  __device__ __forceinline__ double add_to(double a) const { return a + v; }
  // a * b + v and a * b - v
  __device__ __forceinline__ double fma_add(double a, double b) const { return __builtin_fma(a, b, v); }
  __device__ __forceinline__ double fma_sub(double a, double b) const { return __builtin_fma(a, b, -v); }
};
template <> struct Split<float> {
  // a double constant as a float pair hi + lo: (a + hi) + lo rounds like one
  // addition of the double value, so its rounding error varies from event to
  // event instead of biasing all of them the same way
  float hi, lo;
  __device__ __forceinline__ void set(double x) {
    hi = (float)x;
    lo = (float)(x - (double)hi);
  }
  __device__ __forceinline__ float add_to(float a) const { return (a + hi) + lo; }
  // a * b + (hi + lo) and a * b - (hi + lo)
  __device__ __forceinline__ float fma_add(float a, float b) const { return __builtin_fmaf(a, b, hi) + lo; }
  __device__ __forceinline__ float fma_sub(float a, float b) const { return __builtin_fmaf(a, b, -hi) - lo; }
};

__device__ __forceinline__ float neg_abs(float x) { return -__builtin_fabsf(x); }
__device__ __forceinline__ double neg_abs(double x) { return -__builtin_fabs(x); }

template <typename T, int K, int MASK, bool GRAD>
struct MixEv {
  static constexpr int NA = GRAD ? 3 * K : 0;
  static constexpr double kNllScale = -0.69314718055994530942;  // -ln 2: nl holds sum log2 P
  // the log-densities are carried in base 2: lv2 = log2 e * ln(f_j / N_j)
  Split<T> loc[K];  // GAUSS: column reference - mu
  Split<T> cst[K];  // GAUSS: log2 e ln N ; EXP: log2 e (alpha (column reference - a) - ln N)
  T k1[K];          // GAUSS: 1 / sigma ; EXP: log2 e alpha
  T f[K];           // fractions, the last one 1 - sum of the others

  // adds log2 P to nl (the caller scales by -ln 2)
  __device__ __forceinline__ void operator()(T x, T& nl, T* ga) const {
    constexpr T kHalfLog2e = T(-0.5 * 1.44269504088896340736);
    T lv[K], za[K], zb[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if ((MASK >> j) & 1) {
        const T z = loc[j].add_to(x) * k1[j], zz = z * z;
        lv[j] = cst[j].fma_sub(kHalfLog2e, zz);
        za[j] = z;
        zb[j] = zz;
      } else {
        lv[j] = cst[j].fma_add(k1[j], x);
        za[j] = x;
        zb[j] = T(0);
      }
    }
    T q[K];
    if (K == 2) {
      // the larger term has e = 1: one exponential per event
      const T dd = lv[1] - lv[0];
      const bool up = dd > T(0);
      const T eo = Mth<T>::ex2(neg_abs(dd));
      const T m = up ? lv[1] : lv[0];
      const T fa = up ? f[1] : f[0], fb = up ? f[0] : f[1];
      const T s = Mth<T>::fma(fb, eo, fa);
      nl += m + Mth<T>::lg2(s);
      if (GRAD) {
        const T is = Mth<T>::rcp(s), qo = eo * is;
        q[0] = up ? qo : is;
        q[1] = up ? is : qo;
      }
    } else {
      T m = lv[0];
#pragma unroll
      for (int j = 1; j < K; ++j) m = lv[j] > m ? lv[j] : m;
      T e[K], s = T(0);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        e[j] = Mth<T>::ex2(lv[j] - m);
        s = Mth<T>::fma(f[j], e[j], s);
      }
      nl += m + Mth<T>::lg2(s);
      if (GRAD) {
        const T is = Mth<T>::rcp(s);
#pragma unroll
        for (int j = 0; j < K; ++j) q[j] = e[j] * is;
      }
    }
    if (GRAD) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        ga[3 * j] += q[j];
        ga[3 * j + 1] = Mth<T>::fma(q[j], za[j], ga[3 * j + 1]);
        if ((MASK >> j) & 1) ga[3 * j + 2] = Mth<T>::fma(q[j], zb[j], ga[3 * j + 2]);
      }
    }
  }
};

// Constants of a mixture from the staged table (EXP / GAUSS / ADD layouts).
template <typename T, int K, int MASK, bool GRAD>
__device__ __forceinline__ MixEv<T, K, MASK, GRAD> make_mix(const KProgram& P, const CS& cs) {
  constexpr double kLog2e = 1.44269504088896340736;
  MixEv<T, K, MASK, GRAD> ev;
  const KNode& rn = P.node[P.n_nodes - 1];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int c0 = P.node[P.child[rn.child0 + j]].c0;
    if ((MASK >> j) & 1) {
      ev.k1[j] = cs.get<T>(c0 + 1);
      ev.loc[j].set(cs.d[c0]);
      ev.cst[j].set(kLog2e * cs.d[c0 + 2]);
    } else {
      ev.k1[j] = (T)(kLog2e * cs.d[c0 + 1]);
      ev.loc[j].set(0.0);
      ev.cst[j].set(kLog2e * (cs.d[c0 + 1] * cs.d[c0] - cs.d[c0 + 2]));
    }
    ev.f[j] = cs.get<T>(rn.c0 + j);
  }
  return ev;
}

// ------------------------------------------------------------------ leaf evaluators
template <typename T, int OP, bool GRAD>
struct LightLeafEv {  // single EXP / GAUSS leaf
  static constexpr int NA = GRAD ? (OP == OP_EXP ? 1 : 2) : 0;
  static constexpr double kNllScale = 1.0;  // nl holds sum -ln P
  CS cs;
  int c0;
  bool hoisted;
  __device__ __forceinline__ void operator()(T x, T& nl, T* ga) const {
    T dl[2];
    const T lv = OP == OP_EXP ? leaf_exp<T>(cs, c0, hoisted, (double)x, dl)
                              : leaf_gauss<T>(cs, c0, hoisted, (double)x, dl);
    nl -= lv;
#pragma unroll
    for (int j = 0; j < NA; ++j) ga[j] += dl[j];
  }
};

// Kernel variant of OP_TDDP with the trigonometric terms (x free): a
// compile-time choice, so that the x = 0 kernel carries none of their
// registers.
constexpr int OP_TDDP_X = 16;

// Events per thread and step of the single-leaf amplitude kernels: the E
// events share every read of a resonance's constants and every loop step,
// and give the wave E independent instruction chains.
template <typename T, int OP> struct AmpEvents { static constexpr int value = OP == OP_DALITZ ? 2 : 1; };

// A CONV child at x (offset frame) as an unnormalised shape: ln f and
// d ln f / d(slot) in d[0 .. n_slot).
template <typename T>
__device__ __forceinline__ T conv_leaf(const CS& cs, const KNode& cn, double x, T (&d)[8]) {
  if (cn.op == OP_EXP) return leaf_exp<T>(cs, cn.c0, true, x, d);
  if (cn.op == OP_GAUSS) return leaf_gauss<T>(cs, cn.c0, true, x, d);
  return leaf_poly<T>(cs, cn.c0, cn.aux, true, x, d);
}

// Unnormalised shape of an EXP / GAUSS / POLY leaf (a CONV child) with its
// constants read once into registers: ln f and d ln f / d(slot) at v (the
// column's offset frame), the same arithmetic as leaf_exp / leaf_gauss /
// leaf_poly with hoisted = true.
template <typename T, int OP> struct Shape;
template <typename T> struct Shape<T, OP_EXP> {
  double loc;
  T a;
  __device__ __forceinline__ void load(const CS& cs, const KNode& n) {
    loc = cs.d[n.c0];
    a = cs.get<T>(n.c0 + 1);
  }
  __device__ __forceinline__ T eval(double v, T (&d)[4]) const {
    const T u = (T)(v + loc);
    d[0] = u;
    return a * u;
  }
};
template <typename T> struct Shape<T, OP_GAUSS> {
  double loc;
  T isg;
  __device__ __forceinline__ void load(const CS& cs, const KNode& n) {
    loc = cs.d[n.c0];
    isg = cs.get<T>(n.c0 + 1);
  }
  __device__ __forceinline__ T eval(double v, T (&d)[4]) const {
    const T z = (T)(v + loc) * isg;
    d[0] = z * isg;
    d[1] = z * z * isg;
    return T(-0.5) * z * z;
  }
};
template <typename T> struct Shape<T, OP_POLY> {  // degree <= 4
  double loc;
  T a[4];
  int deg;
  __device__ __forceinline__ void load(const CS& cs, const KNode& n) {
    loc = cs.d[n.c0];
    deg = n.aux;
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = k < deg ? cs.get<T>(n.c0 + 1 + k) : T(0);
  }
  __device__ __forceinline__ T eval(double v, T (&d)[4]) const {
    const T u = (T)(v + loc);
    T p = T(0);
#pragma unroll
    for (int k = 3; k >= 0; --k)
      if (k < deg) p = (p + a[k]) * u;
    p += T(1);
    const T ip = Mth<T>::rcp(p);
    T uk = u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < deg) d[k] = uk * ip;
      uk *= u;
    }
    return p > T(0) ? Mth<T>::ln(p) : T(-INFINITY);
  }
};

// Any of the three shapes, the kind chosen at run time (a wave-uniform
// branch per evaluation).
template <typename T> struct ShapeAny {
  double loc;
  T a[4];
  int op, deg;
  __device__ __forceinline__ void load(const CS& cs, const KNode& n) {
    op = n.op;
    loc = cs.d[n.c0];
    deg = op == OP_POLY ? n.aux : (op == OP_GAUSS ? 1 : 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = k < deg ? cs.get<T>(n.c0 + 1 + k) : T(0);
  }
  __device__ __forceinline__ T eval(double v, T (&d)[4]) const {
    if (op == OP_EXP) {
      const T u = (T)(v + loc);
      d[0] = u;
      return a[0] * u;
    }
    if (op == OP_GAUSS) {
      const T isg = a[0];
      const T z = (T)(v + loc) * isg;
      d[0] = z * isg;
      d[1] = z * z * isg;
      return T(-0.5) * z * z;
    }
    const T u = (T)(v + loc);
    T p = T(0);
#pragma unroll
    for (int k = 3; k >= 0; --k)
      if (k < deg) p = (p + a[k]) * u;
    p += T(1);
    const T ip = Mth<T>::rcp(p);
    T uk = u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < deg) d[k] = uk * ip;
      uk *= u;
    }
    return p > T(0) ? Mth<T>::ln(p) : T(-INFINITY);
  }
};

// Visits the grid points k0..k1 of an event's residual window: the first and
// last two take the definition's range test (t_k = lo + (k + 1/2) h and
// x - t_k in double, as written), those between lie inside by the window's
// construction (it is widened by a whole grid step on each side beyond
// rounding) and go untested, their model and resolution arguments
// t_k - ref and x - t_k - ref formed with one fused multiply-add each.
// body(k, t_k - ref, x - t_k - ref) adds a term.
// PAIRS: the untested points are visited two per loop step (then the odd
// one), so that two independent terms are in flight.
template <bool PAIRS = false, class Body>
__device__ __forceinline__ void conv_window(double x, double lo, double hh, double dlo, double dhi, double ref,
                                            int k0, int k1, const Body& body) {
  const auto tested = [&](int k) {
    const double t = conv_grid_point(lo, hh, k), d = x - t;
    if (d >= dlo && d <= dhi) body(k, t - ref, d - ref);
  };
  const int ka = k0 + 2 < k1 + 1 ? k0 + 2 : k1 + 1;  // first untested point
  const int kb = k1 - 2 >= ka ? k1 - 2 : ka - 1;     // last untested point
  for (int k = k0; k < ka; ++k) tested(k);
  const double cM = (lo - ref) + 0.5 * hh, cR = ((x - ref) - lo) - 0.5 * hh;
  const auto untested = [&](int k) {
    const double dk = (double)k;
    body(k, __builtin_fma(dk, hh, cM), __builtin_fma(-dk, hh, cR));
  };
  int k = ka;
  if constexpr (PAIRS)
    for (; k < kb; k += 2) {
      untested(k);
      untested(k + 1);
    }
  for (; k <= kb; ++k) untested(k);
  for (int k = kb + 1; k <= k1; ++k) tested(k);
}

// The model child of one CONV node at every grid point, staged in LDS once
// per row: ln f_M(t_k) - c (c the node's exponent shift) and
// d ln f_M / d(slot j) (zero beyond the model's slots), t_k = lo + (k + 1/2) h
// in the offset frame.  The model does not
// depend on the event, so the term loop then reads it instead of evaluating
// it per term.  Grids of at most kConvTab points qualify (the table fits
// beside the row's LDS accumulators without costing a resident block).
constexpr int kHeavyConvTab = 3;  // the tree interpreter's staged-CONV instantiation
// Array sizes of the staged-CONV interpreter for small trees: 8 slots and 2
// columns (float: 157 instead of 245 registers, three waves per SIMD;
// double: held to 256 registers, two waves per SIMD instead of one)
template <typename T> struct ConvSmall {
  static constexpr int NS = 8;
  static constexpr int NCOL = 2;
};
template <typename T> struct ConvTab {
  T v[5][kConvTab];
};

template <typename T>
__device__ __forceinline__ ConvTab<T>& conv_tab_lds() {
  __shared__ ConvTab<T> t;
  return t;
}

// Stages the first CONV node with at most kConvTab grid points; returns its
// index, or -1 when there is none (every lane of the block takes part).
template <typename T>
__device__ __forceinline__ int conv_stage(const KProgram& P, const CS& cs, ConvTab<T>& tab) {
  int node = -1;
  for (int k = 0; k < P.n_nodes; ++k)
    if (node < 0 && P.node[k].op == OP_CONV && P.node[k].aux <= kConvTab) node = k;
  if (node < 0) return -1;
  const KNode& nd = P.node[node];
  ShapeAny<T> M;
  M.load(cs, P.node[P.child[nd.child0]]);
  const double lo = cs.d[nd.c0], hh = cs.d[nd.c0 + 1], ref = cs.d[nd.c0 + 4];
  const T shift = cs.get<T>(nd.c0 + 5);
  __syncthreads();  // a previous row of this block may still read the table
  for (int k = threadIdx.x; k < nd.aux; k += kBlock) {
    T d[4] = {T(0), T(0), T(0), T(0)};
    const T l = M.eval(conv_grid_point(lo, hh, k) - ref, d);
    tab.v[0][k] = l - shift;
#pragma unroll
    for (int j = 0; j < 4; ++j) tab.v[1 + j][k] = d[j];
  }
  __syncthreads();
  return node;
}

// The grid sum of a CONV node at x (the stored event's value): over
// k in [k0, k1], the terms with the residual x - t_k in [d_lo, d_hi] add
// w = exp(ln f_M(t_k) + ln f_R(x - t_k) - shift) to S and w d ln f / d(slot)
// to the children's slot sums gm (model) and gr (resolution); undef is set
// when the resolution's shape is not positive at a residual in use.
// With TAB the model's values come from the staged table.
template <typename T, int ROP, bool TAB>
__device__ __forceinline__ void conv_terms(const CS& cs, const KNode& cm, const KNode& cr, double x, double lo,
                                           double hh, double dlo, double dhi, double ref, T shift, int k0, int k1,
                                           T& S, T (&gm)[8], T (&gr)[8], bool& undef, const ConvTab<T>* tab) {
  ShapeAny<T> M;
  Shape<T, ROP> R;
  if (!TAB) M.load(cs, cm);
  R.load(cs, cr);
  constexpr int NM = 4;
  constexpr int NR = ROP == OP_EXP ? 1 : (ROP == OP_GAUSS ? 2 : 4);
  if constexpr (TAB && ROP == OP_GAUSS) {
    // Gaussian resolution, u = x - t_k - mu (the residual less the mean, from
    // the offset-frame residual and the staged ref - mu): ln f_R = c u^2 with
    // c = -1/(2 sigma^2), d/dmu = u / sigma^2, d/dsigma = u^2 / sigma^3, so
    // the term adds w, w u and w u^2 and the sums are scaled once per event;
    // the loop is specialised on the model's slot count
    const T isg = R.isg, c = T(-0.5) * isg * isg;
    T su = T(0), su2 = T(0);
    const auto run = [&](auto nms) __attribute__((always_inline)) {
      constexpr int NMS = decltype(nms)::value;
      conv_window<true>(x, lo, hh, dlo, dhi, ref, k0, k1, [&](int k, double, double vr) {
        const T u = (T)(vr + R.loc);
        const T u2 = u * u;
        const T w = Mth<T>::ex(Mth<T>::fma(c, u2, tab->v[0][k]));
        S += w;
        su = Mth<T>::fma(w, u, su);
        su2 = Mth<T>::fma(w, u2, su2);
#pragma unroll
        for (int j = 0; j < NMS; ++j) gm[j] = Mth<T>::fma(w, tab->v[1 + j][k], gm[j]);
      });
    };
    if (cm.n_slot == 1) run(std::integral_constant<int, 1>{});
    else if (cm.n_slot == 2) run(std::integral_constant<int, 2>{});
    else run(std::integral_constant<int, 4>{});
    gr[0] = su * (isg * isg);
    gr[1] = su2 * (isg * isg * isg);
    return;
  }
  if constexpr (TAB && ROP == OP_EXP) {
    // one-sided exponential resolution: ln f_R = a u and d/da = u, the loop
    // specialised on the model's slot count, two points per step
    const auto run = [&](auto nms) __attribute__((always_inline)) {
      constexpr int NMS = decltype(nms)::value;
      conv_window<true>(x, lo, hh, dlo, dhi, ref, k0, k1, [&](int k, double, double vr) {
        T dr[4];
        const T lr = R.eval(vr, dr);
        const T w = Mth<T>::ex(tab->v[0][k] + lr);
        S += w;
        gr[0] = Mth<T>::fma(w, dr[0], gr[0]);
#pragma unroll
        for (int j = 0; j < NMS; ++j) gm[j] = Mth<T>::fma(w, tab->v[1 + j][k], gm[j]);
      });
    };
    if (cm.n_slot == 1) run(std::integral_constant<int, 1>{});
    else if (cm.n_slot == 2) run(std::integral_constant<int, 2>{});
    else run(std::integral_constant<int, 4>{});
    return;
  }
  conv_window(x, lo, hh, dlo, dhi, ref, k0, k1, [&](int k, double vm, double vr) {
    T dm[4], dr[4], lm;
    if constexpr (TAB) {
      lm = tab->v[0][k];  // shift already subtracted
#pragma unroll
      for (int j = 0; j < NM; ++j) dm[j] = tab->v[1 + j][k];
    } else {
      lm = M.eval(vm, dm);
    }
    const T lr = R.eval(vr, dr);
    undef = undef || !(lr > T(-INFINITY));
    const T w = Mth<T>::ex(TAB ? lm + lr : (lm + lr) - shift);
    S += w;
#pragma unroll
    for (int j = 0; j < NM; ++j)
      if (TAB || j < cm.n_slot) gm[j] = Mth<T>::fma(w, dm[j], gm[j]);
#pragma unroll
    for (int j = 0; j < NR; ++j) gr[j] = Mth<T>::fma(w, dr[j], gr[j]);
  });
}

// The same grid sum with a resolution that is a mixture (ADD node cr) of
// K <= 3 Gaussians, each normalised over the residual range (their staged
// ln N and its derivatives): per term and component w_j = exp(ln f_M(t_k)
// + ln g_j(x - t_k) - ln N_j - shift), S += sum f_j w_j; the resolution's
// slot sums gr are ordered as its slots: each Gaussian's (mu, sigma), then
// the K - 1 fractions (d/df_j: w_j - w_K).
template <typename T, bool TAB>
__device__ __forceinline__ void conv_terms_gmix(const CS& cs, const KProgram& P, const KNode& cm, const KNode& cr,
                                                double x, double lo, double hh, double dlo, double dhi, double ref,
                                                T shift, int k0, int k1, T& S, T (&gm)[8], T (&gr)[8],
                                                const ConvTab<T>* tab) {
  ShapeAny<T> M;
  if (!TAB) M.load(cs, cm);
  const int K = cr.n_child;
  double loc[3];
  T isg[3], lnh[3], lnl[3], dmu[3], dsg[3], f[3];
  T last = T(1);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int c0 = cr.res_end[j < K ? j : 0];  // child j's constants
    loc[j] = cs.d[c0];
    isg[j] = cs.get<T>(c0 + 1);
    lnh[j] = cs.get<T>(c0 + 2);
    lnl[j] = cs.get<T>(c0 + 3);
    dmu[j] = cs.get<T>(c0 + 4);
    dsg[j] = cs.get<T>(c0 + 5);
    f[j] = j < K ? cs.get<T>(cr.c0 + j) : T(0);  // the ADD's staged fractions, the last one included
  }
  (void)last;
  if constexpr (TAB) {
    // per component the sums of w_j z_j and w_j z_j^2 (kept in gr[2j] and
    // gr[2j + 1]) and of w_j (the first K - 1 in gr[2K + j], the last in
    // wl); the slot sums f_j (w_j (z_j / sigma_j - dlnN_j/dmu_j)) and
    // f_j (w_j (z_j^2 / sigma_j - dlnN_j/dsigma_j)) and the fractions'
    // w_j - w_K follow once per event
    T wl = T(0);
    // the term loop specialised on the component count (2 or 3)
    const auto run = [&](auto kc) __attribute__((always_inline)) {
      constexpr int KC = decltype(kc)::value;
      conv_window<true>(x, lo, hh, dlo, dhi, ref, k0, k1, [&](int k, double, double v) {
        const T lm = tab->v[0][k];  // shift already subtracted
        T sw = T(0);
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          const T z = (T)(v + loc[j]) * isg[j];
          const T z2 = z * z;
          const T w = Mth<T>::ex(((lm - T(0.5) * z2) - lnh[j]) - lnl[j]);
          sw = Mth<T>::fma(f[j], w, sw);
          gr[2 * j] = Mth<T>::fma(w, z, gr[2 * j]);
          gr[2 * j + 1] = Mth<T>::fma(w, z2, gr[2 * j + 1]);
          if (j + 1 < KC) gr[2 * KC + j] += w;
          else wl += w;
        }
        S += sw;
#pragma unroll
        for (int j = 0; j < 4; ++j) gm[j] = Mth<T>::fma(sw, tab->v[1 + j][k], gm[j]);
      });
    };
    if (K == 2) run(std::integral_constant<int, 2>{});
    else run(std::integral_constant<int, 3>{});
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (j < K) {
        const T wj = j + 1 < K ? gr[2 * K + j] : wl;
        gr[2 * j] = f[j] * (isg[j] * gr[2 * j] - dmu[j] * wj);
        gr[2 * j + 1] = f[j] * (isg[j] * gr[2 * j + 1] - dsg[j] * wj);
      }
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (j + 1 < K) gr[2 * K + j] -= wl;
    return;
  }
  conv_window(x, lo, hh, dlo, dhi, ref, k0, k1, [&](int k, double vm, double v) {
    T dm[4];
    const T lm = M.eval(vm, dm) - shift;
    T w[3], sw = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j < K) {
        const T z = (T)(v + loc[j]) * isg[j];
        w[j] = Mth<T>::ex(((lm - T(0.5) * z * z) - lnh[j]) - lnl[j]);
        const T fw = f[j] * w[j];
        sw += fw;
        gr[2 * j] = Mth<T>::fma(fw, z * isg[j] - dmu[j], gr[2 * j]);
        gr[2 * j + 1] = Mth<T>::fma(fw, z * z * isg[j] - dsg[j], gr[2 * j + 1]);
      }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
      if (j + 1 < K) gr[2 * K + j] += w[j] - w[K - 1];
    S += sw;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < cm.n_slot) gm[j] = Mth<T>::fma(sw, dm[j], gm[j]);
  });
}

// General trees (ADD / PROD over leaves).  Node log-values, adjoints and the
// per-event slot derivatives live in small VGPR arrays indexed by
// wave-uniform node / slot numbers.
// Returns ln P of the root (without the normalisations of hoisted nodes)
// and, with GRAD, its slot derivatives in dl[0 .. P.n_slots).
// HEAVY: 0 light nodes only; 1 adds CONV and COMP; 2 also DALITZ / TDDP;
// kHeavyConvTab as 1 with the CONV node's model read from the row's LDS
// table tab (node tab_node, staged by conv_stage).
template <typename T, int NS, int NCOL, int HEAVY, bool GRAD>
__device__ __forceinline__ T tree_eval(const KProgram& P, const CS& cs, const double* xe, T* dl,
                                       const ConvTab<T>* tab = nullptr, int tab_node = -1) {
    // node capacity of this instantiation; float arrays get 16 entries so
    // that the compiler indexes them with register moves (8 floats become
    // chains of compares and selects, one per entry and access; 8 doubles
    // are already indexed)
    constexpr int NN = HEAVY || sizeof(T) == 4 ? kMaxNodes : 8;
    const int n_nodes = P.n_nodes;
    T lv[NN], adj[NN], resp[NN];
    // forward pass (post-order)
    for (int k = 0; k < n_nodes; ++k) {
      const KNode& nd = P.node[k];
      const int op = nd.op;
      const int c0 = nd.c0, s0 = nd.slot0;
      const bool h = nd.hoisted != 0;
      T v;
      if (op == OP_EXP) {
        T d1[1];
        v = leaf_exp<T>(cs, c0, h, xe[nd.col[0]], d1);
        dl[s0] = d1[0];
      } else if (op == OP_GAUSS) {
        T d2[2];
        v = leaf_gauss<T>(cs, c0, h, xe[nd.col[0]], d2);
        dl[s0] = d2[0];
        dl[s0 + 1] = d2[1];
      } else if (op == OP_POLY) {
        T dp[8];
        v = leaf_poly<T>(cs, c0, nd.aux, h, xe[nd.col[0]], dp);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < nd.aux) dl[s0 + j] = dp[j];
      } else if (HEAVY == 2 && (op == OP_DALITZ || op == OP_TDDP)) {
        const int ns = nd.n_slot;
        const auto emit = [&](int j, const T (&d)[1]) {
          if (j < ns) dl[s0 + j] = d[0];
        };
        const double x12[1] = {xe[nd.col[0]]}, x13[1] = {xe[nd.col[1]]};
        T l1[1];
        if (op == OP_DALITZ) {
          leaf_dalitz<T, 1>(cs, nd, h, x12, x13, l1, emit);
        } else {
          const double xt[1] = {xe[nd.col[2]]}, xs[1] = {xe[nd.col[3]]};
          if (nd.n_slot == 2 * nd.aux + 3) leaf_tddp<T, 1, true>(cs, nd, h, x12, x13, xt, xs, l1, emit);
          else leaf_tddp<T, 1, false>(cs, nd, h, x12, x13, xt, xs, l1, emit);
        }
        v = l1[0];
      } else if (op == OP_PROD) {
        // with leaves that share an observable (aux), unhoisted: minus ln Z
        // of their products and its derivatives in the children's slots
        const bool sub = nd.aux != 0 && !h;
        v = T(0);
        int m = 0;
        for (int j = 0; j < nd.n_child; ++j) {
          const int ch = P.child[nd.child0 + j];
          v += lv[ch];
          resp[ch] = T(1);
          const KNode& cn = P.node[ch];
          if (sub)
            for (int q = 0; q < cn.n_slot; ++q, ++m) dl[cn.slot0 + q] -= cs.get<T>(c0 + 2 + m);
        }
        if (sub) v = (v - cs.get<T>(c0)) - cs.get<T>(c0 + 1);
      } else if (op == OP_MAP) {
        // the child whose range holds x gives the value (increasing
        // boundaries compared with the stored event's value, the column
        // reference added back in double, as the definition takes them);
        // the other children's slot derivatives are dropped (set, not
        // scaled: they may be undefined outside their ranges); unhoisted,
        // ln Z and its slot derivatives are subtracted here
        const int K = nd.n_child;
        const double x = xe[nd.col[0]] + cs.d[c0 + K - 1];
        int sel = 0;
        for (int j = 0; j < K - 1; ++j) sel += x >= cs.d[c0 + j] ? 1 : 0;
        v = T(0);
        int m = 0;
        for (int j = 0; j < K; ++j) {
          const int ch = P.child[nd.child0 + j];
          const bool on = sel == j;
          v = on ? lv[ch] : v;
          resp[ch] = T(1);
          const KNode& cn = P.node[ch];
          for (int q = 0; q < cn.n_slot; ++q, ++m) {
            T d = on ? dl[cn.slot0 + q] : T(0);
            if (!h) d -= cs.get<T>(c0 + K + 2 + m);
            dl[cn.slot0 + q] = d;
          }
        }
        if (!h) v = (v - cs.get<T>(c0 + K)) - cs.get<T>(c0 + K + 1);
      } else if (HEAVY && op == OP_CONV) {
        // numerical convolution: sum over the grid t_k of f_M(t_k) f_R(x - t_k)
        // with the residual in [d_lo, d_hi] and the exponents shifted by c;
        // the children's slots receive the convolution's derivatives
        const int N = nd.aux;
        const int chm = P.child[nd.child0], chr = P.child[nd.child0 + 1];
        const KNode& cm = P.node[chm];
        const KNode& cr = P.node[chr];
        // the resolution's slots: its own, or (a mixture of Gaussians) its
        // Gaussians' and its fractions, contiguous and ending with its own
        const bool mixr = cr.op == OP_ADD;
        const int nm = cm.n_slot, nr = mixr ? 3 * cr.n_child - 1 : cr.n_slot;
        const int r_first = cr.slot0 + cr.n_slot - nr;
        const double lo = cs.d[c0], hh = cs.d[c0 + 1], dlo = cs.d[c0 + 2], dhi = cs.d[c0 + 3], ref = cs.d[c0 + 4];
        const double x = xe[nd.col[0]] + ref;  // the stored event's value
        const T shift = cs.get<T>(c0 + 5);
        T S = T(0), gm[8], gr[8];
        bool undef = false;  // the resolution's shape not positive at a residual in use
#pragma unroll
        for (int j = 0; j < 8; ++j) gm[j] = gr[j] = T(0);
        // Only the grid points whose residual can lie in [d_lo, d_hi] are
        // visited: k in [(x - d_hi - lo)/h - 1/2, (x - d_lo - lo)/h - 1/2],
        // widened by one point on each side so that rounding of these
        // bounds cannot drop one; the range test (t_k and x - t_k in double,
        // as the definition takes them) decides.  Datasets of graphs with a
        // CONV node are stored sorted by x, so a wave's lanes run loops of
        // nearly the same range.
        int k0 = (int)__builtin_ceil((x - dhi - lo) / hh - 0.5) - 1;
        int k1 = (int)__builtin_floor((x - dlo - lo) / hh - 0.5) + 1;
        k0 = k0 < 0 ? 0 : k0;
        k1 = k1 > N - 1 ? N - 1 : k1;
        // the term loop is specialised on the resolution's kind; the
        // children's constants are read once into registers.  The staged
        // instantiation (HEAVY == kHeavyConvTab, chosen on the host for
        // graphs whose one CONV node qualifies) reads the model from the
        // row's LDS table and has no per-term model code: carrying both
        // loops makes the interpreter copy its kernel argument to scratch
#define HF_CONV_CASE(R_, TAB_)                                                                            \
  if (cr.op == R_) conv_terms<T, R_, TAB_>(cs, cm, cr, x, lo, hh, dlo, dhi, ref, shift, k0, k1, S, gm, gr, undef, tab);
        constexpr bool TAB = HEAVY == kHeavyConvTab;
        if (mixr) conv_terms_gmix<T, TAB>(cs, P, cm, cr, x, lo, hh, dlo, dhi, ref, shift, k0, k1, S, gm, gr, tab);
        else HF_CONV_CASE(OP_GAUSS, TAB) else HF_CONV_CASE(OP_EXP, TAB) else HF_CONV_CASE(OP_POLY, TAB)
#undef HF_CONV_CASE
        const T iS = Mth<T>::rcp(S);
        v = S > T(0) && !undef ? Mth<T>::ln(S) : T(-INFINITY);
        v = (v - cs.get<T>(c0 + 6)) - cs.get<T>(c0 + 7);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (j < nm) dl[cm.slot0 + j] = gm[j] * iS - cs.get<T>(c0 + 8 + j);
          if (j < nr) dl[r_first + j] = gr[j] * iS - cs.get<T>(c0 + 8 + nm + j);
        }
        resp[chm] = T(1);
        resp[chr] = T(1);
        // a mixture's Gaussians carry the convolution's derivatives, scaled
        // only by its adjoint in the reverse pass
        if (mixr)
          for (int j = 0; j < cr.n_child; ++j) resp[P.child[cr.child0 + j]] = T(1);
      } else if (op == OP_COMP) {
        // composition f(g(x)): the core's value g = 1 + sum a_j u^j
        // (u = x - x0), the shell's shape at g; the children's slots receive
        // d ln f / dg (x - x0)^j and the shell's own derivatives
        const int chc = P.child[nd.child0], chf = P.child[nd.child0 + 1];
        const KNode& cc = P.node[chc];
        const KNode& cf = P.node[chf];
        const int nc = cc.n_slot, nf = cf.n_slot;
        const T u = (T)(xe[nd.col[0]] + cs.d[cc.c0]);
        T uk[4], gv = T(1), w = T(1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          w *= u;
          uk[j] = w;
          if (j < nc) gv = Mth<T>::fma(cs.get<T>(cc.c0 + 1 + j), w, gv);
        }
        T df[8];
        const double ref = cs.d[c0 + 2];
        const T lf = conv_leaf<T>(cs, cf, (double)gv - ref, df);
        T dfdg;
        if (cf.op == OP_EXP) {
          dfdg = cs.get<T>(cf.c0 + 1);
        } else if (cf.op == OP_GAUSS) {
          dfdg = -df[0];
        } else {
          const T v0 = (T)((double)gv - ref + cs.d[cf.c0]);
          T pv = T(1), dp = T(0), vk = T(1);
#pragma unroll
          for (int j = 1; j <= 4; ++j)
            if (j <= nf) {
              dp = Mth<T>::fma(T(j) * cs.get<T>(cf.c0 + j), vk, dp);
              vk *= v0;
              pv = Mth<T>::fma(cs.get<T>(cf.c0 + j), vk, pv);
            }
          dfdg = dp * Mth<T>::rcp(pv);
        }
        v = (lf - cs.get<T>(c0)) - cs.get<T>(c0 + 1);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < nc) dl[cc.slot0 + j] = dfdg * uk[j] - cs.get<T>(c0 + 3 + j);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < nf) dl[cf.slot0 + j] = df[j] - cs.get<T>(c0 + 3 + nc + j);
        resp[chc] = T(1);
        resp[chf] = T(1);
      } else if (op == OP_DPMAP) {
        // the child of the event's cell on the s12 x s13 grid (row-major;
        // boundaries compared with the stored values, the column references
        // added back in double) gives the value; the other children's slot
        // derivatives are dropped
        const int K = nd.n_child, n13 = nd.aux, n12 = K / n13;
        const double a = xe[nd.col[0]] + cs.d[c0], b = xe[nd.col[1]] + cs.d[c0 + 1];
        int i12 = 0, i13 = 0;
        for (int j = 0; j < n12 - 1; ++j) i12 += a >= cs.d[c0 + 2 + j] ? 1 : 0;
        for (int j = 0; j < n13 - 1; ++j) i13 += b >= cs.d[c0 + 2 + n12 - 1 + j] ? 1 : 0;
        const int sel = i12 * n13 + i13;
        v = T(0);
        for (int j = 0; j < K; ++j) {
          const int ch = P.child[nd.child0 + j];
          const bool on = sel == j;
          v = on ? lv[ch] : v;
          resp[ch] = T(1);
          const KNode& cn = P.node[ch];
          for (int q = 0; q < cn.n_slot; ++q) dl[cn.slot0 + q] = on ? dl[cn.slot0 + q] : T(0);
        }
      } else {  // OP_ADD: log-sum-exp with the largest child as pivot
        const int K = nd.n_child;
        T m = T(-INFINITY);
        for (int j = 0; j < K; ++j) {
          const T x = lv[P.child[nd.child0 + j]];
          m = x > m ? x : m;
        }
        const bool live = m > T(-INFINITY);
        T s = T(0);
        for (int j = 0; j < K; ++j) {
          const int ch = P.child[nd.child0 + j];
          const T w = live ? Mth<T>::ex(lv[ch] - m) : T(0);
          resp[ch] = w;  // e_j for now
          s += cs.get<T>(c0 + j) * w;
        }
        const T is = Mth<T>::rcp(s);
        v = live && s > T(0) ? m + Mth<T>::ln(s) : T(-INFINITY);
        if (!h) v -= cs.get<T>(c0 + K);  // ln of the fractions' sum (hoisted: on the host)
        const T eK = resp[P.child[nd.child0 + K - 1]];
        for (int j = 0; j < K; ++j) {
          const int ch = P.child[nd.child0 + j];
          const T ej = resp[ch];
          if (j < K - 1) dl[s0 + j] = (ej - eK) * is;
          resp[ch] = cs.get<T>(c0 + j) * ej * is;  // responsibility of child j
        }
      }
      lv[k] = v;
    }
    // reverse pass: adjoint of every node, then scale its slots
    const int root = n_nodes - 1;
    adj[root] = T(1);
    for (int k = GRAD ? root : -1; k >= 0; --k) {
      const KNode& nd = P.node[k];
      const T a = adj[k];
      if (nd.op == OP_ADD || nd.op == OP_PROD || nd.op == OP_MAP || nd.op == OP_DPMAP || nd.op == OP_CONV ||
          nd.op == OP_COMP)
        for (int j = 0; j < nd.n_child; ++j) {
          const int ch = P.child[nd.child0 + j];
          adj[ch] = a * resp[ch];
        }
      if (k != root)
        for (int j = 0; j < nd.n_slot; ++j) dl[nd.slot0 + j] = dl[nd.slot0 + j] * a;
    }
    return lv[root];
}

template <typename T, int NS, int NCOL, int HEAVY, bool GRAD>
struct TreeEv {
  CS cs;
  const ConvTab<T>* tab;  // staged CONV model (HEAVY rows), else null
  int tab_node;
  template <class Acc>
  __device__ __forceinline__ void operator()(const KProgram& P, const double* xe, int64_t, const Acc& acc) const {
    const int n_slots = GRAD ? P.n_slots : 0;
    T dl[sizeof(T) == 4 && NS < 16 ? 16 : NS];  // indexed with register moves (see tree_eval)
    const T lr = tree_eval<T, NS, NCOL, HEAVY, GRAD>(P, cs, xe, dl, tab, tab_node);
    acc.add(0, -(double)lr);
#pragma unroll
    for (int j = 0; j < NS; ++j)
      if (j < n_slots) acc.add(1 + j, (double)dl[j]);
  }
};

// Light trees (EXP, GAUSS, POLY leaves under ADD, PROD, MAP and COMP; at most
// 8 nodes, 8 slots and 2 columns; a DPMAP only ever sits beside a DALITZ /
// TDDP node, so never here) for E events per walk of the node
// list: each node's fields are read and its kind decided once for the E
// events, which take the same arithmetic as in tree_eval.  Values, adjoints
// and slot derivatives are [node or slot][event] arrays, so that one index
// serves the E events.
template <typename T, int E, bool GRAD>
__device__ __forceinline__ void tree_eval_light(const KProgram& P, const CS& cs, const double (&xe)[E][2],
                                                T (&dl)[8][E], T (&out)[E]) {
  constexpr int NN = 8;
  const int n_nodes = P.n_nodes;
  T lv[NN][E], adj[NN][E], resp[NN][E];
  for (int k = 0; k < n_nodes; ++k) {
    const KNode& nd = P.node[k];
    const int op = nd.op;
    const int c0 = nd.c0, s0 = nd.slot0;
    const bool h = nd.hoisted != 0;
    T v[E];
    if (op == OP_EXP) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        T d1[1];
        v[e] = leaf_exp<T>(cs, c0, h, (nd.col[0] ? xe[e][1] : xe[e][0]), d1);
        dl[s0][e] = d1[0];
      }
    } else if (op == OP_GAUSS) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        T d2[2];
        v[e] = leaf_gauss<T>(cs, c0, h, (nd.col[0] ? xe[e][1] : xe[e][0]), d2);
        dl[s0][e] = d2[0];
        dl[s0 + 1][e] = d2[1];
      }
    } else if (op == OP_POLY) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        T dp[8];
        v[e] = leaf_poly<T>(cs, c0, nd.aux, h, (nd.col[0] ? xe[e][1] : xe[e][0]), dp);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < nd.aux) dl[s0 + j][e] = dp[j];
      }
    } else if (op == OP_PROD) {
      const bool sub = nd.aux != 0 && !h;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = T(0);
      int m = 0;
      for (int j = 0; j < nd.n_child; ++j) {
        const int ch = P.child[nd.child0 + j];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          v[e] += lv[ch][e];
          resp[ch][e] = T(1);
        }
        const KNode& cn = P.node[ch];
        if (sub)
          for (int q = 0; q < cn.n_slot; ++q, ++m) {
            const T dz = cs.get<T>(c0 + 2 + m);
#pragma unroll
            for (int e = 0; e < E; ++e) dl[cn.slot0 + q][e] -= dz;
          }
      }
      if (sub)
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = (v[e] - cs.get<T>(c0)) - cs.get<T>(c0 + 1);
    } else if (op == OP_MAP) {
      const int K = nd.n_child;
      int sel[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double x = (nd.col[0] ? xe[e][1] : xe[e][0]) + cs.d[c0 + K - 1];
        sel[e] = 0;
        for (int j = 0; j < K - 1; ++j) sel[e] += x >= cs.d[c0 + j] ? 1 : 0;
        v[e] = T(0);
      }
      int m = 0;
      for (int j = 0; j < K; ++j) {
        const int ch = P.child[nd.child0 + j];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          v[e] = sel[e] == j ? lv[ch][e] : v[e];
          resp[ch][e] = T(1);
        }
        const KNode& cn = P.node[ch];
        for (int q = 0; q < cn.n_slot; ++q, ++m) {
#pragma unroll
          for (int e = 0; e < E; ++e) {
            T d = sel[e] == j ? dl[cn.slot0 + q][e] : T(0);
            if (!h) d -= cs.get<T>(c0 + K + 2 + m);
            dl[cn.slot0 + q][e] = d;
          }
        }
      }
      if (!h)
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = (v[e] - cs.get<T>(c0 + K)) - cs.get<T>(c0 + K + 1);
    } else if (op == OP_COMP) {
      // composition f(g(x)), as in tree_eval
      const int chc = P.child[nd.child0], chf = P.child[nd.child0 + 1];
      const KNode& cc = P.node[chc];
      const KNode& cf = P.node[chf];
      const int nc = cc.n_slot, nf = cf.n_slot;
      const double ref = cs.d[c0 + 2];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const T u = (T)((nd.col[0] ? xe[e][1] : xe[e][0]) + cs.d[cc.c0]);
        T uk[4], gv = T(1), w = T(1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          w *= u;
          uk[j] = w;
          if (j < nc) gv = Mth<T>::fma(cs.get<T>(cc.c0 + 1 + j), w, gv);
        }
        T df[8];
        const T lf = conv_leaf<T>(cs, cf, (double)gv - ref, df);
        T dfdg;
        if (cf.op == OP_EXP) {
          dfdg = cs.get<T>(cf.c0 + 1);
        } else if (cf.op == OP_GAUSS) {
          dfdg = -df[0];
        } else {
          const T v0 = (T)((double)gv - ref + cs.d[cf.c0]);
          T pv = T(1), dp = T(0), vk = T(1);
#pragma unroll
          for (int j = 1; j <= 4; ++j)
            if (j <= nf) {
              dp = Mth<T>::fma(T(j) * cs.get<T>(cf.c0 + j), vk, dp);
              vk *= v0;
              pv = Mth<T>::fma(cs.get<T>(cf.c0 + j), vk, pv);
            }
          dfdg = dp * Mth<T>::rcp(pv);
        }
        v[e] = (lf - cs.get<T>(c0)) - cs.get<T>(c0 + 1);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < nc) dl[cc.slot0 + j][e] = dfdg * uk[j] - cs.get<T>(c0 + 3 + j);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < nf) dl[cf.slot0 + j][e] = df[j] - cs.get<T>(c0 + 3 + nc + j);
        resp[chc][e] = T(1);
        resp[chf][e] = T(1);
      }
    } else {  // OP_ADD: log-sum-exp with the largest child as pivot
      const int K = nd.n_child;
      T mx[E], sm[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        mx[e] = T(-INFINITY);
        sm[e] = T(0);
      }
      for (int j = 0; j < K; ++j) {
        const int ch = P.child[nd.child0 + j];
#pragma unroll
        for (int e = 0; e < E; ++e) mx[e] = lv[ch][e] > mx[e] ? lv[ch][e] : mx[e];
      }
      for (int j = 0; j < K; ++j) {
        const int ch = P.child[nd.child0 + j];
        const T fj = cs.get<T>(c0 + j);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const T w = mx[e] > T(-INFINITY) ? Mth<T>::ex(lv[ch][e] - mx[e]) : T(0);
          resp[ch][e] = w;  // e_j for now
          sm[e] += fj * w;
        }
      }
      T is[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        is[e] = Mth<T>::rcp(sm[e]);
        v[e] = mx[e] > T(-INFINITY) && sm[e] > T(0) ? mx[e] + Mth<T>::ln(sm[e]) : T(-INFINITY);
        if (!h) v[e] -= cs.get<T>(c0 + K);
      }
      const int chK = P.child[nd.child0 + K - 1];
      T eK[E];
#pragma unroll
      for (int e = 0; e < E; ++e) eK[e] = resp[chK][e];
      for (int j = 0; j < K; ++j) {
        const int ch = P.child[nd.child0 + j];
        const T fj = cs.get<T>(c0 + j);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const T ej = resp[ch][e];
          if (j < K - 1) dl[s0 + j][e] = (ej - eK[e]) * is[e];
          resp[ch][e] = fj * ej * is[e];  // responsibility of child j
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) lv[k][e] = v[e];
  }
  const int root = n_nodes - 1;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    adj[root][e] = T(1);
    out[e] = lv[root][e];
  }
  for (int k = GRAD ? root : -1; k >= 0; --k) {
    const KNode& nd = P.node[k];
    if (nd.op == OP_ADD || nd.op == OP_PROD || nd.op == OP_MAP || nd.op == OP_COMP)
      for (int j = 0; j < nd.n_child; ++j) {
        const int ch = P.child[nd.child0 + j];
#pragma unroll
        for (int e = 0; e < E; ++e) adj[ch][e] = adj[k][e] * resp[ch][e];
      }
    if (k != root)
      for (int j = 0; j < nd.n_slot; ++j)
#pragma unroll
        for (int e = 0; e < E; ++e) dl[nd.slot0 + j][e] = dl[nd.slot0 + j][e] * adj[k][e];
  }
}

// Row loop of the light-tree kernels: E consecutive chunks per step (a
// thread's E events, the next step's loads in flight); an event past the
// row's end takes the step's first event's values and is not added.
template <typename T, int E, bool GRAD, class Acc>
__device__ __forceinline__ void light_tree_row(const KProgram& P, const CS& cs, const typename Col<T>::S* const* cp,
                                               int ncols, int64_t n, int64_t c0, int64_t c1, const Acc& acc) {
  typedef typename Col<T>::S Sx;
  const int64_t t = threadIdx.x;
  const int n_slots = GRAD ? P.n_slots : 0;
  Sx cur[E][2];
  const auto load = [&](int64_t ch, Sx (&dst)[E][2]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t i = (ch + e) * kBlock + t;
      const bool ok = ch + e < c1 && i < n;
#pragma unroll
      for (int c = 0; c < 2; ++c) dst[e][c] = (c < ncols && ok) ? cp[c][i] : Sx(0);
    }
  };
  if (c0 < c1) load(c0, cur);
#pragma unroll 1
  for (int64_t ch = c0; ch < c1; ch += E) {
    bool ok[E];
    double xe[E][2];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ok[e] = ch + e < c1 && (ch + e) * kBlock + t < n;
#pragma unroll
      for (int c = 0; c < 2; ++c) xe[e][c] = (double)(ok[e] ? cur[e][c] : cur[0][c]);
    }
    if (ch + E < c1) load(ch + E, cur);
    if (!ok[0]) continue;
    T dl[8][E], lr[E];
    tree_eval_light<T, E, GRAD>(P, cs, xe, dl, lr);
    double nl = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (ok[e]) nl -= (double)lr[e];
    acc.add(0, nl);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < n_slots) {
        double g = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (ok[e]) g += (double)dl[j][e];
        acc.add(1 + j, g);
      }
  }
}

// Binned metrics over bin centres with weights w (metric 1: -w ln P; metric
// 2: (w - K P)^2 / max(w, 1)).  ln P is the full log-density: the hoisted
// normalisations L are subtracted here.  Accumulators: [metric, sum over
// bins of dmetric/dlnP x slot derivatives, sum of dmetric/dlnP] -- the last
// carries the hoisted normalisations' derivatives on the host.
template <typename T, int NS, int NCOL, int HEAVY, bool GRAD>
struct BinnedEv {
  CS cs;
  const double* w;
  double K, L;
  int metric;
  template <class Acc>
  __device__ __forceinline__ void operator()(const KProgram& P, const double* xe, int64_t i, const Acc& acc) const {
    const int n_slots = GRAD ? P.n_slots : 0;
    T dl[sizeof(T) == 4 && NS < 16 ? 16 : NS];  // indexed with register moves (see tree_eval)
    const double lp = (double)tree_eval<T, NS, NCOL, HEAVY, GRAD>(P, cs, xe, dl) - L;
    const double wi = w[i];
    double term, dterm;
    if (metric == 1) {
      term = wi != 0.0 ? -wi * lp : 0.0;
      dterm = -wi;
    } else {
      const double E = lp > -INFINITY ? K * ::exp(lp) : 0.0;
      const double r = wi - E, s2 = wi > 1.0 ? wi : 1.0;
      term = r * r / s2;
      dterm = -2.0 * r * E / s2;
    }
    acc.add(0, term);
    if (GRAD) {
#pragma unroll
      for (int j = 0; j < NS; ++j)
        if (j < n_slots) acc.add(1 + j, dterm * (double)dl[j]);
      acc.add(1 + n_slots, dterm);
    }
  }
};

// ------------------------------------------------------------------ rows
constexpr int kUnroll = 8;  // chunks per group in the single-column kernels

template <typename T, int K, int MASK, bool GRAD, bool TM = false>
__device__ __forceinline__ void mix_row(const KProgram& P, const CS& cs, const void* const* cols, int64_t n,
                                        int n_rows, int r, double* __restrict__ out) {
  constexpr int NC = 1 + (GRAD ? 3 * K : 0);
  const auto ev = make_mix<T, K, MASK, GRAD>(P, cs);
  double acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = 0.0;
  int64_t c0, c1;
  row_chunks(n, n_rows, r, c0, c1);
  light_row<T, kUnroll>(ev, (const typename Col<T>::S*)cols[0], n, c0, c1, acc);
  if constexpr (TM) thread_store<NC>(acc, NC, out, out_stride<TM>(n_rows));
  else row_store_lds<NC>(acc, out, n_rows);
}

template <typename T, int OP, bool GRAD, bool TM = false>
__device__ __forceinline__ void light_leaf_row(const KNode& nd, const CS& cs, const void* const* cols, int64_t n,
                                               int n_rows, int r, double* __restrict__ out) {
  typedef LightLeafEv<T, OP, GRAD> Ev;
  constexpr int NC = 1 + Ev::NA;
  Ev ev;
  ev.cs = cs;
  ev.c0 = nd.c0;
  ev.hoisted = nd.hoisted != 0;
  double acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = 0.0;
  int64_t c0, c1;
  row_chunks(n, n_rows, r, c0, c1);
  light_row<T, kUnroll>(ev, (const typename Col<T>::S*)cols[nd.col[0]], n, c0, c1, acc);
  if constexpr (TM) thread_store<NC>(acc, NC, out, out_stride<TM>(n_rows));
  else row_store_lds<NC>(acc, out, n_rows);
}

// Single DALITZ / TDDP leaf (the root: its normalisation is applied on the
// host).  A thread takes event t of E consecutive chunks per step (the next
// step's columns in flight) and adds each slot's E derivatives, summed in
// double, with one LDS add.  Events past the row's end are replaced by the
// step's first event and weighted out; a thread whose first event is past
// the end has none left.
// One (unhoisted) EXP / GAUSS / POLY child of a DPMAP at u: ln P and its
// slot derivatives in d[0 .. n_slot).
template <typename T>
__device__ __forceinline__ T dpmap_child(const CS& cs, const KNode& cn, double u, T (&d)[8]) {
  if (cn.op == OP_EXP) return leaf_exp<T>(cs, cn.c0, false, u, d);
  if (cn.op == OP_GAUSS) return leaf_gauss<T>(cs, cn.c0, false, u, d);
  return leaf_poly<T>(cs, cn.c0, cn.aux, false, u, d);
}

// A DPMAP's cell boundaries and, when every child is a Gaussian, each
// cell's constants, staged in LDS once per row by one lane (reading the
// kernel argument at uniform indices only): per event the cell comes from
// broadcast reads of the boundaries and its constants from one lane-indexed
// read of the table, instead of chains of dependent scalar loads per child.
struct SigLds {
  double r12, r13;           // column references of s12 and s13
  double b[2 * kMaxNodes];   // s12 boundaries, then s13
  double tab[kMaxNodes][8];  // loc = ref - mu, 1/sigma, lnN hi, lnN lo, dlnN/dmu, dlnN/dsigma, first slot
};

template <typename T>
__device__ __forceinline__ bool sig_stage(const KProgram& P, const CS& cs, const KNode& dm, SigLds& L) {
  const int K = dm.n_child, n13 = dm.aux, n12 = K / n13;
  bool all = true;
  for (int j = 0; j < K; ++j) all = all && P.node[P.child[dm.child0 + j]].op == OP_GAUSS;
  if (threadIdx.x == 0) {
    L.r12 = cs.d[dm.c0];
    L.r13 = cs.d[dm.c0 + 1];
    for (int j = 0; j < n12 + n13 - 2; ++j) L.b[j] = cs.d[dm.c0 + 2 + j];
    if (all)
      for (int j = 0; j < K; ++j) {
        const KNode& cn = P.node[P.child[dm.child0 + j]];
        L.tab[j][0] = cs.d[cn.c0];
#pragma unroll
        for (int q = 1; q < 6; ++q) L.tab[j][q] = (double)cs.get<T>(cn.c0 + q);
        L.tab[j][6] = (double)cn.slot0;
      }
  }
  __syncthreads();
  return all;
}

// Cell of the stored values (a, b) on the n12 x n13 grid (row-major).
__device__ __forceinline__ int sig_cell(const SigLds& L, int n12, int n13, double a_off, double b_off) {
  const double a = a_off + L.r12, b = b_off + L.r13;
  int i12 = 0, i13 = 0;
  for (int j = 0; j < n12 - 1; ++j) i12 += a >= L.b[j] ? 1 : 0;
  for (int j = 0; j < n13 - 1; ++j) i13 += b >= L.b[n12 - 1 + j] ? 1 : 0;
  return i12 * n13 + i13;
}

// Time-dependent Dalitz kernels with the sigma_t density that varies across
// the plot (a root PROD of the TDDP node, node 0, and a DPMAP on its s12,
// s13 and sigma_t, the last node but one): the per-event value of the
// event's cell joins ln P in the main loop; the map's slot derivatives are
// summed in a second, light pass over the row (s12, s13 and sigma_t only),
// whose accumulators reuse the LDS of the first.
constexpr int OP_TDDP_S = 17;    // x = 0
constexpr int OP_TDDP_XS = 18;   // x free
constexpr int OP_TDDP_F = 19;    // the full model (its own row function)
template <int OP> struct AmpOp {
  static constexpr int base = OP == OP_TDDP_S ? OP_TDDP : (OP == OP_TDDP_XS ? OP_TDDP_X : OP);
  static constexpr bool sig = OP == OP_TDDP_S || OP == OP_TDDP_XS;
};

template <typename T, int OP, bool GRAD, bool TM = false>
__device__ __forceinline__ void amp_leaf_row(const KProgram& P, const CS& cs, const void* const* cols, int64_t n,
                                             int n_rows, int r, double* __restrict__ out) {
  typedef typename Col<T>::S Sx;
  constexpr int BOP = AmpOp<OP>::base;
  constexpr bool SIG = AmpOp<OP>::sig;
  constexpr int E = AmpEvents<T, BOP>::value;
  constexpr int NCOL = BOP == OP_DALITZ ? 2 : 4;
  constexpr int NS = BOP == OP_DALITZ ? 2 * kMaxRes : (BOP == OP_TDDP ? 2 * kMaxRes + 2 : 2 * kMaxRes + 3);
  constexpr int NC = 1 + NS;
  const KNode& nd = P.node[0];
  // slot columns: 2R coefficient derivatives (+ tau, y); zero derivatives
  // land in the columns up to 2 kMaxRes, so all are cleared.  With the
  // sigma_t map the first pass stores the amplitude node's columns only.
  const int n_slots = GRAD ? (SIG ? nd.n_slot : P.n_slots) : 0;
  const Sx* cp[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) cp[c] = (const Sx*)cols[nd.col[c]];
  __shared__ double accs[NC][kBlock];
  const LdsAcc<NC> acc{accs};
  acc.zero(GRAD ? NC : 1);
  __shared__ SigLds sl;  // sigma_t map (SIG only)
  bool all_gauss = false;
  if constexpr (SIG) all_gauss = sig_stage<T>(P, cs, P.node[P.n_nodes - 2], sl);
  int64_t c0, c1;
  row_chunks(n, n_rows, r, c0, c1);
  const int64_t t = threadIdx.x;
  Sx cur[E][NCOL];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int64_t i = (c0 + e) * kBlock + t;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) cur[e][c] = (c0 + e < c1 && i < n) ? cp[c][i] : Sx(0);
  }
#pragma unroll 1
  for (int64_t ch = c0; ch < c1; ch += E) {
    bool ok[E];
    double x[NCOL][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ok[e] = ch + e < c1 && (ch + e) * kBlock + t < n;
#pragma unroll
      for (int c = 0; c < NCOL; ++c) x[c][e] = (double)(ok[e] ? cur[e][c] : cur[0][c]);
    }
    if (ch + E < c1) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t i1 = (ch + E + e) * kBlock + t;
#pragma unroll
        for (int c = 0; c < NCOL; ++c) cur[e][c] = (ch + E + e < c1 && i1 < n) ? cp[c][i1] : Sx(0);
      }
    }
    if (!ok[0]) continue;
    // sum over the step's valid events, in double
    const auto sum = [&](const T (&v)[E]) {
      double s = (double)v[0];
#pragma unroll
      for (int e = 1; e < E; ++e) s += (double)(ok[e] ? v[e] : T(0));
      return s;
    };
    const auto emit = [&](int j, const T (&v)[E]) {
      if (GRAD) acc.add(1 + j, sum(v));
    };
    T lv[E];
    if constexpr (BOP == OP_DALITZ) leaf_dalitz<T, E>(cs, nd, true, x[0], x[1], lv, emit);
    else leaf_tddp<T, E, BOP == OP_TDDP_X>(cs, nd, true, x[0], x[1], x[2], x[3], lv, emit);
    if constexpr (SIG) {
      const KNode& dm = P.node[P.n_nodes - 2];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int cell = sig_cell(sl, dm.n_child / dm.aux, dm.aux, x[0][e], x[1][e]);
        T v = T(0);
        if (all_gauss) {
          const double* g = sl.tab[cell];
          const T z = (T)(x[3][e] + g[0]) * (T)g[1];
          v = ((T(-0.5) * z * z) - (T)g[2]) - (T)g[3];
        } else {
          for (int j = 0; j < dm.n_child; ++j) {
            T d[8];
            const T lj = dpmap_child<T>(cs, P.node[P.child[dm.child0 + j]], x[3][e], d);
            v = cell == j ? lj : v;
          }
        }
        lv[e] += v;
      }
    }
    acc.add(0, -sum(lv));
  }
  if constexpr (TM) thread_store_acc<NC>(acc, 1 + n_slots, out, out_stride<TM>(n_rows));
  else row_store_acc<NC>(acc, 1 + n_slots, out, n_rows);
  if constexpr (SIG && GRAD) {
    // second pass: the map's slots (columns after the amplitude node's),
    // the selected child's derivatives added to its own columns (all
    // Gaussian: the loads of U chunks issued together; with more, the
    // compiler turns the unrolled selections into lane-indexed reads of the
    // kernel argument and copies it to scratch)
    constexpr int U = 4;
    const KNode& dm = P.node[P.n_nodes - 2];
    const int sb = nd.n_slot, ns2 = P.n_slots - nd.n_slot, n13 = dm.aux, n12 = dm.n_child / n13;
    acc.zero(ns2);
    if (all_gauss) {
#pragma unroll 1
      for (int64_t ch = c0; ch < c1; ch += U) {
        double a[U], b[U], u[U];
#pragma unroll
        for (int e = 0; e < U; ++e) {
          const int64_t i = (ch + e) * kBlock + t;
          const bool ok = ch + e < c1 && i < n;
          a[e] = ok ? (double)cp[0][i] : 0.0;
          b[e] = ok ? (double)cp[1][i] : 0.0;
          u[e] = ok ? (double)cp[3][i] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < U; ++e) {
          if (!(ch + e < c1 && (ch + e) * kBlock + t < n)) continue;
          const double* g = sl.tab[sig_cell(sl, n12, n13, a[e], b[e])];
          const T isg = (T)g[1];
          const T z = (T)(u[e] + g[0]) * isg;
          const int s0 = (int)g[6] - sb;
          acc.add(s0, (double)(z * isg - (T)g[4]));
          acc.add(s0 + 1, (double)(z * z * isg - (T)g[5]));
        }
      }
    } else {
#pragma unroll 1
      for (int64_t ch = c0; ch < c1; ++ch) {
        const int64_t i = ch * kBlock + t;
        if (i >= n) break;
        const double a = (double)cp[0][i], b = (double)cp[1][i], u = (double)cp[3][i];
        const int cell = sig_cell(sl, n12, n13, a, b);
        for (int j = 0; j < dm.n_child; ++j) {
          const KNode& cn = P.node[P.child[dm.child0 + j]];
          T d[8];
          dpmap_child<T>(cs, cn, u, d);
          if (cell == j)
#pragma unroll
            for (int q = 0; q < 8; ++q)
              if (q < cn.n_slot) acc.add(cn.slot0 - sb + q, (double)d[q]);
        }
      }
    }
    if constexpr (TM) thread_store_acc<NC>(acc, ns2, out + (1 + sb) * out_stride<TM>(n_rows), out_stride<TM>(n_rows));
    else row_store_acc<NC>(acc, ns2, out + (int64_t)(1 + sb) * n_rows, n_rows);
  }
}

// Output column (after the 2R coefficient slots) of tail entry j of a full
// node (see leaf_tddp): tau, y, then x, |q/p|, arg q/p and the floating
// shapes where present; -1 for an entry the node does not have.
__device__ __forceinline__ int full_tail_col(const CS& cs, int fb, int j) {
  const int hx = cs.d[fb + kFhx] != 0.0, hq = cs.d[fb + kFhq] != 0.0, nf = (int)cs.d[fb + kFnf];
  if (j < 2) return j;
  if (j == 2) return hx ? 2 : -1;
  if (j < 5) return hq ? 2 + hx + (j - 3) : -1;
  return j - 5 < 2 * nf ? 2 + hx + 2 * hq + (j - 5) : -1;
}

// Single TDDP leaf of the full model (up to kMaxResFull resonances, q/p,
// floating shapes), one event per thread and step.  The NLL and the
// coefficient slots accumulate per thread in LDS (1 + 2 kMaxResFull
// columns), the tail slots (tau, y, x, q/p, shapes) per thread in
// registers; the row store sums both in the same fixed order as the other
// kernels (four waves, then the lanes).
template <typename T, bool GRAD, bool TM = false>
__device__ __forceinline__ void full_leaf_row(const KProgram& P, const CS& cs, const void* const* cols, int64_t n,
                                              int n_rows, int r, double* __restrict__ out) {
  typedef typename Col<T>::S Sx;
  constexpr int NR = kMaxResFull;
  constexpr int NC = 1 + 2 * NR;
  const KNode& nd = P.node[0];
  const int R = nd.aux;
  const int fb = nd.c0 + dz_full_base(R);
  const Sx* cp[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) cp[c] = (const Sx*)cols[nd.col[c]];
  __shared__ double accs[NC][kBlock];
  const LdsAcc<NC> acc{accs};
  acc.zero(GRAD ? NC : 1);
  double tl[kFullTail];
#pragma unroll
  for (int j = 0; j < kFullTail; ++j) tl[j] = 0.0;
  int64_t c0, c1;
  row_chunks(n, n_rows, r, c0, c1);
  const int64_t t = threadIdx.x;
  Sx cur[4];
  {
    const int64_t i = c0 * kBlock + t;
#pragma unroll
    for (int c = 0; c < 4; ++c) cur[c] = (c0 < c1 && i < n) ? cp[c][i] : Sx(0);
  }
#pragma unroll 1
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int64_t i = ch * kBlock + t;
    double x[4][1];
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c][0] = (double)cur[c];
    if (ch + 1 < c1) {
      const int64_t i1 = i + kBlock;
#pragma unroll
      for (int c = 0; c < 4; ++c) cur[c] = i1 < n ? cp[c][i1] : Sx(0);
    }
    if (i >= n) continue;
    const auto emit = [&](int j, const T (&v)[1]) {
      if (GRAD) acc.add(1 + j, (double)v[0]);
    };
    const auto tail = [&](auto j, const T (&v)[1]) {
      constexpr int J = decltype(j)::value;
      if (GRAD) tl[J] += (double)v[0];
    };
    T lv[1];
    leaf_tddp<T, 1, true, NR, true>(cs, nd, true, x[0], x[1], x[2], x[3], lv, emit, tail);
    acc.add(0, -(double)lv[0]);
  }
  const int n_lds = 1 + (GRAD ? 2 * R : 0);
  const int64_t stride = out_stride<TM>(n_rows);
  if constexpr (TM) thread_store_acc<NC>(acc, n_lds, out, stride);
  else row_store_acc<NC>(acc, n_lds, out, n_rows);
  if constexpr (GRAD) {
    if constexpr (TM) {
#pragma unroll
      for (int j = 0; j < kFullTail; ++j) {
        const int col = full_tail_col(cs, fb, j);
        if (col >= 0) out[(int64_t)(1 + 2 * R + col) * stride + threadIdx.x] = tl[j];
      }
    } else {
      __shared__ double red[kBlock / 64][kFullTail];
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
      for (int j = 0; j < kFullTail; ++j) {
        const double v = wave_sum(tl[j]);
        if (lane == 0) red[wave][j] = v;
      }
      __syncthreads();
      const int j = threadIdx.x;
      if (j < kFullTail) {
        const int col = full_tail_col(cs, fb, j);
        if (col >= 0) out[(int64_t)(1 + 2 * R + col) * n_rows] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
      }
      __syncthreads();
    }
  }
}

template <typename T, int NS, int NCOL, int HEAVY, bool GRAD, bool TM = false>
__device__ __forceinline__ void tree_row(const KProgram& P, const CS& cs, const void* const* cols, int64_t n,
                                         int n_rows, int r, double* __restrict__ out) {
  typedef typename Col<T>::S Sx;
  constexpr int NC = 1 + NS;
  ConvTab<T>* tab = nullptr;
  int tab_node = -1;
  if constexpr (HEAVY == kHeavyConvTab) {
    tab = &conv_tab_lds<T>();
    tab_node = conv_stage<T>(P, cs, *tab);
  }
  const TreeEv<T, NS, NCOL, HEAVY, GRAD> ev{cs, tab, tab_node};
  const Sx* cp[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) cp[c] = (const Sx*)cols[c];
  __shared__ double accs[NC][kBlock];
  const LdsAcc<NC> acc{accs};
  const int nc = 1 + (GRAD ? P.n_slots : 0);
  acc.zero(nc);
  int64_t c0, c1;
  row_chunks(n, n_rows, r, c0, c1);
  if constexpr (HEAVY == 0 && !TM) light_tree_row<T, 2, GRAD>(P, cs, cp, P.n_cols, n, c0, c1, acc);
  else heavy_row<T, NCOL>(ev, P, cp, P.n_cols, n, c0, c1, acc);
  if constexpr (TM) thread_store_acc<NC>(acc, nc, out, out_stride<TM>(n_rows));
  else row_store_acc<NC>(acc, nc, out, n_rows);
}

// ------------------------------------------------------------------ kernels (one dataset; one block per row)
// Waves per SIMD the compiler must leave room for: 3 for the float
// time-dependent Dalitz kernel (168 VGPRs instead of 176 keeps three waves
// resident; the others fit as they are).
template <typename T, int OP> struct LeafWaves { static constexpr int value = 1; };
template <> struct LeafWaves<float, OP_TDDP> { static constexpr int value = 3; };
template <> struct LeafWaves<float, OP_TDDP_X> { static constexpr int value = 3; };
template <> struct LeafWaves<float, OP_TDDP_S> { static constexpr int value = 3; };
template <> struct LeafWaves<float, OP_TDDP_XS> { static constexpr int value = 3; };
template <> struct LeafWaves<float, OP_TDDP_F> { static constexpr int value = 2; };

// TM: terms launch (one chunk per row, per-event output, see thread_store);
// the row's output then starts at its first event's place.
template <bool TM>
__device__ __forceinline__ double* row_out(double* partials) {
  return TM ? partials + (int64_t)blockIdx.x * kBlock : partials + blockIdx.x;
}

template <typename T, int OP, bool GRAD, bool TM = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LeafWaves<T, OP>::value)))
void k_leaf(const EvalArgs a) {
  const CS cs{a.prog.c64, a.prog.c32};
  if constexpr (OP == OP_EXP || OP == OP_GAUSS)
    light_leaf_row<T, OP, GRAD, TM>(a.prog.node[0], cs, a.col, a.n_events, a.n_rows, blockIdx.x,
                                    row_out<TM>(a.partials));
  else if constexpr (OP == OP_TDDP_F)
    full_leaf_row<T, GRAD, TM>(a.prog, cs, a.col, a.n_events, a.n_rows, blockIdx.x, row_out<TM>(a.partials));
  else
    amp_leaf_row<T, OP, GRAD, TM>(a.prog, cs, a.col, a.n_events, a.n_rows, blockIdx.x, row_out<TM>(a.partials));
}

// Waves per SIMD the tree kernels must leave room for: 2 for the double
// light-tree kernel (two events per walk fit in 256 registers).
template <typename T, int HEAVY> struct TreeWaves { static constexpr int value = 1; };
template <> struct TreeWaves<double, 0> { static constexpr int value = 2; };
template <> struct TreeWaves<double, 3> { static constexpr int value = 2; };

template <typename T, int NS, int NCOL, int HEAVY, bool GRAD, bool TM = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(TreeWaves<T, HEAVY>::value)))
void k_tree(const EvalArgs a) {
  const CS cs{a.prog.c64, a.prog.c32};
  tree_row<T, NS, NCOL, HEAVY, GRAD, TM>(a.prog, cs, a.col, a.n_events, a.n_rows, blockIdx.x, row_out<TM>(a.partials));
}

template <typename T, int K, int MASK, bool GRAD, bool TM = false>
__global__ __launch_bounds__(kBlock) void k_mix(const EvalArgs a) {
  const CS cs{a.prog.c64, a.prog.c32};
  mix_row<T, K, MASK, GRAD, TM>(a.prog, cs, a.col, a.n_events, a.n_rows, blockIdx.x, row_out<TM>(a.partials));
}

// Single-dataset launches (TM: terms launches) go through hipExtLaunchKernel
// so that timing events (when given) take the dispatch's own start and end
// time stamps.
template <typename T, bool GRAD, bool TM>
inline hipError_t launch_any(int kind, const EvalArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid((unsigned)a.n_rows), block(kBlock);
  switch (kind) {
    case KIND_EXP: hipExtLaunchKernelGGL((k_leaf<T, OP_EXP, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_GAUSS: hipExtLaunchKernelGGL((k_leaf<T, OP_GAUSS, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_TREE_SMALL: hipExtLaunchKernelGGL((k_tree<T, 8, 2, 0, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_DALITZ: hipExtLaunchKernelGGL((k_leaf<T, OP_DALITZ, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_TDDP: hipExtLaunchKernelGGL((k_leaf<T, OP_TDDP, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_TDDPX: hipExtLaunchKernelGGL((k_leaf<T, OP_TDDP_X, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_TDDPS: hipExtLaunchKernelGGL((k_leaf<T, OP_TDDP_S, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_TDDPXS: hipExtLaunchKernelGGL((k_leaf<T, OP_TDDP_XS, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a); break;
    case KIND_TDDPF: return launch_full_leaf(std::is_same<T, float>::value, GRAD, TM, a, st, e0, e1);
    case KIND_TREE:
      hipExtLaunchKernelGGL((k_tree<T, kMaxSlotsTree, kMaxCols, 2, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a);
      break;
    case KIND_TREE_NOAMP:
      hipExtLaunchKernelGGL((k_tree<T, kMaxSlotsTree, kMaxCols, 1, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a);
      break;
    case KIND_TREE_CONV:
      hipExtLaunchKernelGGL((k_tree<T, kMaxSlotsTree, kMaxCols, kHeavyConvTab, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a);
      break;
    case KIND_TREE_CONV_SMALL:
      hipExtLaunchKernelGGL((k_tree<T, ConvSmall<T>::NS, ConvSmall<T>::NCOL, kHeavyConvTab, GRAD, TM>), grid, block, 0,
                            st, e0, e1, 0, a);
      break;
#define HF_MIX(K_, M_)                                                                              \
  case (K_ == 2 ? KIND_MIX2 : KIND_MIX3) + M_:                                                      \
    hipExtLaunchKernelGGL((k_mix<T, K_, M_, GRAD, TM>), grid, block, 0, st, e0, e1, 0, a);              \
    break;
    HF_MIX(2, 0) HF_MIX(2, 1) HF_MIX(2, 2) HF_MIX(2, 3)
    HF_MIX(3, 0) HF_MIX(3, 1) HF_MIX(3, 2) HF_MIX(3, 3) HF_MIX(3, 4) HF_MIX(3, 5) HF_MIX(3, 6) HF_MIX(3, 7)
#undef HF_MIX
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hf
