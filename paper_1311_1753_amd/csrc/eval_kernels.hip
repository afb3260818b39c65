// Per-event likelihood kernels for gfx950 (CDNA4, wave64).
//
// One block of 256 threads owns a fixed tile of TILE = 256 * EPT consecutive
// events; thread t reads events tile*TILE + e*256 + t (e < EPT), so every
// column load is a fully coalesced 256-lane access.  Per event the kernel
// evaluates the flattened PDF tree (forward pass in log space), runs the
// adjoint (reverse pass) to get d ln P / d theta for every gradient slot, and
// accumulates -ln P (Neumaier-compensated) and the slot derivatives in double.
// The block reduces its accumulators with wave64 butterflies (bitwise equal on
// every lane) and a fixed-order merge of the four waves, and stores one row of
// partials per tile.  A second kernel sums the rows of each fit in a fixed
// order.  The partials of a tile depend only on the tile's events and the
// constant table, never on the grid size or on other fits in the same launch,
// so a fit gives bit-identical results alone and batched.
//
// Precision: T = double (FP64 path) or float (FP32-eval path).  In the float
// path events are stored as float offsets from a per-column double
// reference; every location difference (x - a, x - mu, m0^2 - s) is formed in
// double from the stored offset and a double constant, then rounded once.
#include <hip/hip_runtime.h>

#include "device_common.h"
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

// DALITZ: ln |1 + sum c_k A_k|^2 ; dl = d/d(Re c_k), d/d(Im c_k)
template <typename T>
__device__ __forceinline__ T leaf_dalitz(const CS& cs, int c0, int R, bool hoisted, double x12, double x13,
                                         T* dl) {
  const double s12 = x12 + cs.d[c0 + kDzRef12];
  const double s13 = x13 + cs.d[c0 + kDzRef13];
  const double s23 = cs.d[c0 + kDzSsum] - s12 - s13;
  Cx<T> A[kMaxRes];
  dalitz_amps<T, false>(cs, c0, R, s12, s13, s23, A, nullptr);
  const int cb = c0 + dz_coef_base(R, false);
  Cx<T> S = {T(1), T(0)};
#pragma unroll
  for (int k = 0; k < kMaxRes; ++k)
    if (k < R) {
      const Cx<T> c = {cs.get<T>(cb + 2 * k), cs.get<T>(cb + 2 * k + 1)};
      const Cx<T> t = cmul(c, A[k]);
      S.re += t.re;
      S.im += t.im;
    }
  const T a2 = S.re * S.re + S.im * S.im;
  const T inv = T(2) * Mth<T>::rcp(a2);
  T lv = a2 > T(0) ? Mth<T>::ln(a2) : T(-INFINITY);
#pragma unroll
  for (int k = 0; k < kMaxRes; ++k)
    if (k < R) {
      // conj(S) A_k
      const T re = S.re * A[k].re + S.im * A[k].im;
      const T im = S.re * A[k].im - S.im * A[k].re;
      dl[2 * k] = re * inv;
      dl[2 * k + 1] = -im * inv;
      if (!hoisted) {
        dl[2 * k] -= cs.get<T>(c0 + kDzDln + 2 * k);
        dl[2 * k + 1] -= cs.get<T>(c0 + kDzDln + 2 * k + 1);
      }
    }
  if (!hoisted) lv = (lv - cs.get<T>(c0 + kDzLnHi)) - cs.get<T>(c0 + kDzLnLo);
  return lv;
}

// TDDP: ln [a_c C + a_0 E0 + a_s S]; dl = coefficient derivatives, then tau, y
template <typename T>
__device__ __forceinline__ T leaf_tddp(const CS& cs, int c0, int R, bool hoisted, double x12, double x13,
                                       double xt, double xs, T* dl) {
  const double s12 = x12 + cs.d[c0 + kDzRef12];
  const double s13 = x13 + cs.d[c0 + kDzRef13];
  const double s23 = cs.d[c0 + kDzSsum] - s12 - s13;
  Cx<T> A[kMaxRes], Ab[kMaxRes];
  dalitz_amps<T, true>(cs, c0, R, s12, s13, s23, A, Ab);
  const int cb = c0 + dz_coef_base(R, true);
  Cx<T> S = {T(1), T(0)}, Sb = {T(1), T(0)};
#pragma unroll
  for (int k = 0; k < kMaxRes; ++k)
    if (k < R) {
      const Cx<T> c = {cs.get<T>(cb + 2 * k), cs.get<T>(cb + 2 * k + 1)};
      const Cx<T> t = cmul(c, A[k]), tb = cmul(c, Ab[k]);
      S.re += t.re; S.im += t.im;
      Sb.re += tb.re; Sb.im += tb.im;
    }
  const T nA = S.re * S.re + S.im * S.im;
  const T nB = Sb.re * Sb.re + Sb.im * Sb.im;
  const T X = S.re * Sb.re + S.im * Sb.im;  // Re(conj(A) Abar)
  const T as = -X;
  // Decay-time factors, formed in double: C - E(1/tau), S and the tau / y
  // derivative combinations are small differences of nearly equal terms
  // (|y| << 1), and rounding them in float would bias every event the same way.
  const double t = xt, s = xs;
  const int tb = c0 + dz_time_base(R);
  const double g = ::exp(-0.5 * t * t / (s * s));
  double Em, dEm, Ep, dEp, E0, dE0;
  econv<double>(t, s, cs.d[tb + kTdGm], g, Em, dEm);
  econv<double>(t, s, cs.d[tb + kTdGp], g, Ep, dEp);
  econv<double>(t, s, cs.d[tb + kTdG], g, E0, dE0);
  const double Cd = 0.5 * (Em + Ep);
  const double Tm = dEm * cs.d[tb + kTdDGmTau], Tp = dEp * cs.d[tb + kTdDGpTau];
  const double T1 = 0.5 * (Tm + Tp), T0 = dE0 * cs.d[tb + kTdDGTau];
  const double Ym = dEm * cs.d[tb + kTdDGmY], Yp = dEp * cs.d[tb + kTdDGpY];
  const T cc = (T)(Cd + E0);          // d R / d(|A|^2 / 2)
  const T cb_ = (T)(Cd - E0);         // d R / d(|Abar|^2 / 2)
  const T St = (T)(0.5 * (Em - Ep));  // S(t)
  const T tA = (T)(T1 + T0), tB = (T)(T1 - T0), tS = (T)(0.5 * (Tm - Tp));
  const T yAB = (T)(0.5 * (Ym + Yp)), yS = (T)(0.5 * (Ym - Yp));
  // rate = a_c C + a_0 E0 + a_s S = |A|^2 (C + E0)/2 + |Abar|^2 (C - E0)/2 + a_s S
  const T Rv = T(0.5) * nA * cc + T(0.5) * nB * cb_ + as * St;
  const T iR = Mth<T>::rcp(Rv);
  T lv = Rv > T(0) ? Mth<T>::ln(Rv) : T(-INFINITY);
#pragma unroll
  for (int k = 0; k < kMaxRes; ++k)
    if (k < R) {
      // re part: dA = A_k, dAb = Ab_k ; im part: dA = i A_k, dAb = i Ab_k
      const T pA_re = S.re * A[k].re + S.im * A[k].im;     // Re(conj(S) A_k)
      const T pA_im = S.re * A[k].im - S.im * A[k].re;     // Im(conj(S) A_k)
      const T pB_re = Sb.re * Ab[k].re + Sb.im * Ab[k].im;
      const T pB_im = Sb.re * Ab[k].im - Sb.im * Ab[k].re;
      const T x1_re = A[k].re * Sb.re + A[k].im * Sb.im;   // Re(conj(A_k) Sb)
      const T x1_im = A[k].re * Sb.im - A[k].im * Sb.re;   // Im(conj(A_k) Sb)
      const T x2_re = S.re * Ab[k].re + S.im * Ab[k].im;   // Re(conj(S) Ab_k)
      const T x2_im = S.re * Ab[k].im - S.im * Ab[k].re;   // Im(conj(S) Ab_k)
      const T dR_re = cc * pA_re + cb_ * pB_re - (x1_re + x2_re) * St;
      const T dR_im = -cc * pA_im - cb_ * pB_im - (x1_im - x2_im) * St;
      dl[2 * k] = dR_re * iR;
      dl[2 * k + 1] = dR_im * iR;
      if (!hoisted) {
        dl[2 * k] -= cs.get<T>(c0 + kDzDln + 2 * k);
        dl[2 * k + 1] -= cs.get<T>(c0 + kDzDln + 2 * k + 1);
      }
    }
  const T dtau = T(0.5) * nA * tA + T(0.5) * nB * tB + as * tS;
  const T dy = T(0.5) * (nA + nB) * yAB + as * yS;
  dl[2 * R] = dtau * iR;
  dl[2 * R + 1] = dy * iR;
  if (!hoisted) {
    dl[2 * R] -= cs.get<T>(c0 + kDzDln + 2 * R);
    dl[2 * R + 1] -= cs.get<T>(c0 + kDzDln + 2 * R + 1);
    lv = (lv - cs.get<T>(c0 + kDzLnHi)) - cs.get<T>(c0 + kDzLnLo);
  }
  return lv;
}

// ------------------------------------------------------------------ accumulation
struct NeuAcc {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
};

// Error-free sum of two values (Knuth): a + b = s + e exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

// Block reduction of one tile: lanes hold (nll_s, nll_c, slot sums); wave64
// butterflies then a fixed-order merge of the 4 waves.  Row layout written to
// `out`: [nll_s, nll_c, slot_0 .. slot_{S-1}].
template <int S>
__device__ __forceinline__ void tile_store(NeuAcc nll, const double* g, int n_slots, double* __restrict__ out) {
  __shared__ double red[4][S + 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = nll.s, c = nll.c;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double os = __shfl_xor(s, off, 64), oc = __shfl_xor(c, off, 64);
    double ns, e;
    two_sum(s, os, ns, e);
    s = ns;
    c = (c + oc) + e;
  }
  double v[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    v[j] = 0.0;
    if (j < n_slots) {
      double x = g[j];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
      v[j] = x;
    }
  }
  if (lane == 0) {
    red[wave][0] = s;
    red[wave][1] = c;
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (j < n_slots) red[wave][2 + j] = v[j];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t == 0) {
    double ss = red[0][0], cc = red[0][1];
    for (int w = 1; w < 4; ++w) {
      double ns, e;
      two_sum(ss, red[w][0], ns, e);
      ss = ns;
      cc = (cc + red[w][1]) + e;
    }
    out[0] = ss;
    out[1] = cc;
  } else if (t < n_slots + 1) {
    const int j = t - 1;
    out[2 + j] = ((red[0][2 + j] + red[1][2 + j]) + red[2][2 + j]) + red[3][2 + j];
  }
  __syncthreads();  // `red` is reused by the next tile of a persistent block
}

// ------------------------------------------------------------------ single-leaf tiles
template <int OP> struct LeafInfo;
template <> struct LeafInfo<OP_EXP> { static constexpr int ncol = 1, nslot = 1; };
template <> struct LeafInfo<OP_GAUSS> { static constexpr int ncol = 1, nslot = 2; };
template <> struct LeafInfo<OP_DALITZ> { static constexpr int ncol = 2, nslot = 2 * kMaxRes; };
template <> struct LeafInfo<OP_TDDP> { static constexpr int ncol = 4, nslot = 2 * kMaxRes + 2; };

template <typename T, int OP, int EPT, bool GRAD>
__device__ __forceinline__ void leaf_tile(const KNode& nd, const CS& cs, const void* const* cols, int64_t n_events,
                                          int64_t tile, int n_slots_all, double* __restrict__ out) {
  const int n_slots = GRAD ? n_slots_all : 0;
  typedef typename Col<T>::S Sx;
  constexpr int NC = LeafInfo<OP>::ncol;
  constexpr int NS = LeafInfo<OP>::nslot;
  const int64_t base = tile * (int64_t)(kBlock * EPT) + threadIdx.x;
  const bool hoisted = nd.hoisted != 0;
  const int c0 = nd.c0;
  const Sx* cp[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) cp[c] = (const Sx*)cols[nd.col[c]];
  // issue every load of the tile before any arithmetic
  Sx xv[NC][EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t i = base + (int64_t)e * kBlock;
#pragma unroll
    for (int c = 0; c < NC; ++c) xv[c][e] = i < n_events ? cp[c][i] : Sx(0);
  }
  double nll = 0.0;  // <= EPT terms per thread: compensation starts at the tile level
  double g[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) g[j] = 0.0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t i = base + (int64_t)e * kBlock;
    if (i < n_events) {
      T dl[NS];
      T lv;
      if (OP == OP_EXP) lv = leaf_exp<T>(cs, c0, hoisted, (double)xv[0][e], dl);
      else if (OP == OP_GAUSS) lv = leaf_gauss<T>(cs, c0, hoisted, (double)xv[0][e], dl);
      else if (OP == OP_DALITZ) lv = leaf_dalitz<T>(cs, c0, nd.aux, hoisted, (double)xv[0][e], (double)xv[1][e], dl);
      else lv = leaf_tddp<T>(cs, c0, nd.aux, hoisted, (double)xv[0][e], (double)xv[1][e], (double)xv[2][e],
                            (double)xv[3][e], dl);
      nll -= (double)lv;
#pragma unroll
      for (int j = 0; j < NS; ++j)
        if (j < n_slots) g[j] += (double)dl[j];
    }
  }
  tile_store<NS>(NeuAcc{nll, 0.0}, g, n_slots, out);
}

// ------------------------------------------------------------------ tree interpreter tiles
// General trees (ADD / PROD over leaves).  Node log-values, adjoints and the
// per-event slot derivatives live in small VGPR arrays indexed by
// wave-uniform node / slot numbers.
template <typename T, int EPT, int NS, int NCOL, bool HEAVY, bool GRAD>
__device__ __forceinline__ void tree_tile(const KProgram& P, const CS& cs, const void* const* cols, int64_t n_events,
                                          int64_t tile, double* __restrict__ out) {
  typedef typename Col<T>::S Sx;
  constexpr int NN = HEAVY ? kMaxNodes : 8;  // node capacity of this instantiation
  const int64_t base = tile * (int64_t)(kBlock * EPT) + threadIdx.x;
  const int n_nodes = P.n_nodes, n_slots = GRAD ? P.n_slots : 0, n_cols = P.n_cols;
  // one event in flight ahead of the one being evaluated
  Sx cur[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c)
    cur[c] = (c < n_cols && base < n_events) ? ((const Sx*)cols[c])[base] : Sx(0);
  double nll = 0.0;
  double g[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) g[j] = 0.0;
  for (int e = 0; e < EPT; ++e) {
    const int64_t i = base + (int64_t)e * kBlock;
    double xe[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) xe[c] = (double)cur[c];
    if (e + 1 < EPT) {
      const int64_t i1 = i + kBlock;
#pragma unroll
      for (int c = 0; c < NCOL; ++c)
        if (c < n_cols) cur[c] = i1 < n_events ? ((const Sx*)cols[c])[i1] : Sx(0);
    }
    if (i >= n_events) break;
    T lv[NN], adj[NN], resp[NN], dl[NS];
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
      } else if (HEAVY && op == OP_DALITZ) {
        T dd[2 * kMaxRes];
        v = leaf_dalitz<T>(cs, c0, nd.aux, h, xe[nd.col[0]], xe[nd.col[1]], dd);
#pragma unroll
        for (int j = 0; j < 2 * kMaxRes; ++j)
          if (j < 2 * nd.aux) dl[s0 + j] = dd[j];
      } else if (HEAVY && op == OP_TDDP) {
        T dd[2 * kMaxRes + 2];
        v = leaf_tddp<T>(cs, c0, nd.aux, h, xe[nd.col[0]], xe[nd.col[1]], xe[nd.col[2]], xe[nd.col[3]], dd);
#pragma unroll
        for (int j = 0; j < 2 * kMaxRes + 2; ++j)
          if (j < 2 * nd.aux + 2) dl[s0 + j] = dd[j];
      } else if (op == OP_PROD) {
        v = T(0);
        for (int j = 0; j < nd.n_child; ++j) {
          const int ch = P.child[nd.child0 + j];
          v += lv[ch];
          resp[ch] = T(1);
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
      if (nd.op == OP_ADD || nd.op == OP_PROD)
        for (int j = 0; j < nd.n_child; ++j) {
          const int ch = P.child[nd.child0 + j];
          adj[ch] = a * resp[ch];
        }
      if (k != root)
        for (int j = 0; j < nd.n_slot; ++j) dl[nd.slot0 + j] = dl[nd.slot0 + j] * a;
    }
    nll -= (double)lv[root];
#pragma unroll
    for (int j = 0; j < NS; ++j)
      if (j < n_slots) g[j] += (double)dl[j];
  }
  tile_store<NS>(NeuAcc{nll, 0.0}, g, n_slots, out);
}

// ------------------------------------------------------------------ mixture tiles
// Root ADD of K single-column EXP / GAUSS leaves (the signal-plus-background
// shape).  Fully static: the child kinds are wave-uniform branches, the
// accumulators have a fixed layout [2 per child, then K-1 fractions] that the
// host maps back to parameters.
template <typename T> struct Split;
template <> struct Split<double> {
  // double path: the location constant is used as is
  double v;
  __device__ __forceinline__ void set(double x) { v = x; }
  __device__ __forceinline__ double add(double x) const { return x + v; }
};
template <> struct Split<float> {
  // float path: the double location constant as a float pair hi + lo, so that
  // (x + hi) + lo rounds like one addition of the double value (its rounding
  // error varies from event to event instead of biasing all of them)
  float hi, lo;
  __device__ __forceinline__ void set(double x) {
    hi = (float)x;
    lo = (float)(x - (double)hi);
  }
  __device__ __forceinline__ float add(float x) const { return (x + hi) + lo; }
};

// Per-event body of a mixture tile.  MASK bit j set: child j is a Gaussian,
// clear: an exponential (static, so no per-event branching on the kinds);
// FULL: every event of the tile exists (no per-event bound checks).
template <typename T, int EPT, int K, int MASK, bool GRAD, bool FULL>
__device__ __forceinline__ void mix_events(const typename Col<T>::S* __restrict__ xp, int64_t base, int64_t n_events,
                                           const Split<T>* loc, const T* k1, const T* lhi, const T* llo, const T* d0c,
                                           const T* d1c, const T* fr, double& nll, T* gt) {
  typedef typename Col<T>::S Sx;
  Sx xv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t i = base + (int64_t)e * kBlock;
    xv[e] = (FULL || i < n_events) ? xp[i] : Sx(0);
  }
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t i = base + (int64_t)e * kBlock;
    if (!FULL && i >= n_events) break;
    const T x = (T)xv[e];
    T lv[K], d0[K], d1[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const T u = loc[j].add(x);
      if ((MASK >> j) & 1) {
        const T z = u * k1[j], zz = z * z;
        lv[j] = (T(-0.5) * zz - lhi[j]) - llo[j];
        d0[j] = z * k1[j] - d0c[j];
        d1[j] = zz * k1[j] - d1c[j];
      } else {
        lv[j] = (k1[j] * u - lhi[j]) - llo[j];
        d0[j] = u - d0c[j];
      }
    }
    T ej[K], m;
    if (K == 2) {
      // the larger term has e = 1: one exponential per event
      const T dd = lv[1] - lv[0];
      const bool up = dd > T(0);
      const T eo = Mth<T>::ex(up ? -dd : dd);
      ej[0] = up ? eo : T(1);
      ej[1] = up ? T(1) : eo;
      m = up ? lv[1] : lv[0];
    } else {
      m = lv[0];
#pragma unroll
      for (int j = 1; j < K; ++j) m = lv[j] > m ? lv[j] : m;
#pragma unroll
      for (int j = 0; j < K; ++j) ej[j] = Mth<T>::ex(lv[j] - m);
    }
    T ssum = fr[0] * ej[0];
#pragma unroll
    for (int j = 1; j < K; ++j) ssum += fr[j] * ej[j];
    const T v = ssum > T(0) ? m + Mth<T>::ln(ssum) : T(-INFINITY);
    nll -= (double)v;
    if (GRAD) {
      const T is = Mth<T>::rcp(ssum);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const T r = fr[j] * ej[j] * is;
        gt[2 * j] += r * d0[j];
        if ((MASK >> j) & 1) gt[2 * j + 1] += r * d1[j];
        if (j < K - 1) gt[2 * K + j] += (ej[j] - ej[K - 1]) * is;
      }
    }
  }
}

template <typename T, int EPT, int K, int MASK, bool GRAD>
__device__ __forceinline__ void mix_tile(const KProgram& P, const CS& cs, const void* const* cols, int64_t n_events,
                                         int64_t tile, double* __restrict__ out) {
  typedef typename Col<T>::S Sx;
  constexpr int NA = 3 * K - 1;
  const int64_t base = tile * (int64_t)(kBlock * EPT) + threadIdx.x;
  // per-child constants, wave-uniform (constant layouts of EXP / GAUSS above)
  const KNode& rn = P.node[P.n_nodes - 1];
  Split<T> loc[K];
  T k1[K], lhi[K], llo[K], d0c[K], d1c[K], fr[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int c0 = P.node[P.child[rn.child0 + j]].c0;
    loc[j].set(cs.d[c0]);
    k1[j] = cs.get<T>(c0 + 1);
    lhi[j] = cs.get<T>(c0 + 2);
    llo[j] = cs.get<T>(c0 + 3);
    d0c[j] = cs.get<T>(c0 + 4);
    d1c[j] = ((MASK >> j) & 1) ? cs.get<T>(c0 + 5) : T(0);
    fr[j] = cs.get<T>(rn.c0 + j);
  }
  const Sx* xp = (const Sx*)cols[0];
  double nll = 0.0;
  T gt[NA];  // per-thread partial sums over this thread's <= EPT events
#pragma unroll
  for (int j = 0; j < NA; ++j) gt[j] = T(0);
  if (tile * (int64_t)(kBlock * EPT) + (int64_t)kBlock * EPT <= n_events)
    mix_events<T, EPT, K, MASK, GRAD, true>(xp, base, n_events, loc, k1, lhi, llo, d0c, d1c, fr, nll, gt);
  else
    mix_events<T, EPT, K, MASK, GRAD, false>(xp, base, n_events, loc, k1, lhi, llo, d0c, d1c, fr, nll, gt);
  double g[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) g[j] = (double)gt[j];
  tile_store<NA>(NeuAcc{nll, 0.0}, g, GRAD ? NA : 0, out);
}

// ------------------------------------------------------------------ reduction
// Second launch: one 1024-thread block per fit sums that fit's tile rows in a
// fixed order.  Wave w of the 16 works on column w % nc (several waves per
// column when there are fewer than 16 columns, each on a fixed contiguous
// slice of the rows); a lane takes rows lane, lane + 64, ... of its slice with
// 16 loads in flight, two-sum compensated; then a wave64 butterfly and a
// fixed-order merge of the slices of each column.  The NLL is the sum of its
// value and compensation columns.  Result: [nll, slot_0 .. slot_{S-1}].
constexpr int kRedBlock = 1024;
constexpr int kRedWaves = kRedBlock / 64;
constexpr int kMaxRedCols = kMaxSlots + 2;

__device__ __forceinline__ void reduce_fit(const FitRec& fr, int stride, int n_slots) {
  const int nc = n_slots + 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int per_col = nc >= kRedWaves ? 1 : kRedWaves / nc;  // waves per column
  __shared__ double part[kRedWaves][2];
  __shared__ double colsum[kMaxRedCols][kRedWaves][2];
  __shared__ double nll_parts[2];
  // column pass: wave w handles (column, slice) pairs w, w + 16, ...
  for (int task = wave; task < nc * per_col; task += kRedWaves) {
    const int col = task / per_col, slice = task % per_col;
    const int r_begin = (int)((int64_t)fr.n_tiles * slice / per_col);
    const int r_end = (int)((int64_t)fr.n_tiles * (slice + 1) / per_col);
    double s = 0.0, c = 0.0;
    for (int r0 = r_begin; r0 < r_end; r0 += 64 * 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int r = r0 + u * 64 + lane;
        v[u] = r < r_end ? fr.partials[(int64_t)r * stride + col] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        double ns, e;
        two_sum(s, v[u], ns, e);
        s = ns;
        c += e;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double os = __shfl_xor(s, off, 64), oc = __shfl_xor(c, off, 64);
      double ns, e;
      two_sum(s, os, ns, e);
      s = ns;
      c = (c + oc) + e;
    }
    if (lane == 0) {
      colsum[col][slice][0] = s;
      colsum[col][slice][1] = c;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < nc) {
    double s = colsum[t][0][0], c = colsum[t][0][1];
    for (int k = 1; k < per_col; ++k) {
      double ns, e;
      two_sum(s, colsum[t][k][0], ns, e);
      s = ns;
      c = (c + colsum[t][k][1]) + e;
    }
    if (t < 2) nll_parts[t] = s + c;
    else fr.result[t - 1] = s + c;
  }
  __syncthreads();
  if (t == 0) fr.result[0] = nll_parts[0] + nll_parts[1];
  (void)part;
}

__global__ __launch_bounds__(kRedBlock) void k_reduce(const FitRec* __restrict__ fits, int n_fits_max) {
  const FitRec& fr = fits[blockIdx.x];
  if (!fr.active) return;
  reduce_fit(fr, fr.stride, fr.n_slots);
}

__global__ __launch_bounds__(kRedBlock) void k_reduce_one(const FitRec fr) { reduce_fit(fr, fr.stride, fr.n_slots); }

// ------------------------------------------------------------------ kernels
template <typename T, int OP, int EPT, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_leaf(const EvalArgs a) {
  const CS cs{a.prog.c64, a.prog.c32};
  leaf_tile<T, OP, EPT, GRAD>(a.prog.node[0], cs, a.col, a.n_events, blockIdx.x, a.prog.n_slots,
                        a.partials + (int64_t)blockIdx.x * a.stride);
}

template <typename T, int EPT, int NS, int NCOL, bool HEAVY, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_tree(const EvalArgs a) {
  const CS cs{a.prog.c64, a.prog.c32};
  tree_tile<T, EPT, NS, NCOL, HEAVY, GRAD>(a.prog, cs, a.col, a.n_events, blockIdx.x,
                              a.partials + (int64_t)blockIdx.x * a.stride);
}

template <typename T, int EPT, int K, int MASK, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_mix(const EvalArgs a) {
  const CS cs{a.prog.c64, a.prog.c32};
  mix_tile<T, EPT, K, MASK, GRAD>(a.prog, cs, a.col, a.n_events, blockIdx.x,
                                  a.partials + (int64_t)blockIdx.x * a.stride);
}

// Batched: the program structure is shared (kernel argument); constants,
// columns and partials are per fit.  Each block walks a contiguous range of
// global tiles; fits own contiguous tile ranges in fit order.
struct BatchArgs {
  KProgram prog;               // structure only (constants unused)
  const BatchHeader* hdr;      // counts, then the FitRec array
  const double* c64;           // [fit][n_const]
  const float* c32;
  int32_t n_const;
};

__device__ __forceinline__ int find_fit(const FitRec* fits, int n_fits, int gtile) {
  int lo = 0, hi = n_fits - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fits[mid].tile_begin <= gtile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, int OP, int EPT>
__global__ __launch_bounds__(kBlock) void k_leaf_batched(const BatchArgs a) {  // always with gradient
  const int tpb = a.hdr->tiles_per_block, total = a.hdr->total_tiles, n_fits = a.hdr->n_fits;
  const FitRec* fits = (const FitRec*)(a.hdr + 1);
  const int g0 = blockIdx.x * tpb;
  const int g1 = min(g0 + tpb, total);
  if (g0 >= g1) return;
  int f = find_fit(fits, n_fits, g0);
  for (int gt = g0; gt < g1; ++gt) {
    while (gt >= fits[f].tile_begin + fits[f].n_tiles) ++f;
    const FitRec& fr = fits[f];
    const CS cs{a.c64 + (int64_t)f * a.n_const, a.c32 + (int64_t)f * a.n_const};
    const int64_t lt = gt - fr.tile_begin;
    leaf_tile<T, OP, EPT, true>(a.prog.node[0], cs, fr.col, fr.n_events, lt, a.prog.n_slots,
                          fr.partials + lt * (a.prog.n_slots + 2));
  }
}

template <typename T, int EPT, int K, int MASK>
__global__ __launch_bounds__(kBlock) void k_mix_batched(const BatchArgs a) {
  const int tpb = a.hdr->tiles_per_block, total = a.hdr->total_tiles, n_fits = a.hdr->n_fits;
  const FitRec* fits = (const FitRec*)(a.hdr + 1);
  const int g0 = blockIdx.x * tpb;
  const int g1 = min(g0 + tpb, total);
  if (g0 >= g1) return;
  int f = find_fit(fits, n_fits, g0);
  for (int gt = g0; gt < g1; ++gt) {
    while (gt >= fits[f].tile_begin + fits[f].n_tiles) ++f;
    const FitRec& fr = fits[f];
    const CS cs{a.c64 + (int64_t)f * a.n_const, a.c32 + (int64_t)f * a.n_const};
    const int64_t lt = gt - fr.tile_begin;
    mix_tile<T, EPT, K, MASK, true>(a.prog, cs, fr.col, fr.n_events, lt, fr.partials + lt * (a.prog.n_slots + 2));
  }
}

template <typename T, int EPT, int NS, int NCOL, bool HEAVY>
__global__ __launch_bounds__(kBlock) void k_tree_batched(const BatchArgs a) {
  const int tpb = a.hdr->tiles_per_block, total = a.hdr->total_tiles, n_fits = a.hdr->n_fits;
  const FitRec* fits = (const FitRec*)(a.hdr + 1);
  const int g0 = blockIdx.x * tpb;
  const int g1 = min(g0 + tpb, total);
  if (g0 >= g1) return;
  int f = find_fit(fits, n_fits, g0);
  for (int gt = g0; gt < g1; ++gt) {
    while (gt >= fits[f].tile_begin + fits[f].n_tiles) ++f;
    const FitRec& fr = fits[f];
    const CS cs{a.c64 + (int64_t)f * a.n_const, a.c32 + (int64_t)f * a.n_const};
    const int64_t lt = gt - fr.tile_begin;
    tree_tile<T, EPT, NS, NCOL, HEAVY, true>(a.prog, cs, fr.col, fr.n_events, lt, fr.partials + lt * (a.prog.n_slots + 2));
  }
}

// ------------------------------------------------------------------ dispatch
template <typename T, int EPT, bool GRAD>
static hipError_t launch_light(int kind, const EvalArgs& a, int64_t n_tiles, hipStream_t st) {
  const dim3 grid((unsigned)n_tiles), block(kBlock);
  switch (kind) {
    case KIND_EXP: hipLaunchKernelGGL((k_leaf<T, OP_EXP, EPT, GRAD>), grid, block, 0, st, a); break;
    case KIND_GAUSS: hipLaunchKernelGGL((k_leaf<T, OP_GAUSS, EPT, GRAD>), grid, block, 0, st, a); break;
    case KIND_TREE_SMALL: hipLaunchKernelGGL((k_tree<T, EPT, 8, 2, false, GRAD>), grid, block, 0, st, a); break;
#define HF_MIX(K_, M_)                                                                              \
  case (K_ == 2 ? KIND_MIX2 : KIND_MIX3) + M_:                                                      \
    hipLaunchKernelGGL((k_mix<T, EPT, K_, M_, GRAD>), grid, block, 0, st, a);                       \
    break;
    HF_MIX(2, 0) HF_MIX(2, 1) HF_MIX(2, 2) HF_MIX(2, 3)
    HF_MIX(3, 0) HF_MIX(3, 1) HF_MIX(3, 2) HF_MIX(3, 3) HF_MIX(3, 4) HF_MIX(3, 5) HF_MIX(3, 6) HF_MIX(3, 7)
#undef HF_MIX
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int EPT, bool GRAD>
static hipError_t launch_heavy(int kind, const EvalArgs& a, int64_t n_tiles, hipStream_t st) {
  const dim3 grid((unsigned)n_tiles), block(kBlock);
  switch (kind) {
    case KIND_DALITZ: hipLaunchKernelGGL((k_leaf<T, OP_DALITZ, EPT, GRAD>), grid, block, 0, st, a); break;
    case KIND_TDDP: hipLaunchKernelGGL((k_leaf<T, OP_TDDP, EPT, GRAD>), grid, block, 0, st, a); break;
    case KIND_TREE: hipLaunchKernelGGL((k_tree<T, EPT, kMaxSlots, kMaxCols, true, GRAD>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, bool GRAD>
static hipError_t launch_any(int kind, const EvalArgs& a, int64_t n_tiles, hipStream_t st) {
  if (kind_ept(kind) == kEptLight) return launch_light<T, kEptLight, GRAD>(kind, a, n_tiles, st);
  return launch_heavy<T, kEptHeavy, GRAD>(kind, a, n_tiles, st);
}

int kind_ept(int kind) {
  if (kind >= KIND_MIX2) return kEptLight;
  switch (kind) {
    case KIND_EXP: case KIND_GAUSS: case KIND_TREE_SMALL: return kEptLight;
    default: return kEptHeavy;
  }
}

hipError_t launch_eval(int kind, bool fp32, bool grad, const EvalArgs& a, int64_t n_tiles, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (fp32) return grad ? launch_any<float, true>(kind, a, n_tiles, st) : launch_any<float, false>(kind, a, n_tiles, st);
  return grad ? launch_any<double, true>(kind, a, n_tiles, st) : launch_any<double, false>(kind, a, n_tiles, st);
}

template <typename T, int EPT>
static hipError_t launch_b_light(int kind, const BatchArgs& a, int grid, hipStream_t st) {
  switch (kind) {
    case KIND_EXP: hipLaunchKernelGGL((k_leaf_batched<T, OP_EXP, EPT>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case KIND_GAUSS: hipLaunchKernelGGL((k_leaf_batched<T, OP_GAUSS, EPT>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case KIND_TREE_SMALL: hipLaunchKernelGGL((k_tree_batched<T, EPT, 8, 2, false>), dim3(grid), dim3(kBlock), 0, st, a); break;
#define HF_MIX(K_, M_)                                                                              \
  case (K_ == 2 ? KIND_MIX2 : KIND_MIX3) + M_:                                                      \
    hipLaunchKernelGGL((k_mix_batched<T, EPT, K_, M_>), dim3(grid), dim3(kBlock), 0, st, a);        \
    break;
    HF_MIX(2, 0) HF_MIX(2, 1) HF_MIX(2, 2) HF_MIX(2, 3)
    HF_MIX(3, 0) HF_MIX(3, 1) HF_MIX(3, 2) HF_MIX(3, 3) HF_MIX(3, 4) HF_MIX(3, 5) HF_MIX(3, 6) HF_MIX(3, 7)
#undef HF_MIX
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <typename T, int EPT>
static hipError_t launch_b_heavy(int kind, const BatchArgs& a, int grid, hipStream_t st) {
  switch (kind) {
    case KIND_DALITZ: hipLaunchKernelGGL((k_leaf_batched<T, OP_DALITZ, EPT>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case KIND_TDDP: hipLaunchKernelGGL((k_leaf_batched<T, OP_TDDP, EPT>), dim3(grid), dim3(kBlock), 0, st, a); break;
    case KIND_TREE: hipLaunchKernelGGL((k_tree_batched<T, EPT, kMaxSlots, kMaxCols, true>), dim3(grid), dim3(kBlock), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_eval_batched(int kind, bool fp32, const KProgram& prog, const BatchHeader* hdr_dev, const double* c64,
                               const float* c32, int n_const, int grid, hipStream_t st) {
  BatchArgs a;
  a.prog = prog;
  a.hdr = hdr_dev;
  a.c64 = c64;
  a.c32 = c32;
  a.n_const = n_const;
  if (kind_ept(kind) == kEptLight)
    return fp32 ? launch_b_light<float, kEptLight>(kind, a, grid, st) : launch_b_light<double, kEptLight>(kind, a, grid, st);
  return fp32 ? launch_b_heavy<float, kEptHeavy>(kind, a, grid, st) : launch_b_heavy<double, kEptHeavy>(kind, a, grid, st);
}

hipError_t launch_reduce_one(const FitRec& fr, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(kRedBlock), 0, st, fr);
  return hipGetLastError();
}

hipError_t launch_reduce(const FitRec* fits_dev, int n_fits, hipStream_t st) {
  if (n_fits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(n_fits), dim3(kRedBlock), 0, st, fits_dev, n_fits);
  return hipGetLastError();
}

}  // namespace hf
