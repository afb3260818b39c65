// Reference oracle for the unbinned maximum-likelihood hot path.
//
// TEST INFRASTRUCTURE ONLY.  Plain, slow, double-precision CPU code that
// states what the GPU library must compute; only the test suite, the smoke
// check and the benchmark's CPU-baseline leg may load it.  It shares no code,
// header or table with the GPU library.
//
// What it computes (GooFit paper: sections "GooFit code", "Combining
// functions", "Adding new PDFs", "Results"):
//   * a tree of PDF nodes over observables held in a box (the Variable
//     (name, lo, hi) form of the first listing), each node a normalised
//     density P(x; theta) over that box;
//   * the negative log-likelihood NLL = -sum_i ln P_root(x_i; theta) (the
//     maximum-likelihood "metric" of the FitManager section), and its exact
//     gradient with respect to every parameter.
// Every sum over events is a Neumaier-compensated double sum.
//
// Node definitions (each P is normalised over the node's observables):
//   EXP    P = e^{alpha x} / int_a^b e^{alpha x} dx                     (listing 1)
//   GAUSS  P = exp(-(x-mu)^2/(2 sigma^2)) / int_a^b (same) dx          (listing 3)
//   POLY   P = sum_k a_k (x-x0)^k / int (same), a_0 = 1 fixed
//   ADD    P = sum_{j<K} f_j P_j + (1 - sum f_j) P_K                    ("Combining functions")
//   PROD   P = prod_j P_j over disjoint observables                     (listing 2);
//          one-observable EXP / GAUSS / POLY children may share an
//          observable: each such group is renormalised by the integral of
//          its product over the box (numerical, composite Gauss-Legendre)
//   MAP    P(x) = P_j(x) / Z for x in the j-th of K consecutive ranges of the
//          box ([lo, b_1), [b_1, b_2), ..., [b_{K-1}, hi]), children P_j
//          one-observable EXP / GAUSS / POLY leaves normalised over the box,
//          Z = sum_j int_{range j} P_j dx                  ("Combining functions": MappedPdf)
//   DALITZ P = |1 + sum_k c_k A_k(s12, s13)|^2 / N_A, with A_k relativistic
//          Breit-Wigner x Blatt-Weisskopf x Zemach amplitudes and N_A the
//          midpoint sum over a G x G grid of the Dalitz box ("Results": the
//          Dalitz-plot amplitude sum)
//   TDDP   P = [a_c C(t) + a_0 E(t;1/tau) + a_s S(t)] / N_T, the x = 0 mixing
//          rate convolved with a per-event Gaussian resolution ("Results":
//          hyperbolic time terms convolved with Gaussian resolution); with
//          the mixing parameter x the trigonometric terms enter too:
//          P = [a_c C(t) + a_0 Cz(t) + a_s S(t) + b_s Sz(t)] / N_T, Cz / Sz the
//          resolution-convolved e^{-t/tau} cos(x t/tau) / sin(x t/tau),
//          b_s = -Im(conj(A) Abar); the full model of the mixing fit adds
//          complex q/p (Abar -> (q/p) Abar, the amplitude mixed in from the
//          conjugate state) and resonance masses and widths as parameters,
//          whose normalisation is then the grid sum of the time-integrated
//          rate taken at the current parameters ("Results": the ~40-parameter
//          time-dependent fit with 16 complex amplitudes)
//   DPMAP  P(u | s12, s13) = P_c(u): the Dalitz box cut into an n12 x n13
//          grid of rectangles (inner boundaries b12, b13; a boundary belongs
//          to the cell above it), cell c = i12 n13 + i13 taking its own
//          one-observable EXP / GAUSS / POLY leaf on u, normalised over u's
//          box ("Results": the decay-time uncertainty's distribution varies
//          across the Dalitz plot).  A density of u conditional on the plot
//          position; in a PROD with the DALITZ / TDDP node on (s12, s13) it
//          completes the joint density (u may be the TDDP's sigma_t, on
//          which that node is conditional).
//   CONV   numerical convolution of a model M with a resolution R (section
//          "Combining functions": ConvolutionPdf), both one-observable EXP /
//          GAUSS / POLY leaves on x taken as unnormalised shapes f_M, f_R,
//          or ADDs of such leaves (mixtures of the leaves, each normalised
//          over the child's domain: the box for the model, [d_lo, d_hi] for
//          the resolution):
//          P(x) = sum_k f_M(t_k) f_R(x - t_k) / Z over the N midpoints t_k of
//          x's box, the residual x - t_k restricted to [d_lo, d_hi], and
//          Z = sum_k f_M(t_k) int_box f_R(x - t_k) dx (closed forms)
//   COMP   function composition f(g(x)) (section "Combining functions":
//          CompositePdf): g a POLY leaf's value 1 + sum a_j (x - x0)^j, f an
//          EXP / GAUSS / POLY leaf's unnormalised shape evaluated at g,
//          P(x) = f(g(x)) / Z, Z = int_box f(g(x)) dx (numerical, composite
//          Gauss-Legendre)
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cplx;

namespace {

const double kPi = 3.14159265358979323846;

enum Kind { K_EXP = 1, K_GAUSS = 2, K_POLY = 3, K_ADD = 4, K_PROD = 5, K_DALITZ = 6, K_TDDP = 7, K_MAP = 8,
            K_DPMAP = 9, K_CONV = 10, K_COMP = 11 };

// ---------------------------------------------------------------- sums
struct Neumaier {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// ---------------------------------------------------------------- special functions
// erfcx(x) = exp(x^2) erfc(x) for x >= 0.  Below 5 the product form is used;
// above, the classical continued fraction
//   erfc(x) = exp(-x^2)/sqrt(pi) * 1/(x + (1/2)/(x + (2/2)/(x + (3/2)/(x + ...))))
// evaluated from a fixed depth.
double erfcx_pos(double x) {
  if (x < 5.0) return std::exp(x * x) * std::erfc(x);
  double t = x;
  for (int n = 80; n >= 1; --n) t = x + (0.5 * n) / t;
  return 1.0 / (std::sqrt(kPi) * t);
}

// Gaussian-resolution convolution of the unit exponential decay:
//   E(t; G, s) = int_0^inf G0(t') N(t - t'; 0, s) dt',  G0(t') = e^{-G t'}
//             = 1/2 exp(G^2 s^2 / 2 - G t) erfc(w),  w = (G s^2 - t)/(sqrt2 s).
// For w > 0 the equivalent 1/2 exp(-t^2/(2 s^2)) erfcx(w) avoids overflow.
double econv(double t, double G, double s) {
  double w = (G * s * s - t) / (std::sqrt(2.0) * s);
  if (w > 0.0) return 0.5 * std::exp(-t * t / (2.0 * s * s)) * erfcx_pos(w);
  return 0.5 * std::exp(0.5 * G * G * s * s - G * t) * std::erfc(w);
}
// dE/dG = (G s^2 - t) E - s/sqrt(2 pi) exp(-t^2/(2 s^2))
double econv_dG(double t, double G, double s) {
  return (G * s * s - t) * econv(t, G, s) - s / std::sqrt(2.0 * kPi) * std::exp(-t * t / (2.0 * s * s));
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on the
// Legendre polynomial P_n from the usual starting guesses.
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-15) break;
    }
    x[i] = -z; x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// Gaussian-resolution convolution of the oscillating decay, straight from its
// definition:
//   Cz(t) + i Sz(t) = int_0^inf e^{-G u} e^{i w u} N(t - u; 0, s) du
// (Cz convolves e^{-G u} cos(w u), Sz e^{-G u} sin(w u)), and the derivatives
// of both with respect to G and w, by 16-point Gauss-Legendre quadrature on
// segments of width <= s over the window where the Gaussian exceeds e^{-72}
// of its peak.  out = {Cz, Sz, dCz/dG, dSz/dG, dCz/dw, dSz/dw}.
void econv_osc(double t, double G, double w, double s, double* out) {
  struct GL16 { double x[16], w[16]; };
  static const GL16 gl = [] { GL16 g; gauss_legendre(16, g.x, g.w); return g; }();
  const double* gx = gl.x;
  const double* gw = gl.w;
  const double u0 = std::max(0.0, t - 12.0 * s), u1 = std::max(0.0, t) + 12.0 * s;
  const int nseg = std::max(1, (int)std::ceil((u1 - u0) / s));
  const double h = (u1 - u0) / nseg, norm = 1.0 / (std::sqrt(2.0 * kPi) * s);
  Neumaier acc[6];
  for (int k = 0; k < nseg; ++k) {
    const double a = u0 + k * h;
    for (int i = 0; i < 16; ++i) {
      const double u = a + 0.5 * h * (gx[i] + 1.0);
      const double f = 0.5 * h * gw[i] * norm * std::exp(-G * u - (t - u) * (t - u) / (2.0 * s * s));
      const double c = std::cos(w * u), sn = std::sin(w * u);
      acc[0].add(f * c);
      acc[1].add(f * sn);
      acc[2].add(-u * f * c);
      acc[3].add(-u * f * sn);
      acc[4].add(-u * f * sn);
      acc[5].add(u * f * c);
    }
  }
  for (int j = 0; j < 6; ++j) out[j] = acc[j].value();
}

// phi(z) = (e^z - 1)/z, so int_a^b e^{alpha (x-a)} dx = L phi(alpha L).
double phi(double z) { return z == 0.0 ? 1.0 : std::expm1(z) / z; }
// psi(z) = 1/(1 - e^{-z}) - 1/z ; series 1/2 + z/12 - z^3/720 + z^5/30240 near 0.
double psi(double z) {
  if (std::fabs(z) < 1e-2) {
    double z2 = z * z;
    return 0.5 + z / 12.0 - z * z2 / 720.0 + z * z2 * z2 / 30240.0;
  }
  return 1.0 / (-std::expm1(-z)) - 1.0 / z;
}

// ---------------------------------------------------------------- Dalitz kinematics
// p_m0 / p_g0: the parameters holding the mass and width when they float
// (-1: fixed at m0 / g0)
struct Res { int ch; double m0, g0; int J; int p_re, p_im; int p_m0 = -1, p_g0 = -1; };

struct DalitzDef {
  double M, m1, m2, m3, r;
  int grid;
  std::vector<Res> res;
  // grid integrals: I[j][k] = sum conj(A_j) A_k h^2 ; Ib the same with swapped
  // amplitudes; J[j][k] = sum conj(A_j) Abar_k h^2.  Index 0 is the constant.
  std::vector<cplx> I, Ib, Jx;
  int n_amp() const { return (int)res.size() + 1; }
};

double kallen(double a, double b, double c) { return a * a + b * b + c * c - 2 * a * b - 2 * a * c - 2 * b * c; }

// Membership of (s_1x, s_1y) where x is the partner of particle 1 and y the
// bachelor: s_1x in [(m1+mx)^2, (M-my)^2] and s_1y inside the kinematic
// limits at that s_1x (inclusive).
bool inside_pair(const DalitzDef& d, double s1x, double s1y, double mx, double my) {
  double lo = (d.m1 + mx) * (d.m1 + mx), hi = (d.M - my) * (d.M - my);
  if (!(s1x >= lo && s1x <= hi)) return false;
  double rs = std::sqrt(s1x);
  double E1 = (s1x - mx * mx + d.m1 * d.m1) / (2.0 * rs);
  double Ey = (d.M * d.M - s1x - my * my) / (2.0 * rs);
  double p1 = std::sqrt(std::fmax(E1 * E1 - d.m1 * d.m1, 0.0));
  double py = std::sqrt(std::fmax(Ey * Ey - my * my, 0.0));
  double e = E1 + Ey;
  double smin = e * e - (p1 + py) * (p1 + py);
  double smax = e * e - (p1 - py) * (p1 - py);
  return s1y >= smin && s1y <= smax;
}
// A point is in the Dalitz plot when both orderings agree (keeps the
// accepted set exactly symmetric under s12 <-> s13 when m2 = m3).
bool inside(const DalitzDef& d, double s12, double s13) {
  return inside_pair(d, s12, s13, d.m2, d.m3) && inside_pair(d, s13, s12, d.m3, d.m2);
}

// Amplitude of one resonance, B_J(q) * Z_J * BW(s_AB), at mass m0 and
// width g0.  `parts`, when given, receives {Gamma(s), B_J(q), Z_J, Re BW,
// Im BW}; d_m0 / d_g0, when given, the derivatives of the amplitude in m0
// and g0 (the floating-shape parameters of the full time-dependent fit,
// section "Results"), written out from the same formulas:
//   m0 Gamma(s) = W = g0 m0^2 q^{2J+1} P_J(z0) / (q0^{2J+1} sqrt(s) P_J(z)),
//   BW = 1 / D, D = m0^2 - s - i W, B_J = sqrt(P_J(z0) / P_J(z)),
// with z = r^2 q^2, z0 = r^2 q0^2, P_0 = 1, P_1 = 1 + z, P_2 = z^2 + 3z + 9
// and q0^2 = lambda(m0^2, mA^2, mB^2) / (4 m0^2).
cplx res_amp_mg(const DalitzDef& d, const Res& R, double m0, double g0, double s12, double s13, cplx* d_m0,
                cplx* d_g0, double* parts = nullptr) {
  const double M2 = d.M * d.M;
  double s23 = M2 + d.m1 * d.m1 + d.m2 * d.m2 + d.m3 * d.m3 - s12 - s13;
  double sAB, sAC, sBC, mA, mB, mC;
  if (R.ch == 23) { sAB = s23; sAC = s12; sBC = s13; mA = d.m2; mB = d.m3; mC = d.m1; }
  else if (R.ch == 12) { sAB = s12; sAC = s13; sBC = s23; mA = d.m1; mB = d.m2; mC = d.m3; }
  else { sAB = s13; sAC = s12; sBC = s23; mA = d.m1; mB = d.m3; mC = d.m2; }
  double mA2 = mA * mA, mB2 = mB * mB, mC2 = mC * mC;
  double m02 = m0 * m0;
  double lam0 = kallen(m02, mA2, mB2);
  double q = std::sqrt(std::fmax(kallen(sAB, mA2, mB2), 0.0) / (4.0 * sAB));
  double q0 = std::sqrt(std::fmax(lam0, 0.0) / (4.0 * m02));
  double z = (q * d.r) * (q * d.r), z0 = (q0 * d.r) * (q0 * d.r);
  double PJ = 1.0, PJ0 = 1.0, dPJ0 = 0.0;  // P_J(z), P_J(z0), P_J'(z0)
  if (R.J == 1) { PJ = 1.0 + z; PJ0 = 1.0 + z0; dPJ0 = 1.0; }
  else if (R.J == 2) { PJ = z * z + 3.0 * z + 9.0; PJ0 = z0 * z0 + 3.0 * z0 + 9.0; dPJ0 = 2.0 * z0 + 3.0; }
  double B2 = PJ0 / PJ;
  double width = g0 * std::pow(q / q0, 2 * R.J + 1) * (m0 / std::sqrt(sAB)) * B2;
  cplx bw = 1.0 / cplx(m02 - sAB, -m0 * width);
  double Z = 1.0;
  if (R.J >= 1) {
    double z1 = sAC - sBC + (M2 - mC2) * (mB2 - mA2) / sAB;
    Z = z1;
    if (R.J == 2) {
      double ta = sAB - 2.0 * M2 - 2.0 * mC2 + (M2 - mC2) * (M2 - mC2) / sAB;
      double tb = sAB - 2.0 * mA2 - 2.0 * mB2 + (mA2 - mB2) * (mA2 - mB2) / sAB;
      Z = z1 * z1 - ta * tb / 3.0;
    }
  }
  if (parts) { parts[0] = width; parts[1] = std::sqrt(B2); parts[2] = Z; parts[3] = bw.real(); parts[4] = bw.imag(); }
  const cplx A = std::sqrt(B2) * Z * bw;
  if (d_m0 || d_g0) {
    const double W = m0 * width;
    const cplx bw2 = bw * bw;  // dBW = -BW^2 dD
    // W is proportional to g0: dD/dg0 = -i W / g0
    if (d_g0) *d_g0 = std::sqrt(B2) * Z * (-bw2) * cplx(0.0, -W / g0);
    if (d_m0) {
      // m0 enters through m0^2 in D and W, q0 in W and z0 in W and B_J
      const double dq02 = ((2.0 * m02 - 2.0 * mA2 - 2.0 * mB2) / (4.0 * m02) - lam0 / (4.0 * m02 * m02)) * 2.0 * m0;
      const double dlnP0 = dPJ0 / PJ0 * d.r * d.r * dq02;
      const double dlnW = 2.0 / m0 - 0.5 * (2 * R.J + 1) * dq02 / (q0 * q0) + dlnP0;
      const cplx dD(2.0 * m0, -W * dlnW);
      *d_m0 = A * (0.5 * dlnP0) + std::sqrt(B2) * Z * (-bw2) * dD;
    }
  }
  return A;
}

cplx res_amp(const DalitzDef& d, const Res& R, double s12, double s13, double* parts = nullptr) {
  return res_amp_mg(d, R, R.m0, R.g0, s12, s13, nullptr, nullptr, parts);
}

// amps[0] = 1 (constant term), amps[k] = A_k.
void amplitudes(const DalitzDef& d, double s12, double s13, cplx* amps) {
  amps[0] = cplx(1.0, 0.0);
  for (size_t k = 0; k < d.res.size(); ++k) amps[k + 1] = res_amp(d, d.res[k], s12, s13);
}

// The same at theta (floating masses and widths taken from it); dm / dg
// (nullable) receive dA_k/dm0_k and dA_k/dg0_k at [k] (0 for the constant
// term and for fixed shapes).
void amplitudes_th(const DalitzDef& d, const double* th, double s12, double s13, cplx* amps, cplx* dm, cplx* dg) {
  amps[0] = cplx(1.0, 0.0);
  if (dm) dm[0] = 0.0;
  if (dg) dg[0] = 0.0;
  for (size_t k = 0; k < d.res.size(); ++k) {
    const Res& R = d.res[k];
    const bool fl = R.p_m0 >= 0;
    const double m0 = fl ? th[R.p_m0] : R.m0, g0 = fl ? th[R.p_g0] : R.g0;
    cplx a_m = 0.0, a_g = 0.0;
    amps[k + 1] = res_amp_mg(d, R, m0, g0, s12, s13, fl && dm ? &a_m : nullptr, fl && dg ? &a_g : nullptr);
    if (dm) dm[k + 1] = a_m;
    if (dg) dg[k + 1] = a_g;
  }
}

bool floating_shapes(const DalitzDef& d) {
  for (const Res& R : d.res)
    if (R.p_m0 >= 0) return true;
  return false;
}

void build_grid(DalitzDef& d) {
  const int na = d.n_amp();
  d.I.assign(na * na, 0.0);
  d.Ib.assign(na * na, 0.0);
  d.Jx.assign(na * na, 0.0);
  const double lo12 = (d.m1 + d.m2) * (d.m1 + d.m2), hi12 = (d.M - d.m3) * (d.M - d.m3);
  const double lo13 = (d.m1 + d.m3) * (d.m1 + d.m3), hi13 = (d.M - d.m2) * (d.M - d.m2);
  const double h12 = (hi12 - lo12) / d.grid, h13 = (hi13 - lo13) / d.grid;
  const double area = h12 * h13;
  std::vector<cplx> a(na), ab(na);
  // plain row-by-row sum; a Neumaier sum per matrix element and component
  std::vector<Neumaier> sI(2 * na * na), sIb(2 * na * na), sJ(2 * na * na);
  for (int i = 0; i < d.grid; ++i) {
    double s12 = lo12 + (i + 0.5) * h12;
    for (int j = 0; j < d.grid; ++j) {
      double s13 = lo13 + (j + 0.5) * h13;
      if (!inside(d, s12, s13)) continue;
      amplitudes(d, s12, s13, a.data());
      amplitudes(d, s13, s12, ab.data());
      for (int p = 0; p < na; ++p)
        for (int q = 0; q < na; ++q) {
          cplx v = std::conj(a[p]) * a[q], vb = std::conj(ab[p]) * ab[q], vj = std::conj(a[p]) * ab[q];
          int o = 2 * (p * na + q);
          sI[o].add(v.real()); sI[o + 1].add(v.imag());
          sIb[o].add(vb.real()); sIb[o + 1].add(vb.imag());
          sJ[o].add(vj.real()); sJ[o + 1].add(vj.imag());
        }
    }
  }
  for (int e = 0; e < na * na; ++e) {
    d.I[e] = cplx(sI[2 * e].value(), sI[2 * e + 1].value()) * area;
    d.Ib[e] = cplx(sIb[2 * e].value(), sIb[2 * e + 1].value()) * area;
    d.Jx[e] = cplx(sJ[2 * e].value(), sJ[2 * e + 1].value()) * area;
  }
}

// ---------------------------------------------------------------- model
struct Node {
  int kind = 0;
  std::vector<int> child;   // ADD, PROD
  std::vector<int> obs;     // observable columns
  std::vector<int> par;     // EXP: alpha; GAUSS: mu, sigma; POLY: a1..ad; ADD: fractions
  double x0 = 0.0;          // POLY expansion point
  std::vector<double> bounds;  // MAP: the K-1 inner range boundaries; DPMAP: b12
  std::vector<double> bounds2; // DPMAP: b13
  int grid = 0;                // CONV: number of grid points
  double d_lo = 0.0, d_hi = 0.0;  // CONV: residual range
  DalitzDef* dz = nullptr;  // DALITZ, TDDP
  int p_tau = -1, p_y = -1; // TDDP
  int p_x = -1;             // TDDP with the trigonometric terms (x free)
  int p_qm = -1, p_qa = -1; // TDDP with complex q/p = |q/p| e^{i phi}: |q/p|, phi
};

struct Model {
  int n_obs = 0, n_par = 0, root = -1;
  bool direct_norm = false;  // TDDP: the grid sum at theta even with fixed shapes (tests)
  std::vector<double> lo, hi;
  std::vector<Node> nodes;
  ~Model() { for (auto& n : nodes) delete n.dz; }
};

// Per-call normalisation of each node (depends on theta only).
struct NodeNorm { double lnN = 0.0; std::vector<double> dlnN; };

// complex coefficient vector c (c_0 = 1) and its derivative map
void coeffs(const DalitzDef& d, const double* th, std::vector<cplx>& c) {
  c.assign(d.n_amp(), cplx(1.0, 0.0));
  for (size_t k = 0; k < d.res.size(); ++k) c[k + 1] = cplx(th[d.res[k].p_re], th[d.res[k].p_im]);
}

// c^H M c and its derivatives with respect to re/im of c_k (k >= 1).
cplx quad_form(const std::vector<cplx>& M, const std::vector<cplx>& c, int na) {
  cplx s = 0.0;
  for (int j = 0; j < na; ++j)
    for (int k = 0; k < na; ++k) s += std::conj(c[j]) * M[j * na + k] * c[k];
  return s;
}
// d(c^H M c)/d(re c_k) = (c^H M)_k + (M c)_k ; d/d(im c_k) = i[(c^H M)_k - (M c)_k]
void quad_form_grad(const std::vector<cplx>& M, const std::vector<cplx>& c, int na, int k, cplx& dre, cplx& dim) {
  cplx cm = 0.0, mc = 0.0;
  for (int j = 0; j < na; ++j) { cm += std::conj(c[j]) * M[j * na + k]; mc += M[k * na + j] * c[j]; }
  dre = cm + mc;
  dim = cplx(0.0, 1.0) * (cm - mc);
}

// int_u^v f(x) dx of the unnormalised EXP / GAUSS / POLY leaf f (as in
// node_norm below) and its gradient (added into dI, length n_par).
double leaf_integral(const Model& m, const Node& n, const double* th, double u, double v, std::vector<double>& dI) {
  const double a = m.lo[n.obs[0]];
  switch (n.kind) {
    case K_EXP: {
      // e^{alpha (u-a)} L phi(alpha L), L = v - u; d/dalpha ln = (u - a) + L psi(alpha L)
      double al = th[n.par[0]], L = v - u;
      double I = std::exp(al * (u - a)) * L * phi(al * L);
      dI[n.par[0]] += I * ((u - a) + L * psi(al * L));
      return I;
    }
    case K_GAUSS: {
      double mu = th[n.par[0]], sg = th[n.par[1]];
      double zu = (u - mu) / (std::sqrt(2.0) * sg), zv = (v - mu) / (std::sqrt(2.0) * sg);
      double de;
      if (zu > 0.0) de = std::erfc(zu) - std::erfc(zv);
      else if (zv < 0.0) de = std::erfc(-zv) - std::erfc(-zu);
      else de = std::erf(zv) - std::erf(zu);
      double I = sg * std::sqrt(kPi / 2.0) * de;
      double gu = std::exp(-zu * zu), gv = std::exp(-zv * zv);
      dI[n.par[0]] += gu - gv;
      dI[n.par[1]] += I / sg - ((v - mu) * gv - (u - mu) * gu) / sg;
      return I;
    }
    case K_POLY: {
      double I = v - u;
      for (size_t k = 1; k <= n.par.size(); ++k) {
        double w = (std::pow(v - n.x0, (double)(k + 1)) - std::pow(u - n.x0, (double)(k + 1))) / (k + 1);
        I += th[n.par[k - 1]] * w;
        dI[n.par[k - 1]] += w;
      }
      return I;
    }
    default:
      return NAN;
  }
}

// Unnormalised shape f of an EXP / GAUSS / POLY leaf at x (the forms of
// leaf_integral) and d ln f / d theta added into g (dense); a POLY shape may
// come out <= 0 (the caller decides what that means).
double leaf_shape(const Model& m, const Node& n, const double* th, double x, double* g) {
  switch (n.kind) {
    case K_EXP: {
      const double a = m.lo[n.obs[0]];
      g[n.par[0]] += x - a;
      return std::exp(th[n.par[0]] * (x - a));
    }
    case K_GAUSS: {
      const double mu = th[n.par[0]], sg = th[n.par[1]], z = (x - mu) / sg;
      g[n.par[0]] += z / sg;
      g[n.par[1]] += z * z / sg;
      return std::exp(-0.5 * z * z);
    }
    case K_POLY: {
      double f = 1.0;
      for (size_t k = 1; k <= n.par.size(); ++k) f += th[n.par[k - 1]] * std::pow(x - n.x0, (double)k);
      for (size_t k = 1; k <= n.par.size(); ++k) g[n.par[k - 1]] += std::pow(x - n.x0, (double)k) / f;
      return f;
    }
    default:
      return NAN;
  }
}

// A CONV child as a function of v (section "Combining functions": the
// children of a convolution may themselves be combinations): a leaf is its
// unnormalised shape s(v); an ADD of leaves is the mixture
// sum_j f_j s_j(v) / N_j of its components, each normalised over the
// child's domain [dom_lo, dom_hi] (the observable's box for the model, the
// residual range for the resolution), the last fraction 1 - sum of the
// others.  Returns the value and adds d value / d theta into df (dense).
double conv_child(const Model& m, const Node& n, const double* th, double v, double dom_lo, double dom_hi,
                  double* df) {
  const int np = m.n_par;
  // per-call scratch (these run once per grid point and event)
  thread_local std::vector<double> gl, dN, q;
  gl.assign(np, 0.0);
  if (n.kind != K_ADD) {
    const double f = leaf_shape(m, n, th, v, gl.data());
    for (int p = 0; p < np; ++p) df[p] += f * gl[p];
    return f;
  }
  const size_t K = n.child.size();
  q.assign(K, 0.0);
  double flast = 1.0, val = 0.0;
  for (size_t j = 0; j + 1 < K; ++j) flast -= th[n.par[j]];
  for (size_t j = 0; j < K; ++j) {
    const Node& c = m.nodes[n.child[j]];
    gl.assign(np, 0.0);
    dN.assign(np, 0.0);
    const double sj = leaf_shape(m, c, th, v, gl.data());
    const double Nj = leaf_integral(m, c, th, dom_lo, dom_hi, dN);
    q[j] = sj / Nj;
    const double fj = j + 1 < K ? th[n.par[j]] : flast;
    val += fj * q[j];
    for (int p = 0; p < np; ++p) df[p] += fj * q[j] * (gl[p] - dN[p] / Nj);
  }
  for (size_t j = 0; j + 1 < K; ++j) df[n.par[j]] += q[j] - q[K - 1];
  return val;
}

// int_u^v of a CONV child (as conv_child) and its theta derivative (added
// into dI, dense).
double conv_child_integral(const Model& m, const Node& n, const double* th, double u, double v, double dom_lo,
                           double dom_hi, std::vector<double>& dI) {
  if (n.kind != K_ADD) return leaf_integral(m, n, th, u, v, dI);
  const int np = m.n_par;
  const size_t K = n.child.size();
  thread_local std::vector<double> r, dIj, dN;
  r.assign(K, 0.0);
  double flast = 1.0, val = 0.0;
  for (size_t j = 0; j + 1 < K; ++j) flast -= th[n.par[j]];
  for (size_t j = 0; j < K; ++j) {
    const Node& c = m.nodes[n.child[j]];
    dIj.assign(np, 0.0);
    dN.assign(np, 0.0);
    const double Ij = leaf_integral(m, c, th, u, v, dIj);
    const double Nj = leaf_integral(m, c, th, dom_lo, dom_hi, dN);
    r[j] = Ij / Nj;
    const double fj = j + 1 < K ? th[n.par[j]] : flast;
    val += fj * r[j];
    for (int p = 0; p < np; ++p) dI[p] += fj * (dIj[p] / Nj - Ij * dN[p] / (Nj * Nj));
  }
  for (size_t j = 0; j + 1 < K; ++j) dI[n.par[j]] += r[j] - r[K - 1];
  return val;
}

// d ln f / dx of a leaf's unnormalised shape at x.
double leaf_shape_dx(const Node& n, const double* th, double x) {
  switch (n.kind) {
    case K_EXP: return th[n.par[0]];
    case K_GAUSS: return -(x - th[n.par[0]]) / (th[n.par[1]] * th[n.par[1]]);
    case K_POLY: {
      double f = 1.0, df = 0.0;
      for (size_t k = 1; k <= n.par.size(); ++k) {
        f += th[n.par[k - 1]] * std::pow(x - n.x0, (double)k);
        df += k * th[n.par[k - 1]] * std::pow(x - n.x0, (double)(k - 1));
      }
      return df / f;
    }
    default:
      return NAN;
  }
}

// f(g(x)) of a COMP node and d ln f(g(x)) / d theta into gr (dense).
double comp_value(const Model& m, const Node& n, const double* th, double x, double* gr) {
  const Node& C = m.nodes[n.child[0]];
  const Node& F = m.nodes[n.child[1]];
  std::vector<double> gc(m.n_par, 0.0);
  const double gval = leaf_shape(m, C, th, x, gc.data());  // gc = d ln g / d theta
  const double fv = leaf_shape(m, F, th, gval, gr);        // gr = d ln f / d theta (shell)
  const double dfdg = leaf_shape_dx(F, th, gval);
  for (int p = 0; p < m.n_par; ++p) gr[p] += dfdg * gval * gc[p];
  return fv;
}

double node_eval(const Model& m, int id, const double* ev, const double* th, const std::vector<NodeNorm>& nn,
                 double* g);

// threads of the grid sums inside a normalisation (the calling entry
// point's thread count)
int g_norm_threads = 1;
int oracle_threads() { return g_norm_threads; }

// q/p of a TDDP node (1 when it is not a parameter)
cplx tddp_qp(const Node& n, const double* th) {
  return n.p_qm >= 0 ? th[n.p_qm] * cplx(std::cos(th[n.p_qa]), std::sin(th[n.p_qa])) : cplx(1.0, 0.0);
}

// Derivatives of the time-dependent rate
//   r = (|A|^2 + |Ab|^2)/2 C + (|A|^2 - |Ab|^2)/2 Cz - Re(conj(A) Ab) S - Im(conj(A) Ab) Sz
// (Ab = (q/p) B0, B0 = sum_k c_k Abar_k) along the coefficient, q/p and
// floating-shape parameters, added into out[p].  For a parameter moving A
// by dA and Ab by dAb, dr = Re(conj(A) dA + conj(Ab) dAb) C
// + Re(conj(A) dA - conj(Ab) dAb) Cz - Re(X') S - Im(X') Sz with
// X' = conj(dA) Ab + conj(A) dAb.  (C, Cz, S, Sz) are the convolved time
// factors of an event or their integrals over t for the normalisation.
void tddp_tangents(const Node& n, const DalitzDef& d, const double* th, const std::vector<cplx>& c, cplx qp,
                   cplx eph, cplx B0, const std::vector<cplx>& a, const std::vector<cplx>& ab,
                   const std::vector<cplx>& dam, const std::vector<cplx>& dag, const std::vector<cplx>& dbm,
                   const std::vector<cplx>& dbg, cplx A, cplx Ab, double C, double Cz, double S, double Sz,
                   double* out) {
  (void)th;
  const auto dr = [&](cplx dA, cplx dAb) {
    const double dnA = 2.0 * (std::conj(A) * dA).real(), dnB = 2.0 * (std::conj(Ab) * dAb).real();
    const cplx dX = std::conj(dA) * Ab + std::conj(A) * dAb;
    return 0.5 * (dnA + dnB) * C + 0.5 * (dnA - dnB) * Cz - dX.real() * S - dX.imag() * Sz;
  };
  const cplx I(0.0, 1.0);
  for (size_t k = 0; k < d.res.size(); ++k) {
    const Res& R = d.res[k];
    out[R.p_re] += dr(a[k + 1], qp * ab[k + 1]);
    out[R.p_im] += dr(I * a[k + 1], I * qp * ab[k + 1]);
    if (R.p_m0 >= 0) {
      out[R.p_m0] += dr(c[k + 1] * dam[k + 1], qp * c[k + 1] * dbm[k + 1]);
      out[R.p_g0] += dr(c[k + 1] * dag[k + 1], qp * c[k + 1] * dbg[k + 1]);
    }
  }
  if (n.p_qm >= 0) {
    out[n.p_qm] += dr(0.0, eph * B0);  // d(q/p)/d|q/p| = e^{i phi}
    out[n.p_qa] += dr(0.0, I * Ab);    // d(q/p)/dphi = i q/p
  }
}

void node_norm(const Model& m, int id, const double* th, std::vector<NodeNorm>& out) {
  const Node& n = m.nodes[id];
  NodeNorm& r = out[id];
  r.lnN = 0.0;
  r.dlnN.assign(m.n_par, 0.0);
  switch (n.kind) {
    case K_EXP: {
      // N = int_a^b e^{alpha (x-a)} dx = L phi(alpha L); dlnN/dalpha = L psi(alpha L)
      double a = m.lo[n.obs[0]], b = m.hi[n.obs[0]], L = b - a, al = th[n.par[0]];
      r.lnN = std::log(L * phi(al * L));
      r.dlnN[n.par[0]] += L * psi(al * L);
      break;
    }
    case K_GAUSS: {
      double a = m.lo[n.obs[0]], b = m.hi[n.obs[0]], mu = th[n.par[0]], sg = th[n.par[1]];
      double za = (a - mu) / (std::sqrt(2.0) * sg), zb = (b - mu) / (std::sqrt(2.0) * sg);
      double de;  // erf(zb) - erf(za)
      if (za > 0.0) de = std::erfc(za) - std::erfc(zb);
      else if (zb < 0.0) de = std::erfc(-zb) - std::erfc(-za);
      else de = std::erf(zb) - std::erf(za);
      double N = sg * std::sqrt(kPi / 2.0) * de;
      double ga = std::exp(-za * za), gb = std::exp(-zb * zb);
      r.lnN = std::log(N);
      r.dlnN[n.par[0]] += (ga - gb) / N;
      r.dlnN[n.par[1]] += 1.0 / sg - ((b - mu) * gb - (a - mu) * ga) / (sg * N);
      break;
    }
    case K_POLY: {
      double a = m.lo[n.obs[0]], b = m.hi[n.obs[0]];
      double N = (b - n.x0) - (a - n.x0);
      std::vector<double> dN(n.par.size());
      for (size_t k = 1; k <= n.par.size(); ++k) {
        double w = (std::pow(b - n.x0, (double)(k + 1)) - std::pow(a - n.x0, (double)(k + 1))) / (k + 1);
        N += th[n.par[k - 1]] * w;
        dN[k - 1] = w;
      }
      r.lnN = std::log(N);
      for (size_t k = 0; k < n.par.size(); ++k) r.dlnN[n.par[k]] += dN[k] / N;
      break;
    }
    case K_DALITZ: {
      const DalitzDef& d = *n.dz;
      std::vector<cplx> c;
      coeffs(d, th, c);
      int na = d.n_amp();
      double N = quad_form(d.I, c, na).real();
      r.lnN = std::log(N);
      for (size_t k = 0; k < d.res.size(); ++k) {
        cplx dre, dim;
        quad_form_grad(d.I, c, na, (int)k + 1, dre, dim);
        r.dlnN[d.res[k].p_re] += dre.real() / N;
        r.dlnN[d.res[k].p_im] += dim.real() / N;
      }
      break;
    }
    case K_TDDP: {
      // N_T = int dDP int_R dt rate: the time integrals of E(t; G) over R
      // are 1/G, so int C = tau/(1-y^2), int S = y tau/(1-y^2), and with x
      // int Cz = tau/(1+x^2), int Sz = x tau/(1+x^2) (x = 0: int E = tau).
      // The conjugate amplitude carries q/p: Abar' = (q/p) Abar.
      const DalitzDef& d = *n.dz;
      std::vector<cplx> c;
      coeffs(d, th, c);
      int na = d.n_amp();
      double tau = th[n.p_tau], y = th[n.p_y], x = n.p_x >= 0 ? th[n.p_x] : 0.0;
      const cplx qp = tddp_qp(n, th), eph = n.p_qm >= 0 ? cplx(std::cos(th[n.p_qa]), std::sin(th[n.p_qa])) : cplx(1.0, 0.0);
      const double aq = std::abs(qp);
      const int np = m.n_par;
      double kc = tau / (1.0 - y * y), ks = y * tau / (1.0 - y * y);
      double opx = 1.0 + x * x, kz = tau / opx, kzs = x * tau / opx;
      double IAA, IBB, RJ, IJ, N;
      if (!floating_shapes(d) && !m.direct_norm) {
        // grid matrices of the fixed shapes
        cplx QJ0 = quad_form(d.Jx, c, na), QJ = qp * QJ0;
        double IBB0 = quad_form(d.Ib, c, na).real();
        IAA = quad_form(d.I, c, na).real();
        IBB = aq * aq * IBB0;
        RJ = QJ.real();
        IJ = QJ.imag();
        N = 0.5 * (IAA + IBB) * kc + 0.5 * (IAA - IBB) * kz - RJ * ks - IJ * kzs;
        r.lnN = std::log(N);
        for (size_t k = 0; k < d.res.size(); ++k) {
          cplx a1, a2, b1, b2, j1, j2;
          quad_form_grad(d.I, c, na, (int)k + 1, a1, a2);
          quad_form_grad(d.Ib, c, na, (int)k + 1, b1, b2);
          quad_form_grad(d.Jx, c, na, (int)k + 1, j1, j2);
          b1 *= aq * aq; b2 *= aq * aq;
          j1 *= qp; j2 *= qp;
          double dre = 0.5 * (a1.real() + b1.real()) * kc + 0.5 * (a1.real() - b1.real()) * kz - j1.real() * ks -
                       j1.imag() * kzs;
          double dim = 0.5 * (a2.real() + b2.real()) * kc + 0.5 * (a2.real() - b2.real()) * kz - j2.real() * ks -
                       j2.imag() * kzs;
          r.dlnN[d.res[k].p_re] += dre / N;
          r.dlnN[d.res[k].p_im] += dim / N;
        }
        if (n.p_qm >= 0) {
          // dIBB/d|q/p| = 2 |q/p| IBB0, dQJ/d|q/p| = e^{i phi} QJ0, dQJ/dphi = i QJ
          const cplx dq = eph * QJ0;
          r.dlnN[n.p_qm] += (0.5 * 2.0 * aq * IBB0 * (kc - kz) - dq.real() * ks - dq.imag() * kzs) / N;
          r.dlnN[n.p_qa] += (IJ * ks - RJ * kzs) / N;
        }
      } else {
        // the grid sum at theta, cell by cell: the time-integrated rate and
        // its derivatives (the same rule as the matrices: cell centres
        // inside the plot, times the cell area)
        const double lo12 = (d.m1 + d.m2) * (d.m1 + d.m2), hi12 = (d.M - d.m3) * (d.M - d.m3);
        const double lo13 = (d.m1 + d.m3) * (d.m1 + d.m3), hi13 = (d.M - d.m2) * (d.M - d.m2);
        const double h12 = (hi12 - lo12) / d.grid, h13 = (hi13 - lo13) / d.grid, area = h12 * h13;
        const int G = d.grid;
        // per grid row: sums of |A|^2, |Abar'|^2, Re and Im conj(A) Abar', then
        // d(rate)/d theta_p for the coefficient, q/p and shape parameters
        const int nw = 4 + np;
        std::vector<double> rows((size_t)G * nw, 0.0);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(oracle_threads())
#endif
        for (int i = 0; i < G; ++i) {
          std::vector<cplx> a(na), ab(na), dam(na), dag(na), dbm(na), dbg(na);
          std::vector<Neumaier> acc(nw);
          std::vector<double> gp(np);
          const double s12 = lo12 + (i + 0.5) * h12;
          for (int j = 0; j < G; ++j) {
            const double s13 = lo13 + (j + 0.5) * h13;
            if (!inside(d, s12, s13)) continue;
            amplitudes_th(d, th, s12, s13, a.data(), dam.data(), dag.data());
            amplitudes_th(d, th, s13, s12, ab.data(), dbm.data(), dbg.data());
            cplx A = 0.0, B0 = 0.0;
            for (int k = 0; k < na; ++k) { A += c[k] * a[k]; B0 += c[k] * ab[k]; }
            const cplx Ab = qp * B0, X = std::conj(A) * Ab;
            acc[0].add(std::norm(A));
            acc[1].add(std::norm(Ab));
            acc[2].add(X.real());
            acc[3].add(X.imag());
            std::fill(gp.begin(), gp.end(), 0.0);
            tddp_tangents(n, d, th, c, qp, eph, B0, a, ab, dam, dag, dbm, dbg, A, Ab, kc, kz, ks, kzs, gp.data());
            for (int p = 0; p < np; ++p) acc[4 + p].add(gp[p]);
          }
          for (int w = 0; w < nw; ++w) rows[(size_t)i * nw + w] = acc[w].value();
        }
        std::vector<Neumaier> tot(nw);
        for (int i = 0; i < G; ++i)
          for (int w = 0; w < nw; ++w) tot[w].add(rows[(size_t)i * nw + w]);
        IAA = tot[0].value() * area;
        IBB = tot[1].value() * area;
        RJ = tot[2].value() * area;
        IJ = tot[3].value() * area;
        N = 0.5 * (IAA + IBB) * kc + 0.5 * (IAA - IBB) * kz - RJ * ks - IJ * kzs;
        r.lnN = std::log(N);
        for (int p = 0; p < np; ++p) r.dlnN[p] += tot[4 + p].value() * area / N;
      }
      double omy = 1.0 - y * y;
      double dN_dtau = 0.5 * (IAA + IBB) / omy + 0.5 * (IAA - IBB) / opx - RJ * y / omy - IJ * x / opx;
      double dN_dy = 0.5 * (IAA + IBB) * tau * 2.0 * y / (omy * omy) - RJ * tau * (1.0 + y * y) / (omy * omy);
      r.dlnN[n.p_tau] += dN_dtau / N;
      r.dlnN[n.p_y] += dN_dy / N;
      if (n.p_x >= 0) {
        double dN_dx = -0.5 * (IAA - IBB) * tau * 2.0 * x / (opx * opx) - IJ * tau * (1.0 - x * x) / (opx * opx);
        r.dlnN[n.p_x] += dN_dx / N;
      }
      break;
    }
    case K_PROD: {
      // groups of one-observable leaf children on a shared observable:
      // Z_g = int_box prod_{j in g} P_j(x) dx by 200 x 16-point Gauss-Legendre
      for (int ch : n.child) node_norm(m, ch, th, out);
      struct GL16 { double x[16], w[16]; };
      static const GL16 gl = [] { GL16 q; gauss_legendre(16, q.x, q.w); return q; }();
      std::vector<int> done(n.child.size(), 0);
      for (size_t a = 0; a < n.child.size(); ++a) {
        const Node& ca = m.nodes[n.child[a]];
        if (done[a] || ca.obs.size() != 1 || !(ca.kind == K_EXP || ca.kind == K_GAUSS || ca.kind == K_POLY)) continue;
        std::vector<int> grp = {n.child[a]};
        for (size_t b = a + 1; b < n.child.size(); ++b) {
          const Node& cb = m.nodes[n.child[b]];
          if (cb.obs.size() == 1 && cb.obs[0] == ca.obs[0] &&
              (cb.kind == K_EXP || cb.kind == K_GAUSS || cb.kind == K_POLY)) {
            grp.push_back(n.child[b]);
            done[b] = 1;
          }
        }
        if (grp.size() < 2) continue;
        const int o = ca.obs[0];
        const double lo = m.lo[o], hi = m.hi[o];
        const int nseg = 200;
        const double h = (hi - lo) / nseg;
        std::vector<double> ev(m.n_obs, 0.0), gj(m.n_par), gs(m.n_par);
        Neumaier Z;
        std::vector<Neumaier> dZ(m.n_par);
        for (int k = 0; k < nseg; ++k)
          for (int i = 0; i < 16; ++i) {
            ev[o] = lo + h * (k + 0.5 * (gl.x[i] + 1.0));
            double l = 0.0;
            std::fill(gs.begin(), gs.end(), 0.0);
            for (int c : grp) {
              l += node_eval(m, c, ev.data(), th, out, gj.data());
              for (int p = 0; p < m.n_par; ++p) gs[p] += gj[p];
            }
            const double f = 0.5 * h * gl.w[i] * std::exp(l);
            Z.add(f);
            for (int p = 0; p < m.n_par; ++p) dZ[p].add(f * gs[p]);
          }
        const double z = Z.value();
        r.lnN += std::log(z);
        for (int p = 0; p < m.n_par; ++p) r.dlnN[p] += dZ[p].value() / z;
      }
      break;
    }
    case K_MAP: {
      // Z = sum_j I_j / N_j: the children's integrals over their ranges,
      // each child normalised over the whole box (N_j)
      const double lo = m.lo[n.obs[0]], hi = m.hi[n.obs[0]];
      const size_t K = n.child.size();
      double Z = 0.0;
      std::vector<double> dZ(m.n_par, 0.0);
      for (size_t j = 0; j < K; ++j) {
        node_norm(m, n.child[j], th, out);
        const NodeNorm& cn = out[n.child[j]];
        const double u = j == 0 ? lo : n.bounds[j - 1], v = j + 1 == K ? hi : n.bounds[j];
        std::vector<double> dI(m.n_par, 0.0);
        const double I = leaf_integral(m, m.nodes[n.child[j]], th, u, v, dI);
        const double Nj = std::exp(cn.lnN), q = I / Nj;
        Z += q;
        for (int p = 0; p < m.n_par; ++p) dZ[p] += dI[p] / Nj - q * cn.dlnN[p];
      }
      r.lnN = std::log(Z);
      for (int p = 0; p < m.n_par; ++p) r.dlnN[p] = dZ[p] / Z;
      break;
    }
    case K_COMP: {
      // Z = int_box f(g(x)) dx by 200 x 16-point Gauss-Legendre
      struct GL16 { double x[16], w[16]; };
      static const GL16 gl = [] { GL16 q; gauss_legendre(16, q.x, q.w); return q; }();
      const double lo = m.lo[n.obs[0]], hi = m.hi[n.obs[0]];
      const int nseg = 200;
      const double h = (hi - lo) / nseg;
      Neumaier Z;
      std::vector<Neumaier> dZ(m.n_par);
      std::vector<double> gr(m.n_par);
      for (int k = 0; k < nseg; ++k)
        for (int i = 0; i < 16; ++i) {
          const double x = lo + h * (k + 0.5 * (gl.x[i] + 1.0));
          std::fill(gr.begin(), gr.end(), 0.0);
          const double f = 0.5 * h * gl.w[i] * comp_value(m, n, th, x, gr.data());
          Z.add(f);
          for (int p = 0; p < m.n_par; ++p) dZ[p].add(f * gr[p]);
        }
      const double z = Z.value();
      r.lnN = std::log(z);
      for (int p = 0; p < m.n_par; ++p) r.dlnN[p] = dZ[p].value() / z;
      break;
    }
    case K_CONV: {
      // Z = sum_k f_M(t_k) int f_R over the residuals that keep x in the box
      const Node& M = m.nodes[n.child[0]];
      const Node& R = m.nodes[n.child[1]];
      const double lo = m.lo[n.obs[0]], hi = m.hi[n.obs[0]], h = (hi - lo) / n.grid;
      Neumaier Z;
      std::vector<Neumaier> dZ(m.n_par);
      std::vector<double> dfm(m.n_par), dI(m.n_par);
      bool undefined = false;
      for (int k = 0; k < n.grid; ++k) {
        const double t = lo + (k + 0.5) * h;
        const double u = std::max(lo - t, n.d_lo), v = std::min(hi - t, n.d_hi);
        if (!(v > u)) continue;
        std::fill(dfm.begin(), dfm.end(), 0.0);
        std::fill(dI.begin(), dI.end(), 0.0);
        const double fm = conv_child(m, M, th, t, lo, hi, dfm.data());
        // a convolution of densities: a model shape that is not positive at
        // a grid point that enters Z leaves the density undefined
        if (!(fm > 0.0) || !std::isfinite(fm)) {
          undefined = true;
          break;
        }
        const double I = conv_child_integral(m, R, th, u, v, n.d_lo, n.d_hi, dI);
        Z.add(fm * I);
        for (int p = 0; p < m.n_par; ++p) dZ[p].add(dfm[p] * I + fm * dI[p]);
      }
      const double z = Z.value();
      r.lnN = undefined ? INFINITY : std::log(z);  // undefined: ln P = -inf at every event
      for (int p = 0; p < m.n_par; ++p) r.dlnN[p] = undefined ? NAN : dZ[p].value() / z;
      break;
    }
    default:
      break;  // ADD and PROD are normalised through their children
  }
  for (int ch : n.child) node_norm(m, ch, th, out);
}

// ln P_node(event) and its gradient (dense, length n_par).  Returns -inf when
// the density is zero or undefined.
double node_eval(const Model& m, int id, const double* ev, const double* th,
                 const std::vector<NodeNorm>& nn, double* g) {
  const Node& n = m.nodes[id];
  const int np = m.n_par;
  for (int p = 0; p < np; ++p) g[p] = 0.0;
  double lp = -INFINITY;
  switch (n.kind) {
    case K_EXP: {
      double x = ev[n.obs[0]], a = m.lo[n.obs[0]];
      lp = th[n.par[0]] * (x - a) - nn[id].lnN;
      g[n.par[0]] += (x - a);
      break;
    }
    case K_GAUSS: {
      double x = ev[n.obs[0]], mu = th[n.par[0]], sg = th[n.par[1]];
      lp = -0.5 * (x - mu) * (x - mu) / (sg * sg) - nn[id].lnN;
      g[n.par[0]] += (x - mu) / (sg * sg);
      g[n.par[1]] += (x - mu) * (x - mu) / (sg * sg * sg);
      break;
    }
    case K_POLY: {
      double u = ev[n.obs[0]] - n.x0, f = 1.0;
      for (size_t k = 1; k <= n.par.size(); ++k) f += th[n.par[k - 1]] * std::pow(u, (double)k);
      if (!(f > 0.0)) return -INFINITY;
      lp = std::log(f) - nn[id].lnN;
      for (size_t k = 1; k <= n.par.size(); ++k) g[n.par[k - 1]] += std::pow(u, (double)k) / f;
      break;
    }
    case K_ADD: {
      const size_t K = n.child.size();
      std::vector<double> lpj(K), pj(K);
      std::vector<std::vector<double>> gj(K, std::vector<double>(np));
      for (size_t j = 0; j < K; ++j) {
        lpj[j] = node_eval(m, n.child[j], ev, th, nn, gj[j].data());
        pj[j] = std::exp(lpj[j]);
      }
      double flast = 1.0, P = 0.0;
      for (size_t j = 0; j + 1 < K; ++j) { flast -= th[n.par[j]]; P += th[n.par[j]] * pj[j]; }
      P += flast * pj[K - 1];
      if (!(P > 0.0)) return -INFINITY;
      lp = std::log(P);
      for (size_t j = 0; j < K; ++j) {
        double fj = (j + 1 < K) ? th[n.par[j]] : flast;
        if (pj[j] == 0.0) continue;
        for (int p = 0; p < np; ++p) g[p] += fj * pj[j] * gj[j][p] / P;
      }
      for (size_t j = 0; j + 1 < K; ++j) g[n.par[j]] += (pj[j] - pj[K - 1]) / P;
      break;
    }
    case K_MAP: {
      // the child whose range holds x
      const double x = ev[n.obs[0]];
      size_t sel = 0;
      while (sel < n.bounds.size() && x >= n.bounds[sel]) ++sel;
      lp = node_eval(m, n.child[sel], ev, th, nn, g) - nn[id].lnN;
      break;
    }
    case K_COMP: {
      const double f = comp_value(m, n, th, ev[n.obs[0]], g);
      if (!(f > 0.0)) return -INFINITY;
      lp = std::log(f) - nn[id].lnN;
      break;
    }
    case K_CONV: {
      // sum over the grid of f_M(t_k) f_R(x - t_k), residual in [d_lo, d_hi]
      const Node& M = m.nodes[n.child[0]];
      const Node& R = m.nodes[n.child[1]];
      const double x = ev[n.obs[0]], lo = m.lo[n.obs[0]], hi = m.hi[n.obs[0]], h = (hi - lo) / n.grid;
      Neumaier S;
      std::vector<Neumaier> dS(np);
      std::vector<double> dfm(np), dfr(np);
      for (int k = 0; k < n.grid; ++k) {
        const double t = lo + (k + 0.5) * h, d = x - t;
        if (d < n.d_lo || d > n.d_hi) continue;
        std::fill(dfm.begin(), dfm.end(), 0.0);
        std::fill(dfr.begin(), dfr.end(), 0.0);
        const double fr = conv_child(m, R, th, d, n.d_lo, n.d_hi, dfr.data());
        if (!(fr > 0.0)) return -INFINITY;  // resolution shape not positive at a residual in use
        const double fm = conv_child(m, M, th, t, lo, hi, dfm.data());
        S.add(fm * fr);
        for (int p = 0; p < np; ++p) dS[p].add(dfm[p] * fr + fm * dfr[p]);
      }
      const double sv = S.value();
      if (!(sv > 0.0)) return -INFINITY;
      lp = std::log(sv) - nn[id].lnN;
      for (int p = 0; p < np; ++p) g[p] = dS[p].value() / sv;
      break;
    }
    case K_DPMAP: {
      // the cell holding (s12, s13): count the boundaries at or below each
      const double a = ev[n.obs[0]], b = ev[n.obs[1]];
      size_t i12 = 0, i13 = 0;
      for (double v : n.bounds) i12 += a >= v ? 1 : 0;
      for (double v : n.bounds2) i13 += b >= v ? 1 : 0;
      lp = node_eval(m, n.child[i12 * (n.bounds2.size() + 1) + i13], ev, th, nn, g);
      break;
    }
    case K_PROD: {
      std::vector<double> gj(np);
      lp = 0.0;
      for (int ch : n.child) {
        double l = node_eval(m, ch, ev, th, nn, gj.data());
        lp += l;
        for (int p = 0; p < np; ++p) g[p] += gj[p];
      }
      lp -= nn[id].lnN;  // shared-observable groups (0 without)
      break;
    }
    case K_DALITZ: {
      const DalitzDef& d = *n.dz;
      double s12 = ev[n.obs[0]], s13 = ev[n.obs[1]];
      if (!inside(d, s12, s13)) return -INFINITY;
      std::vector<cplx> a(d.n_amp()), c;
      amplitudes(d, s12, s13, a.data());
      coeffs(d, th, c);
      cplx A = 0.0;
      for (int k = 0; k < d.n_amp(); ++k) A += c[k] * a[k];
      double A2 = std::norm(A);
      if (!(A2 > 0.0)) return -INFINITY;
      lp = std::log(A2) - nn[id].lnN;
      // d|A|^2/dx = 2 Re(conj(A) dA/dx); dA/d(re c_k) = A_k, dA/d(im c_k) = i A_k
      for (size_t k = 0; k < d.res.size(); ++k) {
        g[d.res[k].p_re] += 2.0 * (std::conj(A) * a[k + 1]).real() / A2;
        g[d.res[k].p_im] += 2.0 * (std::conj(A) * cplx(0.0, 1.0) * a[k + 1]).real() / A2;
      }
      break;
    }
    case K_TDDP: {
      const DalitzDef& d = *n.dz;
      double s12 = ev[n.obs[0]], s13 = ev[n.obs[1]], t = ev[n.obs[2]], st = ev[n.obs[3]];
      if (!inside(d, s12, s13) || !(st > 0.0)) return -INFINITY;
      const int na = d.n_amp();
      std::vector<cplx> a(na), ab(na), dam(na), dag(na), dbm(na), dbg(na), c;
      amplitudes_th(d, th, s12, s13, a.data(), dam.data(), dag.data());
      amplitudes_th(d, th, s13, s12, ab.data(), dbm.data(), dbg.data());  // CP conjugate: 2 <-> 3 swap
      coeffs(d, th, c);
      const cplx qp = tddp_qp(n, th), eph = n.p_qm >= 0 ? cplx(std::cos(th[n.p_qa]), std::sin(th[n.p_qa])) : cplx(1.0, 0.0);
      cplx A = 0.0, B0 = 0.0;
      for (int k = 0; k < na; ++k) { A += c[k] * a[k]; B0 += c[k] * ab[k]; }
      const cplx Ab = qp * B0;  // the conjugate amplitude with q/p
      double tau = th[n.p_tau], y = th[n.p_y];
      double Gm = (1.0 - y) / tau, Gp = (1.0 + y) / tau, G = 1.0 / tau;
      double Em = econv(t, Gm, st), Ep = econv(t, Gp, st);
      double Ct = 0.5 * (Em + Ep), St = 0.5 * (Em - Ep);
      // trigonometric terms: Cz, Sz convolve e^{-G t} cos / sin(x G t); without
      // x, Cz = E(t; 1/tau) and Sz = 0
      double x = 0.0, oz[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (n.p_x >= 0) {
        x = th[n.p_x];
        econv_osc(t, G, x * G, st, oz);
      } else {
        oz[0] = econv(t, G, st);
        oz[2] = econv_dG(t, G, st);
      }
      double Cz = oz[0], Sz = oz[1];
      double ac = 0.5 * (std::norm(A) + std::norm(Ab));
      double a0 = 0.5 * (std::norm(A) - std::norm(Ab));
      cplx X = std::conj(A) * Ab;
      double as = -X.real(), bs = -X.imag();
      double R = ac * Ct + a0 * Cz + as * St + bs * Sz;
      if (!(R > 0.0)) return -INFINITY;
      lp = std::log(R) - nn[id].lnN;
      // coefficients, q/p and floating shapes: the rate's derivative along
      // (dA, dAbar'), divided by the rate
      std::vector<double> gr(np, 0.0);
      tddp_tangents(n, d, th, c, qp, eph, B0, a, ab, dam, dag, dbm, dbg, A, Ab, Ct, Cz, St, Sz, gr.data());
      for (int p = 0; p < np; ++p) g[p] += gr[p] / R;
      double dEm = econv_dG(t, Gm, st), dEp = econv_dG(t, Gp, st);
      // chain rule through Gm = (1-y)/tau, Gp = (1+y)/tau, G = 1/tau and the
      // oscillation frequency w = x/tau
      double dRm = ac * 0.5 + as * 0.5, dRp = ac * 0.5 - as * 0.5;  // dR/dEm, dR/dEp
      double dG_dtau = -1.0 / (tau * tau), dw_dtau = -x / (tau * tau);
      double dCz_dtau = oz[2] * dG_dtau + oz[4] * dw_dtau, dSz_dtau = oz[3] * dG_dtau + oz[5] * dw_dtau;
      double dR_dtau = dRm * dEm * (-(1.0 - y) / (tau * tau)) + dRp * dEp * (-(1.0 + y) / (tau * tau)) +
                       a0 * dCz_dtau + bs * dSz_dtau;
      double dR_dy = dRm * dEm * (-1.0 / tau) + dRp * dEp * (1.0 / tau);
      g[n.p_tau] += dR_dtau / R;
      g[n.p_y] += dR_dy / R;
      if (n.p_x >= 0) g[n.p_x] += (a0 * oz[4] + bs * oz[5]) / tau / R;
      break;
    }
    default:
      return -INFINITY;
  }
  for (int p = 0; p < np; ++p) g[p] -= nn[id].dlnN[p];
  return lp;
}

}  // namespace

// ====================================================================== C API
extern "C" {

Model* om_new(int n_obs, const double* lo, const double* hi, int n_par) {
  Model* m = new Model;
  m->n_obs = n_obs;
  m->n_par = n_par;
  m->lo.assign(lo, lo + n_obs);
  m->hi.assign(hi, hi + n_obs);
  return m;
}
void om_free(Model* m) { delete m; }
void om_set_root(Model* m, int id) { m->root = id; }

static int push(Model* m, Node n) { m->nodes.push_back(n); return (int)m->nodes.size() - 1; }

int om_exp(Model* m, int obs, int p_alpha) {
  Node n; n.kind = K_EXP; n.obs = {obs}; n.par = {p_alpha}; return push(m, n);
}
int om_gauss(Model* m, int obs, int p_mu, int p_sigma) {
  Node n; n.kind = K_GAUSS; n.obs = {obs}; n.par = {p_mu, p_sigma}; return push(m, n);
}
int om_poly(Model* m, int obs, double x0, int degree, const int* p_coef) {
  Node n; n.kind = K_POLY; n.obs = {obs}; n.x0 = x0; n.par.assign(p_coef, p_coef + degree); return push(m, n);
}
int om_add(Model* m, int n_child, const int* child, const int* p_frac) {
  Node n; n.kind = K_ADD; n.child.assign(child, child + n_child); n.par.assign(p_frac, p_frac + n_child - 1);
  return push(m, n);
}
// MAP over observable `obs`: n_child one-observable leaves and their n_child - 1
// increasing inner boundaries.
int om_map(Model* m, int obs, int n_child, const int* child, const double* bounds) {
  Node n; n.kind = K_MAP; n.obs = {obs}; n.child.assign(child, child + n_child);
  n.bounds.assign(bounds, bounds + n_child - 1);
  return push(m, n);
}
// DPMAP: n12 x n13 children (row-major, s12 index first) on observable u,
// with the n12 - 1 and n13 - 1 inner boundaries of s12 and s13.
int om_dpmap(Model* m, int o12, int o13, int ou, int n12, int n13, const int* child, const double* b12,
             const double* b13) {
  Node n; n.kind = K_DPMAP; n.obs = {o12, o13, ou}; n.child.assign(child, child + n12 * n13);
  n.bounds.assign(b12, b12 + n12 - 1);
  n.bounds2.assign(b13, b13 + n13 - 1);
  return push(m, n);
}
// CONV over observable obs: children model, resolution; N grid points;
// residual range [d_lo, d_hi].
int om_conv(Model* m, int obs, int model, int resolution, int grid, double d_lo, double d_hi) {
  Node n; n.kind = K_CONV; n.obs = {obs}; n.child = {model, resolution}; n.grid = grid; n.d_lo = d_lo;
  n.d_hi = d_hi;
  return push(m, n);
}
// COMP over observable obs: children core (POLY), shell.
int om_comp(Model* m, int obs, int core, int shell) {
  Node n; n.kind = K_COMP; n.obs = {obs}; n.child = {core, shell};
  return push(m, n);
}
int om_prod(Model* m, int n_child, const int* child) {
  Node n; n.kind = K_PROD; n.child.assign(child, child + n_child); return push(m, n);
}
static DalitzDef* make_dalitz(const double* kin, int grid, int n_res, const int* ch, const double* m0,
                              const double* g0, const int* J, const int* p_re, const int* p_im) {
  DalitzDef* d = new DalitzDef;
  d->M = kin[0]; d->m1 = kin[1]; d->m2 = kin[2]; d->m3 = kin[3]; d->r = kin[4];
  d->grid = grid;
  for (int k = 0; k < n_res; ++k) d->res.push_back(Res{ch[k], m0[k], g0[k], J[k], p_re[k], p_im[k]});
  build_grid(*d);
  return d;
}
int om_dalitz(Model* m, int o12, int o13, const double* kin, int grid, int n_res, const int* ch,
              const double* m0, const double* g0, const int* J, const int* p_re, const int* p_im) {
  Node n; n.kind = K_DALITZ; n.obs = {o12, o13};
  n.dz = make_dalitz(kin, grid, n_res, ch, m0, g0, J, p_re, p_im);
  return push(m, n);
}
int om_tddp(Model* m, int o12, int o13, int ot, int osig, const double* kin, int grid, int n_res,
            const int* ch, const double* m0, const double* g0, const int* J, const int* p_re,
            const int* p_im, int p_tau, int p_y, int p_x) {
  Node n; n.kind = K_TDDP; n.obs = {o12, o13, ot, osig};
  n.dz = make_dalitz(kin, grid, n_res, ch, m0, g0, J, p_re, p_im);
  n.p_tau = p_tau; n.p_y = p_y; n.p_x = p_x;
  return push(m, n);
}
// The full time-dependent model: as om_tddp, plus complex q/p = |q/p| e^{i phi}
// (p_qm, p_qa; -1: q/p = 1) and floating masses and widths (p_m0[k], p_g0[k]
// >= 0: resonance k's m0 and Gamma0 are those parameters; m0[k], g0[k] are
// then unused).  With floating shapes the normalisation is the grid sum
// taken at every theta (no matrices).
int om_tddp_full(Model* m, int o12, int o13, int ot, int osig, const double* kin, int grid, int n_res,
                 const int* ch, const double* m0, const double* g0, const int* J, const int* p_re,
                 const int* p_im, const int* p_m0, const int* p_g0, int p_tau, int p_y, int p_x, int p_qm,
                 int p_qa) {
  Node n; n.kind = K_TDDP; n.obs = {o12, o13, ot, osig};
  DalitzDef* d = new DalitzDef;
  d->M = kin[0]; d->m1 = kin[1]; d->m2 = kin[2]; d->m3 = kin[3]; d->r = kin[4];
  d->grid = grid;
  bool fl = false;
  for (int k = 0; k < n_res; ++k) {
    Res R{ch[k], m0[k], g0[k], J[k], p_re[k], p_im[k]};
    R.p_m0 = p_m0[k];
    R.p_g0 = p_g0[k];
    fl = fl || R.p_m0 >= 0;
    d->res.push_back(R);
  }
  if (!fl) build_grid(*d);
  n.dz = d;
  n.p_tau = p_tau; n.p_y = p_y; n.p_x = p_x; n.p_qm = p_qm; n.p_qa = p_qa;
  return push(m, n);
}
// Tests: 1 makes every TDDP normalisation the grid sum at theta.
void om_set_direct_norm(Model* m, int on) { m->direct_norm = on != 0; }

// NLL = -sum ln P_root; grad (nullable) = dNLL/dtheta.  cols[o][i] is
// observable o of event i.  Thread partials are combined in thread order.
double om_nll(Model* m, const double* th, int64_t n, const double* const* cols, double* grad, int n_threads) {
  g_norm_threads = n_threads > 0 ? n_threads : 1;
  std::vector<NodeNorm> nn(m->nodes.size());
  node_norm(*m, m->root, th, nn);
  const int np = m->n_par;
  int nt = n_threads > 0 ? n_threads : 1;
  std::vector<Neumaier> part((size_t)nt * (np + 1));
  bool bad = false;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt) reduction(|| : bad)
#endif
  {
    int tid = 0, T = 1;
#ifdef _OPENMP
    tid = omp_get_thread_num();
    T = omp_get_num_threads();
#endif
    int64_t b = n * tid / T, e = n * (tid + 1) / T;
    std::vector<double> ev(m->n_obs), g(np);
    Neumaier* acc = &part[(size_t)tid * (np + 1)];
    for (int64_t i = b; i < e; ++i) {
      for (int o = 0; o < m->n_obs; ++o) ev[o] = cols[o][i];
      double lp = node_eval(*m, m->root, ev.data(), th, nn, g.data());
      if (!std::isfinite(lp)) { bad = true; continue; }
      acc[0].add(-lp);
      if (grad)
        for (int p = 0; p < np; ++p) acc[1 + p].add(-g[p]);
    }
  }
  if (bad) {
    if (grad) for (int p = 0; p < np; ++p) grad[p] = NAN;
    return INFINITY;
  }
  Neumaier tot[1];
  std::vector<Neumaier> gt(np);
  for (int t = 0; t < nt; ++t) {
    tot[0].add(part[(size_t)t * (np + 1)].value());
    for (int p = 0; p < np; ++p) gt[p].add(part[(size_t)t * (np + 1) + 1 + p].value());
  }
  if (grad) for (int p = 0; p < np; ++p) grad[p] = gt[p].value();
  return tot[0].value();
}

// Binned metrics (the fit-manager metric switch of section "GooFit code"):
// events are bin centres with weights w_i (counts); P is the normalised root
// density.  metric 1: binned NLL = -sum w_i ln P(x_i).  metric 2: chi^2 =
// sum (w_i - K P(x_i))^2 / max(w_i, 1), K = (sum of weights) x bin volume,
// the expected count of a bin being K P at its centre.  grad (nullable) =
// d metric / d theta.  Thread partials are combined in thread order.
double om_binned(Model* m, const double* th, int64_t n, const double* const* cols, const double* w, int metric,
                 double K, double* grad, int n_threads) {
  g_norm_threads = n_threads > 0 ? n_threads : 1;
  std::vector<NodeNorm> nn(m->nodes.size());
  node_norm(*m, m->root, th, nn);
  const int np = m->n_par;
  int nt = n_threads > 0 ? n_threads : 1;
  std::vector<Neumaier> part((size_t)nt * (np + 1));
  bool bad = false;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt) reduction(|| : bad)
#endif
  {
    int tid = 0, T = 1;
#ifdef _OPENMP
    tid = omp_get_thread_num();
    T = omp_get_num_threads();
#endif
    int64_t b = n * tid / T, e = n * (tid + 1) / T;
    std::vector<double> ev(m->n_obs), g(np);
    Neumaier* acc = &part[(size_t)tid * (np + 1)];
    for (int64_t i = b; i < e; ++i) {
      for (int o = 0; o < m->n_obs; ++o) ev[o] = cols[o][i];
      const double lp = node_eval(*m, m->root, ev.data(), th, nn, g.data());
      double term, dterm;  // metric term and its derivative with respect to ln P
      if (metric == 1) {
        if (!std::isfinite(lp)) {
          if (w[i] != 0.0) bad = true;
          continue;
        }
        term = -w[i] * lp;
        dterm = -w[i];
      } else {
        const double E = std::isfinite(lp) ? K * std::exp(lp) : 0.0;
        const double r = w[i] - E, s2 = std::max(w[i], 1.0);
        term = r * r / s2;
        dterm = -2.0 * r * E / s2;
      }
      acc[0].add(term);
      if (grad)
        for (int p = 0; p < np; ++p) acc[1 + p].add(dterm * g[p]);
    }
  }
  if (bad) {
    if (grad) for (int p = 0; p < np; ++p) grad[p] = NAN;
    return INFINITY;
  }
  Neumaier tot;
  std::vector<Neumaier> gt(np);
  for (int t = 0; t < nt; ++t) {
    tot.add(part[(size_t)t * (np + 1)].value());
    for (int p = 0; p < np; ++p) gt[p].add(part[(size_t)t * (np + 1) + 1 + p].value());
  }
  if (grad) for (int p = 0; p < np; ++p) grad[p] = gt[p].value();
  return tot.value();
}

// Per-event ln P_root (and optional per-event gradient rows, n x n_par).
void om_logpdf(Model* m, const double* th, int64_t n, const double* const* cols, double* out, double* grad_rows,
               int n_threads) {
  g_norm_threads = n_threads > 0 ? n_threads : 1;
  std::vector<NodeNorm> nn(m->nodes.size());
  node_norm(*m, m->root, th, nn);
  const int np = m->n_par;
  int nt = n_threads > 0 ? n_threads : 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    std::vector<double> ev(m->n_obs), g(np);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      for (int o = 0; o < m->n_obs; ++o) ev[o] = cols[o][i];
      out[i] = node_eval(*m, m->root, ev.data(), th, nn, g.data());
      if (grad_rows) for (int p = 0; p < np; ++p) grad_rows[i * np + p] = g[p];
    }
  }
}

// ln N and d lnN/dtheta of one node (for tests of the normalisations).
double om_node_lnnorm(Model* m, int id, const double* th, double* dlnN) {
  std::vector<NodeNorm> nn(m->nodes.size());
  node_norm(*m, id, th, nn);
  if (dlnN) for (int p = 0; p < m->n_par; ++p) dlnN[p] = nn[id].dlnN[p];
  return nn[id].lnN;
}

// Grid matrices of a DALITZ/TDDP node: which = 0 -> I, 1 -> Ibar, 2 -> J;
// out holds (n_res+1)^2 complex values as interleaved re, im.
int om_dalitz_matrix(Model* m, int id, int which, double* out) {
  const DalitzDef* d = m->nodes[id].dz;
  if (!d) return -1;
  const std::vector<cplx>& M = which == 0 ? d->I : (which == 1 ? d->Ib : d->Jx);
  for (size_t e = 0; e < M.size(); ++e) { out[2 * e] = M[e].real(); out[2 * e + 1] = M[e].imag(); }
  return (int)M.size();
}

// |A(s12,s13)|^2 (and optionally the conjugate-channel |Abar|^2) at the given
// theta for many points; 0 outside the Dalitz plot.
void om_dalitz_amp2(Model* m, int id, const double* th, int64_t n, const double* s12, const double* s13,
                    double* out, int swapped, int n_threads) {
  const DalitzDef& d = *m->nodes[id].dz;
  int nt = n_threads > 0 ? n_threads : 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    std::vector<cplx> a(d.n_amp()), c;
    coeffs(d, th, c);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      if (!inside(d, s12[i], s13[i])) { out[i] = 0.0; continue; }
      if (swapped) amplitudes(d, s13[i], s12[i], a.data());
      else amplitudes(d, s12[i], s13[i], a.data());
      cplx A = 0.0;
      for (int k = 0; k < d.n_amp(); ++k) A += c[k] * a[k];
      out[i] = std::norm(A);
    }
  }
}

// sum_k |c_k A_k| (the constant term included) at the given theta for many
// points, 0 outside: with |A| it gives the condition number of the
// amplitude sum, the factor by which rounding in the terms can grow in A
// (used to scale per-event tolerances).
void om_dalitz_abs_terms(Model* m, int id, const double* th, int64_t n, const double* s12, const double* s13,
                         double* out) {
  const DalitzDef& d = *m->nodes[id].dz;
  std::vector<cplx> a(d.n_amp()), c;
  coeffs(d, th, c);
  for (int64_t i = 0; i < n; ++i) {
    if (!inside(d, s12[i], s13[i])) { out[i] = 0.0; continue; }
    amplitudes(d, s12[i], s13[i], a.data());
    double t = 0.0;
    for (int k = 0; k < d.n_amp(); ++k) t += std::abs(c[k] * a[k]);
    out[i] = t;
  }
}

// Re(conj(A) Abar) (imag = 0) or Im(conj(A) Abar) (imag = 1) at the given
// theta for many points; 0 outside.
void om_dalitz_cross(Model* m, int id, const double* th, int64_t n, const double* s12, const double* s13,
                     double* out, int imag) {
  const DalitzDef& d = *m->nodes[id].dz;
  std::vector<cplx> a(d.n_amp()), ab(d.n_amp()), c;
  coeffs(d, th, c);
  for (int64_t i = 0; i < n; ++i) {
    if (!inside(d, s12[i], s13[i])) { out[i] = 0.0; continue; }
    amplitudes(d, s12[i], s13[i], a.data());
    amplitudes(d, s13[i], s12[i], ab.data());
    cplx A = 0.0, Ab = 0.0;
    for (int k = 0; k < d.n_amp(); ++k) { A += c[k] * a[k]; Ab += c[k] * ab[k]; }
    out[i] = imag ? (std::conj(A) * Ab).imag() : (std::conj(A) * Ab).real();
  }
}

// The coherent sum A = sum_k c_k A_k (c_0 = 1) at many points; 0 outside.
void om_dalitz_amp(Model* m, int id, const double* th, int64_t n, const double* s12, const double* s13,
                   double* re, double* im) {
  const DalitzDef& d = *m->nodes[id].dz;
  std::vector<cplx> a(d.n_amp()), c;
  coeffs(d, th, c);
  for (int64_t i = 0; i < n; ++i) {
    re[i] = im[i] = 0.0;
    if (!inside(d, s12[i], s13[i])) continue;
    amplitudes(d, s12[i], s13[i], a.data());
    cplx A = 0.0;
    for (int k = 0; k < d.n_amp(); ++k) A += c[k] * a[k];
    re[i] = A.real();
    im[i] = A.imag();
  }
}

// Unsmeared (sigma_t -> 0) decay rate of a TDDP node at (s12, s13, t >= 0)
// (Abar carrying q/p, floating shapes at theta):
// e^{-t/tau}[a_c cosh(y t/tau) + a_0 cos(x t/tau) + a_s sinh(y t/tau)
// + b_s sin(x t/tau)] with the same a_c, a_0, a_s, b_s.
void om_tddp_rate(Model* m, int id, const double* th, int64_t n, const double* s12, const double* s13,
                  const double* t, double* out, int n_threads) {
  const Node& nd = m->nodes[id];
  const DalitzDef& d = *nd.dz;
  double tau = th[nd.p_tau], y = th[nd.p_y], x = nd.p_x >= 0 ? th[nd.p_x] : 0.0;
  int nt = n_threads > 0 ? n_threads : 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    std::vector<cplx> a(d.n_amp()), ab(d.n_amp()), c;
    coeffs(d, th, c);
    const cplx qp = tddp_qp(nd, th);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      if (!inside(d, s12[i], s13[i]) || t[i] < 0.0) { out[i] = 0.0; continue; }
      amplitudes_th(d, th, s12[i], s13[i], a.data(), nullptr, nullptr);
      amplitudes_th(d, th, s13[i], s12[i], ab.data(), nullptr, nullptr);
      cplx A = 0.0, Ab = 0.0;
      for (int k = 0; k < d.n_amp(); ++k) { A += c[k] * a[k]; Ab += c[k] * ab[k]; }
      Ab *= qp;
      double Em = std::exp(-(1.0 - y) * t[i] / tau), Ep = std::exp(-(1.0 + y) * t[i] / tau);
      double E0 = std::exp(-t[i] / tau);
      double ac = 0.5 * (std::norm(A) + std::norm(Ab)), a0 = 0.5 * (std::norm(A) - std::norm(Ab));
      cplx X = std::conj(A) * Ab;
      out[i] = ac * 0.5 * (Em + Ep) + a0 * E0 * std::cos(x * t[i] / tau) - X.real() * 0.5 * (Em - Ep) -
               X.imag() * E0 * std::sin(x * t[i] / tau);
    }
  }
}

// ---- building blocks exposed for invariant tests
int om_inside(const double* kin, double s12, double s13) {
  DalitzDef d; d.M = kin[0]; d.m1 = kin[1]; d.m2 = kin[2]; d.m3 = kin[3]; d.r = kin[4]; d.grid = 0;
  return inside(d, s12, s13) ? 1 : 0;
}
// One resonance amplitude and its derivatives in m0 and g0:
// out = {Re A, Im A, Re dA/dm0, Im dA/dm0, Re dA/dg0, Im dA/dg0}.
void om_res_amp_d(const double* kin, int ch, double m0, double g0, int J, double s12, double s13, double* out) {
  DalitzDef d; d.M = kin[0]; d.m1 = kin[1]; d.m2 = kin[2]; d.m3 = kin[3]; d.r = kin[4]; d.grid = 0;
  Res R{ch, m0, g0, J, 0, 0};
  cplx dm, dg;
  cplx a = res_amp_mg(d, R, m0, g0, s12, s13, &dm, &dg);
  out[0] = a.real(); out[1] = a.imag();
  out[2] = dm.real(); out[3] = dm.imag();
  out[4] = dg.real(); out[5] = dg.imag();
}
// One resonance amplitude: out = {Re A, Im A, Gamma(s), B_J(q), Z_J, Re BW, Im BW}.
void om_res_amp(const double* kin, int ch, double m0, double g0, int J, double s12, double s13, double* out) {
  DalitzDef d; d.M = kin[0]; d.m1 = kin[1]; d.m2 = kin[2]; d.m3 = kin[3]; d.r = kin[4]; d.grid = 0;
  Res R{ch, m0, g0, J, 0, 0};
  cplx a = res_amp(d, R, s12, s13, out + 2);
  out[0] = a.real();
  out[1] = a.imag();
}
double om_econv(double t, double G, double s) { return econv(t, G, s); }
double om_econv_dG(double t, double G, double s) { return econv_dG(t, G, s); }
void om_econv_osc(double t, double G, double w, double s, double* out) { econv_osc(t, G, w, s, out); }
double om_erfcx(double x) { return erfcx_pos(x); }
double om_psi(double z) { return psi(z); }

}  // extern "C"
