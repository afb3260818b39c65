// PDF-tree validation, flattening and per-call staging of the constant table.
//
// The tree of the paper's composite PDFs (sections "Combining functions" and
// "Adding new PDFs") is checked once, re-ordered into post-order with the
// root last, and assigned gradient slots and constant offsets.  Before every
// launch `stage` turns the parameter vector into the constants the kernels
// read: derived per-node values (1/sigma, fractions, resonance constants,
// complex coefficients, decay rates) and the normalisation ln N with its
// gradient, computed here in double from closed forms (exponential, Gaussian,
// polynomial, the time integrals) or from the cached Dalitz grid matrices.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <set>
#include <string>

#include "dp_inside.h"
#include "runtime.h"

namespace hf {

// Masses (A, B; spectator C) of daughter pair c: 0 = 12, 1 = 13, 2 = 23.
static void pair_masses(const DalitzInfo& dz, int c, double& mA, double& mB, double& mC) {
  if (c == 0) { mA = dz.m1; mB = dz.m2; mC = dz.m3; }
  else if (c == 1) { mA = dz.m1; mB = dz.m3; mC = dz.m2; }
  else { mA = dz.m2; mB = dz.m3; mC = dz.m1; }
}

// A resonance's kernel constants (m0^2, Kw B0^2, B0: m0 Gamma(s) = Kw B0^2
// q^{2J+1} / (P_J(z) sqrt(s)) and B_J = B0 / sqrt(P_J(z)), with B0^2 =
// P_J(z0), z0 = r^2 q0^2, P_0 = 1, P_1 = 1 + z, P_2 = z^2 + 3z + 9,
// Kw = m0^2 Gamma0 / q0^{2J+1}) at mass m0 and width g0, and their
// derivatives: d(m0^2)/dm0, d(Kw B0^2)/dm0, d ln B0/dm0 and
// d(Kw B0^2)/dGamma0 (the mass enters through q0 as well).
struct ResConst { double m02, kwb, sqb, dm2, dkw_m, dlb_m, dkw_g; };
static ResConst res_consts(const DalitzInfo& dz, int pair, int J, double m0, double g0) {
  double mA, mB, mC;
  pair_masses(dz, pair, mA, mB, mC);
  const double m02 = m0 * m0, thrP = (mA + mB) * (mA + mB), thrM = (mA - mB) * (mA - mB);
  const double q02 = (m02 - thrP) * (m02 - thrM) / (4.0 * m02);
  // q0^2 = (u - P)(u - M) / (4u), u = m0^2: dq0^2/du = (2u - P - M) / (4u) - q0^2 / u
  const double dq02 = ((2.0 * m02 - thrP - thrM) / (4.0 * m02) - q02 / m02) * 2.0 * m0;
  const double r2 = dz.r * dz.r, z0 = r2 * q02, dz0 = r2 * dq02;
  double bnum = 1.0, dbnum = 0.0;
  if (J == 1) { bnum = 1.0 + z0; dbnum = 1.0; }
  if (J == 2) { bnum = z0 * z0 + 3.0 * z0 + 9.0; dbnum = 2.0 * z0 + 3.0; }
  ResConst c;
  c.m02 = m02;
  c.kwb = m02 * g0 / std::pow(std::sqrt(q02), 2 * J + 1) * bnum;
  c.sqb = std::sqrt(bnum);
  c.dm2 = 2.0 * m0;
  c.dkw_m = c.kwb * (2.0 / m0 - 0.5 * (2 * J + 1) * dq02 / q02 + dbnum / bnum * dz0);
  c.dlb_m = 0.5 * dbnum / bnum * dz0;
  c.dkw_g = c.kwb / g0;
  return c;
}


namespace {

thread_local std::string g_err;

bool finite(double x) { return std::isfinite(x); }

}  // namespace

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return HF_E_HIP;
}
const char* last_error() { return g_err.c_str(); }

int n_free(const pdf_graph* g) {
  int k = 0;
  for (auto& p : g->par) k += p.fixed ? 0 : 1;
  return k;
}

double column_ref(const pdf_graph* g, int col, hf_precision prec) {
  if (prec == HF_FP64) return 0.0;
  // the time-dependent density reads t and sigma_t as stored
  if (g->dz.node >= 0 && g->dz.tddp) {
    const KNode& dn = g->prog.node[g->dz.node];
    if (col == dn.col[2] || col == dn.col[3]) return 0.0;
  }
  const ObsInfo& o = g->obs[g->obs_of_col[col]];
  if (finite(o.lo) && finite(o.hi)) return 0.5 * (o.lo + o.hi);
  return 0.0;
}

// ------------------------------------------------------------------ closed-form normalisations
namespace {

// ln of int_a^b e^{alpha (x - a)} dx and its alpha-derivative.
void exp_norm(double alpha, double L, double& lnN, double& dlnN) {
  const double z = alpha * L;
  if (std::fabs(z) < 1e-3) {
    // expm1(z)/z = 1 + z/2 + z^2/6 + z^3/24 ; d/dalpha ln = L (1/2 + z/12 - z^3/720)
    lnN = std::log(L) + std::log1p(z * (0.5 + z * (1.0 / 6.0 + z / 24.0)));
    dlnN = L * (0.5 + z / 12.0 - z * z * z / 720.0);
  } else {
    lnN = std::log(L) + std::log(std::expm1(z) / z);
    dlnN = L * (1.0 / (-std::expm1(-z)) - 1.0 / z);
  }
}

// ln of int_a^b exp(-(x-mu)^2/(2 s^2)) dx and derivatives in mu and s.
bool gauss_norm(double a, double b, double mu, double s, double& lnN, double& dmu, double& ds) {
  if (!(s > 0.0)) return false;
  const double k = 1.0 / (std::sqrt(2.0) * s);
  const double za = (a - mu) * k, zb = (b - mu) * k;
  double w;  // erf(zb) - erf(za), computed from the tail that avoids cancellation
  if (za >= 0.0) w = std::erfc(za) - std::erfc(zb);
  else if (zb <= 0.0) w = std::erfc(-zb) - std::erfc(-za);
  else w = std::erf(zb) - std::erf(za);
  const double N = s * std::sqrt(M_PI / 2.0) * w;
  if (!(N > 0.0)) return false;
  const double ga = std::exp(-za * za), gb = std::exp(-zb * zb);
  lnN = std::log(N);
  dmu = (ga - gb) / N;
  ds = 1.0 / s - ((b - mu) * gb - (a - mu) * ga) / (s * N);
  return true;
}

// split a double into float hi + float lo
void split(double x, float& hi, float& lo) {
  hi = (float)x;
  lo = (float)(x - (double)hi);
}

}  // namespace

// ------------------------------------------------------------------ Dalitz helpers
bool dalitz_inside(const DalitzInfo& dz, double s12, double s13) {
  return dp_inside(dz.M, dz.m1, dz.m2, dz.m3, s12, s13);
}

int ensure_grid(pdf_graph* g, hipStream_t st) {
  DalitzInfo& dz = g->dz;
  if (dz.node < 0) return HF_OK;
  std::lock_guard<std::mutex> lk(g->grid_mu);
  if (dz.ready) return HF_OK;
  if (dz.full && !dz.fl.empty()) {
    // floating shapes: no matrices; the grid kernel runs with every
    // evaluation over the list of the cells inside the plot (so that no
    // lane of a wave idles on a cell outside) and needs its rows of partials
    const int G = dz.gs.grid;
    std::vector<uint32_t> cells;
    for (int i = 0; i < G; ++i) {
      const double s12 = dz.gs.lo12 + ((double)i + 0.5) * dz.gs.h12;
      for (int j = 0; j < G; ++j) {
        const double s13 = dz.gs.lo13 + ((double)j + 0.5) * dz.gs.h13;
        if (dalitz_inside(dz, s12, s13)) cells.push_back(((uint32_t)i << 16) | (uint32_t)j);
      }
    }
    const int64_t chunks = ((int64_t)cells.size() + kBlock - 1) / kBlock;
    const int R = (int)dz.res.size();
    const int n_col = 1 + 2 * R + 3 + (dz.hq ? 2 : 0) + 2 * (int)dz.fl.size();
    dz.norm_rows = (int32_t)std::max<int64_t>(1, std::min<int64_t>(chunks, 1024));
    dz.norm_cols = n_col;
    hipError_t e = hipMalloc(&dz.norm_cells, std::max<size_t>(cells.size(), 1) * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(normalisation grid cells)");
    e = hipMemcpy(dz.norm_cells, cells.data(), cells.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "copy of the normalisation grid cells");
    dz.n_norm_cells = (int64_t)cells.size();
    dz.ready = true;
    return HF_OK;
  }
  const int na = (int)dz.res.size() + 1, n_mat = dz.tddp ? 3 : 1;
  std::vector<double> out((size_t)n_mat * na * na * 2);
  hipError_t e = dalitz_grid_matrices(dz.gs, g->prog, dz.node, dz.tddp, out.data(), st);
  if (e != hipSuccess) return hip_fail(e, "Dalitz normalisation grid");
  const double area = dz.gs.h12 * dz.gs.h13;
  for (double& v : out) v *= area;
  const size_t m = (size_t)na * na * 2;
  dz.I.assign(out.begin(), out.begin() + m);
  if (dz.tddp) {
    dz.Ib.assign(out.begin() + m, out.begin() + 2 * m);
    dz.J.assign(out.begin() + 2 * m, out.begin() + 3 * m);
  }
  dz.ready = true;
  return HF_OK;
}

namespace {

typedef std::complex<double> cd;

// c^H M c and its gradient with respect to (Re c_k, Im c_k), k >= 1 (c_0 = 1).
// d/dRe c_k = 2 Re-part pieces written out from the bilinear form.
double herm_form(const std::vector<double>& Mf, const std::vector<cd>& c, std::vector<double>& dre,
                 std::vector<double>& dim) {
  const int na = (int)c.size();
  auto M = [&](int p, int q) { return cd(Mf[2 * (p * na + q)], Mf[2 * (p * na + q) + 1]); };
  cd tot = 0.0;
  std::vector<cd> left(na, 0.0), right(na, 0.0);  // (c^H M)_q, (M c)_p
  for (int p = 0; p < na; ++p)
    for (int q = 0; q < na; ++q) {
      const cd m = M(p, q);
      tot += std::conj(c[p]) * m * c[q];
      left[q] += std::conj(c[p]) * m;
      right[p] += m * c[q];
    }
  dre.assign(na, 0.0);
  dim.assign(na, 0.0);
  for (int k = 1; k < na; ++k) {
    // f = Re(c^H M c): d/dRe c_k = Re(left_k + right_k); d/dIm c_k = Re(i left_k - i right_k)
    dre[k] = (left[k] + right[k]).real();
    dim[k] = (cd(0.0, 1.0) * (left[k] - right[k])).real();
  }
  return tot.real();
}

// Im(c^H M c) and its gradient with respect to (Re c_k, Im c_k), k >= 1.
double herm_form_im(const std::vector<double>& Mf, const std::vector<cd>& c, std::vector<double>& dre,
                    std::vector<double>& dim) {
  const int na = (int)c.size();
  auto M = [&](int p, int q) { return cd(Mf[2 * (p * na + q)], Mf[2 * (p * na + q) + 1]); };
  cd tot = 0.0;
  std::vector<cd> left(na, 0.0), right(na, 0.0);
  for (int p = 0; p < na; ++p)
    for (int q = 0; q < na; ++q) {
      const cd m = M(p, q);
      tot += std::conj(c[p]) * m * c[q];
      left[q] += std::conj(c[p]) * m;
      right[p] += m * c[q];
    }
  dre.assign(na, 0.0);
  dim.assign(na, 0.0);
  for (int k = 1; k < na; ++k) {
    dre[k] = (left[k] + right[k]).imag();
    dim[k] = (cd(0.0, 1.0) * (left[k] - right[k])).imag();
  }
  return tot.imag();
}

}  // namespace

// ------------------------------------------------------------------ results
void assemble(const pdf_graph* g, const StagedCall& sc, const double* sums, int64_t n_ev, double* nll, double* grad) {
  const int np = (int)g->par.size(), S = g->prog.n_slots;
  const double n = (double)n_ev;
  *nll = (sums ? sums[0] : 0.0) + n * sc.ht.lnN;  // the kernels sum -ln P
  if (!grad) return;
  for (int p = 0; p < np; ++p) grad[p] = n * sc.ht.dlnN[p];
  if (sums && g->mix.K > 0) {
    // mixture sums per child j: S0 = sum q_j, S1 = sum q_j z (EXP: q_j x),
    // S2 = sum q_j z^2; the derivatives of ln L are
    //   f_j (S1 / sigma - dlnN/dmu S0), f_j (S2 / sigma - dlnN/dsigma S0)  (GAUSS)
    //   f_j (S1 + (column reference - a - dlnN/dalpha) S0)                  (EXP)
    //   S0_j - S0_{K-1}                                                      (fraction j)
    const MixInfo& mx = g->mix;
    const double* c = sc.prog.c64;
    const int K = mx.K, rc0 = sc.prog.node[mx.root].c0;
    for (int j = 0; j < K; ++j) {
      const double fj = c[rc0 + j];
      const NodeInfo& cn = g->nodes[mx.child[j]];
      const int c0 = sc.prog.node[mx.child[j]].c0;
      const double S0 = sums[1 + 3 * j], S1 = sums[2 + 3 * j], S2 = sums[3 + 3 * j];
      if (mx.gauss[j]) {
        grad[cn.par[0]] -= fj * (c[c0 + 1] * S1 - c[c0 + 4] * S0);
        grad[cn.par[1]] -= fj * (c[c0 + 1] * S2 - c[c0 + 5] * S0);
      } else {
        grad[cn.par[0]] -= fj * (S1 + (c[c0] - c[c0 + 4]) * S0);
      }
    }
    const NodeInfo& rn = g->nodes[mx.root];
    for (int j = 0; j < K - 1; ++j) grad[rn.par[j]] -= sums[1 + 3 * j] - sums[1 + 3 * (K - 1)];
  } else if (sums) {
    for (int j = 0; j < S; ++j)
      if (g->slot_par[j] >= 0) grad[g->slot_par[j]] -= sums[1 + j];  // slots hold sum d ln P
  }
  for (int p = 0; p < np; ++p)
    if (g->par[p].fixed) grad[p] = 0.0;
}

void assemble_binned(const pdf_graph* g, const StagedCall& sc, const double* sums, double* value, double* grad) {
  const int np = (int)g->par.size(), S = g->n_slots_tree;
  *value = sums ? sums[0] : 0.0;
  if (!grad) return;
  for (int p = 0; p < np; ++p) grad[p] = sums ? -sc.ht.dlnN[p] * sums[1 + S] : 0.0;
  if (sums)
    for (int j = 0; j < S; ++j)
      if (g->slot_par_tree[j] >= 0) grad[g->slot_par_tree[j]] += sums[1 + j];
  for (int p = 0; p < np; ++p)
    if (g->par[p].fixed) grad[p] = 0.0;
}

int32_t rows_for(int kind, hf_precision prec, int64_t n) {
  if (n <= 0) return 0;
  static std::atomic<int> cus[64];
  static std::atomic<int> resident[64][2][KIND_COUNT];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (cus[dev].load() <= 0) {
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0) cu = 256;
    cus[dev].store(cu);
  }
  // rows per compute unit: kRowsPerCU, or HIPFIT_ROWS_PER_CU (1..64) for
  // tuning; at most the kernels' resident blocks per compute unit
  static const int per_cu_env = [] {
    const char* v = std::getenv("HIPFIT_ROWS_PER_CU");
    const int k = v ? std::atoi(v) : 0;
    return k >= 1 && k <= 64 ? k : 0;
  }();
  int per_cu = per_cu_env ? per_cu_env : kRowsPerCU;
  const bool fp32 = prec == HF_FP32_EVAL;
  if (!per_cu_env && kind >= 0 && kind < KIND_COUNT) {
    std::atomic<int>& r = resident[dev][fp32 ? 1 : 0][kind];
    if (r.load() == 0) {
      const int nb = resident_blocks_per_cu(kind, fp32);
      r.store(nb > 0 ? nb : -1);
    }
    const int nb = r.load();
    if (nb > 0 && nb < per_cu) per_cu = nb;
  }
  const int64_t nch = (n + kBlock - 1) / kBlock;
  const int64_t minc = kind_light(kind) ? kMinChunksLight : 1;
  const int64_t want = (nch + minc - 1) / minc;
  const int64_t cap = (int64_t)cus[dev].load() * per_cu;
  return (int32_t)(want < cap ? want : cap);
}

// ------------------------------------------------------------------ staging
namespace {

int subtree_slots(const std::vector<NodeInfo>& all, int k);


// One-observable leaf that a PROD may multiply with others on the same observable.
bool is_leaf1(const NodeInfo& n) {
  return (n.op == OP_EXP || n.op == OP_GAUSS || n.op == OP_POLY) && n.obs.size() == 1;
}

// Groups of a PROD's children (indices into n.child) that are one-observable
// leaves sharing an observable; only groups of two or more.
std::vector<std::vector<int>> shared_groups(const std::vector<NodeInfo>& all, const NodeInfo& n) {
  std::vector<std::vector<int>> out;
  std::vector<int> done(n.child.size(), 0);
  for (size_t a = 0; a < n.child.size(); ++a) {
    if (done[a] || !is_leaf1(all[n.child[a]])) continue;
    std::vector<int> grp = {(int)a};
    for (size_t b = a + 1; b < n.child.size(); ++b)
      if (!done[b] && is_leaf1(all[n.child[b]]) && all[n.child[b]].obs[0] == all[n.child[a]].obs[0]) {
        grp.push_back((int)b);
        done[b] = 1;
      }
    if (grp.size() >= 2) out.push_back(grp);
  }
  return out;
}

}  // namespace

// Share q = int_u^v f / int_box f of a one-observable EXP / GAUSS / POLY leaf
// f on [u, v] inside its box, and dq/d(slot) for the leaf's slots (the
// parameter values are those the kernels see: `rnd` rounds to float on the
// FP32 path).  False when the box integral is not positive.
template <class Rnd>
static bool leaf_share(const pdf_graph* g, const NodeInfo& nd, const double* th, const Rnd& rnd, bool fp32, double u,
                       double v, double& q, std::vector<double>& dq) {
  const ObsInfo& o = g->obs[nd.obs[0]];
  q = 0.0;
  switch (nd.op) {
    case OP_EXP: {
      // ln q = alpha (u - lo) + ln int_0^{v-u} e^{alpha y} dy - ln int_0^L e^{alpha y} dy
      const double alpha = rnd(th[nd.par[0]]);
      double lnI, dI, lnN, dN;
      exp_norm(alpha, v - u, lnI, dI);
      exp_norm(alpha, o.hi - o.lo, lnN, dN);
      q = std::exp(alpha * (u - o.lo) + lnI - lnN);
      dq.assign(1, q * ((u - o.lo) + dI - dN));
      return true;
    }
    case OP_GAUSS: {
      const double mu = th[nd.par[0]];
      const double s = fp32 ? 1.0 / rnd(1.0 / th[nd.par[1]]) : th[nd.par[1]];
      double lnN, dmN, dsN, lnI, dmI, dsI;
      if (!gauss_norm(o.lo, o.hi, mu, s, lnN, dmN, dsN)) return false;
      dq.assign(2, 0.0);
      if (!gauss_norm(u, v, mu, s, lnI, dmI, dsI)) return true;  // far tail: q = 0
      q = std::exp(lnI - lnN);
      dq[0] = q * (dmI - dmN);
      dq[1] = q * (dsI - dsN);
      return true;
    }
    case OP_POLY: {
      const double x0 = nd.consts[0];
      const int d = (int)nd.par.size();
      double I = v - u, N = o.hi - o.lo;
      std::vector<double> wI(d), wN(d);
      for (int j = 1; j <= d; ++j) {
        const double a = rnd(th[nd.par[j - 1]]);
        wI[j - 1] = (std::pow(v - x0, j + 1) - std::pow(u - x0, j + 1)) / (j + 1);
        wN[j - 1] = (std::pow(o.hi - x0, j + 1) - std::pow(o.lo - x0, j + 1)) / (j + 1);
        I += a * wI[j - 1];
        N += a * wN[j - 1];
      }
      if (!(N > 0.0)) return false;
      q = I / N;
      dq.assign(d, 0.0);
      for (int j = 0; j < d; ++j) dq[j] = (wI[j] - q * wN[j]) / N;
      return true;
    }
    default:
      return false;
  }
}

// A one-observable EXP / GAUSS / POLY leaf with the parameter values the
// kernels see: ln P(x), normalised over the observable's box, and its slot
// derivatives.
struct HostLeaf {
  int op = 0, n_slot = 0;
  double p[8] = {0.0}, x0 = 0.0, s = 1.0, lnN = 0.0, dN[8] = {0.0};
  // false where P(x) = 0 (a polynomial at or below zero)
  bool eval(double x, double& l, double* d) const {
    switch (op) {
      case OP_EXP:
        l = p[0] * (x - x0) - lnN;
        d[0] = (x - x0) - dN[0];
        return true;
      case OP_GAUSS: {
        const double z = (x - p[0]) / s;
        l = -0.5 * z * z - lnN;
        d[0] = z / s - dN[0];
        d[1] = z * z / s - dN[1];
        return true;
      }
      default: {
        double f = 1.0, u = 1.0;
        double pw[8];
        for (int j = 0; j < n_slot; ++j) {
          u *= x - x0;
          pw[j] = u;
          f += p[j] * u;
        }
        if (!(f > 0.0)) return false;
        l = std::log(f) - lnN;
        for (int j = 0; j < n_slot; ++j) d[j] = pw[j] / f - dN[j];
        return true;
      }
    }
  }
};

template <class Rnd>
static HostLeaf host_leaf(const pdf_graph* g, const NodeInfo& nd, const double* th, const Rnd& rnd, bool fp32,
                          bool& ok) {
  const ObsInfo& o = g->obs[nd.obs[0]];
  HostLeaf h;
  h.op = nd.op;
  switch (nd.op) {
    case OP_EXP:
      h.n_slot = 1;
      h.p[0] = rnd(th[nd.par[0]]);
      h.x0 = o.lo;
      exp_norm(h.p[0], o.hi - o.lo, h.lnN, h.dN[0]);
      break;
    case OP_GAUSS:
      h.n_slot = 2;
      h.p[0] = th[nd.par[0]];
      h.s = fp32 ? 1.0 / rnd(1.0 / th[nd.par[1]]) : th[nd.par[1]];
      if (!gauss_norm(o.lo, o.hi, h.p[0], h.s, h.lnN, h.dN[0], h.dN[1])) ok = false;
      break;
    default: {
      h.n_slot = (int)nd.par.size();
      h.x0 = nd.consts[0];
      double N = o.hi - o.lo;
      for (int j = 1; j <= h.n_slot; ++j) {
        h.p[j - 1] = rnd(th[nd.par[j - 1]]);
        h.dN[j - 1] = (std::pow(o.hi - h.x0, j + 1) - std::pow(o.lo - h.x0, j + 1)) / (j + 1);
        N += h.p[j - 1] * h.dN[j - 1];
      }
      if (!(N > 0.0)) { ok = false; N = 1.0; }
      h.lnN = std::log(N);
      for (int j = 0; j < h.n_slot; ++j) h.dN[j] /= N;
    }
  }
  return h;
}

// int_u^v f of the unnormalised shape f of an EXP / GAUSS / POLY leaf (the
// kernels' forms: EXP e^{alpha (x - lo)}, GAUSS e^{-(x - mu)^2 / (2 s^2)},
// POLY 1 + sum a_j (x - x0)^j) and d/d(slot) of that integral; 0 when
// v <= u.  `h` carries the parameters as the kernels see them.
static double raw_integral(const HostLeaf& h, double lo, double u, double v, double* dI) {
  for (int j = 0; j < h.n_slot; ++j) dI[j] = 0.0;
  if (!(v > u)) return 0.0;
  switch (h.op) {
    case OP_EXP: {
      double lnI, dln;
      exp_norm(h.p[0], v - u, lnI, dln);
      const double I = std::exp(h.p[0] * (u - lo) + lnI);
      dI[0] = I * ((u - lo) + dln);
      return I;
    }
    case OP_GAUSS: {
      double lnI, dm, ds;
      if (!gauss_norm(u, v, h.p[0], h.s, lnI, dm, ds)) return 0.0;
      const double I = std::exp(lnI);
      dI[0] = I * dm;
      dI[1] = I * ds;
      return I;
    }
    default: {
      double I = v - u;
      for (int j = 1; j <= h.n_slot; ++j) {
        const double w = (std::pow(v - h.x0, j + 1) - std::pow(u - h.x0, j + 1)) / (j + 1);
        I += h.p[j - 1] * w;
        dI[j - 1] = w;
      }
      return I;
    }
  }
}

// 16-point Gauss-Legendre nodes (first 16) and weights (next 16) on [-1, 1].
static const double* gl16() {
  static const double* const gl = [] {
    // nodes (first 16) and weights (next 16) on [-1, 1] by Newton on P_16
    static double q[32];
    const int n = 16;
    for (int i = 0; i < n; ++i) {
      double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= n; ++k) {
          const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (x * p1 - p0) / (x * x - 1.0);
        const double dx = p1 / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
      q[i] = x;
      q[n + i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return q;
  }();
  return gl;
}

// Z = int_box prod_j P_j(x) dx over a group of one-observable leaves on one
// observable, by composite 16-point Gauss-Legendre on segments no wider than
// two of the narrowest Gaussian's widths and four decay lengths of the
// steepest exponential (32 .. 4096 segments), and dZ/d(slot) / Z for the
// leaves' slots in order.  False when Z is not positive.
static bool shared_norm(const std::vector<HostLeaf>& lf, double lo, double hi, double& lnZ,
                        std::vector<double>& dz) {
  const double* const gl = gl16();
  const double L = hi - lo;
  double h = L / 32.0;
  for (const HostLeaf& f : lf) {
    if (f.op == OP_GAUSS) h = std::min(h, 2.0 * f.s);
    if (f.op == OP_EXP && f.p[0] != 0.0) h = std::min(h, 4.0 / std::fabs(f.p[0]));
  }
  const int nseg = (int)std::min(4096.0, std::ceil(L / h));
  h = L / nseg;
  int ns = 0;
  for (const HostLeaf& f : lf) ns += f.n_slot;
  std::vector<double> acc(ns, 0.0), d(ns);
  double Z = 0.0;
  for (int k = 0; k < nseg; ++k)
    for (int i = 0; i < 16; ++i) {
      const double x = lo + h * (k + 0.5 * (gl[i] + 1.0));
      double l = 0.0, li;
      bool live = true;
      for (size_t j = 0, m = 0; j < lf.size(); m += lf[j].n_slot, ++j) {
        live = live && lf[j].eval(x, li, d.data() + m);
        l += li;
      }
      if (!live) continue;
      const double w = 0.5 * h * gl[16 + i] * std::exp(l);
      Z += w;
      for (int m = 0; m < ns; ++m) acc[m] += w * d[m];
    }
  if (!(Z > 0.0) || !std::isfinite(Z)) return false;
  lnZ = std::log(Z);
  dz.resize(ns);
  for (int m = 0; m < ns; ++m) dz[m] = acc[m] / Z;
  return true;
}

void stage(const pdf_graph* g, const double* th, hf_precision prec, StagedCall& sc, bool generic) {
  sc.prog = g->prog;
  sc.ok = true;
  sc.ht.lnN = 0.0;
  sc.ht.dlnN.assign(g->par.size(), 0.0);
  KProgram& P = sc.prog;
  const bool fp32 = prec == HF_FP32_EVAL;
  // The float path sees parameter-derived factors (rates, 1/sigma,
  // fractions, polynomial and amplitude coefficients) rounded to float.  They
  // are rounded here first and every normalisation is computed from the
  // rounded values, so the float density is exactly normalised: its NLL is
  // the NLL at a nearby parameter point, without offsets that jump as the
  // rounding changes.
  auto rnd = [&](double v) { return fp32 ? (double)(float)v : v; };
  constexpr double kLog2e = 1.44269504088896340736;
  auto setc = [&](int i, double v) {
    P.c64[i] = v;
    P.c32[i] = (float)v;
  };
  auto set_ln = [&](int i_hi, int i_lo, double v) {
    P.c64[i_hi] = v;
    P.c64[i_lo] = 0.0;
    float h, l;
    split(v, h, l);
    P.c32[i_hi] = h;
    P.c32[i_lo] = l;
  };
  // children of CONV nodes enter as unnormalised shapes: no normalisation
  // of their own (and no domain check over the box)
  std::vector<char> conv_child(P.n_nodes, 0);
  for (int k = 0; k < P.n_nodes; ++k)
    if (P.node[k].op == OP_CONV || P.node[k].op == OP_COMP)
      for (int c : g->nodes[k].child) conv_child[c] = 1;
  // the Gaussians of a CONV resolution mixture are normalised over the
  // CONV's residual range (index of that CONV node, else -1)
  std::vector<int> res_comp_of(P.n_nodes, -1);
  for (int k = 0; k < P.n_nodes; ++k)
    if (P.node[k].op == OP_CONV && g->nodes[g->nodes[k].child[1]].op == OP_ADD)
      for (int c : g->nodes[g->nodes[k].child[1]].child) res_comp_of[c] = k;
  for (int k = 0; k < P.n_nodes; ++k) {
    const KNode& kn = P.node[k];
    const NodeInfo& nd = g->nodes[k];
    const int c0 = kn.c0;
    const bool hoist = kn.hoisted != 0;
    const bool shape_only = conv_child[k] != 0;
    // n_max: entries of the node's dlnN block (-1: one per derivative; the
    // full time-dependent node, always hoisted, has more derivatives than
    // entries)
    auto norm_terms = [&](double lnN, const std::vector<std::pair<int, double>>& d, int i_hi, int i_lo,
                          int i_d0, int n_max = -1) {
      const int nd_ = n_max < 0 ? (int)d.size() : std::min((int)d.size(), n_max);
      if (shape_only) {
        set_ln(i_hi, i_lo, 0.0);
        for (int j = 0; j < nd_; ++j) setc(i_d0 + j, 0.0);
      } else if (hoist) {
        sc.ht.lnN += lnN;
        for (auto& pd : d) sc.ht.dlnN[pd.first] += pd.second;
        set_ln(i_hi, i_lo, 0.0);
        for (int j = 0; j < nd_; ++j) setc(i_d0 + j, 0.0);
      } else {
        set_ln(i_hi, i_lo, lnN);
        for (int j = 0; j < nd_; ++j) setc(i_d0 + j, d[j].second);
      }
    };
    switch (kn.op) {
      case OP_EXP: {
        const int col = kn.col[0];
        const ObsInfo& o = g->obs[g->obs_of_col[col]];
        // the mixture kernel uses log2(e) alpha rounded to float
        const bool mixc = !generic && g->mix.K > 0 && k != g->mix.root;
        const double alpha = !fp32 ? th[nd.par[0]]
                                   : (mixc ? (double)(float)(kLog2e * th[nd.par[0]]) / kLog2e : rnd(th[nd.par[0]]));
        P.c64[c0] = column_ref(g, col, prec) - o.lo;
        P.c32[c0] = 0.0f;
        setc(c0 + 1, alpha);
        double lnN, dlnN;
        exp_norm(alpha, o.hi - o.lo, lnN, dlnN);
        norm_terms(lnN, {{nd.par[0], dlnN}}, c0 + 2, c0 + 3, c0 + 4);
        break;
      }
      case OP_GAUSS: {
        const int col = kn.col[0];
        const ObsInfo& o = g->obs[g->obs_of_col[col]];
        const double mu = th[nd.par[0]];
        const double k1 = rnd(1.0 / th[nd.par[1]]);
        const double s = fp32 ? 1.0 / k1 : th[nd.par[1]];
        double lnN = 0, dmu = 0, ds = 0;
        // over the box, or over the residual range for a component of a
        // CONV resolution mixture
        const int rk = res_comp_of[k];
        const double nlo = rk >= 0 ? g->nodes[rk].consts[1] : o.lo, nhi = rk >= 0 ? g->nodes[rk].consts[2] : o.hi;
        if (!(s > 0.0) || (!gauss_norm(nlo, nhi, mu, s, lnN, dmu, ds) && !shape_only)) sc.ok = false;
        P.c64[c0] = column_ref(g, col, prec) - mu;
        P.c32[c0] = 0.0f;
        setc(c0 + 1, k1);
        norm_terms(lnN, {{nd.par[0], dmu}, {nd.par[1], ds}}, c0 + 2, c0 + 3, c0 + 4);
        break;
      }
      case OP_POLY: {
        const int col = kn.col[0];
        const ObsInfo& o = g->obs[g->obs_of_col[col]];
        const double x0 = nd.consts[0];
        const int d = kn.aux;
        P.c64[c0] = column_ref(g, col, prec) - x0;
        P.c32[c0] = 0.0f;
        double N = (o.hi - x0) - (o.lo - x0);
        std::vector<double> w(d);
        for (int j = 1; j <= d; ++j) {
          w[j - 1] = (std::pow(o.hi - x0, j + 1) - std::pow(o.lo - x0, j + 1)) / (j + 1);
          const double a = rnd(th[nd.par[j - 1]]);
          N += a * w[j - 1];
          setc(c0 + j, a);
        }
        if (!(N > 0.0)) { sc.ok = sc.ok && shape_only; N = 1.0; }
        std::vector<std::pair<int, double>> dv;
        for (int j = 0; j < d; ++j) dv.push_back({nd.par[j], w[j] / N});
        norm_terms(std::log(N), dv, c0 + d + 1, c0 + d + 2, c0 + d + 3);
        break;
      }
      case OP_ADD: {
        // fractions as the kernels see them; ln of their sum (1 up to the
        // rounding) normalises the sum: added per event by the tree kernel,
        // or on the host when the node is hoisted
        double last = 1.0, sum = 0.0;
        const int K = kn.n_child;
        for (int j = 0; j < K - 1; ++j) {
          const double f = rnd(th[nd.par[j]]);
          setc(c0 + j, f);
          last -= th[nd.par[j]];
          sum += f;
        }
        setc(c0 + K - 1, rnd(last));
        sum += rnd(last);
        const double lnsum = sum > 0.0 ? std::log(sum) : 0.0;
        if (hoist) {
          sc.ht.lnN += lnsum;
          setc(c0 + K, 0.0);
        } else {
          setc(c0 + K, lnsum);
        }
        break;
      }
      case OP_PROD: {
        if (!kn.aux) break;
        // shared-observable groups: ln Z of each group's product and its
        // slot derivatives, per child slot in child order (zero for the
        // children outside every group)
        std::vector<int> base(kn.n_child + 1, 0);
        for (int j = 0; j < kn.n_child; ++j) base[j + 1] = base[j] + P.node[nd.child[j]].n_slot;
        std::vector<double> dslot(base[kn.n_child], 0.0);
        double lnZ = 0.0;
        for (const std::vector<int>& grp : shared_groups(g->nodes, nd)) {
          std::vector<HostLeaf> lf;
          bool ok = true;
          for (int j : grp) lf.push_back(host_leaf(g, g->nodes[nd.child[j]], th, rnd, fp32, ok));
          const ObsInfo& o = g->obs[g->nodes[nd.child[grp[0]]].obs[0]];
          double lz = 0.0;
          std::vector<double> dz;
          if (!ok || !shared_norm(lf, o.lo, o.hi, lz, dz)) { sc.ok = false; continue; }
          lnZ += lz;
          for (size_t j = 0, m = 0; j < grp.size(); m += lf[j].n_slot, ++j)
            for (int q = 0; q < lf[j].n_slot; ++q) dslot[base[grp[j]] + q] = dz[m + q];
        }
        for (int j = 0, m = 0; j < kn.n_child; ++j) {
          const NodeInfo& cn = g->nodes[nd.child[j]];
          for (int q = 0; q < P.node[nd.child[j]].n_slot; ++q, ++m) {
            if (hoist) {
              if (dslot[m] != 0.0) sc.ht.dlnN[cn.par[q]] += dslot[m];
              setc(c0 + 2 + m, 0.0);
            } else {
              setc(c0 + 2 + m, dslot[m]);
            }
          }
        }
        if (hoist) {
          sc.ht.lnN += lnZ;
          set_ln(c0, c0 + 1, 0.0);
        } else {
          set_ln(c0, c0 + 1, lnZ);
        }
        break;
      }
      case OP_COMP: {
        // Z = int_box f(g(x)) dx, composite 16-point Gauss-Legendre on 128
        // segments, with d ln Z / d(slot) for the core's and the shell's slots
        const int col = kn.col[0];
        const ObsInfo& o = g->obs[g->obs_of_col[col]];
        // (the core is a function, the shell is evaluated at its values: the
        // box normalisations host_leaf checks do not apply)
        bool ok = true, ok_c = true, ok_f = true;
        HostLeaf C = host_leaf(g, g->nodes[nd.child[0]], th, rnd, fp32, ok_c);
        HostLeaf F = host_leaf(g, g->nodes[nd.child[1]], th, rnd, fp32, ok_f);
        if (F.op == OP_GAUSS && !(F.s > 0.0)) ok = false;
        C.lnN = F.lnN = 0.0;
        for (int j = 0; j < 8; ++j) C.dN[j] = F.dN[j] = 0.0;
        const int nc = C.n_slot, nf = F.n_slot;
        const double* gl = gl16();
        const int nseg = 128;
        const double hs = (o.hi - o.lo) / nseg;
        double Z = 0.0;
        std::vector<double> dZ(nc + nf, 0.0);
        double dc[8], df[8];
        for (int q = 0; q < nseg && ok; ++q)
          for (int i = 0; i < 16; ++i) {
            const double x = o.lo + hs * (q + 0.5 * (gl[i] + 1.0));
            // core value and its slot derivatives (d g / d a_j = (x - x0)^j)
            double gv = 1.0, uk = 1.0;
            for (int j = 0; j < nc; ++j) {
              uk *= x - C.x0;
              dc[j] = uk;
              gv += C.p[j] * uk;
            }
            double lf;
            if (!F.eval(gv, lf, df)) { ok = false; break; }
            // d ln f / dg of the shell's shape
            double dfdg;
            if (F.op == OP_EXP) dfdg = F.p[0];
            else if (F.op == OP_GAUSS) dfdg = -(gv - F.p[0]) / (F.s * F.s);
            else {
              double pv = 1.0, dp = 0.0, w = 1.0;
              for (int j = 1; j <= nf; ++j) {
                dp += j * F.p[j - 1] * w;
                w *= gv - F.x0;
                pv += F.p[j - 1] * w;
              }
              dfdg = dp / pv;
            }
            const double wq = 0.5 * hs * gl[16 + i] * std::exp(lf);
            Z += wq;
            for (int j = 0; j < nc; ++j) dZ[j] += wq * dfdg * dc[j];
            for (int j = 0; j < nf; ++j) dZ[nc + j] += wq * df[j];
          }
        if (!ok || !(Z > 0.0) || !std::isfinite(Z)) { sc.ok = false; Z = 1.0; }
        const double lnZ = std::log(Z);
        setc(c0 + 2, column_ref(g, col, prec));
        for (int j = 0; j < nc + nf; ++j) {
          const double dz = dZ[j] / Z;
          const NodeInfo& cn = g->nodes[nd.child[j < nc ? 0 : 1]];
          if (hoist) {
            sc.ht.dlnN[cn.par[j < nc ? j : j - nc]] += dz;
            setc(c0 + 3 + j, 0.0);
          } else {
            setc(c0 + 3 + j, dz);
          }
        }
        if (hoist) {
          sc.ht.lnN += lnZ;
          set_ln(c0, c0 + 1, 0.0);
        } else {
          set_ln(c0, c0 + 1, lnZ);
        }
        break;
      }
      case OP_CONV: {
        // grid t_k = lo + (k + 1/2) h; Z = sum_k f_M(t_k) int_{box} f_R(x - t_k) dx
        const int N = kn.aux, col = kn.col[0];
        const ObsInfo& o = g->obs[g->obs_of_col[col]];
        const double ref = column_ref(g, col, prec), h = (o.hi - o.lo) / N;
        const double dlo = nd.consts[1], dhi = nd.consts[2];
        // (the box normalisations host_leaf checks are the model's; the
        // resolution lives on the residual range)
        bool ok = true, ok_r = true;
        HostLeaf M = host_leaf(g, g->nodes[nd.child[0]], th, rnd, fp32, ok);
        const NodeInfo& rn = g->nodes[nd.child[1]];
        const bool mixr = rn.op == OP_ADD;  // resolution: a mixture of Gaussians
        HostLeaf R = host_leaf(g, mixr ? g->nodes[rn.child[0]] : rn, th, rnd, fp32, ok_r);
        if (R.op == OP_GAUSS && !(R.s > 0.0)) ok = false;
        M.lnN = R.lnN = 0.0;  // shapes
        for (int j = 0; j < 8; ++j) M.dN[j] = R.dN[j] = 0.0;
        // mixture components (normalised over [d_lo, d_hi]) and fractions as
        // the kernels see them (the ADD's staged constants)
        const int KR = mixr ? (int)rn.child.size() : 0;
        std::vector<HostLeaf> RC(KR);
        std::vector<double> fr(KR), Nr(KR), dNr(2 * KR);
        for (int j = 0; j < KR; ++j) {
          bool okc = true;
          RC[j] = host_leaf(g, g->nodes[rn.child[j]], th, rnd, fp32, okc);
          if (!(RC[j].s > 0.0)) ok = false;
          RC[j].lnN = 0.0;
          RC[j].dN[0] = RC[j].dN[1] = 0.0;
          double dn[8];
          Nr[j] = raw_integral(RC[j], o.lo, dlo, dhi, dn);
          dNr[2 * j] = dn[0];
          dNr[2 * j + 1] = dn[1];
          if (!(Nr[j] > 0.0)) { ok = false; Nr[j] = 1.0; }
          fr[j] = P.c64[P.node[nd.child[1]].c0 + j];
        }
        const int nm = M.n_slot, nr = mixr ? 3 * KR - 1 : R.n_slot;
        // the resolution's integral over [u, v] and its slot derivatives
        // (mixture slots: each Gaussian's (mu, sigma), then the fractions)
        auto res_integral = [&](double u, double v, double* dI) {
          if (!mixr) return raw_integral(R, o.lo, u, v, dI);
          double I = 0.0, rj[3];
          for (int j = 0; j < KR; ++j) {
            double di[8];
            const double Ij = raw_integral(RC[j], o.lo, u, v, di);
            rj[j] = Ij / Nr[j];
            I += fr[j] * rj[j];
            dI[2 * j] = fr[j] * (di[0] - rj[j] * dNr[2 * j]) / Nr[j];
            dI[2 * j + 1] = fr[j] * (di[1] - rj[j] * dNr[2 * j + 1]) / Nr[j];
          }
          for (int j = 0; j + 1 < KR; ++j) dI[2 * KR + j] = rj[j] - rj[KR - 1];
          return I;
        };
        // exponent shift: the shapes' maxima over the grid and the residual range
        double cm = -INFINITY, cr = -INFINITY, l, d[8];
        for (int k = 0; k < N; ++k)
          if (M.eval(o.lo + (k + 0.5) * h, l, d)) cm = std::max(cm, l);
        if (mixr) {
          for (int j = 0; j < KR; ++j) cr = std::max(cr, -std::log(Nr[j]));  // a component's peak, 1 / N_j
        } else {
          for (int k = 0; k <= 256; ++k)
            if (R.eval(dlo + (dhi - dlo) * k / 256.0, l, d)) cr = std::max(cr, l);
          if (R.op == OP_GAUSS && R.p[0] > dlo && R.p[0] < dhi) cr = std::max(cr, 0.0);
        }
        const double shift = std::isfinite(cm) && std::isfinite(cr) ? cm + cr : 0.0;
        double Z = 0.0;
        std::vector<double> dZ(nm + nr, 0.0);
        double dm[8], dI[8];
        for (int k = 0; k < N; ++k) {
          const double t = o.lo + (k + 0.5) * h;
          const double u = std::max(o.lo - t, dlo), v = std::min(o.hi - t, dhi);
          if (!(v > u)) continue;  // no residual of this grid point keeps x in the box
          // a convolution of densities: the model's shape must be positive at
          // every grid point that enters Z, else the density is undefined
          if (!M.eval(t, l, dm)) {
            ok = false;
            continue;
          }
          const double I = res_integral(u, v, dI);
          if (I == 0.0) continue;
          const double fm = std::exp(l);
          Z += fm * I;
          for (int j = 0; j < nm; ++j) dZ[j] += fm * dm[j] * I;
          for (int j = 0; j < nr; ++j) dZ[nm + j] += fm * dI[j];
        }
        if (!ok || !(Z > 0.0) || !std::isfinite(Z)) { sc.ok = false; Z = 1.0; }
        // the kernel forms t_k = lo + (k + 1/2) h and x - t_k in double from
        // the stored event's value, as here and in the definition
        P.c64[c0] = o.lo;
        P.c32[c0] = (float)P.c64[c0];
        setc(c0 + 1, h);
        setc(c0 + 2, dlo);
        setc(c0 + 3, dhi);
        setc(c0 + 4, ref);
        setc(c0 + 5, shift);
        const double lnZ = std::log(Z);
        // the children's slots in order: the model's, then the resolution's
        // subtree (its mixture's Gaussians, then its fractions)
        const KNode& rk = P.node[nd.child[1]];
        const int r_first = rk.slot0 + rk.n_slot - nr;
        for (int j = 0; j < nm + nr; ++j) {
          const double dz = dZ[j] / Z;
          const int slot = j < nm ? P.node[nd.child[0]].slot0 + j : r_first + (j - nm);
          if (hoist) {
            if (g->slot_par[slot] >= 0) sc.ht.dlnN[g->slot_par[slot]] += dz;
            setc(c0 + 8 + j, 0.0);
          } else {
            setc(c0 + 8 + j, dz);
          }
        }
        if (hoist) {
          sc.ht.lnN += lnZ;
          set_ln(c0 + 6, c0 + 7, -shift);
        } else {
          set_ln(c0 + 6, c0 + 7, lnZ - shift);
        }
        break;
      }
      case OP_DPMAP: {
        // the column references of s12 and s13 (the kernel adds them back
        // to the stored values), then the cell boundaries
        const int n12 = (int)nd.consts[0], n13 = (int)nd.consts[1];
        setc(c0, column_ref(g, kn.col[0], prec));
        setc(c0 + 1, column_ref(g, kn.col[1], prec));
        for (int j = 0; j < n12 - 1; ++j) setc(c0 + 2 + j, nd.consts[2 + j]);
        for (int j = 0; j < n13 - 1; ++j) setc(c0 + 2 + n12 - 1 + j, nd.consts[n12 + 1 + j]);
        break;
      }
      case OP_MAP: {
        // boundaries, then the column reference (the kernel adds it back to
        // the stored value); Z = sum of the children's shares of their
        // ranges (each child normalised over the box)
        const int K = kn.n_child, col = kn.col[0];
        const ObsInfo& o = g->obs[g->obs_of_col[col]];
        for (int j = 0; j < K - 1; ++j) setc(c0 + j, nd.consts[j]);
        setc(c0 + K - 1, column_ref(g, col, prec));
        double Z = 0.0;
        std::vector<std::vector<double>> dq(K);
        for (int j = 0; j < K; ++j) {
          const double u = j == 0 ? o.lo : nd.consts[j - 1], v = j + 1 == K ? o.hi : nd.consts[j];
          double q = 0.0;
          if (!leaf_share(g, g->nodes[nd.child[j]], th, rnd, fp32, u, v, q, dq[j])) sc.ok = false;
          Z += q;
        }
        if (!(Z > 0.0)) { sc.ok = false; Z = 1.0; }
        const double lnZ = std::log(Z);
        int m = 0;
        for (int j = 0; j < K; ++j) {
          const NodeInfo& cn = g->nodes[nd.child[j]];
          for (size_t q = 0; q < dq[j].size(); ++q, ++m) {
            const double dz = dq[j][q] / Z;
            if (hoist) {
              sc.ht.dlnN[cn.par[q]] += dz;
              setc(c0 + K + 2 + m, 0.0);
            } else {
              setc(c0 + K + 2 + m, dz);
            }
          }
        }
        if (hoist) {
          sc.ht.lnN += lnZ;
          set_ln(c0 + K, c0 + K + 1, 0.0);
        } else {
          set_ln(c0 + K, c0 + K + 1, lnZ);
        }
        break;
      }
      case OP_DALITZ:
      case OP_TDDP: {
        const DalitzInfo& dz = g->dz;
        const bool td = kn.op == OP_TDDP;
        const int R = kn.aux;
        P.c64[c0 + kDzRef12] = column_ref(g, kn.col[0], prec);
        P.c64[c0 + kDzRef13] = column_ref(g, kn.col[1], prec);
        std::vector<cd> c(R + 1, cd(1.0, 0.0));
        const int cb = c0 + dz_coef_base(R, td);
        for (int j = 0; j < R; ++j) {
          c[j + 1] = cd(rnd(th[nd.par[2 * j]]), rnd(th[nd.par[2 * j + 1]]));
          setc(cb + 2 * j, c[j + 1].real());
          setc(cb + 2 * j + 1, c[j + 1].imag());
        }
        std::vector<std::pair<int, double>> dv;
        double lnN = 0.0;
        if (!td) {
          std::vector<double> dre, dim;
          const double N = herm_form(dz.I, c, dre, dim);
          if (!(N > 0.0)) sc.ok = false;
          lnN = std::log(N);
          for (int j = 0; j < R; ++j) {
            dv.push_back({nd.par[2 * j], dre[j + 1] / N});
            dv.push_back({nd.par[2 * j + 1], dim[j + 1] / N});
          }
        } else {
          // parameters: 2R coefficients, tau, y and (optionally) x; the full
          // model adds q/p = |q/p| e^{i phi} and floating masses and widths
          const bool hx = dz.p_x >= 0;
          const double tau = th[dz.p_tau], y = th[dz.p_y], x = hx ? th[dz.p_x] : 0.0;
          if (!(tau > 0.0) || !(std::fabs(y) < 1.0)) sc.ok = false;
          double qr = 1.0, qi = 0.0, qm = 1.0, ph = 0.0;
          if (dz.hq) {
            qm = th[dz.p_qm];
            ph = th[dz.p_qa];
            if (!(qm > 0.0) || !std::isfinite(ph)) sc.ok = false;
            qr = qm * std::cos(ph);
            qi = qm * std::sin(ph);
          }
          // time integrals over the real line: int C = tau/(1-y^2),
          // int S = y tau/(1-y^2), int Cz = tau/(1+x^2), int Sz = x tau/(1+x^2)
          const double den = 1.0 - y * y, opx = 1.0 + x * x;
          const double kc = tau / den, ks = y * tau / den, kz = tau / opx, kzs = x * tau / opx;
          if (dz.full) {
            const int fb = c0 + dz_full_base(R);
            setc(fb + kFqRe, qr);
            setc(fb + kFqIm, qi);
            setc(fb + kFiq, qm > 0.0 ? 1.0 / qm : 0.0);
            setc(fb + kFhx, hx ? 1.0 : 0.0);
            setc(fb + kFhq, dz.hq ? 1.0 : 0.0);
            setc(fb + kFnf, (double)dz.fl.size());
            setc(fb + kFkc, kc);
            setc(fb + kFkz, kz);
            setc(fb + kFks, ks);
            setc(fb + kFkzs, kzs);
            // floating resonances: their constants and Jacobians at theta
            for (size_t f = 0; f < dz.fl.size(); ++f) {
              const FloatRes& fr = dz.fl[f];
              const double m0 = th[fr.p_m0], g0 = th[fr.p_g0];
              double mA, mB, mC;
              pair_masses(dz, fr.pair, mA, mB, mC);
              if (!(m0 > mA + mB) || !(g0 > 0.0) || !std::isfinite(m0) || !std::isfinite(g0)) {
                sc.ok = false;
                continue;
              }
              const ResConst rcn = res_consts(dz, fr.pair, fr.J, m0, g0);
              const int rb = c0 + dz_res_base(R, true) + fr.place * kResStride;
              setc(rb + kResM02, rcn.m02);
              setc(rb + kResKwB, rcn.kwb);
              setc(rb + kResSqB, rcn.sqb);
              const int lb = fb + kFlBase + (int)f * kFlStride;
              setc(lb + kFlRes, fr.place);
              setc(lb + kFlPair, fr.pair);
              setc(lb + kFlJ, fr.J);
              setc(lb + kFlDm2, rcn.dm2);
              setc(lb + kFlDkwM, rcn.dkw_m);
              setc(lb + kFlDlbM, rcn.dlb_m);
              setc(lb + kFlDkwG, rcn.dkw_g);
            }
          }
          if (dz.full && !dz.fl.empty()) {
            // normalisation from the grid kernel at this theta (eval_one)
            sc.grid_norm = true;
            sc.tint[0] = kc;
            sc.tint[1] = kz;
            sc.tint[2] = ks;
            sc.tint[3] = kzs;
          } else {
            std::vector<double> aR, aI, bR, bI, jR, jI, kR, kI;
            const double IA = herm_form(dz.I, c, aR, aI);
            const double IB0 = herm_form(dz.Ib, c, bR, bI);
            const double X0 = herm_form(dz.J, c, jR, jI);     // Re c^H J c
            const double Y0 = herm_form_im(dz.J, c, kR, kI);  // Im c^H J c
            // with q/p: Ibar scales by |q/p|^2, the cross term c^H J c by q/p
            const double IB = qm * qm * IB0, X = qr * X0 - qi * Y0, Y = qr * Y0 + qi * X0;
            const double N = 0.5 * (IA + IB) * kc + 0.5 * (IA - IB) * kz - X * ks - Y * kzs;
            if (!(N > 0.0)) sc.ok = false;
            lnN = std::log(N);
            for (int j = 1; j <= R; ++j) {
              const double br = qm * qm * bR[j], bi = qm * qm * bI[j];
              const double xr = qr * jR[j] - qi * kR[j], yr = qr * kR[j] + qi * jR[j];
              const double xi = qr * jI[j] - qi * kI[j], yi = qr * kI[j] + qi * jI[j];
              const double dr = 0.5 * (aR[j] + br) * kc + 0.5 * (aR[j] - br) * kz - xr * ks - yr * kzs;
              const double di = 0.5 * (aI[j] + bi) * kc + 0.5 * (aI[j] - bi) * kz - xi * ks - yi * kzs;
              dv.push_back({nd.par[2 * j - 2], dr / N});
              dv.push_back({nd.par[2 * j - 1], di / N});
            }
            const double dtau = 0.5 * (IA + IB) / den + 0.5 * (IA - IB) / opx - X * y / den - Y * x / opx;
            const double dy = 0.5 * (IA + IB) * tau * 2.0 * y / (den * den) - X * tau * (1.0 + y * y) / (den * den);
            dv.push_back({dz.p_tau, dtau / N});
            dv.push_back({dz.p_y, dy / N});
            if (hx) {
              const double dx = -0.5 * (IA - IB) * tau * 2.0 * x / (opx * opx) - Y * tau * (1.0 - x * x) / (opx * opx);
              dv.push_back({dz.p_x, dx / N});
            }
            if (dz.hq) {
              // d/d|q/p|: Ibar' = 2 |q/p| Ibar0, cross' = e^{i phi} c^H J c;
              // d/dphi: cross' = i q/p c^H J c
              const double er = std::cos(ph), ei = std::sin(ph);
              const double dq = (0.5 * 2.0 * qm * IB0 * (kc - kz) - (er * X0 - ei * Y0) * ks - (er * Y0 + ei * X0) * kzs);
              dv.push_back({dz.p_qm, dq / N});
              dv.push_back({dz.p_qa, (Y * ks - X * kzs) / N});
            }
          }
          const int tb = c0 + dz_time_base(R, dz.full ? kMaxResFull : kMaxRes);
          setc(tb + kTdGm, (1.0 - y) / tau);
          setc(tb + kTdGp, (1.0 + y) / tau);
          setc(tb + kTdG, 1.0 / tau);
          setc(tb + kTdDGmTau, -(1.0 - y) / (tau * tau));
          setc(tb + kTdDGpTau, -(1.0 + y) / (tau * tau));
          setc(tb + kTdDGTau, -1.0 / (tau * tau));
          setc(tb + kTdDGmY, -1.0 / tau);
          setc(tb + kTdDGpY, 1.0 / tau);
          setc(tb + kTdW, x / tau);
          setc(tb + kTdDWTau, -x / (tau * tau));
          setc(tb + kTdDWX, hx ? 1.0 / tau : 0.0);
        }
        norm_terms(lnN, dv, c0 + kDzLnHi, c0 + kDzLnLo, c0 + kDzDln, dz_n_dln(R, td));
        break;
      }
    }
  }
}

// ------------------------------------------------------------------ creation
namespace {

int node_slots(const NodeInfo& n) {
  switch (n.op) {
    case OP_EXP: return 1;
    case OP_GAUSS: return 2;
    case OP_POLY: return (int)n.par.size();
    case OP_ADD: return (int)n.child.size() - 1;
    case OP_PROD: return 0;
    default: return (int)n.par.size();
  }
}

// A TDDP node of the full time-dependent model (the full constant form, or
// more resonances than the plain kernels hold): evaluated by the full
// kernel, as the root only.
bool tddp_full(const NodeInfo& n) {
  if (n.op != OP_TDDP) return false;
  const int R = (int)n.consts[6];
  return R > kMaxRes || (int)n.consts.size() == 8 + 5 * R;
}

// Slots of a node and everything below it (a CONV child: a leaf, or a
// mixture of leaves).
int subtree_slots(const std::vector<NodeInfo>& all, int k) {
  int s = node_slots(all[k]);
  for (int c : all[k].child) s += subtree_slots(all, c);
  return s;
}

int node_consts(const std::vector<NodeInfo>& all, const NodeInfo& n) {
  switch (n.op) {
    case OP_MAP: {
      int slots = 0;
      for (int c : n.child) slots += node_slots(all[c]);
      return (int)n.child.size() + 2 + slots;
    }
    case OP_PROD: {
      // with shared groups: lnZ_hi, lnZ_lo, then dlnZ/d(slot) of every child slot
      if (shared_groups(all, n).empty()) return 0;
      int slots = 0;
      for (int c : n.child) slots += node_slots(all[c]);
      return 2 + slots;
    }
    case OP_DPMAP: return (int)n.consts[0] + (int)n.consts[1];
    case OP_CONV: return 8 + subtree_slots(all, n.child[0]) + subtree_slots(all, n.child[1]);
    case OP_COMP: return 3 + node_slots(all[n.child[0]]) + node_slots(all[n.child[1]]);
    case OP_EXP: return 5;
    case OP_GAUSS: return 6;
    case OP_POLY: return 2 * (int)n.par.size() + 3;
    case OP_ADD: return (int)n.child.size() + 1;
    case OP_DALITZ: return dz_n_const((int)n.consts[6], false);
    default: return tddp_full(n) ? dz_n_const_full((int)n.consts[6]) : dz_n_const((int)n.consts[6], true);
  }
}

// (pair, spin) group 3 * pair + J of resonance j of a Dalitz node (the
// node's constant block holds per resonance: pair 12 / 13 / 23, m0, Gamma0, J).
int res_group_of(const NodeInfo& n, int j) {
  const double ch = n.consts[7 + 4 * j];
  return 3 * (ch == 12 ? 0 : (ch == 13 ? 1 : 2)) + (int)n.consts[10 + 4 * j];
}

// Stable reordering of a Dalitz node's resonances into (pair, spin) groups,
// each resonance's two coefficient parameters moving with it: the kernels
// evaluate every group in a loop of its own with the pair and spin fixed.
// The density does not depend on the order of the terms of the coherent sum.
void group_resonances(NodeInfo& n, int R) {
  std::vector<int> idx(R);
  for (int j = 0; j < R; ++j) idx[j] = j;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return res_group_of(n, a) < res_group_of(n, b); });
  const std::vector<double> c = n.consts;
  const std::vector<int> p = n.par;
  for (int j = 0; j < R; ++j) {
    for (int i = 0; i < 4; ++i) n.consts[7 + 4 * j + i] = c[7 + 4 * idx[j] + i];
    n.par[2 * j] = p[2 * idx[j]];
    n.par[2 * j + 1] = p[2 * idx[j] + 1];
  }
  if ((int)c.size() == 8 + 5 * R) {
    // full form: the floating-shape flags move with their resonances, and so
    // do the (m0, Gamma0) parameter pairs at the end of the list (given in
    // resonance order)
    const int fl = (int)c[7 + 4 * R];
    const int tail0 = 2 * R + 2 + (fl & 1) + 2 * ((fl >> 1) & 1);
    std::vector<int> pair_of(R, -1);
    for (int j = 0, f = 0; j < R; ++j)
      if (c[8 + 4 * R + j] == 1) pair_of[j] = f++;
    for (int j = 0, f = 0; j < R; ++j) {
      n.consts[8 + 4 * R + j] = c[8 + 4 * R + idx[j]];
      if (pair_of[idx[j]] >= 0) {
        n.par[tail0 + 2 * f] = p[tail0 + 2 * pair_of[idx[j]]];
        n.par[tail0 + 2 * f + 1] = p[tail0 + 2 * pair_of[idx[j]] + 1];
        ++f;
      }
    }
  }
}

}  // namespace

}  // namespace hf

using namespace hf;

extern "C" int pdf_graph_create(const hf_obs* obs, int32_t n_obs, const hf_param* par, int32_t n_par,
                                const hf_node* nodes, int32_t n_nodes, int32_t root, pdf_graph** out) {
  try {
    if (!obs || !par || !nodes || !out) return fail(HF_E_INVALID, "pdf_graph_create: NULL argument");
    if (n_obs < 1 || n_obs > 64) return fail(HF_E_INVALID, "pdf_graph_create: n_obs out of range");
    if (n_par < 0 || n_par > kMaxPar) return fail(HF_E_INVALID, "pdf_graph_create: n_par out of range (max 64)");
    if (n_nodes < 1 || n_nodes > kMaxNodes) return fail(HF_E_GRAPH, "pdf_graph_create: 1..16 nodes allowed");
    if (root < 0 || root >= n_nodes) return fail(HF_E_GRAPH, "pdf_graph_create: root index out of range");
    std::unique_ptr<pdf_graph> g(new pdf_graph);
    for (int i = 0; i < n_obs; ++i) {
      const hf_obs& o = obs[i];
      if (std::isnan(o.lo) || std::isnan(o.hi) || !(o.lo < o.hi))
        return fail(HF_E_GRAPH, "observable " + std::to_string(i) + ": need lo < hi");
      g->obs.push_back({o.name ? o.name : "", o.lo, o.hi});
    }
    for (int i = 0; i < n_par; ++i) {
      const hf_param& p = par[i];
      if (!std::isfinite(p.init)) return fail(HF_E_GRAPH, "parameter " + std::to_string(i) + ": init not finite");
      if (p.lo != p.hi && !(p.lo < p.hi)) return fail(HF_E_GRAPH, "parameter " + std::to_string(i) + ": lo > hi");
      if (p.lo != p.hi && (p.init < p.lo || p.init > p.hi))
        return fail(HF_E_GRAPH, "parameter " + std::to_string(i) + ": init outside [lo, hi]");
      g->par.push_back({p.name ? p.name : "", p.init, p.step > 0 ? p.step : 0.1, p.lo, p.hi, p.fixed != 0});
    }
    // copy + per-node checks
    std::vector<NodeInfo> in(n_nodes);
    for (int k = 0; k < n_nodes; ++k) {
      const hf_node& n = nodes[k];
      NodeInfo& ni = in[k];
      ni.op = n.op;
      const std::string where = "node " + std::to_string(k) + ": ";
      if (n.n_child < 0 || n.n_par < 0 || n.n_obs < 0 || n.n_const < 0) return fail(HF_E_GRAPH, where + "negative count");
      if ((n.n_child && !n.child) || (n.n_par && !n.par) || (n.n_obs && !n.obs) || (n.n_const && !n.consts))
        return fail(HF_E_GRAPH, where + "NULL array");
      ni.child.assign(n.child, n.child + n.n_child);
      ni.par.assign(n.par, n.par + n.n_par);
      ni.obs.assign(n.obs, n.obs + n.n_obs);
      ni.consts.assign(n.consts, n.consts + n.n_const);
      for (int c : ni.child)
        if (c < 0 || c >= k) return fail(HF_E_GRAPH, where + "child index must refer to an earlier node");
      for (int p : ni.par)
        if (p < 0 || p >= n_par) return fail(HF_E_GRAPH, where + "parameter index out of range");
      for (int o : ni.obs)
        if (o < 0 || o >= n_obs) return fail(HF_E_GRAPH, where + "observable index out of range");
      auto need = [&](bool ok, const char* m) { return ok ? 0 : fail(HF_E_GRAPH, where + m); };
      auto finite_box = [&](int o) { return std::isfinite(g->obs[o].lo) && std::isfinite(g->obs[o].hi); };
      int rc = 0;
      switch (n.op) {
        case OP_EXP:
          rc = need(n.n_child == 0 && n.n_par == 1 && n.n_obs == 1, "EXP takes 1 parameter and 1 observable");
          if (!rc) rc = need(finite_box(ni.obs[0]), "EXP needs a finite observable box");
          break;
        case OP_GAUSS:
          rc = need(n.n_child == 0 && n.n_par == 2 && n.n_obs == 1, "GAUSS takes 2 parameters and 1 observable");
          if (!rc) rc = need(finite_box(ni.obs[0]), "GAUSS needs a finite observable box");
          break;
        case OP_POLY:
          rc = need(n.n_child == 0 && n.n_par >= 1 && n.n_par <= 8 && n.n_obs == 1 && n.n_const == 1,
                    "POLY takes 1..8 coefficients, 1 observable and the constant x0");
          if (!rc) rc = need(finite_box(ni.obs[0]) && std::isfinite(ni.consts[0]), "POLY needs a finite box and x0");
          break;
        case OP_ADD:
          rc = need(n.n_child >= 2 && n.n_par == n.n_child - 1 && n.n_obs == 0,
                    "ADD takes K >= 2 children and K-1 fractions");
          break;
        case OP_PROD:
          rc = need(n.n_child >= 2 && n.n_par == 0 && n.n_obs == 0, "PROD takes K >= 2 children and no parameters");
          break;
        case OP_MAP: {
          rc = need(n.n_child >= 2 && n.n_par == 0 && n.n_obs == 1 && n.n_const == n.n_child - 1,
                    "MAP takes K >= 2 children, one observable, K-1 boundaries and no parameters");
          if (!rc) rc = need(finite_box(ni.obs[0]), "MAP needs a finite observable box");
          if (!rc) {
            const ObsInfo& o = g->obs[ni.obs[0]];
            double prev = o.lo;
            for (double b : ni.consts) {
              rc = need(std::isfinite(b) && b > prev, "MAP boundaries must increase strictly inside the box");
              if (rc) break;
              prev = b;
            }
            if (!rc) rc = need(prev < o.hi, "MAP boundaries must increase strictly inside the box");
          }
          for (int c : ni.child) {
            if (rc) break;
            const NodeInfo& cn = in[c];
            rc = need((cn.op == OP_EXP || cn.op == OP_GAUSS || cn.op == OP_POLY) && cn.obs.size() == 1 &&
                          cn.obs[0] == ni.obs[0],
                      "MAP children must be EXP / GAUSS / POLY leaves on the MAP's observable");
          }
          break;
        }
        case OP_COMP: {
          // children = (core POLY, shell leaf) on obs
          rc = need(n.n_child == 2 && n.n_par == 0 && n.n_obs == 1 && n.n_const == 0,
                    "COMP takes a core and a shell, one observable, no parameters or constants");
          if (!rc) rc = need(finite_box(ni.obs[0]), "COMP needs a finite observable box");
          if (!rc) {
            const NodeInfo& cc = in[ni.child[0]];
            const NodeInfo& cf = in[ni.child[1]];
            rc = need(cc.op == OP_POLY && cc.obs.size() == 1 && cc.obs[0] == ni.obs[0] && cc.par.size() <= 4 &&
                          (cf.op == OP_EXP || cf.op == OP_GAUSS || cf.op == OP_POLY) && cf.obs.size() == 1 &&
                          cf.obs[0] == ni.obs[0] && cf.par.size() <= 4,
                      "COMP: a POLY core (degree <= 4) and an EXP / GAUSS / POLY shell, both on its observable");
          }
          break;
        }
        case OP_CONV: {
          // consts = (N, d_lo, d_hi); children = (model, resolution) leaves on obs
          rc = need(n.n_child == 2 && n.n_par == 0 && n.n_obs == 1 && n.n_const == 3,
                    "CONV takes a model and a resolution, one observable and (N, d_lo, d_hi)");
          if (!rc) rc = need(finite_box(ni.obs[0]), "CONV needs a finite observable box");
          if (!rc)
            rc = need(ni.consts[0] >= 2 && ni.consts[0] <= kMaxConvGrid && ni.consts[0] == std::floor(ni.consts[0]) &&
                          std::isfinite(ni.consts[1]) && std::isfinite(ni.consts[2]) && ni.consts[1] < ni.consts[2],
                      "CONV: 2..4096 grid points and a residual range d_lo < d_hi");
          for (int j = 0; j < (int)ni.child.size() && !rc; ++j) {
            const NodeInfo& cn = in[ni.child[j]];
            // the resolution may be a mixture of 2 or 3 Gaussians on the
            // observable (each normalised over the residual range)
            if (j == 1 && cn.op == OP_ADD) {
              rc = need(cn.child.size() >= 2 && cn.child.size() <= 3,
                        "a CONV resolution mixture takes 2 or 3 Gaussians");
              for (int c : cn.child) {
                if (rc) break;
                const NodeInfo& gc = in[c];
                rc = need(gc.op == OP_GAUSS && gc.obs.size() == 1 && gc.obs[0] == ni.obs[0],
                          "a CONV resolution mixture takes Gaussians on the convolution's observable");
              }
              continue;
            }
            rc = need((cn.op == OP_EXP || cn.op == OP_GAUSS || cn.op == OP_POLY) && cn.obs.size() == 1 &&
                          cn.obs[0] == ni.obs[0] && cn.par.size() <= 4,
                      "CONV children must be EXP / GAUSS / POLY (degree <= 4) leaves on its observable (the "
                      "resolution also a mixture of Gaussians)");
          }
          break;
        }
        case OP_DPMAP: {
          // obs = (s12, s13, u); consts = (n12, n13, b12..., b13...)
          rc = need(n.n_par == 0 && n.n_obs == 3 && n.n_const >= 2, "DPMAP takes (s12, s13, u), no parameters");
          if (rc) break;
          const double a12 = ni.consts[0], a13 = ni.consts[1];
          rc = need(a12 >= 1 && a13 >= 1 && a12 <= kMaxNodes && a13 <= kMaxNodes && a12 == std::floor(a12) &&
                        a13 == std::floor(a13) && n.n_const == (int)(a12 + a13) &&
                        n.n_child == (int)(a12 * a13) && n.n_child >= 2,
                    "DPMAP: consts (n12, n13, n12-1 s12 boundaries, n13-1 s13 boundaries), n12 x n13 >= 2 children");
          for (int ax = 0; ax < 2 && !rc; ++ax) {
            const int o = ni.obs[ax];
            rc = need(finite_box(o), "DPMAP: s12 and s13 need finite boxes");
            const int nb = (int)(ax == 0 ? a12 : a13) - 1, b0 = ax == 0 ? 2 : 2 + (int)a12 - 1;
            double prev = g->obs[o].lo;
            for (int j = 0; j < nb && !rc; ++j) {
              const double b = ni.consts[b0 + j];
              rc = need(std::isfinite(b) && b > prev, "DPMAP boundaries must increase strictly inside the box");
              prev = b;
            }
            if (!rc) rc = need(prev < g->obs[o].hi, "DPMAP boundaries must increase strictly inside the box");
          }
          for (int c : ni.child) {
            if (rc) break;
            const NodeInfo& cn = in[c];
            rc = need((cn.op == OP_EXP || cn.op == OP_GAUSS || cn.op == OP_POLY) && cn.obs.size() == 1 &&
                          cn.obs[0] == ni.obs[2],
                      "DPMAP children must be EXP / GAUSS / POLY leaves on its third observable");
          }
          break;
        }
        case OP_DALITZ:
        case OP_TDDP: {
          const bool td = n.op == OP_TDDP;
          rc = need(n.n_child == 0 && n.n_const >= 7, "Dalitz node needs the constant block");
          if (rc) break;
          const int R = (int)ni.consts[6];
          const int rmax = td ? kMaxResFull : kMaxRes;
          // the full time-dependent form adds a block of 1 + R constants:
          // flags (1: x, 2: q/p), then 1 for each resonance whose mass and
          // width are parameters
          const bool ext = td && R >= 1 && n.n_const == 8 + 5 * R;
          rc = need(R >= 1 && R <= rmax && (n.n_const == 7 + 4 * R || ext),
                    td ? "time-dependent Dalitz: 1..16 resonances, 7 + 4R (full form 8 + 5R) constants"
                       : "Dalitz: 1..8 resonances, 7 + 4R constants");
          if (!rc && ext) {
            const double fl = ni.consts[7 + 4 * R];
            rc = need(fl == 0 || fl == 1 || fl == 2 || fl == 3, "time-dependent Dalitz: flags must be 0..3");
            int nf = 0;
            for (int j = 0; j < R && !rc; ++j) {
              const double v = ni.consts[8 + 4 * R + j];
              rc = need(v == 0 || v == 1, "time-dependent Dalitz: floating-shape flags must be 0 or 1");
              nf += v == 1;
            }
            if (!rc) rc = need(nf <= kMaxFloat, "time-dependent Dalitz: at most 4 resonances with floating shapes");
            if (!rc) {
              const int hx = ((int)fl & 1) != 0, hq = ((int)fl & 2) != 0;
              rc = need(n.n_par == 2 * R + 2 + hx + 2 * hq + 2 * nf,
                        "time-dependent Dalitz (full form): 2R + tau, y (+ x) (+ |q/p|, arg q/p) + 2 per "
                        "floating resonance parameters");
            }
          } else if (!rc) {
            rc = need(td ? (n.n_par == 2 * R + 2 || n.n_par == 2 * R + 3) : n.n_par == 2 * R,
                      "Dalitz: 2R parameters; time-dependent: 2R + tau, y (+ x)");
          }
          if (!rc) rc = need(n.n_obs == (td ? 4 : 2), "Dalitz: observables (s12, s13[, t, sigma_t])");
          if (!rc) rc = need(finite_box(ni.obs[0]) && finite_box(ni.obs[1]), "Dalitz: s12, s13 need finite boxes");
          if (rc) break;
          const double M = ni.consts[0], m1 = ni.consts[1], m2 = ni.consts[2], m3 = ni.consts[3];
          const double G = ni.consts[5];
          rc = need(m1 > 0 && m2 > 0 && m3 > 0 && M > m1 + m2 + m3 && ni.consts[4] >= 0,
                    "Dalitz: need positive masses with M > m1 + m2 + m3 and r >= 0");
          if (!rc) rc = need(G >= 2 && G <= 4096 && G == std::floor(G), "Dalitz: grid size 2..4096");
          for (int j = 0; j < R && !rc; ++j) {
            const double ch = ni.consts[7 + 4 * j], m0 = ni.consts[8 + 4 * j], g0 = ni.consts[9 + 4 * j],
                         J = ni.consts[10 + 4 * j];
            rc = need(ch == 12 || ch == 13 || ch == 23, "Dalitz: channel must be 12, 13 or 23");
            if (!rc) rc = need(J == 0 || J == 1 || J == 2, "Dalitz: J must be 0, 1 or 2");
            if (!rc) {
              const double mA = ch == 23 ? m2 : m1, mB = ch == 12 ? m2 : m3;
              rc = need(m0 > mA + mB && g0 > 0, "Dalitz: resonance mass above threshold and width > 0");
            }
          }
          if (!rc) group_resonances(ni, R);
          break;
        }
        default:
          rc = fail(HF_E_GRAPH, where + "unknown op");
      }
      if (rc) return rc;
    }
    // a root PROD of a DPMAP and a TDDP node lists the TDDP node first (the
    // product is symmetric; the fused kernel expects it as node 0)
    if (in[root].op == OP_PROD && in[root].child.size() == 2 && in[in[root].child[0]].op == OP_DPMAP &&
        in[in[root].child[1]].op == OP_TDDP)
      std::swap(in[root].child[0], in[root].child[1]);
    // reachable nodes in post-order (children before parents, root last)
    std::vector<int> order, used(n_nodes, 0);
    std::function<int(int)> visit = [&](int k) -> int {
      if (used[k]) return fail(HF_E_GRAPH, "node " + std::to_string(k) + " is used twice");
      used[k] = 1;
      for (int c : in[k].child)
        if (int rc = visit(c)) return rc;
      order.push_back(k);
      return 0;
    };
    if (int rc = visit(root)) return rc;
    if ((int)order.size() > kMaxNodes) return fail(HF_E_GRAPH, "too many nodes");
    std::vector<int> newidx(n_nodes, -1);
    for (size_t i = 0; i < order.size(); ++i) newidx[order[i]] = (int)i;
    for (int k : order) {
      NodeInfo n = in[k];
      for (int& c : n.child) c = newidx[c];
      g->nodes.push_back(n);
    }
    const int NN = (int)g->nodes.size();
    // observable sets; ADD children share one, PROD children are disjoint
    // apart from groups of one-observable leaves
    std::vector<std::set<int>> os(NN);
    std::vector<int> dpmap_ok(NN, 0);
    int n_heavy = 0;
    for (int k = 0; k < NN; ++k) {
      NodeInfo& n = g->nodes[k];
      if (n.op == OP_ADD || n.op == OP_PROD) {
        // PROD: one-observable EXP / GAUSS / POLY children may share their
        // observable (renormalised numerically); a DPMAP child conditions on
        // the (s12, s13) of a DALITZ / TDDP sibling and may describe that
        // TDDP's sigma_t; any other overlap is an error
        std::set<int> leaf_only, claimed;
        int dzc = -1;
        if (n.op == OP_PROD)
          for (int c : n.child)
            if (g->nodes[c].op == OP_DALITZ || g->nodes[c].op == OP_TDDP) dzc = c;
        for (int c : n.child) {
          if (n.op == OP_ADD && os[c] != os[n.child[0]])
            return fail(HF_E_GRAPH, "ADD children must share the same observables");
          // the observables this child adds to the product
          std::set<int> own = os[c];
          if (g->nodes[c].op == OP_DPMAP) {
            const NodeInfo& dm = g->nodes[c];
            if (n.op != OP_PROD || dzc < 0 || g->nodes[dzc].obs[0] != dm.obs[0] ||
                g->nodes[dzc].obs[1] != dm.obs[1])
              return fail(HF_E_GRAPH,
                          "a DPMAP must be a PROD child beside the DALITZ / TDDP node on the same (s12, s13)");
            dpmap_ok[c] = 1;
            own = {dm.obs[2]};
            if (g->nodes[dzc].op == OP_TDDP && g->nodes[dzc].obs[3] == dm.obs[2]) own.clear();
          }
          const bool l1 = is_leaf1(g->nodes[c]);
          for (int o : own) {
            if (n.op == OP_PROD && claimed.count(o) && !(l1 && leaf_only.count(o)))
              return fail(HF_E_GRAPH,
                          "PROD children must have disjoint observables, except one-observable EXP / GAUSS / POLY "
                          "leaves, which may share one");
            if (!claimed.count(o) && l1) leaf_only.insert(o);
            claimed.insert(o);
          }
          for (int o : os[c]) os[k].insert(o);
        }
      } else {
        for (int o : n.obs) {
          if (os[k].count(o)) return fail(HF_E_GRAPH, "a node uses an observable twice");
          os[k].insert(o);
        }
      }
      if (n.op == OP_DALITZ || n.op == OP_TDDP) ++n_heavy;
    }
    if (n_heavy > 1) return fail(HF_E_GRAPH, "at most one DALITZ/TDDP node per graph");
    for (int k = 0; k < NN; ++k)
      if (g->nodes[k].op == OP_DPMAP && !dpmap_ok[k])
        return fail(HF_E_GRAPH, "a DPMAP must be a PROD child beside the DALITZ / TDDP node on the same (s12, s13)");
    // columns: used observables in index order
    g->col_of_obs.assign(n_obs, -1);
    for (int o = 0; o < n_obs; ++o)
      if (os[NN - 1].count(o)) {
        g->col_of_obs[o] = (int)g->obs_of_col.size();
        g->obs_of_col.push_back(o);
      }
    if ((int)g->obs_of_col.size() > kMaxCols) return fail(HF_E_GRAPH, "more than 8 observables used");
    // hoisting: every ancestor is a PROD
    std::vector<int> hoist(NN, 0);
    hoist[NN - 1] = 1;
    for (int k = NN - 1; k >= 0; --k)
      for (int c : g->nodes[k].child) hoist[c] = hoist[k] && g->nodes[k].op == OP_PROD;
    // flatten
    KProgram& P = g->prog;
    std::memset(&P, 0, sizeof(P));
    P.n_nodes = NN;
    P.root = NN - 1;
    P.n_cols = (int)g->obs_of_col.size();
    int slot = 0, cst = 0, chl = 0;
    for (int k = 0; k < NN; ++k) {
      const NodeInfo& n = g->nodes[k];
      KNode& kn = P.node[k];
      kn.op = (int32_t)n.op;
      kn.n_child = (int32_t)n.child.size();
      kn.child0 = (int32_t)chl;
      for (int c : n.child) P.child[chl++] = (int32_t)c;
      kn.slot0 = (int32_t)slot;
      kn.n_slot = (int32_t)node_slots(n);
      kn.c0 = (int32_t)cst;
      for (int j = 0; j < 4; ++j) kn.col[j] = j < (int)n.obs.size() ? (int32_t)g->col_of_obs[n.obs[j]] : 0;
      kn.hoisted = (int32_t)hoist[k];
      kn.aux = 0;
      if (n.op == OP_POLY) kn.aux = (int32_t)n.par.size();
      if (n.op == OP_PROD) kn.aux = shared_groups(g->nodes, n).empty() ? 0 : 1;
      if (n.op == OP_DPMAP) kn.aux = (int32_t)n.consts[1];
      if (n.op == OP_CONV) kn.aux = (int32_t)n.consts[0];
      // ADD: the first children's constant offsets (read with compile-time
      // indices by the CONV resolution mixture, whose Gaussians they are)
      if (n.op == OP_ADD)
        for (int j = 0; j < (int)n.child.size() && j < kNumGroups; ++j) kn.res_end[j] = P.node[n.child[j]].c0;
      if (n.op == OP_DALITZ || n.op == OP_TDDP) {
        const int R = (int)n.consts[6];
        kn.aux = (int32_t)R;
        int cnt[kNumGroups] = {0};
        for (int j = 0; j < R; ++j) ++cnt[res_group_of(n, j)];
        for (int gi = 0, e = 0; gi < kNumGroups; ++gi) kn.res_end[gi] = (int32_t)(e += cnt[gi]);
      }
      // gradient slot -> parameter
      if (n.op == OP_ADD) for (int j = 0; j < kn.n_slot; ++j) g->slot_par.push_back(n.par[j]);
      else for (int j = 0; j < kn.n_slot; ++j) g->slot_par.push_back(n.par[j]);
      slot += kn.n_slot;
      cst += node_consts(g->nodes, n);
      if (slot > kMaxSlots) return fail(HF_E_GRAPH, "more than 48 gradient slots");
      if (cst > kMaxConst) return fail(HF_E_GRAPH, "constant table overflow (too many resonances or nodes)");
    }
    P.n_slots = slot;
    g->n_const = cst;
    // static Dalitz constants
    for (int k = 0; k < NN; ++k) {
      const NodeInfo& n = g->nodes[k];
      if (n.op != OP_DALITZ && n.op != OP_TDDP) continue;
      DalitzInfo& dz = g->dz;
      dz.node = k;
      dz.tddp = n.op == OP_TDDP;
      dz.M = n.consts[0]; dz.m1 = n.consts[1]; dz.m2 = n.consts[2]; dz.m3 = n.consts[3]; dz.r = n.consts[4];
      dz.grid = (int)n.consts[5];
      const int R = (int)n.consts[6];
      for (int j = 0; j < R; ++j)
        dz.res.push_back({(int)n.consts[7 + 4 * j], n.consts[8 + 4 * j], n.consts[9 + 4 * j], (int)n.consts[10 + 4 * j]});
      if (dz.tddp) {
        dz.p_tau = n.par[2 * R];
        dz.p_y = n.par[2 * R + 1];
      }
      if (tddp_full(n)) {
        if (NN != 1) return fail(HF_E_GRAPH, "the full time-dependent Dalitz node must be the graph's only node");
        dz.full = true;
        const bool ext = (int)n.consts.size() == 8 + 5 * R;
        const int flags = ext ? (int)n.consts[7 + 4 * R] : ((int)n.par.size() == 2 * R + 3 ? 1 : 0);
        dz.hx = (flags & 1) != 0;
        dz.hq = (flags & 2) != 0;
        int q = 2 * R + 2;
        if (dz.hx) dz.p_x = n.par[q++];
        if (dz.hq) {
          dz.p_qm = n.par[q++];
          dz.p_qa = n.par[q++];
        }
        for (int j = 0; ext && j < R; ++j)
          if (n.consts[8 + 4 * R + j] == 1) {
            const int ch = (int)n.consts[7 + 4 * j];
            dz.fl.push_back({j, ch == 12 ? 0 : (ch == 13 ? 1 : 2), (int)n.consts[10 + 4 * j], n.par[q], n.par[q + 1]});
            q += 2;
          }
      } else if (dz.tddp && (int)n.par.size() == 2 * R + 3) {
        dz.p_x = n.par[2 * R + 2];
      }
      const double lo12 = (dz.m1 + dz.m2) * (dz.m1 + dz.m2), hi12 = (dz.M - dz.m3) * (dz.M - dz.m3);
      const double lo13 = (dz.m1 + dz.m3) * (dz.m1 + dz.m3), hi13 = (dz.M - dz.m2) * (dz.M - dz.m2);
      dz.gs = GridSpec{lo12, (hi12 - lo12) / dz.grid, lo13, (hi13 - lo13) / dz.grid, dz.M, dz.m1, dz.m2, dz.m3, dz.grid};
      const int c0 = P.node[k].c0;
      auto setc = [&](int i, double v) { P.c64[i] = v; P.c32[i] = (float)v; };
      const double M2 = dz.M * dz.M;
      setc(c0 + kDzSsum, M2 + dz.m1 * dz.m1 + dz.m2 * dz.m2 + dz.m3 * dz.m3);
      setc(c0 + kDzR2, dz.r * dz.r);
      // pair constants: 12 = (m1, m2; spectator m3), 13 = (m1, m3; m2), 23 = (m2, m3; m1)
      const int chb = c0 + dz_ch_base(R, dz.tddp);
      for (int c = 0; c < kNumCh; ++c) {
        double mA, mB, mC;
        pair_masses(dz, c, mA, mB, mC);
        const int cb = chb + c * kChStride;
        setc(cb + kChThrP, (mA + mB) * (mA + mB));
        setc(cb + kChThrM, (mA - mB) * (mA - mB));
        setc(cb + kChZc1, (M2 - mC * mC) * (mB * mB - mA * mA));
        setc(cb + kChZtaC, 2.0 * M2 + 2.0 * mC * mC);
        setc(cb + kChZtaD, (M2 - mC * mC) * (M2 - mC * mC));
        setc(cb + kChZtbC, 2.0 * mA * mA + 2.0 * mB * mB);
        setc(cb + kChZtbD, (mA * mA - mB * mB) * (mA * mA - mB * mB));
      }
      const int rbase = c0 + dz_res_base(R, dz.tddp);
      for (int j = 0; j < R; ++j) {
        const ResInfo& r = dz.res[j];
        const int c = r.ch == 12 ? 0 : (r.ch == 13 ? 1 : 2);
        const int rb = rbase + j * kResStride;
        const ResConst rcn = res_consts(dz, c, r.J, r.m0, r.g0);
        setc(rb + kResM02, rcn.m02);
        setc(rb + kResKwB, rcn.kwb);
        setc(rb + kResSqB, rcn.sqb);
      }
    }
    // the generic slot layout (the tree interpreter's, used by binned datasets)
    g->slot_par_tree = g->slot_par;
    g->n_slots_tree = P.n_slots;
    // parameters that the float path sees rounded to float (through 1/sigma,
    // fractions, rates, coefficients); Gaussian means and the decay time,
    // width and mass differences of the time-dependent density enter through
    // double constants only
    g->par_rounded.assign(g->par.size(), false);
    for (const NodeInfo& n : g->nodes)
      for (size_t j = 0; j < n.par.size(); ++j) {
        const bool exact = (n.op == OP_GAUSS && j == 0) || (n.op == OP_TDDP && j >= 2 * (size_t)n.consts[6]);
        if (!exact) g->par_rounded[n.par[j]] = true;
      }
    // kernel family
    const NodeInfo& rootn = g->nodes[NN - 1];
    bool heavy = g->dz.node >= 0;
    // the general interpreter only (a DPMAP also implies a DALITZ / TDDP node;
    // the light-tree kernels have no DPMAP code)
    for (const NodeInfo& n : g->nodes) heavy = heavy || n.op == OP_CONV || n.op == OP_DPMAP;
    // mixture of single-column EXP/GAUSS leaves: static kernel with its own
    // accumulator layout [3 per child], combined on the host (MixInfo)
    bool mix = rootn.op == OP_ADD && (NN == 3 || NN == 4) && (int)rootn.child.size() == NN - 1 && P.n_cols == 1;
    for (int c : rootn.child)
      if (mix && g->nodes[c].op != OP_EXP && g->nodes[c].op != OP_GAUSS) mix = false;
    if (mix) {
      const int K = (int)rootn.child.size();
      g->mix.K = K;
      g->mix.root = NN - 1;
      for (int j = 0; j < K; ++j) {
        g->mix.child[j] = rootn.child[j];
        g->mix.gauss[j] = g->nodes[rootn.child[j]].op == OP_GAUSS;
      }
      g->slot_par.assign(3 * K, -1);
      P.n_slots = 3 * K;
      int mask = 0;
      for (int j = 0; j < K; ++j)
        if (g->nodes[rootn.child[j]].op == OP_GAUSS) mask |= 1 << j;
      g->kind = (K == 2 ? KIND_MIX2 : KIND_MIX3) + mask;
      *out = g.release();
      return HF_OK;
    }
    if (NN == 1 && rootn.op == OP_EXP) g->kind = KIND_EXP;
    else if (NN == 1 && rootn.op == OP_GAUSS) g->kind = KIND_GAUSS;
    else if (NN == 1 && rootn.op == OP_DALITZ) g->kind = KIND_DALITZ;
    else if (NN == 1 && rootn.op == OP_TDDP && g->dz.full) g->kind = KIND_TDDPF;
    else if (NN == 1 && rootn.op == OP_TDDP)
      g->kind = (int)rootn.par.size() == 2 * (int)rootn.consts[6] + 3 ? KIND_TDDPX : KIND_TDDP;
    else if (NN >= 5 && rootn.op == OP_PROD && rootn.child.size() == 2 && P.node[0].op == OP_TDDP &&
             P.node[NN - 2].op == OP_DPMAP && P.node[NN - 2].n_child == NN - 3 &&
             P.node[NN - 2].col[2] == P.node[0].col[3])
      // TDDP x sigma_t density of the event's Dalitz-plot cell: fused kernel
      g->kind = (int)g->nodes[0].par.size() == 2 * (int)g->nodes[0].consts[6] + 3 ? KIND_TDDPXS : KIND_TDDPS;
    else if (!heavy && P.n_slots <= 8 && P.n_cols <= 2 && NN <= 8) g->kind = KIND_TREE_SMALL;
    else g->kind = g->dz.node >= 0 ? KIND_TREE : KIND_TREE_NOAMP;
    if (g->kind == KIND_TREE_NOAMP) {
      // one CONV node with a grid small enough for the row's LDS table: the
      // interpreter that reads the model's grid values from that table
      int n_conv = 0;
      bool fits = true;
      for (int k = 0; k < P.n_nodes; ++k)
        if (P.node[k].op == OP_CONV) {
          ++n_conv;
          fits = fits && P.node[k].aux <= kConvTab;
        }
      if (n_conv == 1 && fits)
        g->kind = P.n_slots <= 8 && P.n_cols <= 2 && NN <= 8 ? KIND_TREE_CONV_SMALL : KIND_TREE_CONV;
    }
    if ((g->kind == KIND_TREE || g->kind == KIND_TREE_NOAMP || g->kind == KIND_TREE_CONV) &&
        P.n_slots > kMaxSlotsTree)
      return fail(HF_E_GRAPH, "more than 32 gradient slots in a tree of several nodes");
    *out = g.release();
    return HF_OK;
  } catch (const std::exception& e) {
    return fail(HF_E_INVALID, std::string("pdf_graph_create: ") + e.what());
  }
}

extern "C" void pdf_graph_destroy(pdf_graph* g) { delete g; }

extern "C" int pdf_graph_shape(const pdf_graph* g, int32_t* n_obs, int32_t* n_par) {
  if (!g) return fail(HF_E_INVALID, "pdf_graph_shape: NULL graph");
  if (n_obs) *n_obs = (int32_t)g->obs.size();
  if (n_par) *n_par = (int32_t)g->par.size();
  return HF_OK;
}

extern "C" int hf_dalitz_inside(const pdf_graph* g, int32_t node, int64_t n, const double* s12, const double* s13,
                                uint8_t* out) {
  if (!g || (n > 0 && (!s12 || !s13 || !out))) return fail(HF_E_INVALID, "hf_dalitz_inside: NULL argument");
  if (g->dz.node < 0) return fail(HF_E_INVALID, "hf_dalitz_inside: graph has no Dalitz node");
  (void)node;
  for (int64_t i = 0; i < n; ++i) out[i] = dalitz_inside(g->dz, s12[i], s13[i]) ? 1 : 0;
  return HF_OK;
}

extern "C" const char* hf_last_error(void) { return hf::last_error(); }
extern "C" const char* last_error_message(void) { return hf::last_error(); }
extern "C" const char* hf_version(void) { return "hipfit 0.1 (gfx950)"; }
