// Variable-metric minimiser (BFGS with sine transforms for bounded
// parameters), ask/tell form.  See minimiser.h.
#include "minimiser.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace hf {

bool spd_inverse(const std::vector<double>& A, int n, std::vector<double>& inv) {
  std::vector<double> L(A.size(), 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
      if (i == j) {
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        L[i * n + i] = std::sqrt(s);
      } else {
        L[i * n + j] = s / L[j * n + j];
      }
    }
  // inverse of L, then inv = L^-T L^-1
  std::vector<double> Li(A.size(), 0.0);
  for (int i = 0; i < n; ++i) {
    Li[i * n + i] = 1.0 / L[i * n + i];
    for (int j = 0; j < i; ++j) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s -= L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = s / L[i * n + i];
    }
  }
  inv.assign(A.size(), 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += Li[k * n + i] * Li[k * n + j];
      inv[i * n + j] = inv[j * n + i] = s;
    }
  return true;
}

namespace {
bool bounded(const MinParam& p) { return p.lo != p.hi; }
}  // namespace

double Minimiser::to_ext(int j, double u) const {
  const MinParam& p = ps_[j];
  if (!bounded(p)) return u;
  return p.lo + (p.hi - p.lo) * (std::sin(u) + 1.0) * 0.5;
}

double Minimiser::to_int(int j, double x) const {
  const MinParam& p = ps_[j];
  if (!bounded(p)) return x;
  double v = 2.0 * (x - p.lo) / (p.hi - p.lo) - 1.0;
  v = std::min(std::max(v, -1.0 + 1e-9), 1.0 - 1e-9);
  return std::asin(v);
}

double Minimiser::dxdu(int j, double u) const {
  const MinParam& p = ps_[j];
  if (!bounded(p)) return 1.0;
  return (p.hi - p.lo) * 0.5 * std::cos(u);
}

void Minimiser::ext_point(const std::vector<double>& u, std::vector<double>& x) const {
  x = x_best;
  for (int k = 0; k < nf_; ++k) x[free_[k]] = to_ext(free_[k], u[k]);
}

void Minimiser::int_grad(const std::vector<double>& u, const std::vector<double>& gext, std::vector<double>& gu) const {
  gu.resize(nf_);
  for (int k = 0; k < nf_; ++k) gu[k] = gext[free_[k]] * dxdu(free_[k], u[k]);
}

double Minimiser::sigma_ext(int p) const {
  for (int k = 0; k < nf_; ++k)
    if (free_[k] == p) {
      if (!V_.empty() && V_[k * nf_ + k] > 0.0) return std::sqrt(V_[k * nf_ + k]) * std::fabs(dxdu(p, u_[k]));
      return ps_[p].step;
    }
  return ps_[p].step;
}

void Minimiser::start(const std::vector<MinParam>& ps, const double* x0, const MinOptions& o) {
  ps_ = ps;
  o_ = o;
  n_ = (int)ps.size();
  free_.clear();
  for (int j = 0; j < n_; ++j)
    if (!ps[j].fixed) free_.push_back(j);
  nf_ = (int)free_.size();
  x_best.assign(x0, x0 + n_);
  u_.assign(nf_, 0.0);
  for (int k = 0; k < nf_; ++k) u_[k] = to_int(free_[k], x0[free_[k]]);
  // start from the transformed point so that x_best is exactly representable
  for (int k = 0; k < nf_; ++k) x_best[free_[k]] = to_ext(free_[k], u_[k]);
  V_.clear();
  Hext_.clear();
  Cfree_.clear();
  gext_best_.assign(n_, 0.0);
  err.assign(n_, 0.0);
  cov.assign((size_t)n_ * n_, 0.0);
  status = RUNNING;
  phase_ = EVAL0;
  n_iter = n_eval = 0;
  n_fail_ = 0;
  polish_ = 0;
  edm_polish_ = INFINITY;
  f_best = 0.0;
  edm = 0.0;
}

bool Minimiser::ask(std::vector<double>& x) {
  std::vector<double> u;
  switch (phase_) {
    case EVAL0:
      ext_point(u_, x);
      break;
    case HESS0:
      u = u_;
      u[k_] += hstep_[k_];
      ext_point(u, x);
      break;
    case LINE:
      u.resize(nf_);
      for (int k = 0; k < nf_; ++k) u[k] = u0_[k] + alpha_ * p_[k];
      ext_point(u, x);
      break;
    case FINAL_H: {
      x = x_best;
      const int j = free_[k_ / 2];
      x[j] += (k_ % 2 == 0 ? 1.0 : -1.0) * hstep_[k_ / 2];
      break;
    }
    case POLISH:
      x = x_pend_;
      break;
    case DONE:
      return false;
  }
  if (phase_ != POLISH) x_pend_ = x;
  return true;
}

void Minimiser::reset_metric_diag() {
  V_.assign((size_t)nf_ * nf_, 0.0);
  for (int k = 0; k < nf_; ++k) {
    const double d = std::fabs(dxdu(free_[k], u_[k]));
    const double s = ps_[free_[k]].step / std::max(d, 1e-12);
    V_[k * nf_ + k] = s * s;
  }
}

void Minimiser::finish(int st) {
  status = st;
  phase_ = DONE;
  if (Hext_.empty()) {
    // errors from the variable metric when no final Hessian was taken
    for (int k = 0; k < nf_; ++k) {
      const int j = free_[k];
      if (!V_.empty() && V_[k * nf_ + k] > 0.0)
        err[j] = std::sqrt(2.0 * o_.up * V_[k * nf_ + k]) * std::fabs(dxdu(j, u_[k]));
    }
  }
}

// EDM below which the evaluation cannot resolve the minimum: one rounding
// unit of every parameter the evaluation rounds (relative precision eps),
// measured in errors, with a factor 4 of margin; at least edm_tol.
double Minimiser::edm_target() const {
  double r = 0.0;
  for (int k = 0; k < nf_; ++k) {
    const int j = free_[k];
    const double eps = o_.param_eps > 0.0 ? o_.param_eps : (o_.param_eps < 0.0 ? 0.0 : ps_[j].eps);
    if (eps <= 0.0) continue;
    const double sg = sigma_ext(j);
    if (sg > 0.0 && std::isfinite(sg)) r += eps * std::fabs(x_best[j]) / sg;
  }
  return std::max(o_.edm_tol, 2.0 * r * r);
}

void Minimiser::begin_line() {
  p_.assign(nf_, 0.0);
  double slope = 0.0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    slope = 0.0;
    for (int i = 0; i < nf_; ++i) {
      double s = 0.0;
      for (int j = 0; j < nf_; ++j) s -= V_[i * nf_ + j] * gu_[j];
      p_[i] = s;
      slope += s * gu_[i];
    }
    if (slope < 0.0 || attempt == 1) break;
    reset_metric_diag();
  }
  edm = -0.5 * slope;
  if (!(slope < 0.0) || edm < edm_target()) {
    begin_final();
    return;
  }
  if (n_iter >= o_.max_iter) {
    status = MAX_ITER;
    begin_final();
    return;
  }
  u0_ = u_;
  f0_ = f_;
  g0_ = gu_;
  slope0_ = slope;
  alpha_ = 1.0;
  // keep sine-transformed coordinates within one half period per step
  double pmax = 0.0;
  for (int k = 0; k < nf_; ++k)
    if (bounded(ps_[free_[k]])) pmax = std::max(pmax, std::fabs(p_[k]));
  if (pmax > 1.5) alpha_ = 1.5 / pmax;
  alpha_hi_ = -1.0;
  n_back_ = 0;
  phase_ = LINE;
}

// Step of the final Hessian's central differences for parameter j with error
// scale s: a tenth of it (the NLL is close to quadratic over that range, and
// the step is large against rounding noise in the gradient), above the
// parameter's rounding in the evaluation (relative precision eps: kept below
// 1e-4 of the step) and at most a quarter of the distance to a bound.
double Minimiser::hess_step(int j, double s) const {
  if (!(s > 0.0) || !std::isfinite(s)) s = ps_[j].step;
  double h = 0.1 * s;
  h = std::max(h, 1e-12 * (std::fabs(x_best[j]) + 1.0));
  const double eps = o_.param_eps > 0.0 ? o_.param_eps : (o_.param_eps < 0.0 ? 0.0 : ps_[j].eps);
  h = std::max(h, 1e4 * eps * std::fabs(x_best[j]));
  if (bounded(ps_[j])) h = std::min(h, 0.25 * std::min(x_best[j] - ps_[j].lo, ps_[j].hi - x_best[j]));
  return h;
}

void Minimiser::begin_final() {
  if (!o_.want_errors) {
    finish(status == RUNNING ? CONVERGED : status);
    return;
  }
  // first pass: steps from the variable metric's (marginal) errors
  hstep_.assign(nf_, 0.0);
  for (int k = 0; k < nf_; ++k) hstep_[k] = hess_step(free_[k], sigma_ext(free_[k]));
  h_refined_ = false;
  H1_.clear();
  Hcols_.assign((size_t)nf_ * nf_, 0.0);
  k_ = 0;
  phase_ = FINAL_H;
}

// HIPFIT_TRACE=1 prints every evaluation the minimiser is told about.
static bool trace_on() {
  static const bool on = [] {
    const char* v = std::getenv("HIPFIT_TRACE");
    return v && v[0] == '1';
  }();
  return on;
}

void Minimiser::tell(double f, const std::vector<double>& g) {
  ++n_eval;
  if (trace_on()) {
    static const char* names[] = {"EVAL0", "HESS0", "LINE", "FINAL_H", "POLISH", "DONE"};
    std::fprintf(stderr, "[minimiser] eval %d phase %s f %.12g f_best %.12g edm %.3g alpha %.3g\n", n_eval,
                 names[phase_], f, f_best, edm, alpha_);
  }
  switch (phase_) {
    case EVAL0: {
      if (!std::isfinite(f)) {
        finish(FAILED);
        return;
      }
      f_ = f;
      f_best = f;
      gext_best_ = g;
      int_grad(u_, g, gu_);
      if (nf_ == 0) {
        finish(CONVERGED);
        return;
      }
      hstep_.assign(nf_, 0.0);
      for (int k = 0; k < nf_; ++k) {
        const double d = std::fabs(dxdu(free_[k], u_[k]));
        hstep_[k] = 1e-3 * ps_[free_[k]].step / std::max(d, 1e-12);
      }
      Hcols_.assign((size_t)nf_ * nf_, 0.0);
      k_ = 0;
      phase_ = HESS0;
      return;
    }
    case HESS0: {
      std::vector<double> u = u_, gu;
      u[k_] += hstep_[k_];
      if (std::isfinite(f)) {
        int_grad(u, g, gu);
        for (int i = 0; i < nf_; ++i) Hcols_[i * nf_ + k_] = (gu[i] - gu_[i]) / hstep_[k_];
      }
      if (++k_ < nf_) return;
      std::vector<double> H((size_t)nf_ * nf_);
      for (int i = 0; i < nf_; ++i)
        for (int j = 0; j < nf_; ++j) H[i * nf_ + j] = 0.5 * (Hcols_[i * nf_ + j] + Hcols_[j * nf_ + i]);
      if (!spd_inverse(H, nf_, V_)) {
        reset_metric_diag();
        for (int k = 0; k < nf_; ++k)
          if (H[k * nf_ + k] > 0.0) V_[k * nf_ + k] = 1.0 / H[k * nf_ + k];
      }
      begin_line();
      return;
    }
    case LINE: {
      std::vector<double> u(nf_), gu;
      for (int k = 0; k < nf_; ++k) u[k] = u0_[k] + alpha_ * p_[k];
      const double allow = o_.f_noise * (std::fabs(f0_) + 1.0);
      bool armijo = std::isfinite(f) && f <= f0_ + 1e-4 * alpha_ * slope0_ + allow;
      if (!armijo && std::isfinite(f) && f <= f0_ + 100.0 * allow) {
        // f moved by no more than its rounding noise: judge the step by the
        // gradient, with the quadratic-model change f(a) - f(0) = a (phi'(0) + phi'(a)) / 2
        int_grad(u, g, gu);
        double dnew = 0.0;
        for (int k = 0; k < nf_; ++k) dnew += gu[k] * p_[k];
        armijo = 0.5 * alpha_ * (slope0_ + dnew) <= 1e-4 * alpha_ * slope0_;
      }
      if (!armijo) {
        alpha_hi_ = alpha_;
        if (++n_back_ > 40) {
          // no decrease found: at the noise floor of f, or a poor metric
          if (n_fail_++ == 0) {
            reset_metric_diag();
            begin_line();
          } else {
            if (edm > 10.0 * edm_target()) status = MAX_ITER;
            begin_final();
          }
          return;
        }
        double a = 0.2 * alpha_;
        if (std::isfinite(f)) {
          const double den = 2.0 * (f - f0_ - slope0_ * alpha_);
          if (den > 0.0) a = -slope0_ * alpha_ * alpha_ / den;
          a = std::min(std::max(a, 0.1 * alpha_), 0.5 * alpha_);
        }
        alpha_ = a;
        return;
      }
      int_grad(u, g, gu);
      // BFGS update of the inverse Hessian
      std::vector<double> s(nf_), y(nf_), Vy(nf_, 0.0);
      double sy = 0.0, ss = 0.0, yy = 0.0;
      for (int k = 0; k < nf_; ++k) {
        s[k] = u[k] - u0_[k];
        y[k] = gu[k] - g0_[k];
        sy += s[k] * y[k];
        ss += s[k] * s[k];
        yy += y[k] * y[k];
      }
      if (sy > 1e-14 * std::sqrt(ss * yy)) {
        const double rho = 1.0 / sy;
        double yVy = 0.0;
        for (int i = 0; i < nf_; ++i) {
          for (int j = 0; j < nf_; ++j) Vy[i] += V_[i * nf_ + j] * y[j];
          yVy += y[i] * Vy[i];
        }
        for (int i = 0; i < nf_; ++i)
          for (int j = 0; j < nf_; ++j)
            V_[i * nf_ + j] += rho * ((1.0 + rho * yVy) * s[i] * s[j] - (Vy[i] * s[j] + s[i] * Vy[j]));
      }
      u_ = u;
      f_ = f;
      gu_ = gu;
      ext_point(u_, x_best);
      f_best = f;
      gext_best_ = g;
      ++n_iter;
      begin_line();
      return;
    }
    case FINAL_H: {
      const int k = k_ / 2;
      if (k_ % 2 == 0) {
        gplus_ = g;
      } else {
        for (int i = 0; i < nf_; ++i) {
          const int j = free_[i];
          Hcols_[i * nf_ + k] = std::isfinite(f) ? (gplus_[j] - g[j]) / (2.0 * hstep_[k]) : NAN;
        }
      }
      if (++k_ < 2 * nf_) return;
      Hext_.assign((size_t)nf_ * nf_, 0.0);
      for (int i = 0; i < nf_; ++i)
        for (int j = 0; j < nf_; ++j) Hext_[i * nf_ + j] = 0.5 * (Hcols_[i * nf_ + j] + Hcols_[j * nf_ + i]);
      if (!h_refined_) {
        // second pass where a parameter's conditional error sqrt(2 up / H_jj)
        // is much smaller than its marginal one (strongly correlated
        // parameters): the first steps were long against the range over
        // which the NLL is quadratic along that parameter alone
        h_refined_ = true;
        bool again = false;
        std::vector<double> hn(nf_);
        for (int k = 0; k < nf_; ++k) {
          const double hkk = Hext_[k * nf_ + k];
          hn[k] = hkk > 0.0 && std::isfinite(hkk) ? hess_step(free_[k], std::sqrt(2.0 * o_.up / hkk)) : hstep_[k];
          again = again || hn[k] < 0.5 * hstep_[k];
        }
        if (again) {
          H1_ = Hext_;
          hstep_ = hn;
          k_ = 0;
          return;
        }
      } else if (!H1_.empty()) {
        // the shorter steps cost more rounding noise in the gradient; they
        // are kept only where they change an error by more than 1 % (the
        // NLL is not quadratic over the first steps), else the first
        // pass's Hessian stands
        std::vector<double> C1, C2;
        if (spd_inverse(H1_, nf_, C1) && spd_inverse(Hext_, nf_, C2)) {
          double dmax = 0.0;
          for (int a = 0; a < nf_; ++a)
            dmax = std::max(dmax, std::fabs(std::sqrt(C2[a * nf_ + a] / C1[a * nf_ + a]) - 1.0));
          if (!(dmax > 1e-2)) Hext_ = H1_;
        }
        H1_.clear();
      }
      std::vector<double> C;
      if (!spd_inverse(Hext_, nf_, C)) {
        Hext_.clear();
        finish(status == RUNNING ? CONVERGED : status);
        return;
      }
      Cfree_ = C;
      for (int a = 0; a < nf_; ++a) {
        // covariance 2 up H^-1 (up = 0.5: likelihoods, 1: chi^2)
        err[free_[a]] = std::sqrt(2.0 * o_.up * C[a * nf_ + a]);
        for (int b = 0; b < nf_; ++b) cov[(size_t)free_[a] * n_ + free_[b]] = 2.0 * o_.up * C[a * nf_ + b];
      }
      start_polish();
      return;
    }
    case POLISH: {
      const double allow = o_.f_noise * (std::fabs(f_best) + 1.0);
      bool ok = std::isfinite(f) && f <= f_best + allow;
      if (!ok && std::isfinite(f) && f <= f_best + 100.0 * allow) {
        // within the noise of f: trapezoid estimate of the change from the gradients
        double d = 0.0;
        for (int k = 0; k < nf_; ++k) {
          const int j = free_[k];
          d += 0.5 * (g[j] + gext_best_[j]) * (x_pend_[j] - x_best[j]);
        }
        ok = d <= 0.0;
      }
      if (ok) {
        x_best = x_pend_;
        f_best = f;
        gext_best_ = g;
        for (int k = 0; k < nf_; ++k) u_[k] = to_int(free_[k], x_best[free_[k]]);
        ++polish_;
        start_polish();
      } else {
        finish(status == RUNNING ? CONVERGED : status);
      }
      return;
    }
    case DONE:
      return;
  }
}

// Newton step with the final Hessian while the exact EDM is above tolerance.
void Minimiser::start_polish() {
  double e = 0.0;
  std::vector<double> step(nf_, 0.0);
  for (int a = 0; a < nf_; ++a) {
    for (int b = 0; b < nf_; ++b) step[a] += Cfree_[a * nf_ + b] * gext_best_[free_[b]];
    e += 0.5 * gext_best_[free_[a]] * step[a];
  }
  const double prev = edm_polish_;
  edm = e;
  edm_polish_ = e;
  // Newton steps with the exact Hessian shrink the EDM quadratically; when a
  // step no longer does, the gradient is at its rounding-noise floor and the
  // point is as good as the evaluation allows (accepted if within ~5e-4 sigma)
  const bool floor = polish_ >= 1 && e > 0.25 * prev && e < 1e-7;
  const double tgt = edm_target();
  if (edm < tgt || floor || polish_ >= 3) {
    int st = status;
    const bool ok = edm < 10.0 * tgt || floor;
    if (st == RUNNING) st = ok ? CONVERGED : MAX_ITER;
    else if (st == MAX_ITER && ok) st = CONVERGED;
    finish(st);
    return;
  }
  x_pend_ = x_best;
  for (int a = 0; a < nf_; ++a) {
    const int j = free_[a];
    double v = x_best[j] - step[a];
    if (bounded(ps_[j])) v = std::min(std::max(v, ps_[j].lo), ps_[j].hi);
    x_pend_[j] = v;
  }
  phase_ = POLISH;
}

}  // namespace hf
