// fit(): one maximum-likelihood fit driven through the minimiser state
// machine (the FitManager role of the paper's section "GooFit code").
// grad_mode 0 uses the analytic adjoint gradient (nll_grad); grad_mode 1 is
// the plain numerical path: central differences of nll_eval, 2 n_free extra
// evaluations per gradient.
#include <cmath>
#include <algorithm>
#include <cstring>
#include <vector>

#include "minimiser.h"
#include "runtime.h"

namespace hf {

std::vector<MinParam> min_params(const pdf_graph* g, hf_precision prec) {
  std::vector<MinParam> ps;
  for (size_t i = 0; i < g->par.size(); ++i) {
    const auto& p = g->par[i];
    ps.push_back({p.init, p.step, p.lo, p.hi, p.fixed, prec == HF_FP32_EVAL && g->par_rounded[i] ? 0x1p-24 : 0.0});
  }
  return ps;
}

MinOptions min_options(const hf_fit_opts* o, hf_precision prec) {
  MinOptions m;
  if (o) {
    if (o->max_iter > 0) m.max_iter = o->max_iter;
    if (o->edm_tol > 0) m.edm_tol = o->edm_tol;
    m.want_errors = o->want_errors != 0;
  }
  // the float path's NLL carries rounding noise of order sqrt(n) 1e-7 |ln P|:
  // let the line search accept steps within that noise and stop on the gradient
  m.f_noise = prec == HF_FP32_EVAL ? 1e-9 : 1e-13;
  // 0: per-parameter defaults (min_params); > 0 overrides; < 0: all exact
  m.param_eps = o ? o->param_eps : 0.0;
  return m;
}

int status_code(int st) {
  switch (st) {
    case Minimiser::CONVERGED: return HF_OK;
    case Minimiser::MAX_ITER: return HF_E_NOT_CONVERGED;
    default: return HF_E_DOMAIN;
  }
}

}  // namespace hf

using namespace hf;

extern "C" int fit(const pdf_graph* g, const dataset* d, const hf_fit_opts* opts, void* hip_stream,
                   double* params_inout, double* errors_out, double* cov_out, hf_fit_summary* summary) {
  try {
    if (!g || !d || !params_inout) return fail(HF_E_INVALID, "fit: NULL argument");
    if (d->g != g) return fail(HF_E_SHAPE, "fit: dataset was uploaded for another graph");
    const int np = (int)g->par.size();
    for (int p = 0; p < np; ++p)
      if (!std::isfinite(params_inout[p])) return fail(HF_E_INVALID, "fit: start value not finite");
    const int mode = opts ? opts->grad_mode : 0;
    if (mode != 0 && mode != 1) return fail(HF_E_INVALID, "fit: grad_mode must be 0 or 1");
    hipStream_t st = (hipStream_t)hip_stream;
    Minimiser m;
    MinOptions mo = min_options(opts, d->prec);
    if (d->metric == HF_METRIC_CHI2) {
      mo.up = 1.0;
      // chi^2 amplifies the rounding of ln P by (w - K P) K P / w per bin: in
      // the float path its noise is ~1e-6 of the value, not ~1e-9
      if (d->prec == HF_FP32_EVAL) mo.f_noise = 1e-5;
    }
    m.start(min_params(g, d->prec), params_inout, mo);
    std::vector<double> x(np), gr(np), xp(np);
    int n_eval = 0;
    while (m.ask(x)) {
      double f = 0.0;
      int rc;
      if (mode == 0) {
        rc = eval_one(g, d, x.data(), st, true, &f, gr.data());
        ++n_eval;
      } else {
        rc = eval_one(g, d, x.data(), st, false, &f, nullptr);
        ++n_eval;
        for (int p = 0; p < np && rc == HF_OK; ++p) {
          gr[p] = 0.0;
          if (g->par[p].fixed) continue;
          const double sg = m.sigma_ext(p);
          double h = 1e-3 * (sg > 0 && std::isfinite(sg) ? sg : g->par[p].step);
          h = std::max(h, 1e-10 * (std::fabs(x[p]) + 1.0));
          double fp = 0.0, fm = 0.0;
          xp = x;
          xp[p] = x[p] + h;
          int r1 = eval_one(g, d, xp.data(), st, false, &fp, nullptr);
          xp[p] = x[p] - h;
          int r2 = eval_one(g, d, xp.data(), st, false, &fm, nullptr);
          n_eval += 2;
          if (r1 == HF_E_DOMAIN || r2 == HF_E_DOMAIN) { f = INFINITY; break; }
          if (r1 != HF_OK) { rc = r1; break; }
          if (r2 != HF_OK) { rc = r2; break; }
          gr[p] = (fp - fm) / (2.0 * h);
        }
      }
      if (rc == HF_E_DOMAIN) f = INFINITY;
      else if (rc != HF_OK) return rc;
      m.tell(f, gr);
    }
    std::memcpy(params_inout, m.x_best.data(), np * sizeof(double));
    if (errors_out) std::memcpy(errors_out, m.err.data(), np * sizeof(double));
    if (cov_out) std::memcpy(cov_out, m.cov.data(), (size_t)np * np * sizeof(double));
    if (summary) {
      summary->nll = m.f_best;
      summary->edm = m.edm;
      summary->n_iter = m.n_iter;
      summary->n_eval = n_eval;
      summary->status = status_code(m.status);
    }
    const int rc = status_code(m.status);
    if (rc == HF_E_NOT_CONVERGED) set_error("fit: iteration limit reached");
    if (rc == HF_E_DOMAIN) set_error("fit: start point outside the density's domain");
    return rc;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("fit: ") + ex.what());
  }
}

extern "C" int hf_minimize(int32_t n, const hf_param* params, const double* x0, const hf_fit_opts* opts,
                           double f_noise, hf_fg_fn fn, void* user, double* x_out, double* errors_out,
                           double* cov_out, hf_fit_summary* summary) {
  try {
    if (n < 0 || n > kMaxPar || (n > 0 && !params) || !fn || !x_out)
      return fail(HF_E_INVALID, "hf_minimize: bad argument");
    std::vector<MinParam> ps;
    std::vector<double> start(n);
    for (int i = 0; i < n; ++i) {
      const hf_param& p = params[i];
      ps.push_back({p.init, p.step > 0 ? p.step : 0.1, p.lo, p.hi, p.fixed != 0, 0.0});
      start[i] = x0 ? x0[i] : p.init;
      if (!std::isfinite(start[i])) return fail(HF_E_INVALID, "hf_minimize: start value not finite");
    }
    MinOptions mo = min_options(opts, HF_FP64);
    if (f_noise > 0) mo.f_noise = f_noise;
    Minimiser m;
    m.start(ps, start.data(), mo);
    std::vector<double> x(n), g(n);
    while (m.ask(x)) {
      double f = 0.0;
      std::fill(g.begin(), g.end(), 0.0);
      if (fn(x.data(), &f, g.data(), user) != 0) return fail(HF_E_INVALID, "hf_minimize: callback failed");
      m.tell(f, g);
    }
    std::memcpy(x_out, m.x_best.data(), n * sizeof(double));
    if (errors_out) std::memcpy(errors_out, m.err.data(), n * sizeof(double));
    if (cov_out) std::memcpy(cov_out, m.cov.data(), (size_t)n * n * sizeof(double));
    if (summary) {
      summary->nll = m.f_best;
      summary->edm = m.edm;
      summary->n_iter = m.n_iter;
      summary->n_eval = m.n_eval;
      summary->status = status_code(m.status);
    }
    return status_code(m.status);
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("hf_minimize: ") + ex.what());
  }
}
