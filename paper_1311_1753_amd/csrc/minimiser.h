// Quasi-Newton minimiser written as a resumable state machine.
//
// The paper hands the likelihood to MINUIT's variable-metric Migrad
// (section "GooFit code": FitManager defines the parameters and calls
// mnmigr).  This replacement keeps Migrad's structure -- a variable-metric
// (BFGS) update of the inverse Hessian, sine transforms for bounded
// parameters, the estimated distance to minimum EDM = g^T V g / 2 as the stop
// rule, and a final Hessian for the errors -- but asks for one
// (value, gradient) pair at a time through ask()/tell(), so that a single
// fit, or hundreds of fits batched into one GPU launch, drive the same code.
#pragma once
#include <cstdint>
#include <vector>

namespace hf {

struct MinParam {
  double init, step, lo, hi;  // lo == hi: unbounded
  bool fixed;
  double eps = 0.0;           // relative precision with which the evaluation sees it (0: exact)
};

struct MinOptions {
  int max_iter = 500;
  double edm_tol = 1e-10;
  bool want_errors = true;
  double f_noise = 1e-13;  // relative noise of f tolerated by the line search
  double param_eps = 0.0;  // > 0: overrides every MinParam::eps; < 0: all exact
  double up = 0.5;         // objective change that defines one error (0.5: likelihoods, 1: chi^2)
};

class Minimiser {
 public:
  enum Status { RUNNING = 0, CONVERGED = 1, MAX_ITER = 2, FAILED = 3 };

  void start(const std::vector<MinParam>& ps, const double* x0, const MinOptions& o);
  // Fills x (all parameters, external values) with the next point at which
  // the caller must evaluate f and its gradient; false once finished.
  bool ask(std::vector<double>& x);
  // Result at the point of the last ask(); g has all parameters (entries of
  // fixed parameters are ignored).  A non-finite f means "outside the domain".
  void tell(double f, const std::vector<double>& g);

  // current estimate of the error of each parameter (external units)
  double sigma_ext(int p) const;

  int status = RUNNING;
  bool done() const { return phase_ == DONE; }
  std::vector<double> x_best;        // external
  std::vector<double> err, cov;      // external; cov is n x n row-major
  double f_best = 0.0, edm = 0.0;
  int n_iter = 0, n_eval = 0;

 private:
  enum Phase { EVAL0, HESS0, LINE, FINAL_H, POLISH, DONE };
  int n_ = 0, nf_ = 0;
  std::vector<MinParam> ps_;
  std::vector<int> free_;            // indices of free parameters
  MinOptions o_;
  Phase phase_ = EVAL0;
  // internal state
  std::vector<double> u_, gu_, V_;   // internal point, gradient, inverse Hessian (nf x nf)
  double f_ = 0.0;
  std::vector<double> u0_, g0_;      // start of current line search
  double f0_ = 0.0;
  std::vector<double> p_;            // search direction
  double alpha_ = 1.0, slope0_ = 0.0, alpha_hi_ = -1.0;
  int n_back_ = 0, n_ext_ = 0, n_fail_ = 0;
  int k_ = 0;                        // column counter for Hessians
  std::vector<double> hstep_, Hcols_, gplus_;
  bool h_refined_ = false;  // the final Hessian's second pass (conditional-error steps) was taken
  std::vector<double> H1_;  // the first pass's Hessian while the second runs
  double hess_step(int j, double s) const;
  std::vector<double> x_pend_;       // point handed out by ask()
  int polish_ = 0;
  double edm_polish_ = 0.0;          // EDM before the last Newton polish
  std::vector<double> Hext_;         // final external Hessian (free parameters)
  std::vector<double> Cfree_;        // its inverse
  std::vector<double> gext_best_;    // gradient at x_best (external)

  double to_ext(int j, double u) const;
  double to_int(int j, double x) const;
  double dxdu(int j, double u) const;
  void ext_point(const std::vector<double>& u, std::vector<double>& x) const;
  void int_grad(const std::vector<double>& u, const std::vector<double>& gext, std::vector<double>& gu) const;
  void reset_metric_diag();
  void begin_line();
  double edm_target() const;
  void begin_final();
  void finish(int st);
  void start_polish();
};

// Symmetric positive-definite inverse via Cholesky; false if not PD.
bool spd_inverse(const std::vector<double>& A, int n, std::vector<double>& inv);

}  // namespace hf
