// Host runtime objects behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hipfit.h"
#include "internal.h"
#include "kernels.h"

namespace hf {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

struct ObsInfo { std::string name; double lo, hi; };
struct ParInfo { std::string name; double init, step, lo, hi; bool fixed; };

struct NodeInfo {
  int op;
  std::vector<int> child, par, obs;
  std::vector<double> consts;
};

// Resonance description (Dalitz nodes).
struct ResInfo { int ch; double m0, g0; int J; };
// A resonance of the full time-dependent model whose mass and width are
// parameters: its place in the grouped order, pair (0, 1, 2 for 12, 13,
// 23), spin and the two parameter indices.
struct FloatRes { int place, pair, J, p_m0, p_g0; };

struct DalitzInfo {
  int node = -1;          // index of the DALITZ / TDDP node
  bool tddp = false;
  double M, m1, m2, m3, r;
  int grid;
  std::vector<ResInfo> res;
  GridSpec gs;
  bool ready = false;     // matrices computed
  // I, Ibar, J (na x na complex, area included), row-major
  std::vector<double> I, Ib, J;
  // full time-dependent model (KIND_TDDPF): x and q/p present, their
  // parameters, the floating resonances; with floating shapes the
  // normalisation is the grid kernel's sum at every evaluation over the
  // cells inside the plot (device list, made with the first call), into
  // norm_rows rows of partials that each dataset holds (dataset::norm_partials)
  bool full = false, hx = false, hq = false;
  int p_tau = -1, p_y = -1, p_x = -1, p_qm = -1, p_qa = -1;
  std::vector<FloatRes> fl;
  int32_t norm_rows = 0;
  int32_t norm_cols = 0;
  uint32_t* norm_cells = nullptr;  // the grid cells inside the plot, (i << 16) | j (device)
  int64_t n_norm_cells = 0;
};

// Host-side terms added after the device reduction (normalisations of the
// nodes whose ancestors are all products).
struct HostTerms {
  double lnN = 0.0;                 // per event
  std::vector<double> dlnN;         // per event, per parameter
};

// Root ADD of K single-column EXP / GAUSS leaves evaluated by the static
// mixture kernel: per child the kernel sums q, q z (EXP: q x) and q z^2,
// which the host turns into parameter derivatives.
struct MixInfo {
  int K = 0;            // 0: not a mixture
  int root = -1;
  int child[3] = {-1, -1, -1};
  bool gauss[3] = {false, false, false};
};

struct StagedCall {
  KProgram prog;                    // structure + constants for this call
  HostTerms ht;
  bool ok = true;                   // false: parameters outside the density's domain
  bool grid_norm = false;           // the full model's normalisation comes from the grid kernel
  double tint[4] = {0, 0, 0, 0};    // ... with these time integrals kc, kz, ks, kzs
};

}  // namespace hf

struct pdf_graph {
  std::vector<hf::ObsInfo> obs;
  std::vector<hf::ParInfo> par;
  std::vector<hf::NodeInfo> nodes;   // post-order, root last (re-indexed)
  hf::KProgram prog;                 // structure; static constants filled
  std::vector<int> slot_par;         // gradient slot -> parameter index
  std::vector<int> slot_par_tree;    // the same for the tree interpreter's slot layout
  int n_slots_tree = 0;
  std::vector<bool> par_rounded;     // parameter reaches the float kernels rounded to float
  int kind = 0;
  int n_const = 0;
  std::vector<int> col_of_obs;       // observable -> column (-1: unused)
  std::vector<int> obs_of_col;
  hf::DalitzInfo dz;
  hf::MixInfo mix;
  std::mutex grid_mu;
  ~pdf_graph() {
    if (dz.norm_cells) (void)hipFree(dz.norm_cells);
  }
};

struct dataset {
  const pdf_graph* g = nullptr;
  hf_precision prec = HF_FP64;
  int64_t n = 0;
  int n_cols = 0;
  void* block = nullptr;                      // device allocation (columns + partials)
  const void* col[hf::kMaxCols] = {nullptr};
  double ref[hf::kMaxCols] = {0.0};           // per-column reference (float path)
  double* partials = nullptr;
  int32_t n_rows = 0;                         // one block per row (see rows_for)
  int64_t bytes = 0;
  double* res_host = nullptr;                 // pinned, device-mapped: result row, then the completion flag
  double* norm_partials = nullptr;            // full model with floating shapes: the grid kernel's rows (device)
  double* res_dev = nullptr;
  int64_t seq = 0;                            // completion flag value of the last evaluation
  int metric = 0;                             // 0: unbinned; 1 binned NLL; 2 chi^2 (HF_METRIC_*)
  const double* wcol = nullptr;               // binned: weights (device, in the block)
  double wsum = 0.0, volume = 0.0;            // binned: total weight, bin volume
};

namespace hf {

// Column reference used by the float path (0 for unbounded observables).
double column_ref(const pdf_graph* g, int col, hf_precision prec);
// Fills the constant table of `sc.prog` for parameters `theta`.
// generic: constants for the tree interpreter even when the graph has a
// static mixture kernel (binned datasets).
void stage(const pdf_graph* g, const double* theta, hf_precision prec, StagedCall& sc, bool generic = false);
// Makes sure the Dalitz normalisation matrices exist (runs the grid kernels once).
int ensure_grid(pdf_graph* g, hipStream_t st);
// Host membership test of the Dalitz plot (same rule as the grid).
bool dalitz_inside(const DalitzInfo& dz, double s12, double s13);
// nll / gradient on one dataset (want_grad false: NLL-only kernels).
int eval_one(const pdf_graph* g, const dataset* d, const double* theta, hipStream_t st, bool want_grad, double* nll,
             double* grad);
int n_free(const pdf_graph* g);
// Rows of a dataset of n events for a graph of kernel kind `kind` in
// precision `prec` on the current device.
int32_t rows_for(int kind, hf_precision prec, int64_t n);
// NLL and gradient from the reduced sums [sum(-ln P), slot sums] of one
// evaluation (sums may be null for an empty dataset); grad may be null.
void assemble(const pdf_graph* g, const StagedCall& sc, const double* sums, int64_t n, double* nll, double* grad);
// The same for a binned dataset: sums = [metric, slot sums, sum of dmetric/dlnP]
// over the tree interpreter's slots.
void assemble_binned(const pdf_graph* g, const StagedCall& sc, const double* sums, double* value, double* grad);

}  // namespace hf
