// Host-side entry points of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hf {

// Kernel family chosen for a graph at creation.
enum KernelKind {
  KIND_EXP = 0,         // single EXP leaf
  KIND_GAUSS = 1,       // single GAUSS leaf
  KIND_TREE_SMALL = 2,  // tree of light nodes, <= 8 gradient slots, <= 2 columns
  KIND_DALITZ = 3,      // single DALITZ leaf
  KIND_TDDP = 4,        // single TDDP leaf
  KIND_TREE = 5,        // any tree
  KIND_TDDPX = 6,       // single TDDP leaf with x free (trigonometric terms)
  KIND_TDDPS = 7,       // PROD of a TDDP leaf (x = 0) and a DPMAP on its s12, s13, sigma_t
  KIND_TDDPXS = 12,     // the same with x free
  KIND_TREE_NOAMP = 13, // any tree without DALITZ / TDDP nodes (the general interpreter minus the amplitude code)
  KIND_TDDPF = 14,      // single TDDP leaf of the full model (up to 16 resonances, q/p, floating shapes)
  KIND_TREE_CONV = 15,  // KIND_TREE_NOAMP with one CONV node of at most kConvTab grid points (model staged in LDS)
  // root ADD of 2 (3) single-column EXP/GAUSS leaves: KIND_MIX2 (KIND_MIX3)
  // plus a mask with bit j set when child j is a GAUSS
  KIND_MIX2 = 8,
  KIND_MIX3 = 16,
  // KIND_TREE_CONV within the light trees' sizes (at most 8 nodes, 8 slots,
  // 2 columns): the staged-model interpreter with arrays of that size
  KIND_TREE_CONV_SMALL = 24,
  KIND_COUNT = 25
};

// Rows (blocks) per dataset: at most kRowsPerCU per compute unit (fewer when
// fewer blocks of the kind's kernels fit on a compute unit at once, so that
// every row is resident from the start), and at least kMinChunksLight chunks
// of 256 events per row for the light kinds.
constexpr int kRowsPerCU = 4;
constexpr int kMinChunksLight = 4;

// true for the single-column kinds (EXP, GAUSS, small trees, mixtures)
bool kind_light(int kind);
// Blocks of a kind's kernels that fit on one compute unit at once (current
// device); 0 when unknown (mixtures, or the occupancy query failed).
int resident_blocks_per_cu(int kind, bool fp32);

// e0 / e1 (nullable): events that receive the dispatch's start / end time
hipError_t launch_eval(int kind, bool fp32, bool grad, const EvalArgs& a, hipStream_t st, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr);
// Terms launch of nll_terms: a.n_rows = the dataset's chunks (one per row);
// a.partials receives [1 + accumulators][n_rows x 256] per-event terms.
hipError_t launch_terms(int kind, bool fp32, const EvalArgs& a, hipStream_t st);
hipError_t launch_reduce_one(const FitRec& fr, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Binned datasets: the tree interpreter with the binned metric; `heavy`
// selects the general instantiation (32 slots, 8 columns): 1 without, 2 with
// the amplitude nodes.
hipError_t launch_binned(bool fp32, bool grad, int heavy, const EvalArgs& a, hipStream_t st, hipEvent_t e0 = nullptr,
                         hipEvent_t e1 = nullptr);
hipError_t launch_reduce(const FitRec* fits_dev, int n_fits, hipStream_t st);
hipError_t launch_eval_batched(int kind, bool fp32, const KProgram& prog, const BatchHeader* hdr_dev, const double* c64,
                               const float* c32, int n_const, int grid, hipStream_t st);

// Device-side toy generation.  Factors (the children of a root PROD, or the
// root alone) each fill one column; a factor is one leaf, or an ADD of up to
// kMaxGenLeaf leaves on one observable picked with the cumulative fractions.
constexpr int kMaxGenLeaf = 4;
constexpr int kMaxGenLeaves = kMaxCols * kMaxGenLeaf;
struct GenLeaf {
  int32_t op;        // OP_EXP or OP_GAUSS
  int32_t pad;
  double cum;        // cumulative fraction up to this leaf (the factor's last leaf: unused)
  double lo, hi;     // the observable's box
  double p0, p1, p2, p3;  // EXP: alpha, e^{alpha L} - 1; GAUSS: mu, sqrt(2) sigma, erf(z_lo), erf(z_hi)
};
struct GenArgs {
  int64_t n;
  uint32_t key0, key1;                 // Philox key (the seed's low and high words)
  int32_t n_factor, fp32;
  int32_t first[kMaxCols], n_leaf[kMaxCols], col[kMaxCols];
  double ref[kMaxCols];                // FP32-eval storage reference per factor's column
  void* out[kMaxCols];                 // per factor: its column (double, or float offsets)
  GenLeaf leaf[kMaxGenLeaves];
};
hipError_t launch_generate(const GenArgs& a, hipStream_t st);

// Accept-reject toy generation for any graph whose observables have finite
// boxes: candidates uniform over the columns' boxes, the density from the
// tree interpreter in double (FP64 constants of `prog`).
struct GenArArgs {
  KProgram prog;
  int64_t n;
  uint32_t key0, key1;
  int32_t max_trials, n_cols, fp32, dalitz;  // dalitz: test (s12, s13) = columns c12, c13
  int32_t c12, c13;
  double lo[kMaxCols], hi[kMaxCols], ref[kMaxCols];
  double env, ln_hoist;        // envelope; normalisation applied on the host (subtracted here)
  double M, m1, m2, m3;        // Dalitz kinematics
  void* out[kMaxCols];
  int32_t* fail;               // bit 0: trials exhausted; bit 1: density above the envelope
};
static_assert(sizeof(GenArArgs) <= 4096, "kernel arguments are limited to 4 KiB");
hipError_t launch_generate_ar(const GenArArgs& a, hipStream_t st);

// Dalitz normalisation grid: M[w][p][q] for w in {I, Ibar, J} (n_mat of them),
// complex, unscaled by the cell area.  `out_host` receives n_mat * na * na * 2
// doubles.  Blocking.
struct GridSpec {
  double lo12, h12, lo13, h13;   // cell centre = lo + (i + 0.5) h
  double M, m1, m2, m3;
  int grid;
};
hipError_t dalitz_grid_matrices(const GridSpec& gs, const KProgram& prog, int node, bool tddp, double* out_host,
                                hipStream_t st);

// The full time-dependent model: its likelihood kernels (tm: terms launch)
// and, with floating resonance shapes, the grid normalisation at the
// current parameters (see full_kernels.hip): partials receive
// [|A|^2, 2R coefficient derivatives, |Abar'|^2, a_s, b_s, (|q/p|, arg q/p),
// (m0, Gamma0 per floating resonance)] per row, before the cell area.
struct NormArgs {
  KProgram prog;      // the evaluation's constants, column references 0
  GridSpec gs;
  const uint32_t* cells;  // the cells inside the plot, (i << 16) | j
  int64_t n_cells;
  double* partials;       // [column][row]
  int32_t n_rows;
};
static_assert(sizeof(NormArgs) <= 4096, "kernel arguments are limited to 4 KiB");
hipError_t launch_full_leaf(bool fp32, bool grad, bool tm, const EvalArgs& a, hipStream_t st, hipEvent_t e0,
                            hipEvent_t e1);
const void* full_leaf_kernel(bool fp32, bool grad);
hipError_t launch_full_norm(bool grad, const NormArgs& a, hipStream_t st);

}  // namespace hf
