// Internal layout shared by the host runtime and the gfx950 kernels.
//
// A PDF tree is flattened into a KProgram: nodes in post-order (children
// before parents, root last), each with its opcode, child list, the columns
// it reads, the slots of the per-event gradient it owns and an offset into a
// constant table.  The host rewrites the constant table from the parameter
// vector before every launch (double values for the FP64 path, float copies
// for the FP32-eval path, location constants always in double); the whole
// program travels as a kernel argument, so each launch reads it through the
// scalar cache with no extra copy.  This replaces the paper's global
// parameter array and per-PDF index arrays read by double indirection
// (section "Adding new PDFs").
#pragma once
#include <cstdint>

namespace hf {

constexpr int kBlock = 256;          // threads per block (4 wave64)
constexpr int kMaxNodes = 16;
constexpr int kMaxCols = 8;
constexpr int kMaxSlots = 48;       // gradient slots of a graph
constexpr int kMaxSlotsTree = 32;   // ... evaluated by the tree interpreter
constexpr int kMaxConst = 192;
constexpr int kMaxRes = 8;          // resonances of DALITZ / TDDP nodes in the plain kernels
constexpr int kMaxResFull = 16;     // ... of the full time-dependent kernel (the mixing fit)
constexpr int kMaxFloat = 4;        // resonances with floating mass and width
constexpr int kMaxPar = 64;
constexpr int kNumGroups = 9;        // (pair, spin) groups of Dalitz resonances
constexpr int kConvTab = 512;        // grid points of a CONV model that a row stages in LDS

enum Op : int16_t {
  OP_EXP = 1, OP_GAUSS = 2, OP_POLY = 3, OP_ADD = 4, OP_PROD = 5, OP_DALITZ = 6, OP_TDDP = 7, OP_MAP = 8,
  OP_DPMAP = 9, OP_CONV = 10, OP_COMP = 11
};
constexpr int kMaxConvGrid = 4096;  // CONV grid points

// Node fields are 32-bit so that the kernels read them from the kernel
// argument with scalar loads at wave-uniform node indices (16-bit fields at
// runtime offsets become per-lane memory loads whose values the compiler can
// no longer treat as uniform).
struct KNode {
  int32_t op;
  int32_t n_child;
  int32_t child0;    // first index into KProgram::child
  int32_t slot0;     // first per-event gradient slot owned by this node
  int32_t n_slot;
  int32_t c0;        // first constant of this node
  int32_t col[4];    // observable columns read
  int32_t hoisted;   // 1: normalisation applied on the host (every ancestor is PROD)
  int32_t aux;       // POLY: degree; DALITZ/TDDP: number of resonances
  // DALITZ/TDDP: the resonances are stored grouped by (pair, spin), group
  // g = 3 * pair + J (pairs 12, 13, 23 = 0, 1, 2); group g holds resonances
  // [res_end[g - 1], res_end[g]) with res_end[-1] = 0 and res_end[8] = R.
  // ADD: res_end[j] is child j's first constant (c0).
  int32_t res_end[kNumGroups];
};

struct KProgram {
  int32_t n_nodes, root, n_slots, n_cols;
  KNode node[kMaxNodes];
  int32_t child[kMaxNodes];
  double c64[kMaxConst];
  float c32[kMaxConst];
};

// Constant layouts (offsets relative to KNode::c0).
//   EXP    0 loc = ref - a (double), 1 alpha, 2 lnN_hi, 3 lnN_lo, 4 dlnN/dalpha
//   GAUSS  0 loc = ref - mu (double), 1 1/sigma, 2 lnN_hi, 3 lnN_lo, 4 dlnN/dmu, 5 dlnN/dsigma
//   POLY   0 loc = ref - x0 (double), 1..d a_k, d+1 lnN_hi, d+2 lnN_lo, d+3.. dlnN/da_k
//   ADD    0..K-1 fractions (the last one 1 - sum of the others)
//   MAP    0..K-2 inner range boundaries, K-1 column reference (added back
//          to the stored value before the range test), K lnZ_hi, K+1 lnZ_lo,
//          then dlnZ/d(slot) for every slot of the children in child order
//          (not hoisted; zeros when hoisted)
//   PROD   with leaves sharing an observable: 0 lnZ_hi, 1 lnZ_lo, then
//          dlnZ/d(slot) for every slot of the children in child order
//          (zeros when hoisted); otherwise none
//   DPMAP  0, 1 column references of s12 and s13, then n12-1 s12 cell
//          boundaries and n13-1 s13 boundaries; aux = n13
//   CONV   0 box lower end lo (grid t_k = lo + (k + 1/2) h), 1 grid step h,
//          2 d_lo, 3 d_hi,
//          4 column reference, 5 shift c of the exponents, 6 (lnZ - c)_hi,
//          7 (lnZ - c)_lo, then dlnZ/d(slot) for the model's and the
//          resolution's slots (not hoisted; zeros when hoisted); aux = N
//   COMP   0 lnZ_hi, 1 lnZ_lo, 2 column reference, then dlnZ/d(slot) for the
//          core's and the shell's slots (zeros when hoisted)
//   DALITZ/TDDP: see the kDz* offsets below.
// For the float path lnN is split into a float pair (hi + lo) so that the
// rounding of the constant does not bias every event in the same direction.
// kDzR2: squared barrier radius r^2 (all resonances)
constexpr int kDzRef12 = 0, kDzRef13 = 1, kDzSsum = 2, kDzLnHi = 3, kDzLnLo = 4, kDzR2 = 5, kDzDln = 6;
// channel blocks (pairs 12, 13, 23 in that order) after the 2R (+2 for TDDP)
// dlnN entries: constants that depend only on the pair's masses
constexpr int kChThrP = 0, kChThrM = 1, kChZc1 = 2, kChZtaC = 3, kChZtaD = 4, kChZtbC = 5, kChZtbD = 6,
              kChStride = 7, kNumCh = 3;
// per resonance block (stride kResStride) after the channel blocks, in the
// group order of KNode::res_end: m0^2, Kw B0^2 (B0 = the barrier polynomial's
// square root at q0, 1 for J = 0), B0
constexpr int kResM02 = 0, kResKwB = 1, kResSqB = 2, kResStride = 3;
// TDDP time constants after the coefficients: the decay rates G-/+ = (1 -/+ y)/tau
// and G = 1/tau with their tau and y derivatives, and the oscillation
// frequency W = x/tau of the trigonometric terms with its tau and x
// derivatives (zero without x)
constexpr int kTdGm = 0, kTdGp = 1, kTdG = 2, kTdDGmTau = 3, kTdDGpTau = 4, kTdDGTau = 5,
              kTdDGmY = 6, kTdDGpY = 7, kTdW = 8, kTdDWTau = 9, kTdDWX = 10, kTdCount = 11;

// dlnN entries: 2R coefficients (+ tau, y, x for TDDP; the x entry stays
// unused without x)
constexpr int dz_n_dln(int R, bool tddp) { return 2 * R + (tddp ? 3 : 0); }
constexpr int dz_ch_base(int R, bool tddp) { return kDzDln + dz_n_dln(R, tddp); }
constexpr int dz_res_base(int R, bool tddp) { return dz_ch_base(R, tddp) + kNumCh * kChStride; }
// the coefficient block always has room for NR coefficients (NR = kMaxRes,
// or kMaxResFull for the full model); those of absent resonances stay zero,
// so the kernels sum over all NR places
constexpr int dz_coef_base(int R, bool tddp) { return dz_res_base(R, tddp) + R * kResStride; }
constexpr int dz_time_base(int R, int NR = kMaxRes) { return dz_coef_base(R, true) + 2 * NR; }
constexpr int dz_n_const(int R, bool tddp) { return dz_coef_base(R, tddp) + 2 * kMaxRes + (tddp ? kTdCount : 0); }

// Full time-dependent model (the mixing fit: up to kMaxResFull resonances,
// complex q/p, floating masses and widths), after the time constants:
//   kFqRe, kFqIm   q/p (1, 0 without q/p);  kFiq  1 / |q/p|
//   kFhx, kFhq     1.0 when x (q/p) is a parameter;  kFnf  floating resonances
//   kFkc..kFkzs    time integrals of C, Cz, S, Sz over the real line
//   then per floating resonance f (stride kFlStride): its place, pair
//   (0, 1, 2 for 12, 13, 23) and spin, d(m0^2)/dm0, d(Kw B0^2)/dm0,
//   d ln B0/dm0 and d(Kw B0^2)/dGamma0
constexpr int kFqRe = 0, kFqIm = 1, kFiq = 2, kFhx = 3, kFhq = 4, kFnf = 5, kFkc = 6, kFkz = 7, kFks = 8,
              kFkzs = 9, kFlBase = 10;
constexpr int kFlRes = 0, kFlPair = 1, kFlJ = 2, kFlDm2 = 3, kFlDkwM = 4, kFlDlbM = 5, kFlDkwG = 6, kFlStride = 7;
constexpr int dz_full_base(int R) { return dz_time_base(R, kMaxResFull) + kTdCount; }
constexpr int dz_n_const_full(int R) { return dz_full_base(R) + kFlBase + kFlStride * kMaxFloat; }
// slots of a full node: 2R coefficients, tau, y, (x), (|q/p|, arg q/p), then
// (m0, Gamma0) per floating resonance; at most this many after the
// coefficients
constexpr int kFullTail = 5 + 2 * kMaxFloat;

// Arguments of one evaluation launch over one dataset.
struct EvalArgs {
  KProgram prog;
  const void* col[kMaxCols];   // device columns (double or float)
  int64_t n_events;
  double* partials;            // column-major [n_slots + 1][n_rows]: sum(-ln P), slot sums
  int32_t n_rows;              // one block per row
  int32_t metric;              // 0: unbinned NLL; binned: 1 weighted NLL, 2 chi^2
  const double* wcol;          // binned: bin weights (counts)
  double kfac;                 // binned chi^2: expected count = kfac * P
  double lnL;                  // binned: normalisations of hoisted nodes (ln P = kernel value - lnL)
};

// Header of a batched launch's device table, followed by the FitRec array.
struct BatchHeader {
  int32_t n_fits, total_rows, pad0, pad1;
};

// Per-fit record of a batched launch (device memory).
struct FitRec {
  const void* col[kMaxCols];
  int64_t n_events;
  double* partials;            // column-major, column stride n_rows
  int32_t row_begin;           // first global row of this fit
  int32_t n_rows;
  double* result;              // n_slots + 1 doubles
  int32_t n_slots;             // slot columns to reduce (0: NLL only)
  int32_t active;
  int64_t* flag;               // nullable: set to `seq` after the result is visible to the host
  int64_t seq;
};

}  // namespace hf
