// Likelihood kernels for gfx950: single-dataset, binned and batched launches,
// the fixed-order reduction, accept-reject toy generation, and their host
// dispatch.  The per-event evaluators and row loops are in eval_device.h.
#include <algorithm>

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "eval_device.h"
#include "philox.h"

namespace hf {

// ------------------------------------------------------------------ accept-reject toys
// Event i takes trials j = 0, 1, ...: its uniforms j (C + 1) + c place the
// candidate's column c in the box, number j (C + 1) + C decides acceptance
// (u * envelope < P in double); the first accepted candidate is the event,
// so the output does not depend on the launch shape.  An event that runs out
// of trials, or a density above the envelope, sets a flag bit.
template <int H>
__global__ __launch_bounds__(256) void k_generate_ar(const GenArArgs a) {
  const CS cs{a.prog.c64, a.prog.c32};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    EventStream rs{(uint32_t)((uint64_t)i & 0xFFFFFFFFu), (uint32_t)((uint64_t)i >> 32), a.key0, a.key1};
    double x[kMaxCols];
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c) x[c] = 0.0;
    bool done = false;
    int flag = 0;
    for (int j = 0; j < a.max_trials && !done; ++j) {
#pragma unroll
      for (int c = 0; c < kMaxCols; ++c)
        if (c < a.n_cols) x[c] = __dadd_rn(a.lo[c], __dmul_rn(rs.next(), a.hi[c] - a.lo[c]));  // no fma: as written
      const double ua = rs.next();
      bool in = true;
      if (a.dalitz) {
        double s12 = 0.0, s13 = 0.0;
#pragma unroll
        for (int c = 0; c < kMaxCols; ++c) {
          s12 = c == a.c12 ? x[c] : s12;
          s13 = c == a.c13 ? x[c] : s13;
        }
        in = dp_inside(a.M, a.m1, a.m2, a.m3, s12, s13);
      }
      if (in) {
        double dl[kMaxSlotsTree];
        const double p = ::exp(tree_eval<double, kMaxSlotsTree, kMaxCols, H, false>(a.prog, cs, x, dl) - a.ln_hoist);
        if (p > a.env) flag |= 2;
        if (__dmul_rn(ua, a.env) < p) done = true;
      }
    }
    if (!done) flag |= 1;
    if (flag) atomicOr(a.fail, flag);
#pragma unroll
    for (int c = 0; c < kMaxCols; ++c)
      if (c < a.n_cols) {
        if (a.fp32) ((float*)a.out[c])[i] = (float)(x[c] - a.ref[c]);
        else ((double*)a.out[c])[i] = x[c];
      }
  }
}

hipError_t launch_generate_ar(const GenArArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  const int64_t blocks = (a.n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
  if (a.dalitz) hipLaunchKernelGGL(k_generate_ar<2>, dim3(grid), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_generate_ar<1>, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ reduction
// Second launch: one 1024-thread block per fit sums that fit's rows in a
// fixed order.  Wave w of the 16 works on column w % nc (several waves per
// column when there are fewer than 16 columns, each on a fixed contiguous
// slice of the rows); a lane takes rows lane, lane + 64, ... of its slice
// (contiguous in the column-major layout) with 16 loads in flight,
// two-sum compensated; then a wave64 butterfly and a fixed-order merge of the
// slices of each column.  Result: [nll, slot_0 .. slot_{S-1}].
constexpr int kRedBlock = 1024;
constexpr int kRedWaves = kRedBlock / 64;
constexpr int kMaxRedCols = kMaxSlots + 1;

// Error-free sum of two values (Knuth): a + b = s + e exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

__device__ __forceinline__ void reduce_fit(const FitRec& fr) {
  const int nc = fr.n_slots + 1;
  const int R = fr.n_rows;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int per_col = nc >= kRedWaves ? 1 : kRedWaves / nc;  // waves per column
  __shared__ double colsum[kMaxRedCols][kRedWaves][2];
  for (int task = wave; task < nc * per_col; task += kRedWaves) {
    const int col = task / per_col, slice = task % per_col;
    const int r_begin = (int)((int64_t)R * slice / per_col);
    const int r_end = (int)((int64_t)R * (slice + 1) / per_col);
    const double* src = fr.partials + (int64_t)col * R;
    double s = 0.0, c = 0.0;
    for (int r0 = r_begin; r0 < r_end; r0 += 64 * 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int r = r0 + u * 64 + lane;
        v[u] = r < r_end ? src[r] : 0.0;
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
  __shared__ double fin[kMaxRedCols];
  const int t = threadIdx.x;
  if (t < nc) {
    double s = colsum[t][0][0], c = colsum[t][0][1];
    for (int k = 1; k < per_col; ++k) {
      double ns, e;
      two_sum(s, colsum[t][k][0], ns, e);
      s = ns;
      c = (c + colsum[t][k][1]) + e;
    }
    fin[t] = s + c;
  }
  __syncthreads();
  // one thread stores the result, then (system-scope release) the flag the
  // host may spin on
  if (t == 0) {
    for (int j = 0; j < nc; ++j) fr.result[j] = fin[j];
    if (fr.flag) {
      __threadfence_system();
      *(volatile int64_t*)fr.flag = fr.seq;
    }
  }
}

__global__ __launch_bounds__(kRedBlock) void k_reduce(const FitRec* __restrict__ fits, int n_fits_max) {
  const FitRec& fr = fits[blockIdx.x];
  if (!fr.active) return;
  reduce_fit(fr);
}

__global__ __launch_bounds__(kRedBlock) void k_reduce_one(const FitRec fr) { reduce_fit(fr); }

// Binned datasets (any tree): the tree interpreter with the binned metric.
template <typename T, int NS, int NCOL, int HEAVY, bool GRAD>
__global__ __launch_bounds__(kBlock) void k_binned(const EvalArgs a) {
  typedef typename Col<T>::S Sx;
  constexpr int NC = NS + 2;
  const CS cs{a.prog.c64, a.prog.c32};
  const BinnedEv<T, NS, NCOL, HEAVY, GRAD> ev{cs, a.wcol, a.kfac, a.lnL, a.metric};
  const Sx* cp[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) cp[c] = (const Sx*)a.col[c];
  __shared__ double accs[NC][kBlock];
  const LdsAcc<NC> acc{accs};
  const int nc = GRAD ? a.prog.n_slots + 2 : 1;
  acc.zero(nc);
  int64_t c0, c1;
  row_chunks(a.n_events, a.n_rows, blockIdx.x, c0, c1);
  heavy_row<T, NCOL>(ev, a.prog, cp, a.prog.n_cols, a.n_events, c0, c1, acc);
  row_store_acc<NC>(acc, nc, a.partials + blockIdx.x, a.n_rows);
}

// Batched: the program structure is shared (kernel argument); constants,
// columns and partials are per fit.  Fits own contiguous ranges of the global
// row list in fit order; each block walks global rows blockIdx.x,
// blockIdx.x + gridDim.x, ...
struct BatchArgs {
  KProgram prog;               // structure only (constants unused)
  const BatchHeader* hdr;      // counts, then the FitRec array
  const double* c64;           // [fit][n_const]
  const float* c32;
  int32_t n_const;
};

__device__ __forceinline__ int find_fit(const FitRec* fits, int n_fits, int grow) {
  int lo = 0, hi = n_fits - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fits[mid].row_begin <= grow) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_leaf_batched(const BatchArgs a) {  // always with gradient
  const int total = a.hdr->total_rows, n_fits = a.hdr->n_fits;
  const FitRec* fits = (const FitRec*)(a.hdr + 1);
  for (int gr = blockIdx.x; gr < total; gr += gridDim.x) {
    const int f = find_fit(fits, n_fits, gr);
    const FitRec& fr = fits[f];
    const CS cs{a.c64 + (int64_t)f * a.n_const, a.c32 + (int64_t)f * a.n_const};
    const int r = gr - fr.row_begin;
    if constexpr (OP == OP_EXP || OP == OP_GAUSS)
      light_leaf_row<T, OP, true>(a.prog.node[0], cs, fr.col, fr.n_events, fr.n_rows, r, fr.partials + r);
    else
      amp_leaf_row<T, OP, true>(a.prog, cs, fr.col, fr.n_events, fr.n_rows, r, fr.partials + r);
  }
}

template <typename T, int K, int MASK>
__global__ __launch_bounds__(kBlock) void k_mix_batched(const BatchArgs a) {
  const int total = a.hdr->total_rows, n_fits = a.hdr->n_fits;
  const FitRec* fits = (const FitRec*)(a.hdr + 1);
  for (int gr = blockIdx.x; gr < total; gr += gridDim.x) {
    const int f = find_fit(fits, n_fits, gr);
    const FitRec& fr = fits[f];
    const CS cs{a.c64 + (int64_t)f * a.n_const, a.c32 + (int64_t)f * a.n_const};
    const int r = gr - fr.row_begin;
    mix_row<T, K, MASK, true>(a.prog, cs, fr.col, fr.n_events, fr.n_rows, r, fr.partials + r);
  }
}

template <typename T, int NS, int NCOL, int HEAVY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(TreeWaves<T, HEAVY>::value)))
void k_tree_batched(const BatchArgs a) {
  const int total = a.hdr->total_rows, n_fits = a.hdr->n_fits;
  const FitRec* fits = (const FitRec*)(a.hdr + 1);
  for (int gr = blockIdx.x; gr < total; gr += gridDim.x) {
    const int f = find_fit(fits, n_fits, gr);
    const FitRec& fr = fits[f];
    const CS cs{a.c64 + (int64_t)f * a.n_const, a.c32 + (int64_t)f * a.n_const};
    const int r = gr - fr.row_begin;
    tree_row<T, NS, NCOL, HEAVY, true>(a.prog, cs, fr.col, fr.n_events, fr.n_rows, r, fr.partials + r);
  }
}

// ------------------------------------------------------------------ dispatch
bool kind_light(int kind) {
  if ((kind >= KIND_MIX2 && kind < KIND_MIX2 + 4) || (kind >= KIND_MIX3 && kind < KIND_MIX3 + 8)) return true;
  return kind == KIND_EXP || kind == KIND_GAUSS || kind == KIND_TREE_SMALL;
}

// Resident blocks per compute unit of a kind's kernels (the smaller of the
// NLL-only and gradient instantiations), from the occupancy calculator.
template <typename T, bool GRAD>
static const void* kernel_of(int kind) {
  switch (kind) {
    case KIND_EXP: return (const void*)&k_leaf<T, OP_EXP, GRAD>;
    case KIND_GAUSS: return (const void*)&k_leaf<T, OP_GAUSS, GRAD>;
    case KIND_TREE_SMALL: return (const void*)&k_tree<T, 8, 2, 0, GRAD>;
    case KIND_DALITZ: return (const void*)&k_leaf<T, OP_DALITZ, GRAD>;
    case KIND_TDDP: return (const void*)&k_leaf<T, OP_TDDP, GRAD>;
    case KIND_TDDPX: return (const void*)&k_leaf<T, OP_TDDP_X, GRAD>;
    case KIND_TDDPS: return (const void*)&k_leaf<T, OP_TDDP_S, GRAD>;
    case KIND_TDDPXS: return (const void*)&k_leaf<T, OP_TDDP_XS, GRAD>;
    case KIND_TREE: return (const void*)&k_tree<T, kMaxSlotsTree, kMaxCols, 2, GRAD>;
    case KIND_TREE_NOAMP: return (const void*)&k_tree<T, kMaxSlotsTree, kMaxCols, 1, GRAD>;
    case KIND_TREE_CONV: return (const void*)&k_tree<T, kMaxSlotsTree, kMaxCols, kHeavyConvTab, GRAD>;
    case KIND_TREE_CONV_SMALL: return (const void*)&k_tree<T, ConvSmall<T>::NS, ConvSmall<T>::NCOL, kHeavyConvTab, GRAD>;
    case KIND_TDDPF: return full_leaf_kernel(std::is_same<T, float>::value, GRAD);
    default: return nullptr;  // mixtures: light, never below kRowsPerCU
  }
}

int resident_blocks_per_cu(int kind, bool fp32) {
  int best = 0;
  for (int grad = 0; grad < 2; ++grad) {
    const void* f = fp32 ? (grad ? kernel_of<float, true>(kind) : kernel_of<float, false>(kind))
                         : (grad ? kernel_of<double, true>(kind) : kernel_of<double, false>(kind));
    if (!f) continue;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kBlock, 0) != hipSuccess || nb <= 0) continue;
    best = best == 0 ? nb : std::min(best, nb);
  }
  return best;
}

hipError_t launch_eval(int kind, bool fp32, bool grad, const EvalArgs& a, hipStream_t st, hipEvent_t e0,
                       hipEvent_t e1) {
  if (a.n_rows <= 0) return hipSuccess;
  if (fp32)
    return grad ? launch_any<float, true, false>(kind, a, st, e0, e1) : launch_any<float, false, false>(kind, a, st, e0, e1);
  return grad ? launch_any<double, true, false>(kind, a, st, e0, e1)
              : launch_any<double, false, false>(kind, a, st, e0, e1);
}

template <typename T, bool GRAD>
static hipError_t launch_binned_t(int heavy, const EvalArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid((unsigned)a.n_rows), block(kBlock);
  if (heavy >= 2)
    hipExtLaunchKernelGGL((k_binned<T, kMaxSlotsTree, kMaxCols, 2, GRAD>), grid, block, 0, st, e0, e1, 0, a);
  else if (heavy == 1)
    hipExtLaunchKernelGGL((k_binned<T, kMaxSlotsTree, kMaxCols, 1, GRAD>), grid, block, 0, st, e0, e1, 0, a);
  else
    hipExtLaunchKernelGGL((k_binned<T, 8, 2, 0, GRAD>), grid, block, 0, st, e0, e1, 0, a);
  return hipGetLastError();
}

hipError_t launch_binned(bool fp32, bool grad, int heavy, const EvalArgs& a, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1) {
  if (a.n_rows <= 0) return hipSuccess;
  if (fp32)
    return grad ? launch_binned_t<float, true>(heavy, a, st, e0, e1) : launch_binned_t<float, false>(heavy, a, st, e0, e1);
  return grad ? launch_binned_t<double, true>(heavy, a, st, e0, e1) : launch_binned_t<double, false>(heavy, a, st, e0, e1);
}

template <typename T>
static hipError_t launch_b(int kind, const BatchArgs& a, int grid, hipStream_t st) {
  const dim3 g(grid), b(kBlock);
  switch (kind) {
    case KIND_EXP: hipLaunchKernelGGL((k_leaf_batched<T, OP_EXP>), g, b, 0, st, a); break;
    case KIND_GAUSS: hipLaunchKernelGGL((k_leaf_batched<T, OP_GAUSS>), g, b, 0, st, a); break;
    case KIND_TREE_SMALL: hipLaunchKernelGGL((k_tree_batched<T, 8, 2, 0>), g, b, 0, st, a); break;
    case KIND_DALITZ: hipLaunchKernelGGL((k_leaf_batched<T, OP_DALITZ>), g, b, 0, st, a); break;
    case KIND_TDDP: hipLaunchKernelGGL((k_leaf_batched<T, OP_TDDP>), g, b, 0, st, a); break;
    case KIND_TDDPX: hipLaunchKernelGGL((k_leaf_batched<T, OP_TDDP_X>), g, b, 0, st, a); break;
    case KIND_TDDPS: hipLaunchKernelGGL((k_leaf_batched<T, OP_TDDP_S>), g, b, 0, st, a); break;
    case KIND_TDDPXS: hipLaunchKernelGGL((k_leaf_batched<T, OP_TDDP_XS>), g, b, 0, st, a); break;
    case KIND_TREE: hipLaunchKernelGGL((k_tree_batched<T, kMaxSlotsTree, kMaxCols, 2>), g, b, 0, st, a); break;
    case KIND_TREE_NOAMP: hipLaunchKernelGGL((k_tree_batched<T, kMaxSlotsTree, kMaxCols, 1>), g, b, 0, st, a); break;
    case KIND_TREE_CONV:
      hipLaunchKernelGGL((k_tree_batched<T, kMaxSlotsTree, kMaxCols, kHeavyConvTab>), g, b, 0, st, a);
      break;
    case KIND_TREE_CONV_SMALL:
      hipLaunchKernelGGL((k_tree_batched<T, ConvSmall<T>::NS, ConvSmall<T>::NCOL, kHeavyConvTab>), g, b, 0, st, a);
      break;
#define HF_MIX(K_, M_)                                                                              \
  case (K_ == 2 ? KIND_MIX2 : KIND_MIX3) + M_:                                                      \
    hipLaunchKernelGGL((k_mix_batched<T, K_, M_>), g, b, 0, st, a);                                 \
    break;
    HF_MIX(2, 0) HF_MIX(2, 1) HF_MIX(2, 2) HF_MIX(2, 3)
    HF_MIX(3, 0) HF_MIX(3, 1) HF_MIX(3, 2) HF_MIX(3, 3) HF_MIX(3, 4) HF_MIX(3, 5) HF_MIX(3, 6) HF_MIX(3, 7)
#undef HF_MIX
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
  return fp32 ? launch_b<float>(kind, a, grid, st) : launch_b<double>(kind, a, grid, st);
}

hipError_t launch_reduce_one(const FitRec& fr, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  hipExtLaunchKernelGGL(k_reduce_one, dim3(1), dim3(kRedBlock), 0, st, e0, e1, 0, fr);
  return hipGetLastError();
}

hipError_t launch_reduce(const FitRec* fits_dev, int n_fits, hipStream_t st) {
  if (n_fits <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(n_fits), dim3(kRedBlock), 0, st, fits_dev, n_fits);
  return hipGetLastError();
}

}  // namespace hf
