// The full time-dependent model of the mixing fit (section "Results": 16
// complex amplitudes, the mixing parameters, complex q/p and floating
// resonance masses and widths): its likelihood kernels, and the grid kernel
// that re-computes its normalisation at every evaluation when resonance
// shapes float (the grid matrices of the plain kernels hold only while the
// shapes are fixed).
//
// Normalisation: N = sum over the G x G midpoint cells inside the plot of
// the time-integrated rate, |A|^2 (kc + kz)/2 + |Abar'|^2 (kc - kz)/2
// + a_s ks + b_s kzs, times the cell area (kc, kz, ks, kzs the integrals of
// C, Cz, S, Sz over the real line).  One thread per cell of the list of
// cells inside the plot (made once per graph on the host with the same
// membership rule), rows of consecutive list entries as a dataset's rows of
// events; per row the sums of
// |A|^2, |Abar'|^2, a_s, b_s and the derivatives of the rate in the
// coefficient, q/p and shape slots, reduced by the same fixed-order
// reduction as the likelihood.  The tau, y and x derivatives follow on the
// host from the four sums.
#include "eval_device.h"

namespace hf {

namespace {

// Output column (after the 2R coefficient slots) of tail entry j of a grid
// launch: |Abar'|^2, a_s, b_s, then |q/p|, arg q/p and the shapes where
// present; -1 for an entry the node does not have.
__device__ __forceinline__ int norm_tail_col(const CS& cs, int fb, int j) {
  const int hq = cs.d[fb + kFhq] != 0.0, nf = (int)cs.d[fb + kFnf];
  if (j < 3) return j;
  if (j < 5) return hq ? j : -1;
  return j - 5 < 2 * nf ? 3 + 2 * hq + (j - 5) : -1;
}

template <bool GRAD>
__global__ __launch_bounds__(kBlock) void k_full_norm(const NormArgs a) {
  constexpr int NR = kMaxResFull;
  constexpr int NC = 1 + 2 * NR;
  const CS cs{a.prog.c64, a.prog.c32};
  const KNode& nd = a.prog.node[0];
  const int R = nd.aux;
  const int fb = nd.c0 + dz_full_base(R);
  const int64_t n_cells = a.n_cells;
  __shared__ double accs[NC][kBlock];
  const LdsAcc<NC> acc{accs};
  acc.zero(GRAD ? NC : 1);
  double tl[kFullTail];
#pragma unroll
  for (int j = 0; j < kFullTail; ++j) tl[j] = 0.0;
  int64_t c0, c1;
  row_chunks(n_cells, a.n_rows, blockIdx.x, c0, c1);
#pragma unroll 1
  for (int64_t ch = c0; ch < c1; ++ch) {
    const int64_t c = ch * kBlock + threadIdx.x;
    if (c >= n_cells) continue;
    const uint32_t cell = a.cells[c];
    const int i = (int)(cell >> 16), j = (int)(cell & 0xffffu);
    double s12, s13;
    {
#pragma clang fp contract(off)
      s12 = a.gs.lo12 + ((double)i + 0.5) * a.gs.h12;
      s13 = a.gs.lo13 + ((double)j + 0.5) * a.gs.h13;
    }
    const double x12[1] = {s12}, x13[1] = {s13}, xz[1] = {0.0}, xs[1] = {1.0};
    const auto emit = [&](int k, const double (&v)[1]) {
      if (GRAD) acc.add(1 + k, v[0]);
    };
    const auto tail = [&](auto jj, const double (&v)[1]) {
      constexpr int J = decltype(jj)::value;
      if (GRAD || J < 3) tl[J] += v[0];
    };
    double nA[1];
    leaf_tddp<double, 1, true, NR, true, true>(cs, nd, true, x12, x13, xz, xs, nA, emit, tail);
    acc.add(0, nA[0]);
  }
  const int n_lds = 1 + (GRAD ? 2 * R : 0);
  row_store_acc<NC>(acc, n_lds, a.partials + blockIdx.x, a.n_rows);
  __shared__ double red[kBlock / 64][kFullTail];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kFullTail; ++j) {
    const double v = wave_sum(tl[j]);
    if (lane == 0) red[wave][j] = v;
  }
  __syncthreads();
  const int j = threadIdx.x;
  if (j < kFullTail && (GRAD || j < 3)) {
    const int col = norm_tail_col(cs, fb, j);
    if (col >= 0)
      a.partials[(int64_t)(n_lds + col) * a.n_rows + blockIdx.x] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
  }
}

template <typename T, bool GRAD, bool TM>
hipError_t launch_leaf(const EvalArgs& a, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  hipExtLaunchKernelGGL((k_leaf<T, OP_TDDP_F, GRAD, TM>), dim3((unsigned)a.n_rows), dim3(kBlock), 0, st, e0, e1, 0,
                        a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_full_leaf(bool fp32, bool grad, bool tm, const EvalArgs& a, hipStream_t st, hipEvent_t e0,
                            hipEvent_t e1) {
  if (tm) return fp32 ? launch_leaf<float, true, true>(a, st, e0, e1) : launch_leaf<double, true, true>(a, st, e0, e1);
  if (fp32)
    return grad ? launch_leaf<float, true, false>(a, st, e0, e1) : launch_leaf<float, false, false>(a, st, e0, e1);
  return grad ? launch_leaf<double, true, false>(a, st, e0, e1) : launch_leaf<double, false, false>(a, st, e0, e1);
}

const void* full_leaf_kernel(bool fp32, bool grad) {
  if (fp32) return grad ? (const void*)&k_leaf<float, OP_TDDP_F, true> : (const void*)&k_leaf<float, OP_TDDP_F, false>;
  return grad ? (const void*)&k_leaf<double, OP_TDDP_F, true> : (const void*)&k_leaf<double, OP_TDDP_F, false>;
}

hipError_t launch_full_norm(bool grad, const NormArgs& a, hipStream_t st) {
  if (grad) hipLaunchKernelGGL(k_full_norm<true>, dim3((unsigned)a.n_rows), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL(k_full_norm<false>, dim3((unsigned)a.n_rows), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

}  // namespace hf
