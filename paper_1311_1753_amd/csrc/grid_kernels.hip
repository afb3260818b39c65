// Dalitz-plot normalisation integrals on the G x G midpoint grid (double).
//
// For the basis amplitudes a_0 = 1, a_k = A_k (k = 1..R) and their CP
// conjugates abar_k(s12, s13) = a_k(s13, s12), the kernels form
//   I_pq    = sum_cells conj(a_p) a_q
//   Ibar_pq = sum_cells conj(abar_p) abar_q      (TDDP only)
//   J_pq    = sum_cells conj(a_p) abar_q         (TDDP only)
// over the cells whose centre lies in the Dalitz plot; the host multiplies by
// the cell area.  With these, the normalisation of a coherent sum with
// coefficients c is c^H I c, and that of the time-dependent density is a
// linear combination of c^H I c, c^H Ibar c and Re c^H J c.  The grid depends
// only on the resonance shapes, so it is computed once per graph.
//
// Pass 1: a block takes 128 cells of one grid row, evaluates their
// amplitudes into LDS, and its threads each sum matrix elements (n_mat *
// na^2 of them, so more than one per thread beyond 15 resonances) over
// those cells.  Pass 2: one block per matrix element sums the row
// partials in a fixed order.  Both passes are deterministic.
#include <hip/hip_runtime.h>

#include <vector>

#include "device_common.h"
#include "dp_inside.h"
#include "internal.h"
#include "kernels.h"

namespace hf {

constexpr int kGridCells = 128;

struct GridArgs {
  KProgram prog;
  GridSpec gs;
  int node, c0, R, tddp, n_chunks;
  double2* part;     // [row * n_chunks + chunk][n_mat * na * na]
};

template <int NR>
__global__ __launch_bounds__(kBlock) void k_grid_rows(const GridArgs a) {
  const int na = a.R + 1;
  const int n_mat = a.tddp ? 3 : 1;
  const int row = blockIdx.x / a.n_chunks, chunk = blockIdx.x % a.n_chunks;
  __shared__ double2 sa[kGridCells][NR + 1];
  __shared__ double2 sb[kGridCells][NR + 1];
  const CS cs{a.prog.c64, a.prog.c32};
  const int t = threadIdx.x;
  if (t < kGridCells) {
    const int col = chunk * kGridCells + t;
    bool in = false;
    double s12 = 0.0, s13 = 0.0;
    if (col < a.gs.grid) {
#pragma clang fp contract(off)
      s12 = a.gs.lo12 + ((double)row + 0.5) * a.gs.h12;
      s13 = a.gs.lo13 + ((double)col + 0.5) * a.gs.h13;
      in = dp_inside(a.gs.M, a.gs.m1, a.gs.m2, a.gs.m3, s12, s13);
    }
    AmpArr<double, NR> a0, b0;
    if (in) {
      const double p12[1] = {s12}, p13[1] = {s13}, p23[1] = {cs.d[a.c0 + kDzSsum] - s12 - s13};
      if (a.tddp) dalitz_amps<double, true, 1, NR>(cs, a.prog.node[a.node], p12, p13, p23, a0, a0, b0, b0);
      else dalitz_amps<double, false, 1, NR>(cs, a.prog.node[a.node], p12, p13, p23, a0, a0, b0, b0);
    }
    sa[t][0] = make_double2(in ? 1.0 : 0.0, 0.0);
    sb[t][0] = sa[t][0];
    for (int k = 0; k < a.R; ++k) {
      sa[t][k + 1] = in ? make_double2(a0[2 * k], a0[2 * k + 1]) : make_double2(0.0, 0.0);
      sb[t][k + 1] = (in && a.tddp) ? make_double2(b0[2 * k], b0[2 * k + 1]) : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  const int n_el = n_mat * na * na;
  for (int el = t; el < n_el; el += kBlock) {
    const int w = el / (na * na), pq = el % (na * na), p = pq / na, q = pq % na;
    double re = 0.0, im = 0.0;
    for (int c = 0; c < kGridCells; ++c) {
      const double2 x = (w == 1) ? sb[c][p] : sa[c][p];
      const double2 y = (w == 0) ? sa[c][q] : sb[c][q];
      // conj(x) * y
      re += x.x * y.x + x.y * y.y;
      im += x.x * y.y - x.y * y.x;
    }
    a.part[(int64_t)blockIdx.x * n_el + el] = make_double2(re, im);
  }
}

__device__ __forceinline__ void two_sum_g(double a, double b, double& s, double& e) {
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

__global__ __launch_bounds__(kBlock) void k_grid_sum(const double2* __restrict__ part, int n_rows, int n_el,
                                                     double2* __restrict__ out) {
  const int el = blockIdx.x;
  double sr = 0.0, cr = 0.0, si = 0.0, ci = 0.0;
  for (int r = threadIdx.x; r < n_rows; r += kBlock) {
    const double2 v = part[(int64_t)r * n_el + el];
    double ns, e;
    two_sum_g(sr, v.x, ns, e); sr = ns; cr += e;
    two_sum_g(si, v.y, ns, e); si = ns; ci += e;
  }
  __shared__ double4 red[kBlock];
  red[threadIdx.x] = make_double4(sr, cr, si, ci);
  __syncthreads();
  for (int half = kBlock / 2; half >= 1; half >>= 1) {
    if (threadIdx.x < half) {
      const double4 x = red[threadIdx.x], y = red[threadIdx.x + half];
      double s1, e1, s2, e2;
      two_sum_g(x.x, y.x, s1, e1);
      two_sum_g(x.z, y.z, s2, e2);
      red[threadIdx.x] = make_double4(s1, (x.y + y.y) + e1, s2, (x.w + y.w) + e2);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[el] = make_double2(red[0].x + red[0].y, red[0].z + red[0].w);
}

hipError_t dalitz_grid_matrices(const GridSpec& gs, const KProgram& prog, int node, bool tddp, double* out_host,
                                hipStream_t st) {
  const KNode& nd = prog.node[node];
  const int R = nd.aux, na = R + 1, n_mat = tddp ? 3 : 1;
  const int n_el = n_mat * na * na;
  GridArgs a;
  a.prog = prog;
  a.gs = gs;
  a.node = node;
  a.c0 = nd.c0;
  a.R = R;
  a.tddp = tddp ? 1 : 0;
  a.n_chunks = (gs.grid + kGridCells - 1) / kGridCells;
  const int n_rows = gs.grid * a.n_chunks;
  double2* part = nullptr;
  double2* out = nullptr;
  hipError_t e = hipMalloc(&part, (size_t)n_rows * n_el * sizeof(double2));
  if (e != hipSuccess) return e;
  e = hipMalloc(&out, (size_t)n_el * sizeof(double2));
  if (e != hipSuccess) { hipFree(part); return e; }
  a.part = part;
  if (R > kMaxRes) hipLaunchKernelGGL(k_grid_rows<kMaxResFull>, dim3(n_rows), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL(k_grid_rows<kMaxRes>, dim3(n_rows), dim3(kBlock), 0, st, a);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_grid_sum, dim3(n_el), dim3(kBlock), 0, st, part, n_rows, n_el, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out_host, out, (size_t)n_el * sizeof(double2), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(part);
  hipFree(out);
  return e;
}

}  // namespace hf
