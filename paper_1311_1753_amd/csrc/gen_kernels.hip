// Device-side toy generation: events of a sampleable PDF tree drawn in HBM,
// for the toy fits of the serving loop (the paper's pseudo-experiment
// studies) without moving their events over PCIe.
//
// Random numbers: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011), a counter-based
// generator: uniform number m of event i comes from the block with counter
// (i mod 2^32, i div 2^32, m div 2, 0) under the key (seed low word, seed
// high word), words 0-1 for even m and 2-3 for odd m, as
// u = (floor((w_a 2^32 + w_b) / 2^11) + 1/2) 2^-53 in (0, 1).  Every event is
// independent of the others, so the grid can be any shape.
//
// Sampling: the factors of a root PROD in order; in a factor that is an ADD
// one uniform picks the child (the first j with u < f_0 + ... + f_j, the last
// taking the rest), then one uniform feeds the child's inverse CDF:
//   EXP   x = lo + ln(1 + u (e^{alpha L} - 1)) / alpha   (lo + u L at alpha = 0)
//   GAUSS x = mu + sqrt(2) sigma erfinv(erf(z_lo) + u (erf(z_hi) - erf(z_lo)))
// clamped to the box.  Each lane evaluates every child of its factor with its
// own u and keeps the picked one: the children's constants are read at
// wave-uniform indices only.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "philox.h"

namespace hf {
namespace {

__device__ __forceinline__ double inv_cdf(const GenLeaf& L, double u) {
  double x;
  if (L.op == OP_EXP)
    x = L.p0 == 0.0 ? L.lo + u * (L.hi - L.lo) : L.lo + ::log1p(u * L.p1) / L.p0;
  else
    x = L.p0 + L.p1 * ::erfinv(L.p2 + u * (L.p3 - L.p2));
  return fmin(fmax(x, L.lo), L.hi);
}

__global__ __launch_bounds__(256) void k_generate(const GenArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
    EventStream rs{(uint32_t)((uint64_t)i & 0xFFFFFFFFu), (uint32_t)((uint64_t)i >> 32), a.key0, a.key1};
    for (int f = 0; f < a.n_factor; ++f) {
      const int first = a.first[f], nl = a.n_leaf[f];
      int pick = 0;
      if (nl > 1) {
        const double u = rs.next();
        pick = nl - 1;
        for (int q = nl - 2; q >= 0; --q) pick = u < a.leaf[first + q].cum ? q : pick;
      }
      const double u = rs.next();
      double x = 0.0;
      for (int q = 0; q < nl; ++q) {
        const double xq = inv_cdf(a.leaf[first + q], u);
        x = q == pick ? xq : x;
      }
      if (a.fp32) ((float*)a.out[f])[i] = (float)(x - a.ref[f]);
      else ((double*)a.out[f])[i] = x;
    }
  }
}

}  // namespace

hipError_t launch_generate(const GenArgs& a, hipStream_t st) {
  if (a.n <= 0) return hipSuccess;
  const int64_t blocks = (a.n + 255) / 256;
  const unsigned grid = (unsigned)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(k_generate, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace hf
