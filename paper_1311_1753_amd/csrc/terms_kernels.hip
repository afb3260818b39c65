// Per-event terms launches (nll_terms): the same kernels as the likelihood
// evaluation, instantiated with per-event output.  A terms launch has one
// 256-event chunk per row, so every thread evaluates exactly one event with
// the evaluation kernels' own code and writes that event's accumulator terms
// (-ln P without the host-applied normalisations, then the kind's gradient
// accumulators) to [column][event] instead of summing them; the host turns
// each event's terms into ln P and d ln P / d theta with the same assembly
// as the summed result.
#include "eval_device.h"

namespace hf {

hipError_t launch_terms(int kind, bool fp32, const EvalArgs& a, hipStream_t st) {
  if (a.n_rows <= 0) return hipSuccess;
  return fp32 ? launch_any<float, true, true>(kind, a, st, nullptr, nullptr)
              : launch_any<double, true, true>(kind, a, st, nullptr, nullptr);
}

}  // namespace hf
