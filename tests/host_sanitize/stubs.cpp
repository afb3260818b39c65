// Host stand-ins for the library's kernel-launch entry points (kernels.h),
// so that the host runtime (graph validation and staging, the minimiser,
// the ABI's argument checks, the batch engine's bookkeeping) can be built
// with the address and undefined-behaviour sanitizers and run without a
// GPU.  Every launch reports hipErrorNotSupported; callers must turn that
// into an HF_E_HIP return, never a crash.
#include "../../paper_1311_1753_amd/csrc/kernels.h"

namespace hf {

bool kind_light(int kind) {
  return (kind >= KIND_MIX2 && kind < KIND_MIX2 + 4) || (kind >= KIND_MIX3 && kind < KIND_MIX3 + 8) || kind == KIND_EXP ||
         kind == KIND_GAUSS || kind == KIND_TREE_SMALL;
}
int resident_blocks_per_cu(int, bool) { return 0; }
hipError_t launch_eval(int, bool, bool, const EvalArgs&, hipStream_t, hipEvent_t, hipEvent_t) {
  return hipErrorNotSupported;
}
hipError_t launch_terms(int, bool, const EvalArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reduce_one(const FitRec&, hipStream_t, hipEvent_t, hipEvent_t) { return hipErrorNotSupported; }
hipError_t launch_binned(bool, bool, int, const EvalArgs&, hipStream_t, hipEvent_t, hipEvent_t) {
  return hipErrorNotSupported;
}
hipError_t launch_reduce(const FitRec*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_eval_batched(int, bool, const KProgram&, const BatchHeader*, const double*, const float*, int, int,
                               hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_generate(const GenArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_full_leaf(bool, bool, bool, const EvalArgs&, hipStream_t, hipEvent_t, hipEvent_t) {
  return hipErrorNotSupported;
}
const void* full_leaf_kernel(bool, bool) { return nullptr; }
hipError_t launch_full_norm(bool, const NormArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_generate_ar(const GenArArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t dalitz_grid_matrices(const GridSpec&, const KProgram&, int, bool, double*, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace hf
