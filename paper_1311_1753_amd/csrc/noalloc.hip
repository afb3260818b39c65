// nll_grad over caller-owned device columns with no device allocation: the
// evaluation kernels' partial rows and the reduction's result row live in a
// fixed file-scope device array instead of a dataset's workspace, and the
// result reaches the host by a stream copy instead of a mapped host buffer.
// For callers that cannot allocate device memory (code under stream
// capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace hf {

// Capacity of the scratch array in doubles: partial rows of at most
// 65536 - 33 = 65503 doubles (n_rows x (slots + 1)), then one result row of
// slots + 1 <= 33 doubles.  512 KiB per GPU, held until the process ends.
constexpr int64_t kScratchDoubles = 65536;
constexpr int64_t kResultDoubles = kMaxSlots + 1;

}  // namespace hf

static __device__ __align__(256) double scratch[hf::kScratchDoubles];

namespace hf {
namespace {

// Device address of `scratch` per device ordinal, looked up once per device
// with that device current (each GPU holds its own copy of the array).
std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {nullptr};

int scratch_on_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "nll_grad_noalloc: hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(HF_E_INVALID, "nll_grad_noalloc: device ordinal above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "nll_grad_noalloc: hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return HF_OK;
}

}  // namespace
}  // namespace hf

using namespace hf;

extern "C" int nll_grad_noalloc(const pdf_graph* g, void* const* dev_cols, int64_t n_events, hf_precision prec,
                                const double* params, void* hip_stream, double* nll, double* grad) {
  try {
    if (!g || !params || !nll || !grad) return fail(HF_E_INVALID, "nll_grad_noalloc: NULL argument");
    if (n_events < 0 || n_events > (int64_t(1) << 36))
      return fail(HF_E_INVALID, "nll_grad_noalloc: n_events out of range");
    if (prec != HF_FP64 && prec != HF_FP32_EVAL) return fail(HF_E_INVALID, "nll_grad_noalloc: bad precision");
    const int np = (int)g->par.size(), nc = (int)g->obs_of_col.size();
    for (int p = 0; p < np; ++p)
      if (std::isnan(params[p])) return fail(HF_E_INVALID, "nll_grad_noalloc: parameter is NaN");
    if (n_events > 0 && !dev_cols) return fail(HF_E_INVALID, "nll_grad_noalloc: NULL dev_cols");
    const size_t es = prec == HF_FP32_EVAL ? 4 : 8;
    for (int c = 0; c < nc && n_events > 0; ++c) {
      const void* p = dev_cols[g->obs_of_col[c]];
      if (!p) return fail(HF_E_INVALID, "nll_grad_noalloc: NULL column for a used observable");
      if ((uintptr_t)p % es) return fail(HF_E_INVALID, "nll_grad_noalloc: column not aligned to its element size");
    }
    for (int k = 0; k < g->prog.n_nodes; ++k)
      if (g->prog.node[k].op == OP_CONV)
        return fail(HF_E_INVALID, "nll_grad_noalloc: graphs with a convolution need their events sorted "
                                  "(use dataset_upload)");
    if (g->dz.full && !g->dz.fl.empty())
      return fail(HF_E_INVALID, "nll_grad_noalloc: floating resonance shapes re-compute the normalisation grid "
                                "with every evaluation (use nll_grad on an uploaded dataset)");
    if (g->dz.node >= 0 && !g->dz.ready)
      return fail(HF_E_INVALID, "nll_grad_noalloc: the Dalitz normalisation grid is not computed yet (it is, "
                                "once, by the first nll_eval / nll_grad / fit on a dataset of this graph)");
    hipStream_t st = (hipStream_t)hip_stream;
    StagedCall sc;
    stage(g, params, prec, sc, false);
    if (!sc.ok) {
      *nll = INFINITY;
      for (int p = 0; p < np; ++p) grad[p] = NAN;
      return fail(HF_E_DOMAIN, "nll_grad_noalloc: parameters outside the density's domain");
    }
    const int S = g->prog.n_slots;
    double sums[kMaxSlots + 1] = {0.0};
    if (n_events > 0) {
      const int32_t n_rows = rows_for(g->kind, prec, n_events);
      if ((int64_t)n_rows * (S + 1) > kScratchDoubles - kResultDoubles)
        return fail(HF_E_INVALID, "nll_grad_noalloc: the partial rows exceed the 512 KiB scratch array "
                                  "(more than 65503 doubles: rows x (slots + 1))");
      double* sp = nullptr;
      if (int rc = scratch_on_current_device(&sp)) return rc;
      EvalArgs a;
      std::memset(&a, 0, sizeof(a));
      a.prog = sc.prog;
      for (int c = 0; c < nc; ++c) a.col[c] = dev_cols[g->obs_of_col[c]];
      a.n_events = n_events;
      a.partials = sp;
      a.n_rows = n_rows;
      hipError_t e = launch_eval(g->kind, prec == HF_FP32_EVAL, true, a, st);
      if (e != hipSuccess) return hip_fail(e, "nll_grad_noalloc: launch of the likelihood kernel");
      // every row of the partials is written by the kernel before the
      // reduction reads it, so the scratch array needs no clearing
      FitRec fr;
      std::memset(&fr, 0, sizeof(fr));
      fr.partials = sp;
      fr.n_rows = n_rows;
      fr.result = sp + (kScratchDoubles - kResultDoubles);
      fr.n_slots = S;
      fr.active = 1;
      fr.flag = nullptr;
      e = launch_reduce_one(fr, st);
      if (e != hipSuccess) return hip_fail(e, "nll_grad_noalloc: launch of the reduction kernel");
      e = hipMemcpyAsync(sums, fr.result, (S + 1) * sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(e, "nll_grad_noalloc: result copy");
    }
    double v = 0.0, gtmp[kMaxPar];
    assemble(g, sc, n_events > 0 ? sums : nullptr, n_events, &v, gtmp);
    if (!std::isfinite(v)) {
      *nll = INFINITY;
      for (int p = 0; p < np; ++p) grad[p] = gtmp[p];
      return fail(HF_E_DOMAIN, "nll_grad_noalloc: density <= 0 or not finite at some event");
    }
    *nll = v;
    for (int p = 0; p < np; ++p) grad[p] = gtmp[p];
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("nll_grad_noalloc: ") + ex.what());
  }
}
