// Batched likelihood evaluations and the continuous-batching fit engine.
//
// All active fits of one graph are evaluated by one launch of the row
// kernel (each block walks the concatenated row list with a grid stride)
// followed by one launch of the per-fit reduction.  The host side of a step
// writes a fixed-size header, the per-fit records and the per-fit constant
// tables into pinned memory; the device side -- three copies and two kernels
// -- is captured once into a HIP graph and replayed every step, so its shape
// never changes: fit counts and row counts are read from the header in
// device memory, the eval grid is fixed and surplus blocks exit at once.
// Results are written by the reduction straight into mapped pinned memory.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "minimiser.h"
#include "runtime.h"

namespace hf {

std::vector<MinParam> min_params(const pdf_graph* g, hf_precision prec);
MinOptions min_options(const hf_fit_opts* o, hf_precision prec);
int status_code(int st);

// Device-side tables of one batched launch.
struct BatchTables {
  int max_fits = 0, n_const = 0, S = 0;
  BatchHeader* hdr_h = nullptr;
  BatchHeader* hdr_d = nullptr;   // header followed by max_fits FitRec
  double* c64_h = nullptr;
  double* c64_d = nullptr;
  float* c32_h = nullptr;
  float* c32_d = nullptr;
  double* res_h = nullptr;        // mapped pinned, [max_fits][S + 2]: result row, completion flag
  double* res_d = nullptr;
  int64_t seq = 0;                // completion flag value of the last step
  int RS() const { return S + 2; }
  size_t tab_bytes = 0;

  FitRec* fits_h() { return (FitRec*)(hdr_h + 1); }
  FitRec* fits_d() { return (FitRec*)(hdr_d + 1); }

  int alloc(int mf, int nc, int s) {
    max_fits = mf;
    n_const = std::max(nc, 1);
    S = s;
    tab_bytes = sizeof(BatchHeader) + (size_t)mf * sizeof(FitRec);
    hipError_t e;
    if ((e = hipHostMalloc((void**)&hdr_h, tab_bytes, hipHostMallocDefault)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = hipMalloc((void**)&hdr_d, tab_bytes)) != hipSuccess) return hip_fail(e, "batch tables");
    if ((e = hipHostMalloc((void**)&c64_h, (size_t)mf * n_const * 8, hipHostMallocDefault)) != hipSuccess) return hip_fail(e, "batch constants");
    if ((e = hipMalloc((void**)&c64_d, (size_t)mf * n_const * 8)) != hipSuccess) return hip_fail(e, "batch constants");
    if ((e = hipHostMalloc((void**)&c32_h, (size_t)mf * n_const * 4, hipHostMallocDefault)) != hipSuccess) return hip_fail(e, "batch constants");
    if ((e = hipMalloc((void**)&c32_d, (size_t)mf * n_const * 4)) != hipSuccess) return hip_fail(e, "batch constants");
    if ((e = hipHostMalloc((void**)&res_h, (size_t)mf * (S + 2) * 8, hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
      return hip_fail(e, "batch results");
    std::memset(res_h, 0, (size_t)mf * (S + 2) * 8);
    if ((e = hipHostGetDevicePointer((void**)&res_d, res_h, 0)) != hipSuccess) return hip_fail(e, "batch results");
    std::memset(hdr_h, 0, tab_bytes);
    return HF_OK;
  }
  void release() {
    if (hdr_h) hipHostFree(hdr_h);
    if (hdr_d) hipFree(hdr_d);
    if (c64_h) hipHostFree(c64_h);
    if (c64_d) hipFree(c64_d);
    if (c32_h) hipHostFree(c32_h);
    if (c32_d) hipFree(c32_d);
    if (res_h) hipHostFree(res_h);
    hdr_h = nullptr; hdr_d = nullptr; c64_h = nullptr; c64_d = nullptr; c32_h = nullptr; c32_d = nullptr; res_h = nullptr;
  }
};

// Fixed launch shape of the batched eval kernel.
constexpr int kBatchGrid = 2048;

// Enqueues copies + eval + reduce for the tables as filled on the host.
static hipError_t enqueue_step(const pdf_graph* g, bool fp32, BatchTables& t, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(t.hdr_d, t.hdr_h, t.tab_bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t.c64_d, t.c64_h, (size_t)t.max_fits * t.n_const * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(t.c32_d, t.c32_h, (size_t)t.max_fits * t.n_const * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = launch_eval_batched(g->kind, fp32, g->prog, t.hdr_d, t.c64_d, t.c32_d, t.n_const, kBatchGrid, st);
  if (e == hipSuccess) e = launch_reduce(t.fits_d(), t.max_fits, st);
  return e;
}

// Fills the host tables for n fits (datasets ds, staged constants sc).
static void fill_tables(const pdf_graph* g, BatchTables& t, const std::vector<const dataset*>& ds,
                        const std::vector<const StagedCall*>& sc) {
  const int n = (int)ds.size();
  FitRec* fr = t.fits_h();
  int row = 0;
  t.seq += 1;
  for (int i = 0; i < t.max_fits; ++i) {
    std::memset(&fr[i], 0, sizeof(FitRec));
    if (i < n) {
      for (int c = 0; c < kMaxCols; ++c) fr[i].col[c] = ds[i]->col[c];
      fr[i].n_events = ds[i]->n;
      fr[i].partials = ds[i]->partials;
      fr[i].row_begin = row;
      fr[i].n_rows = ds[i]->n_rows;
      fr[i].result = t.res_d + (size_t)i * t.RS();
      fr[i].flag = (int64_t*)(t.res_d + (size_t)i * t.RS() + t.S + 1);
      fr[i].seq = t.seq;
      fr[i].n_slots = g->prog.n_slots;
      fr[i].active = 1;
      row += ds[i]->n_rows;
      std::memcpy(t.c64_h + (size_t)i * t.n_const, sc[i]->prog.c64, g->n_const * sizeof(double));
      std::memcpy(t.c32_h + (size_t)i * t.n_const, sc[i]->prog.c32, g->n_const * sizeof(float));
    }
  }
  t.hdr_h->n_fits = n;
  t.hdr_h->total_rows = row;
}

// Waits until the reduction has set the completion flag of each of the first
// n fits (spinning on mapped host memory, asking the stream every 4096 spins).
static hipError_t wait_fits(const BatchTables& t, int n, hipStream_t st) {
  for (int k = 0; k < n; ++k) {
    const volatile int64_t* flag = (const volatile int64_t*)(t.res_h + (size_t)k * t.RS() + t.S + 1);
    for (uint64_t spin = 1; *flag != t.seq; ++spin) {
      if ((spin & 4095) == 0) {
        const hipError_t e = hipStreamQuery(st);
        if (e == hipSuccess) {
          if (*flag == t.seq) break;
          return hipErrorUnknown;
        }
        if (e != hipErrorNotReady) return e;
      }
      __builtin_ia32_pause();
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return hipSuccess;
}

static void finish_fit(const pdf_graph* g, const dataset* d, const StagedCall& sc, const double* row, double* nll,
                       double* grad) {
  double v = 0.0;
  assemble(g, sc, d->n > 0 ? row : nullptr, d->n, &v, grad);
  *nll = std::isfinite(v) ? v : INFINITY;
}

}  // namespace hf

using namespace hf;

extern "C" int nll_grad_batched(const pdf_graph* g, const dataset* const* d, int32_t n_fits, const double* params,
                                void* hip_stream, double* nll, double* grad) {
  try {
    if (!g || (n_fits > 0 && (!d || !params || !nll || !grad)) || n_fits < 0)
      return fail(HF_E_INVALID, "nll_grad_batched: bad argument");
    if (n_fits == 0) return HF_OK;
    if (g->kind == KIND_TDDPF)
      return fail(HF_E_INVALID, "nll_grad_batched: the full time-dependent model is evaluated one dataset at a time");
    const int np = (int)g->par.size();
    for (int i = 0; i < n_fits; ++i) {
      if (!d[i] || d[i]->g != g) return fail(HF_E_SHAPE, "nll_grad_batched: dataset of another graph");
      if (d[i]->prec != d[0]->prec) return fail(HF_E_SHAPE, "nll_grad_batched: mixed precisions");
      if (d[i]->metric != 0) return fail(HF_E_INVALID, "nll_grad_batched: binned datasets are evaluated one at a time");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (int rc = ensure_grid(const_cast<pdf_graph*>(g), st)) return rc;
    std::vector<StagedCall> sc(n_fits);
    std::vector<const dataset*> ds;
    std::vector<const StagedCall*> scp;
    std::vector<int> which;
    for (int i = 0; i < n_fits; ++i) {
      stage(g, params + (size_t)i * np, d[i]->prec, sc[i]);
      if (sc[i].ok && d[i]->n > 0) {
        ds.push_back(d[i]);
        scp.push_back(&sc[i]);
        which.push_back(i);
      }
    }
    std::vector<double> rows((size_t)n_fits * (g->prog.n_slots + 1), 0.0);
    // A dataset's partial rows serve one fit per launch: fits that repeat a
    // dataset already in the launch go to a following launch (each result
    // is still the one nll_grad gives alone).
    while (!ds.empty()) {
      std::vector<const dataset*> run_ds, rest_ds;
      std::vector<const StagedCall*> run_sc, rest_sc;
      std::vector<int> run_which, rest_which;
      for (size_t k = 0; k < ds.size(); ++k) {
        const bool seen = std::find(run_ds.begin(), run_ds.end(), ds[k]) != run_ds.end();
        (seen ? rest_ds : run_ds).push_back(ds[k]);
        (seen ? rest_sc : run_sc).push_back(scp[k]);
        (seen ? rest_which : run_which).push_back(which[k]);
      }
      BatchTables t;
      int rc = t.alloc((int)run_ds.size(), g->n_const, g->prog.n_slots);
      if (rc) { t.release(); return rc; }
      fill_tables(g, t, run_ds, run_sc);
      hipError_t e = enqueue_step(g, d[0]->prec == HF_FP32_EVAL, t, st);
      if (e == hipSuccess) e = wait_fits(t, (int)run_ds.size(), st);
      if (e != hipSuccess) { t.release(); return hip_fail(e, "nll_grad_batched"); }
      for (size_t k = 0; k < run_ds.size(); ++k)
        std::memcpy(&rows[(size_t)run_which[k] * (g->prog.n_slots + 1)], t.res_h + k * t.RS(),
                    (t.S + 1) * sizeof(double));
      t.release();
      ds.swap(rest_ds);
      scp.swap(rest_sc);
      which.swap(rest_which);
    }
    for (int i = 0; i < n_fits; ++i) {
      if (!sc[i].ok) {
        nll[i] = INFINITY;
        for (int p = 0; p < np; ++p) grad[(size_t)i * np + p] = NAN;
        continue;
      }
      finish_fit(g, d[i], sc[i], &rows[(size_t)i * (g->prog.n_slots + 1)], &nll[i], &grad[(size_t)i * np]);
    }
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("nll_grad_batched: ") + ex.what());
  }
}

// ---------------------------------------------------------------------- engine
struct batch_engine {
  struct Slot {
    bool used = false, running = false;
    const dataset* d = nullptr;
    int64_t tag = 0;
    Minimiser m;
    std::vector<double> x, g;
    StagedCall sc;
    int64_t bytes = 0;
    int n_eval = 0;
    int status_override = 0;  // nonzero: the fit ended by an injected failure
  };
  // Failure injection from the host (HIPFIT_FAULT="tag:eval:kind" at
  // batch_create): when the fit with that tag receives its eval-th
  // evaluation, "domain" replaces the result by NLL = +inf (as a density <= 0
  // would: the fit's line search backs off), "abort" ends that fit with
  // status HF_E_HIP.  The kernels are untouched; the other fits must not
  // notice (their results stay bitwise the same).
  struct Fault {
    int64_t tag = -1;
    int eval = -1;
    int kind = 0;  // 1 domain, 2 abort
  } fault;
  const pdf_graph* g = nullptr;
  int max_slots = 0;
  int64_t budget = 0, in_use = 0;
  hipStream_t st = nullptr;
  bool prec_set = false;
  hf_precision prec = HF_FP64;
  std::vector<Slot> slots;
  BatchTables t;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
};

extern "C" int batch_create(const pdf_graph* g, int32_t max_slots, int64_t hbm_budget_bytes, void* hip_stream,
                            batch_engine** out) {
  try {
    if (!g || !out) return fail(HF_E_INVALID, "batch_create: NULL argument");
    if (max_slots < 1 || max_slots > 4096) return fail(HF_E_INVALID, "batch_create: max_slots out of range");
    if (hbm_budget_bytes <= 0) return fail(HF_E_INVALID, "batch_create: budget must be positive");
    (void)hip_stream;
    std::unique_ptr<batch_engine> b(new batch_engine);
    b->g = g;
    b->max_slots = max_slots;
    b->budget = hbm_budget_bytes;
    b->slots.resize(max_slots);
    const char* ng = std::getenv("HIPFIT_NO_GRAPH");
    b->use_graph = !(ng && ng[0] == '1');
    if (const char* fe = std::getenv("HIPFIT_FAULT")) {
      long long tag = -1;
      int ev = -1;
      char kind[16] = {0};
      if (std::sscanf(fe, "%lld:%d:%15s", &tag, &ev, kind) != 3 || ev < 0 ||
          (std::strcmp(kind, "domain") != 0 && std::strcmp(kind, "abort") != 0))
        return fail(HF_E_INVALID, "batch_create: HIPFIT_FAULT must be tag:eval:domain or tag:eval:abort");
      b->fault.tag = tag;
      b->fault.eval = ev;
      b->fault.kind = std::strcmp(kind, "domain") == 0 ? 1 : 2;
    }
    hipError_t e = hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "batch_create: stream");
    if (int rc = b->t.alloc(max_slots, g->n_const, g->prog.n_slots)) {
      b->t.release();
      hipStreamDestroy(b->st);
      return rc;
    }
    *out = b.release();
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("batch_create: ") + ex.what());
  }
}

extern "C" void batch_destroy(batch_engine* b) {
  if (!b) return;
  if (b->st) hipStreamSynchronize(b->st);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->t.release();
  if (b->st) hipStreamDestroy(b->st);
  delete b;
}

extern "C" int batch_admit(batch_engine* b, const dataset* d, const double* params_init, const hf_fit_opts* opts,
                           int64_t tag, int32_t* slot_out) {
  try {
    if (!b || !d || !params_init) return fail(HF_E_INVALID, "batch_admit: NULL argument");
    if (d->g != b->g) return fail(HF_E_SHAPE, "batch_admit: dataset of another graph");
    if (d->metric != 0) return fail(HF_E_INVALID, "batch_admit: binned datasets are fitted one at a time");
    if (b->g->kind == KIND_TDDPF)
      return fail(HF_E_INVALID, "batch_admit: the full time-dependent model is fitted one dataset at a time");
    if (opts && opts->grad_mode != 0) return fail(HF_E_INVALID, "batch_admit: only the analytic gradient is batched");
    if (b->prec_set && d->prec != b->prec) return fail(HF_E_INVALID, "batch_admit: precision differs from the engine's");
    if (d->bytes > b->budget) return fail(HF_E_INVALID, "batch_admit: dataset larger than the whole budget");
    for (auto& s : b->slots)
      if (s.used && s.d == d) return fail(HF_E_INVALID, "batch_admit: dataset already admitted");
    int free_slot = -1;
    for (int i = 0; i < b->max_slots; ++i)
      if (!b->slots[i].used) { free_slot = i; break; }
    if (free_slot < 0) return fail(HF_E_FULL, "batch_admit: no free slot");
    if (b->in_use + d->bytes > b->budget) return fail(HF_E_BUDGET, "batch_admit: budget exhausted");
    for (size_t p = 0; p < b->g->par.size(); ++p)
      if (!std::isfinite(params_init[p])) return fail(HF_E_INVALID, "batch_admit: start value not finite");
    auto& s = b->slots[free_slot];
    s.used = true;
    s.running = true;
    s.d = d;
    s.tag = tag;
    s.bytes = d->bytes;
    s.n_eval = 0;
    s.status_override = 0;
    s.m.start(min_params(b->g, d->prec), params_init, min_options(opts, d->prec));
    b->in_use += d->bytes;
    b->prec = d->prec;
    b->prec_set = true;
    if (slot_out) *slot_out = free_slot;
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("batch_admit: ") + ex.what());
  }
}

static void retire_running(batch_engine* b, batch_engine::Slot& s) {
  s.running = false;
  b->in_use -= s.bytes;
}

// The injected failure, if this evaluation of this fit is the chosen one:
// true when the fit was ended ("abort"); f replaced by +inf ("domain").
static bool inject_fault(batch_engine* b, batch_engine::Slot& s, double& f) {
  if (s.tag != b->fault.tag || s.n_eval != b->fault.eval) return false;
  if (b->fault.kind == 1) {
    f = INFINITY;
    for (double& v : s.g) v = 0.0;  // as the host answers a point outside the domain
    return false;
  }
  s.status_override = HF_E_HIP;
  retire_running(b, s);
  return true;
}

extern "C" int batch_step(batch_engine* b, int32_t* n_active_out, int32_t* n_done_out) {
  try {
    if (!b) return fail(HF_E_INVALID, "batch_step: NULL engine");
    const pdf_graph* g = b->g;
    if (int rc = ensure_grid(const_cast<pdf_graph*>(g), b->st)) return rc;
    const int np = (int)g->par.size();
    std::vector<const dataset*> ds;
    std::vector<const StagedCall*> scp;
    std::vector<int> idx;
    for (int i = 0; i < b->max_slots; ++i) {
      auto& s = b->slots[i];
      if (!s.running) continue;
      // points outside the domain, and empty datasets, are answered on the host
      while (s.running) {
        if (!s.m.ask(s.x)) { retire_running(b, s); break; }
        stage(g, s.x.data(), s.d->prec, s.sc);
        if (s.sc.ok && s.d->n > 0) break;
        s.g.assign(np, 0.0);
        double f = INFINITY;
        if (s.sc.ok) finish_fit(g, s.d, s.sc, nullptr, &f, s.g.data());
        ++s.n_eval;
        if (inject_fault(b, s, f)) break;
        s.m.tell(f, s.g);
      }
      if (!s.running) continue;
      ds.push_back(s.d);
      scp.push_back(&s.sc);
      idx.push_back(i);
    }
    if (!ds.empty()) {
      fill_tables(g, b->t, ds, scp);
      hipError_t e = hipSuccess;
      const bool fp32 = b->prec == HF_FP32_EVAL;
      if (b->use_graph) {
        if (!b->exec) {
          e = hipStreamBeginCapture(b->st, hipStreamCaptureModeRelaxed);
          if (e == hipSuccess) {
            hipError_t e2 = enqueue_step(g, fp32, b->t, b->st);
            e = hipStreamEndCapture(b->st, &b->graph);
            if (e2 != hipSuccess) e = e2;
          }
          if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
          if (e != hipSuccess) return hip_fail(e, "batch_step: graph capture");
        }
        e = hipGraphLaunch(b->exec, b->st);
      } else {
        e = enqueue_step(g, fp32, b->t, b->st);
      }
      if (e == hipSuccess) e = wait_fits(b->t, (int)ds.size(), b->st);
      if (e != hipSuccess) return hip_fail(e, "batch_step: launch");
      for (size_t k = 0; k < ds.size(); ++k) {
        auto& s = b->slots[idx[k]];
        s.g.assign(np, 0.0);
        double f;
        finish_fit(g, s.d, s.sc, b->t.res_h + k * b->t.RS(), &f, s.g.data());
        ++s.n_eval;
        if (inject_fault(b, s, f)) continue;
        s.m.tell(f, s.g);
        if (s.m.done()) retire_running(b, s);
      }
    }
    int act = 0, done = 0;
    for (auto& s : b->slots) {
      if (s.used && s.running) ++act;
      if (s.used && !s.running) ++done;
    }
    if (n_active_out) *n_active_out = act;
    if (n_done_out) *n_done_out = done;
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("batch_step: ") + ex.what());
  }
}

extern "C" int batch_poll(batch_engine* b, int32_t max, int64_t* tags, int32_t* status, double* params,
                          double* errors, double* nll, int32_t* n_eval) {
  if (!b) return fail(HF_E_INVALID, "batch_poll: NULL engine");
  const int np = (int)b->g->par.size();
  int k = 0;
  for (auto& s : b->slots) {
    if (k >= max) break;
    if (!s.used || s.running) continue;
    if (tags) tags[k] = s.tag;
    if (status) status[k] = s.status_override ? s.status_override : status_code(s.m.status);
    if (params) std::memcpy(params + (size_t)k * np, s.m.x_best.data(), np * sizeof(double));
    if (errors) std::memcpy(errors + (size_t)k * np, s.m.err.data(), np * sizeof(double));
    if (nll) nll[k] = s.m.f_best;
    if (n_eval) n_eval[k] = s.n_eval;
    s.used = false;
    s.d = nullptr;
    ++k;
  }
  return k;
}

extern "C" int batch_cancel(batch_engine* b, int64_t tag) {
  if (!b) return fail(HF_E_INVALID, "batch_cancel: NULL engine");
  for (auto& s : b->slots)
    if (s.used && s.tag == tag) {
      if (s.running) retire_running(b, s);
      s.used = false;
      s.d = nullptr;
      return HF_OK;
    }
  return fail(HF_E_INVALID, "batch_cancel: no fit with that tag");
}
