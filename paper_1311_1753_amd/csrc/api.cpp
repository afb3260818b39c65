// Datasets and likelihood evaluations of the C ABI.
//
// A dataset is one device allocation: structure-of-arrays event columns
// (each 256-byte aligned, float offsets from a per-column double reference in
// the FP32-eval path, raw doubles in the FP64 path) followed by the per-tile
// partial rows of the reduction.  An evaluation stages the constant table on
// the host, launches the tile kernel and the fixed-order reduction on the
// caller's stream, and reads the reduced row from pinned, device-mapped host
// memory written directly by the reduction kernel.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "runtime.h"

namespace hf {

namespace {

// Pinned staging buffer shared by uploads (serialised by a mutex).
std::mutex g_stage_mu;
void* g_stage = nullptr;
size_t g_stage_bytes = 0;
constexpr size_t kStageChunk = size_t(32) << 20;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Optional kernel timing (hf_profile): HIP events that take the start and
// end time stamps of the likelihood kernel's and the reduction's dispatches
// (hipExtLaunchKernel) of every `every`-th eval_one.  The evaluation itself
// waits as usual (on the completion flag); its time stamps are read at the
// next profiled evaluation or when the profile is read, by when they are
// complete, so profiling adds no synchronisation to the timed calls.
struct Profile {
  bool on = false;
  bool init = false;
  bool pending = false;  // events of a profiled evaluation not yet read
  int every = 1;
  int64_t calls = 0;
  hipEvent_t e[4];
  double eval_ms = 0.0, reduce_ms = 0.0;
  int64_t n = 0;
};
static Profile g_prof;
static std::mutex g_prof_mu;

static hipError_t prof_harvest() {
  if (!g_prof.pending) return hipSuccess;
  hipError_t e = hipEventSynchronize(g_prof.e[3]);
  if (e != hipSuccess) return e;
  float t1 = 0.f, t2 = 0.f;
  if ((e = hipEventElapsedTime(&t1, g_prof.e[0], g_prof.e[1])) != hipSuccess) return e;
  if ((e = hipEventElapsedTime(&t2, g_prof.e[2], g_prof.e[3])) != hipSuccess) return e;
  g_prof.eval_ms += t1;
  g_prof.reduce_ms += t2;
  g_prof.n += 1;
  g_prof.pending = false;
  return hipSuccess;
}

// Layout of a dataset's mapped result row: the reduced sums of an
// evaluation and their completion flag, then (the full time-dependent model
// with floating shapes) the reduced grid sums of its normalisation and
// their flag.
constexpr int kResFlag = kMaxSlots + 1;
constexpr int kNormRes = kMaxSlots + 2;
constexpr int kNormFlag = kNormRes + kMaxSlots + 1;
constexpr int kResultDoubles = kNormFlag + 1;

// Waits for the reduction of one evaluation: spins on the flag that the
// reduction kernel sets after its result is visible in mapped host memory,
// asking the stream every 4096 spins (errors, or a finished stream without
// the flag, end the wait).
static hipError_t wait_result(const dataset* d, hipStream_t st, int flag_at = kResFlag) {
  const volatile int64_t* flag = (const volatile int64_t*)(d->res_host + flag_at);
  for (uint64_t spin = 1;; ++spin) {
    if (*flag == d->seq) {
      std::atomic_thread_fence(std::memory_order_acquire);
      return hipSuccess;
    }
    if ((spin & 4095) == 0) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        if (*flag == d->seq) {
          std::atomic_thread_fence(std::memory_order_acquire);
          return hipSuccess;
        }
        return hipErrorUnknown;
      }
      if (e != hipErrorNotReady) return e;
    }
    __builtin_ia32_pause();
  }
}

static int ensure_result_buffer(const dataset* dc) {
  dataset* d = const_cast<dataset*>(dc);
  if (d->res_host) return HF_OK;
  void* h = nullptr;
  hipError_t e = hipHostMalloc(&h, kResultDoubles * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(result row)");
  std::memset(h, 0, kResultDoubles * sizeof(double));  // flags 0: no evaluation finished yet
  void* dv = nullptr;
  e = hipHostGetDevicePointer(&dv, h, 0);
  if (e != hipSuccess) {
    hipHostFree(h);
    return hip_fail(e, "hipHostGetDevicePointer");
  }
  d->res_host = (double*)h;
  d->res_dev = (double*)dv;
  return HF_OK;
}

// One evaluation of a binned dataset: the tree interpreter with the metric,
// then the reduction of its [metric, slots, sum of dmetric/dlnP] columns.
static int eval_binned(const pdf_graph* g, const dataset* d, const StagedCall& sc, hipStream_t st, bool want_grad,
                       double* value, double* grad) {
  const int S = g->n_slots_tree;
  std::vector<double> sums(S + 2, 0.0);
  if (d->n > 0) {
    if (int rc = ensure_result_buffer(d)) return rc;
    EvalArgs a;
    std::memset(&a, 0, sizeof(a));
    a.prog = sc.prog;
    a.prog.n_slots = S;
    for (int c = 0; c < kMaxCols; ++c) a.col[c] = d->col[c];
    a.n_events = d->n;
    a.partials = d->partials;
    a.n_rows = d->n_rows;
    a.metric = d->metric;
    a.wcol = d->wcol;
    a.kfac = d->wsum * d->volume;
    a.lnL = sc.ht.lnN;
    bool heavy = g->dz.node >= 0 || S > 8 || g->prog.n_cols > 2 || g->prog.n_nodes > 8;
    for (int k = 0; k < g->prog.n_nodes; ++k)
      heavy = heavy || g->prog.node[k].op == OP_CONV;
    hipError_t e = launch_binned(d->prec == HF_FP32_EVAL, want_grad, heavy ? (g->dz.node >= 0 ? 2 : 1) : 0, a, st);
    if (e != hipSuccess) return hip_fail(e, "launch of the binned kernel");
    FitRec fr;
    std::memset(&fr, 0, sizeof(fr));
    fr.partials = d->partials;
    fr.n_rows = d->n_rows;
    fr.result = d->res_dev;
    fr.n_slots = want_grad ? S + 1 : 0;
    fr.active = 1;
    dataset* dm = const_cast<dataset*>(d);
    dm->seq += 1;
    fr.flag = (int64_t*)(d->res_dev + kResFlag);
    fr.seq = d->seq;
    e = launch_reduce_one(fr, st);
    if (e != hipSuccess) return hip_fail(e, "launch of the reduction kernel");
    e = wait_result(d, st);
    if (e != hipSuccess) return hip_fail(e, "waiting for the reduction");
    for (int j = 0; j < (want_grad ? S + 2 : 1); ++j) sums[j] = d->res_host[j];
  }
  double v = 0.0;
  assemble_binned(g, sc, d->n > 0 ? sums.data() : nullptr, &v, grad);
  if (!std::isfinite(v)) {
    *value = INFINITY;
    return fail(HF_E_DOMAIN, "density <= 0 or not finite at a bin with weight");
  }
  *value = v;
  return HF_OK;
}

// The full time-dependent model with floating resonance shapes: the grid
// kernel at this theta (constants of `sc`, column references 0) and its
// reduction into the normalisation area of the dataset's result row, which
// the reduction marks with the dataset's next sequence number (the caller's
// evaluation then uses the same number for its own flag).
static int launch_grid_norm(const pdf_graph* g, const dataset* d, const StagedCall& sc, bool want_grad,
                            hipStream_t st) {
  const DalitzInfo& dz = g->dz;
  if (!d->norm_partials) {
    // the dataset's own rows, so that evaluations of different datasets of
    // one graph may overlap
    dataset* dm = const_cast<dataset*>(d);
    hipError_t e = hipMalloc(&dm->norm_partials, (size_t)dz.norm_cols * dz.norm_rows * sizeof(double));
    if (e != hipSuccess) {
      dm->norm_partials = nullptr;
      return hip_fail(e, "hipMalloc(normalisation grid partials)");
    }
  }
  const KNode& kn = sc.prog.node[dz.node];
  NormArgs na;
  std::memset(&na, 0, sizeof(na));
  na.prog = sc.prog;
  for (int i : {kDzRef12, kDzRef13}) {
    na.prog.c64[kn.c0 + i] = 0.0;
    na.prog.c32[kn.c0 + i] = 0.0f;
  }
  na.gs = dz.gs;
  na.cells = dz.norm_cells;
  na.n_cells = dz.n_norm_cells;
  na.partials = d->norm_partials;
  na.n_rows = dz.norm_rows;
  hipError_t e = launch_full_norm(want_grad, na, st);
  if (e != hipSuccess) return hip_fail(e, "launch of the normalisation grid kernel");
  const int R = (int)dz.res.size();
  FitRec fr;
  std::memset(&fr, 0, sizeof(fr));
  fr.partials = d->norm_partials;
  fr.n_rows = dz.norm_rows;
  fr.result = d->res_dev + kNormRes;
  fr.n_slots = want_grad ? 2 * R + 3 + (dz.hq ? 2 : 0) + 2 * (int)dz.fl.size() : 3;
  fr.active = 1;
  fr.flag = (int64_t*)(d->res_dev + kNormFlag);
  fr.seq = d->seq + 1;
  e = launch_reduce_one(fr, st);
  if (e != hipSuccess) return hip_fail(e, "launch of the normalisation reduction");
  return HF_OK;
}

// ln N and its derivatives from the grid sums (read after the reduction's
// flag): N = area [sum |A|^2 (kc + kz)/2 + sum |Abar'|^2 (kc - kz)/2 +
// sum a_s ks + sum b_s kzs], the coefficient, q/p and shape derivatives
// summed by the kernel, those in tau, y and x from the four sums.
static int grid_norm_terms(const pdf_graph* g, const dataset* d, const double* th, bool want_grad, StagedCall& sc) {
  const DalitzInfo& dz = g->dz;
  const double* v = d->res_host + kNormRes;
  const int R = (int)dz.res.size();
  const int nl = want_grad ? 1 + 2 * R : 1;  // |Abar'|^2 follows the LDS columns
  const double area = dz.gs.h12 * dz.gs.h13;
  const double IA = area * v[0], IB = area * v[nl], AS = area * v[nl + 1], BS = area * v[nl + 2];
  const double kc = sc.tint[0], kz = sc.tint[1], ks = sc.tint[2], kzs = sc.tint[3];
  const double N = 0.5 * (IA + IB) * kc + 0.5 * (IA - IB) * kz + AS * ks + BS * kzs;
  if (!(N > 0.0) || !std::isfinite(N)) return fail(HF_E_DOMAIN, "normalisation <= 0 or not finite");
  sc.ht.lnN += std::log(N);
  if (!want_grad) return HF_OK;
  const NodeInfo& nd = g->nodes[dz.node];
  for (int j = 0; j < 2 * R; ++j) sc.ht.dlnN[nd.par[j]] += area * v[1 + j] / N;
  int q = nl + 3;
  if (dz.hq) {
    sc.ht.dlnN[dz.p_qm] += area * v[q] / N;
    sc.ht.dlnN[dz.p_qa] += area * v[q + 1] / N;
    q += 2;
  }
  for (const FloatRes& f : dz.fl) {
    sc.ht.dlnN[f.p_m0] += area * v[q] / N;
    sc.ht.dlnN[f.p_g0] += area * v[q + 1] / N;
    q += 2;
  }
  const double tau = th[dz.p_tau], y = th[dz.p_y], x = dz.p_x >= 0 ? th[dz.p_x] : 0.0;
  const double X = -AS, Y = -BS, den = 1.0 - y * y, opx = 1.0 + x * x;
  const double dtau = 0.5 * (IA + IB) / den + 0.5 * (IA - IB) / opx - X * y / den - Y * x / opx;
  const double dy = 0.5 * (IA + IB) * tau * 2.0 * y / (den * den) - X * tau * (1.0 + y * y) / (den * den);
  sc.ht.dlnN[dz.p_tau] += dtau / N;
  sc.ht.dlnN[dz.p_y] += dy / N;
  if (dz.p_x >= 0)
    sc.ht.dlnN[dz.p_x] += (-0.5 * (IA - IB) * tau * 2.0 * x / (opx * opx) - Y * tau * (1.0 - x * x) / (opx * opx)) / N;
  return HF_OK;
}

int eval_one(const pdf_graph* g, const dataset* d, const double* th, hipStream_t st, bool want_grad, double* nll,
             double* grad) {
  const int np = (int)g->par.size();
  if (int rc = ensure_grid(const_cast<pdf_graph*>(g), st)) return rc;
  StagedCall sc;
  stage(g, th, d->prec, sc, d->metric != 0);
  if (!sc.ok) {
    *nll = INFINITY;
    if (grad) for (int p = 0; p < np; ++p) grad[p] = NAN;
    return fail(HF_E_DOMAIN, "parameters outside the density's domain");
  }
  if (d->metric != 0) return eval_binned(g, d, sc, st, want_grad, nll, grad);
  const int S = g->prog.n_slots;
  std::vector<double> sums(S + 1, 0.0);
  if (d->n > 0) {
    if (int rc = ensure_result_buffer(d)) return rc;
    EvalArgs a;
    a.prog = sc.prog;
    for (int c = 0; c < kMaxCols; ++c) a.col[c] = d->col[c];
    a.n_events = d->n;
    a.partials = d->partials;
    a.n_rows = d->n_rows;
    a.metric = 0;
    a.wcol = nullptr;
    a.kfac = 0.0;
    a.lnL = 0.0;
    const bool prof = g_prof.on && (g_prof.calls++ % g_prof.every) == 0;
    if (prof) {
      hipError_t e = prof_harvest();
      if (e != hipSuccess) return hip_fail(e, "profile events");
    }
    if (sc.grid_norm)
      if (int rc = launch_grid_norm(g, d, sc, want_grad, st)) return rc;
    hipError_t e = launch_eval(g->kind, d->prec == HF_FP32_EVAL, want_grad, a, st, prof ? g_prof.e[0] : nullptr,
                               prof ? g_prof.e[1] : nullptr);
    if (e != hipSuccess) return hip_fail(e, "launch of the likelihood kernel");
    FitRec fr;
    std::memset(&fr, 0, sizeof(fr));
    fr.partials = d->partials;
    fr.n_rows = d->n_rows;
    fr.result = d->res_dev;
    fr.n_slots = want_grad ? S : 0;
    fr.active = 1;
    dataset* dm = const_cast<dataset*>(d);
    dm->seq += 1;
    fr.flag = (int64_t*)(d->res_dev + kResFlag);
    fr.seq = d->seq;
    e = launch_reduce_one(fr, st, prof ? g_prof.e[2] : nullptr, prof ? g_prof.e[3] : nullptr);
    if (e != hipSuccess) return hip_fail(e, "launch of the reduction kernel");
    e = wait_result(d, st);
    if (e == hipSuccess && sc.grid_norm) e = wait_result(d, st, kNormFlag);
    if (e != hipSuccess) return hip_fail(e, "waiting for the reduction");
    if (prof) g_prof.pending = true;
    for (int j = 0; j < (want_grad ? S + 1 : 1); ++j) sums[j] = d->res_host[j];
    if (sc.grid_norm)
      if (int rc = grid_norm_terms(g, d, th, want_grad, sc)) {
        *nll = INFINITY;
        return rc;
      }
  }
  double v = 0.0;
  assemble(g, sc, d->n > 0 ? sums.data() : nullptr, d->n, &v, grad);
  if (!std::isfinite(v)) {
    *nll = INFINITY;
    return fail(HF_E_DOMAIN, "density <= 0 or not finite at some event");
  }
  *nll = v;
  return HF_OK;
}

}  // namespace hf

using namespace hf;

// Upload of an unbinned dataset (metric 0) or of bin centres with weights
// (metric 1 or 2).
// Allocates a dataset of n events for graph g: one device block holding the
// columns (256-byte aligned, storage format of `prec`), the binned weights
// (metric != 0) and the partial rows of the evaluation kernels.
// Sizes of that block's parts.
struct DatasetLayout {
  int32_t n_rows;
  size_t col_bytes, w_bytes, part_bytes, total;
};
static DatasetLayout dataset_layout(const pdf_graph* g, int64_t n, hf_precision prec, int metric) {
  DatasetLayout L;
  const int nc = (int)g->obs_of_col.size();
  const size_t es = prec == HF_FP32_EVAL ? 4 : 8;
  // binned datasets run the tree interpreter: one event per chunk and
  // thread, partial columns [metric, tree slots, sum of dmetric/dlnP]
  L.n_rows = rows_for(metric ? (int)KIND_TREE : g->kind, prec, n);
  const int part_cols = metric ? g->n_slots_tree + 2 : g->prog.n_slots + 1;
  L.col_bytes = align256((size_t)n * es);
  L.w_bytes = metric ? align256((size_t)n * sizeof(double)) : 0;
  L.part_bytes = align256((size_t)std::max<int32_t>(L.n_rows, 1) * part_cols * sizeof(double));
  L.total = L.col_bytes * nc + L.w_bytes + L.part_bytes;
  return L;
}

static int make_dataset(const pdf_graph* g, int64_t n, hf_precision prec, int metric, double volume, const char* who,
                        std::unique_ptr<dataset>& d) {
  d.reset(new dataset);
  const int nc = (int)g->obs_of_col.size();
  d->g = g;
  d->prec = prec;
  d->n = n;
  d->n_cols = nc;
  d->metric = metric;
  d->volume = volume;
  const DatasetLayout L = dataset_layout(g, n, prec, metric);
  d->n_rows = L.n_rows;
  const size_t col_bytes = L.col_bytes, w_bytes = L.w_bytes, total = L.total;
  void* blk = nullptr;
  hipError_t e = hipMalloc(&blk, total);
  if (e != hipSuccess) {
    d.reset();
    return fail(HF_E_OOM, std::string(who) + ": hipMalloc: " + hipGetErrorString(e));
  }
  d->block = blk;
  d->bytes = (int64_t)total;
  char* base = (char*)blk;
  for (int c = 0; c < nc; ++c) {
    d->col[c] = base + c * col_bytes;
    d->ref[c] = column_ref(g, c, prec);
  }
  d->partials = (double*)(base + nc * col_bytes + w_bytes);
  if (metric) d->wcol = (const double*)(base + nc * col_bytes);
  return HF_OK;
}

static int upload(const pdf_graph* g, const double* const* host_cols, int64_t n, hf_precision prec,
                  void* hip_stream, int metric, const double* weights, double volume, dataset** out) {
  try {
    if (!g || !out || (n > 0 && !host_cols)) return fail(HF_E_INVALID, "dataset_upload: NULL argument");
    if (n < 0 || n > (int64_t(1) << 36)) return fail(HF_E_INVALID, "dataset_upload: n_events out of range");
    if (prec != HF_FP64 && prec != HF_FP32_EVAL) return fail(HF_E_INVALID, "dataset_upload: bad precision");
    hipStream_t st = (hipStream_t)hip_stream;
    const int nc = (int)g->obs_of_col.size();
    // validation on the host: every value inside its box, Dalitz points inside the plot
    for (int c = 0; c < nc && n > 0; ++c) {
      const int o = g->obs_of_col[c];
      const double* x = host_cols[o];
      if (!x) return fail(HF_E_INVALID, "dataset_upload: NULL column for a used observable");
      const double lo = g->obs[o].lo, hi = g->obs[o].hi;
      for (int64_t i = 0; i < n; ++i)
        if (!(x[i] >= lo && x[i] <= hi) || !std::isfinite(x[i]))
          return fail(HF_E_DOMAIN, "dataset_upload: event " + std::to_string(i) + " outside the box of '" +
                                       g->obs[o].name + "'");
    }
    if (g->dz.node >= 0 && n > 0) {
      const NodeInfo& nd = g->nodes[g->dz.node];
      const double* a = host_cols[nd.obs[0]];
      const double* b = host_cols[nd.obs[1]];
      for (int64_t i = 0; i < n; ++i)
        if (!dalitz_inside(g->dz, a[i], b[i]))
          return fail(HF_E_DOMAIN, "dataset_upload: event " + std::to_string(i) + " outside the Dalitz plot");
      if (g->dz.tddp) {
        const double* s = host_cols[nd.obs[3]];
        for (int64_t i = 0; i < n; ++i)
          if (!(s[i] > 0.0)) return fail(HF_E_DOMAIN, "dataset_upload: sigma_t must be > 0");
      }
    }
    std::unique_ptr<dataset> d;
    if (int rc = make_dataset(g, n, prec, metric, volume, "dataset_upload", d)) return rc;
    const size_t es = prec == HF_FP32_EVAL ? 4 : 8;
    void* blk = d->block;
    hipError_t e = hipSuccess;
    if (metric) {
      double ws = 0.0;
      for (int64_t i = 0; i < n; ++i) ws += weights[i];
      d->wsum = ws;
      if (n > 0) {
        e = hipMemcpy((void*)d->wcol, weights, (size_t)n * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) { hipFree(blk); return hip_fail(e, "dataset_upload_binned: weights"); }
      }
    }

    // events of graphs with a CONV node are stored sorted by that node's
    // observable (the likelihood is a sum over events; neighbouring events
    // then share their grid ranges, and a wave skips the grid points none of
    // its events reaches)
    std::vector<int64_t> perm;
    if (!metric && n > 1)
      for (const NodeInfo& nd : g->nodes)
        if (nd.op == OP_CONV) {
          const double* key = host_cols[nd.obs[0]];
          perm.resize(n);
          for (int64_t i = 0; i < n; ++i) perm[i] = i;
          std::stable_sort(perm.begin(), perm.end(), [key](int64_t a, int64_t b) { return key[a] < key[b]; });
          break;
        }
    // convert through the pinned staging buffer, one chunk at a time
    if (n > 0) {
      std::lock_guard<std::mutex> lk(g_stage_mu);
      if (!g_stage) {
        e = hipHostMalloc(&g_stage, kStageChunk, hipHostMallocDefault);
        if (e != hipSuccess) { g_stage = nullptr; hipFree(blk); return hip_fail(e, "hipHostMalloc(staging)"); }
        g_stage_bytes = kStageChunk;
      }
      const int64_t per = (int64_t)(g_stage_bytes / es);
      for (int c = 0; c < nc; ++c) {
        const double* x = host_cols[g->obs_of_col[c]];
        const double ref = d->ref[c];
        for (int64_t b = 0; b < n; b += per) {
          const int64_t m = std::min(per, n - b);
          if (!perm.empty()) {
            if (es == 4) {
              float* s = (float*)g_stage;
              for (int64_t i = 0; i < m; ++i) s[i] = (float)(x[perm[b + i]] - ref);
            } else {
              double* s = (double*)g_stage;
              for (int64_t i = 0; i < m; ++i) s[i] = x[perm[b + i]];
            }
          } else if (es == 4) {
            float* s = (float*)g_stage;
            for (int64_t i = 0; i < m; ++i) s[i] = (float)(x[b + i] - ref);
          } else {
            std::memcpy(g_stage, x + b, (size_t)m * 8);
          }
          e = hipMemcpyAsync((char*)d->col[c] + b * es, g_stage, (size_t)m * es, hipMemcpyHostToDevice, st);
          if (e == hipSuccess) e = hipStreamSynchronize(st);
          if (e != hipSuccess) { hipFree(blk); return hip_fail(e, "dataset_upload: copy"); }
        }
      }
    }
    *out = d.release();
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("dataset_upload: ") + ex.what());
  }
}

extern "C" int dataset_upload(const pdf_graph* g, const double* const* host_cols, int64_t n, hf_precision prec,
                              void* hip_stream, dataset** out) {
  return upload(g, host_cols, n, prec, hip_stream, 0, nullptr, 0.0, out);
}

extern "C" int dataset_upload_binned(const pdf_graph* g, const double* const* centres, const double* weights,
                                     int64_t n_bins, double bin_volume, int32_t metric, hf_precision prec,
                                     void* hip_stream, dataset** out) {
  if (metric != HF_METRIC_BNLL && metric != HF_METRIC_CHI2)
    return fail(HF_E_INVALID, "dataset_upload_binned: metric must be HF_METRIC_BNLL or HF_METRIC_CHI2");
  if (!(bin_volume > 0.0) || !std::isfinite(bin_volume))
    return fail(HF_E_INVALID, "dataset_upload_binned: bin volume must be positive");
  if (!g) return fail(HF_E_INVALID, "dataset_upload_binned: NULL graph");
  if (g->n_slots_tree + 2 > kMaxSlotsTree + 1)
    return fail(HF_E_GRAPH, "dataset_upload_binned: more than 31 gradient slots");
  if (g->dz.full) return fail(HF_E_GRAPH, "dataset_upload_binned: the full time-dependent model is unbinned only");
  if (n_bins > 0 && !weights) return fail(HF_E_INVALID, "dataset_upload_binned: NULL weights");
  for (int64_t i = 0; i < n_bins; ++i)
    if (!(weights[i] >= 0.0) || !std::isfinite(weights[i]))
      return fail(HF_E_INVALID, "dataset_upload_binned: weights must be finite and >= 0");
  return upload(g, centres, n_bins, prec, hip_stream, metric, weights, bin_volume, out);
}

// ---------------------------------------------------------------- toy generation
namespace {

// Sampling table of a graph at parameters th: the factors (root PROD
// children, or the root) with their leaves.  HF_E_GRAPH for a tree that is
// not sampleable, HF_E_DOMAIN for parameters outside the density's domain.
int gen_table(const pdf_graph* g, const double* th, GenArgs& a) {
  const int NN = (int)g->nodes.size();
  const NodeInfo& root = g->nodes[NN - 1];
  std::vector<int> factors;
  if (root.op == OP_PROD) factors = root.child;
  else factors = {NN - 1};
  if ((int)factors.size() > kMaxCols) return fail(HF_E_GRAPH, "dataset_generate: too many factors");
  const char* kShape =
      "dataset_generate: sampleable graphs are EXP / GAUSS leaves, ADDs of up to 4 such leaves on one "
      "observable, and PRODs of those";
  int nl = 0;
  a.n_factor = (int)factors.size();
  for (int f = 0; f < a.n_factor; ++f) {
    const NodeInfo& fn = g->nodes[factors[f]];
    std::vector<int> leaves;
    if (fn.op == OP_ADD) leaves = fn.child;
    else leaves = {factors[f]};
    if ((int)leaves.size() > kMaxGenLeaf) return fail(HF_E_GRAPH, kShape);
    a.first[f] = nl;
    a.n_leaf[f] = (int)leaves.size();
    double cum = 0.0;
    for (size_t q = 0; q < leaves.size(); ++q) {
      const NodeInfo& ln = g->nodes[leaves[q]];
      if (!(ln.op == OP_EXP || ln.op == OP_GAUSS)) return fail(HF_E_GRAPH, kShape);
      if (ln.obs[0] != g->nodes[leaves[0]].obs[0]) return fail(HF_E_GRAPH, kShape);
      GenLeaf& L = a.leaf[nl++];
      const ObsInfo& o = g->obs[ln.obs[0]];
      L.op = ln.op;
      L.pad = 0;
      L.lo = o.lo;
      L.hi = o.hi;
      if (fn.op == OP_ADD && q + 1 < leaves.size()) {
        const double fq = th[fn.par[q]];
        if (!(fq >= 0.0)) return fail(HF_E_DOMAIN, "dataset_generate: fractions must be >= 0");
        cum += fq;
      }
      L.cum = fn.op == OP_ADD && q + 1 < leaves.size() ? cum : 2.0;
      if (ln.op == OP_EXP) {
        const double al = th[ln.par[0]];
        L.p0 = al;
        L.p1 = std::expm1(al * (o.hi - o.lo));
        L.p2 = L.p3 = 0.0;
      } else {
        const double mu = th[ln.par[0]], sg = th[ln.par[1]];
        if (!(sg > 0.0)) return fail(HF_E_DOMAIN, "dataset_generate: sigma must be > 0");
        L.p0 = mu;
        L.p1 = std::sqrt(2.0) * sg;
        L.p2 = std::erf((o.lo - mu) / L.p1);
        L.p3 = std::erf((o.hi - mu) / L.p1);
        if (!(L.p3 > L.p2)) return fail(HF_E_DOMAIN, "dataset_generate: Gaussian without weight in its box");
      }
    }
    if (fn.op == OP_ADD && cum > 1.0) return fail(HF_E_DOMAIN, "dataset_generate: fractions sum above 1");
    a.col[f] = g->col_of_obs[g->nodes[leaves[0]].obs[0]];
    for (int h = 0; h < f; ++h)
      if (a.col[h] == a.col[f])
        return fail(HF_E_GRAPH, "dataset_generate: product factors on a shared observable are not sampleable");
  }
  return HF_OK;
}

}  // namespace

extern "C" int dataset_generate(const pdf_graph* g, const double* params, int64_t n, uint64_t seed,
                                hf_precision prec, void* hip_stream, dataset** out) {
  try {
    if (!g || !params || !out) return fail(HF_E_INVALID, "dataset_generate: NULL argument");
    if (n < 0 || n > (int64_t(1) << 36)) return fail(HF_E_INVALID, "dataset_generate: n_events out of range");
    if (prec != HF_FP64 && prec != HF_FP32_EVAL) return fail(HF_E_INVALID, "dataset_generate: bad precision");
    for (size_t p = 0; p < g->par.size(); ++p)
      if (!std::isfinite(params[p])) return fail(HF_E_INVALID, "dataset_generate: parameter not finite");
    GenArgs a;
    std::memset(&a, 0, sizeof(a));
    if (int rc = gen_table(g, params, a)) return rc;
    std::unique_ptr<dataset> d;
    if (int rc = make_dataset(g, n, prec, 0, 0.0, "dataset_generate", d)) return rc;
    a.n = n;
    a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(seed >> 32);
    a.fp32 = prec == HF_FP32_EVAL ? 1 : 0;
    for (int f = 0; f < a.n_factor; ++f) {
      a.out[f] = const_cast<void*>(d->col[a.col[f]]);
      a.ref[f] = d->ref[a.col[f]];
    }
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = launch_generate(a, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      hipFree(d->block);
      return hip_fail(e, "dataset_generate");
    }
    *out = d.release();
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("dataset_generate: ") + ex.what());
  }
}

extern "C" int dataset_generate_ar(pdf_graph* g, const double* params, int64_t n, uint64_t seed, double envelope,
                                   int32_t max_trials, hf_precision prec, void* hip_stream, dataset** out) {
  try {
    if (!g || !params || !out) return fail(HF_E_INVALID, "dataset_generate_ar: NULL argument");
    if (n < 0 || n > (int64_t(1) << 36)) return fail(HF_E_INVALID, "dataset_generate_ar: n_events out of range");
    if (prec != HF_FP64 && prec != HF_FP32_EVAL) return fail(HF_E_INVALID, "dataset_generate_ar: bad precision");
    if (!(envelope > 0.0) || !std::isfinite(envelope))
      return fail(HF_E_INVALID, "dataset_generate_ar: envelope must be positive and finite");
    if (max_trials < 1) return fail(HF_E_INVALID, "dataset_generate_ar: max_trials must be >= 1");
    for (size_t p = 0; p < g->par.size(); ++p)
      if (!std::isfinite(params[p])) return fail(HF_E_INVALID, "dataset_generate_ar: parameter not finite");
    const int nc = (int)g->obs_of_col.size();
    for (int c = 0; c < nc; ++c) {
      const ObsInfo& o = g->obs[g->obs_of_col[c]];
      if (!std::isfinite(o.lo) || !std::isfinite(o.hi))
        return fail(HF_E_GRAPH, "dataset_generate_ar: every observable needs a finite box");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (int rc = ensure_grid(g, st)) return rc;
    StagedCall sc;
    stage(g, params, HF_FP64, sc, true);
    if (!sc.ok) return fail(HF_E_DOMAIN, "dataset_generate_ar: parameters outside the density's domain");
    std::unique_ptr<GenArArgs> a(new GenArArgs);
    std::memset(a.get(), 0, sizeof(GenArArgs));
    a->prog = sc.prog;
    a->n = n;
    a->key0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a->key1 = (uint32_t)(seed >> 32);
    a->max_trials = max_trials;
    a->n_cols = nc;
    a->fp32 = prec == HF_FP32_EVAL ? 1 : 0;
    a->env = envelope;
    a->ln_hoist = sc.ht.lnN;
    if (g->dz.node >= 0) {
      const NodeInfo& dn = g->nodes[g->dz.node];
      a->dalitz = 1;
      a->c12 = g->col_of_obs[dn.obs[0]];
      a->c13 = g->col_of_obs[dn.obs[1]];
      a->M = g->dz.M;
      a->m1 = g->dz.m1;
      a->m2 = g->dz.m2;
      a->m3 = g->dz.m3;
    }
    std::unique_ptr<dataset> d;
    if (int rc = make_dataset(g, n, prec, 0, 0.0, "dataset_generate_ar", d)) return rc;
    for (int c = 0; c < nc; ++c) {
      const ObsInfo& o = g->obs[g->obs_of_col[c]];
      a->lo[c] = o.lo;
      a->hi[c] = o.hi;
      a->ref[c] = d->ref[c];
      a->out[c] = const_cast<void*>(d->col[c]);
    }
    int32_t* flag = nullptr;
    hipError_t e = hipMalloc(&flag, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, sizeof(int32_t), st);
    a->fail = flag;
    if (e == hipSuccess) e = launch_generate_ar(*a, st);
    int32_t fl = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&fl, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (flag) hipFree(flag);
    if (e != hipSuccess) {
      hipFree(d->block);
      return hip_fail(e, "dataset_generate_ar");
    }
    if (fl) {
      hipFree(d->block);
      return fail(HF_E_DOMAIN, (fl & 2) ? "dataset_generate_ar: the density exceeds the envelope"
                                        : "dataset_generate_ar: an event ran out of trials");
    }
    *out = d.release();
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("dataset_generate_ar: ") + ex.what());
  }
}

extern "C" int dataset_read_column(const dataset* d, int32_t obs, void* hip_stream, double* host_out) {
  try {
    if (!d || !host_out) return fail(HF_E_INVALID, "dataset_read_column: NULL argument");
    const pdf_graph* g = d->g;
    if (obs < 0 || obs >= (int)g->obs.size() || g->col_of_obs[obs] < 0)
      return fail(HF_E_INVALID, "dataset_read_column: observable not stored");
    if (d->metric) return fail(HF_E_INVALID, "dataset_read_column: binned datasets hold bin centres only");
    const int c = g->col_of_obs[obs];
    const size_t es = d->prec == HF_FP32_EVAL ? 4 : 8;
    if (d->n == 0) return HF_OK;
    std::vector<char> buf((size_t)d->n * es);
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(buf.data(), d->col[c], buf.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "dataset_read_column");
    if (es == 8) {
      std::memcpy(host_out, buf.data(), buf.size());
    } else {
      const float* f = (const float*)buf.data();
      for (int64_t i = 0; i < d->n; ++i) host_out[i] = (double)f[i] + d->ref[c];
    }
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("dataset_read_column: ") + ex.what());
  }
}

extern "C" int hf_column_ref(const pdf_graph* g, int32_t obs, hf_precision prec, double* ref) {
  if (!g || !ref || obs < 0 || obs >= (int32_t)g->obs.size()) return fail(HF_E_INVALID, "hf_column_ref: bad argument");
  if (prec != HF_FP64 && prec != HF_FP32_EVAL) return fail(HF_E_INVALID, "hf_column_ref: bad precision");
  const int c = g->col_of_obs[obs];
  *ref = c < 0 ? 0.0 : column_ref(g, c, prec);
  return HF_OK;
}

extern "C" int dataset_wrap_device(const pdf_graph* g, void* const* dev_cols, int64_t n, hf_precision prec,
                                   dataset** out) {
  try {
    if (!g || !out || (n > 0 && !dev_cols)) return fail(HF_E_INVALID, "dataset_wrap_device: NULL argument");
    if (n < 0 || n > (int64_t(1) << 36)) return fail(HF_E_INVALID, "dataset_wrap_device: n_events out of range");
    if (prec != HF_FP64 && prec != HF_FP32_EVAL) return fail(HF_E_INVALID, "dataset_wrap_device: bad precision");
    const int nc = (int)g->obs_of_col.size();
    const size_t es = prec == HF_FP32_EVAL ? 4 : 8;
    std::unique_ptr<dataset> d(new dataset);
    d->g = g;
    d->prec = prec;
    d->n = n;
    d->n_cols = nc;
    for (int c = 0; c < nc; ++c) {
      void* p = n > 0 ? dev_cols[g->obs_of_col[c]] : nullptr;
      if (n > 0 && !p) return fail(HF_E_INVALID, "dataset_wrap_device: NULL column for a used observable");
      if ((uintptr_t)p % es != 0) return fail(HF_E_INVALID, "dataset_wrap_device: misaligned column");
      d->col[c] = p;
      d->ref[c] = column_ref(g, c, prec);
    }
    d->n_rows = rows_for(g->kind, prec, n);
    const size_t part_bytes = align256((size_t)std::max<int32_t>(d->n_rows, 1) * (g->prog.n_slots + 1) * sizeof(double));
    void* blk = nullptr;
    hipError_t e = hipMalloc(&blk, part_bytes);
    if (e != hipSuccess) return fail(HF_E_OOM, std::string("dataset_wrap_device: hipMalloc: ") + hipGetErrorString(e));
    d->block = blk;
    d->partials = (double*)blk;
    d->bytes = (int64_t)part_bytes;
    *out = d.release();
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("dataset_wrap_device: ") + ex.what());
  }
}

extern "C" void dataset_free(dataset* d) {
  if (!d) return;
  if (d->block) hipFree(d->block);
  if (d->res_host) hipHostFree(d->res_host);
  if (d->norm_partials) hipFree(d->norm_partials);
  delete d;
}

extern "C" int64_t dataset_device_bytes(const dataset* d) { return d ? d->bytes : 0; }

extern "C" int dataset_bytes_needed(const pdf_graph* g, int64_t n_events, hf_precision prec, int64_t* bytes) {
  if (!g || !bytes) return fail(HF_E_INVALID, "dataset_bytes_needed: NULL argument");
  if (n_events < 0 || n_events > (int64_t(1) << 36)) return fail(HF_E_INVALID, "dataset_bytes_needed: n_events out of range");
  if (prec != HF_FP64 && prec != HF_FP32_EVAL) return fail(HF_E_INVALID, "dataset_bytes_needed: bad precision");
  *bytes = (int64_t)dataset_layout(g, n_events, prec, 0).total;
  return HF_OK;
}

static int check_call(const pdf_graph* g, const dataset* d, const double* params) {
  if (!g || !d || !params) return fail(HF_E_INVALID, "NULL graph, dataset or params");
  if (d->g != g) return fail(HF_E_SHAPE, "dataset was uploaded for another graph");
  for (size_t p = 0; p < g->par.size(); ++p)
    if (std::isnan(params[p])) return fail(HF_E_INVALID, "parameter is NaN");
  return HF_OK;
}

extern "C" int nll_eval(const pdf_graph* g, const dataset* d, const double* params, void* hip_stream, double* nll) {
  try {
    if (int rc = check_call(g, d, params)) return rc;
    if (!nll) return fail(HF_E_INVALID, "nll_eval: NULL output");
    return eval_one(g, d, params, (hipStream_t)hip_stream, false, nll, nullptr);
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("nll_eval: ") + ex.what());
  }
}

extern "C" int nll_grad(const pdf_graph* g, const dataset* d, const double* params, void* hip_stream, double* nll,
                        double* grad) {
  try {
    if (int rc = check_call(g, d, params)) return rc;
    if (!nll || !grad) return fail(HF_E_INVALID, "nll_grad: NULL output");
    return eval_one(g, d, params, (hipStream_t)hip_stream, true, nll, grad);
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("nll_grad: ") + ex.what());
  }
}

// Per-event terms: the evaluation kernels instantiated with per-event output
// (launch_terms), over slices of the dataset so that the device buffer stays
// bounded; each event's terms are assembled like a one-event dataset.
extern "C" int nll_terms(const pdf_graph* g, const dataset* d, const double* params, void* hip_stream, double* lnp,
                         double* dlnp) {
  try {
    if (int rc = check_call(g, d, params)) return rc;
    if (!lnp) return fail(HF_E_INVALID, "nll_terms: NULL lnp");
    if (d->metric != 0) return fail(HF_E_INVALID, "nll_terms: binned dataset (only unbinned datasets have terms)");
    hipStream_t st = (hipStream_t)hip_stream;
    const int np = (int)g->par.size();
    if (int rc = ensure_grid(const_cast<pdf_graph*>(g), st)) return rc;
    StagedCall sc;
    stage(g, params, d->prec, sc, false);
    if (!sc.ok) {  // the density is undefined at every event
      for (int64_t i = 0; i < d->n; ++i) {
        lnp[i] = -INFINITY;
        if (dlnp)
          for (int p = 0; p < np; ++p) dlnp[i * np + p] = NAN;
      }
      return fail(HF_E_DOMAIN, "nll_terms: parameters outside the density's domain");
    }
    if (d->n == 0) return HF_OK;
    if (sc.grid_norm) {
      if (int rc = ensure_result_buffer(d)) return rc;
      if (int rc = launch_grid_norm(g, d, sc, dlnp != nullptr, st)) return rc;
      const_cast<dataset*>(d)->seq += 1;
      hipError_t e = wait_result(d, st, kNormFlag);
      if (e != hipSuccess) return hip_fail(e, "nll_terms: normalisation grid");
      if (int rc = grid_norm_terms(g, d, params, dlnp != nullptr, sc)) return rc;
    }
    const int S = g->prog.n_slots, nc = 1 + S;
    const int64_t kSlice = int64_t(1) << 18;  // events per terms launch
    const int64_t slice_cap = std::min<int64_t>(kSlice, d->n);
    const int64_t cap_rows = (slice_cap + kBlock - 1) / kBlock;
    const size_t col_stride = (size_t)cap_rows * kBlock;
    double* buf = nullptr;
    hipError_t e = hipMalloc((void**)&buf, col_stride * nc * sizeof(double));
    if (e != hipSuccess) return fail(HF_E_OOM, std::string("nll_terms: hipMalloc: ") + hipGetErrorString(e));
    std::vector<double> host(col_stride * nc), sums(nc), gr(np);
    const size_t es = d->prec == HF_FP32_EVAL ? 4 : 8;
    bool bad = false;
    int rc = HF_OK;
    for (int64_t e0 = 0; e0 < d->n && rc == HF_OK; e0 += kSlice) {
      const int64_t m = std::min<int64_t>(kSlice, d->n - e0);
      EvalArgs a;
      std::memset(&a, 0, sizeof(a));
      a.prog = sc.prog;
      for (int c = 0; c < kMaxCols; ++c)
        a.col[c] = d->col[c] ? (const void*)((const char*)d->col[c] + (size_t)e0 * es) : nullptr;
      a.n_events = m;
      a.n_rows = (int32_t)((m + kBlock - 1) / kBlock);
      a.partials = buf;
      const size_t stride = (size_t)a.n_rows * kBlock;
      e = launch_terms(g->kind, d->prec == HF_FP32_EVAL, a, st);
      if (e == hipSuccess) e = hipMemcpyAsync(host.data(), buf, stride * (dlnp ? nc : 1) * sizeof(double),
                                              hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        rc = hip_fail(e, "nll_terms: terms launch");
        break;
      }
      for (int64_t i = 0; i < m; ++i) {
        for (int j = 0; j < (dlnp ? nc : 1); ++j) sums[j] = host[(size_t)j * stride + i];
        double v = 0.0;
        assemble(g, sc, sums.data(), 1, &v, dlnp ? gr.data() : nullptr);
        lnp[e0 + i] = -v;
        if (dlnp)
          for (int p = 0; p < np; ++p) dlnp[(e0 + i) * np + p] = gr[p] == 0.0 ? 0.0 : -gr[p];
        bad = bad || !std::isfinite(v);
      }
    }
    hipFree(buf);
    if (rc != HF_OK) return rc;
    if (bad) return fail(HF_E_DOMAIN, "nll_terms: density <= 0 or not finite at some event");
    return HF_OK;
  } catch (const std::exception& ex) {
    return fail(HF_E_INVALID, std::string("nll_terms: ") + ex.what());
  }
}

extern "C" int hf_profile(int32_t enable, double* eval_ms, double* reduce_ms, int64_t* n_launch) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_prof.init) {
    hipError_t e = prof_harvest();
    if (e != hipSuccess) return hip_fail(e, "hf_profile: profile events");
  }
  if (eval_ms) *eval_ms = g_prof.eval_ms;
  if (reduce_ms) *reduce_ms = g_prof.reduce_ms;
  if (n_launch) *n_launch = g_prof.n;
  if (enable >= 1) {
    if (!g_prof.init) {
      for (int i = 0; i < 4; ++i) {
        hipError_t e = hipEventCreate(&g_prof.e[i]);
        if (e != hipSuccess) return hip_fail(e, "hf_profile: hipEventCreate");
      }
      g_prof.init = true;
    }
    g_prof.eval_ms = g_prof.reduce_ms = 0.0;
    g_prof.n = 0;
    g_prof.calls = 0;
    g_prof.every = enable;
    g_prof.on = true;
  } else if (enable == 0) {
    g_prof.on = false;
  }
  return HF_OK;
}
