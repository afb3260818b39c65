// Host-runtime checks under the address and undefined-behaviour sanitizers
// (no GPU): graph creation and validation for every node kind, staging of
// the constant tables and the host assembly of results in both precisions,
// the minimiser on smooth, bounded, fixed-parameter and failing objectives,
// and the ABI's error paths (uploads and launches that cannot reach a GPU
// must return an error code, never crash).  Exit status 0 and no sanitizer
// report mean success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/hipfit.h"
#include "../../paper_1311_1753_amd/csrc/runtime.h"

static int g_fail = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);      \
      ++g_fail;                                                               \
    }                                                                         \
  } while (0)

// A graph description kept alive while pdf_graph_create copies it.
struct Spec {
  std::vector<hf_obs> obs;
  std::vector<hf_param> par;
  std::vector<std::vector<int32_t>> child, pars, obsi;
  std::vector<std::vector<double>> consts;
  std::vector<int32_t> op;
  int add(int o, std::vector<int32_t> ch, std::vector<int32_t> p, std::vector<int32_t> ob, std::vector<double> c = {}) {
    op.push_back(o);
    child.push_back(ch);
    pars.push_back(p);
    obsi.push_back(ob);
    consts.push_back(c);
    return (int)op.size() - 1;
  }
  int create(pdf_graph** g, int root = -1) {
    std::vector<hf_node> nodes(op.size());
    for (size_t i = 0; i < op.size(); ++i) {
      nodes[i].op = op[i];
      nodes[i].n_child = (int32_t)child[i].size();
      nodes[i].child = child[i].data();
      nodes[i].n_par = (int32_t)pars[i].size();
      nodes[i].par = pars[i].data();
      nodes[i].n_obs = (int32_t)obsi[i].size();
      nodes[i].obs = obsi[i].data();
      nodes[i].n_const = (int32_t)consts[i].size();
      nodes[i].consts = consts[i].data();
    }
    return pdf_graph_create(obs.data(), (int32_t)obs.size(), par.data(), (int32_t)par.size(), nodes.data(),
                            (int32_t)nodes.size(), root < 0 ? (int32_t)nodes.size() - 1 : root, g);
  }
};

static hf_param P(const char* n, double init, double step, double lo = 0.0, double hi = 0.0) {
  return hf_param{n, init, step, lo, hi, 0};
}

static std::vector<double> dalitz_consts(bool tddp_unused) {
  (void)tddp_unused;
  // M, m1, m2, m3, r, grid, R, then (channel, m0, Gamma0, J)
  return {1.865, 0.4976, 0.1396, 0.1396, 1.5, 100, 3, 23, 0.775, 0.149, 1, 12, 0.892, 0.05, 1, 13, 0.892, 0.05, 1};
}

// Staging and assembly of one graph at its start values and at a shifted
// point, in both precisions; Dalitz grids get a synthetic Hermitian matrix.
static void stage_both(pdf_graph* g) {
  using namespace hf;
  if (g->dz.node >= 0) {
    const int na = (int)g->dz.res.size() + 1;
    auto herm = [&](std::vector<double>& M) {
      M.assign((size_t)na * na * 2, 0.0);
      for (int p = 0; p < na; ++p)
        for (int q = 0; q < na; ++q) {
          M[2 * (p * na + q)] = p == q ? 2.0 + p : 0.1 / (1 + p + q);
          M[2 * (p * na + q) + 1] = p == q ? 0.0 : (p < q ? 0.01 : -0.01);
        }
    };
    herm(g->dz.I);
    herm(g->dz.Ib);
    herm(g->dz.J);
    g->dz.ready = true;
  }
  const int np = (int)g->par.size();
  std::vector<double> th(np), gr(np), sums(kMaxSlots + 2, 0.1);
  for (int p = 0; p < np; ++p) th[p] = g->par[p].init;
  for (int shift = 0; shift < 2; ++shift) {
    for (int p = 0; p < np; ++p) th[p] = g->par[p].init * (shift ? 1.01 : 1.0) + (shift ? 1e-3 : 0.0);
    for (hf_precision pr : {HF_FP64, HF_FP32_EVAL}) {
      StagedCall sc;
      stage(g, th.data(), pr, sc, false);
      StagedCall sb;
      stage(g, th.data(), pr, sb, true);
      double v = 0.0;
      assemble(g, sc, sums.data(), 1000, &v, gr.data());
      assemble(g, sc, nullptr, 0, &v, gr.data());
      assemble_binned(g, sb, sums.data(), &v, gr.data());
      int64_t bytes = 0;
      CHECK(dataset_bytes_needed(g, 12345, pr, &bytes) == HF_OK && bytes > 0);
      for (int o = 0; o < (int)g->obs.size(); ++o) {
        double ref = -1.0;
        CHECK(hf_column_ref(g, o, pr, &ref) == HF_OK);
      }
    }
  }
}

static void graphs() {
  // exponential
  {
    Spec s;
    s.obs = {{"x", 0.0, 10.0}};
    s.par = {P("alpha", -2.0, 0.1, -10, 10)};
    s.add(HF_OP_EXP, {}, {0}, {0});
    pdf_graph* g = nullptr;
    CHECK(s.create(&g) == HF_OK);
    int32_t no = 0, np = 0;
    CHECK(pdf_graph_shape(g, &no, &np) == HF_OK && no == 1 && np == 1);
    stage_both(g);
    // uploads cannot reach a device here: an error code, not a crash
    std::vector<double> x = {1.0, 2.0, 3.0};
    const double* cols[1] = {x.data()};
    dataset* d = nullptr;
    const int rc = dataset_upload(g, cols, 3, HF_FP64, nullptr, &d);
    CHECK(rc != HF_OK && d == nullptr);
    std::vector<double> bad = {1.0, 11.0};
    const double* bc[1] = {bad.data()};
    CHECK(dataset_upload(g, bc, 2, HF_FP64, nullptr, &d) == HF_E_DOMAIN);
    CHECK(dataset_upload(g, nullptr, 2, HF_FP64, nullptr, &d) == HF_E_INVALID);
    CHECK(dataset_upload(g, cols, -1, HF_FP64, nullptr, &d) == HF_E_INVALID);
    double v = 0.0, gg[1];
    CHECK(nll_grad(g, nullptr, &s.par[0].init, nullptr, &v, gg) == HF_E_INVALID);
    CHECK(std::strlen(hf_last_error()) > 0);
    pdf_graph_destroy(g);
  }
  // Gaussian + exponential, a polynomial, a map, shared-observable product
  {
    Spec s;
    s.obs = {{"x", 0.0, 10.0}};
    s.par = {P("mu", 5.0, 0.1), P("sigma", 1.0, 0.1, 0.01, 5), P("beta", -0.2, 0.1), P("f", 0.4, 0.05, 0, 1),
             P("a1", 0.1, 0.01), P("a2", -0.01, 0.01)};
    const int ga = s.add(HF_OP_GAUSS, {}, {0, 1}, {0});
    const int ex = s.add(HF_OP_EXP, {}, {2}, {0});
    s.add(HF_OP_ADD, {ga, ex}, {3}, {});
    pdf_graph* g = nullptr;
    CHECK(s.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);

    Spec m;
    m.obs = s.obs;
    m.par = s.par;
    const int e1 = m.add(HF_OP_EXP, {}, {2}, {0});
    const int g1 = m.add(HF_OP_GAUSS, {}, {0, 1}, {0});
    const int p1 = m.add(HF_OP_POLY, {}, {4, 5}, {0}, {8.5});
    m.add(HF_OP_MAP, {e1, g1, p1}, {}, {0}, {4.0, 7.0});
    CHECK(m.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);

    Spec sh;
    sh.obs = s.obs;
    sh.par = s.par;
    const int pa = sh.add(HF_OP_POLY, {}, {4, 5}, {0}, {5.0});
    const int gb = sh.add(HF_OP_GAUSS, {}, {0, 1}, {0});
    sh.add(HF_OP_PROD, {pa, gb}, {}, {});
    CHECK(sh.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);
  }
  // convolution and composition
  {
    Spec s;
    s.obs = {{"x", 0.0, 10.0}};
    s.par = {P("alpha", -0.4, 0.05), P("rmu", 0.05, 0.01), P("rsg", 0.3, 0.01, 0.01, 2), P("a1", 0.5, 0.01),
             P("a2", 0.05, 0.01)};
    const int m = s.add(HF_OP_EXP, {}, {0}, {0});
    const int r = s.add(HF_OP_GAUSS, {}, {1, 2}, {0});
    s.add(HF_OP_CONV, {m, r}, {}, {0}, {400, -2.0, 2.0});
    pdf_graph* g = nullptr;
    CHECK(s.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);

    Spec c;
    c.obs = s.obs;
    c.par = s.par;
    const int core = c.add(HF_OP_POLY, {}, {3, 4}, {0}, {5.0});
    const int shell = c.add(HF_OP_GAUSS, {}, {1, 2}, {0});
    c.add(HF_OP_COMP, {core, shell}, {}, {0});
    CHECK(c.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);
  }
  // Dalitz, time-dependent Dalitz with x, and the sigma_t map beside it
  {
    Spec s;
    s.obs = {{"s12", 0.406, 2.977}, {"s13", 0.406, 2.977}, {"t", -INFINITY, INFINITY}, {"st", 0.02, 0.2}};
    for (int k = 0; k < 3; ++k) {
      s.par.push_back(P("re", 0.3, 0.05));
      s.par.push_back(P("im", 0.1, 0.05));
    }
    s.add(HF_OP_DALITZ, {}, {0, 1, 2, 3, 4, 5}, {0, 1}, dalitz_consts(false));
    pdf_graph* g = nullptr;
    CHECK(s.create(&g) == HF_OK);
    stage_both(g);
    std::vector<double> a = {0.5, 1.0, 2.9, 0.1}, b = {0.5, 1.2, 2.9, 0.1};
    std::vector<uint8_t> in(4);
    CHECK(hf_dalitz_inside(g, 0, 4, a.data(), b.data(), in.data()) == HF_OK);
    pdf_graph_destroy(g);

    Spec t = s;
    t.op.clear();
    t.child.clear();
    t.pars.clear();
    t.obsi.clear();
    t.consts.clear();
    t.par.push_back(P("tau", 0.41, 0.01, 0.1, 2.0));
    t.par.push_back(P("y", 0.01, 0.005, -0.2, 0.2));
    t.par.push_back(P("x", 0.008, 0.005, -0.2, 0.2));
    t.add(HF_OP_TDDP, {}, {0, 1, 2, 3, 4, 5, 6, 7, 8}, {0, 1, 2, 3}, dalitz_consts(true));
    CHECK(t.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);

    // the full form: x and q/p (flags 3), the second resonance's mass and
    // width as parameters (given after |q/p|, arg q/p), with and without
    // floating shapes; a bad flag and a wrong parameter count are errors
    Spec f = t;
    f.consts.clear();
    f.op.clear();
    f.child.clear();
    f.pars.clear();
    f.obsi.clear();
    f.par.push_back(P("qm", 0.9, 0.01, 0.5, 1.5));
    f.par.push_back(P("qa", 0.2, 0.01, -1.0, 1.0));
    f.par.push_back(P("m0", 0.89, 0.002, 0.8, 0.95));
    f.par.push_back(P("g0", 0.05, 0.002, 0.03, 0.08));
    std::vector<double> fc = dalitz_consts(true);
    fc.push_back(3);
    fc.insert(fc.end(), {0, 1, 0});
    f.add(HF_OP_TDDP, {}, {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12}, {0, 1, 2, 3}, fc);
    CHECK(f.create(&g) == HF_OK);
    CHECK(g->dz.full && g->dz.hq && g->dz.hx && g->dz.fl.size() == 1);
    stage_both(g);
    {
      // floating shapes: staging leaves the normalisation to the grid kernel
      using namespace hf;
      std::vector<double> th(g->par.size());
      for (size_t p = 0; p < th.size(); ++p) th[p] = g->par[p].init;
      StagedCall sc;
      stage(g, th.data(), HF_FP32_EVAL, sc, false);
      CHECK(sc.ok && sc.grid_norm);
      th[11] = 0.2;  // mass below the K pi threshold
      stage(g, th.data(), HF_FP64, sc, false);
      CHECK(!sc.ok);
    }
    pdf_graph_destroy(g);
    f.op.clear();
    f.child.clear();
    f.pars.clear();
    f.obsi.clear();
    f.consts.clear();
    fc[fc.size() - 2] = 0;  // no floating shape: the q/p matrices path
    f.add(HF_OP_TDDP, {}, {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10}, {0, 1, 2, 3}, fc);
    CHECK(f.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);
    f.op.clear();
    f.child.clear();
    f.pars.clear();
    f.obsi.clear();
    f.consts.clear();
    fc[fc.size() - 4] = 7;  // flags 0..3 only
    f.add(HF_OP_TDDP, {}, {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10}, {0, 1, 2, 3}, fc);
    CHECK(f.create(&g) == HF_E_GRAPH);

    Spec u = s;
    u.op.clear();
    u.child.clear();
    u.pars.clear();
    u.obsi.clear();
    u.consts.clear();
    u.par.push_back(P("tau", 0.41, 0.01, 0.1, 2.0));
    u.par.push_back(P("y", 0.01, 0.005, -0.2, 0.2));
    for (int c = 0; c < 4; ++c) {
      u.par.push_back(P("smu", 0.1, 0.01));
      u.par.push_back(P("ssg", 0.04, 0.01, 0.001, 1.0));
    }
    const int td = u.add(HF_OP_TDDP, {}, {0, 1, 2, 3, 4, 5, 6, 7}, {0, 1, 2, 3}, dalitz_consts(true));
    std::vector<int32_t> cells;
    for (int c = 0; c < 4; ++c) cells.push_back(u.add(HF_OP_GAUSS, {}, {8 + 2 * c, 9 + 2 * c}, {3}));
    const int dm = u.add(HF_OP_DPMAP, cells, {}, {0, 1, 3}, {2, 2, 1.5, 1.5});
    u.add(HF_OP_PROD, {td, dm}, {}, {});
    CHECK(u.create(&g) == HF_OK);
    stage_both(g);
    pdf_graph_destroy(g);
  }
  // invalid trees
  {
    Spec s;
    s.obs = {{"x", 0.0, 1.0}};
    s.par = {P("a", -1.0, 0.1)};
    s.add(HF_OP_EXP, {1}, {0}, {0});  // child index not earlier than the node
    s.add(HF_OP_EXP, {}, {0}, {0});
    pdf_graph* g = nullptr;
    CHECK(s.create(&g, 1) == HF_E_GRAPH && g == nullptr);
    Spec w;
    w.obs = {{"x", 1.0, 0.0}};  // lo >= hi
    w.par = {P("a", -1.0, 0.1)};
    w.add(HF_OP_EXP, {}, {0}, {0});
    CHECK(w.create(&g) != HF_OK);
    Spec q;
    q.obs = {{"x", 0.0, 1.0}};
    q.par = {P("a", -1.0, 0.1)};
    q.add(HF_OP_GAUSS, {}, {0}, {0});  // one parameter for a Gaussian
    CHECK(q.create(&g) == HF_E_GRAPH);
    Spec big;
    big.obs = {{"x", 0.0, 1.0}};
    big.par = {P("a", -1.0, 0.1), P("f", 0.5, 0.1, 0, 1)};
    int prev = big.add(HF_OP_EXP, {}, {0}, {0});
    for (int k = 0; k < 16; ++k) {
      const int e = big.add(HF_OP_EXP, {}, {0}, {0});
      prev = big.add(HF_OP_ADD, {prev, e}, {1}, {});
    }
    CHECK(big.create(&g) != HF_OK);  // more than 16 nodes
    CHECK(pdf_graph_create(nullptr, 0, nullptr, 0, nullptr, 0, 0, &g) != HF_OK);
  }
}

// ------------------------------------------------------------------ minimiser
static int quad(const double* x, double* f, double* g, void*) {
  *f = 0.0;
  for (int i = 0; i < 5; ++i) {
    const double d = x[i] - 0.5 * i;
    *f += (i + 1) * d * d;
    g[i] = 2.0 * (i + 1) * d;
  }
  return 0;
}
static int rosen(const double* x, double* f, double* g, void*) {
  const double a = 1.0 - x[0], b = x[1] - x[0] * x[0];
  *f = a * a + 100.0 * b * b;
  g[0] = -2.0 * a - 400.0 * x[0] * b;
  g[1] = 200.0 * b;
  return 0;
}
static int nan_left(const double* x, double* f, double* g, void*) {
  if (x[0] < 0.0) {
    *f = NAN;
    g[0] = 0.0;
    return 0;
  }
  *f = (x[0] - 2.0) * (x[0] - 2.0);
  g[0] = 2.0 * (x[0] - 2.0);
  return 0;
}
static int fails(const double*, double*, double*, void*) { return 1; }

static void minimiser() {
  hf_fit_opts o{0, 0.0, 0, 1, 0.0};
  hf_fit_summary sm;
  std::vector<hf_param> p5;
  for (int i = 0; i < 5; ++i) p5.push_back(P("p", 3.0, 0.1));
  p5[2].fixed = 1;
  std::vector<double> x(5), e(5), cov(25);
  CHECK(hf_minimize(5, p5.data(), nullptr, &o, 0.0, quad, nullptr, x.data(), e.data(), cov.data(), &sm) == HF_OK);
  CHECK(std::fabs(x[0]) < 1e-6 && std::fabs(x[4] - 2.0) < 1e-6 && x[2] == 3.0 && e[2] == 0.0);
  std::vector<hf_param> p2 = {P("x", -1.2, 0.1, -2.0, 2.0), P("y", 1.0, 0.1)};
  std::vector<double> y(2), ye(2);
  o.max_iter = 2000;
  const int rc = hf_minimize(2, p2.data(), nullptr, &o, 0.0, rosen, nullptr, y.data(), ye.data(), nullptr, &sm);
  CHECK(rc == HF_OK || rc == HF_E_NOT_CONVERGED);
  std::vector<hf_param> p1 = {P("x", 5.0, 1.0)};
  double z = 0.0, ze = 0.0;
  CHECK(hf_minimize(1, p1.data(), nullptr, &o, 0.0, nan_left, nullptr, &z, &ze, nullptr, &sm) == HF_OK);
  CHECK(std::fabs(z - 2.0) < 1e-5);
  CHECK(hf_minimize(1, p1.data(), nullptr, &o, 0.0, fails, nullptr, &z, &ze, nullptr, &sm) == HF_E_INVALID);
  CHECK(hf_minimize(-1, p1.data(), nullptr, &o, 0.0, quad, nullptr, &z, &ze, nullptr, &sm) == HF_E_INVALID);
  CHECK(hf_minimize(1, p1.data(), nullptr, &o, 0.0, nullptr, nullptr, &z, &ze, nullptr, &sm) == HF_E_INVALID);
}

int main() {
  graphs();
  minimiser();
  std::printf("host sanitizer checks: %s (%d failed)\n", g_fail ? "FAILED" : "ok", g_fail);
  return g_fail ? 1 : 0;
}
