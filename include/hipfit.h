/*
 * hipfit.h -- C ABI of the MI355X (gfx950) unbinned maximum-likelihood library.
 *
 * The library evaluates, on one GPU, the negative log-likelihood
 *     NLL(theta) = -sum_i ln P(x_i; theta)
 * of a tree of normalised probability densities P over a set of events, and
 * its exact gradient, and minimises it.  The split of the interface follows
 * the four components of a GooFit program (paper, section "GooFit code"):
 * variables (hf_obs / hf_param), the PDF (pdf_graph), the data (dataset) and
 * the fit manager (fit, batch_*).
 *
 * Conventions for every entry point:
 *   - return 0 (HF_OK) on success or a negative hf_status;
 *   - on error, out-parameters are left untouched (except where stated) and
 *     hf_last_error() returns a message for the calling thread;
 *   - no C++ exception and no abort crosses this interface;
 *   - all pointers are host pointers unless the name says "dev";
 *   - `hip_stream` is a hipStream_t (NULL = the default stream);
 *   - handles are owned by the caller and released with the matching
 *     destroy/free call;
 *   - calls that use one dataset (or one batch engine) must not overlap in
 *     time: each holds a per-object device workspace.
 */
#ifndef HIPFIT_H
#define HIPFIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum hf_status {
  HF_OK = 0,
  HF_E_INVALID = -1,        /* bad argument (NULL handle, size out of range) */
  HF_E_GRAPH = -2,          /* invalid PDF tree (see pdf_graph_create) */
  HF_E_SHAPE = -3,          /* dataset / parameter shape does not match the graph */
  HF_E_OOM = -4,            /* device or pinned host allocation failed */
  HF_E_HIP = -5,            /* a HIP runtime call failed (message has the HIP error) */
  HF_E_DOMAIN = -6,         /* event outside its box / Dalitz plot, or density <= 0 or not finite */
  HF_E_NOT_CONVERGED = -7,  /* minimiser hit its iteration limit */
  HF_E_BUDGET = -8,         /* batch admission: the fit does not fit the device-memory budget now */
  HF_E_FULL = -9            /* batch admission: no free slot */
};

/* Arithmetic of the per-event evaluation.  The reductions, normalisations
 * and minimiser are always double precision. */
typedef enum {
  HF_FP64 = 0,              /* events stored and evaluated in double */
  HF_FP32_EVAL = 1          /* events stored as float offsets from a per-column double
                               reference; location differences (x - mu, s - m0^2) formed in
                               double, the rest of the per-event arithmetic in float,
                               accumulation in double with compensated sums */
} hf_precision;

/* Binned metrics (the fit-manager metric switch of the paper's "GooFit code"
 * section; binned fits as in its results section).  Events are bin centres
 * with weights w_i (counts); P is the normalised density of the graph.
 *   HF_METRIC_BNLL: binned NLL = -sum_i w_i ln P(x_i)
 *   HF_METRIC_CHI2: chi^2 = sum_i (w_i - K P(x_i))^2 / max(w_i, 1), with
 *                   K = (sum of the weights) x bin volume the expected
 *                   count of a bin per unit density at its centre.
 * Fits of chi^2 use up = 1 (errors sqrt(diag(2 H^-1))), the likelihoods up
 * = 0.5 (sqrt(diag(H^-1))). */
typedef enum { HF_METRIC_BNLL = 1, HF_METRIC_CHI2 = 2 } hf_metric;

/* Node kinds of the PDF tree (paper, sections "GooFit code", "Combining
 * functions", "Results").  Every node is a density normalised over its
 * observables' box. */
enum hf_op {
  HF_OP_EXP = 1,     /* e^{alpha x}/int_box; par = {alpha}; obs = {x}                    */
  HF_OP_GAUSS = 2,   /* exp(-(x-mu)^2/(2 sigma^2))/int_box; par = {mu, sigma}; obs = {x}   */
  HF_OP_POLY = 3,    /* (1 + sum_k a_k (x-x0)^k)/int_box; par = {a_1..a_d}; obs = {x};
                        consts = {x0}; density <= 0 at an event is a domain error           */
  HF_OP_ADD = 4,     /* sum_{j<K} f_j P_j + (1 - sum f_j) P_K; K >= 2 children; par = the
                        K-1 fractions; children over the same box, each normalised          */
  HF_OP_PROD = 5,    /* prod_j P_j / prod_g Z_g; K >= 2 children; no par; children use
                        disjoint observables, except that one-observable EXP / GAUSS / POLY
                        leaves may share one: each such group g (two or more leaves on one
                        observable x) is renormalised by Z_g = int_box prod_{j in g} P_j dx
                        (section "Combining functions"), computed on the host by composite
                        16-point Gauss-Legendre quadrature on at most 4096 segments; any
                        other overlap is HF_E_GRAPH                                          */
  HF_OP_DALITZ = 6,  /* |1 + sum_k c_k A_k(s12, s13)|^2 / N_A over the Dalitz plot;
                        obs = {s12, s13}; par = {Re c_1, Im c_1, ..., Re c_R, Im c_R};
                        consts = DALITZ block (below)                                       */
  HF_OP_TDDP = 7     /* time-dependent Dalitz density with per-event Gaussian resolution:
                        [a_c C(t) + a_0 Cz(t) + a_s S(t) + b_s Sz(t)] / N_T, where
                        a_c = (|A|^2+|Abar|^2)/2, a_0 = (|A|^2-|Abar|^2)/2, a_s = -Re(A* Abar),
                        b_s = -Im(A* Abar), Abar(s12,s13) = A(s13,s12), C/S = (E(G-) +/- E(G+))/2,
                        G-/+ = (1 -/+ y)/tau, E(t; G, sigma_t) the Gaussian-convolved decay
                        e^{-G t}, and Cz + i Sz the Gaussian-convolved e^{-t/tau} e^{i x t/tau}
                        (section "Results": hyperbolic and trigonometric terms); t is
                        normalised over the real line; obs = {s12, s13, t, sigma_t};
                        par = {Re c_1, Im c_1, ..., tau, y} (x = 0: Cz = E(t; 1/tau), Sz = 0)
                        or {..., tau, y, x}; consts = DALITZ block.
                        Full form (the mixing fit of section "Results": up to 16 resonances,
                        complex q/p, floating resonance shapes): the DALITZ block followed by
                        flags (1: x is a parameter, 2: q/p is) and R floating-shape flags
                        (1: resonance k's mass and width are parameters); par = {2R
                        coefficients, tau, y, (x), (|q/p|, arg q/p), then (m0, Gamma0) of each
                        floating resonance in resonance order}; at most 4 floating.  q/p
                        multiplies the conjugate amplitude: Abar -> (q/p) Abar in every term
                        above and in N_T.  With floating shapes N_T is re-computed on the grid
                        at every evaluation (grid kernel, FP64) instead of from the cached
                        grid matrices.  A full-form node (or a TDDP node with more than 8
                        resonances) must be the graph's only node; binned datasets,
                        nll_grad_batched, the batch engine and nll_grad_noalloc with floating
                        shapes reject it (HF_E_GRAPH / HF_E_INVALID).  Domain: |q/p| > 0,
                        m0 above the pair's threshold, Gamma0 > 0 (else HF_E_DOMAIN)    */,
  HF_OP_MAP = 8      /* piecewise density (section "Combining functions": MappedPdf):
                        P(x) = P_j(x) / Z for x in the j-th of the K ranges [lo, b_1),
                        [b_1, b_2), ..., [b_{K-1}, hi] of observable x's box; children = K >= 2
                        one-observable EXP / GAUSS / POLY leaves on x, each normalised over
                        the box; Z = sum_j int_{range j} P_j dx; obs = {x}; no par;
                        consts = {b_1 < ... < b_{K-1}}, strictly inside the box             */,
  HF_OP_DPMAP = 9    /* density of an observable u that varies across the Dalitz plot
                        (section "Results": the decay-time uncertainty's distribution):
                        P(u | s12, s13) = P_c(u), c = i12 n13 + i13 the event's cell of the
                        n12 x n13 grid cut at the inner boundaries b12 of s12 and b13 of s13
                        (a boundary belongs to the cell above it); obs = {s12, s13, u};
                        children = the n12 n13 cells' one-observable EXP / GAUSS / POLY leaves
                        on u (row-major, s12 index first), each normalised over u's box; no
                        par; consts = {n12, n13, b12 (n12 - 1, increasing), b13 (n13 - 1)}.
                        Only as a PROD child beside the DALITZ / TDDP node on the same
                        (s12, s13); u may be that TDDP's sigma_t (which it then describes)
                        or an observable no other child uses                                */,
  HF_OP_CONV = 10    /* numerical convolution (section "Combining functions": ConvolutionPdf):
                        P(x) = sum_k f_M(t_k) f_R(x - t_k) / Z over the N midpoints t_k of x's
                        box, the residual x - t_k restricted to [d_lo, d_hi]; children =
                        {model, resolution}, one-observable EXP / GAUSS / POLY (degree <= 4)
                        leaves on x taken as unnormalised shapes f (EXP e^{alpha (v - lo)},
                        GAUSS e^{-(v - mu)^2 / (2 sigma^2)}, POLY 1 + sum a_j (v - x0)^j, v
                        the model's t or the resolution's residual); the resolution may
                        also be an ADD of 2 or 3 GAUSS leaves on x, a mixture whose
                        components are each normalised over [d_lo, d_hi];
                        Z = sum_k f_M(t_k) int_box f_R(x - t_k) dx (closed forms, on the
                        host); obs = {x}; no par; consts = {N (2..4096), d_lo, d_hi}; the
                        per-event sum visits only the points whose residual can lie in
                        [d_lo, d_hi] (cost ~ N (d_hi - d_lo) / box width per event), and a
                        graph whose one CONV node has N <= 512 reads the model's values at
                        the grid points from a table each block builds once; range
                        tests take t_k = lo + (k + 1/2) h and x - t_k in double on the
                        stored event value; a model shape <= 0 at a grid point whose
                        residual window meets the box is a domain error of the parameters,
                        a resolution shape <= 0 at a residual an event uses makes that
                        event's density undefined (domain error)                            */,
  HF_OP_COMP = 11    /* function composition (section "Combining functions": CompositePdf):
                        P(x) = f(g(x)) / Z with the core g(x) = 1 + sum_j a_j (x - x0)^j, a
                        POLY leaf's value (degree <= 4), and f an EXP / GAUSS / POLY (degree
                        <= 4) leaf's unnormalised shape (as for HF_OP_CONV) evaluated at g;
                        Z = int_box f(g(x)) dx by 16-point Gauss-Legendre on 128 segments on
                        the host; children = {core, shell} on x; obs = {x}; no par or consts */
};

/* DALITZ block of node constants:
 *   {M, m1, m2, m3, r, G, R, then R times (channel, m0, Gamma0, J)}
 * M: parent mass; m1..m3: daughter masses (GeV); r: Blatt-Weisskopf radius
 * (1/GeV); G: normalisation grid size (G x G midpoint cells over the box
 * [(m1+m2)^2, (M-m3)^2] x [(m1+m3)^2, (M-m2)^2], a cell counting when its
 * centre is inside the plot in both orderings); R <= 8 resonances (16 for a
 * TDDP node; the full form appends 1 + R constants, see HF_OP_TDDP); channel
 * 12, 13 or 23 (pair of daughters); J in {0, 1, 2}.  Amplitude of a
 * resonance: B_J(q) Z_J BW(s_AB) with the mass-dependent width
 * Gamma(s) = Gamma0 (q/q0)^{2J+1} (m0/sqrt s) B_J^2, Blatt-Weisskopf ratios
 * B_J and Zemach spin factors Z_J.  The constant term has c_0 = 1. */

/* Observable: Variable(name, lower limit, upper limit) of the paper's first
 * listing.  lo < hi; infinite limits are allowed only for the t and sigma_t
 * observables of a TDDP node. */
typedef struct { const char* name; double lo, hi; } hf_obs;

/* Fit parameter: Variable(name, initial value, step size, lower, upper) of the
 * first listing.  lo == hi means unbounded.  fixed != 0 keeps it at `init`
 * in fits (its gradient entry is 0). */
typedef struct { const char* name; double init, step, lo, hi; int32_t fixed; } hf_param;

/* One node of the tree, in post-order (children before parents). */
typedef struct {
  int32_t op;                        /* hf_op */
  int32_t n_child; const int32_t* child;   /* indices of earlier nodes */
  int32_t n_par;   const int32_t* par;     /* indices into the hf_param array */
  int32_t n_obs;   const int32_t* obs;     /* indices into the hf_obs array */
  int32_t n_const; const double* consts;   /* op-specific constants (above) */
} hf_node;

typedef struct pdf_graph pdf_graph;
typedef struct dataset dataset;
typedef struct batch_engine batch_engine;

/* ------------------------------------------------------------------ graph
 * Validates and flattens the tree into the per-launch opcode / constant
 * table.  Errors (HF_E_GRAPH): child index not earlier than its parent or
 * used twice, root not the last reachable node, PROD children sharing an
 * observable, ADD children over different observables, wrong par/obs/const
 * counts for the op, lo >= hi, an unbounded box for an EXP/GAUSS/POLY/DALITZ
 * observable, more than 16 nodes, 48 gradient slots (32 in a graph of several
 * nodes) or 8 observables, a constant table beyond 192 entries.  The
 * arrays are copied; no GPU work is done here. */
int pdf_graph_create(const hf_obs* obs, int32_t n_obs, const hf_param* par, int32_t n_par,
                     const hf_node* nodes, int32_t n_nodes, int32_t root, pdf_graph** out);
void pdf_graph_destroy(pdf_graph* g);
/* Number of observables and parameters of a graph. */
int pdf_graph_shape(const pdf_graph* g, int32_t* n_obs, int32_t* n_par);

/* ------------------------------------------------------------------ data
 * Copies n_events events given as n_obs host columns (host_cols[o][i] is
 * observable o of event i, double) to device memory as structure-of-arrays
 * columns in the requested precision (the paper's setData step, section
 * "GooFit code").  Every value must lie inside its observable's box (and
 * Dalitz events inside the plot): otherwise HF_E_DOMAIN and nothing is
 * allocated.  Event order is preserved.  n_events may be 0.  Blocks until the
 * copy is done; the caller keeps ownership of the host columns. */
/* (Graphs with a CONV node: the events are stored sorted by that node's
 * observable, all columns permuted alike; the likelihood does not depend on
 * the order, and dataset_read_column returns the stored order.) */
int dataset_upload(const pdf_graph* g, const double* const* host_cols, int64_t n_events,
                   hf_precision prec, void* hip_stream, dataset** out);
/* Borrows columns that already live in device memory (e.g. tensors of a
 * framework) instead of copying: dev_cols[o] is the device address of
 * observable o's column (n_events values; unused observables may be NULL).
 * HF_FP64: doubles, the observable's values.  HF_FP32_EVAL: floats, each
 * the value minus hf_column_ref(g, o, HF_FP32_EVAL), rounded once.  The
 * columns are not validated (events outside an observable's box or the
 * Dalitz plot give meaningless densities); they must stay allocated and
 * unchanged while the dataset is used, and stay owned by the caller
 * (dataset_free releases only the library's workspace).  Columns must be
 * aligned to their element size. */
int dataset_wrap_device(const pdf_graph* g, void* const* dev_cols, int64_t n_events, hf_precision prec,
                        dataset** out);
/* The reference subtracted from observable obs in the FP32-eval storage (the
 * middle of its box, 0 for an unbounded or unused observable; always 0 for
 * HF_FP64). */
int hf_column_ref(const pdf_graph* g, int32_t obs, hf_precision prec, double* ref);
/* Binned dataset: n_bins bin centres (host columns as for dataset_upload,
 * validated the same way) with weights[n_bins] >= 0 (finite), equal bins of
 * volume bin_volume > 0, and the metric that nll_eval / nll_grad / fit then
 * evaluate for it (the "NLL" outputs carry the metric's value).  Any graph
 * with at most 31 gradient slots; binned datasets are evaluated one at a
 * time (nll_grad_batched and the batch engine reject them). */
int dataset_upload_binned(const pdf_graph* g, const double* const* centres, const double* weights,
                          int64_t n_bins, double bin_volume, int32_t metric, hf_precision prec, void* hip_stream,
                          dataset** out);
/* Device-side toy generation (the toy / pseudo-experiment fits of the
 * paper's sections on fitting and of the serving loop, without moving their
 * events over PCIe): a dataset of n_events events drawn from graph g's
 * density at parameters params (n_par doubles), written in device memory on
 * hip_stream in the storage format of prec; the call returns when they are
 * written.  Sampleable graphs: an EXP or GAUSS leaf, an ADD of up to 4 such
 * leaves on one observable, or a PROD of those over their observables.
 * Random numbers: Philox4x32-10 (Salmon et al., SC 2011); uniform m of
 * event i is taken from the block with counter (i mod 2^32, i div 2^32,
 * m div 2, 0) and key (seed mod 2^32, seed div 2^32), words 0-1 (even m) or
 * 2-3 (odd m) as u = (floor((w_a 2^32 + w_b) / 2^11) + 1/2) 2^-53.  Per event,
 * the PROD's factors in order; an ADD takes one uniform to pick its child
 * (the first j with u < f_0 + ... + f_j, the last child taking the rest);
 * a leaf takes one uniform through its inverse CDF (EXP:
 * lo + ln(1 + u (e^{alpha L} - 1)) / alpha; GAUSS:
 * mu + sqrt(2) sigma erfinv(erf(z_lo) + u (erf(z_hi) - erf(z_lo)))), clamped
 * to the box.  HF_E_GRAPH for other graphs; HF_E_DOMAIN for sigma <= 0,
 * negative fractions or fractions summing above 1.  The same (graph, params,
 * n, seed) give the same events; event i does not depend on n. */
int dataset_generate(const pdf_graph* g, const double* params, int64_t n_events, uint64_t seed,
                     hf_precision prec, void* hip_stream, dataset** out);
/* Accept-reject toy generation on the device for any graph whose used
 * observables all have finite boxes (DALITZ, MAP, CONV, COMP, ... included;
 * not the time-dependent density): event i takes trials j = 0, 1, ...
 * (at most max_trials); with C used observables (column order = observable
 * index order), its uniforms j (C + 1) + c (numbered as for
 * dataset_generate) place the candidate's column c at lo + u (hi - lo), and
 * uniform j (C + 1) + C accepts the candidate when u * envelope < P(candidate)
 * (double precision; P = 0 outside the Dalitz plot).  envelope must bound
 * the normalised density over the box.  HF_E_DOMAIN when an event runs out
 * of trials or a candidate's density exceeds the envelope (no dataset is
 * returned), HF_E_GRAPH for an unbounded observable.  The first call on a
 * Dalitz graph computes its normalisation grid. */
int dataset_generate_ar(pdf_graph* g, const double* params, int64_t n_events, uint64_t seed, double envelope,
                        int32_t max_trials, hf_precision prec, void* hip_stream, dataset** out);
/* Copies observable obs of an unbinned dataset to the host as doubles (the
 * stored value, plus the column reference for HF_FP32_EVAL); host_out holds
 * n_events doubles.  Blocking on hip_stream. */
int dataset_read_column(const dataset* d, int32_t obs, void* hip_stream, double* host_out);
void dataset_free(dataset* d);
/* Device bytes held by a dataset (columns + workspace). */
int64_t dataset_device_bytes(const dataset* d);
/* Device bytes that dataset_upload / dataset_generate / dataset_generate_ar
 * would allocate for an unbinned dataset of n_events events of graph g in
 * precision prec (what dataset_device_bytes then reports), so that a caller
 * can reserve device memory before it uploads.  HF_E_INVALID for NULL
 * pointers, a negative or too large n_events or an unknown precision. */
int dataset_bytes_needed(const pdf_graph* g, int64_t n_events, hf_precision prec, int64_t* bytes);

/* ------------------------------------------------------------------ likelihood
 * params: n_par doubles (external values, fixed ones included).  Runs the
 * per-event evaluation and the deterministic two-pass reduction on
 * `hip_stream` and blocks until the result is on the host (the calling thread
 * spins on a flag that the reduction sets in mapped host memory, checking the
 * stream for errors while it waits).  One dataset must not be evaluated from
 * two threads at once.  A density <= 0 or
 * not finite at any event sets *nll = +INF and returns HF_E_DOMAIN.
 * Results are bitwise reproducible for the same inputs. */
int nll_eval(const pdf_graph* g, const dataset* d, const double* params, void* hip_stream,
             double* nll);
/* As nll_eval, plus grad[n_par] = dNLL/dtheta from the per-event adjoint
 * (0 for fixed parameters), including the derivative of the normalisation. */
int nll_grad(const pdf_graph* g, const dataset* d, const double* params, void* hip_stream,
             double* nll, double* grad);
/* n_fits independent evaluations (same graph, own datasets and parameters,
 * params is n_fits x n_par row-major) in one launch; each result is bitwise
 * equal to what nll_grad returns for that fit alone.  nll[n_fits],
 * grad[n_fits x n_par]; per-fit domain errors give +INF for that fit only
 * (the call still returns HF_OK).  A dataset may appear several times (for
 * example one dataset at several parameter points): each repeat is
 * evaluated by a following launch, as its partial sums have one workspace. */
int nll_grad_batched(const pdf_graph* g, const dataset* const* d, int32_t n_fits,
                     const double* params, void* hip_stream, double* nll, double* grad);
/* Per-event terms of the likelihood (the metric's per-event values, paper
 * section "GooFit code": the PDF evaluated at each event before the sum):
 * lnp[i] = ln P(x_i; params) and, when dlnp is not NULL, dlnp[i * n_par + p]
 * = d ln P(x_i) / d params[p] (0 for fixed parameters), for the n_events
 * events of an unbinned dataset in its stored order.  They come from the
 * evaluation kernels themselves, run so that each thread handles one event
 * and writes its terms instead of adding them, followed by the same host
 * assembly of normalisations as nll_grad; so nll_grad's NLL and gradient are
 * sums of exactly these per-event values (up to the order of summation).
 * Uses a temporary device buffer of at most 2^18 x (gradient slots + 1)
 * doubles.  Blocking on hip_stream.  HF_E_INVALID for a binned dataset or a
 * NULL lnp; HF_E_DOMAIN (all outputs still written, -INF where the density
 * is <= 0, and at every event with NaN derivatives when the parameters are
 * outside the density's domain) when the density is not positive and finite
 * at some event. */
int nll_terms(const pdf_graph* g, const dataset* d, const double* params, void* hip_stream, double* lnp,
              double* dlnp);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): nll_grad over
 * columns the caller already holds in device memory (dev_cols as for
 * dataset_wrap_device, in the storage format of prec; NULL allowed for
 * unused observables), with no dataset object and no allocation.  The
 * evaluation kernels' partial rows and the result row live in a fixed
 * 512 KiB device array of the library (one per GPU, kept until the process
 * ends); the result comes back by a copy on hip_stream, and the call blocks
 * until it is on the host.  Results are bitwise those of nll_grad on a
 * dataset holding the same events.  Calls that overlap in time on one GPU
 * share that array and race: serialise them.  HF_E_INVALID for NULL
 * arguments, misaligned or missing used columns, more partial rows than the
 * array holds (rows x (gradient slots + 1) > 65503 doubles; the default
 * row count, 4 per compute unit, needs at most 33792), graphs with a CONV
 * node (their events must be stored sorted) and Dalitz graphs whose
 * normalisation grid has not been computed by an earlier nll_eval /
 * nll_grad / fit; HF_E_DOMAIN as for nll_grad.  The columns are not
 * validated. */
int nll_grad_noalloc(const pdf_graph* g, void* const* dev_cols, int64_t n_events, hf_precision prec,
                     const double* params, void* hip_stream, double* nll, double* grad);

/* ------------------------------------------------------------------ fit
 * Quasi-Newton (BFGS) minimisation with MINUIT-style sine transforms for
 * bounded parameters, a bracketing line search, and a final Hessian from
 * central differences of the gradient (the MINUIT role of the paper's
 * FitManager section).  Errors are sqrt(diag(H^-1)), H the NLL Hessian. */
typedef struct {
  int32_t max_iter;     /* BFGS iterations (<= 0: 500) */
  double edm_tol;       /* stop when 0.5 g^T H^-1 g < edm_tol (<= 0: 1e-10) */
  int32_t grad_mode;    /* 0: analytic gradient (nll_grad); 1: central differences of nll_eval,
                           2 n_free extra evaluations per gradient */
  int32_t want_errors;  /* nonzero: compute the final Hessian, errors and covariance */
  double param_eps;     /* relative precision with which the evaluation sees the parameters:
                           the final Hessian's difference steps are at least 1e4 param_eps |x|,
                           so that rounding the parameters does not disturb them.  0: the
                           default (fit / batch_admit on FP32-eval datasets: 2^-24 for the
                           parameters the float kernels see rounded -- all but Gaussian means
                           and the decay time and width difference; otherwise exact);
                           > 0: this value for every parameter; < 0: exact */
} hf_fit_opts;

typedef struct {
  double nll, edm;
  int32_t n_iter, n_eval, status;   /* n_eval counts likelihood evaluations; status hf_status */
} hf_fit_summary;

/* params_inout: start values in, fitted values out (n_par).  errors_out
 * (n_par, nullable) and cov_out (n_par x n_par row-major, nullable) are 0 for
 * fixed parameters.  Returns HF_OK, HF_E_NOT_CONVERGED (results still
 * written) or an error. */
int fit(const pdf_graph* g, const dataset* d, const hf_fit_opts* opts, void* hip_stream,
        double* params_inout, double* errors_out, double* cov_out, hf_fit_summary* summary);

/* The same minimiser on any function: fn(x, &f, g, user) must set f and the
 * gradient g[n] at x (return 0; nonzero aborts with HF_E_INVALID; a non-finite
 * f means "outside the domain").  params gives start values, steps, bounds
 * and fixed flags (as for a graph); x0 (nullable) overrides the start values.
 * Host only: no GPU work. */
typedef int (*hf_fg_fn)(const double* x, double* f, double* g, void* user);
int hf_minimize(int32_t n, const hf_param* params, const double* x0, const hf_fit_opts* opts, double f_noise,
                hf_fg_fn fn, void* user, double* x_out, double* errors_out, double* cov_out,
                hf_fit_summary* summary);

/* ------------------------------------------------------------------ batched serving
 * A batch engine holds up to max_slots concurrent fits of one graph.  Each
 * batch_step advances every active fit's minimiser by one likelihood
 * evaluation, all of them in one graph-captured launch, so fits that are
 * admitted while others run share the device.  Admission is by device
 * memory: the datasets of the active fits may hold at most hbm_budget_bytes.
 * The engine borrows the datasets; the caller frees them after the fit is
 * polled. */
int batch_create(const pdf_graph* g, int32_t max_slots, int64_t hbm_budget_bytes, void* hip_stream,
                 batch_engine** out);
void batch_destroy(batch_engine* b);
/* Starts a fit of dataset d from params_init (n_par).  HF_E_FULL: no slot;
 * HF_E_BUDGET: not enough budget now (retry later); HF_E_INVALID: the dataset
 * alone exceeds the whole budget or its precision differs from the engine's
 * first dataset. */
int batch_admit(batch_engine* b, const dataset* d, const double* params_init, const hf_fit_opts* opts,
                int64_t tag, int32_t* slot_out);
/* One evaluation for every active fit; blocks until done.  n_active_out: fits
 * still running after the step; n_done_out: fits finished and waiting for
 * batch_poll. */
int batch_step(batch_engine* b, int32_t* n_active_out, int32_t* n_done_out);
/* Returns up to max finished fits and frees their slots and budget.  For each
 * i < return value: tags[i], status[i], params[i*n_par..], errors[i*n_par..],
 * nll[i], n_eval[i] (any output pointer may be NULL).  Returns the count
 * (>= 0) or an error. */
int batch_poll(batch_engine* b, int32_t max, int64_t* tags, int32_t* status, double* params,
               double* errors, double* nll, int32_t* n_eval);
/* Cancels an active fit by tag (its slot and budget are freed at once). */
int batch_cancel(batch_engine* b, int64_t tag);
/* Failure injection for tests of the engine's per-fit isolation, from the
 * host only: with HIPFIT_FAULT="tag:eval:domain" set when batch_create runs,
 * the fit with that tag receives NLL = +inf at its eval-th evaluation (as
 * from a density <= 0: its line search backs off); with "tag:eval:abort" the
 * fit ends there with status HF_E_HIP.  Other fits are unaffected.  A
 * malformed value makes batch_create fail with HF_E_INVALID. */

/* ------------------------------------------------------------------ misc
 * Dalitz-plot membership (the same rule as the normalisation grid) of n
 * points for the DALITZ/TDDP node `node` of a graph: out[i] = 1 inside. */
int hf_dalitz_inside(const pdf_graph* g, int32_t node, int64_t n, const double* s12,
                     const double* s13, uint8_t* out);
/* Kernel timing for measurement: enable = k >= 1 resets the counters and
 * starts timing the likelihood kernel and the reduction of every k-th
 * nll_eval / nll_grad with HIP events that take the dispatches' own start and
 * end time stamps (those calls wait on the completion flag as usual; their
 * time stamps are read at the next timed call or by the next hf_profile
 * call); enable = 0 stops; a negative value only reads.  Outputs (nullable):
 * total milliseconds of the likelihood kernels and of the reductions, and the
 * number of timed calls so far (all complete when read).  Not for concurrent
 * use from several threads. */
int hf_profile(int32_t enable, double* eval_ms, double* reduce_ms, int64_t* n_launch);
/* Last error message of the calling thread ("" if none); valid until the
 * thread's next call into the library.  last_error_message is the same
 * function under the boundary's plain name. */
const char* hf_last_error(void);
const char* last_error_message(void);
/* Library version string. */
const char* hf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HIPFIT_H */
