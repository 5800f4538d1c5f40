// C ABI of the solver (include/voxcap.h): problem lifecycle, GMRES driver (restarted,
// several right-hand sides in lock-step, right-preconditioned with eq. (14)), FP32/FP64
// iterative refinement, capacitance of eq. (8) and its adjoint permittivity derivative.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mvp_kernels.h"
#include "problem.h"

namespace vc {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

static const double kEps0 = 8.8541878128e-12;   // F/m

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------------------ GMRES
struct SolveSpec {
  vc_precision mvp;     // VC_FP64 or VC_FP32 product
  int transpose;
  int precond;          // 0 none, 1 block-diagonal-diagonal, 2 diagonal
  double rtol;
  int restart, max_iter;
};

static vc_status ensure_workspace(vc_problem* P, int nrhs, int restart) {
  if (P->s_nrhs >= nrhs && P->s_restart >= restart) return VC_OK;
  const int64_t N = npanels(P);
  const int r = std::max(restart, P->s_restart), k = std::max(nrhs, P->s_nrhs);
  if (k > 64) { set_error("at most 64 right-hand sides per solve"); return VC_ERR_ARG; }
  P->drop_graphs();   // captured graphs hold pointers into the old workspace
  VC_HIP(P->s_V.alloc((size_t)(r + 1) * k * N * sizeof(double)));
  VC_HIP(P->s_w.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_z.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_r.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_b.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_x.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_tmp.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_rr.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_dd.alloc((size_t)k * N * sizeof(double)));
  VC_HIP(P->s_h.alloc((size_t)2 * (r + 2) * k * sizeof(double)));
  VC_HIP(P->s_y2.alloc((size_t)(r + 2) * k * sizeof(double)));
  VC_HIP(P->s_partial.alloc((size_t)std::max(gemv_t_partial_size(N, r + 2, k), colnorm_partial_size(N, k)) *
                            sizeof(double)));
  VC_HIP(P->s_norm.alloc((size_t)4 * k * sizeof(double)));
  VC_HIP(P->s_active.alloc((size_t)k * sizeof(int)));
  // device-side cycle state: H, cs, sn, g, bn, rn, rre, scal (doubles); kd, iters,
  // act_cycle, act_step (ints) + skip[2], bad
  const size_t nd = (size_t)k * ((size_t)(r + 1) * r + 2 * r + (r + 1) + 4) + 1;
  VC_HIP(P->s_cyc.alloc(nd * sizeof(double)));
  VC_HIP(P->s_cyci.alloc(((size_t)4 * k + 4) * sizeof(int)));
  P->s_nrhs = k;
  P->s_restart = r;
  return VC_OK;
}

// views of the cycle state for one (nrhs, restart) solve
struct Cyc {
  double *H, *cs, *sn, *g, *bn, *rn, *rre, *scal, *rtol;
  int *kd, *iters, *act_cycle, *act_step, *skip, *bad;
};
static Cyc cycle_views(vc_problem* P, int nrhs, int m) {
  Cyc c{};
  double* d = P->s_cyc.as<double>();
  c.H = d; d += (size_t)nrhs * (m + 1) * m;
  c.cs = d; d += (size_t)nrhs * m;
  c.sn = d; d += (size_t)nrhs * m;
  c.g = d; d += (size_t)nrhs * (m + 1);
  c.bn = d; d += nrhs;
  c.rn = d; d += nrhs;
  c.rre = d; d += nrhs;
  c.scal = d; d += nrhs;
  c.rtol = d;
  int* q = P->s_cyci.as<int>();
  c.kd = q; q += nrhs;
  c.iters = q; q += nrhs;
  c.act_cycle = q; q += nrhs;
  c.act_step = q; q += nrhs;
  c.skip = q; q += 2;
  c.bad = q;
  return c;
}

// z = R v (if preconditioned), w = A z; skipped entirely when *skip
static vc_status op_with_precond(vc_problem* P, const SolveSpec& sp, const double* v, double* z, double* w, int nrhs,
                                 hipStream_t st, const int* skip = nullptr) {
  const double* src = v;
  if (sp.precond) {
    P->pc.mode = sp.precond;
    vc_status s = apply_precond(P, sp.transpose, v, z, nrhs, st, skip);
    if (s != VC_OK) return s;
    src = z;
  }
  return apply_op(P, sp.transpose, sp.mvp, src, w, nrhs, st, skip);
}

// r = b - A x
static vc_status residual(vc_problem* P, const SolveSpec& sp, const double* b, const double* x, double* r, int nrhs,
                          hipStream_t st) {
  const int64_t N = npanels(P);
  vc_status s = apply_op(P, sp.transpose, sp.mvp, x, r, nrhs, st);
  if (s != VC_OK) return s;
  VC_HIP(launch_axpy_cols(r, b, N, nrhs, nullptr, 1, st));
  return VC_OK;
}

static vc_status col_norms(vc_problem* P, const double* w, int64_t N, int nrhs, double* d_out, std::vector<double>& h,
                           hipStream_t st) {
  VC_HIP(launch_colnorm(w, N, N, nrhs, d_out, P->s_partial.as<double>(), st));
  h.resize(nrhs);
  VC_HIP(hipMemcpyAsync(h.data(), d_out, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  VC_HIP(hipStreamSynchronize(st));
  return VC_OK;
}

// One GMRES(m) restart cycle, every step on the device (so it can be captured):
// residual and its norms, cycle start (masks, g, skip flags), m Arnoldi steps with
// classical Gram-Schmidt applied twice and the Givens update, then x += R V y for the
// columns that were active at the start.  Columns freeze once converged; when all
// have, the remaining steps' products are skipped by the device flag.
static vc_status issue_cycle(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs,
                             hipStream_t st) {
  const int64_t N = npanels(P);
  const int m = sp.restart;
  const Cyc c = cycle_views(P, nrhs, m);
  double* V = P->s_V.as<double>();
  double* w = P->s_w.as<double>();
  double* z = P->s_z.as<double>();
  double* r = P->s_r.as<double>();
  double* hd = P->s_h.as<double>();
  double* y2 = P->s_y2.as<double>();
  double* nrm = P->s_norm.as<double>();
  const int64_t ldv = (int64_t)nrhs * N;
  const int ldh = m + 2;
  vc_status s = residual(P, sp, b, x, r, nrhs, st);
  if (s != VC_OK) return s;
  VC_HIP(launch_colnorm(r, N, N, nrhs, c.rn, P->s_partial.as<double>(), st));
  VC_HIP(launch_cycle_start(nrhs, m, c.rn, c.bn, c.rtol, c.act_cycle, c.act_step, c.g, c.scal, c.kd, c.skip, c.rre,
                            st));
  VC_HIP(launch_scale_copy(V, r, N, nrhs, c.scal, c.skip, st));   // V_0 = r / |r|
  for (int j = 0; j < m; ++j) {
    s = op_with_precond(P, sp, V + j * ldv, z, w, nrhs, st, c.skip + 1);
    if (s != VC_OK) return s;
    VC_HIP(launch_gemv_t(V, ldv, N, j + 1, w, N, nrhs, hd, ldh, c.act_step, P->s_partial.as<double>(), st));
    VC_HIP(launch_gemv_n_sub(V, ldv, N, j + 1, hd, ldh, w, N, nrhs, c.act_step, 0, st));
    VC_HIP(launch_gemv_t(V, ldv, N, j + 1, w, N, nrhs, hd + (size_t)ldh * nrhs, ldh, c.act_step,
                         P->s_partial.as<double>(), st));
    VC_HIP(launch_gemv_n_sub(V, ldv, N, j + 1, hd + (size_t)ldh * nrhs, ldh, w, N, nrhs, c.act_step, 0, st));
    VC_HIP(launch_colnorm(w, N, N, nrhs, nrm, P->s_partial.as<double>(), st));
    VC_HIP(launch_arnoldi(j, nrhs, m, hd, hd + (size_t)ldh * nrhs, ldh, nrm, c.H, c.cs, c.sn, c.g, c.bn, c.rtol,
                          c.act_step, c.kd, c.iters, c.scal, c.skip, c.bad, st));
    if (j + 1 < m) VC_HIP(launch_scale_copy(V + (j + 1) * ldv, w, N, nrhs, c.scal, c.skip + 1, st));
  }
  // x += R V y, y = R_H^{-1} g over each column's steps
  VC_HIP(launch_backsolve(nrhs, m, c.H, c.g, c.kd, c.act_cycle, y2, ldh, st));
  VC_HIP(launch_zero(w, (int64_t)nrhs * N, st));
  VC_HIP(launch_gemv_n_sub(V, ldv, N, m, y2, ldh, w, N, nrhs, c.act_cycle, 0, st));   // w = V y
  const double* upd = w;
  if (sp.precond) {
    P->pc.mode = sp.precond;
    s = apply_precond(P, sp.transpose, w, z, nrhs, st, c.skip);
    if (s != VC_OK) return s;
    upd = z;
  }
  VC_HIP(launch_add_active(x, upd, N, nrhs, c.act_cycle, c.skip, st));
  return VC_OK;
}

// Solve A x = b (x holds the initial guess).  iters/rre: per column outputs.  With
// graphs on, every cycle replays one graph captured at the first solve of this shape
// (rtol is read from device memory, so solves to any tolerance share it); an eager
// product before the capture settles the autotuned launch configuration.
static vc_status gmres(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs,
                       std::vector<int>& iters, std::vector<double>& rre, hipStream_t st) {
  const int64_t N = npanels(P);
  const int m = sp.restart;
  vc_status s = ensure_workspace(P, nrhs, m);
  if (s != VC_OK) return s;
  const Cyc c = cycle_views(P, nrhs, m);
  VC_HIP(hipMemcpyAsync(c.rtol, &sp.rtol, sizeof(double), hipMemcpyHostToDevice, st));
  VC_HIP(launch_colnorm(b, N, N, nrhs, c.bn, P->s_partial.as<double>(), st));
  VC_HIP(hipMemsetAsync(c.iters, 0, (size_t)nrhs * sizeof(int), st));
  VC_HIP(hipMemsetAsync(c.bad, 0, sizeof(int), st));
  std::vector<int> it(nrhs), skip(2);
  rre.assign(nrhs, 0.0);
  int bad = 0;
  vc_problem::GraphKey key{(int)sp.mvp, sp.transpose, sp.precond, nrhs, m, b, x};
  for (int cycle = 0;; ++cycle) {
    if (P->use_graphs) {
      hipGraphExec_t ex = P->find_graph(key);
      if (!ex) {
        // eager product first: launch configurations chosen (and timed, with the
        // autotuner) outside the capture
        s = apply_op(P, sp.transpose, sp.mvp, b, P->s_tmp.as<double>(), nrhs, st);
        if (s != VC_OK) return s;
        VC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        vc_status sc = issue_cycle(P, sp, b, x, nrhs, st);
        hipGraph_t gr = nullptr;
        const hipError_t ee = hipStreamEndCapture(st, &gr);
        if (sc != VC_OK) { if (gr) (void)hipGraphDestroy(gr); return sc; }
        if (ee != hipSuccess) { set_error("graph capture failed: %s", hipGetErrorString(ee)); return VC_ERR_HIP; }
        const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
          (void)hipGraphDestroy(gr);
          set_error("graph instantiation failed: %s", hipGetErrorString(ei));
          return VC_ERR_HIP;
        }
        P->add_graph(key, gr, ex);
      }
      VC_HIP(hipGraphLaunch(ex, st));
    } else {
      s = issue_cycle(P, sp, b, x, nrhs, st);
      if (s != VC_OK) return s;
    }
    VC_HIP(hipMemcpyAsync(rre.data(), c.rre, (size_t)nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    VC_HIP(hipMemcpyAsync(it.data(), c.iters, (size_t)nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
    VC_HIP(hipMemcpyAsync(skip.data(), c.skip, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    VC_HIP(hipMemcpyAsync(&bad, c.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    VC_HIP(hipStreamSynchronize(st));
    iters = it;
    for (int k = 0; k < nrhs; ++k)
      if (!std::isfinite(rre[k])) { set_error("non-finite residual in column %d", k); return VC_ERR_NUMERIC; }
    if (bad) { set_error("non-finite Arnoldi coefficient"); return VC_ERR_NUMERIC; }
    if (skip[0]) return VC_OK;   // every column met rtol at the start of this cycle
    const int total = *std::max_element(it.begin(), it.end());
    if (total >= sp.max_iter) {
      // this cycle already advanced x: report the residual it starts from
      set_error("GMRES did not reach rtol %.3g in %d iterations (worst rre %.3g at the last restart)", sp.rtol,
                total, *std::max_element(rre.begin(), rre.end()));
      return VC_ERR_NOT_CONVERGED;
    }
  }
}

// the (blocking, default-priority) stream the solves run on: graphs cannot be captured
// on the null stream, and a blocking stream stays ordered with null-stream copies
static hipStream_t get_solve_stream(vc_problem* P) {
  if (!P->solve_stream && hipStreamCreate(&P->solve_stream) != hipSuccess) P->solve_stream = nullptr;
  return P->solve_stream;
}

// FP64 solve, or FP32-product GMRES inside FP64 refinement (VC_MIXED).
static vc_status solve(vc_problem* P, const vc_solve_opts& o, int transpose, const double* b, double* x, int nrhs,
                       vc_stats* stats, hipStream_t st) {
  const int64_t N = npanels(P);
  SolveSpec sp{};
  sp.transpose = transpose;
  sp.precond = o.use_precond;
  sp.restart = o.restart;
  sp.max_iter = o.max_iter;
  std::vector<int> it;
  std::vector<double> rre;
  P->use_graphs = o.graph == 0;
  if (!st) st = get_solve_stream(P);
  if (!st) { set_error("could not create the solve stream"); return VC_ERR_HIP; }
  VC_HIP(hipMemsetAsync(x, 0, (size_t)nrhs * N * sizeof(double), st));
  int ir_steps = 0;
  vc_status s;
  if (o.prec != VC_MIXED) {
    sp.mvp = o.prec == VC_FP32 ? VC_FP32 : VC_FP64;
    sp.rtol = o.rtol;
    s = gmres(P, sp, b, x, nrhs, it, rre, st);
  } else {
    // outer FP64 refinement: r = b - A x (FP64 product), inner FP32 GMRES on A d = r, x += d
    s = ensure_workspace(P, nrhs, o.restart);
    if (s != VC_OK) return s;
    double* rrp = P->s_rr.as<double>();   // stable buffers: the inner solves reuse their graph
    double* ddp = P->s_dd.as<double>();
    std::vector<int> tot(nrhs, 0);
    SolveSpec s64 = sp;
    s64.mvp = VC_FP64;
    std::vector<double> bn, rn;
    s = col_norms(P, b, N, nrhs, P->s_norm.as<double>(), bn, st);
    if (s != VC_OK) return s;
    VC_HIP(hipMemcpyAsync(rrp, b, (size_t)nrhs * N * sizeof(double), hipMemcpyDeviceToDevice, st));
    s = VC_ERR_NOT_CONVERGED;
    rre.assign(nrhs, 1.0);
    for (ir_steps = 0; ir_steps < o.ir_max; ++ir_steps) {
      SolveSpec s32 = sp;
      s32.mvp = VC_FP32;
      s32.rtol = o.inner_rtol;
      VC_HIP(hipMemsetAsync(ddp, 0, (size_t)nrhs * N * sizeof(double), st));
      vc_status si = gmres(P, s32, rrp, ddp, nrhs, it, rre, st);
      if (si != VC_OK && si != VC_ERR_NOT_CONVERGED) return si;
      for (int c = 0; c < nrhs; ++c) tot[c] += it[c];
      std::vector<double> ones(nrhs, 1.0);
      VC_HIP(hipMemcpyAsync(P->s_norm.as<double>() + nrhs, ones.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
      VC_HIP(launch_axpy_cols(x, ddp, N, nrhs, P->s_norm.as<double>() + nrhs, 0, st));
      vc_status sr = residual(P, s64, b, x, rrp, nrhs, st);
      if (sr != VC_OK) return sr;
      sr = col_norms(P, rrp, N, nrhs, P->s_norm.as<double>(), rn, st);
      if (sr != VC_OK) return sr;
      bool ok = true;
      for (int c = 0; c < nrhs; ++c) {
        rre[c] = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
        if (rre[c] > o.rtol) ok = false;
      }
      if (ok) { s = VC_OK; ++ir_steps; break; }
    }
    it = tot;
    if (s != VC_OK) set_error("refinement did not reach rtol %.3g in %d steps", o.rtol, o.ir_max);
  }
  if (stats) {
    for (int c = 0; c < nrhs && c < 64; ++c) {
      stats->iters[c] = c < (int)it.size() ? it[c] : 0;
      stats->final_rre[c] = c < (int)rre.size() ? rre[c] : 0.0;
    }
    stats->ir_steps = ir_steps;
  }
  return s;
}

static vc_solve_opts fill_defaults(const vc_solve_opts* in) {
  vc_solve_opts o{};
  if (in) o = *in;
  if (o.rtol <= 0) o.rtol = 1e-12;
  if (o.restart <= 0) o.restart = 35;
  if (o.max_iter <= 0) o.max_iter = 2000;
  if (o.inner_rtol <= 0) o.inner_rtol = 1e-5;
  if (o.ir_max <= 0) o.ir_max = 20;
  if (!in) o.use_precond = 1;
  return o;
}

}  // namespace vc

using namespace vc;

#define VC_CHECK_PROBLEM(p)                                          \
  do {                                                               \
    if (!(p)) { set_error("null problem"); return VC_ERR_ARG; }      \
    if ((p)->hip_failed) { set_error("problem unusable after a HIP error"); return VC_ERR_HIP; } \
  } while (0)

static vc_status mark(vc_problem* p, vc_status s) {
  if (s == VC_ERR_HIP && p) p->hip_failed = true;
  return s;
}

extern "C" {

const char* vc_status_string(vc_status s) {
  switch (s) {
    case VC_OK: return "ok";
    case VC_ERR_ARG: return "invalid argument";
    case VC_ERR_GEOMETRY: return "invalid geometry";
    case VC_ERR_HIP: return "HIP runtime error";
    case VC_ERR_OOM: return "out of memory";
    case VC_ERR_NOT_CONVERGED: return "not converged";
    case VC_ERR_NUMERIC: return "numerical breakdown";
    case VC_ERR_STATE: return "call out of order";
  }
  return "unknown status";
}

const char* vc_last_error(void) { return g_err.c_str(); }

vc_status vc_problem_create(const vc_geometry* g, int device, vc_problem** out) {
  if (!g || !out || !g->cond_id || !g->eps_r) { set_error("null argument"); return VC_ERR_ARG; }
  *out = nullptr;
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || !(g->dv > 0.0)) { set_error("grid sizes and dv must be > 0"); return VC_ERR_ARG; }
  const int64_t nv = (int64_t)g->nx * g->ny * g->nz;
  if (nv > (int64_t)1 << 31) { set_error("grid too large"); return VC_ERR_ARG; }
  vc_problem* p = new (std::nothrow) vc_problem();
  if (!p) { set_error("host allocation failed"); return VC_ERR_OOM; }
  p->device = device;
  p->nx = g->nx; p->ny = g->ny; p->nz = g->nz;
  p->dv = g->dv;
  p->eps_b = g->eps_background > 0 ? g->eps_background : (g->eps_background == 0 ? 1.0 : g->eps_background);
  p->cond_id.assign(g->cond_id, g->cond_id + nv);
  p->eps_r.assign(g->eps_r, g->eps_r + nv);
  vc_status s = panelize(p);
  if (s == VC_OK) s = choose_sizes(p, nullptr);
  if (s != VC_OK) { delete p; return s; }
  *out = p;
  return VC_OK;
}

vc_status vc_problem_destroy(vc_problem* p) {
  if (!p) return VC_OK;
  if (p->setup_done) (void)hipSetDevice(p->device);
  delete p;
  return VC_OK;
}

vc_status vc_panel_counts(const vc_problem* p, int64_t* n_cond, int64_t* n_diel, int32_t* m) {
  if (!p) { set_error("null problem"); return VC_ERR_ARG; }
  if (n_cond) *n_cond = p->n_cond;
  if (n_diel) *n_diel = p->n_diel;
  if (m) *m = p->m;
  return VC_OK;
}

vc_status vc_panels(const vc_problem* p, vc_panel* out) {
  if (!p || !out) { set_error("null argument"); return VC_ERR_ARG; }
  std::memcpy(out, p->panels.data(), p->panels.size() * sizeof(vc_panel));
  return VC_OK;
}

vc_status vc_fft_size(const vc_problem* p, int32_t out_m[3]) {
  if (!p || !out_m) { set_error("null argument"); return VC_ERR_ARG; }
  for (int a = 0; a < 3; ++a) out_m[a] = p->M[a];
  return VC_OK;
}

vc_status vc_setup(vc_problem* p, const vc_setup_opts* opts, void* stream) {
  VC_CHECK_PROBLEM(p);
  vc_setup_opts o{};
  if (opts) o = *opts;
  if (o.tucker_tol < 0) { set_error("tucker_tol must be >= 0"); return VC_ERR_ARG; }
  const double t0 = now_s();
  VC_HIP(hipSetDevice(p->device));
  p->drop_graphs();   // they hold pointers to tables and work arrays set up again below
  hipStream_t st = (hipStream_t)stream;
  vc_status s = choose_sizes(p, (o.fft_size[0] || o.fft_size[1] || o.fft_size[2]) ? o.fft_size : nullptr);
  if (s != VC_OK) return s;
  for (int a = 0; a < 3; ++a) p->nv[a] = o.nv[a] > 0 ? o.nv[a] : 8;
  const int prec = o.precisions ? o.precisions : 3;
  p->tk.clear();
  p->tucker_tol = 0.0;
  s = build_spectra(p, (prec & 1) != 0, (prec & 2) != 0, o.tucker_tol, st);
  if (s != VC_OK) return mark(p, s);
  p->max_rhs = o.max_rhs > 0 ? o.max_rhs : p->m;
  p->autotune = o.autotune != 0;
  p->sand_choice.clear();
  const bool diel = p->n_diel > 0;
  p->ncomp_F = diel ? 6 : 3;
  p->ncomp_O = diel ? 6 : 3;
  p->rhs_stride = (int64_t)p->n1[0] * p->M[1] * p->H;
  p->comp_stride = p->rhs_stride * p->max_rhs;
  const size_t cb = 16;   // complex double
  VC_HIP(p->work_F.alloc((size_t)p->ncomp_F * p->comp_stride * cb));
  VC_HIP(p->work_O.alloc((size_t)p->ncomp_O * p->comp_stride * cb));
  s = build_precond(p, st);
  if (s != VC_OK) return mark(p, s);
  VC_HIP(hipStreamSynchronize(st));
  p->setup_done = true;
  p->t_setup = now_s() - t0;
  return VC_OK;
}

vc_status vc_apply(vc_problem* p, int transpose, vc_precision prec, const double* x, double* y, int32_t nrhs,
                   void* stream) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_apply before vc_setup"); return VC_ERR_STATE; }
  if (!x || !y || nrhs <= 0 || nrhs > p->max_rhs) { set_error("bad x/y or nrhs (1..%d)", p->max_rhs); return VC_ERR_ARG; }
  if (prec != VC_FP64 && prec != VC_FP32) { set_error("prec must be VC_FP64 or VC_FP32"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(p->device));
  return mark(p, apply_op(p, transpose, prec, x, y, nrhs, (hipStream_t)stream));
}

vc_status vc_apply_precond(vc_problem* p, int transpose, const double* x, double* y, int32_t nrhs, void* stream) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_apply_precond before vc_setup"); return VC_ERR_STATE; }
  if (!x || !y || nrhs <= 0) { set_error("bad arguments"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(p->device));
  p->pc.mode = 1;
  return mark(p, apply_precond(p, transpose, x, y, nrhs, (hipStream_t)stream));
}

static vc_status capacitance_impl(vc_problem* p, const vc_solve_opts* opts, double* C, double* rho_dev, vc_stats* stats,
                                  std::vector<double>* rho_host) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_capacitance before vc_setup"); return VC_ERR_STATE; }
  if (!C) { set_error("null C"); return VC_ERR_ARG; }
  vc_solve_opts o = fill_defaults(opts);
  if ((o.prec == VC_FP32 || o.prec == VC_MIXED) && !p->have32) { set_error("FP32 spectra not built"); return VC_ERR_STATE; }
  if (p->m > p->max_rhs) { set_error("setup max_rhs < number of conductors"); return VC_ERR_STATE; }
  VC_HIP(hipSetDevice(p->device));
  const double t0 = now_s();
  hipStream_t st = get_solve_stream(p);
  if (!st) { set_error("could not create the solve stream"); return VC_ERR_HIP; }
  const int64_t N = npanels(p);
  const int m = p->m;
  p->mvp_count = 0;
  vc_status s = ensure_workspace(p, m, o.restart);
  if (s != VC_OK) return mark(p, s);
  std::vector<double> B((size_t)m * N, 0.0);
  for (int64_t k = 0; k < N; ++k)
    if (p->panels[k].kind == 0) B[(size_t)p->panels[k].cond * N + k] = 1.0;
  VC_HIP(hipMemcpy(p->s_b.p, B.data(), B.size() * sizeof(double), hipMemcpyHostToDevice));
  if (stats) std::memset(stats, 0, sizeof(vc_stats));
  s = solve(p, o, 0, p->s_b.as<double>(), p->s_x.as<double>(), m, stats, st);
  if (s != VC_OK && s != VC_ERR_NOT_CONVERGED) return mark(p, s);
  DevMem dC;
  VC_HIP(dC.alloc((size_t)m * m * sizeof(double)));
  VC_HIP(launch_cap_reduce(p->s_x.as<double>(), N, m, p->d_cond_panels.as<int32_t>(), p->d_cond_ptr.as<int32_t>(),
                           p->d_weight.as<double>(), 4.0 * M_PI * kEps0 * p->dv, dC.as<double>(), st));
  VC_HIP(hipMemcpy(C, dC.p, (size_t)m * m * sizeof(double), hipMemcpyDeviceToHost));
  if (rho_dev) VC_HIP(hipMemcpy(rho_dev, p->s_x.p, (size_t)m * N * sizeof(double), hipMemcpyDeviceToDevice));
  if (rho_host) {
    rho_host->resize((size_t)m * N);
    VC_HIP(hipMemcpy(rho_host->data(), p->s_x.p, (size_t)m * N * sizeof(double), hipMemcpyDeviceToHost));
  }
  if (stats) {
    stats->mvp_count = p->mvp_count;
    stats->t_setup_s = p->t_setup;
    stats->t_solve_s = now_s() - t0;
    stats->spectra_bytes = p->spectra_bytes;
    int rmax = 0;
    for (const auto& t : p->tk) rmax = std::max(rmax, std::max(t.r[0], std::max(t.r[1], t.r[2])));
    stats->tucker_rank_max = rmax;
  }
  return s;
}

vc_status vc_capacitance(vc_problem* p, const vc_solve_opts* opts, double* C, double* rho_dev, vc_stats* stats) {
  return capacitance_impl(p, opts, C, rho_dev, stats, nullptr);
}

vc_status vc_capacitance_grad_eps(vc_problem* p, const vc_solve_opts* opts, const int32_t* block_of_voxel,
                                  int32_t nblocks, double* dC, double* C_out, vc_stats* stats) {
  VC_CHECK_PROBLEM(p);
  if (!block_of_voxel || nblocks <= 0 || !dC) { set_error("bad gradient arguments"); return VC_ERR_ARG; }
  const int m = p->m;
  const int64_t N = npanels(p);
  std::vector<double> C((size_t)m * m);
  vc_status s = capacitance_impl(p, opts, C.data(), nullptr, stats, nullptr);
  if (s != VC_OK) return s;
  if (C_out) std::memcpy(C_out, C.data(), C.size() * sizeof(double));
  DevMem rho;
  VC_HIP(rho.alloc((size_t)m * N * sizeof(double)));
  VC_HIP(hipMemcpy(rho.p, p->s_x.p, (size_t)m * N * sizeof(double), hipMemcpyDeviceToDevice));
  // adjoint solves A^T lambda_i = w_i, w_i = eps_adj on the panels of conductor i
  vc_solve_opts o = fill_defaults(opts);
  std::vector<double> W((size_t)m * N, 0.0);
  for (int64_t k = 0; k < N; ++k)
    if (p->panels[k].kind == 0) W[(size_t)p->panels[k].cond * N + k] = p->panels[k].eps_adj;
  VC_HIP(hipMemcpy(p->s_b.p, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice));
  s = solve(p, o, 1, p->s_b.as<double>(), p->s_x.as<double>(), m, nullptr, get_solve_stream(p));
  if (s != VC_OK) return mark(p, s);
  // per-block entries of the derivative (index bookkeeping on the host, sums on the GPU):
  //   conductor panel k: d w_{cond k} / d eps(non-conductor side block) = 1 (eq. 8)
  //   dielectric panel k: d I_kk / d eps_lo = -4 pi eps_hi / (eps_lo - eps_hi)^2,
  //                       d I_kk / d eps_hi = +4 pi eps_lo / (eps_lo - eps_hi)^2 (eq. 7)
  auto vox = [&](int i, int j, int k) -> int32_t {
    if (i < 0 || j < 0 || k < 0 || i >= p->nx || j >= p->ny || k >= p->nz) return -1;
    return block_of_voxel[((int64_t)i * p->ny + j) * p->nz + k];
  };
  std::vector<std::vector<int32_t>> ek(nblocks), ec(nblocks);
  std::vector<std::vector<double>> ef(nblocks);
  for (int64_t k = 0; k < N; ++k) {
    const vc_panel& pn = p->panels[k];
    int lo[3] = {pn.i, pn.j, pn.k};
    lo[pn.dir] -= 1;
    const int32_t blo = vox(lo[0], lo[1], lo[2]);
    const int32_t bhi = vox(pn.i, pn.j, pn.k);
    if (pn.kind == 0) {
      const int32_t b = pn.eps_lo == 0.0 ? bhi : blo;   // non-conductor side
      if (b < 0 || b >= nblocks) continue;
      ek[b].push_back((int32_t)k); ec[b].push_back(pn.cond); ef[b].push_back(1.0);
    } else {
      const double el = pn.eps_lo, eh = pn.eps_hi, dd = (el - eh) * (el - eh);
      const double d[2] = {-4.0 * M_PI * eh / dd, 4.0 * M_PI * el / dd};
      for (int side = 0; side < 2; ++side) {
        const int32_t b = side == 0 ? blo : bhi;
        if (b < 0 || b >= nblocks) continue;
        ek[b].push_back((int32_t)k); ec[b].push_back(-1); ef[b].push_back(d[side]);
      }
    }
  }
  std::vector<int32_t> bptr(nblocks + 1, 0), fk, fc;
  std::vector<double> ff;
  for (int b = 0; b < nblocks; ++b) {
    fk.insert(fk.end(), ek[b].begin(), ek[b].end());
    fc.insert(fc.end(), ec[b].begin(), ec[b].end());
    ff.insert(ff.end(), ef[b].begin(), ef[b].end());
    bptr[b + 1] = (int32_t)fk.size();
  }
  DevMem d_bptr, d_k, d_c, d_f, d_dC;
  VC_HIP(d_bptr.alloc(bptr.size() * sizeof(int32_t)));
  VC_HIP(d_k.alloc(std::max<size_t>(1, fk.size()) * sizeof(int32_t)));
  VC_HIP(d_c.alloc(std::max<size_t>(1, fc.size()) * sizeof(int32_t)));
  VC_HIP(d_f.alloc(std::max<size_t>(1, ff.size()) * sizeof(double)));
  VC_HIP(d_dC.alloc((size_t)nblocks * m * m * sizeof(double)));
  VC_HIP(hipMemcpy(d_bptr.p, bptr.data(), bptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (!fk.empty()) {
    VC_HIP(hipMemcpy(d_k.p, fk.data(), fk.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    VC_HIP(hipMemcpy(d_c.p, fc.data(), fc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    VC_HIP(hipMemcpy(d_f.p, ff.data(), ff.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  VC_HIP(launch_grad_eps(d_bptr.as<int32_t>(), d_k.as<int32_t>(), d_c.as<int32_t>(), d_f.as<double>(),
                         rho.as<double>(), p->s_x.as<double>(), N, m, nblocks, 4.0 * M_PI * kEps0 * p->dv,
                         d_dC.as<double>(), nullptr));
  VC_HIP(hipMemcpy(dC, d_dC.p, (size_t)nblocks * m * m * sizeof(double), hipMemcpyDeviceToHost));
  return VC_OK;
}

vc_status vc_charges_to_capacitance(vc_problem* p, const double* rho_dev, int32_t nrhs, double* C_dev, void* stream) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_setup first"); return VC_ERR_STATE; }
  if (!rho_dev || !C_dev || nrhs <= 0) { set_error("bad arguments"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(p->device));
  VC_HIP(launch_cap_reduce_n(rho_dev, npanels(p), p->m, nrhs, p->d_cond_panels.as<int32_t>(),
                             p->d_cond_ptr.as<int32_t>(), p->d_weight.as<double>(), 4.0 * M_PI * kEps0 * p->dv, C_dev,
                             (hipStream_t)stream));
  return VC_OK;
}

vc_status vc_charges_to_capacitance_adjoint(vc_problem* p, const double* gC_dev, int32_t nrhs, double* grho_dev,
                                            void* stream) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_setup first"); return VC_ERR_STATE; }
  if (!gC_dev || !grho_dev || nrhs <= 0) { set_error("bad arguments"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(p->device));
  VC_HIP(launch_cap_reduce_adj(gC_dev, npanels(p), nrhs, p->d_pcond.as<int32_t>(), p->d_weight.as<double>(),
                               4.0 * M_PI * kEps0 * p->dv, grho_dev, (hipStream_t)stream));
  return VC_OK;
}

vc_status vc_tucker_info(vc_problem* p, int32_t* npairs, int32_t ranks[45], double* stored_numbers,
                         double* full_numbers, double* rebuild_ms, int32_t* rebuilds) {
  VC_CHECK_PROBLEM(p);
  if (!npairs || !ranks || !stored_numbers || !full_numbers || !rebuild_ms || !rebuilds) {
    set_error("null argument");
    return VC_ERR_ARG;
  }
  for (auto& e : p->tk_pending) {
    VC_HIP(hipEventSynchronize(e.second));
    float t = 0.f;
    VC_HIP(hipEventElapsedTime(&t, e.first, e.second));
    p->tk_ms += t;
    p->tk_count += 1;
    p->ev_free.push_back(e.first);
    p->ev_free.push_back(e.second);
  }
  p->tk_pending.clear();
  *npairs = (int32_t)p->tk.size();
  for (int i = 0; i < 45; ++i) ranks[i] = 0;
  double st = 0.0, full = 0.0;
  const double D[3] = {(double)p->Hx, (double)p->Hy, (double)p->H};
  for (size_t q = 0; q < p->tk.size() && q < 15; ++q) {
    const auto& t = p->tk[q];
    for (int m = 0; m < 3; ++m) ranks[3 * q + m] = t.r[m];
    st += (double)t.r[0] * t.r[1] * t.r[2] + D[0] * t.r[0] + D[1] * t.r[1] + D[2] * t.r[2];
    full += D[0] * D[1] * D[2];
  }
  *stored_numbers = st;
  *full_numbers = full;
  *rebuild_ms = p->tk_ms;
  *rebuilds = p->tk_count;
  return VC_OK;
}

vc_status vc_profile_enable(vc_problem* p, int enable) {
  VC_CHECK_PROBLEM(p);
  p->prof = enable != 0;
  return VC_OK;
}

vc_status vc_pass_times(vc_problem* p, double ms[5], int32_t launches[5], double bytes[5]) {
  VC_CHECK_PROBLEM(p);
  if (!ms || !launches || !bytes) { set_error("null argument"); return VC_ERR_ARG; }
  for (int i = 0; i < 5; ++i) { ms[i] = 0.0; launches[i] = 0; bytes[i] = p->pass_bytes[i]; }
  for (auto& ev : p->ev_pending) {
    VC_HIP(hipEventSynchronize(ev[5]));
    for (int i = 0; i < 5; ++i) {
      float t = 0.f;
      VC_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms[i] += t;
      launches[i] += 1;
    }
    for (hipEvent_t e : ev) p->ev_free.push_back(e);
  }
  p->ev_pending.clear();
  return VC_OK;
}

vc_status vc_xpass_candidates(vc_problem* p, vc_precision prec, int transpose, int32_t* out, int32_t max_rows,
                              int32_t* n_rows) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_setup first"); return VC_ERR_STATE; }
  if (!n_rows || (max_rows > 0 && !out)) { set_error("null argument"); return VC_ERR_ARG; }
  if (prec != VC_FP64 && prec != VC_FP32) { set_error("prec must be VC_FP64 or VC_FP32"); return VC_ERR_ARG; }
  const int elem = prec == VC_FP32 ? 4 : 8;
  const int nin = (transpose && p->n_diel > 0) ? 6 : 3;
  const std::vector<vc::SandCfg> cand = vc::sandwich_candidates(p->M[0], elem, nin, p->n1[0], vc::kLdsBudget);
  *n_rows = (int32_t)cand.size();
  for (int32_t r = 0; r < (int32_t)cand.size() && r < max_rows; ++r) {
    int32_t* row = out + 8 * r;
    for (int k = 0; k < 8; ++k) row[k] = 0;
    row[0] = cand[r].nst;
    for (int s2 = 0; s2 < cand[r].nst; ++s2) row[1 + s2] = (int32_t)((cand[r].radpack >> (5 * s2)) & 31u);
    row[7] = 1 << cand[r].lgc;
  }
  return VC_OK;
}

vc_status vc_xpass_set(vc_problem* p, vc_precision prec, int transpose, int32_t nrhs, const int32_t cfg[8]) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_setup first"); return VC_ERR_STATE; }
  if (!cfg || nrhs <= 0 || nrhs > p->max_rhs) { set_error("bad cfg or nrhs"); return VC_ERR_ARG; }
  if (prec != VC_FP64 && prec != VC_FP32) { set_error("prec must be VC_FP64 or VC_FP32"); return VC_ERR_ARG; }
  const int elem = prec == VC_FP32 ? 4 : 8;
  const int nin = (transpose && p->n_diel > 0) ? 6 : 3;
  const std::vector<vc::SandCfg> cand = vc::sandwich_candidates(p->M[0], elem, nin, p->n1[0], vc::kLdsBudget);
  for (const vc::SandCfg& g : cand) {
    bool same = cfg[0] == g.nst && cfg[7] == (1 << g.lgc);
    for (int s2 = 0; s2 < 6 && same; ++s2)
      same = cfg[1 + s2] == (s2 < g.nst ? (int32_t)((g.radpack >> (5 * s2)) & 31u) : 0);
    if (!same) continue;
    const int t = (transpose && p->n_diel > 0) ? 1 : 0;   // without dielectric rows A is symmetric
    const int key = (nrhs << 2) | (t << 1) | (elem == 8 ? 1 : 0);
    p->sand_choice[key] = vc_problem::SandChoice{g.nst, g.tl, g.lgc, g.nthr, g.radpack, false, 0.0, 0.0};
    return VC_OK;
  }
  set_error("not an x-pass configuration of this problem (see vc_xpass_candidates)");
  return VC_ERR_ARG;
}

vc_status vc_tuning_report(vc_problem* p, char* buf, int32_t len) {
  VC_CHECK_PROBLEM(p);
  if (!buf || len <= 0) { set_error("null or empty buffer"); return VC_ERR_ARG; }
  std::string out;
  char line[256];
  for (const auto& kv : p->sand_choice) {
    const auto& c = kv.second;
    std::string rad;
    for (int s = 0; s < c.nst; ++s) {
      if (s) rad += "x";
      rad += std::to_string((int)((c.radpack >> (5 * s)) & 31u));
    }
    std::snprintf(line, sizeof line, "x-pass %s %s nrhs=%d radices=%s cols=%d threads=%d %s", (kv.first & 1) ? "fp64" : "fp32",
                  (kv.first & 2) ? "transpose" : "forward", kv.first >> 2, rad.c_str(), 1 << c.lgc, c.nthr,
                  c.tuned ? "tuned" : "default");
    out += line;
    if (c.tuned) {
      std::snprintf(line, sizeof line, " best_ms=%.4f default_ms=%.4f", c.ms_best, c.ms_default);
      out += line;
    }
    out += "\n";
  }
  std::snprintf(buf, (size_t)len, "%s", out.c_str());
  return VC_OK;
}

}  // extern "C"
