// GMRES driver of the solve: restarted, several right-hand sides in lock-step,
// right-preconditioned with eq. (14) (Sec. II.D); every step of a restart cycle runs on
// the device (capturable as a graph); FP32-product GMRES inside FP64 refinement.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "mvp_kernels.h"
#include "problem.h"
#include "solver.h"

namespace vc {

// Arnoldi steps per captured segment of a restart cycle: after each segment the host
// reads whether any column still iterates (one small read-back per segment).
constexpr int kCycleSeg = 8;
static int cycle_segments(int m) { return (m + kCycleSeg - 1) / kCycleSeg; }


double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------------------ GMRES

size_t solve_ws_layout(int64_t N, int k, int r, char* base, SolveWs* ws) {
  size_t off = 0;
  // next region of n elements of type T (256-byte aligned)
  auto take = [&](auto*& ptr, size_t n) {
    using T = std::remove_reference_t<decltype(*ptr)>;
    off = (off + 255) & ~(size_t)255;
    ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
  };
  SolveWs w{};
  const size_t kN = (size_t)k * (size_t)N;
  take(w.V, (size_t)(r + 1) * kN);
  for (double** v : {&w.w, &w.z, &w.r, &w.b, &w.x, &w.tmp, &w.rr, &w.dd}) take(*v, kN);
  take(w.h, (size_t)2 * (r + 2) * k);
  take(w.y2, (size_t)(r + 2) * k);
  take(w.partial, (size_t)std::max({gemv_t_partial_size(N, r + 2, k), colnorm_partial_size(N, k),
                                    cgs_partial_size(N, r + 1, k)}));
  take(w.norm, (size_t)4 * k);
  // device-side cycle state: H, cs, sn, g, bn, rn, rre, scal (doubles); kd, iters,
  // act_cycle, act_step (ints) + skip[2], bad
  take(w.cyc, (size_t)k * ((size_t)(r + 1) * r + 2 * r + (r + 1) + 4) + 1);
  take(w.dC, (size_t)k * k);
  take(w.rx, (size_t)k + 2);
  take(w.active, (size_t)k);
  take(w.cyci, (size_t)4 * k + 5);
  take(w.cnt, (size_t)cgs_counter_size(r + 1, k));
  w.nrhs = k;
  w.restart = r;
  if (ws) *ws = w;
  return (off + 255) & ~(size_t)255;
}

vc_status ensure_workspace(vc_problem* P, int nrhs, int restart) {
  if (P->ws.nrhs >= nrhs && P->ws.restart >= restart) return VC_OK;
  if (P->ws_static) {
    set_error("the static scratch holds a smaller solve than asked for");
    return VC_ERR_STATE;
  }
  const int64_t N = npanels(P);
  const int r = std::max(restart, P->ws.restart), k = std::max(nrhs, P->ws.nrhs);
  if (k > 256) { set_error("at most 256 right-hand sides per solve"); return VC_ERR_ARG; }
  P->drop_graphs();   // captured graphs hold pointers into the old workspace
  const size_t bytes = solve_ws_layout(N, k, r, nullptr, nullptr);
  VC_HIP(P->s_all.alloc(bytes));
  solve_ws_layout(N, k, r, P->s_all.as<char>(), &P->ws_own);
  // vectors start at zero (rows a product never writes, the padding rows of a packed
  // set, then stay zero through every update), and so do the counters
  VC_HIP(hipMemset(P->s_all.p, 0, bytes));
  P->ws = P->ws_own;
  return VC_OK;
}

Cyc cycle_views(vc_problem* P, int nrhs, int m) {
  Cyc c{};
  double* d = P->ws.cyc;
  c.H = d; d += (size_t)nrhs * (m + 1) * m;
  c.cs = d; d += (size_t)nrhs * m;
  c.sn = d; d += (size_t)nrhs * m;
  c.g = d; d += (size_t)nrhs * (m + 1);
  c.bn = d; d += nrhs;
  c.rn = d; d += nrhs;
  c.rre = d; d += nrhs;
  c.scal = d; d += nrhs;
  c.rtol = d;
  int* q = P->ws.cyci;
  c.kd = q; q += nrhs;
  c.iters = q; q += nrhs;
  c.act_cycle = q; q += nrhs;
  c.act_step = q; q += nrhs;
  c.skip = q; q += 3;   // [0] cycle-level, [1] step-level, [2] whole solve disabled (cleared per solve)
  c.bad = q;
  return c;
}

// z = R v (if preconditioned), w = A z; skipped entirely when *skip
// (act: optional per-column activity; the product skips inactive columns)
vc_status op_with_precond(vc_problem* P, const SolveSpec& sp, const double* v, double* z, double* w, int nrhs,
                          hipStream_t st, const int* skip, const int* act) {
  const double* src = v;
  if (sp.precond) {
    P->pc.mode = sp.precond;
    vc_status s = apply_precond(P, sp.transpose, v, z, nrhs, st, skip);
    if (s != VC_OK) return s;
    src = z;
  }
  return apply_op(P, sp.transpose, sp.mvp, src, w, nrhs, st, skip, act);
}

// r = b - A x
vc_status residual(vc_problem* P, const SolveSpec& sp, const double* b, const double* x, double* r, int nrhs,
                   hipStream_t st, const int* skip) {
  const int64_t N = npanels(P);
  vc_status s = apply_op(P, sp.transpose, sp.mvp, x, r, nrhs, st, skip);
  if (s != VC_OK) return s;
  VC_HIP(launch_axpy_cols(r, b, N, nrhs, nullptr, 1, st, skip));
  return VC_OK;
}

vc_status col_norms(vc_problem* P, const double* w, int64_t N, int nrhs, double* d_out, std::vector<double>& h,
                           hipStream_t st) {
  VC_HIP(launch_colnorm(w, N, N, nrhs, d_out, P->ws.partial, st));
  h.resize(nrhs);
  VC_HIP(hipMemcpyAsync(h.data(), d_out, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  VC_HIP(hipStreamSynchronize(st));
  return VC_OK;
}

// One GMRES(m) restart cycle, every step on the device (so it can be captured), in parts
// so that the last cycle of a solve (which only finds every column converged) costs one
// residual, and a cycle whose columns all converge early stops issuing steps:
//   part 0:            residual and its norms, cycle start (masks, g, skip flags),
//                      V_0 = r / |r|;
//   part -1:           the same for a zero x (r = b, no product: a solve's first cycle);
//   parts 1..nseg:     Arnoldi steps [kCycleSeg (part - 1), kCycleSeg part) with
//                      classical Gram-Schmidt applied twice and the Givens update;
//   part nseg + 1:     x += R V y for the columns that were active at the start.
// Columns freeze once converged; when all have, the remaining steps' kernels return at
// once (device flag), and the host, which reads that flag after each segment, issues no
// further segment.
vc_status issue_cycle(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs, hipStream_t st,
                      int part) {
  const int64_t N = npanels(P);
  const int m = sp.restart;
  const Cyc c = cycle_views(P, nrhs, m);
  double* V = P->ws.V;
  double* w = P->ws.w;
  double* z = P->ws.z;
  double* r = P->ws.r;
  double* hd = P->ws.h;
  double* y2 = P->ws.y2;
  double* nrm = P->ws.norm;
  const int64_t ldv = (int64_t)nrhs * N;
  const int ldh = m + 2;
  vc_status s;
  if (part == 0 || part == -1) {
    if (part == 0) {
      s = residual(P, sp, b, x, r, nrhs, st, c.skip + 2);
      if (s != VC_OK) return s;
    } else {
      VC_HIP(launch_zero(r, (int64_t)nrhs * N, st));
      VC_HIP(launch_axpy_cols(r, b, N, nrhs, nullptr, 1, st, c.skip + 2));   // r = b - 0
    }
    VC_HIP(launch_colnorm(r, N, N, nrhs, c.rn, P->ws.partial, st, c.skip + 2));
    VC_HIP(launch_cycle_start(nrhs, m, c.rn, c.bn, c.rtol, c.act_cycle, c.act_step, c.g, c.scal, c.kd, c.skip, c.rre,
                              st));
    VC_HIP(launch_scale_copy(V, r, N, nrhs, c.scal, c.skip, st));   // V_0 = r / |r|
    return VC_OK;
  }
  const int nseg = cycle_segments(m);
  if (part <= nseg) {
    const int j1 = std::min(m, part * kCycleSeg);
    for (int j = (part - 1) * kCycleSeg; j < j1; ++j) {
      s = op_with_precond(P, sp, V + j * ldv, z, w, nrhs, st, c.skip + 1, c.act_step);
      if (s != VC_OK) return s;
      // classical Gram-Schmidt twice, |w| and the Givens update (three launches)
      VC_HIP(launch_cgs_step(V, ldv, N, j + 1, w, nrhs, hd, hd + (size_t)ldh * nrhs, ldh, P->ws.partial,
                             P->ws.cnt, j, m, c.H, c.cs, c.sn, c.g, c.bn, c.rtol, c.act_step, c.kd,
                             c.iters, c.scal, c.skip, c.bad, nrm, st));
      if (j + 1 < m) VC_HIP(launch_scale_copy(V + (j + 1) * ldv, w, N, nrhs, c.scal, c.skip + 1, st));
    }
    if (sp.relax)
      VC_HIP(launch_relax_state(nrhs, m, c.g, c.kd, c.act_step, c.bn, c.iters, c.skip, P->ws.rx, st));
    return VC_OK;
  }
  // x += R V y, y = R_H^{-1} g over each column's steps
  VC_HIP(launch_backsolve(nrhs, m, c.H, c.g, c.kd, c.act_cycle, y2, ldh, st));
  VC_HIP(launch_zero(w, (int64_t)nrhs * N, st));
  VC_HIP(launch_gemv_n_sub(V, ldv, N, m, y2, ldh, w, N, nrhs, c.act_cycle, 0, st, c.kd));   // w = V y
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

// The captured part of a restart cycle for this solve shape (captured and
// instantiated on first use).  An eager product first settles the launch
// configurations (and runs the autotuner) outside the capture.
vc_status cycle_graph(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs, hipStream_t st,
                      int part, hipGraph_t* g_out, hipGraphExec_t* e_out) {
  vc_problem::GraphKey key{(int)sp.mvp, sp.transpose, sp.precond, nrhs, sp.restart, part, b, x, sp.relax};
  for (const auto& e : P->graphs)
    if (e.key == key) {
      *g_out = e.graph;
      *e_out = e.exec;
      return VC_OK;
    }
  if (part != -1) {   // (part -1 has no product)
    vc_status s = apply_op(P, sp.transpose, sp.mvp, b, P->ws.tmp, nrhs, st);
    if (s != VC_OK) return s;
  }
  VC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  vc_status sc = issue_cycle(P, sp, b, x, nrhs, st, part);
  hipGraph_t gr = nullptr;
  const hipError_t ee = hipStreamEndCapture(st, &gr);
  if (sc != VC_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return sc;
  }
  if (ee != hipSuccess) { set_error("graph capture failed: %s", hipGetErrorString(ee)); return VC_ERR_HIP; }
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(gr);
    set_error("graph instantiation failed: %s", hipGetErrorString(ei));
    return VC_ERR_HIP;
  }
  P->add_graph(key, gr, ex);
  *g_out = gr;
  *e_out = ex;
  return VC_OK;
}

static vc_status run_part(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs, hipStream_t st,
                          int part) {
  if (!P->use_graphs) return issue_cycle(P, sp, b, x, nrhs, st, part);
  hipGraph_t gr = nullptr;
  hipGraphExec_t ex = nullptr;
  vc_status s = cycle_graph(P, sp, b, x, nrhs, st, part, &gr, &ex);
  if (s != VC_OK) return s;
  VC_HIP(hipGraphLaunch(ex, st));
  return VC_OK;
}

// Solve A x = b (x holds the initial guess).  iters/rre: per column outputs.  With
// graphs on, every cycle replays one graph captured at the first solve of this shape
// (rtol is read from device memory, so solves to any tolerance share it); an eager
// product before the capture settles the autotuned launch configuration.
//
// Relaxed mixed form (sp.relax): each segment's products are FP32 when the largest
// residual estimate of an iterating column (read after the previous segment, or the
// true residual at the cycle start) is at most sp.relax_thr, FP64 otherwise; the cycle
// starts compute the true residual with FP64 products.  A cycle that starts in FP32
// and does not halve the largest true residual sends the rest of the solve to FP64.
// steps32: Arnoldi steps taken with FP32 products (largest over columns, per segment).
vc_status gmres(vc_problem* P, const SolveSpec& sp, const double* b, double* x, int nrhs,
                       std::vector<int>& iters, std::vector<double>& rre, hipStream_t st, int* steps32, bool x_zero) {
  const int64_t N = npanels(P);
  const int m = sp.restart;
  vc_status s = ensure_workspace(P, nrhs, m);
  if (s != VC_OK) return s;
  const Cyc c = cycle_views(P, nrhs, m);
  VC_HIP(hipMemcpyAsync(c.rtol, &sp.rtol, sizeof(double), hipMemcpyHostToDevice, st));
  VC_HIP(launch_colnorm(b, N, N, nrhs, c.bn, P->ws.partial, st));
  VC_HIP(hipMemsetAsync(c.iters, 0, (size_t)nrhs * sizeof(int), st));
  VC_HIP(hipMemsetAsync(c.bad, 0, sizeof(int), st));
  VC_HIP(hipMemsetAsync(c.skip + 2, 0, sizeof(int), st));
  std::vector<int> it(nrhs), skip(2);
  rre.assign(nrhs, 0.0);
  int bad = 0;
  const bool relax = sp.relax != 0;
  std::vector<double> rx(relax ? nrhs + 2 : 0);
  std::vector<int> it_seg(nrhs, 0);   // iteration counts before the current segment
  double est = INFINITY;              // worst residual estimate of an iterating column
  double start_prev = INFINITY;       // worst true residual at the previous cycle start
  bool force64 = false, start32 = false, seg32 = false;
  int n32 = 0;
  // FP32 steps of the segment just run: the largest per-column count increase
  auto count32 = [&](const int* now, bool was32) {
    int d = 0;
    for (int c = 0; c < nrhs; ++c) d = std::max(d, now[c] - it_seg[c]);
    if (was32) n32 += d;
    std::copy(now, now + nrhs, it_seg.begin());
  };
  std::vector<int> itv(nrhs);
  // start of the first cycle (x = 0 given: r = b without a product); each later round
  // runs the previous cycle's steps and the next cycle's start before one host read-back
  s = run_part(P, sp, b, x, nrhs, st, x_zero ? -1 : 0);
  if (s != VC_OK) return s;
  const int nseg = cycle_segments(m);
  for (int cycle = 0;; ++cycle) {
    if (cycle > 0) {
      // the steps segment by segment, until no column is still iterating
      for (int seg = 1; seg <= nseg; ++seg) {
        SolveSpec ss = sp;
        if (relax) {
          seg32 = !force64 && est <= sp.relax_thr;
          ss.mvp = seg32 ? VC_FP32 : VC_FP64;
          if (seg == 1) start32 = seg32;
        }
        s = run_part(P, ss, b, x, nrhs, st, seg);
        if (s != VC_OK) return s;
        if (seg == nseg) break;
        int step_done = 0;
        if (relax) {
          VC_HIP(hipMemcpyAsync(rx.data(), P->ws.rx, rx.size() * sizeof(double), hipMemcpyDeviceToHost, st));
          VC_HIP(hipStreamSynchronize(st));
          est = rx[0];
          step_done = rx[1] != 0.0;
          for (int k = 0; k < nrhs; ++k) itv[k] = (int)rx[2 + k];
          count32(itv.data(), seg32);
        } else {
          VC_HIP(hipMemcpyAsync(&step_done, c.skip + 1, sizeof(int), hipMemcpyDeviceToHost, st));
          VC_HIP(hipStreamSynchronize(st));
        }
        if (step_done) break;
      }
      s = run_part(P, sp, b, x, nrhs, st, nseg + 1);
      if (s != VC_OK) return s;
      s = run_part(P, sp, b, x, nrhs, st, 0);
      if (s != VC_OK) return s;
    }
    VC_HIP(hipMemcpyAsync(rre.data(), c.rre, (size_t)nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    VC_HIP(hipMemcpyAsync(it.data(), c.iters, (size_t)nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
    VC_HIP(hipMemcpyAsync(skip.data(), c.skip, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    VC_HIP(hipMemcpyAsync(&bad, c.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    VC_HIP(hipStreamSynchronize(st));
    iters = it;
    if (relax) {
      if (cycle > 0) count32(it.data(), seg32);   // the cycle's last segment
      // the next cycle's columns are those above rtol; their worst true residual
      double worst = 0.0;
      for (int k = 0; k < nrhs; ++k)
        if (rre[k] > sp.rtol) worst = std::max(worst, rre[k]);
      if (cycle > 0 && start32 && !(worst <= 0.5 * start_prev)) force64 = true;
      start_prev = worst;
      est = worst;
    }
    if (steps32) *steps32 = relax ? n32 : (sp.mvp == VC_FP32 ? *std::max_element(it.begin(), it.end()) : 0);
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
hipStream_t get_solve_stream(vc_problem* P) {
  if (!P->solve_stream && hipStreamCreate(&P->solve_stream) != hipSuccess) P->solve_stream = nullptr;
  return P->solve_stream;
}

// FP64 solve, or VC_MIXED: FP32-product GMRES inside FP64 refinement, or the relaxed
// form (one GMRES whose Arnoldi products turn FP32 as the residual shrinks).
vc_status solve(vc_problem* P, const vc_solve_opts& o, int transpose, const double* b, double* x, int nrhs,
                       vc_stats* stats, hipStream_t st, std::vector<int>* it_out, std::vector<double>* rre_out) {
  const int64_t N = npanels(P);
  SolveSpec sp{};
  sp.transpose = transpose;
  sp.precond = o.use_precond;
  sp.restart = o.restart;
  sp.max_iter = o.max_iter;
  std::vector<int> it;
  std::vector<double> rre;
  // a call without allocation (static scratch) issues every cycle eagerly on the
  // caller's stream: capturing and instantiating graphs, and creating a stream, allocate
  P->use_graphs = o.graph == 0 && !P->ws_static;
  if (!st && !P->ws_static) {
    st = get_solve_stream(P);
    if (!st) { set_error("could not create the solve stream"); return VC_ERR_HIP; }
  }
  if (o.use_precond < 0 || o.use_precond > 3) { set_error("use_precond must be 0, 1, 2 or 3"); return VC_ERR_ARG; }
  if (o.use_precond == 3) {
    if (P->ws_static) { set_error("use_precond 3 builds its blocks (allocates) on first use"); return VC_ERR_ARG; }
    if (P->pack) { set_error("packed sets use the block-diagonal-diagonal or diagonal preconditioner"); return VC_ERR_ARG; }
    // built on first use, before any restart cycle is captured
    const vc_status bs = build_precond_full(P, st);
    if (bs != VC_OK) return bs;
  }
  if (o.mixed_form < 0 || o.mixed_form > VC_MIXED_RELAXED) {
    set_error("mixed_form must be 0 (automatic), 1 (refinement) or 2 (relaxed)");
    return VC_ERR_ARG;
  }
  VC_HIP(hipMemsetAsync(x, 0, (size_t)nrhs * N * sizeof(double), st));
  int ir_steps = 0, n32 = 0, form = 0;
  vc_status s;
  if (o.prec == VC_MIXED) {
    form = o.mixed_form;
    if (form == 0) {
      // relaxed where FP64 products are small enough to be bound by latency and cache
      const double b64 = P->pack ? pack_product_bytes(P, 8) : product_bytes_model(P, 8, nrhs);
      form = b64 <= VC_MIXED_RELAXED_MAX_BYTES ? VC_MIXED_RELAXED : VC_MIXED_REFINEMENT;
    }
  }
  if (o.prec != VC_MIXED) {
    sp.mvp = o.prec == VC_FP32 ? VC_FP32 : VC_FP64;
    sp.rtol = o.rtol;
    s = gmres(P, sp, b, x, nrhs, it, rre, st, &n32, true);   // x was zeroed above
  } else if (form == VC_MIXED_RELAXED) {
    // one GMRES on the FP64 system: FP64 residuals at the restarts, FP32 Arnoldi
    // products once the residual estimate is below rtol / inner_rtol (an FP32 product's
    // relative error is taken as inner_rtol)
    sp.mvp = VC_FP64;
    sp.rtol = o.rtol;
    sp.relax = 1;
    sp.relax_thr = o.rtol / o.inner_rtol;
    s = gmres(P, sp, b, x, nrhs, it, rre, st, &n32, true);
  } else {
    // outer FP64 refinement: r = b - A x (FP64 product), inner FP32 GMRES on A d = r, x += d
    s = ensure_workspace(P, nrhs, o.restart);
    if (s != VC_OK) return s;
    double* rrp = P->ws.rr;   // stable buffers: the inner solves reuse their graph
    double* ddp = P->ws.dd;
    std::vector<int> tot(nrhs, 0);
    SolveSpec s64 = sp;
    s64.mvp = VC_FP64;
    std::vector<double> bn, rn, keep(nrhs), ones(nrhs, 1.0);
    s = col_norms(P, b, N, nrhs, P->ws.norm, bn, st);
    if (s != VC_OK) return s;
    VC_HIP(hipMemcpyAsync(rrp, b, (size_t)nrhs * N * sizeof(double), hipMemcpyDeviceToDevice, st));
    s = VC_ERR_NOT_CONVERGED;
    rre.assign(nrhs, 1.0);
    double worst = 1.0;   // largest relative residual of a column still above rtol
    for (ir_steps = 0; ir_steps < o.ir_max; ++ir_steps) {
      SolveSpec s32 = sp;
      s32.mvp = VC_FP32;
      // reduce the residual no further than this step needs (half of rtol / worst),
      // and no further than FP32 products can (inner_rtol)
      s32.rtol = std::max(o.inner_rtol, 0.5 * o.rtol / worst);
      s32.max_iter = std::min(o.max_iter, 4 * o.restart);
      VC_HIP(hipMemsetAsync(ddp, 0, (size_t)nrhs * N * sizeof(double), st));
      int k32 = 0;
      vc_status si = gmres(P, s32, rrp, ddp, nrhs, it, rre, st, &k32, true);   // ddp zeroed above
      if (si != VC_OK && si != VC_ERR_NOT_CONVERGED) return si;
      n32 += k32;
      for (int c = 0; c < nrhs; ++c) tot[c] += it[c];
      VC_HIP(hipMemcpyAsync(P->ws.norm + nrhs, ones.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
      VC_HIP(launch_axpy_cols(x, ddp, N, nrhs, P->ws.norm + nrhs, 0, st));
      vc_status sr = residual(P, s64, b, x, rrp, nrhs, st);
      if (sr != VC_OK) return sr;
      sr = col_norms(P, rrp, N, nrhs, P->ws.norm, rn, st);
      if (sr != VC_OK) return sr;
      bool ok = true;
      worst = 0.0;
      for (int c = 0; c < nrhs; ++c) {
        rre[c] = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
        keep[c] = rre[c] > o.rtol ? 1.0 : 0.0;
        if (rre[c] > o.rtol) ok = false;
        worst = std::max(worst, rre[c]);
      }
      if (ok) { s = VC_OK; ++ir_steps; break; }
      // columns already within rtol get a zero residual: the next inner solve leaves them
      VC_HIP(hipMemcpyAsync(P->ws.norm + 2 * nrhs, keep.data(), nrhs * sizeof(double),
                            hipMemcpyHostToDevice, st));
      VC_HIP(launch_scale_cols(rrp, N, N, nrhs, P->ws.norm + 2 * nrhs, 0, st));
    }
    it = tot;
    if (s != VC_OK) set_error("refinement did not reach rtol %.3g in %d steps", o.rtol, o.ir_max);
  }
  if (it_out) *it_out = it;
  if (rre_out) *rre_out = rre;
  if (stats) {
    for (int c = 0; c < nrhs && c < 64; ++c) {
      stats->iters[c] = c < (int)it.size() ? it[c] : 0;
      stats->final_rre[c] = c < (int)rre.size() ? rre[c] : 0.0;
    }
    stats->ir_steps = ir_steps;
    stats->mixed_form = form;
    stats->steps_fp32 = n32;
  }
  return s;
}

vc_solve_opts fill_defaults(const vc_solve_opts* in) {
  vc_solve_opts o{};
  if (in) o = *in;
  if (o.rtol <= 0) o.rtol = 1e-12;
  if (o.restart <= 0) o.restart = 35;
  if (o.max_iter <= 0) o.max_iter = 2000;
  if (o.inner_rtol <= 0) o.inner_rtol = 1e-6;
  if (o.ir_max <= 0) o.ir_max = 20;
  if (!in) o.use_precond = 1;
  return o;
}

}  // namespace vc
