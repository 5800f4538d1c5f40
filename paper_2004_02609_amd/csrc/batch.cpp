// Many independent problems of uneven size solved together (the batched form).
//
// Each problem keeps its own GMRES state on the device.  One graph holds the captured
// restart cycle of every problem as an independent branch (the branches share no
// data, so the runtime overlaps small problems the GPU would otherwise run mostly
// idle); it is instantiated once and launched once per round.  A problem that has
// finished is parked by its device flags: every kernel of its branch returns at
// entry.  Between rounds the host reads each problem's residuals and advances its
// state: converged, iteration cap, or (mixed precision) the FP64 refinement step
// r = b - A x that starts the next inner FP32 solve.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mvp_kernels.h"
#include "problem.h"
#include "solver.h"

namespace vc {

namespace {

struct Scene {
  vc_problem* P = nullptr;
  int m = 0;
  bool mixed = false;
  SolveSpec sp{};                  // the GMRES whose cycles the rounds replay
  const double* b = nullptr;       // its right-hand sides and unknowns
  double* x = nullptr;
  hipGraph_t g = nullptr;
  std::vector<double> bn_outer;    // mixed: |b| of the outer system
  std::vector<int> iters_total;
  std::vector<double> rre;
  int ir_steps = 0;
  bool done = false;
  vc_status status = VC_OK;
};

// start (or restart, for the next refinement step) the GMRES of scene s: cycle state
// reset and |b| on the device
vc_status begin_gmres(Scene& s, hipStream_t st) {
  vc_problem* P = s.P;
  const int64_t N = npanels(P);
  const Cyc c = cycle_views(P, s.m, s.sp.restart);
  VC_HIP(hipMemcpyAsync(c.rtol, &s.sp.rtol, sizeof(double), hipMemcpyHostToDevice, st));
  VC_HIP(launch_colnorm(s.b, N, N, s.m, c.bn, P->s_partial.as<double>(), st));
  VC_HIP(hipMemsetAsync(c.iters, 0, (size_t)s.m * sizeof(int), st));
  VC_HIP(hipMemsetAsync(c.bad, 0, sizeof(int), st));
  VC_HIP(hipMemsetAsync(c.skip + 2, 0, sizeof(int), st));   // enabled
  return VC_OK;
}

// park a finished problem: its branch of the round graph becomes a no-op
vc_status park(Scene& s, hipStream_t st) {
  static const int on[3] = {1, 1, 1};
  const Cyc c = cycle_views(s.P, s.m, s.sp.restart);
  VC_HIP(hipMemcpyAsync(c.skip, on, sizeof(on), hipMemcpyHostToDevice, st));
  VC_HIP(hipStreamSynchronize(st));   // `on` must not be read after this returns
  return VC_OK;
}

vc_status init_scene(Scene& s, const vc_solve_opts& o, hipStream_t st) {
  vc_problem* P = s.P;
  if (!P->setup_done) { set_error("batch: problem not set up"); return VC_ERR_STATE; }
  if (P->m > P->max_rhs) { set_error("batch: setup max_rhs < number of conductors"); return VC_ERR_STATE; }
  s.m = P->m;
  const int64_t N = npanels(P);
  vc_status r = ensure_workspace(P, s.m, o.restart);
  if (r != VC_OK) return r;
  P->use_graphs = true;
  std::vector<double> B((size_t)s.m * N, 0.0);
  for (int64_t k = 0; k < N; ++k)
    if (P->panels[k].kind == 0) B[(size_t)P->panels[k].cond * N + k] = 1.0;
  VC_HIP(hipMemcpyAsync(P->s_b.p, B.data(), B.size() * sizeof(double), hipMemcpyHostToDevice, st));
  VC_HIP(hipMemsetAsync(P->s_x.p, 0, (size_t)s.m * N * sizeof(double), st));
  s.sp.transpose = 0;
  s.sp.precond = o.use_precond;
  s.sp.restart = o.restart;
  s.sp.max_iter = o.max_iter;
  s.mixed = o.prec == VC_MIXED;
  s.iters_total.assign(s.m, 0);
  s.rre.assign(s.m, 1.0);
  if (!s.mixed) {
    s.sp.mvp = o.prec == VC_FP32 ? VC_FP32 : VC_FP64;
    s.sp.rtol = o.rtol;
    s.b = P->s_b.as<double>();
    s.x = P->s_x.as<double>();
  } else {
    // outer FP64 refinement on b; the inner FP32 GMRES solves A d = r
    s.sp.mvp = VC_FP32;
    s.sp.rtol = o.inner_rtol;
    VC_HIP(hipMemcpyAsync(P->s_rr.p, P->s_b.p, (size_t)s.m * N * sizeof(double), hipMemcpyDeviceToDevice, st));
    VC_HIP(hipMemsetAsync(P->s_dd.p, 0, (size_t)s.m * N * sizeof(double), st));
    r = col_norms(P, P->s_b.as<double>(), N, s.m, P->s_norm.as<double>(), s.bn_outer, st);
    if (r != VC_OK) return r;
    s.b = P->s_rr.as<double>();
    s.x = P->s_dd.as<double>();
  }
  hipGraphExec_t ex = nullptr;
  r = cycle_graph(P, s.sp, s.b, s.x, s.m, st, &s.g, &ex);
  if (r != VC_OK) return r;
  return begin_gmres(s, st);
}

// after an inner FP32 solve converged: x += d, r = b - A x in FP64, outer check, and
// (if not done) restart the inner solve on the new residual
vc_status refine_step(Scene& s, const vc_solve_opts& o, hipStream_t st) {
  vc_problem* P = s.P;
  const int64_t N = npanels(P);
  std::vector<double> ones(s.m, 1.0), rn;
  VC_HIP(hipMemcpyAsync(P->s_norm.as<double>() + s.m, ones.data(), s.m * sizeof(double), hipMemcpyHostToDevice, st));
  VC_HIP(launch_axpy_cols(P->s_x.as<double>(), P->s_dd.as<double>(), N, s.m, P->s_norm.as<double>() + s.m, 0, st));
  SolveSpec s64 = s.sp;
  s64.mvp = VC_FP64;
  vc_status r = residual(P, s64, P->s_b.as<double>(), P->s_x.as<double>(), P->s_rr.as<double>(), s.m, st);
  if (r != VC_OK) return r;
  r = col_norms(P, P->s_rr.as<double>(), N, s.m, P->s_norm.as<double>(), rn, st);
  if (r != VC_OK) return r;
  ++s.ir_steps;
  bool ok = true;
  for (int c = 0; c < s.m; ++c) {
    s.rre[c] = s.bn_outer[c] > 0 ? rn[c] / s.bn_outer[c] : 0.0;
    if (!(s.rre[c] <= o.rtol)) ok = false;
  }
  if (ok) {
    s.done = true;
    return VC_OK;
  }
  if (s.ir_steps >= o.ir_max) {
    set_error("refinement did not reach rtol %.3g in %d steps", o.rtol, o.ir_max);
    s.done = true;
    return VC_ERR_NOT_CONVERGED;
  }
  VC_HIP(hipMemsetAsync(P->s_dd.p, 0, (size_t)s.m * N * sizeof(double), st));
  return begin_gmres(s, st);
}

}  // namespace

vc_status batch_capacitance(vc_problem* const* problems, int n, const vc_solve_opts* opts, double* const* C_out,
                            vc_stats* stats) {
  const vc_solve_opts o = fill_defaults(opts);
  if (n <= 0 || !problems || !C_out) { set_error("batch: bad arguments"); return VC_ERR_ARG; }
  for (int k = 0; k < n; ++k) {
    if (!problems[k] || !C_out[k]) { set_error("batch: null problem or output %d", k); return VC_ERR_ARG; }
    if (problems[k]->device != problems[0]->device) { set_error("batch: problems on different devices"); return VC_ERR_ARG; }
    if (problems[k]->hip_failed) { set_error("batch: problem %d unusable after a HIP error", k); return VC_ERR_HIP; }
    for (int j = 0; j < k; ++j)
      if (problems[j] == problems[k]) { set_error("batch: problem %d listed twice", k); return VC_ERR_ARG; }
  }
  if ((o.prec == VC_FP32 || o.prec == VC_MIXED))
    for (int k = 0; k < n; ++k)
      if (!problems[k]->have32) { set_error("batch: FP32 spectra not built for problem %d", k); return VC_ERR_STATE; }
  VC_HIP(hipSetDevice(problems[0]->device));
  const double t0 = now_s();
  hipStream_t st = get_solve_stream(problems[0]);
  if (!st) { set_error("could not create the solve stream"); return VC_ERR_HIP; }
  std::vector<Scene> sc(n);
  for (int k = 0; k < n; ++k) {
    sc[k].P = problems[k];
    problems[k]->mvp_count = 0;
    vc_status r = init_scene(sc[k], o, st);
    if (r != VC_OK) return r;
  }
  // the round graph: every problem's restart cycle as an independent branch
  hipGraph_t rg = nullptr;
  hipGraphExec_t re = nullptr;
  VC_HIP(hipGraphCreate(&rg, 0));
  for (int k = 0; k < n; ++k) {
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddChildGraphNode(&node, rg, nullptr, 0, sc[k].g);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(rg);
      set_error("batch: adding problem %d to the round graph failed: %s", k, hipGetErrorString(e));
      return VC_ERR_HIP;
    }
  }
  {
    const hipError_t e = hipGraphInstantiate(&re, rg, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(rg);
      set_error("batch: round graph instantiation failed: %s", hipGetErrorString(e));
      return VC_ERR_HIP;
    }
  }
  vc_status first_err = VC_OK;
  struct Readback {
    std::vector<double> rre;
    std::vector<int> it;
    int skip[2];
    int bad;
  };
  std::vector<Readback> rb(n);
  vc_status loop_err = VC_OK;
  for (int round = 0;; ++round) {
    std::vector<int> act;
    for (int k = 0; k < n; ++k)
      if (!sc[k].done) act.push_back(k);
    if (act.empty()) break;
    const hipError_t le = hipGraphLaunch(re, st);
    if (le != hipSuccess) {
      set_error("batch: round graph launch failed: %s", hipGetErrorString(le));
      loop_err = VC_ERR_HIP;
      break;
    }
    for (int k : act) {
      Scene& s = sc[k];
      const Cyc c = cycle_views(s.P, s.m, s.sp.restart);
      rb[k].rre.resize(s.m);
      rb[k].it.resize(s.m);
      VC_HIP(hipMemcpyAsync(rb[k].rre.data(), c.rre, (size_t)s.m * sizeof(double), hipMemcpyDeviceToHost, st));
      VC_HIP(hipMemcpyAsync(rb[k].it.data(), c.iters, (size_t)s.m * sizeof(int), hipMemcpyDeviceToHost, st));
      VC_HIP(hipMemcpyAsync(rb[k].skip, c.skip, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      VC_HIP(hipMemcpyAsync(&rb[k].bad, c.bad, sizeof(int), hipMemcpyDeviceToHost, st));
    }
    VC_HIP(hipStreamSynchronize(st));
    for (int k : act) {
      Scene& s = sc[k];
      bool finite = true;
      for (double v : rb[k].rre) finite = finite && std::isfinite(v);
      if (!finite || rb[k].bad) {
        set_error("batch: non-finite residual in problem %d", k);
        s.status = VC_ERR_NUMERIC;
        s.done = true;
        continue;
      }
      if (rb[k].skip[0]) {   // this GMRES met its tolerance at the start of the cycle
        for (int c = 0; c < s.m; ++c) s.iters_total[c] += rb[k].it[c];
        if (!s.mixed) {
          s.rre = rb[k].rre;
          s.done = true;
        } else {
          const vc_status r = refine_step(s, o, st);
          if (r != VC_OK) s.status = r;
        }
        continue;
      }
      const int total = *std::max_element(rb[k].it.begin(), rb[k].it.end());
      if (total >= s.sp.max_iter) {
        set_error("batch: GMRES of problem %d did not reach rtol %.3g in %d iterations", k, s.sp.rtol, total);
        for (int c = 0; c < s.m; ++c) s.iters_total[c] += rb[k].it[c];
        s.rre = rb[k].rre;
        s.status = VC_ERR_NOT_CONVERGED;
        s.done = true;
      }
    }
    for (int k : act)
      if (sc[k].done) {
        const vc_status r = park(sc[k], st);
        if (r != VC_OK) { loop_err = r; break; }
      }
    if (loop_err != VC_OK) break;
  }
  (void)hipGraphExecDestroy(re);
  (void)hipGraphDestroy(rg);
  if (loop_err != VC_OK) return loop_err;
  // C of eq. (8) for every problem
  for (int k = 0; k < n; ++k) {
    Scene& s = sc[k];
    vc_problem* P = s.P;
    const int64_t N = npanels(P);
    DevMem dC;
    VC_HIP(dC.alloc((size_t)s.m * s.m * sizeof(double)));
    VC_HIP(launch_cap_reduce(P->s_x.as<double>(), N, s.m, P->d_cond_panels.as<int32_t>(), P->d_cond_ptr.as<int32_t>(),
                             P->d_weight.as<double>(), 4.0 * M_PI * kEps0 * P->dv, dC.as<double>(), st));
    VC_HIP(hipMemcpyAsync(C_out[k], dC.p, (size_t)s.m * s.m * sizeof(double), hipMemcpyDeviceToHost, st));
    VC_HIP(hipStreamSynchronize(st));
    if (stats) {
      vc_stats& t = stats[k];
      std::memset(&t, 0, sizeof(vc_stats));
      for (int c = 0; c < s.m && c < 64; ++c) {
        t.iters[c] = s.iters_total[c];
        t.final_rre[c] = s.rre[c];
      }
      t.ir_steps = s.ir_steps;
      t.mvp_count = P->mvp_count;
      t.t_setup_s = P->t_setup;
      t.t_solve_s = now_s() - t0;
      t.spectra_bytes = P->spectra_bytes;
    }
    if (s.status != VC_OK && first_err == VC_OK) first_err = s.status;
  }
  return first_err;
}

}  // namespace vc
