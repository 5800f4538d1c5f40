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
#include "solver.h"

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
  note_device_lds(p->device);
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
  p->y_choice.clear();
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
  p->tune_cache = o.tune_cache ? o.tune_cache : "";
  if (!p->tune_cache.empty()) {
    int32_t nl = 0;
    s = vc_tuning_load(p, p->tune_cache.c_str(), &nl);
    if (s != VC_OK) return s;
  }
  return VC_OK;
}

vc_status vc_setup_time(const vc_problem* p, double* total_s, double* toeplitz_s) {
  if (!p) { set_error("null problem"); return VC_ERR_ARG; }
  if (!p->setup_done) { set_error("vc_setup has not run"); return VC_ERR_STATE; }
  if (total_s) *total_s = p->t_setup;
  if (toeplitz_s) *toeplitz_s = p->t_toeplitz;
  return VC_OK;
}

vc_status vc_memory_info(const vc_problem* p, double* spectra_bytes, double* work_bytes) {
  if (!p) { set_error("null problem"); return VC_ERR_ARG; }
  if (!p->setup_done) { set_error("vc_setup has not run"); return VC_ERR_STATE; }
  if (spectra_bytes) *spectra_bytes = p->spectra_bytes;
  if (work_bytes) *work_bytes = (double)(p->work_F.bytes + p->work_O.bytes + p->s_all.bytes);
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
  if (!x || !y || x == y || nrhs <= 0 || nrhs > p->max_rhs) {
    set_error("bad x/y (null or the same array) or nrhs (1..%d)", p->max_rhs);
    return VC_ERR_ARG;
  }
  VC_HIP(hipSetDevice(p->device));
  p->pc.mode = 1;
  return mark(p, apply_precond(p, transpose, x, y, nrhs, (hipStream_t)stream));
}

vc_status vc_apply_precond_kind(vc_problem* p, int32_t kind, int transpose, const double* x, double* y, int32_t nrhs,
                                void* stream) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_apply_precond_kind before vc_setup"); return VC_ERR_STATE; }
  if (!x || !y || x == y || nrhs <= 0 || nrhs > p->max_rhs) {
    set_error("bad x/y (null or the same array) or nrhs (1..%d)", p->max_rhs);
    return VC_ERR_ARG;
  }
  if (kind < 1 || kind > 3) { set_error("preconditioner kind must be 1, 2 or 3"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(p->device));
  if (kind == 3) {
    if (p->pack) { set_error("packed sets use the block-diagonal-diagonal or diagonal preconditioner"); return VC_ERR_ARG; }
    const vc_status s = build_precond_full(p, (hipStream_t)stream);
    if (s != VC_OK) return mark(p, s);
  }
  p->pc.mode = kind;
  return mark(p, apply_precond(p, transpose, x, y, nrhs, (hipStream_t)stream));
}

vc_status vc_precond_info(vc_problem* p, int32_t kind, int64_t* nbox, int64_t* nblock, int64_t* bytes) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done || p->pack) { set_error("vc_precond_info needs a set-up single problem"); return VC_ERR_STATE; }
  if (kind != 1 && kind != 3) { set_error("preconditioner kind must be 1 or 3"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(p->device));
  const int64_t N = npanels(p);
  if (kind == 1) {
    const Precond& pc = p->pc;
    if (nbox) *nbox = pc.nbox;
    if (nblock) *nblock = pc.nblock;
    // distinct inverses, box panel lists and pointers, block table, dielectric diagonal
    if (bytes)
      *bytes = pc.block_doubles * 8 + (int64_t)pc.h_box_panels.size() * 4 + (int64_t)(pc.nbox + 1) * 4 +
               (int64_t)pc.nbox * 4 + (int64_t)pc.nblock * 12 + N * 8;
    return VC_OK;
  }
  const vc_status s = build_precond_full(p, nullptr);
  if (s != VC_OK) return mark(p, s);
  const FullBlocks& fb = p->pc.full;
  if (nbox) *nbox = fb.nbox;
  if (nblock) *nblock = fb.nblock;
  if (bytes)
    *bytes = fb.block_doubles * 8 + N * 4 + (int64_t)(fb.nbox + 1) * 4 + (int64_t)fb.nbox * 4 + (int64_t)fb.nblock * 12;
  return VC_OK;
}

}  // extern "C"

vc_status vc::capacitance_check(vc_problem* p, const vc_solve_opts* opts, const double* C, vc_solve_opts* o) {
  if (!p->setup_done) { set_error("vc_capacitance before vc_setup"); return VC_ERR_STATE; }
  if (!C) { set_error("null C"); return VC_ERR_ARG; }
  *o = fill_defaults(opts);
  if ((o->prec == VC_FP32 || o->prec == VC_MIXED) && !p->have32) { set_error("FP32 spectra not built"); return VC_ERR_STATE; }
  if (p->m > p->max_rhs) { set_error("setup max_rhs < number of conductors"); return VC_ERR_STATE; }
  return VC_OK;
}

vc_status vc::capacitance_run(vc_problem* p, const vc_solve_opts& o, double* C, double* rho_dev, vc_stats* stats,
                          hipStream_t st, std::vector<double>* rho_host, double t0) {
  const int64_t N = npanels(p);
  const int m = p->m;
  p->mvp_count = 0;
  // unit potential on conductor j: b[j N + k] = 1 on the panels of conductor j (Sec. II.A)
  VC_HIP(launch_unit_rhs(p->ws.b, p->d_pcond.as<int32_t>(), N, m, st));
  if (stats) std::memset(stats, 0, sizeof(vc_stats));
  vc_status s = solve(p, o, 0, p->ws.b, p->ws.x, m, stats, st);
  if (s != VC_OK && s != VC_ERR_NOT_CONVERGED) return s;
  VC_HIP(launch_cap_reduce(p->ws.x, N, m, p->d_cond_panels.as<int32_t>(), p->d_cond_ptr.as<int32_t>(),
                           p->d_weight.as<double>(), 4.0 * M_PI * kEps0 * p->dv, p->ws.dC, st));
  VC_HIP(hipMemcpyAsync(C, p->ws.dC, (size_t)m * m * sizeof(double), hipMemcpyDeviceToHost, st));
  if (rho_dev) VC_HIP(hipMemcpyAsync(rho_dev, p->ws.x, (size_t)m * N * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (rho_host) {
    rho_host->resize((size_t)m * N);
    VC_HIP(hipMemcpyAsync(rho_host->data(), p->ws.x, (size_t)m * N * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  VC_HIP(hipStreamSynchronize(st));
  if (stats) {
    stats->mvp_count = p->mvp_count;
    stats->t_setup_s = p->t_setup;
    stats->t_solve_s = now_s() - t0;
    stats->spectra_bytes = p->spectra_bytes;
    int rmax = 0;
    for (const auto& t : p->tk) rmax = std::max(rmax, std::max(t.r[0], std::max(t.r[1], t.r[2])));
    stats->tucker_rank_max = rmax;
    stats->bytes_model = product_bytes_model(p, o.prec == VC_FP64 ? 8 : 4, m);
  }
  return s;
}

extern "C" {

static vc_status capacitance_impl(vc_problem* p, const vc_solve_opts* opts, double* C, double* rho_dev, vc_stats* stats,
                                  std::vector<double>* rho_host) {
  VC_CHECK_PROBLEM(p);
  vc_solve_opts o;
  vc_status s = capacitance_check(p, opts, C, &o);
  if (s != VC_OK) return s;
  VC_HIP(hipSetDevice(p->device));
  const double t0 = now_s();
  hipStream_t st = get_solve_stream(p);
  if (!st) { set_error("could not create the solve stream"); return VC_ERR_HIP; }
  s = ensure_workspace(p, p->m, o.restart);
  if (s != VC_OK) return mark(p, s);
  s = capacitance_run(p, o, C, rho_dev, stats, st, rho_host, t0);
  return s == VC_OK || s == VC_ERR_NOT_CONVERGED ? s : mark(p, s);
}

vc_status vc_pack_create(vc_problem* const* problems, int32_t n, vc_pack** out) {
  if (!out) { set_error("null output"); return VC_ERR_ARG; }
  *out = nullptr;
  vc_problem* q = nullptr;
  const vc_status s = pack_create(problems, n, &q);
  if (s != VC_OK) return s;
  *out = reinterpret_cast<vc_pack*>(q);
  return VC_OK;
}

vc_status vc_pack_destroy(vc_pack* pk) {
  delete reinterpret_cast<vc_problem*>(pk);
  return VC_OK;
}

vc_status vc_pack_info(const vc_pack* pk, int32_t out[6]) {
  if (!pk || !out) { set_error("null argument"); return VC_ERR_ARG; }
  pack_info(reinterpret_cast<const vc_problem*>(pk), out);
  return VC_OK;
}

vc_status vc_pack_apply(vc_pack* pk, vc_precision prec, const double* x, double* y, void* stream) {
  vc_problem* q = reinterpret_cast<vc_problem*>(pk);
  VC_CHECK_PROBLEM(q);
  if (!q->pack) { set_error("not a packed set"); return VC_ERR_ARG; }
  if (!x || !y) { set_error("null x/y"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(q->device));
  return mark(q, apply_op(q, 0, prec, x, y, q->m, (hipStream_t)stream));
}

vc_status vc_pack_capacitance(vc_pack* pk, const vc_solve_opts* opts, double* const* C_out, vc_stats* stats) {
  vc_problem* q = reinterpret_cast<vc_problem*>(pk);
  VC_CHECK_PROBLEM(q);
  if (!q->pack) { set_error("not a packed set"); return VC_ERR_ARG; }
  return mark(q, pack_capacitance(q, opts, C_out, stats));
}

vc_status vc_capacitance_batch(vc_problem* const* problems, int32_t n, const vc_solve_opts* opts, double* const* C_out,
                               vc_stats* stats) {
  vc_pack* pk = nullptr;
  vc_status s = vc_pack_create(problems, n, &pk);
  if (s != VC_OK) return s;
  s = vc_pack_capacitance(pk, opts, C_out, stats);
  vc_pack_destroy(pk);
  return s;
}

vc_status vc_batch_capacitance(vc_problem* const* problems, int32_t n, const vc_solve_opts* opts, double* const* C_out,
                               vc_stats* stats) {
  return vc_capacitance_batch(problems, n, opts, C_out, stats);
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
  VC_HIP(hipMemcpy(rho.p, p->ws.x, (size_t)m * N * sizeof(double), hipMemcpyDeviceToDevice));
  // adjoint solves A^T lambda_i = w_i, w_i = eps_adj on the panels of conductor i
  vc_solve_opts o = fill_defaults(opts);
  std::vector<double> W((size_t)m * N, 0.0);
  for (int64_t k = 0; k < N; ++k)
    if (p->panels[k].kind == 0) W[(size_t)p->panels[k].cond * N + k] = p->panels[k].eps_adj;
  VC_HIP(hipMemcpy(p->ws.b, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice));
  s = solve(p, o, 1, p->ws.b, p->ws.x, m, nullptr, get_solve_stream(p));
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
                         rho.as<double>(), p->ws.x, N, m, nblocks, 4.0 * M_PI * kEps0 * p->dv,
                         d_dC.as<double>(), nullptr));
  VC_HIP(hipMemcpy(dC, d_dC.p, (size_t)nblocks * m * m * sizeof(double), hipMemcpyDeviceToHost));
  return VC_OK;
}

vc_status vc_update_eps(vc_problem* p, const double* eps_r, double eps_background, void* stream) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_update_eps before vc_setup"); return VC_ERR_STATE; }
  if (p->pack) { set_error("vc_update_eps on a packed set"); return VC_ERR_ARG; }
  if (!eps_r) { set_error("null eps_r"); return VC_ERR_ARG; }
  // the panel list of the new permittivities (host only), compared with the current one
  vc_problem q;
  q.nx = p->nx; q.ny = p->ny; q.nz = p->nz;
  q.dv = p->dv;
  q.eps_b = eps_background;
  q.cond_id = p->cond_id;
  q.eps_r.assign(eps_r, eps_r + p->cond_id.size());
  const vc_status s = panelize(&q);
  if (s != VC_OK) return s;
  bool same = q.panels.size() == p->panels.size();
  for (size_t k = 0; same && k < q.panels.size(); ++k) {
    const vc_panel &a = q.panels[k], &b = p->panels[k];
    same = a.i == b.i && a.j == b.j && a.k == b.k && a.dir == b.dir && a.kind == b.kind && a.cond == b.cond;
  }
  if (!same) {
    set_error("the new permittivities change the panel list (a dielectric face appears or vanishes): "
              "create a new problem");
    return VC_ERR_ARG;
  }
  VC_HIP(hipSetDevice(p->device));
  hipStream_t st = (hipStream_t)stream;
  // finish any work that still reads the current arrays, then rewrite them in place (the
  // allocations stay, so captured graphs keep pointing at valid, updated data)
  VC_HIP(hipStreamSynchronize(st));
  const int64_t N = (int64_t)p->panels.size();
  p->eps_r.swap(q.eps_r);
  p->eps_b = eps_background;
  p->panels.swap(q.panels);
  p->diag.swap(q.diag);
  p->weight.swap(q.weight);
  std::vector<double> dinv(N, 0.0), dinv_diag(N, 0.0);
  for (int64_t k = 0; k < N; ++k) {
    if (p->panels[k].kind == 1) dinv[k] = dinv_diag[k] = 1.0 / p->diag[k];
    else dinv_diag[k] = 1.0 / p->pc.pself;
  }
  const size_t nb = (size_t)N * sizeof(double);
  VC_HIP(hipMemcpyAsync(p->d_diag.p, p->diag.data(), nb, hipMemcpyHostToDevice, st));
  VC_HIP(hipMemcpyAsync(p->d_weight.p, p->weight.data(), nb, hipMemcpyHostToDevice, st));
  VC_HIP(hipMemcpyAsync(p->pc.dinv.p, dinv.data(), nb, hipMemcpyHostToDevice, st));
  VC_HIP(hipMemcpyAsync(p->pc.dinv_diag.p, dinv_diag.data(), nb, hipMemcpyHostToDevice, st));
  VC_HIP(hipStreamSynchronize(st));
  // the comparison preconditioner's blocks hold the eq. (7) diagonal: rebuilt at next use
  // (graphs captured with it point at its blocks, so they go too)
  if (p->pc.full.built) {
    p->drop_graphs();
    p->pc.full = FullBlocks();
    if (p->pc.mode == 3) p->pc.mode = 1;
  }
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
  if (enable < 0 || enable > 2) { set_error("profiling level must be 0, 1 or 2"); return VC_ERR_ARG; }
  p->prof = enable;
  return VC_OK;
}

vc_status vc_pass_times(vc_problem* p, double ms[5], int32_t launches[5], double bytes[5]) {
  VC_CHECK_PROBLEM(p);
  if (!ms || !launches || !bytes) { set_error("null argument"); return VC_ERR_ARG; }
  for (int i = 0; i < 5; ++i) { ms[i] = 0.0; launches[i] = 0; bytes[i] = p->pass_bytes[i]; }
  for (auto& ev : p->ev_pending) {
    for (int i = 5; i >= 0; --i)
      if (ev[i]) { VC_HIP(hipEventSynchronize(ev[i])); break; }
    for (int i = 0; i < 5; ++i) {
      if (!ev[i] || !ev[i + 1]) continue;   // pass not bracketed at this profiling level
      float t = 0.f;
      VC_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms[i] += t;
      launches[i] += 1;
    }
    for (hipEvent_t e : ev)
      if (e) p->ev_free.push_back(e);
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
  const std::vector<vc::SandCfg> cand = vc::xpass_candidate_list(p, elem, nin);
  *n_rows = (int32_t)cand.size();
  for (int32_t r = 0; r < (int32_t)cand.size() && r < max_rows; ++r) {
    int32_t* row = out + 8 * r;
    for (int k = 0; k < 8; ++k) row[k] = 0;
    row[0] = cand[r].nst;
    for (int s2 = 0; s2 < cand[r].nst; ++s2) row[1 + s2] = (int32_t)((cand[r].radpack >> (5 * s2)) & 31u);
    row[7] = cand[r].stage ? -cand[r].ncol : cand[r].ncol;   // negative: the staged form
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
  const std::vector<vc::SandCfg> cand = vc::xpass_candidate_list(p, elem, nin);
  for (const vc::SandCfg& g : cand) {
    bool same = cfg[0] == g.nst && cfg[7] == (g.stage ? -g.ncol : g.ncol);
    for (int s2 = 0; s2 < 6 && same; ++s2)
      same = cfg[1 + s2] == (s2 < g.nst ? (int32_t)((g.radpack >> (5 * s2)) & 31u) : 0);
    if (!same) continue;
    const int t = (transpose && p->n_diel > 0) ? 1 : 0;   // without dielectric rows A is symmetric
    const int key = (nrhs << 2) | (t << 1) | (elem == 8 ? 1 : 0);
    p->sand_choice[key] = vc_problem::SandChoice{g.nst, g.tl, g.ncol, g.nthr, g.radpack, false, 0.0, 0.0};
    p->sand_choice[key].stage = g.stage;
    return VC_OK;
  }
  set_error("not an x-pass configuration of this problem (see vc_xpass_candidates)");
  return VC_ERR_ARG;
}

vc_status vc_ypass_set(vc_problem* p, vc_precision prec, int transpose, int inverse, int32_t nrhs, int32_t kernel,
                       int32_t cols, int32_t xcd_group) {
  VC_CHECK_PROBLEM(p);
  if (!p->setup_done) { set_error("vc_setup first"); return VC_ERR_STATE; }
  if (nrhs <= 0 || nrhs > p->max_rhs) { set_error("nrhs outside 1..max_rhs"); return VC_ERR_ARG; }
  if (prec != VC_FP64 && prec != VC_FP32) { set_error("prec must be VC_FP64 or VC_FP32"); return VC_ERR_ARG; }
  if (kernel != 0 && kernel != 1) { set_error("kernel must be 0 (LDS tiles) or 1 (register edge)"); return VC_ERR_ARG; }
  if (cols < 0 || cols > 32 || (cols & (cols - 1))) { set_error("cols must be 0 or a power of two <= 32"); return VC_ERR_ARG; }
  if (xcd_group != 1 && xcd_group != 2 && xcd_group != 4 && xcd_group != -1) {
    set_error("xcd_group must be 1, 2, 4 or -1 (every tile of a row)");
    return VC_ERR_ARG;
  }
  const int t = (transpose && p->n_diel > 0) ? 1 : 0;   // without dielectric rows A is symmetric
  const int key = (nrhs << 3) | (t << 2) | ((inverse ? 1 : 0) << 1) | (prec == VC_FP64 ? 1 : 0);
  p->y_choice[key] = vc_problem::YChoice{kernel, false, {0.0, 0.0}, cols, xcd_group};
  return VC_OK;
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
    std::snprintf(line, sizeof line, "x-pass %s %s nrhs=%d radices=%s cols=%d threads=%d%s %s", (kv.first & 1) ? "fp64" : "fp32",
                  (kv.first & 2) ? "transpose" : "forward", kv.first >> 2, rad.c_str(), c.ncol, c.nthr,
                  c.stage ? " staged" : "", c.from_file ? "cached" : (c.tuned ? "tuned" : "default"));
    out += line;
    if (c.tuned) {
      std::snprintf(line, sizeof line, " best_ms=%.4f default_ms=%.4f", c.ms_best, c.ms_default);
      out += line;
    }
    out += "\n";
  }
  for (const auto& kv : p->y_choice) {
    const auto& c = kv.second;
    std::snprintf(line, sizeof line, "y-pass %s %s%s nrhs=%d kernel=%s%s %s", (kv.first & 1) ? "fp64" : "fp32",
                  (kv.first & 2) ? "inverse" : "forward", (kv.first & 4) ? " (transposed product)" : "",
                  kv.first >> 3, c.impl ? "register-edge" : "lds-tiles",
                  ((c.impl && c.ncol > 0) ? " cols=" + std::to_string(c.ncol) : std::string()).append(
                      (c.impl && (c.xg > 1 || c.xg < 0)) ? (c.xg < 0 ? std::string(" xcd_group=row")
                                                                    : " xcd_group=" + std::to_string(c.xg))
                                                         : std::string()).c_str(),
                  c.from_file ? "cached" : (c.tuned ? "tuned" : "default"));
    out += line;
    if (c.tuned || c.from_file) {
      std::snprintf(line, sizeof line, " lds_ms=%.4f register_ms=%.4f", c.ms[0], c.ms[1]);
      out += line;
    }
    out += "\n";
  }
  std::snprintf(buf, (size_t)len, "%s", out.c_str());
  return VC_OK;
}

}  // extern "C"
