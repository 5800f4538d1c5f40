// Setup of the FFT product (Sec. II.B, App. B) and of the preconditioner (Sec. II.D).
//
// Kernel spectra.  For each observer/source normal pair the Toeplitz tensor of App. B
// (Algorithm 1: the integral of eq. 5 or eq. 6 for every index lag, source centre
// offset from Tab. VII) is embedded in a circulant of length M_a >= 2 N_a + 1 per axis
// (lag l at index l mod M_a; Tab. VIII-X are this embedding for M_a = 2(N_a+1)) and
// transformed in FP64.  Every tensor is even in the lag components (odd along the
// observer normal for eq. 6), so after removing the half-voxel phase
// exp(-i pi k_alpha/M_alpha) exp(+i pi k_beta/M_beta) (and a factor i for eq. 6) its
// spectrum is real and has a definite parity under k_a -> M_a - k_a; only the octant
// 0 <= k_a <= M_a/2 is stored.  Eq. (12) is the statement that the pair (beta, alpha)
// is the complex conjugate of (alpha, beta): only 6 of the 9 P spectra are stored.
//
// Preconditioner.  The box is cut into nv voxel boxes; the conductor panels owned by a
// box (those on a conductor voxel of that box) form one dense block of eq. (5) values,
// which is Cholesky-factored and inverted in FP64.  Identical panel patterns share one
// inverse.  Dielectric rows use the inverse of the eq. (7) diagonal.
#include <atomic>
#include <thread>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "mvp_kernels.h"
#include "octant_kernels.h"
#include "problem.h"

namespace vc {

int pair_index_P(int a, int b) { return a == b ? a : 2 + a + b; }
int pair_index_E(int a, int b) { return 6 + 3 * a + b; }

int pair_odd_bits(int q) {
  if (q < 3) return 0;
  if (q < 6) {
    const int s = q - 2;   // a + b
    const int a = (s == 1 || s == 2) ? 0 : 1;
    const int b = s - a;
    return (1 << a) | (1 << b);
  }
  const int a = (q - 6) / 3, b = (q - 6) % 3;
  return a == b ? (1 << a) : (1 << b);
}

void pair_axes(int q, int* a, int* b, int* want) {
  if (q < 3) { *a = *b = q; *want = 0; return; }
  if (q < 6) {
    const int s = q - 2;
    *a = (s == 1 || s == 2) ? 0 : 1;
    *b = s - *a;
    *want = 0;
    return;
  }
  *a = (q - 6) / 3;
  *b = (q - 6) % 3;
  *want = 1;
}

void gauss_legendre_table(std::vector<double>& gl) {
  gl.assign(11 * 24, 0.0);
  for (int n = 1; n <= 10; ++n) {
    for (int i = 0; i < n; ++i) {
      long double x = cosl(M_PI * (i + 0.75L) / (n + 0.5L));
      for (int it = 0; it < 100; ++it) {
        long double p0 = 1.0L, p1 = x;
        for (int k = 2; k <= n; ++k) {
          long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        if (n == 1) { p0 = 1.0L; p1 = x; }
        long double dp = n * (x * p1 - p0) / (x * x - 1.0L);
        long double dx = p1 / dp;
        x -= dx;
        if (fabsl(dx) < 1e-19L) break;
      }
      long double p0 = 1.0L, p1 = x;
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2.0L * k - 1.0L) * x * p1 - (k - 1.0L) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p0 = 1.0L; p1 = x; }
      long double dp = n * (x * p1 - p0) / (x * x - 1.0L);
      long double w = 2.0L / ((1.0L - x * x) * dp * dp);
      gl[n * 24 + i] = (double)(0.5L * x);
      gl[n * 24 + 12 + i] = (double)(0.5L * w);
    }
  }
}

template <typename T>
static hipError_t upload_axis(AxisTables& t, int L, int axis) {
  (void)axis;
  t.plan = make_plan(L, Tune<T>::maxr);
  std::vector<T> tw(2 * L), ph(2 * L);
  for (int k = 0; k < L; ++k) {
    const long double a = 2.0L * (long double)M_PI * k / L;
    tw[2 * k] = (T)cosl(a);
    tw[2 * k + 1] = (T)(-sinl(a));
    const long double b = (long double)M_PI * k / L;
    ph[2 * k] = (T)cosl(b);
    ph[2 * k + 1] = (T)sinl(b);
  }
  hipError_t e = t.tw.alloc(tw.size() * sizeof(T));
  if (e != hipSuccess) return e;
  e = hipMemcpy(t.tw.p, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = t.ph.alloc(ph.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(t.ph.p, ph.data(), ph.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Largest tile (columns per workgroup) whose LDS use fits `budget` bytes and whose
// element count L*ncol stays within emax per thread for at most 1024 threads.
// Among feasible tiles, prefer little padding waste (tiles past the last column) and
// enough workgroups (other_blocks = product of the other grid dimensions) to fill the
// chip several times over; then the widest tile.
static size_t g_lds_ext = kLdsBudget;

size_t lds_ext_budget() { return g_lds_ext; }

void note_device_lds(int device) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess &&
      (size_t)v > kLdsBudget)
    g_lds_ext = (size_t)v;
}

bool pick_tile(int L, int elem_bytes, int emax, int ncols_total, int* ncol, int* nthr, size_t budget,
               int64_t other_blocks, int max_thr) {
  // nothing fits the preferred budget: use the device's per-workgroup maximum
  const size_t one = (size_t)elem_bytes * ((size_t)L + 2 * (size_t)L * 2);
  if (one > budget && budget < g_lds_ext) budget = g_lds_ext;
  int best = 0;
  double best_score = -1e30;
  for (int c : {32, 16, 8, 4, 2, 1}) {
    const size_t lds = (size_t)elem_bytes * ((size_t)L + 2 * (size_t)L * (c + 1));
    const int64_t thr = ((int64_t)L * c + emax - 1) / emax;
    if (lds > budget || thr > max_thr) continue;
    const int64_t tiles = (ncols_total + c - 1) / c;
    const double waste = (double)(tiles * c - ncols_total) / (double)(tiles * c);
    const double wgs = (double)tiles * (double)(other_blocks > 0 ? other_blocks : 1);
    double score = std::log2((double)c) - 8.0 * waste;
    if (wgs < 1024.0) score -= 2.0 * std::log2(1024.0 / wgs);
    if (score > best_score) { best_score = score; best = c; }
  }
  if (best == 0) { set_error("no FFT tile fits length %d", L); return false; }
  int64_t thr = ((int64_t)L * best + emax - 1) / emax;
  thr = ((thr + 63) / 64) * 64;
  if (thr < 64) thr = 64;
  *ncol = best;
  *nthr = (int)thr;
  return (int64_t)L * best <= (int64_t)emax * thr && thr <= max_thr;
}

template <typename T>
static vc_status upload(DevMem& d, const std::vector<T>& h) {
  VC_HIP(d.alloc(h.size() * sizeof(T)));
  if (!h.empty()) VC_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return VC_OK;
}

vc_status build_spectra(vc_problem* P, int want64, int want32, double tucker_tol, hipStream_t st) {
  const int Mx = P->M[0], My = P->M[1], Mz = P->M[2];
  const int H = P->H, Hx = P->Hx, Hy = P->Hy;
  // index maps
  vc_status s;
  if ((s = upload(P->d_line_ptr, P->line_ptr)) != VC_OK) return s;
  if ((s = upload(P->d_items, P->items)) != VC_OK) return s;
  if ((s = upload(P->d_lflag, P->lflag)) != VC_OK) return s;
  if ((s = upload(P->d_pflag, P->pflag)) != VC_OK) return s;
  if ((s = upload(P->d_pk, P->pk)) != VC_OK) return s;
  if ((s = upload(P->d_pkind, P->pkind)) != VC_OK) return s;
  if ((s = upload(P->d_diag, P->diag)) != VC_OK) return s;
  if ((s = upload(P->d_cond_ptr, P->cond_ptr)) != VC_OK) return s;
  if ((s = upload(P->d_cond_panels, P->cond_panels)) != VC_OK) return s;
  if ((s = upload(P->d_weight, P->weight)) != VC_OK) return s;
  {
    std::vector<int32_t> pc(P->panels.size());
    for (size_t k = 0; k < pc.size(); ++k) pc[k] = P->panels[k].kind == 0 ? P->panels[k].cond : -1;
    if ((s = upload(P->d_pcond, pc)) != VC_OK) return s;
  }
  std::vector<double> gl;
  gauss_legendre_table(gl);
  if ((s = upload(P->d_gl, gl)) != VC_OK) return s;
  for (int a = 0; a < 3; ++a) {
    VC_HIP(upload_axis<double>(P->t64.ax[a], P->M[a], a));
    VC_HIP(upload_axis<float>(P->t32.ax[a], P->M[a], a));
    if (P->t64.ax[a].plan.nst < 0) { set_error("FFT size %d not 7-smooth", P->M[a]); return VC_ERR_ARG; }
  }
  const int npairs = P->n_diel > 0 ? 15 : 6;
  const int64_t per_pair = (int64_t)Hy * H * Hx;
  P->have64 = want64;
  P->have32 = want32;
  P->spectra_bytes = 0;
  const bool tucker = tucker_tol > 0.0;
  // the Tucker form keeps no spectra: each x-pass workgroup builds its tile's from the
  // factors (eq. 13); uncompressed, every stored pair is kept
  P->t64.R.reset();
  P->t32.R.reset();
  if (!tucker) {
    if (want64) { VC_HIP(P->t64.R.alloc((size_t)15 * per_pair * sizeof(double))); P->spectra_bytes += (double)npairs * per_pair * 8; }
    if (want32) { VC_HIP(P->t32.R.alloc((size_t)15 * per_pair * sizeof(float))); P->spectra_bytes += (double)npairs * per_pair * 4; }
  }
  DevMem circ, spec, resid, one;   // one: a pair's FP64 spectrum when compressing
  if (tucker) {
    VC_HIP(one.alloc((size_t)per_pair * sizeof(double)));
    if ((s = tucker_begin(P, tucker_tol)) != VC_OK) return s;
  }
  VC_HIP(circ.alloc((size_t)Mx * My * Mz * sizeof(double)));
  VC_HIP(spec.alloc((size_t)Mx * My * H * 2 * sizeof(double)));
  // Toeplitz source: the panel integrals on this grid, or a cache's octants cropped to it
  const vc_toeplitz_cache* tzc = P->tz_cache;
  const int ngrid[3] = {P->nx, P->ny, P->nz};
  DevMem oct;
  if (tzc) {
    if (tzc->device != P->device || ngrid[0] > tzc->nmax[0] || ngrid[1] > tzc->nmax[1] || ngrid[2] > tzc->nmax[2]) {
      set_error("the Toeplitz cache does not cover this grid on this device");
      return VC_ERR_ARG;
    }
    VC_HIP(oct.alloc((size_t)(ngrid[0] + 1) * (ngrid[1] + 1) * (ngrid[2] + 1) * sizeof(double)));
  }
  P->t_toeplitz = 0.0;
  VC_HIP(resid.alloc(sizeof(double)));
  VC_HIP(hipMemsetAsync(resid.p, 0, sizeof(double), st));
  const int n[3] = {P->nx, P->ny, P->nz};
  const double scale = 1.0 / ((double)Mx * My * Mz);
  for (int q = 0; q < npairs; ++q) {
    int a, b, want;
    pair_axes(q, &a, &b, &want);
    FillArgs fa{};
    fa.alpha = a; fa.beta = b; fa.want = want;
    fa.Mx = Mx; fa.My = My; fa.Mz = Mz;
    for (int ax = 0; ax < 3; ++ax) {
      fa.no[ax] = n[ax] + (ax == a);
      fa.ns[ax] = n[ax] + (ax == b);
    }
    fa.scale = scale;
    VC_HIP(hipStreamSynchronize(st));
    const auto tt0 = std::chrono::steady_clock::now();
    if (tzc) {
      if ((s = toeplitz_restore(tzc, q, ngrid, oct.as<double>(), st)) != VC_OK) return s;
      OctArgs oa{};
      oa.alpha = a; oa.beta = b; oa.want = want;
      for (int ax = 0; ax < 3; ++ax) oa.D[ax] = ngrid[ax] + 1;
      VC_HIP(launch_embed_octant(circ.as<double>(), oct.as<double>(), fa, oa, st));
    } else {
      VC_HIP(launch_fill_circulant(circ.as<double>(), fa, P->d_gl.as<double>(), st));
    }
    VC_HIP(hipStreamSynchronize(st));
    P->t_toeplitz += std::chrono::duration<double>(std::chrono::steady_clock::now() - tt0).count();
    int ncol, nthr;
    if (!pick_tile(Mz, 16, Tune<double>::emax, (Mx * My + 1) / 2, &ncol, &nthr, kLdsBudget, 1)) return VC_ERR_ARG;
    VC_HIP(launch_zr2c_dense(circ.as<double>(), spec.p, Mx * My, H, P->t64.ax[2].plan, P->t64.ax[2].tw.p, ncol, nthr, st));
    CompSet cs{};
    cs.n = 1;
    StridedArgs sa{};
    sa.comp_stride = 0; sa.rhs_stride = 0;
    sa.ncols = H; sa.nrhs = 1; sa.inverse = 0; sa.n1x = 0; sa.n1y = 0;
    // y pass over all Mx planes
    if (!pick_tile(My, 16, Tune<double>::emax, H, &ncol, &nthr, kLdsBudget, Mx)) return VC_ERR_ARG;
    sa.plane_stride = (int64_t)My * H; sa.row_stride = H; sa.ncol = ncol; sa.nin = My; sa.nout = My;
    VC_HIP(launch_strided<double>(spec.p, sa, cs, Mx, P->t64.ax[1].plan, P->t64.ax[1].tw.p, nullptr, nullptr, nthr, st));
    // x pass over all My planes
    if (!pick_tile(Mx, 16, Tune<double>::emax, H, &ncol, &nthr, kLdsBudget, My)) return VC_ERR_ARG;
    sa.plane_stride = H; sa.row_stride = (int64_t)My * H; sa.ncol = ncol; sa.nin = Mx; sa.nout = Mx;
    VC_HIP(launch_strided<double>(spec.p, sa, cs, My, P->t64.ax[0].plan, P->t64.ax[0].tw.p, nullptr, nullptr, nthr, st));
    ExtractArgs ea{};
    ea.Mx = Mx; ea.My = My; ea.Mz = Mz; ea.H = H; ea.Hx = Hx; ea.Hy = Hy;
    ea.kind = want == 1 ? 2 : (a == b ? 0 : 1);
    ea.alpha = a; ea.beta = b;
    if (tucker) {
      ea.pair_off = 0;
      VC_HIP(launch_extract(spec.p, one.as<double>(), nullptr, ea, resid.as<double>(), st));
      if ((s = tucker_compress_pair(P, one.as<double>(), st)) != VC_OK) return s;
    } else {
      ea.pair_off = (int64_t)q * per_pair;
      VC_HIP(launch_extract(spec.p, want64 ? P->t64.R.as<double>() : nullptr, want32 ? P->t32.R.as<float>() : nullptr,
                            ea, resid.as<double>(), st));
    }
  }
  if (tucker) {
    if ((s = tucker_end(P)) != VC_OK) return s;
    // resident: every device buffer of the Tucker form (cores and factors in FP64 and
    // FP32, the padded U1 copies) and the rebuild's T1 / T2 strips
    for (const TuckerPair& tp : P->tk) {
      P->spectra_bytes += (double)(tp.S64.bytes + tp.S32.bytes + tp.U1p64.bytes + tp.U1t32.bytes);
      for (int m = 0; m < 3; ++m) P->spectra_bytes += (double)(tp.U64[m].bytes + tp.U32[m].bytes);
    }
    P->spectra_bytes += (double)(P->tk_T1.bytes + P->tk_T2[0].bytes + P->tk_T2[1].bytes);
  }
  double r = 0.0;
  VC_HIP(hipMemcpyAsync(&r, resid.p, sizeof(double), hipMemcpyDeviceToHost, st));
  VC_HIP(hipStreamSynchronize(st));
  P->extract_resid = r;
  return VC_OK;
}

// ------------------------------------------------------------------------------ preconditioner
static bool cholesky_inverse(std::vector<double>& A, int n) {
  // A (n x n, row-major, symmetric positive definite) -> A^{-1}
  std::vector<double> L(A);
  for (int j = 0; j < n; ++j) {
    double d = L[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0)) return false;
    d = std::sqrt(d);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = L[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = s / d;
    }
  }
  // inverse of L (lower)
  std::vector<double> Li((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Li[(size_t)j * n + j] = 1.0 / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s -= L[(size_t)i * n + k] * Li[(size_t)k * n + j];
      Li[(size_t)i * n + j] = s / L[(size_t)i * n + i];
    }
  }
  // A^{-1} = Li^T Li
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
      A[(size_t)i * n + j] = s;
      A[(size_t)j * n + i] = s;
    }
  return true;
}

// The same tables read from a Toeplitz cache: each pair's octant restored for
// min(nv_a, n_a) offsets per axis (a panel lag along axis a never exceeds n_a; entries
// of lags the grid cannot hold stay 0), then every lag's entry taken at |d| with the
// sign of eq. (6) in d_alpha.  Eq. (5) with a > b reads the octant of (b, a): the
// kernel is even, so both orders have the same values at the same |d|.
static vc_status lag_tables_cached(vc_problem* P, const vc_toeplitz_cache* C, int want, std::vector<double>& tab,
                                   int64_t nl, hipStream_t st) {
  const int nv[3] = {P->nv[0], P->nv[1], P->nv[2]};
  const int ng[3] = {P->nx, P->ny, P->nz};
  int c[3];
  for (int ax = 0; ax < 3; ++ax) c[ax] = std::min(nv[ax], ng[ax]);
  const int64_t no = (int64_t)(c[0] + 1) * (c[1] + 1) * (c[2] + 1);
  DevMem doct;
  VC_HIP(doct.alloc(no * sizeof(double)));
  std::vector<double> oct(no);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int q = want == 0 ? pair_index_P(std::min(a, b), std::max(a, b)) : pair_index_E(a, b);
      vc_status s = toeplitz_restore(C, q, c, doct.as<double>(), st);   // synchronizes
      if (s != VC_OK) return s;
      VC_HIP(hipMemcpy(oct.data(), doct.p, no * sizeof(double), hipMemcpyDeviceToHost));
      int64_t t = 0;
      for (int lx = -nv[0]; lx <= nv[0]; ++lx)
        for (int ly = -nv[1]; ly <= nv[1]; ++ly)
          for (int lz = -nv[2]; lz <= nv[2]; ++lz, ++t) {
            const int l[3] = {lx, ly, lz};
            int o[3];
            bool inside = true, neg_a = false;
            for (int ax = 0; ax < 3; ++ax) {
              // twice the offset, d = l - 1/2 on the observer normal and l + 1/2 on the
              // source normal of an orthogonal pair; o = |d| - h
              const int d2 = 2 * l[ax] + (a != b ? (ax == a ? -1 : (ax == b ? 1 : 0)) : 0);
              o[ax] = (d2 < 0 ? -d2 : d2) / 2;
              if (ax == a) neg_a = d2 < 0;
              inside = inside && o[ax] <= c[ax];
            }
            if (!inside) continue;
            const double v = oct[((int64_t)o[0] * (c[1] + 1) + o[1]) * (c[2] + 1) + o[2]];
            tab[(size_t)(3 * a + b) * nl + t] = (want == 1 && neg_a) ? -v : v;
          }
    }
  return VC_OK;
}

// The eq. (5) (want 0) or eq. (6) (want 1) integral for every observer/source normal
// pair and every index lag in [-nv, nv] per axis: tab[(3 a + b) nl + t], lag t in
// x-major order over the (2 nv + 1)^3 box of lags.  With a Toeplitz cache the values
// come from its octants, else from the panel integrals.
static vc_status lag_tables(vc_problem* P, int want, std::vector<double>& tab, int64_t* nl_out, hipStream_t st,
                            const vc_toeplitz_cache* C = nullptr) {
  const int nvx = P->nv[0], nvy = P->nv[1], nvz = P->nv[2];
  const int ex = 2 * nvx + 1, ey = 2 * nvy + 1, ez = 2 * nvz + 1;
  const int64_t nl = (int64_t)ex * ey * ez;
  *nl_out = nl;
  tab.assign(9 * nl, 0.0);
  if (C) return lag_tables_cached(P, C, want, tab, nl, st);
  std::vector<double> d(3 * nl);
  DevMem dd, dout;
  VC_HIP(dd.alloc(d.size() * sizeof(double)));
  VC_HIP(dout.alloc(nl * sizeof(double)));
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      int64_t t = 0;
      for (int lx = -nvx; lx <= nvx; ++lx)
        for (int ly = -nvy; ly <= nvy; ++ly)
          for (int lz = -nvz; lz <= nvz; ++lz, ++t) {
            double o[3] = {(double)lx, (double)ly, (double)lz};
            if (a != b) { o[a] -= 0.5; o[b] += 0.5; }
            d[3 * t] = o[0]; d[3 * t + 1] = o[1]; d[3 * t + 2] = o[2];
          }
      VC_HIP(hipMemcpy(dd.p, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice));
      VC_HIP(launch_kernel_table(dd.as<double>(), (int)nl, a, b, want, dout.as<double>(), P->d_gl.as<double>(), st));
      VC_HIP(hipMemcpyAsync(&tab[(size_t)(3 * a + b) * nl], dout.p, nl * sizeof(double), hipMemcpyDeviceToHost, st));
      VC_HIP(hipStreamSynchronize(st));
    }
  return VC_OK;
}

vc_status build_precond(vc_problem* P, hipStream_t st) {
  Precond& pc = P->pc;
  const int nvx = P->nv[0], nvy = P->nv[1], nvz = P->nv[2];
  const int64_t N = npanels(P);
  // kernel table of eq. (5) for every lag inside a box: lag in [-nv, nv] per axis
  const int ey = 2 * nvy + 1, ez = 2 * nvz + 1;
  int64_t nl = 0;
  std::vector<double> tab;
  {
    // the cache is only known to be alive during vc_setup, which is where this runs
    const vc_status ts = lag_tables(P, 0, tab, &nl, st, P->tz_cache);
    if (ts != VC_OK) return ts;
  }
  // group conductor panels by owning box
  const int nbx = (P->nx + nvx - 1) / nvx, nby = (P->ny + nvy - 1) / nvy, nbz = (P->nz + nvz - 1) / nvz;
  std::map<int64_t, std::vector<int32_t>> boxes;
  for (int64_t p = 0; p < N; ++p) {
    const vc_panel& pn = P->panels[p];
    if (pn.kind != 0) continue;
    int v[3] = {pn.i, pn.j, pn.k};
    if (pn.eps_lo == 0.0) v[pn.dir] -= 1;   // conductor on the -axis side
    const int64_t key = ((int64_t)(v[0] / nvx) * nby + v[1] / nvy) * nbz + v[2] / nvz;
    boxes[key].push_back((int32_t)p);
  }
  (void)nbx;
  std::map<std::vector<int32_t>, int> uniq;
  pc.h_box_ptr.assign(1, 0);
  pc.h_box_panels.clear();
  pc.h_box_block.clear();
  pc.h_block_n.clear();
  pc.h_block_off.clear();
  pc.h_blocks.clear();
  for (auto& kv : boxes) {
    const int64_t key = kv.first;
    const int bz = (int)(key % nbz), by = (int)((key / nbz) % nby), bx = (int)(key / ((int64_t)nbz * nby));
    const int ox = bx * nvx, oy = by * nvy, oz = bz * nvz;
    const auto& pl = kv.second;
    const int nb = (int)pl.size();
    if (nb > 4096) { set_error("preconditioner box holds %d panels (> 4096); use smaller nv", nb); return VC_ERR_ARG; }
    std::vector<int32_t> pat;
    pat.reserve(4 * nb);
    for (int32_t p : pl) {
      const vc_panel& pn = P->panels[p];
      pat.push_back(pn.dir); pat.push_back(pn.i - ox); pat.push_back(pn.j - oy); pat.push_back(pn.k - oz);
    }
    auto it = uniq.find(pat);
    int blk;
    if (it == uniq.end()) {
      std::vector<double> A((size_t)nb * nb);
      for (int r = 0; r < nb; ++r)
        for (int c = 0; c < nb; ++c) {
          const vc_panel& pr = P->panels[pl[r]];
          const vc_panel& pcn = P->panels[pl[c]];
          const int lx = pr.i - pcn.i, ly = pr.j - pcn.j, lz = pr.k - pcn.k;
          const int64_t t = ((int64_t)(lx + nvx) * ey + (ly + nvy)) * ez + (lz + nvz);
          A[(size_t)r * nb + c] = tab[(size_t)(3 * pr.dir + pcn.dir) * nl + t];
        }
      if (!cholesky_inverse(A, nb)) { set_error("preconditioner block not positive definite"); return VC_ERR_NUMERIC; }
      blk = (int)pc.h_block_n.size();
      uniq.emplace(std::move(pat), blk);
      pc.h_block_n.push_back(nb);
      pc.h_block_off.push_back((int64_t)pc.h_blocks.size());
      // stored transposed (column i of the inverse contiguous): the apply kernel's lanes
      // then read consecutive addresses
      const size_t o = pc.h_blocks.size();
      pc.h_blocks.resize(o + (size_t)nb * nb);
      for (int r = 0; r < nb; ++r)
        for (int c = 0; c < nb; ++c) pc.h_blocks[o + (size_t)c * nb + r] = A[(size_t)r * nb + c];
    } else {
      blk = it->second;
    }
    for (int32_t p : pl) pc.h_box_panels.push_back(p);
    pc.h_box_ptr.push_back((int32_t)pc.h_box_panels.size());
    pc.h_box_block.push_back(blk);
  }
  pc.nbox = (int)pc.h_box_block.size();
  pc.nblock = (int)pc.h_block_n.size();
  pc.block_doubles = (int64_t)pc.h_blocks.size();
  std::vector<double> dinv(N, 0.0), dinv_diag(N, 0.0);
  const double pself = tab[(size_t)0 * nl + ((int64_t)nvx * ey + nvy) * ez + nvz];
  pc.pself = pself;
  for (int64_t p = 0; p < N; ++p) {
    if (P->panels[p].kind == 1) dinv[p] = dinv_diag[p] = 1.0 / P->diag[p];
    else dinv_diag[p] = 1.0 / pself;
  }
  vc_status s;
  if ((s = upload(pc.box_ptr, pc.h_box_ptr)) != VC_OK) return s;
  if ((s = upload(pc.box_panels, pc.h_box_panels)) != VC_OK) return s;
  if ((s = upload(pc.box_block, pc.h_box_block)) != VC_OK) return s;
  if ((s = upload(pc.block_off, pc.h_block_off)) != VC_OK) return s;
  if ((s = upload(pc.block_n, pc.h_block_n)) != VC_OK) return s;
  if ((s = upload(pc.blocks, pc.h_blocks)) != VC_OK) return s;
  if ((s = upload(pc.dinv, dinv)) != VC_OK) return s;
  if ((s = upload(pc.dinv_diag, dinv_diag)) != VC_OK) return s;
  pc.built = 1;
  return VC_OK;
}

// A^{-1} of a general n x n matrix (row-major) by Gauss-Jordan elimination with partial
// pivoting, in place; false if a pivot vanishes.
static bool lu_inverse(std::vector<double>& A, int n) {
  std::vector<double> Inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + k]) > best) { best = std::fabs(A[(size_t)i * n + k]); piv = i; }
    if (!(best > 0.0)) return false;
    if (piv != k)
      for (int j = 0; j < n; ++j) {
        std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
        std::swap(Inv[(size_t)k * n + j], Inv[(size_t)piv * n + j]);
      }
    const double ip = 1.0 / A[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) { A[(size_t)k * n + j] *= ip; Inv[(size_t)k * n + j] *= ip; }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = A[(size_t)i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
        Inv[(size_t)i * n + j] -= f * Inv[(size_t)k * n + j];
      }
    }
  }
  A.swap(Inv);
  return true;
}

// The conventional block-diagonal preconditioner of the comparison in Sec. III.A: the
// same nv voxel boxes, but every panel joins a box (a conductor panel the box of its
// conductor voxel, a dielectric panel the box of the voxel on its -axis side, or +axis
// side on the grid's low face), and each box's block is the full row of eq. (4)
// restricted to the box: eq. (5) values on conductor rows, the eq. (7) diagonal plus
// eq. (6) values on dielectric rows (+axis normal, as the product's rows).  The blocks
// are unsymmetric; their inverses are stored transposed like the conductor blocks, and
// identical (pattern, permittivity) boxes share one inverse.
vc_status build_precond_full(vc_problem* P, hipStream_t st) {
  FullBlocks& fb = P->pc.full;
  if (fb.built) return VC_OK;
  const int nvx = P->nv[0], nvy = P->nv[1], nvz = P->nv[2];
  const int64_t N = npanels(P);
  const int ey = 2 * nvy + 1, ez = 2 * nvz + 1;
  int64_t nl = 0;
  std::vector<double> tp, te;
  vc_status s;
  if ((s = lag_tables(P, 0, tp, &nl, st)) != VC_OK) return s;
  if ((s = lag_tables(P, 1, te, &nl, st)) != VC_OK) return s;
  const int nby = (P->ny + nvy - 1) / nvy, nbz = (P->nz + nvz - 1) / nvz;
  std::map<int64_t, std::vector<int32_t>> boxes;
  for (int64_t p = 0; p < N; ++p) {
    const vc_panel& pn = P->panels[p];
    int v[3] = {pn.i, pn.j, pn.k};
    if (pn.kind == 0) {
      if (pn.eps_lo == 0.0) v[pn.dir] -= 1;   // conductor on the -axis side
    } else if (v[pn.dir] > 0) {
      v[pn.dir] -= 1;
    }
    const int64_t key = ((int64_t)(v[0] / nvx) * nby + v[1] / nvy) * nbz + v[2] / nvz;
    boxes[key].push_back((int32_t)p);
  }
  std::map<std::vector<int64_t>, int> uniq;
  std::vector<int32_t> box_ptr(1, 0), box_panels, box_block, block_n;
  std::vector<const std::vector<int32_t>*> block_src;   // panels of the box that defines each block
  for (auto& kv : boxes) {
    const int64_t key = kv.first;
    const int bz = (int)(key % nbz), by = (int)((key / nbz) % nby), bx = (int)(key / ((int64_t)nbz * nby));
    const int ox = bx * nvx, oy = by * nvy, oz = bz * nvz;
    const auto& pl = kv.second;
    const int nb = (int)pl.size();
    if (nb > 4096) { set_error("preconditioner box holds %d panels (> 4096); use smaller nv", nb); return VC_ERR_ARG; }
    std::vector<int64_t> pat;
    pat.reserve(5 * nb);
    for (int32_t p : pl) {
      const vc_panel& pn = P->panels[p];
      int64_t dbits = 0;
      std::memcpy(&dbits, &P->diag[p], sizeof(double));
      pat.push_back(pn.kind * 4 + pn.dir); pat.push_back(pn.i - ox); pat.push_back(pn.j - oy); pat.push_back(pn.k - oz);
      pat.push_back(dbits);
    }
    auto it = uniq.find(pat);
    int blk;
    if (it == uniq.end()) {
      blk = (int)block_n.size();
      uniq.emplace(std::move(pat), blk);
      block_n.push_back(nb);
      block_src.push_back(&pl);
    } else {
      blk = it->second;
    }
    for (int32_t p : pl) box_panels.push_back(p);
    box_ptr.push_back((int32_t)box_panels.size());
    box_block.push_back(blk);
  }
  const int nblk = (int)block_n.size();
  std::vector<int64_t> block_off(nblk);
  int64_t total = 0;
  for (int b = 0; b < nblk; ++b) { block_off[b] = total; total += (int64_t)block_n[b] * block_n[b]; }
  std::vector<double> blocks((size_t)total);
  // assemble and invert the distinct blocks on the host's cores
  std::atomic<int> next{0}, bad{0};
  auto work = [&]() {
    std::vector<double> A;
    for (int b = next++; b < nblk && !bad; b = next++) {
      const std::vector<int32_t>& pl = *block_src[b];
      const int nb = block_n[b];
      A.assign((size_t)nb * nb, 0.0);
      for (int r = 0; r < nb; ++r) {
        const vc_panel& pr = P->panels[pl[r]];
        const std::vector<double>& tab = pr.kind == 0 ? tp : te;
        for (int c = 0; c < nb; ++c) {
          const vc_panel& pcn = P->panels[pl[c]];
          const int lx = pr.i - pcn.i, ly = pr.j - pcn.j, lz = pr.k - pcn.k;
          const int64_t t = ((int64_t)(lx + nvx) * ey + (ly + nvy)) * ez + (lz + nvz);
          A[(size_t)r * nb + c] = tab[(size_t)(3 * pr.dir + pcn.dir) * nl + t] + (r == c ? P->diag[pl[r]] : 0.0);
        }
      }
      if (!lu_inverse(A, nb)) { bad = 1; return; }
      double* o = blocks.data() + block_off[b];
      for (int r = 0; r < nb; ++r)
        for (int c = 0; c < nb; ++c) o[(size_t)c * nb + r] = A[(size_t)r * nb + c];
    }
  };
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (int t = 1; t < std::min(nth, nblk); ++t) pool.emplace_back(work);
  work();
  for (auto& t : pool) t.join();
  if (bad) { set_error("block-diagonal preconditioner: singular block"); return VC_ERR_NUMERIC; }
  fb.nbox = (int)box_block.size();
  fb.nblock = (int)block_n.size();
  fb.block_doubles = (int64_t)blocks.size();
  if ((s = upload(fb.box_ptr, box_ptr)) != VC_OK) return s;
  if ((s = upload(fb.box_panels, box_panels)) != VC_OK) return s;
  if ((s = upload(fb.box_block, box_block)) != VC_OK) return s;
  if ((s = upload(fb.block_off, block_off)) != VC_OK) return s;
  if ((s = upload(fb.block_n, block_n)) != VC_OK) return s;
  if ((s = upload(fb.blocks, blocks)) != VC_OK) return s;
  fb.built = 1;
  return VC_OK;
}

}  // namespace vc
