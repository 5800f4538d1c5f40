// Tucker compression of the stored kernel spectra at setup and their rebuild before
// each product (eq. 13, Sec. II.C).
//
// Compression (FP64, once): the sequentially truncated HOSVD.  For modes kx, ky, kz in
// turn the current tensor's unfolding goes through an SVD (rocSOLVER gesvd), the
// smallest rank whose discarded squared singular values sum to at most
// tol^2 ||X||^2 / 3 is kept, and the tensor is projected onto those singular vectors
// (rocBLAS GEMM); what is left is the core.  The three budgets add up to
// ||X - X_hat|| <= tol ||X||.
//
// Rebuild (every product, FP32 or FP64): three GEMM steps on the matrix cores
// (tucker_kernels.hip) write each stored pair back into the spectra buffer the x pass
// reads; each step is one launch covering every stored pair (a device table of the
// pairs' GEMMs), so a rebuild is three launches whatever the number of pairs.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mvp_kernels.h"
#include "problem.h"

namespace vc {

#define VC_RB(expr)                                                          \
  do {                                                                       \
    const rocblas_status _s = (expr);                                        \
    if (_s != rocblas_status_success) {                                      \
      set_error("%s failed (rocblas status %d)", #expr, (int)_s);            \
      return VC_ERR_HIP;                                                     \
    }                                                                        \
  } while (0)

// Leading right singular vectors of A (m x n column-major, lda = m; destroyed): the
// smallest r whose discarded squared singular values sum to at most budget (directions
// beyond min(m, n) carry none).  Singular vectors straight from the SVD of the
// unfolding (not from the eigenvectors of its Gram matrix, whose squared condition
// number limits the small components the spectra need to ~1e-8 of the largest).
// U: n x r row-major on the device (U[i][a] = component i of vector a).
static vc_status leading_subspace(rocblas_handle h, double* A, int m, int n, double budget, DevMem& U, int* r_out,
                                  hipStream_t st) {
  const int k = std::min(m, n);
  DevMem sv, vt, e, info;
  VC_HIP(sv.alloc((size_t)k * sizeof(double)));
  VC_HIP(vt.alloc((size_t)n * n * sizeof(double)));
  VC_HIP(e.alloc((size_t)std::max(k - 1, 1) * sizeof(double)));
  VC_HIP(info.alloc(sizeof(rocblas_int)));
  VC_RB(rocsolver_dgesvd(h, rocblas_svect_none, rocblas_svect_all, m, n, A, m, sv.as<double>(), nullptr, 1,
                         vt.as<double>(), n, e.as<double>(), rocblas_outofplace, info.as<rocblas_int>()));
  std::vector<double> s(k), v((size_t)n * n);
  rocblas_int inf = 0;
  VC_HIP(hipMemcpyAsync(s.data(), sv.p, (size_t)k * sizeof(double), hipMemcpyDeviceToHost, st));
  VC_HIP(hipMemcpyAsync(v.data(), vt.p, v.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  VC_HIP(hipMemcpyAsync(&inf, info.p, sizeof(rocblas_int), hipMemcpyDeviceToHost, st));
  VC_HIP(hipStreamSynchronize(st));
  if (inf != 0) { set_error("SVD did not converge (info %d)", (int)inf); return VC_ERR_NUMERIC; }
  // singular values descending: drop from the smallest while the dropped energy fits
  int r = k;
  double acc = 0.0;
  while (r > 1) {
    acc += s[r - 1] * s[r - 1];
    if (acc > budget) break;
    --r;
  }
  // row a of V^T (element (a, i) at a + i n) is right singular vector a
  std::vector<double> u((size_t)n * r);
  for (int a = 0; a < r; ++a)
    for (int i = 0; i < n; ++i) u[(size_t)i * r + a] = v[(size_t)a + (size_t)i * n];
  VC_HIP(U.alloc(u.size() * sizeof(double)));
  VC_HIP(hipMemcpyAsync(U.p, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, st));
  VC_HIP(hipStreamSynchronize(st));
  *r_out = r;
  return VC_OK;
}

// Compress one tensor X (device, D1 x D2 x D3 row-major: [kx][ky][kz]).  The mode-i
// unfolding's transpose is handed to the SVD as a column-major matrix: X itself for
// mode 1, a copy with the first two indices swapped for modes 2 and 3.
static vc_status compress_one(rocblas_handle h, const double* X, int D1, int D2, int D3, double tol, TuckerPair& tp,
                              hipStream_t st) {
  const int64_t K1 = (int64_t)D2 * D3;
  const double one = 1.0, zero = 0.0;
  double nrm2 = 0.0;
  VC_RB(rocblas_ddot(h, (rocblas_int)(D1 * K1), X, 1, X, 1, &nrm2));   // host result: synchronizes
  const double budget = tol * tol * nrm2 / 3.0;
  // mode 1: A = X (D2 D3 x D1 column-major)
  DevMem A;
  VC_HIP(A.alloc((size_t)D1 * K1 * sizeof(double)));
  VC_HIP(hipMemcpyAsync(A.p, X, (size_t)D1 * K1 * sizeof(double), hipMemcpyDeviceToDevice, st));
  vc_status s = leading_subspace(h, A.as<double>(), (int)K1, D1, budget, tp.U64[0], &tp.r[0], st);
  if (s != VC_OK) return s;
  const int r1 = tp.r[0];
  // X1 (r1 x D2 D3) = U1^T X
  DevMem X1;
  VC_HIP(X1.alloc((size_t)r1 * K1 * sizeof(double)));
  VC_RB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)K1, r1, D1, &one, X,
                      (rocblas_int)K1, tp.U64[0].as<double>(), r1, &zero, X1.as<double>(), (rocblas_int)K1));
  // mode 2: A[ky][a][kz] (r1 D3 x D2 column-major)
  VC_HIP(launch_swap01(X1.as<double>(), A.as<double>(), r1, D2, D3, st));
  s = leading_subspace(h, A.as<double>(), r1 * D3, D2, budget, tp.U64[1], &tp.r[1], st);
  if (s != VC_OK) return s;
  const int r2 = tp.r[1];
  // X2[a] (r2 x D3) = U2^T X1[a]
  DevMem X2;
  VC_HIP(X2.alloc((size_t)r1 * r2 * D3 * sizeof(double)));
  VC_RB(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_transpose, D3, r2, D2, &one,
                                      X1.as<double>(), D3, K1, tp.U64[1].as<double>(), r2, 0, &zero, X2.as<double>(),
                                      D3, (rocblas_stride)r2 * D3, r1));
  // mode 3: A[kz][(a, b)] (r1 r2 x D3 column-major)
  VC_HIP(launch_swap01(X2.as<double>(), A.as<double>(), r1 * r2, D3, 1, st));
  s = leading_subspace(h, A.as<double>(), r1 * r2, D3, budget, tp.U64[2], &tp.r[2], st);
  if (s != VC_OK) return s;
  const int r3 = tp.r[2];
  // core S (r1 r2 x r3) = Y U3 with Y = X2 as (r1 r2 x D3)
  VC_HIP(tp.S64.alloc((size_t)r1 * r2 * r3 * sizeof(double)));
  VC_RB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, r3, r1 * r2, D3, &one,
                      tp.U64[2].as<double>(), r3, X2.as<double>(), D3, &zero, tp.S64.as<double>(), r3));
  VC_HIP(hipStreamSynchronize(st));
  return VC_OK;
}

vc_status tucker_compress_tensor(const double* X, int D1, int D2, int D3, double tol, TuckerPair& tp,
                                 hipStream_t st) {
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) { set_error("rocblas_create_handle failed"); return VC_ERR_HIP; }
  rocblas_set_stream(h, st);
  const vc_status s = compress_one(h, X, D1, D2, D3, tol, tp, st);
  rocblas_destroy_handle(h);
  return s;
}

vc_status tucker_begin(vc_problem* P, double tol) {
  P->tucker_tol = tol;
  P->tk.clear();
  P->tk_ms = 0.0;
  P->tk_count = 0;
  return VC_OK;
}

vc_status tucker_compress_pair(vc_problem* P, const double* X, hipStream_t st) {
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) { set_error("rocblas_create_handle failed"); return VC_ERR_HIP; }
  rocblas_set_stream(h, st);
  P->tk.emplace_back();
  TuckerPair& tp = P->tk.back();
  vc_status s = compress_one(h, X, P->Hx, P->Hy, P->H, P->tucker_tol, tp, st);
  rocblas_destroy_handle(h);
  if (s != VC_OK) return s;
  // FP32 copies of the core and factors
  const int64_t ns = (int64_t)tp.r[0] * tp.r[1] * tp.r[2];
  VC_HIP(tp.S32.alloc((size_t)ns * sizeof(float)));
  VC_HIP(launch_to_f32(tp.S64.as<double>(), tp.S32.as<float>(), ns, st));
  const int D[3] = {P->Hx, P->Hy, P->H};
  for (int m = 1; m < 3; ++m) {
    const int64_t nu = (int64_t)D[m] * tp.r[m];
    VC_HIP(tp.U32[m].alloc((size_t)nu * sizeof(float)));
    VC_HIP(launch_to_f32(tp.U64[m].as<double>(), tp.U32[m].as<float>(), nu, st));
  }
  // U1 for the fused x pass: FP64 with rows padded to a multiple of 4, FP32 transposed
  // with r1 padded to a multiple of 16 and Hx to a multiple of 64 (zero filled)
  const int r1 = tp.r[0];
  tp.r1p = (r1 + 3) & ~3;
  tp.r1q = (r1 + 15) & ~15;
  tp.hxp = (D[0] + 63) & ~63;
  std::vector<double> u((size_t)D[0] * r1), u64((size_t)D[0] * tp.r1p, 0.0);
  VC_HIP(hipMemcpyAsync(u.data(), tp.U64[0].p, u.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  VC_HIP(hipStreamSynchronize(st));
  std::vector<float> u32t((size_t)tp.r1q * tp.hxp, 0.0f);
  for (int x = 0; x < D[0]; ++x)
    for (int a = 0; a < r1; ++a) {
      u64[(size_t)x * tp.r1p + a] = u[(size_t)x * r1 + a];
      u32t[(size_t)a * tp.hxp + x] = (float)u[(size_t)x * r1 + a];
    }
  VC_HIP(tp.U1p64.alloc(u64.size() * sizeof(double)));
  VC_HIP(tp.U1t32.alloc(u32t.size() * sizeof(float)));
  VC_HIP(hipMemcpy(tp.U1p64.p, u64.data(), u64.size() * sizeof(double), hipMemcpyHostToDevice));
  VC_HIP(hipMemcpy(tp.U1t32.p, u32t.data(), u32t.size() * sizeof(float), hipMemcpyHostToDevice));
  return VC_OK;
}

// scratch of the rebuild: each pair its own T1 (r1 r2 x D3) and T2 (D2 x D3 x r1p)
// regions, so the two GEMM steps of every pair can run as two launches; T1 sized in
// FP64 elements and reused by FP32, T2 one per precision.  The fused x pass reads T2 and U1 through a per-pair device
// table (one per precision).
vc_status tucker_end(vc_problem* P) {
  int64_t t1 = 0, t2 = 0;
  P->tk_o1.clear();
  P->tk_o2.clear();
  for (const TuckerPair& tp : P->tk) {
    P->tk_o1.push_back(t1);
    P->tk_o2.push_back(t2);
    t1 += (int64_t)tp.r[0] * tp.r[1] * P->H;
    t2 += (int64_t)tp.r1p * P->Hy * P->H;
  }
  VC_HIP(P->tk_T1.alloc((size_t)std::max<int64_t>(t1, 1) * sizeof(double)));
  VC_HIP(P->tk_T2[0].alloc((size_t)std::max<int64_t>(t2, 1) * sizeof(float)));
  VC_HIP(P->tk_T2[1].alloc((size_t)std::max<int64_t>(t2, 1) * sizeof(double)));
  // T2's padding entries (r1 <= r < r1p) are never written: they stay zero
  for (auto& t : P->tk_T2) VC_HIP(hipMemset(t.p, 0, t.bytes));
  for (auto& tt : P->tk_tab) tt.built = false;   // rebuilt on next use
  for (int prec = 0; prec < 2; ++prec) {
    const bool f64 = prec == 1;
    std::vector<TkPairDev> v(P->tk.size());
    for (size_t q = 0; q < P->tk.size(); ++q) {
      const TuckerPair& tp = P->tk[q];
      v[q].U1 = tp.U1p64.p;
      v[q].U1t = tp.U1t32.p;
      v[q].r1q = tp.r1q;
      v[q].hxp = tp.hxp;
      v[q].T2 = f64 ? (const void*)(P->tk_T2[1].as<double>() + P->tk_o2[q])
                    : (const void*)(P->tk_T2[0].as<float>() + P->tk_o2[q]);
      v[q].r1 = tp.r[0];
      v[q].r1p = tp.r1p;
    }
    VC_HIP(P->tk_dev[prec].alloc(std::max<size_t>(v.size(), 1) * sizeof(TkPairDev)));
    if (!v.empty()) VC_HIP(hipMemcpy(P->tk_dev[prec].p, v.data(), v.size() * sizeof(TkPairDev), hipMemcpyHostToDevice));
  }
  return VC_OK;
}

// the two GEMM tables of one precision (built on first use)
template <typename T>
static vc_status rebuild_tables(vc_problem* P) {
  vc_problem::TkTables& tt = P->tk_tab[sizeof(T) == 8 ? 1 : 0];
  if (tt.built) return VC_OK;
  const int D2 = P->Hy, D3 = P->H;
  T* T1 = P->tk_T1.as<T>();
  T* T2 = P->tk_T2[sizeof(T) == 8 ? 1 : 0].as<T>();
  std::vector<GemmDesc> g1, g2;
  for (size_t q = 0; q < P->tk.size(); ++q) {
    const TuckerPair& tp = P->tk[q];
    const int r1 = tp.r[0], r2 = tp.r[1], r3 = tp.r[2];
    const void* S = sizeof(T) == 8 ? tp.S64.p : tp.S32.p;
    const void* U2 = sizeof(T) == 8 ? tp.U64[1].p : tp.U32[1].p;
    const void* U3 = sizeof(T) == 8 ? tp.U64[2].p : tp.U32[2].p;
    T* t1 = T1 + P->tk_o1[q];
    T* t2 = T2 + P->tk_o2[q];
    GemmDesc d{};
    // T1 (r1 r2 x D3) = S (r1 r2 x r3) U3^T
    d.A = S; d.B = U3; d.C = t1;
    d.M = r1 * r2; d.N = D3; d.K = r3; d.batch = 1;
    d.sam = r3; d.sak = 1; d.sbk = 1; d.sbn = r3; d.scm = D3; d.scn = 1;
    g1.push_back(d);
    // T2[.][.][a] (D2 x D3, element stride r1p) = U2 (D2 x r2) T1[a] (r2 x D3)
    d = GemmDesc{};
    d.A = U2; d.B = t1; d.C = t2;
    d.M = D2; d.N = D3; d.K = r2; d.batch = r1;
    d.sam = r2; d.sak = 1; d.sbk = D3; d.sbn = 1; d.scm = (int64_t)D3 * tp.r1p; d.scn = tp.r1p;
    d.bsa = 0; d.bsb = (int64_t)r2 * D3; d.bsc = 1;
    g2.push_back(d);
  }
  std::vector<GemmDesc>* all[2] = {&g1, &g2};
  for (int i = 0; i < 2; ++i) {
    std::vector<GemmDesc>& v = *all[i];
    const int nb = gemm_table_layout(v.data(), (int)v.size());
    if (nb < 0) return VC_ERR_ARG;
    VC_HIP(tt.tab[i].alloc(std::max<size_t>(v.size(), 1) * sizeof(GemmDesc)));
    if (!v.empty()) VC_HIP(hipMemcpy(tt.tab[i].p, v.data(), v.size() * sizeof(GemmDesc), hipMemcpyHostToDevice));
    tt.n[i] = (int)v.size();
    tt.nblk[i] = nb;
  }
  tt.built = true;
  return VC_OK;
}

// T1 and T2 of every stored pair (the x-mode product X = U1 T2 runs inside the x pass)
template <typename T>
vc_status tucker_rebuild(vc_problem* P, hipStream_t st, const int* skip) {
  const int D2 = P->Hy, D3 = P->H;
  // two launches for all pairs when every rank fits the register strip
  if (rebuild_tables<T>(P) == VC_OK) {
    const vc_problem::TkTables& tt = P->tk_tab[sizeof(T) == 8 ? 1 : 0];
    for (int i = 0; i < 2; ++i)
      VC_HIP(launch_mfma_gemm_multi<T>(tt.tab[i].as<GemmDesc>(), tt.n[i], tt.nblk[i], skip, st));
    return VC_OK;
  }
  // ranks above the strip: one pair after another with the general kernel
  T* T1 = P->tk_T1.as<T>();
  T* T2 = P->tk_T2[sizeof(T) == 8 ? 1 : 0].as<T>();
  for (size_t q = 0; q < P->tk.size(); ++q) {
    const TuckerPair& tp = P->tk[q];
    const int r1 = tp.r[0], r2 = tp.r[1], r3 = tp.r[2];
    const T* S = sizeof(T) == 8 ? (const T*)tp.S64.p : (const T*)tp.S32.p;
    const T* U2 = sizeof(T) == 8 ? (const T*)tp.U64[1].p : (const T*)tp.U32[1].p;
    const T* U3 = sizeof(T) == 8 ? (const T*)tp.U64[2].p : (const T*)tp.U32[2].p;
    T* t1 = T1 + P->tk_o1[q];
    T* t2 = T2 + P->tk_o2[q];
    GemmArgs g{};
    g.M = r1 * r2; g.N = D3; g.K = r3; g.batch = 1;
    g.sam = r3; g.sak = 1; g.sbk = 1; g.sbn = r3; g.scm = D3; g.scn = 1;
    g.skip = skip;
    VC_HIP(launch_mfma_gemm<T>(S, U3, t1, g, st));
    g = GemmArgs{};
    g.M = D2; g.N = D3; g.K = r2; g.batch = r1;
    g.sam = r2; g.sak = 1; g.sbk = D3; g.sbn = 1; g.scm = (int64_t)D3 * tp.r1p; g.scn = tp.r1p;
    g.bsa = 0; g.bsb = (int64_t)r2 * D3; g.bsc = 1;
    g.skip = skip;
    VC_HIP(launch_mfma_gemm<T>(U2, t1, t2, g, st));
  }
  return VC_OK;
}

template vc_status tucker_rebuild<float>(vc_problem*, hipStream_t, const int*);
template vc_status tucker_rebuild<double>(vc_problem*, hipStream_t, const int*);

}  // namespace vc
