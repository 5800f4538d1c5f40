// Toeplitz setup path (Sec. II.C and Tab. I): the block Toeplitz tensors of App. B are
// computed once over a largest grid, Tucker-compressed (eq. 13) and kept, on disk if
// wanted; a problem's setup then restores them cropped to its own grid and embeds them
// in its circulants instead of evaluating the panel integrals again.
//
// What is stored per pair is one octant: the kernel at the non-negative centre offsets
// d_a = t_a + h_a (t_a = 0..nmax_a, h_a = 1/2 on the two normal axes of an orthogonal
// pair).  The kernel of eq. (5) is even in every offset component and that of eq. (6)
// odd in d_alpha and even in the rest, so the octant holds every value a grid of at
// most nmax voxels per axis needs.  A Tucker factor is indexed by one axis' offset, so
// the tensor of a smaller grid is the same core with the leading n_a + 1 rows of each
// factor: cropping costs nothing and adds no error.  In the dimensionless form (voxel
// edge 1) the tensors do not depend on the voxel size, so the rescaling by powers of
// the voxel edge that a dimensional store needs is the identity here.
#include <rocblas/rocblas.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mvp_kernels.h"
#include "octant_kernels.h"
#include "problem.h"

namespace vc {

namespace {

const char kMagic[8] = {'V', 'C', 'T', 'O', 'E', 'P', '0', '1'};

struct Rocblas {
  rocblas_handle h = nullptr;
  ~Rocblas() {
    if (h) rocblas_destroy_handle(h);
  }
};

#define VC_RB(expr)                                                          \
  do {                                                                       \
    const rocblas_status _s = (expr);                                        \
    if (_s != rocblas_status_success) {                                      \
      set_error("%s failed (rocblas status %d)", #expr, (int)_s);            \
      return VC_ERR_HIP;                                                     \
    }                                                                        \
  } while (0)

vc_status make_handle(Rocblas& rb, hipStream_t st) {
  if (rocblas_create_handle(&rb.h) != rocblas_status_success) {
    rb.h = nullptr;
    set_error("rocblas_create_handle failed");
    return VC_ERR_HIP;
  }
  rocblas_set_stream(rb.h, st);
  return VC_OK;
}

bool pair_ok(int q) { return q >= 0 && q < kToeplitzPairs; }

}  // namespace

// out (c0 x c1 x c2 row-major) = S x_1 U0[:c0] x_2 U1[:c1] x_3 U2[:c2]: three GEMMs,
// the innermost mode first.  Y1: r0 r1 c2 doubles, Y2: r0 c1 c2 doubles.
static vc_status restore_crop(rocblas_handle h, const TuckerPair& tp, const int c[3], double* out, double* Y1,
                              double* Y2) {
  const int r0 = tp.r[0], r1 = tp.r[1], r2 = tp.r[2];
  const double one = 1.0, zero = 0.0;
  // Y1[a][b][t2] = sum_c S[a][b][c] U2[t2][c]
  VC_RB(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, c[2], r0 * r1, r2, &one,
                      tp.U64[2].as<double>(), r2, tp.S64.as<double>(), r2, &zero, Y1, c[2]));
  // Y2[a][t1][t2] = sum_b U1[t1][b] Y1[a][b][t2]
  VC_RB(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, c[2], c[1], r1, &one, Y1,
                                      c[2], (rocblas_stride)r1 * c[2], tp.U64[1].as<double>(), r1, 0, &zero, Y2,
                                      c[2], (rocblas_stride)c[1] * c[2], r0));
  // out[t0][t1 t2] = sum_a U0[t0][a] Y2[a][t1 t2]
  VC_RB(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, c[1] * c[2], c[0], r0, &one, Y2,
                      c[1] * c[2], tp.U64[0].as<double>(), r0, &zero, out, c[1] * c[2]));
  return VC_OK;
}

vc_status toeplitz_restore(const vc_toeplitz_cache* C, int q, const int n[3], double* out, hipStream_t st) {
  if (!pair_ok(q)) { set_error("pair %d outside 0..14", q); return VC_ERR_ARG; }
  int c[3];
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > C->nmax[a]) {
      set_error("grid %d x %d x %d exceeds the cache's %d x %d x %d", n[0], n[1], n[2], C->nmax[0], C->nmax[1],
                C->nmax[2]);
      return VC_ERR_ARG;
    }
    c[a] = n[a] + 1;
  }
  const TuckerPair& tp = C->pair[q];
  DevMem Y1, Y2;
  VC_HIP(Y1.alloc((size_t)tp.r[0] * tp.r[1] * c[2] * sizeof(double)));
  VC_HIP(Y2.alloc((size_t)tp.r[0] * c[1] * c[2] * sizeof(double)));
  Rocblas rb;
  vc_status s = make_handle(rb, st);
  if (s != VC_OK) return s;
  s = restore_crop(rb.h, tp, c, out, Y1.as<double>(), Y2.as<double>());
  if (s != VC_OK) return s;
  VC_HIP(hipStreamSynchronize(st));   // the scratch is freed on return
  return VC_OK;
}

vc_status toeplitz_octant(int q, const int n[3], double* out, const double* gl, hipStream_t st) {
  OctArgs o{};
  pair_axes(q, &o.alpha, &o.beta, &o.want);
  for (int a = 0; a < 3; ++a) o.D[a] = n[a] + 1;
  VC_HIP(launch_fill_octant(out, o, gl, st));
  return VC_OK;
}

}  // namespace vc

using namespace vc;

static double wall_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// host copies of a pair's core and factors (for saving)
static vc_status download_pair(const TuckerPair& tp, const int D[3], std::vector<double>& S,
                               std::vector<double> (&U)[3], hipStream_t st) {
  S.resize((size_t)tp.r[0] * tp.r[1] * tp.r[2]);
  VC_HIP(hipMemcpyAsync(S.data(), tp.S64.p, S.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  for (int m = 0; m < 3; ++m) {
    U[m].resize((size_t)D[m] * tp.r[m]);
    VC_HIP(hipMemcpyAsync(U[m].data(), tp.U64[m].p, U[m].size() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  VC_HIP(hipStreamSynchronize(st));
  return VC_OK;
}

extern "C" vc_status vc_toeplitz_cache_build(const int32_t nmax[3], double tol, int device, void* stream,
                                             vc_toeplitz_cache** out) {
  if (!nmax || !out) { set_error("null argument"); return VC_ERR_ARG; }
  *out = nullptr;
  if (!(tol > 0.0) || tol >= 1.0) { set_error("tol must be in (0, 1)"); return VC_ERR_ARG; }
  for (int a = 0; a < 3; ++a)
    if (nmax[a] < 1 || nmax[a] > 4096) { set_error("nmax[%d] = %d outside 1..4096", a, nmax[a]); return VC_ERR_ARG; }
  // the compression hands the octant's size to rocBLAS / rocSOLVER as 32-bit integers
  const int64_t oct_elems = (int64_t)(nmax[0] + 1) * (nmax[1] + 1) * (nmax[2] + 1);
  if (oct_elems >= ((int64_t)1 << 31)) {
    set_error("octant of %d x %d x %d offsets exceeds 2^31 elements", nmax[0] + 1, nmax[1] + 1, nmax[2] + 1);
    return VC_ERR_ARG;
  }
  const double t0 = wall_s();
  VC_HIP(hipSetDevice(device));
  hipStream_t st = (hipStream_t)stream;
  auto C = std::make_unique<vc_toeplitz_cache>();
  C->device = device;
  C->tol = tol;
  int D[3];
  for (int a = 0; a < 3; ++a) {
    C->nmax[a] = nmax[a];
    D[a] = nmax[a] + 1;
  }
  std::vector<double> gl;
  gauss_legendre_table(gl);
  DevMem dgl, oct;
  VC_HIP(dgl.alloc(gl.size() * sizeof(double)));
  VC_HIP(hipMemcpy(dgl.p, gl.data(), gl.size() * sizeof(double), hipMemcpyHostToDevice));
  VC_HIP(oct.alloc((size_t)D[0] * D[1] * D[2] * sizeof(double)));
  for (int q = 0; q < kToeplitzPairs; ++q) {
    const int n[3] = {nmax[0], nmax[1], nmax[2]};
    vc_status s = toeplitz_octant(q, n, oct.as<double>(), dgl.as<double>(), st);
    if (s != VC_OK) return s;
    s = tucker_compress_tensor(oct.as<double>(), D[0], D[1], D[2], tol, C->pair[q], st);
    if (s != VC_OK) return s;
    s = download_pair(C->pair[q], D, C->hS[q], C->hU[q], st);
    if (s != VC_OK) return s;
  }
  C->build_s = wall_s() - t0;
  *out = C.release();
  return VC_OK;
}

extern "C" vc_status vc_toeplitz_cache_destroy(vc_toeplitz_cache* c) {
  if (c) {
    (void)hipSetDevice(c->device);
    delete c;
  }
  return VC_OK;
}

extern "C" vc_status vc_toeplitz_cache_save(const vc_toeplitz_cache* c, const char* path) {
  if (!c || !path) { set_error("null argument"); return VC_ERR_ARG; }
  FILE* f = std::fopen(path, "wb");
  if (!f) { set_error("cannot open %s for writing", path); return VC_ERR_ARG; }
  bool ok = std::fwrite(kMagic, 1, 8, f) == 8;
  const int32_t hdr[4] = {c->nmax[0], c->nmax[1], c->nmax[2], kToeplitzPairs};
  ok = ok && std::fwrite(hdr, sizeof hdr, 1, f) == 1;
  ok = ok && std::fwrite(&c->tol, sizeof(double), 1, f) == 1;
  for (int q = 0; ok && q < kToeplitzPairs; ++q) {
    const int32_t r[3] = {c->pair[q].r[0], c->pair[q].r[1], c->pair[q].r[2]};
    ok = std::fwrite(r, sizeof r, 1, f) == 1;
    ok = ok && std::fwrite(c->hS[q].data(), sizeof(double), c->hS[q].size(), f) == c->hS[q].size();
    for (int m = 0; ok && m < 3; ++m)
      ok = std::fwrite(c->hU[q][m].data(), sizeof(double), c->hU[q][m].size(), f) == c->hU[q][m].size();
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) { set_error("write to %s failed", path); return VC_ERR_ARG; }
  return VC_OK;
}

static vc_status upload_vec(DevMem& d, const std::vector<double>& h) {
  VC_HIP(d.alloc(h.size() * sizeof(double)));
  VC_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  return VC_OK;
}

extern "C" vc_status vc_toeplitz_cache_load(const char* path, int device, vc_toeplitz_cache** out) {
  if (!path || !out) { set_error("null argument"); return VC_ERR_ARG; }
  *out = nullptr;
  const double t0 = wall_s();
  FILE* f = std::fopen(path, "rb");
  if (!f) { set_error("cannot open %s", path); return VC_ERR_ARG; }
  auto C = std::make_unique<vc_toeplitz_cache>();
  C->device = device;
  char mg[8];
  int32_t hdr[4];
  bool ok = std::fread(mg, 1, 8, f) == 8 && std::memcmp(mg, kMagic, 8) == 0;
  ok = ok && std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[3] == kToeplitzPairs;
  ok = ok && std::fread(&C->tol, sizeof(double), 1, f) == 1;
  int D[3] = {0, 0, 0};
  for (int a = 0; ok && a < 3; ++a) {
    ok = hdr[a] >= 1 && hdr[a] <= 4096;
    C->nmax[a] = hdr[a];
    D[a] = hdr[a] + 1;
  }
  for (int q = 0; ok && q < kToeplitzPairs; ++q) {
    int32_t r[3];
    ok = std::fread(r, sizeof r, 1, f) == 1;
    for (int m = 0; ok && m < 3; ++m) ok = r[m] >= 1 && r[m] <= D[m];
    if (!ok) break;
    for (int m = 0; m < 3; ++m) C->pair[q].r[m] = r[m];
    C->hS[q].resize((size_t)r[0] * r[1] * r[2]);
    ok = std::fread(C->hS[q].data(), sizeof(double), C->hS[q].size(), f) == C->hS[q].size();
    for (int m = 0; ok && m < 3; ++m) {
      C->hU[q][m].resize((size_t)D[m] * r[m]);
      ok = std::fread(C->hU[q][m].data(), sizeof(double), C->hU[q][m].size(), f) == C->hU[q][m].size();
    }
  }
  char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;   // nothing after the last pair
  std::fclose(f);
  if (!ok) { set_error("%s is not a Toeplitz cache of this library (bad header, size or ranks)", path); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(device));
  for (int q = 0; q < kToeplitzPairs; ++q) {
    vc_status s = upload_vec(C->pair[q].S64, C->hS[q]);
    for (int m = 0; s == VC_OK && m < 3; ++m) s = upload_vec(C->pair[q].U64[m], C->hU[q][m]);
    if (s != VC_OK) return s;
  }
  C->build_s = wall_s() - t0;
  *out = C.release();
  return VC_OK;
}

extern "C" vc_status vc_toeplitz_cache_info(const vc_toeplitz_cache* c, int32_t nmax[3], double* tol,
                                            int32_t ranks[45], double* stored_numbers, double* seconds) {
  if (!c) { set_error("null cache"); return VC_ERR_ARG; }
  if (nmax)
    for (int a = 0; a < 3; ++a) nmax[a] = c->nmax[a];
  if (tol) *tol = c->tol;
  double n = 0.0;
  for (int q = 0; q < kToeplitzPairs; ++q) {
    const TuckerPair& tp = c->pair[q];
    if (ranks)
      for (int m = 0; m < 3; ++m) ranks[3 * q + m] = tp.r[m];
    n += (double)tp.r[0] * tp.r[1] * tp.r[2];
    for (int m = 0; m < 3; ++m) n += (double)(c->nmax[m] + 1) * tp.r[m];
  }
  if (stored_numbers) *stored_numbers = n;
  if (seconds) *seconds = c->build_s;
  return VC_OK;
}

extern "C" vc_status vc_toeplitz_cache_restore(const vc_toeplitz_cache* c, int32_t pair, const int32_t n[3],
                                               double* out, void* stream) {
  if (!c || !n || !out) { set_error("null argument"); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(c->device));
  const int nn[3] = {n[0], n[1], n[2]};
  return toeplitz_restore(c, pair, nn, out, (hipStream_t)stream);
}

extern "C" vc_status vc_toeplitz_octant(int32_t pair, const int32_t n[3], int device, double* out, void* stream) {
  if (!n || !out) { set_error("null argument"); return VC_ERR_ARG; }
  if (!(pair >= 0 && pair < kToeplitzPairs)) { set_error("pair %d outside 0..14", pair); return VC_ERR_ARG; }
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1 || n[a] > 4096) { set_error("n[%d] = %d outside 1..4096", a, n[a]); return VC_ERR_ARG; }
  VC_HIP(hipSetDevice(device));
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> gl;
  gauss_legendre_table(gl);
  DevMem dgl;
  VC_HIP(dgl.alloc(gl.size() * sizeof(double)));
  VC_HIP(hipMemcpy(dgl.p, gl.data(), gl.size() * sizeof(double), hipMemcpyHostToDevice));
  const int nn[3] = {n[0], n[1], n[2]};
  vc_status s = toeplitz_octant(pair, nn, out, dgl.as<double>(), st);
  if (s != VC_OK) return s;
  VC_HIP(hipStreamSynchronize(st));   // the node table is freed on return
  return VC_OK;
}

extern "C" vc_status vc_setup_toeplitz_source(vc_problem* p, const vc_toeplitz_cache* c) {
  if (!p) { set_error("null problem"); return VC_ERR_ARG; }
  if (c) {
    if (c->device != p->device) { set_error("cache on device %d, problem on device %d", c->device, p->device); return VC_ERR_ARG; }
    if (p->nx > c->nmax[0] || p->ny > c->nmax[1] || p->nz > c->nmax[2]) {
      set_error("grid %d x %d x %d exceeds the cache's %d x %d x %d", p->nx, p->ny, p->nz, c->nmax[0], c->nmax[1],
                c->nmax[2]);
      return VC_ERR_ARG;
    }
  }
  p->tz_cache = c;
  return VC_OK;
}
