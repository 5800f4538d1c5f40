// Host-visible declarations of the FFT-product pass kernels (see mvp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_core.hpp"

namespace vc {

// Elements a thread stages per FFT stage of the z and strided kernels (launches keep
// L*ncol <= emax*threads), chosen so no kernel needs scratch memory under a 1024-thread
// launch bound (128 VGPRs).
template <typename T> struct Tune {
  static constexpr int emax = sizeof(T) == 4 ? 16 : 8;
  // largest FFT radix compiled into the z and strided kernels (register budget)
  static constexpr int maxr = sizeof(T) == 4 ? 21 : 12;
};
// Dynamic LDS per workgroup: tiles are chosen within 64 KiB (several workgroups per
// CU); a transform too long for that falls back to the device's per-workgroup maximum
// (160 KiB on gfx950), queried at setup.
constexpr size_t kLdsBudget = 64 * 1024;
size_t lds_ext_budget();
void note_device_lds(int device);

// Up to six field components handled by one strided launch (blockIdx.z = comp*nrhs+rhs).
struct CompSet {
  int n;
  int comp[6];   // component index in the work array
  int axis[6];   // panel normal axis of the component (selects its line/plane flags)
  int min_[6];   // flag bits a row must have to be loaded (0 = load all rows < nin)
  int mout[6];   // flag bits a row must have to be stored (0 = store all rows < nout)
};

struct StridedArgs {
  int64_t comp_stride, rhs_stride, plane_stride, row_stride;
  int ncols;      // columns along the contiguous axis (H)
  int ncol;       // columns per workgroup tile
  int nin, nout;  // rows loaded (rest zero) / rows stored
  int nrhs;
  int inverse;
  int n1x, n1y;   // flag array extents (planes x rows)
  int lgc;        // log2(ncol), set by the launcher
  const int* skip;   // optional device flag: when set, the launch does nothing
  const int* act;    // optional per right-hand side activity: workgroups of inactive ones return
  // optional half-voxel phase along the transformed axis (L complex; null: none): the
  // components of normal axis phax take ph[k] on the forward outputs and conj(ph[k]) on
  // the inverse inputs
  const void* ph;
  int phax;
};

// y pass with register-edge stages (ypass_impl.hpp): blockIdx = (kz tile, x plane,
// component * nrhs + rhs)
struct YArgs {
  int64_t comp_stride, rhs_stride, plane_stride, row_stride;
  int ncols;        // kz columns (H)
  int ncol;         // columns per workgroup, 1..32
  int nin, nout;    // rows loaded (rest zero) / rows stored, each also filtered by line flags
  int nrhs, inverse, n1x, n1y;
  int L, nst, tl;   // y length, stages (radices f0 >= ... >= RS in radpack), L / RS
  uint32_t radpack;
  CompSet cs;
  const int* skip;  // optional device flag: when set, the launch does nothing
  const int* act;   // optional per right-hand side activity
  int xg;           // 2 or 4: that many consecutive tiles of a row (which share cache
                    // lines) per XCD, issued together; -1: all tiles of a row; 0 or 1:
                    // the launch order
  const void* ph;   // optional half-voxel phase along y, as StridedArgs::ph
  int phax;
};
template <typename T>
hipError_t launch_ypass(void* data, const YArgs& a, const void* tw, const uint8_t* lflag, const uint8_t* pflag,
                        int nplanes, int nthr, hipStream_t st);
// the register-edge y pass of several scenes in one launch (members with last radix rs)
struct YScene {
  YArgs a;            // a.skip / a.act unused: the call's flags apply
  void* data;
  const void* tw;
  const uint8_t* lflag;
  const uint8_t* pflag;
  int c0, gx, gy, blk0;   // first column; tiles, planes; first linear workgroup
};
template <typename T>
// cpt: columns per thread of the kernel that will run (ypass_cols_per_thread; the
// multi-scene kernel always takes 1)
bool ypass_args_ok(const YArgs& a, int nthr, bool flags, size_t* lds, int cpt = 1);
template <typename T>
hipError_t launch_ypass_multi(const YScene* tab, int nscene, int nblocks, int rs, int nthr, size_t lds,
                              const int* skip, const int* act, hipStream_t st);
// plan and tile of the y pass for length L over ncols kz columns (fewest stages, largest
// last radix, then the tile that keeps lanes and columns busy and reads whole 128-byte
// row lines); false when none fits
bool ypass_config(int L, int elem, int ncols, size_t budget, YArgs* a, int* nthr);

// Tucker form of one stored pair for the fused x pass (eq. 13): the factor U1 (Hx x r1p,
// row-major) and the strip T2 = S x2 U2 x3 U3 (Hy x H x r1p, r fastest), in the
// product's precision; r1p = r1 rounded up to 4, zero past r1 in both
struct TkPairDev {
  const void* U1;    // [Hx][r1p] (FP64 table)
  const void* T2;    // [Hy][H][r1p]
  const void* U1t;   // FP32 table: U1 transposed, [r1q][hxp] (zero filled)
  int r1, r1p, r1q, hxp;
};

struct SandArgs {
  int64_t comp_stride, rhs_stride, pair_stride;
  int nrhs, n1x, Mx, My, H, Hx, Hy;
  int ncol;       // (ky, kz) columns per workgroup, 1..32
  int adjoint;
  int nin, nout;
  // x transform: radices r_0 >= ... >= r_{nst-1} (product Mx), r_s in bits 5s..5s+4
  // of radpack (a packed word, so the kernel never indexes an argument array); the
  // last one is the register stage, tl = Mx / r_{nst-1} threads per column
  int nst, tl;
  uint32_t radpack;
  // bits 3q..3q+2: stored spectrum of pair q is odd under k_a -> M_a - k_a (bit a)
  uint64_t oddmask;
  const int* skip;   // optional device flag: when set, the launch does nothing
  const int* act;    // optional per right-hand side activity: workgroups of inactive ones return
  // Tucker-fused form (null: the stored spectra R): per stored pair its U1 and T2
  // (device table of npairs entries); one workgroup per tile runs every right-hand side
  const TkPairDev* tk;
  int npairs;
  int tk_r1max;   // largest x-mode rank r1 over the pairs
  // staged form (stored spectra, tk null): one workgroup per tile copies the tile's
  // stored spectra of the npairs pairs into LDS once and runs every right-hand side
  // against them (the fused form's structure, with a copy in place of the build)
  int stage;
};
// dynamic LDS of the sandwich: twiddle table (+ the x phases in FP32) + one [L][ncol]
// tile + 3 n1x plane flags
inline size_t sandwich_lds_bytes(int L, int ncol, int elem, int n1x) {
  return (size_t)2 * elem * ((size_t)(elem == 4 ? 2 : 1) * L + (size_t)L * ncol) + (size_t)3 * n1x;
}
// the fused form: the tile's spectra [npairs][Hx][ncol] (16-byte aligned) + one [L][ncol]
// tile + 3 n1x plane flags (the twiddles and x phases stay in global memory)
inline size_t sandwich_tk_lds_bytes(int L, int ncol, int elem, int n1x, int npairs, int Hx) {
  return (((size_t)npairs * Hx * ncol * elem + 15) & ~(size_t)15) + (size_t)2 * elem * L * ncol + (size_t)3 * n1x;
}
// x-transform plan of the sandwich for one precision / variant (see sandwich_impl.hpp):
// fewest stages with the first radix <= rmax, middle radices <= rmid and the last
// (smallest) radix <= rs_max, at most max_tl threads per column; nst = -1 when none
AxisPlan make_sandwich_plan(int L, int rmax, int rmid, int rs_max, int max_tl);
constexpr int kSandMaxStages = 6;
constexpr int sandwich_rmid(int elem) { return elem == 4 ? 10 : 10; }
// Register-edge transform plans (x pass and y pass) compiled with their radices, stage
// count and length as constants (entry 0: the generic kernels, which read them from
// their arguments).  A launch whose runtime plan equals an entry uses that entry's
// kernel; every other plan runs the generic one.
// `wide`: the FP32 three-input x-pass kernel of the plan is compiled for workgroups of up
// to 1024 threads (its registers fit 128 VGPRs), so long transforms, which need L/RS
// threads per column, still get several columns per workgroup.
struct SandFixedPlan {
  int L, nst, r[4];
  bool wide;
};
constexpr SandFixedPlan kSandFixed[] = {
    {0, 0, {0, 0, 0, 0}, false},
    {36, 3, {4, 3, 3, 0}, false},
    {140, 3, {7, 5, 4, 0}, false},
    {270, 3, {9, 6, 5, 0}, false},
    {540, 3, {10, 9, 6, 0}, false},
    {540, 4, {10, 6, 3, 3}, true},
    {1050, 4, {7, 6, 5, 5}, true},
    {36, 2, {6, 6, 0, 0}, false},
};
constexpr int kSandNumFixed = (int)(sizeof(kSandFixed) / sizeof(kSandFixed[0]));
constexpr uint32_t sand_fixed_pack(int id) {
  uint32_t p = 0;
  for (int s = 0; s < kSandFixed[id].nst; ++s) p |= (uint32_t)kSandFixed[id].r[s] << (5 * s);
  return p;
}
constexpr int sand_fixed_last(int id) { return kSandFixed[id].nst > 0 ? kSandFixed[id].r[kSandFixed[id].nst - 1] : 0; }
// table entry of a runtime plan (0: none)
inline int sand_fixed_id(int L, int nst, uint32_t radpack) {
  for (int id = 1; id < kSandNumFixed; ++id)
    if (kSandFixed[id].L == L && kSandFixed[id].nst == nst && sand_fixed_pack(id) == radpack) return id;
  return 0;
}
// most threads per workgroup of the x-pass kernel that runs a plan
constexpr int sand_max_threads_fixed(int id, int elem, int nin) {
  return (id > 0 && kSandFixed[id].wide && elem == 4 && nin == 3) ? 1024 : 512;
}
inline int sand_max_threads(int L, int nst, uint32_t radpack, int elem, int nin) {
  return sand_max_threads_fixed(sand_fixed_id(L, nst, radpack), elem, nin);
}
// Columns per thread of the single-scene register-edge y pass: 2 for FP32 tiles of even
// width whose plan is compiled (each thread transforms two adjacent columns, so a tile
// needs half the threads), else 1.
inline int ypass_cols_per_thread(int L, int nst, uint32_t radpack, int tl, int ncol, int elem) {
  const int id = sand_fixed_id(L, nst, radpack);
  return (elem == 4 && id > 0 && ncol % 2 == 0 && tl * sand_fixed_last(id) == L) ? 2 : 1;
}

template <typename T>
hipError_t launch_zfwd(const double* x, int64_t N, int nrhs, int mode, const int32_t* items, int nitems,
                       const int32_t* line_ptr, const int32_t* pk, const int8_t* pkind, void* F, int64_t comp_stride,
                       int64_t rhs_stride, int n1x, int n1y, int My, int H, const AxisPlan& pl, const void* tw, int ncol,
                       int nthr, const int* skip, hipStream_t st, const int* act = nullptr, const void* ph = nullptr);
template <typename T>
hipError_t launch_strided(void* data, const StridedArgs& a, const CompSet& cs, int nplanes, const AxisPlan& pl,
                          const void* tw, const uint8_t* lflag, const uint8_t* pflag, int nthr, hipStream_t st);
// e0 / e1 (optional): events the launch itself stamps at the kernel's start and end
// (no separate event packets around it)
template <typename T>
hipError_t launch_sandwich(const void* Fin, void* Fout, const void* R, const SandArgs& a, const void* tw,
                           const void* phx, const uint8_t* pflag, int nthr,
                           hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// a sandwich launch configuration (plan, tile, threads)
struct SandCfg {
  int nst, tl, ncol, nthr;
  uint32_t radpack;
  int stage = 0;   // the staged form of the stored spectra (SandArgs::stage)
};
// one sandwich variant (NIN input / NOUT output components, TK: Tucker-fused), last-stage
// radix rs
template <typename T, int NIN, int NOUT, int TK>
hipError_t launch_sandwich_v(const void* Fin, void* Fout, const void* R, const SandArgs& a, const void* tw,
                             const void* phx, const uint8_t* pflag, int nthr,
                             size_t lds, int rs, hipStream_t st, hipEvent_t e0, hipEvent_t e1);
// largest last-stage radix compiled for each sandwich variant (registers: NIN x RS held values)
constexpr int sandwich_rs_max(int elem, int nin) { return elem == 4 ? (nin == 3 ? 6 : 7) : (nin == 3 ? 5 : 3); }
constexpr int sandwich_rmax(int elem) { return elem == 4 ? 10 : 10; }
template <typename T>
hipError_t launch_zinv(const void* O, double* y, const double* x, int64_t N, int nrhs, int mode, const int32_t* items,
                       int nitems, const int32_t* line_ptr, const int32_t* pk, const int8_t* pkind,
                       const double* diag, const uint8_t* lflag, int64_t comp_stride, int64_t rhs_stride, int n1x,
                       int n1y, int My, int H, const AxisPlan& pl, const void* tw, int ncol, int nthr,
                       const int* skip, hipStream_t st, const int* act = nullptr, const void* ph = nullptr);

// ---- one launch per pass over several independent problems ("scenes") of different
// sizes: a device table holds every scene's arguments and its first linear workgroup
// (blk0, increasing); a workgroup finds its scene by binary search on blk0.
// z pass of one scene (forward scatter + R2C, or C2R + gather); the panel vectors of
// scene s are columns c0 .. c0+nrhs-1 of the call's x / y (column stride ldx).
struct ZScene {
  const int32_t* items;
  const int32_t* line_ptr;
  const int32_t* pk;
  const int8_t* pkind;
  const double* diag;
  const uint8_t* lflag;
  void* F;            // spectral work array (written by the forward pass, read by the inverse)
  const void* tw;
  const void* ph;     // half-voxel phase along z (null: none): z-normal components take ph[kz]
                      // after the forward transform and conj(ph[kz]) before the inverse
  AxisPlan pl;
  int64_t comp_stride, rhs_stride;
  int nitems, nrhs, n1x, n1y, My, H, lgc;
  int c0;             // first column of the scene
  int gx;             // workgroups along the line items (the rest index right-hand sides)
  int blk0;
};
struct StridedScene {
  StridedArgs a;      // a.act is unused: the call's activity array (offset by c0) applies
  CompSet cs;
  AxisPlan pl;
  void* data;
  const void* tw;
  const uint8_t* lflag;
  const uint8_t* pflag;
  int c0, gx, gy, blk0;
};
struct SandScene {
  SandArgs a;         // a.skip / a.act unused: the call's flags apply
  const void* Fin;
  void* Fout;
  const void* R;
  const void* tw;
  const void* phx;
  const uint8_t* pflag;
  int c0, ntiles, blk0;
};
template <typename T>
hipError_t launch_zfwd_multi(const ZScene* tab, int nscene, int nblocks, const double* x, int64_t ldx,
                             const int* skip, const int* act, int nthr, size_t lds, hipStream_t st);
template <typename T>
hipError_t launch_zinv_multi(const ZScene* tab, int nscene, int nblocks, const double* x, double* y, int64_t ldx,
                             const int* skip, const int* act, int nthr, size_t lds, hipStream_t st);
template <typename T>
hipError_t launch_strided_multi(const StridedScene* tab, int nscene, int nblocks, const int* skip, const int* act,
                                int nthr, size_t lds, hipStream_t st);
template <typename T, int NIN, int NOUT>
hipError_t launch_sandwich_multi_v(const SandScene* tab, int nscene, int nblocks, const int* skip, const int* act,
                                   int nthr, size_t lds, int rs, hipStream_t st);
// LDS bytes of the z / strided kernels for transform length L and ncol lines
size_t zs_lds_bytes(int elem, int L, int ncol);
// host-side check of one sandwich configuration (what the kernel assumes); false = invalid
template <typename T> bool sandwich_args_ok(const SandArgs& a, int nthr);

// setup kernels (setup_kernels.hip)
struct FillArgs {
  int alpha, beta, want;   // want 0 = P (eq. 5), 1 = E (eq. 6)
  int Mx, My, Mz;
  int no[3], ns[3];        // observer / source panel counts per axis
  double scale;            // folded inverse-FFT normalisation 1/(Mx My Mz)
};
hipError_t launch_fill_circulant(double* C, const FillArgs& a, const double* gl_nodes, hipStream_t st);
hipError_t launch_zr2c_dense(const double* in, void* out, int nlines, int H, const AxisPlan& pl, const void* tw,
                             int ncol, int nthr, hipStream_t st);
struct ExtractArgs {
  int Mx, My, Mz, H, Hx, Hy;
  int kind;                // 0: P diagonal pair, 1: P off-diagonal, 2: E
  int alpha, beta;
  int64_t pair_off;        // element offset of this pair in the stored arrays
};
hipError_t launch_extract(const void* spec, double* R64, float* R32, const ExtractArgs& a, double* resid,
                          hipStream_t st);
// panel-integral kernel for host tables (preconditioner blocks): out[i] = K(alpha,beta,d_i)
hipError_t launch_kernel_table(const double* d, int n, int alpha, int beta, int want, double* out,
                               const double* gl_nodes, hipStream_t st);

// solver kernels (solver_kernels.hip)
hipError_t launch_gemv_t(const double* V, int64_t ldv, int64_t N, int k, const double* w, int64_t ldw, int nrhs,
                         double* h, int64_t ldh, const int* active, double* partial, hipStream_t st);
int64_t gemv_t_partial_size(int64_t N, int kmax, int nrhs);
hipError_t launch_gemv_n_sub(const double* V, int64_t ldv, int64_t N, int k, const double* h, int64_t ldh,
                             double* w, int64_t ldw, int nrhs, const int* active, int accumulate_into_h2,
                             hipStream_t st, const int* kcol = nullptr);
hipError_t launch_colnorm(const double* w, int64_t ldw, int64_t N, int nrhs, double* out, double* partial,
                          hipStream_t st, const int* skip = nullptr);
int64_t colnorm_partial_size(int64_t N, int nrhs);
hipError_t launch_scale_cols(double* w, int64_t ldw, int64_t N, int nrhs, const double* s, int mode,
                             hipStream_t st);
hipError_t launch_axpy_cols(double* y, const double* x, int64_t N, int nrhs, const double* a, int sub,
                            hipStream_t st, const int* skip = nullptr);
hipError_t launch_diag_scale(const double* x, double* y, const double* dinv, int64_t N, int nrhs, const int* skip,
                             hipStream_t st, int64_t dinv_ld = 0);
hipError_t launch_block_apply(const double* x, double* y, int64_t N, int nrhs, const int32_t* box_ptr,
                              const int32_t* box_panels, const int32_t* box_block, const int64_t* block_off,
                              const int32_t* block_n, const double* blocks, int nbox, const int* skip,
                              hipStream_t st, const int32_t* box_c0 = nullptr, const int32_t* box_nc = nullptr,
                              int trans = 0);
// device-side GMRES cycle (one thread per right-hand side, nrhs <= 256)
hipError_t launch_cycle_start(int nrhs, int m, const double* rn, const double* bn, const double* rtol, int* act_cycle,
                              int* act_step, double* g, double* scal, int* kd, int* skip, double* rre_out,
                              hipStream_t st);
// what the host reads after a segment of the relaxed mixed form (2 + nrhs doubles):
// the largest residual estimate of an iterating column, the step-level skip flag,
// iteration counts
hipError_t launch_relax_state(int nrhs, int m, const double* g, const int* kd, const int* act_step, const double* bn,
                              const int* iters, const int* skip, double* out, hipStream_t st);
hipError_t launch_arnoldi(int j, int nrhs, int m, const double* h1, const double* h2, int ldh, const double* hn,
                          double* H, double* cs, double* sn, double* g, const double* bn, const double* rtol,
                          int* act_step, int* kd, int* iters, double* scal, int* skip, int* bad, hipStream_t st);
// One Arnoldi step after the product w = A z: CGS twice, |w| and the Givens update in
// three launches (k = j + 1 basis vectors, nrhs <= 256).  cnt: cgs_counter_size(kmax,
// nrhs) zeroed unsigned counters (each launch leaves them zero); partial: as for
// launch_gemv_t; nrm_out: |w| per active column.
hipError_t launch_cgs_step(const double* V, int64_t ldv, int64_t N, int k, double* w, int nrhs, double* h1,
                           double* h2, int ldh, double* partial, unsigned* cnt, int j, int m, double* H, double* cs,
                           double* sn, double* g, const double* bn, const double* rtol, int* act_step, int* kd,
                           int* iters, double* scal, int* skip, int* bad, double* nrm_out, hipStream_t st);
int64_t cgs_counter_size_a(int kmax, int nrhs);
// partials of the Gram-Schmidt launches (doubles), k <= kmax basis vectors
int64_t cgs_partial_size(int64_t N, int kmax, int nrhs);
int64_t cgs_counter_size(int kmax, int nrhs);
hipError_t launch_backsolve(int nrhs, int m, const double* H, const double* g, const int* kd, const int* act_cycle,
                            double* y, int ldy, hipStream_t st);
hipError_t launch_scale_copy(double* dst, const double* src, int64_t N, int nrhs, const double* s, const int* skip,
                             hipStream_t st);
hipError_t launch_zero(double* p, int64_t n, hipStream_t st);
// b[j N + k] = 1 where pcond[k] == j, else 0 (k < N, j < m): the unit-potential
// right-hand sides of the m conductors
hipError_t launch_unit_rhs(double* b, const int32_t* pcond, int64_t N, int m, hipStream_t st);
// p[0..n) = 0 (a kernel: no memset node when captured)
hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t st);
hipError_t launch_add_active(double* x, const double* z, int64_t N, int nrhs, const int* act, const int* skip,
                             hipStream_t st);
hipError_t launch_cap_reduce(const double* rho, int64_t N, int m, const int32_t* cond_panels,
                             const int32_t* cond_ptr, const double* weight, double scale, double* C,
                             hipStream_t st);

// Tucker rebuild GEMMs (tucker_kernels.hip): C[z] = A[z] B[z] with element strides
struct GemmArgs {
  int M, N, K, batch;
  int64_t sam, sak, sbk, sbn, scm, scn;   // A[m][k], B[k][n], C[m][n]
  int64_t bsa, bsb, bsc;                  // batch strides
  const int* skip;                        // optional device flag: when set, the launch does nothing
};
template <typename T>
hipError_t launch_mfma_gemm(const T* A, const T* B, T* C, const GemmArgs& g, hipStream_t st);
// one GEMM of a multi-GEMM launch: C[z] = A[z] B[z] (element strides as GemmArgs)
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int M, N, K, batch;
  int64_t sam, sak, sbk, sbn, scm, scn;
  int64_t bsa, bsb, bsc;
  int gx, gy, blk0;   // set by gemm_table_layout
};
int gemm_table_layout(GemmDesc* d, int n);
template <typename T>
hipError_t launch_mfma_gemm_multi(const GemmDesc* tab, int ndesc, int nblocks, const int* skip, hipStream_t st);
hipError_t launch_to_f32(const double* in, float* out, int64_t n, hipStream_t st);
hipError_t launch_swap01(const double* in, double* out, int A, int B, int C, hipStream_t st);

hipError_t launch_cap_reduce_n(const double* rho, int64_t N, int m, int nrhs, const int32_t* cond_panels,
                               const int32_t* cond_ptr, const double* weight, double scale, double* C,
                               hipStream_t st);
hipError_t launch_cap_reduce_adj(const double* gC, int64_t N, int nrhs, const int32_t* pcond, const double* weight,
                                 double scale, double* grho, hipStream_t st);
hipError_t launch_grad_eps(const int32_t* bptr, const int32_t* ek, const int32_t* econd, const double* ecoef,
                           const double* rho, const double* lam, int64_t N, int m, int nblocks, double scale,
                           double* dC, hipStream_t st);

}  // namespace vc
