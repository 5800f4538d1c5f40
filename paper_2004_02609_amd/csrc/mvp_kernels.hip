// Pass kernels of the FFT product of eq. (11) (Sec. II.B) for gfx950.
//
// Data layout of every spectral work array (one per field component and right-hand
// side): [x < n1x][ky < My][kz < H] complex, kz contiguous, H = Mz/2 + 1.  Only x
// planes that can hold panels (x < n1x = Nx + 1) are ever stored: the inputs are zero
// beyond them and the outputs are only needed there, so the x transform (the middle
// "sandwich" pass) reads and writes half of the x extent.
//
//  k_zfwd     scatter panel charges into z lines and transform them (R2C along z),
//             two real lines per complex transform
//  k_strided  C2C along a strided axis (y, or x during setup) on tiles of `ncol`
//             consecutive kz columns, with row pruning from per-line flags
//  (the x transform with the block multiply is in sandwich_impl.hpp)
//  k_zinv     inverse z transform (C2R) of the lines that hold panels, fused with the
//             gather, the jump term of eq. (7) and the FP64 result
#include "fft_core.hpp"
#include "mvp_kernels.h"

namespace vc {

template <typename T> __device__ __forceinline__ C2<T> ld(const C2<T>* p) { return *p; }

// Panels of one tile of z lines.  Items are the lines holding panels in line order and
// line_ptr is the panels' CSR over all lines, so the panels of the tile's consecutive
// items form one contiguous range; lp[c] is the first panel of tile column c and lp[nc]
// one past the last, sl[c] the line of column c.  Returns nc (columns of this tile, >= 1
// whenever item0 < nitems).
__device__ __forceinline__ int tile_panels(const int32_t* __restrict__ items, const int32_t* __restrict__ line_ptr,
                                           int item0, int nitems, int ncol, int* lp, int* sl) {
  const int nc = min(ncol, nitems - item0);
  const int tid = threadIdx.x;
  if (nc > 0 && tid <= nc) {
    const int line = items[item0 + (tid < nc ? tid : nc - 1)];
    if (tid < nc) sl[tid] = line;
    lp[tid] = line_ptr[tid < nc ? line : line + 1];
  }
  __syncthreads();
  return nc;
}
// tile column of panel p: the last c < nc with lp[c] <= p (every line of the tile holds
// a panel, so lp is strictly increasing); nc <= 32
__device__ __forceinline__ int panel_col(const int* lp, int nc, int p) {
  int c = 0;
#pragma unroll
  for (int st = 16; st > 0; st >>= 1)
    if (c + st < nc && lp[c + st] <= p) c += st;
  return c;
}

// ------------------------------------------------------------------------------ z forward
// Tiles hold 2^lgc lines; divisions by non-powers of two use fdiv (exact in range).
// Workgroup (bx, by): lines bx*ncol .. of the item list, right-hand side(s) by (two per
// complex transform in mode 0).  x: the scene's first column, column stride ldx.
template <typename T>
__device__ __forceinline__ void zfwd_body(const ZScene& a, int mode, const double* __restrict__ x, int64_t ldx,
                                          const int* __restrict__ act, int bx, int by) {
  const int nrhs = a.nrhs;
  const int ra = (mode == 0) ? 2 * by : by;
  const int rb = (mode == 0) ? ra + 1 : -1;
  if (act && !act[ra] && !(rb >= 0 && rb < nrhs && act[rb])) return;   // uniform per workgroup
  extern __shared__ char smem_raw[];
  const AxisPlan& pl = a.pl;
  const int L = pl.L;
  const int lgc = a.lgc, ncol = 1 << lgc, ncolp = ncol + 1;
  const int nitems = a.nitems, n1x = a.n1x, n1y = a.n1y, My = a.My, H = a.H;
  const int64_t comp_stride = a.comp_stride, rhs_stride = a.rhs_stride;
  const int32_t* __restrict__ items = a.items;
  const int32_t* __restrict__ line_ptr = a.line_ptr;
  const int32_t* __restrict__ pk = a.pk;
  const int8_t* __restrict__ pkind = a.pkind;
  C2<T>* __restrict__ F = static_cast<C2<T>*>(a.F);
  const C2<T>* __restrict__ twg = static_cast<const C2<T>*>(a.tw);
  const C2<T>* __restrict__ phz = static_cast<const C2<T>*>(a.ph);
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  C2<T>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  __shared__ int lp[33], sl[32];
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  for (int e = tid; e < L * ncolp; e += nthr) buf[e] = C2<T>{T(0), T(0)};
  const int item0 = bx * ncol;
  const int nc = tile_panels(items, line_ptr, item0, nitems, ncol, lp, sl);   // (synchronises)
  // scatter: all threads over the tile's panels at once
  for (int p = (nc > 0 ? lp[0] : 0) + tid; nc > 0 && p < lp[nc]; p += nthr) {
    const int c = panel_col(lp, nc, p);
    const int k = pk[p];
    double re, im;
    if (mode == 0) {
      re = x[(int64_t)ra * ldx + p];
      im = (rb < nrhs) ? x[(int64_t)rb * ldx + p] : 0.0;
    } else {
      const double v = x[(int64_t)ra * ldx + p];
      re = pkind[p] == 0 ? v : 0.0;
      im = pkind[p] == 0 ? 0.0 : v;
    }
    buf[k * ncolp + c] = C2<T>{T(re), T(im)};
  }
  __syncthreads();
  const C2<T>* res = lds_fft<T, Tune<T>::maxr>(buf, buf2, tw, pl, lgc, ncolp, false);
  const int plane = n1x * n1y;
  const float invH = 1.0f / (float)H, invPl = 1.0f / (float)plane, invN1y = 1.0f / (float)n1y;
  for (int e = tid; e < H * ncol; e += nthr) {
    const int c = fdiv(e, invH), k = e - c * H;
    if (c >= nc) continue;
    const int line = sl[c];
    const int axis = fdiv(line, invPl);
    const int rem = line - axis * plane;
    const int xi = fdiv(rem, invN1y), yi = rem - xi * n1y;
    const C2<T> Z = res[k * ncolp + c];
    const C2<T> Zc = cconj(res[(k == 0 ? 0 : L - k) * ncolp + c]);
    C2<T> A = {T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y + Zc.y)};
    C2<T> B = {T(0.5) * (Z.y - Zc.y), T(-0.5) * (Z.x - Zc.x)};
    if (phz && axis == 2) {
      // half-voxel shift of the z-normal component to the common lattice
      const C2<T> w = phz[k];
      A = cmul(A, w);
      B = cmul(B, w);
    }
    const int64_t off = ((int64_t)xi * My + yi) * H + k;
    if (mode == 0) {
      F[axis * comp_stride + ra * rhs_stride + off] = A;
      if (rb < nrhs) F[axis * comp_stride + rb * rhs_stride + off] = B;
    } else {
      F[axis * comp_stride + ra * rhs_stride + off] = A;
      F[(3 + axis) * comp_stride + ra * rhs_stride + off] = B;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(1024)
k_zfwd(ZScene a, int mode, const double* __restrict__ x, int64_t ldx, const int* __restrict__ skip,
       const int* __restrict__ act) {
  if (skip && *skip) return;
  zfwd_body<T>(a, mode, x, ldx, act, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ void __launch_bounds__(1024)
k_zfwd_multi(const ZScene* __restrict__ tab, int nscene, const double* __restrict__ x, int64_t ldx,
             const int* __restrict__ skip, const int* __restrict__ act) {
  if (skip && *skip) return;
  const int lin = blockIdx.x;
  const ZScene& a = tab[find_scene(tab, nscene, lin)];
  const int local = lin - a.blk0;
  const int by = local / a.gx, bx = local - by * a.gx;
  zfwd_body<T>(a, 0, x + (int64_t)a.c0 * ldx, ldx, act ? act + a.c0 : nullptr, bx, by);
}

// ------------------------------------------------------------------------------ strided C2C
// Workgroup (bx, plane, bz = component * nrhs + rhs).
template <typename T>
__device__ __forceinline__ void strided_body(C2<T>* __restrict__ data, const StridedArgs& a, const CompSet& cs,
                                             const AxisPlan& pl, const C2<T>* __restrict__ twg,
                                             const uint8_t* __restrict__ lflag, const uint8_t* __restrict__ pflag,
                                             const int* __restrict__ act, int bx, int plane, int bz) {
  const int nrhs = a.nrhs;
  const int cz = bz / nrhs, rhs = bz - cz * nrhs;
  if (act && !act[rhs]) return;   // uniform per workgroup
  const int comp = cs.comp[cz], axis = cs.axis[cz];
  const int min_ = cs.min_[cz], mout = cs.mout[cz];
  const int need = a.inverse ? mout : min_;
  const int n1x = a.n1x, n1y = a.n1y;
  if (pflag && need && !(pflag[axis * n1x + plane] & need)) return;  // uniform per block
  extern __shared__ char smem_raw[];
  const int L = pl.L;
  const int lgc = a.lgc, ncol = 1 << lgc, ncolp = ncol + 1, cmask = ncol - 1;
  const int nin = a.nin, nout = a.nout, ncols = a.ncols, inverse = a.inverse;
  const int64_t row_stride = a.row_stride;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  C2<T>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  C2<T>* base = data + comp * a.comp_stride + rhs * a.rhs_stride + plane * a.plane_stride;
  const int col0 = bx * ncol;
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  const uint8_t* lf = lflag ? lflag + ((int64_t)axis * n1x + plane) * n1y : nullptr;
  // half-voxel phase of this component along the transformed axis (null: none)
  const C2<T>* __restrict__ ph = (a.ph && axis == a.phax) ? static_cast<const C2<T>*>(a.ph) : nullptr;
  for (int e = tid; e < (L << lgc); e += nthr) {
    const int r = e >> lgc, c = e & cmask;
    C2<T> v = {T(0), T(0)};
    const int col = col0 + c;
    if (r < nin && col < ncols) {
      bool ok = true;
      if (lf && min_) ok = (lf[r] & min_) != 0;
      if (ok) v = base[(int64_t)r * row_stride + col];
      if (ok && ph && inverse) v = cmul(v, cconj(ph[r]));
    }
    buf[r * ncolp + c] = v;
  }
  __syncthreads();
  const C2<T>* res = lds_fft<T, Tune<T>::maxr>(buf, buf2, tw, pl, lgc, ncolp, inverse != 0);
  for (int e = tid; e < (nout << lgc); e += nthr) {
    const int r = e >> lgc, c = e & cmask;
    const int col = col0 + c;
    if (col >= ncols) continue;
    if (lf && mout && !(lf[r] & mout)) continue;
    C2<T> v = res[r * ncolp + c];
    if (ph && !inverse) v = cmul(v, ph[r]);
    base[(int64_t)r * row_stride + col] = v;
  }
}

template <typename T>
__global__ void __launch_bounds__(1024)
k_strided(C2<T>* __restrict__ data, StridedArgs a, CompSet cs, AxisPlan pl, const C2<T>* __restrict__ twg,
          const uint8_t* __restrict__ lflag, const uint8_t* __restrict__ pflag) {
  if (a.skip && *a.skip) return;
  strided_body<T>(data, a, cs, pl, twg, lflag, pflag, a.act, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T>
__global__ void __launch_bounds__(1024)
k_strided_multi(const StridedScene* __restrict__ tab, int nscene, const int* __restrict__ skip,
                const int* __restrict__ act) {
  if (skip && *skip) return;
  const int lin = blockIdx.x;
  const StridedScene& sc = tab[find_scene(tab, nscene, lin)];
  const int local = lin - sc.blk0;
  const int gxy = sc.gx * sc.gy;
  const int bz = local / gxy, rem = local - bz * gxy;
  const int by = rem / sc.gx, bx = rem - by * sc.gx;
  strided_body<T>(static_cast<C2<T>*>(sc.data), sc.a, sc.cs, sc.pl, static_cast<const C2<T>*>(sc.tw), sc.lflag,
                  sc.pflag, act ? act + sc.c0 : nullptr, bx, by, bz);
}

// ------------------------------------------------------------------------------ z inverse + gather
// Workgroup (bx, by): lines bx*ncol .. of the item list, right-hand side(s) by.  x is
// the product's input (jump term of eq. (7)), y its output, both from the scene's
// first column with column stride ldx.
template <typename T>
__device__ __forceinline__ void zinv_body(const ZScene& a, int mode, const double* __restrict__ x,
                                          double* __restrict__ y, int64_t ldx, const int* __restrict__ act, int bx,
                                          int by) {
  const int nrhs = a.nrhs;
  const int ra = (mode == 0) ? by : 2 * by;
  const int rb = (mode == 0) ? -1 : ra + 1;
  if (act && !act[ra] && !(rb >= 0 && rb < nrhs && act[rb])) return;   // uniform per workgroup
  extern __shared__ char smem_raw[];
  const AxisPlan& pl = a.pl;
  const int L = pl.L;
  const int lgc = a.lgc, ncol = 1 << lgc, ncolp = ncol + 1;
  const int nitems = a.nitems, n1x = a.n1x, n1y = a.n1y, My = a.My, H = a.H;
  const int64_t comp_stride = a.comp_stride, rhs_stride = a.rhs_stride;
  const int32_t* __restrict__ items = a.items;
  const int32_t* __restrict__ line_ptr = a.line_ptr;
  const int32_t* __restrict__ pk = a.pk;
  const int8_t* __restrict__ pkind = a.pkind;
  const double* __restrict__ diag = a.diag;
  const uint8_t* __restrict__ lflag = a.lflag;
  const C2<T>* __restrict__ O = static_cast<const C2<T>*>(a.F);
  const C2<T>* __restrict__ twg = static_cast<const C2<T>*>(a.tw);
  const C2<T>* __restrict__ phz = static_cast<const C2<T>*>(a.ph);
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  C2<T>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  __shared__ int lp[33], sl[32];
  __shared__ uint8_t sf[32];
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  const int item0 = bx * ncol;
  if (tid < ncol && item0 + tid < nitems) sf[tid] = lflag[items[item0 + tid]];   // line flags of the tile
  const int nc = tile_panels(items, line_ptr, item0, nitems, ncol, lp, sl);   // (synchronises)
  const int plane = n1x * n1y;
  const float invH = 1.0f / (float)H, invPl = 1.0f / (float)plane, invN1y = 1.0f / (float)n1y;
  for (int e = tid; e < H * ncol; e += nthr) {
    const int c = fdiv(e, invH), k = e - c * H;
    C2<T> Cv = {T(0), T(0)}, Dv = {T(0), T(0)};
    if (c < nc) {
      const int line = sl[c];
      const int axis = fdiv(line, invPl);
      const int rem = line - axis * plane;
      const int xi = fdiv(rem, invN1y), yi = rem - xi * n1y;
      const int64_t off = ((int64_t)xi * My + yi) * H + k;
      if (mode == 0) {
        const uint8_t f = sf[c];
        if (f & 1) Cv = O[axis * comp_stride + ra * rhs_stride + off];
        if (f & 2) Dv = O[(3 + axis) * comp_stride + ra * rhs_stride + off];
      } else {
        Cv = O[axis * comp_stride + ra * rhs_stride + off];
        if (rb < nrhs) Dv = O[axis * comp_stride + rb * rhs_stride + off];
      }
      if (phz && axis == 2) {
        // back from the common lattice: the conjugate half-voxel shift
        const C2<T> w = cconj(phz[k]);
        Cv = cmul(Cv, w);
        Dv = cmul(Dv, w);
      }
    }
    // Z = C + i D on the half spectrum, Hermitian completion for the other half
    buf[k * ncolp + c] = C2<T>{Cv.x - Dv.y, Cv.y + Dv.x};
    if (k > 0 && k < L - k) buf[(L - k) * ncolp + c] = C2<T>{Cv.x + Dv.y, Dv.x - Cv.y};
  }
  __syncthreads();
  const C2<T>* res = lds_fft<T, Tune<T>::maxr>(buf, buf2, tw, pl, lgc, ncolp, true);
  // gather: all threads over the tile's panels at once
  for (int p = (nc > 0 ? lp[0] : 0) + tid; nc > 0 && p < lp[nc]; p += nthr) {
    const int c = panel_col(lp, nc, p);
    const C2<T> Z = res[pk[p] * ncolp + c];
    const double dg = diag[p];
    if (mode == 0) {
      const int64_t o = (int64_t)ra * ldx + p;
      y[o] = pkind[p] == 0 ? double(Z.x) : double(Z.y) + dg * x[o];
    } else {
      const int64_t oa = (int64_t)ra * ldx + p;
      y[oa] = double(Z.x) + dg * x[oa];
      if (rb < nrhs) {
        const int64_t ob = (int64_t)rb * ldx + p;
        y[ob] = double(Z.y) + dg * x[ob];
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(1024)
k_zinv(ZScene a, int mode, const double* __restrict__ x, double* __restrict__ y, int64_t ldx,
       const int* __restrict__ skip, const int* __restrict__ act) {
  if (skip && *skip) return;
  zinv_body<T>(a, mode, x, y, ldx, act, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ void __launch_bounds__(1024)
k_zinv_multi(const ZScene* __restrict__ tab, int nscene, const double* __restrict__ x, double* __restrict__ y,
             int64_t ldx, const int* __restrict__ skip, const int* __restrict__ act) {
  if (skip && *skip) return;
  const int lin = blockIdx.x;
  const ZScene& a = tab[find_scene(tab, nscene, lin)];
  const int local = lin - a.blk0;
  const int by = local / a.gx, bx = local - by * a.gx;
  const int64_t o = (int64_t)a.c0 * ldx;
  zinv_body<T>(a, 0, x + o, y + o, ldx, act ? act + a.c0 : nullptr, bx, by);
}

static inline int ilog2(int n) {
  int l = 0;
  while ((1 << (l + 1)) <= n) ++l;
  return l;
}

// ------------------------------------------------------------------------------ host launchers
template <typename T>
static size_t lds_bytes(int L, int ncol) {
  return sizeof(C2<T>) * ((size_t)L + 2 * (size_t)L * (ncol + 1));   // twiddles + ping-pong tiles
}

// launches above the default 64 KiB of dynamic LDS declare it first
template <typename K>
static hipError_t allow_lds(K kernel, size_t lds) {
  if (lds <= kLdsBudget) return hipSuccess;
  if (lds > lds_ext_budget()) return hipErrorInvalidValue;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

size_t zs_lds_bytes(int elem, int L, int ncol) {
  return (size_t)2 * elem * ((size_t)L + 2 * (size_t)L * (ncol + 1));
}

template <typename T>
hipError_t launch_zfwd(const double* x, int64_t N, int nrhs, int mode, const int32_t* items, int nitems,
                       const int32_t* line_ptr, const int32_t* pk, const int8_t* pkind, void* F, int64_t comp_stride,
                       int64_t rhs_stride, int n1x, int n1y, int My, int H, const AxisPlan& pl, const void* tw, int ncol,
                       int nthr, const int* skip, hipStream_t st, const int* act, const void* ph) {
  if (nitems == 0) return hipSuccess;
  if (ncol < 1 || ncol > 32 || (ncol & (ncol - 1)) || nthr < 64) return hipErrorInvalidValue;   // tile of <= 32 lines
  ZScene a{};
  a.items = items; a.line_ptr = line_ptr; a.pk = pk; a.pkind = pkind; a.F = F; a.tw = tw; a.pl = pl; a.ph = ph;
  a.comp_stride = comp_stride; a.rhs_stride = rhs_stride;
  a.nitems = nitems; a.nrhs = nrhs; a.n1x = n1x; a.n1y = n1y; a.My = My; a.H = H; a.lgc = ilog2(ncol);
  dim3 grid((nitems + ncol - 1) / ncol, mode == 0 ? (nrhs + 1) / 2 : nrhs);
  const hipError_t e = allow_lds(k_zfwd<T>, lds_bytes<T>(pl.L, ncol));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zfwd<T>), grid, dim3(nthr), lds_bytes<T>(pl.L, ncol), st, a, mode, x, N, skip, act);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_strided(void* data, const StridedArgs& a, const CompSet& cs, int nplanes, const AxisPlan& pl,
                          const void* tw, const uint8_t* lflag, const uint8_t* pflag, int nthr, hipStream_t st) {
  dim3 grid((a.ncols + a.ncol - 1) / a.ncol, nplanes, cs.n * a.nrhs);
  StridedArgs b = a;
  b.lgc = ilog2(a.ncol);
  if ((1 << b.lgc) != a.ncol) return hipErrorInvalidValue;
  const hipError_t e = allow_lds(k_strided<T>, lds_bytes<T>(pl.L, a.ncol));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_strided<T>), grid, dim3(nthr), lds_bytes<T>(pl.L, a.ncol), st, (C2<T>*)data, b, cs,
                     pl, (const C2<T>*)tw, lflag, pflag);
  return hipGetLastError();
}

template <typename T>
bool sandwich_args_ok(const SandArgs& a, int nthr) {
  // the kernel assumes every one of these
  if (a.nst < 1 || a.nst > kSandMaxStages || a.ncol < 1 || a.ncol > 32 || nthr < 64 || (nthr & 63) ||
      nthr > sand_max_threads(a.Mx, a.nst, a.radpack, (int)sizeof(T), a.nin))
    return false;
  long prod = 1;
  int prev = 1 << 30;
  for (int s = 0; s < a.nst; ++s) {
    const int r = (int)((a.radpack >> (5 * s)) & 31u);
    if (r < 2 || r > prev) return false;
    if (s == 0 && r > sandwich_rmax((int)sizeof(T))) return false;
    if (s > 0 && s < a.nst - 1 && r > sandwich_rmid((int)sizeof(T))) return false;
    prev = r;
    prod *= r;
  }
  const int rs = (int)((a.radpack >> (5 * (a.nst - 1))) & 31u);
  if (prod != a.Mx || (long)a.tl * rs != a.Mx || (long)a.tl * a.ncol > nthr) return false;
  if (a.nst == 1 && a.tl != 1) return false;
  if (rs > sandwich_rs_max((int)sizeof(T), a.nin)) return false;
  // 32-bit byte offsets inside one (component, rhs) slab and one stored pair, each slab
  // small enough for the out-of-range offset of the buffer views (0xFFFFFFF0)
  if ((uint64_t)a.n1x * a.My * a.H * 2 * sizeof(T) > 0xFFFFFF00ull ||
      (!a.tk && (uint64_t)a.pair_stride * sizeof(T) > 0xFFFFFF00ull))
    return false;
  // the fused and staged forms: their stored pairs, and the tile's spectra within the
  // device's LDS (the staged form copies the stored octants: all npairs of them in the
  // buffer view, whose byte size must fit the view's 32-bit range)
  if (a.tk && a.stage) return false;
  if ((a.tk || a.stage) &&
      (a.npairs < 1 || a.npairs > 15 ||
       sandwich_tk_lds_bytes(a.Mx, a.ncol, (int)sizeof(T), a.n1x, a.npairs, a.Hx) > lds_ext_budget()))
    return false;
  if (a.stage && (uint64_t)a.npairs * a.pair_stride * sizeof(T) > 0xFFFFFF00ull) return false;
  return true;
}

template <typename T>
hipError_t launch_sandwich(const void* Fin, void* Fout, const void* R, const SandArgs& a, const void* tw,
                           const void* phx, const uint8_t* pflag, int nthr,
                           hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  if (!sandwich_args_ok<T>(a, nthr)) return hipErrorInvalidValue;
  const int rs = (int)((a.radpack >> (5 * (a.nst - 1))) & 31u);
  if (a.tk || a.stage) {
    const size_t lds = sandwich_tk_lds_bytes(a.Mx, a.ncol, (int)sizeof(T), a.n1x, a.npairs, a.Hx);
    if (!a.adjoint && a.nin == 3 && a.nout == 6)
      return launch_sandwich_v<T, 3, 6, 1>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, rs, st, e0, e1);
    if (!a.adjoint && a.nin == 3 && a.nout == 3)
      return launch_sandwich_v<T, 3, 3, 1>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, rs, st, e0, e1);
    if (a.adjoint && a.nin == 6 && a.nout == 3)
      return launch_sandwich_v<T, 6, 3, 1>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, rs, st, e0, e1);
    return hipErrorInvalidValue;
  }
  const size_t lds = sandwich_lds_bytes(a.Mx, a.ncol, (int)sizeof(T), a.n1x);
  if (!a.adjoint && a.nin == 3 && a.nout == 6)
    return launch_sandwich_v<T, 3, 6, 0>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, rs, st, e0, e1);
  if (!a.adjoint && a.nin == 3 && a.nout == 3)
    return launch_sandwich_v<T, 3, 3, 0>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, rs, st, e0, e1);
  if (a.adjoint && a.nin == 6 && a.nout == 3)
    return launch_sandwich_v<T, 6, 3, 0>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, rs, st, e0, e1);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_zinv(const void* O, double* y, const double* x, int64_t N, int nrhs, int mode, const int32_t* items,
                       int nitems, const int32_t* line_ptr, const int32_t* pk, const int8_t* pkind,
                       const double* diag, const uint8_t* lflag, int64_t comp_stride, int64_t rhs_stride, int n1x,
                       int n1y, int My, int H, const AxisPlan& pl, const void* tw, int ncol, int nthr,
                       const int* skip, hipStream_t st, const int* act, const void* ph) {
  if (nitems == 0) return hipSuccess;
  if (ncol < 1 || ncol > 32 || (ncol & (ncol - 1)) || nthr < 64) return hipErrorInvalidValue;   // tile of <= 32 lines
  ZScene a{};
  a.items = items; a.line_ptr = line_ptr; a.pk = pk; a.pkind = pkind; a.diag = diag; a.lflag = lflag;
  a.F = const_cast<void*>(O); a.tw = tw; a.pl = pl; a.ph = ph;
  a.comp_stride = comp_stride; a.rhs_stride = rhs_stride;
  a.nitems = nitems; a.nrhs = nrhs; a.n1x = n1x; a.n1y = n1y; a.My = My; a.H = H; a.lgc = ilog2(ncol);
  dim3 grid((nitems + ncol - 1) / ncol, mode == 0 ? nrhs : (nrhs + 1) / 2);
  const hipError_t e = allow_lds(k_zinv<T>, lds_bytes<T>(pl.L, ncol));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zinv<T>), grid, dim3(nthr), lds_bytes<T>(pl.L, ncol), st, a, mode, x, y, N, skip, act);
  return hipGetLastError();
}

// multi-scene launches: the table (device memory) was checked and laid out by the host
template <typename T>
hipError_t launch_zfwd_multi(const ZScene* tab, int nscene, int nblocks, const double* x, int64_t ldx,
                             const int* skip, const int* act, int nthr, size_t lds, hipStream_t st) {
  if (nscene <= 0 || nblocks <= 0) return hipSuccess;
  const hipError_t e = allow_lds(k_zfwd_multi<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zfwd_multi<T>), dim3(nblocks), dim3(nthr), lds, st, tab, nscene, x, ldx, skip, act);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_zinv_multi(const ZScene* tab, int nscene, int nblocks, const double* x, double* y, int64_t ldx,
                             const int* skip, const int* act, int nthr, size_t lds, hipStream_t st) {
  if (nscene <= 0 || nblocks <= 0) return hipSuccess;
  const hipError_t e = allow_lds(k_zinv_multi<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_zinv_multi<T>), dim3(nblocks), dim3(nthr), lds, st, tab, nscene, x, y, ldx, skip, act);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_strided_multi(const StridedScene* tab, int nscene, int nblocks, const int* skip, const int* act,
                                int nthr, size_t lds, hipStream_t st) {
  if (nscene <= 0 || nblocks <= 0) return hipSuccess;
  const hipError_t e = allow_lds(k_strided_multi<T>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_strided_multi<T>), dim3(nblocks), dim3(nthr), lds, st, tab, nscene, skip, act);
  return hipGetLastError();
}

#define VC_INST(T)                                                                                                \
  template hipError_t launch_zfwd<T>(const double*, int64_t, int, int, const int32_t*, int, const int32_t*,        \
                                     const int32_t*, const int8_t*, void*, int64_t, int64_t, int, int, int, int,   \
                                     const AxisPlan&, const void*, int, int, const int*, hipStream_t, const int*,  \
                                     const void*);                                                                \
  template hipError_t launch_strided<T>(void*, const StridedArgs&, const CompSet&, int, const AxisPlan&,          \
                                        const void*, const uint8_t*, const uint8_t*, int, hipStream_t);            \
  template hipError_t launch_sandwich<T>(const void*, void*, const void*, const SandArgs&, const void*, const void*, \
                                         const uint8_t*, int, hipStream_t, hipEvent_t, hipEvent_t);                 \
  template hipError_t launch_zinv<T>(const void*, double*, const double*, int64_t, int, int, const int32_t*, int, \
                                     const int32_t*, const int32_t*, const int8_t*, const double*, const uint8_t*, \
                                     int64_t, int64_t, int, int, int, int, const AxisPlan&, const void*, int, int, \
                                     const int*, hipStream_t, const int*, const void*);                            \
  template hipError_t launch_zfwd_multi<T>(const ZScene*, int, int, const double*, int64_t, const int*,           \
                                           const int*, int, size_t, hipStream_t);                                 \
  template hipError_t launch_zinv_multi<T>(const ZScene*, int, int, const double*, double*, int64_t, const int*,  \
                                           const int*, int, size_t, hipStream_t);                                 \
  template hipError_t launch_strided_multi<T>(const StridedScene*, int, int, const int*, const int*, int, size_t, \
                                              hipStream_t);                                                       \
  template bool sandwich_args_ok<T>(const SandArgs&, int);
VC_INST(float)
VC_INST(double)

}  // namespace vc
