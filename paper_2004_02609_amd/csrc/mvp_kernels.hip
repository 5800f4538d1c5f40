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
//  k_xsandwich forward x transform of the inputs, the per-frequency block multiply,
//             inverse x transform of each output, all in one LDS tile of (ky, kz) columns
//  k_zinv     inverse z transform (C2R) of the lines that hold panels, fused with the
//             gather, the jump term of eq. (7) and the FP64 result
#include "fft_core.hpp"
#include "mvp_kernels.h"

namespace vc {

template <typename T> __device__ __forceinline__ C2<T> ld(const C2<T>* p) { return *p; }

// ------------------------------------------------------------------------------ z forward
// Tiles hold 2^lgc lines; divisions by non-powers of two use fdiv (exact in range).
template <typename T, int EMAX>
__global__ void __launch_bounds__(1024)
k_zfwd(const double* __restrict__ x, int64_t N, int nrhs, int mode, const int32_t* __restrict__ items, int nitems,
       const int32_t* __restrict__ line_ptr, const int32_t* __restrict__ pk, const int8_t* __restrict__ pkind,
       C2<T>* __restrict__ F, int64_t comp_stride, int64_t rhs_stride, int n1x, int n1y, int My, int H, AxisPlan pl,
       const C2<T>* __restrict__ twg, int lgc) {
  extern __shared__ char smem_raw[];
  const int L = pl.L;
  const int ncol = 1 << lgc, ncolp = ncol + 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  C2<T>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  for (int e = tid; e < L * ncolp; e += nthr) buf[e] = C2<T>{T(0), T(0)};
  __syncthreads();
  const int ra = (mode == 0) ? 2 * blockIdx.y : blockIdx.y;
  const int rb = (mode == 0) ? ra + 1 : -1;
  const int item0 = blockIdx.x * ncol;
  for (int c = 0; c < ncol; ++c) {
    const int it = item0 + c;
    if (it >= nitems) break;
    const int line = items[it];
    const int p0 = line_ptr[line], p1 = line_ptr[line + 1];
    for (int p = p0 + tid; p < p1; p += nthr) {
      const int k = pk[p];
      double re, im;
      if (mode == 0) {
        re = x[(int64_t)ra * N + p];
        im = (rb < nrhs) ? x[(int64_t)rb * N + p] : 0.0;
      } else {
        const double v = x[(int64_t)ra * N + p];
        re = pkind[p] == 0 ? v : 0.0;
        im = pkind[p] == 0 ? 0.0 : v;
      }
      buf[k * ncolp + c] = C2<T>{T(re), T(im)};
    }
  }
  __syncthreads();
  const C2<T>* res = lds_fft<T, Tune<T>::maxr>(buf, buf2, tw, pl, lgc, ncolp, false);
  const int plane = n1x * n1y;
  const float invH = 1.0f / (float)H, invPl = 1.0f / (float)plane, invN1y = 1.0f / (float)n1y;
  for (int e = tid; e < H * ncol; e += nthr) {
    const int c = fdiv(e, invH), k = e - c * H;
    const int it = item0 + c;
    if (it >= nitems) continue;
    const int line = items[it];
    const int axis = fdiv(line, invPl);
    const int rem = line - axis * plane;
    const int xi = fdiv(rem, invN1y), yi = rem - xi * n1y;
    const C2<T> Z = res[k * ncolp + c];
    const C2<T> Zc = cconj(res[(k == 0 ? 0 : L - k) * ncolp + c]);
    const C2<T> A = {T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y + Zc.y)};
    const C2<T> B = {T(0.5) * (Z.y - Zc.y), T(-0.5) * (Z.x - Zc.x)};
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

// ------------------------------------------------------------------------------ strided C2C
template <typename T, int EMAX>
__global__ void __launch_bounds__(1024)
k_strided(C2<T>* __restrict__ data, StridedArgs a, CompSet cs, AxisPlan pl, const C2<T>* __restrict__ twg,
          const uint8_t* __restrict__ lflag, const uint8_t* __restrict__ pflag) {
  extern __shared__ char smem_raw[];
  const int L = pl.L;
  const int lgc = a.lgc, ncol = 1 << lgc, ncolp = ncol + 1, cmask = ncol - 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  C2<T>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int plane = blockIdx.y;
  const int cz = blockIdx.z / a.nrhs, rhs = blockIdx.z - cz * a.nrhs;
  const int comp = cs.comp[cz], axis = cs.axis[cz];
  const int min_ = cs.min_[cz], mout = cs.mout[cz];
  const int need = a.inverse ? mout : min_;
  if (pflag && need && !(pflag[axis * a.n1x + plane] & need)) return;  // uniform per block
  C2<T>* base = data + comp * a.comp_stride + rhs * a.rhs_stride + plane * a.plane_stride;
  const int col0 = blockIdx.x * ncol;
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  const uint8_t* lf = lflag ? lflag + ((int64_t)axis * a.n1x + plane) * a.n1y : nullptr;
  for (int e = tid; e < (L << lgc); e += nthr) {
    const int r = e >> lgc, c = e & cmask;
    C2<T> v = {T(0), T(0)};
    const int col = col0 + c;
    if (r < a.nin && col < a.ncols) {
      bool ok = true;
      if (lf && min_) ok = (lf[r] & min_) != 0;
      if (ok) v = base[(int64_t)r * a.row_stride + col];
    }
    buf[r * ncolp + c] = v;
  }
  __syncthreads();
  const C2<T>* res = lds_fft<T, Tune<T>::maxr>(buf, buf2, tw, pl, lgc, ncolp, a.inverse != 0);
  for (int e = tid; e < (a.nout << lgc); e += nthr) {
    const int r = e >> lgc, c = e & cmask;
    const int col = col0 + c;
    if (col >= a.ncols) continue;
    if (lf && mout && !(lf[r] & mout)) continue;
    base[(int64_t)r * a.row_stride + col] = res[r * ncolp + c];
  }
}

// ------------------------------------------------------------------------------ x sandwich
// A workgroup owns 2^lgc consecutive (ky, kz) columns of the [x][ky][kz] arrays (for a
// fixed x they are contiguous, so tiles never straddle a row end) and every kx.
// Stored kernel spectra are real after a separable half-voxel phase (see setup); the
// value for frequency (kx, ky, kz) of pair q is par(q, kx) * par(q, ky) * R[q][ky'][kz][kx'],
// kx' contiguous, so the multiply maps consecutive threads to consecutive kx.
template <typename T>
__device__ __forceinline__ T rget(const T* __restrict__ R, const SandArgs& a, int q, int kx, int kyp, int kz,
                                  int yflip) {
  int kxp = kx;
  const unsigned odd = (unsigned)(a.oddmask >> (3 * q)) & 7u;   // bit a: odd in k_a
  bool neg = yflip && ((odd >> 1) & 1u);
  if (kx > a.Mx / 2) {
    kxp = a.Mx - kx;
    if (odd & 1u) neg = !neg;
  }
  const T v = R[(int64_t)q * a.pair_stride + ((int64_t)kyp * a.H + kz) * a.Hx + kxp];
  return neg ? -v : v;
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear id; this maps linear id
// -> work index so that each XCD gets one contiguous range (neighbouring column tiles,
// which share cache lines and spectra, then meet in the same L2).
__device__ __forceinline__ int xcd_remap(int lin, int n) {
  const int xcd = lin & 7, idx = lin >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// One workgroup = one right-hand side x 2^lgc (ky, kz) columns x all kx.  The inputs'
// global loads for component b+1 are issued before the transform of component b so
// they are in flight while it runs; transformed inputs stay in registers (rows-fastest
// mapping: thread element j is kx = er[j] of column ec[j]).
template <typename T, int EMAX, int NIN, int NOUT, int NTHR>
__global__ void __launch_bounds__(NTHR, (sizeof(T) == 8 || NIN == 6) ? 2 : 4)
k_xsandwich(const C2<T>* __restrict__ Fin, C2<T>* __restrict__ Fout, const T* __restrict__ R, SandArgs a,
            AxisPlan pl, const C2<T>* __restrict__ twg, const C2<T>* __restrict__ phx, const C2<T>* __restrict__ phy,
            const C2<T>* __restrict__ phz, const uint8_t* __restrict__ pflag) {
  extern __shared__ char smem_raw[];
  const int L = pl.L;  // = Mx
  const int lgc = a.lgc, ncol = 1 << lgc, ncolp = ncol + 1, cmask = ncol - 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  C2<T>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x;
  const int ntiles = gridDim.x;
  const int work = xcd_remap(blockIdx.y * ntiles + blockIdx.x, ntiles * gridDim.y);
  const int rhs = work / ntiles, tile = work - rhs * ntiles;
  const int ncols = a.My * a.H;                 // flattened (ky, kz) columns
  const int col0 = tile * ncol;
  const int64_t rowst = (int64_t)a.My * a.H;    // stride between x rows
  const float invL = 1.0f / (float)L, invH = 1.0f / (float)a.H;
  for (int t = tid; t < L; t += NTHR) tw[t] = twg[t];
  const int nel = L << lgc;
  C2<T> q[NIN][EMAX];
  C2<T> pre[EMAX];
  // global -> registers for input component b (columns fastest: contiguous reads)
#define VC_FETCH(b)                                                                                  \
  {                                                                                                  \
    const int fax = (b) % 3;                                                                         \
    const int fmsk = NIN == 3 ? 3 : ((b) < 3 ? 1 : 2);                                               \
    const C2<T>* src = Fin + (b) * a.comp_stride + rhs * a.rhs_stride;                               \
    _Pragma("unroll") for (int j = 0; j < EMAX; ++j) {                                               \
      const int e = tid + j * NTHR;                                                                  \
      const int r = e >> lgc, col = col0 + (e & cmask);                                              \
      C2<T> v = {T(0), T(0)};                                                                        \
      if (e < nel && r < a.n1x && col < ncols && (pflag[fax * a.n1x + r] & fmsk)) v = src[r * rowst + col]; \
      pre[j] = v;                                                                                    \
    }                                                                                                \
  }
  VC_FETCH(0)
#pragma unroll
  for (int b = 0; b < NIN; ++b) {
    const int axis = b % 3;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {
      const int e = tid + j * NTHR;
      if (e < nel) buf[(e >> lgc) * ncolp + (e & cmask)] = pre[j];
    }
    __syncthreads();
    if (b + 1 < NIN) VC_FETCH(b + 1)
    const C2<T>* res = lds_fft<T, Tune<T>::maxr_sand>(buf, buf2, tw, pl, lgc, ncolp, false);
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {            // rows fastest: contiguous spectra reads
      const int e = tid + j * NTHR;
      if (e < nel) {
        const int c = fdiv(e, invL), r = e - c * L;
        const int col = min(col0 + c, ncols - 1);
        const int ky = fdiv(col, invH), kz = col - ky * a.H;
        // half-voxel phase of the input component (shift to the common lattice)
        const C2<T> ph = axis == 0 ? phx[r] : (axis == 1 ? phy[ky] : phz[kz]);
        q[b][j] = cmul(res[r * ncolp + c], ph);
      } else {
        q[b][j] = C2<T>{T(0), T(0)};
      }
    }
  }
#undef VC_FETCH
  for (int o = 0; o < NOUT; ++o) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {
      const int e = tid + j * NTHR;
      if (e < nel) {
        const int c = fdiv(e, invL), r = e - c * L;
        const int col = min(col0 + c, ncols - 1);
        const int ky = fdiv(col, invH), kz = col - ky * a.H;
        const int yflip = ky > a.My / 2;
        const int kyp = yflip ? a.My - ky : ky;
        C2<T> acc = {T(0), T(0)};
        int oax;
        if (NIN == 3) {
          // o < 3: C_alpha = sum_b P(alpha,b) Q'_b ; o >= 3: D_alpha = i sum_b E(alpha,b) Q'_b
          const int al = o < 3 ? o : o - 3;
          oax = al;
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const int qi = o < 3 ? (al == b ? al : 2 + al + b) : 6 + 3 * al + b;
            const T rv = rget(R, a, qi, r, kyp, kz, yflip);
            acc.x += rv * q[b][j].x;
            acc.y += rv * q[b][j].y;
          }
          if (o >= 3) acc = C2<T>{-acc.y, acc.x};
        } else {
          // adjoint: out_b = sum_al P(al,b) X'C_al - i sum_al E(al,b) X'D_al
          const int bb = o;
          oax = bb;
          C2<T> accE = {T(0), T(0)};
#pragma unroll
          for (int al = 0; al < 3; ++al) {
            const int qp = al == bb ? al : 2 + al + bb;
            const T rp = rget(R, a, qp, r, kyp, kz, yflip);
            acc.x += rp * q[al][j].x;
            acc.y += rp * q[al][j].y;
            const T re = rget(R, a, 6 + 3 * al + bb, r, kyp, kz, yflip);
            accE.x += re * q[(NIN > 3 ? 3 : 0) + al][j].x;
            accE.y += re * q[(NIN > 3 ? 3 : 0) + al][j].y;
          }
          acc.x += accE.y;   // -i * accE
          acc.y -= accE.x;
        }
        // output phase: conj of the half-voxel shift of the output component
        const C2<T> ph = oax == 0 ? phx[r] : (oax == 1 ? phy[ky] : phz[kz]);
        buf[r * ncolp + c] = cmul(acc, cconj(ph));
      }
    }
    __syncthreads();
    const C2<T>* res = lds_fft<T, Tune<T>::maxr_sand>(buf, buf2, tw, pl, lgc, ncolp, true);
    const int axis = o % 3, msk = NIN == 3 ? (o < 3 ? 1 : 2) : 3;
    C2<T>* dst = Fout + o * a.comp_stride + rhs * a.rhs_stride;
    for (int e = tid; e < (a.n1x << lgc); e += NTHR) {
      const int r = e >> lgc, c = e & cmask;
      const int col = col0 + c;
      if (col >= ncols) continue;
      if (!(pflag[axis * a.n1x + r] & msk)) continue;
      dst[r * rowst + col] = res[r * ncolp + c];
    }
  }
}

// ------------------------------------------------------------------------------ z inverse + gather
template <typename T, int EMAX>
__global__ void __launch_bounds__(1024)
k_zinv(const C2<T>* __restrict__ O, double* __restrict__ y, const double* __restrict__ x, int64_t N, int nrhs,
       int mode, const int32_t* __restrict__ items, int nitems, const int32_t* __restrict__ line_ptr,
       const int32_t* __restrict__ pk, const int8_t* __restrict__ pkind, const double* __restrict__ diag,
       const uint8_t* __restrict__ lflag, int64_t comp_stride, int64_t rhs_stride, int n1x, int n1y, int My, int H,
       AxisPlan pl, const C2<T>* __restrict__ twg, int lgc) {
  extern __shared__ char smem_raw[];
  const int L = pl.L;
  const int ncol = 1 << lgc, ncolp = ncol + 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  C2<T>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  const int ra = (mode == 0) ? blockIdx.y : 2 * blockIdx.y;
  const int rb = (mode == 0) ? -1 : ra + 1;
  const int item0 = blockIdx.x * ncol;
  const int plane = n1x * n1y;
  const float invH = 1.0f / (float)H, invPl = 1.0f / (float)plane, invN1y = 1.0f / (float)n1y;
  for (int e = tid; e < H * ncol; e += nthr) {
    const int c = fdiv(e, invH), k = e - c * H;
    const int it = item0 + c;
    C2<T> Cv = {T(0), T(0)}, Dv = {T(0), T(0)};
    if (it < nitems) {
      const int line = items[it];
      const int axis = fdiv(line, invPl);
      const int rem = line - axis * plane;
      const int xi = fdiv(rem, invN1y), yi = rem - xi * n1y;
      const int64_t off = ((int64_t)xi * My + yi) * H + k;
      if (mode == 0) {
        const uint8_t f = lflag[line];
        if (f & 1) Cv = O[axis * comp_stride + ra * rhs_stride + off];
        if (f & 2) Dv = O[(3 + axis) * comp_stride + ra * rhs_stride + off];
      } else {
        Cv = O[axis * comp_stride + ra * rhs_stride + off];
        if (rb < nrhs) Dv = O[axis * comp_stride + rb * rhs_stride + off];
      }
    }
    // Z = C + i D on the half spectrum, Hermitian completion for the other half
    buf[k * ncolp + c] = C2<T>{Cv.x - Dv.y, Cv.y + Dv.x};
    if (k > 0 && k < L - k) buf[(L - k) * ncolp + c] = C2<T>{Cv.x + Dv.y, Dv.x - Cv.y};
  }
  __syncthreads();
  const C2<T>* res = lds_fft<T, Tune<T>::maxr>(buf, buf2, tw, pl, lgc, ncolp, true);
  for (int c = 0; c < ncol; ++c) {
    const int it = item0 + c;
    if (it >= nitems) break;
    const int line = items[it];
    const int p0 = line_ptr[line], p1 = line_ptr[line + 1];
    for (int p = p0 + tid; p < p1; p += nthr) {
      const C2<T> Z = res[pk[p] * ncolp + c];
      const double dg = diag[p];
      if (mode == 0) {
        const int64_t o = (int64_t)ra * N + p;
        y[o] = pkind[p] == 0 ? double(Z.x) : double(Z.y) + dg * x[o];
      } else {
        const int64_t oa = (int64_t)ra * N + p;
        y[oa] = double(Z.x) + dg * x[oa];
        if (rb < nrhs) {
          const int64_t ob = (int64_t)rb * N + p;
          y[ob] = double(Z.y) + dg * x[ob];
        }
      }
    }
  }
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

template <typename T>
hipError_t launch_zfwd(const double* x, int64_t N, int nrhs, int mode, const int32_t* items, int nitems,
                       const int32_t* line_ptr, const int32_t* pk, const int8_t* pkind, void* F, int64_t comp_stride,
                       int64_t rhs_stride, int n1x, int n1y, int My, int H, const AxisPlan& pl, const void* tw, int ncol,
                       int nthr, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  dim3 grid((nitems + ncol - 1) / ncol, mode == 0 ? (nrhs + 1) / 2 : nrhs);
  hipLaunchKernelGGL((k_zfwd<T, Tune<T>::emax>), grid, dim3(nthr), lds_bytes<T>(pl.L, ncol), st, x, N, nrhs, mode, items,
                     nitems, line_ptr, pk, pkind, (C2<T>*)F, comp_stride, rhs_stride, n1x, n1y, My, H, pl,
                     (const C2<T>*)tw, ilog2(ncol));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_strided(void* data, const StridedArgs& a, const CompSet& cs, int nplanes, const AxisPlan& pl,
                          const void* tw, const uint8_t* lflag, const uint8_t* pflag, int nthr, hipStream_t st) {
  dim3 grid((a.ncols + a.ncol - 1) / a.ncol, nplanes, cs.n * a.nrhs);
  StridedArgs b = a;
  b.lgc = ilog2(a.ncol);
  if ((1 << b.lgc) != a.ncol) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_strided<T, Tune<T>::emax>), grid, dim3(nthr), lds_bytes<T>(pl.L, a.ncol), st, (C2<T>*)data, b, cs,
                     pl, (const C2<T>*)tw, lflag, pflag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sandwich(const void* Fin, void* Fout, const void* R, const SandArgs& a, const AxisPlan& pl,
                           const void* tw, const void* phx, const void* phy, const void* phz, const uint8_t* pflag,
                           int nthr, hipStream_t st) {
  dim3 grid((a.My * a.H + a.ncol - 1) / a.ncol, a.nrhs);
  size_t lds = lds_bytes<T>(pl.L, a.ncol);
  SandArgs b = a;
  b.lgc = ilog2(a.ncol);
  if ((1 << b.lgc) != a.ncol) return hipErrorInvalidValue;
  constexpr int E = Tune<T>::emax_sand;
#define VC_SAND(NI, NO, NT)                                                                                   \
  hipLaunchKernelGGL((k_xsandwich<T, E, NI, NO, NT>), grid, dim3(NT), lds, st, (const C2<T>*)Fin,            \
                     (C2<T>*)Fout, (const T*)R, b, pl, (const C2<T>*)tw, (const C2<T>*)phx, (const C2<T>*)phy, \
                     (const C2<T>*)phz, pflag)
#define VC_SAND_T(NI, NO)                 \
  if (nthr == 256) VC_SAND(NI, NO, 256);  \
  else if (nthr == 512) VC_SAND(NI, NO, 512); \
  else VC_SAND(NI, NO, 1024);
  if ((long)pl.L * a.ncol > (long)E * nthr || (nthr != 256 && nthr != 512 && nthr != 1024))
    return hipErrorInvalidValue;
  if (!a.adjoint && a.nout == 6) { VC_SAND_T(3, 6) }
  else if (!a.adjoint && a.nout == 3) { VC_SAND_T(3, 3) }
  else if (a.adjoint && a.nin == 6) { VC_SAND_T(6, 3) }
  else return hipErrorInvalidValue;
#undef VC_SAND_T
#undef VC_SAND
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zinv(const void* O, double* y, const double* x, int64_t N, int nrhs, int mode, const int32_t* items,
                       int nitems, const int32_t* line_ptr, const int32_t* pk, const int8_t* pkind,
                       const double* diag, const uint8_t* lflag, int64_t comp_stride, int64_t rhs_stride, int n1x,
                       int n1y, int My, int H, const AxisPlan& pl, const void* tw, int ncol, int nthr,
                       hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  dim3 grid((nitems + ncol - 1) / ncol, mode == 0 ? nrhs : (nrhs + 1) / 2);
  hipLaunchKernelGGL((k_zinv<T, Tune<T>::emax>), grid, dim3(nthr), lds_bytes<T>(pl.L, ncol), st, (const C2<T>*)O, y, x, N,
                     nrhs, mode, items, nitems, line_ptr, pk, pkind, diag, lflag, comp_stride, rhs_stride, n1x, n1y,
                     My, H, pl, (const C2<T>*)tw, ilog2(ncol));
  return hipGetLastError();
}

#define VC_INST(T)                                                                                                \
  template hipError_t launch_zfwd<T>(const double*, int64_t, int, int, const int32_t*, int, const int32_t*,        \
                                     const int32_t*, const int8_t*, void*, int64_t, int64_t, int, int, int, int,   \
                                     const AxisPlan&, const void*, int, int, hipStream_t);                         \
  template hipError_t launch_strided<T>(void*, const StridedArgs&, const CompSet&, int, const AxisPlan&,          \
                                        const void*, const uint8_t*, const uint8_t*, int, hipStream_t);            \
  template hipError_t launch_sandwich<T>(const void*, void*, const void*, const SandArgs&, const AxisPlan&,       \
                                         const void*, const void*, const void*, const void*, const uint8_t*, int,  \
                                         hipStream_t);                                                             \
  template hipError_t launch_zinv<T>(const void*, double*, const double*, int64_t, int, int, const int32_t*, int, \
                                     const int32_t*, const int32_t*, const int8_t*, const double*, const uint8_t*, \
                                     int64_t, int64_t, int, int, int, int, const AxisPlan&, const void*, int, int, \
                                     hipStream_t);
VC_INST(float)
VC_INST(double)

}  // namespace vc
