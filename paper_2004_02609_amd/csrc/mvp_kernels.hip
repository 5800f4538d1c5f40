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
//             inverse x transform of each output, all in one LDS tile per (ky, kz-tile)
//  k_zinv     inverse z transform (C2R) of the lines that hold panels, fused with the
//             gather, the jump term of eq. (7) and the FP64 result
#include "fft_core.hpp"
#include "mvp_kernels.h"

namespace vc {

template <typename T> __device__ __forceinline__ C2<T> ld(const C2<T>* p) { return *p; }

// ------------------------------------------------------------------------------ z forward
template <typename T, int EMAX>
__global__ void __launch_bounds__(1024)
k_zfwd(const double* __restrict__ x, int64_t N, int nrhs, int mode, const int32_t* __restrict__ items, int nitems,
       const int32_t* __restrict__ line_ptr, const int32_t* __restrict__ pk, const int8_t* __restrict__ pkind,
       C2<T>* __restrict__ F, int64_t comp_stride, int64_t rhs_stride, int n1x, int n1y, int My, int H, AxisPlan pl,
       const C2<T>* __restrict__ twg, int ncol) {
  extern __shared__ char smem_raw[];
  const int L = pl.L;
  const int ncolp = ncol + 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
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
  lds_fft<T, EMAX>(buf, tw, pl, ncol, ncolp, false);
  const int plane = n1x * n1y;
  for (int e = tid; e < H * ncol; e += nthr) {
    const int c = e / H, k = e - c * H;
    const int it = item0 + c;
    if (it >= nitems) continue;
    const int line = items[it];
    const int axis = line / plane;
    const int rem = line - axis * plane;
    const int xi = rem / n1y, yi = rem - xi * n1y;
    const C2<T> Z = buf[k * ncolp + c];
    const C2<T> Zc = cconj(buf[((L - k) % L) * ncolp + c]);
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
  const int ncol = a.ncol, ncolp = ncol + 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
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
  for (int e = tid; e < L * ncol; e += nthr) {
    const int r = e / ncol, c = e - r * ncol;
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
  lds_fft<T, EMAX>(buf, tw, pl, ncol, ncolp, a.inverse != 0);
  for (int e = tid; e < a.nout * ncol; e += nthr) {
    const int r = e / ncol, c = e - r * ncol;
    const int col = col0 + c;
    if (col >= a.ncols) continue;
    if (lf && mout && !(lf[r] & mout)) continue;
    base[(int64_t)r * a.row_stride + col] = buf[r * ncolp + c];
  }
}

// ------------------------------------------------------------------------------ x sandwich
// Stored kernel spectra are real after a separable half-voxel phase (see setup); the
// value for frequency (kx, ky, kz) of pair q is par(q, kx) * par(q, ky) * R[q][ky'][kz][kx'].
template <typename T>
__device__ __forceinline__ T rget(const T* __restrict__ R, const SandArgs& a, int q, int kx, int kyp, int kz,
                                  T sy) {
  int kxp = kx;
  T s = sy;
  if (kx > a.Mx / 2) {
    kxp = a.Mx - kx;
    if (a.odd[q] & 1) s = -s;
  }
  return s * R[(int64_t)q * a.pair_stride + ((int64_t)kyp * a.H + kz) * a.Hx + kxp];
}

template <typename T, int EMAX, int NIN, int NOUT>
__global__ void __launch_bounds__(1024)
k_xsandwich(const C2<T>* __restrict__ Fin, C2<T>* __restrict__ Fout, const T* __restrict__ R, SandArgs a,
            AxisPlan pl, const C2<T>* __restrict__ twg, const C2<T>* __restrict__ phx, const C2<T>* __restrict__ phy,
            const C2<T>* __restrict__ phz, const uint8_t* __restrict__ pflag) {
  extern __shared__ char smem_raw[];
  const int L = pl.L;  // = Mx
  const int ncol = a.ncol, ncolp = ncol + 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int ky = blockIdx.y;
  const int col0 = blockIdx.x * ncol;
  const int kyp = ky > a.My / 2 ? a.My - ky : ky;
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  const C2<T> py = phy[ky];
  const int nel = L * ncol;
  for (int rhs = 0; rhs < a.nrhs; ++rhs) {
    C2<T> q[NIN][EMAX];
    for (int b = 0; b < NIN; ++b) {
      const int comp = a.in_comp[b];
      const int axis = a.in_axis[b];
      const int msk = a.in_mask[b];
      const C2<T>* src = Fin + comp * a.comp_stride + rhs * a.rhs_stride;
      __syncthreads();
      for (int e = tid; e < nel; e += nthr) {
        const int r = e / ncol, c = e - r * ncol;
        const int col = col0 + c;
        C2<T> v = {T(0), T(0)};
        if (r < a.n1x && col < a.H && (!msk || (pflag[axis * a.n1x + r] & msk)))
          v = src[((int64_t)r * a.My + ky) * a.H + col];
        buf[r * ncolp + c] = v;
      }
      __syncthreads();
      lds_fft<T, EMAX>(buf, tw, pl, ncol, ncolp, false);
#pragma unroll
      for (int j = 0; j < EMAX; ++j) {
        const int e = tid + j * nthr;
        if (e < nel) {
          const int r = e / ncol, c = e - r * ncol;
          const int col = col0 + c < a.H ? col0 + c : a.H - 1;
          // half-voxel phase of the input component (shift to the common lattice)
          const int ax = a.in_axis[b];
          C2<T> ph = ax == 0 ? phx[r] : (ax == 1 ? py : phz[col]);
          q[b][j] = cmul(buf[r * ncolp + c], ph);
        } else {
          q[b][j] = C2<T>{T(0), T(0)};
        }
      }
    }
    for (int o = 0; o < NOUT; ++o) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < EMAX; ++j) {
        const int e = tid + j * nthr;
        if (e < nel) {
          const int r = e / ncol, c = e - r * ncol;
          const int kz = col0 + c < a.H ? col0 + c : a.H - 1;
          const T sy = T(1);
          C2<T> acc = {T(0), T(0)};
          int oax;
          if (!a.adjoint) {
            // forward: o < 3 -> C_alpha = sum_b P(alpha,b) Q'_b ; o >= 3 -> D_alpha = i sum_b E(alpha,b) Q'_b
            const int al = o < 3 ? o : o - 3;
            oax = al;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const int qi = o < 3 ? (al == b ? al : 2 + al + b) : 6 + 3 * al + b;
              T ys = (ky > a.My / 2 && ((a.odd[qi] >> 1) & 1)) ? T(-1) : sy;
              const T rv = rget(R, a, qi, r, kyp, kz, ys);
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
              T ys = (ky > a.My / 2 && ((a.odd[qp] >> 1) & 1)) ? T(-1) : sy;
              const T rp = rget(R, a, qp, r, kyp, kz, ys);
              acc.x += rp * q[al][j].x;
              acc.y += rp * q[al][j].y;
              if (NIN > 3) {
                const int qe = 6 + 3 * al + bb;
                T ye = (ky > a.My / 2 && ((a.odd[qe] >> 1) & 1)) ? T(-1) : sy;
                const T re = rget(R, a, qe, r, kyp, kz, ye);
                accE.x += re * q[3 + al][j].x;
                accE.y += re * q[3 + al][j].y;
              }
            }
            acc.x += accE.y;   // -i * accE
            acc.y -= accE.x;
          }
          // output phase: conj of the half-voxel shift of the output component
          const C2<T> ph = oax == 0 ? phx[r] : (oax == 1 ? py : phz[kz]);
          buf[r * ncolp + c] = cmul(acc, cconj(ph));
        }
      }
      __syncthreads();
      lds_fft<T, EMAX>(buf, tw, pl, ncol, ncolp, true);
      const int comp = a.out_comp[o], axis = a.out_axis[o], msk = a.out_mask[o];
      C2<T>* dst = Fout + comp * a.comp_stride + rhs * a.rhs_stride;
      for (int e = tid; e < a.n1x * ncol; e += nthr) {
        const int r = e / ncol, c = e - r * ncol;
        const int col = col0 + c;
        if (col >= a.H) continue;
        if (msk && !(pflag[axis * a.n1x + r] & msk)) continue;
        dst[((int64_t)r * a.My + ky) * a.H + col] = buf[r * ncolp + c];
      }
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
       AxisPlan pl, const C2<T>* __restrict__ twg, int ncol) {
  extern __shared__ char smem_raw[];
  const int L = pl.L;
  const int ncolp = ncol + 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  const int ra = (mode == 0) ? blockIdx.y : 2 * blockIdx.y;
  const int rb = (mode == 0) ? -1 : ra + 1;
  const int item0 = blockIdx.x * ncol;
  const int plane = n1x * n1y;
  for (int e = tid; e < H * ncol; e += nthr) {
    const int c = e / H, k = e - c * H;
    const int it = item0 + c;
    C2<T> Cv = {T(0), T(0)}, Dv = {T(0), T(0)};
    if (it < nitems) {
      const int line = items[it];
      const int axis = line / plane;
      const int rem = line - axis * plane;
      const int xi = rem / n1y, yi = rem - xi * n1y;
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
  lds_fft<T, EMAX>(buf, tw, pl, ncol, ncolp, true);
  for (int c = 0; c < ncol; ++c) {
    const int it = item0 + c;
    if (it >= nitems) break;
    const int line = items[it];
    const int p0 = line_ptr[line], p1 = line_ptr[line + 1];
    for (int p = p0 + tid; p < p1; p += nthr) {
      const C2<T> Z = buf[pk[p] * ncolp + c];
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

// ------------------------------------------------------------------------------ host launchers
template <typename T>
static size_t lds_bytes(int L, int ncol) {
  return sizeof(C2<T>) * ((size_t)L + (size_t)L * (ncol + 1));
}

template <typename T>
hipError_t launch_zfwd(const double* x, int64_t N, int nrhs, int mode, const int32_t* items, int nitems,
                       const int32_t* line_ptr, const int32_t* pk, const int8_t* pkind, void* F, int64_t comp_stride,
                       int64_t rhs_stride, int n1x, int n1y, int My, int H, const AxisPlan& pl, const void* tw, int ncol,
                       int nthr, hipStream_t st) {
  if (nitems == 0) return hipSuccess;
  dim3 grid((nitems + ncol - 1) / ncol, mode == 0 ? (nrhs + 1) / 2 : nrhs);
  hipLaunchKernelGGL((k_zfwd<T, kEmax>), grid, dim3(nthr), lds_bytes<T>(pl.L, ncol), st, x, N, nrhs, mode, items,
                     nitems, line_ptr, pk, pkind, (C2<T>*)F, comp_stride, rhs_stride, n1x, n1y, My, H, pl,
                     (const C2<T>*)tw, ncol);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_strided(void* data, const StridedArgs& a, const CompSet& cs, int nplanes, const AxisPlan& pl,
                          const void* tw, const uint8_t* lflag, const uint8_t* pflag, int nthr, hipStream_t st) {
  dim3 grid((a.ncols + a.ncol - 1) / a.ncol, nplanes, cs.n * a.nrhs);
  hipLaunchKernelGGL((k_strided<T, kEmax>), grid, dim3(nthr), lds_bytes<T>(pl.L, a.ncol), st, (C2<T>*)data, a, cs,
                     pl, (const C2<T>*)tw, lflag, pflag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sandwich(const void* Fin, void* Fout, const void* R, const SandArgs& a, const AxisPlan& pl,
                           const void* tw, const void* phx, const void* phy, const void* phz, const uint8_t* pflag,
                           int nthr, hipStream_t st) {
  dim3 grid((a.H + a.ncol - 1) / a.ncol, a.My);
  size_t lds = lds_bytes<T>(pl.L, a.ncol);
#define VC_SAND(NI, NO)                                                                                       \
  hipLaunchKernelGGL((k_xsandwich<T, kEmaxSand, NI, NO>), grid, dim3(nthr), lds, st, (const C2<T>*)Fin,       \
                     (C2<T>*)Fout, (const T*)R, a, pl, (const C2<T>*)tw, (const C2<T>*)phx, (const C2<T>*)phy, \
                     (const C2<T>*)phz, pflag)
  if (!a.adjoint && a.nout == 6) VC_SAND(3, 6);
  else if (!a.adjoint && a.nout == 3) VC_SAND(3, 3);
  else if (a.adjoint && a.nin == 6) VC_SAND(6, 3);
  else VC_SAND(3, 3);
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
  hipLaunchKernelGGL((k_zinv<T, kEmax>), grid, dim3(nthr), lds_bytes<T>(pl.L, ncol), st, (const C2<T>*)O, y, x, N,
                     nrhs, mode, items, nitems, line_ptr, pk, pkind, diag, lflag, comp_stride, rhs_stride, n1x, n1y,
                     My, H, pl, (const C2<T>*)tw, ncol);
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
