// x "sandwich" pass of the FFT product of eq. (11) (Sec. II.B): forward x transform of
// the input components, the per-frequency block multiply with the stored kernel
// spectra, and the inverse x transform of every output component, for one tile of
// (ky, kz) columns and one right-hand side per workgroup.
//
// The x transform of length L = Mx runs as a Stockham mixed-radix FFT with radices
// f[0] >= f[1] >= ... >= f[S-1] = RS (RS a compile-time radix).  Thread (i, c) of the
// workgroup owns butterfly i < L/RS of column c (columns fastest across lanes, so
// every global access touches ncol consecutive complex values of one x row):
//
//   forward stage 0 (p = 1):   HBM rows i + q L/f0 -> registers -> radix f0 -> LDS
//   forward stages 1..S-2:     LDS -> LDS in place
//   forward stage S-1 (RS):    LDS -> registers; the thread now holds X[i + q L/RS]
//   block multiply:            in registers, one output component at a time
//   inverse stage 0 (RS, p=1): its inputs are exactly the values the thread holds,
//                              so it runs in registers -> LDS
//   inverse stages 1..S-2:     LDS -> LDS in place
//   inverse stage S-1 (f0):    LDS -> registers -> HBM rows i + q L/f0
//
// Each transform makes one round trip through LDS (plus one per middle stage), and the
// first and last butterflies touch HBM directly.  With S = 1 (L = RS) no LDS is used.
#pragma once
#include "fft_core.hpp"
#include "mvp_kernels.h"

namespace vc {

// Largest radix compiled into the LDS stages of the sandwich, per precision.
template <typename T> struct SandTune {
  static constexpr int rmax = sandwich_rmax((int)sizeof(T));
};

// Workgroups are dispatched to the 8 XCDs round-robin by linear id; this maps linear id
// -> work index so that each XCD gets one contiguous range of work.
__device__ __forceinline__ int xcd_remap(int lin, int n) {
  const int xcd = lin & 7, idx = lin >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Loads / stores at a uniform base plus a 32-bit per-lane byte offset (the launcher
// checks every array the sandwich touches is below 4 GiB), so the addresses take one
// VGPR each instead of a 64-bit pair.
template <typename V>
__device__ __forceinline__ V ldo(const V* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename V>
__device__ __forceinline__ void sto(V* __restrict__ base, uint32_t byte_off, V v) {
  *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// Stored real spectrum of pair q at (kx, ky, kz), ky already folded to kyp <= My/2
// (yflip set when it was), layout [q][kxp < Hx][kyp < Hy][kz < H]: the folds use the
// parity of the pair's spectrum under k_a -> M_a - k_a (bit a of its 3-bit field).
template <typename T>
__device__ __forceinline__ T rget(const T* __restrict__ R, const SandArgs& a, int q, int kx, int kyp, int kz,
                                  int yflip) {
  int kxp = kx;
  const unsigned odd = (unsigned)(a.oddmask >> (3 * q)) & 7u;
  bool neg = yflip && ((odd >> 1) & 1u);
  if (kx > a.Mx / 2) {
    kxp = a.Mx - kx;
    if (odd & 1u) neg = !neg;
  }
  const T v = ldo(R + (int64_t)q * a.pair_stride, (uint32_t)(((kxp * a.Hy + kyp) * a.H + kz) * (int)sizeof(T)));
  return neg ? -v : v;
}

// component-wise select (a select of whole structs by a runtime flag can be lowered to
// a small table in scratch memory)
template <typename T>
__device__ __forceinline__ C2<T> csel(bool f, C2<T> a, C2<T> b) {
  return C2<T>{f ? a.x : b.x, f ? a.y : b.y};
}

// v[q] *= w^(q ts), w = exp(-+2 pi i / L) from the table (conjugated for sg = +1)
template <typename T, int R>
__device__ __forceinline__ void tw_mul(C2<T>* v, const C2<T>* __restrict__ tw, int ts, T sg) {
#pragma unroll
  for (int q = 1; q < R; ++q) {
    C2<T> w = tw[q * ts];
    w.y *= -sg;
    v[q] = cmul(v[q], w);
  }
}

// forward stage 0 (p = 1): butterfly i of column c straight from HBM (rows >= nrows or
// without the flag bits are zero), outputs y[i R + q] to LDS
template <typename T, int R>
__device__ __forceinline__ void sw_first(const C2<T>* __restrict__ src, uint32_t off0, uint32_t rowb,
                                         const uint8_t* __restrict__ pfl, int msk, int nrows, int L, int i,
                                         bool colok, C2<T>* __restrict__ buf, int ncolp, int c) {
  asm volatile("" : "+v"(i), "+v"(c));   // keep this stage's address arithmetic here (no hoisting)
  const int LR = L / R;
  if (i >= LR) return;
  C2<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = i + q * LR;
    v[q] = C2<T>{T(0), T(0)};
    if (colok && r < nrows && (pfl[r] & msk)) v[q] = ldo(src, off0 + (uint32_t)r * rowb);
  }
  Dft<T, R>::run(v, T(-1));
#pragma unroll
  for (int q = 0; q < R; ++q) buf[(i * R + q) * ncolp + c] = v[Dft<T, R>::pos(q)];
}

// a middle Stockham stage in place in LDS: all reads, barrier, all writes, barrier
template <typename T, int R>
__device__ __forceinline__ void sw_mid(C2<T>* __restrict__ buf, const C2<T>* __restrict__ tw, int L, int p,
                                       float invp, int i, int c, int ncolp, T sg) {
  asm volatile("" : "+v"(i), "+v"(c));   // keep this stage's address arithmetic here (no hoisting)
  const int LR = L / R;
  const bool act = i < LR;
  C2<T> v[R];
  int j = 0;
  if (act) {
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = buf[(i + q * LR) * ncolp + c];
    const int ip = fdiv(i, invp), k = i - ip * p;
    tw_mul<T, R>(v, tw, k * (LR / p), sg);
    Dft<T, R>::run(v, sg);
    j = ip * p * R + k;
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int q = 0; q < R; ++q) buf[(j + q * p) * ncolp + c] = v[Dft<T, R>::pos(q)];
  }
  __syncthreads();
}

// inverse last stage (radix R = f0, p = L/R): LDS -> butterfly -> HBM rows i + q L/R
template <typename T, int R>
__device__ __forceinline__ void sw_last_inv(const C2<T>* __restrict__ buf, const C2<T>* __restrict__ tw, int L, int i,
                                            int c, int ncolp, C2<T>* __restrict__ dst, uint32_t off0, uint32_t rowb,
                                            const uint8_t* __restrict__ pfl, int msk, int nrows, bool colok) {
  asm volatile("" : "+v"(i), "+v"(c));   // keep this stage's address arithmetic here (no hoisting)
  const int LR = L / R;
  if (i >= LR) return;
  C2<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = buf[(i + q * LR) * ncolp + c];
  tw_mul<T, R>(v, tw, i, T(1));
  Dft<T, R>::run(v, T(1));
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = i + q * LR;
    if (colok && r < nrows && (pfl[r] & msk)) sto(dst, off0 + (uint32_t)r * rowb, v[Dft<T, R>::pos(q)]);
  }
}

// radix dispatch for the LDS stages: first / last stage radices in [RS, rmax], middle
// ones in [RS, rmid]
#define VC_SW_SWITCH(RADIX, CALL, HI)                                                                     \
  switch (RADIX) {                                                                                        \
    VC_SW_CASE(2, CALL, HI) VC_SW_CASE(3, CALL, HI) VC_SW_CASE(4, CALL, HI) VC_SW_CASE(5, CALL, HI)       \
    VC_SW_CASE(6, CALL, HI) VC_SW_CASE(7, CALL, HI) VC_SW_CASE(8, CALL, HI) VC_SW_CASE(9, CALL, HI)       \
    VC_SW_CASE(10, CALL, HI) VC_SW_CASE(12, CALL, HI) VC_SW_CASE(14, CALL, HI) VC_SW_CASE(15, CALL, HI)   \
    VC_SW_CASE(16, CALL, HI) VC_SW_CASE(18, CALL, HI) VC_SW_CASE(20, CALL, HI) VC_SW_CASE(21, CALL, HI)   \
    VC_SW_CASE(25, CALL, HI) VC_SW_CASE(27, CALL, HI)                                                     \
    default: break;                                                                                       \
  }
#define VC_SW_CASE(RR, CALL, HI)                   \
  case RR:                                         \
    if constexpr (RR >= RS && RR <= HI) { CALL(RR) } \
    break;

__device__ __forceinline__ int srad(const SandArgs& a, int s) { return (int)((a.radpack >> (5 * s)) & 31u); }

template <typename T, int NIN, int NOUT, int RS>
__global__ void __launch_bounds__(512, (sizeof(T) == 8 || NIN == 6) ? 2 : 3)
k_xsandwich(const C2<T>* __restrict__ Fin, C2<T>* __restrict__ Fout, const T* __restrict__ R, SandArgs a,
            const C2<T>* __restrict__ twg, const C2<T>* __restrict__ phx, const C2<T>* __restrict__ phy,
            const C2<T>* __restrict__ phz, const uint8_t* __restrict__ pflag) {
  constexpr int RMAX = sandwich_rmax((int)sizeof(T)), RMID = sandwich_rmid((int)sizeof(T));
  extern __shared__ char smem_raw[];
  const int L = a.Mx, tl = a.tl, S = a.nst;
  const int lgc = a.lgc, ncol = 1 << lgc, ncolp = ncol + 1;
  C2<T>* tw = reinterpret_cast<C2<T>*>(smem_raw);
  C2<T>* buf = tw + L;
  uint8_t* sflag = reinterpret_cast<uint8_t*>(buf + L * ncolp);   // plane flags of the 3 axes
  const int tid = threadIdx.x;
  const int c_ = tid & (ncol - 1), i_ = tid >> lgc;
  const bool valid = i_ < tl;
  // right-hand sides fastest: the workgroups that read one tile's spectra run together
  // on one XCD, so those spectra come from HBM once per tile rather than once per RHS
  const int ntiles = gridDim.x;
  const int work = xcd_remap(blockIdx.y * ntiles + blockIdx.x, ntiles * gridDim.y);
  const int tile = work / a.nrhs, rhs = work - tile * a.nrhs;
  const int ncols = a.My * a.H;                 // flattened (ky, kz) columns
  const int col = (tile << lgc) + c_;
  const bool colok = col < ncols;
  const int colc = colok ? col : ncols - 1;
  const int ky = fdiv(colc, 1.0f / (float)a.H), kz = colc - ky * a.H;
  const int yflip = ky > a.My / 2;
  const int kyp = yflip ? a.My - ky : ky;
  const uint32_t rowb = (uint32_t)ncols * (uint32_t)sizeof(C2<T>);   // bytes between x rows
  const uint32_t off0 = (uint32_t)colc * (uint32_t)sizeof(C2<T>);
  const int r0 = srad(a, 0);
  for (int t = tid; t < L; t += blockDim.x) tw[t] = twg[t];
  for (int t = tid; t < 3 * a.n1x; t += blockDim.x) sflag[t] = pflag[t];
  __syncthreads();
  const C2<T> phy_t = phy[ky], phz_t = phz[kz];

  C2<T> q[NIN][RS];
#pragma unroll 1
  for (int b = 0; b < NIN; ++b) {
    // opaque per-iteration copies: without them the compiler hoists the address
    // arithmetic of every radix case out of the loop and keeps it all live
    int i = i_, c = c_;
    asm volatile("" : "+v"(i), "+v"(c));
    const int fax = b % 3;
    const int fmsk = NIN == 3 ? 3 : (b < 3 ? 1 : 2);
    const C2<T>* src = Fin + b * a.comp_stride + rhs * a.rhs_stride;
    const uint8_t* pfl = sflag + fax * a.n1x;
    C2<T> v[RS];
    if (S == 1) {
      if (valid) {
#pragma unroll
        for (int m = 0; m < RS; ++m) {
          v[m] = C2<T>{T(0), T(0)};
          if (colok && m < a.n1x && (pfl[m] & fmsk)) v[m] = ldo(src, off0 + (uint32_t)m * rowb);
        }
        Dft<T, RS>::run(v, T(-1));
      }
    } else {
      if (b > 0) __syncthreads();   // readers of the previous component are done with buf
#define VC_CALL(RR) sw_first<T, RR>(src, off0, rowb, pfl, fmsk, a.n1x, L, i, colok, buf, ncolp, c);
      VC_SW_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
      __syncthreads();
      int p = r0;
      for (int s = 1; s < S - 1; ++s) {
        const int rs = srad(a, s);
        const float invp = 1.0f / (float)p;
#define VC_CALL(RR) sw_mid<T, RR>(buf, tw, L, p, invp, i, c, ncolp, T(-1));
        VC_SW_SWITCH(rs, VC_CALL, RMID)
#undef VC_CALL
        p *= rs;
      }
      if (valid) {
        // last forward stage (radix RS, p = tl): butterfly i reads rows i + q tl,
        // twiddle exponent q i, outputs X[i + q tl]
#pragma unroll
        for (int m = 0; m < RS; ++m) v[m] = buf[(i + m * tl) * ncolp + c];
        tw_mul<T, RS>(v, tw, i, T(-1));
        Dft<T, RS>::run(v, T(-1));
      }
    }
    // half-voxel phase of the input component (shift to the common lattice); slot
    // pos(m) holds X[i + m tl]
    if (valid) {
      const C2<T> phyz = csel(fax == 1, phy_t, phz_t);
#pragma unroll
      for (int m = 0; m < RS; ++m) {
        const C2<T> ph = fax == 0 ? phx[i + m * tl] : phyz;
        const C2<T> w = cmul(v[Dft<T, RS>::pos(m)], ph);
#pragma unroll
        for (int bb = 0; bb < NIN; ++bb)
          if (bb == b) q[bb][m] = w;
      }
    }
  }

#pragma unroll 1
  for (int o = 0; o < NOUT; ++o) {
    int i = i_, c = c_;
    asm volatile("" : "+v"(i), "+v"(c));
    const int oax = NIN == 3 ? (o < 3 ? o : o - 3) : o;
    C2<T> z[RS];
    if (valid) {
      const C2<T> phyz = csel(oax == 1, phy_t, phz_t);
#pragma unroll
      for (int m = 0; m < RS; ++m) {
        const int kx = i + m * tl;
        C2<T> acc = {T(0), T(0)};
        if (NIN == 3) {
          // o < 3: C_alpha = sum_b P(alpha,b) Q'_b ; o >= 3: D_alpha = i sum_b E(alpha,b) Q'_b
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            const int qi = o < 3 ? (oax == b ? oax : 2 + oax + b) : 6 + 3 * oax + b;
            const T rv = rget(R, a, qi, kx, kyp, kz, yflip);
            acc.x += rv * q[b][m].x;
            acc.y += rv * q[b][m].y;
          }
          if (o >= 3) acc = C2<T>{-acc.y, acc.x};
        } else {
          // transposed product: out_b = sum_al P(al,b) X'C_al - i sum_al E(al,b) X'D_al
          C2<T> accE = {T(0), T(0)};
#pragma unroll
          for (int al = 0; al < 3; ++al) {
            const int qp = al == oax ? al : 2 + al + oax;
            const T rp = rget(R, a, qp, kx, kyp, kz, yflip);
            acc.x += rp * q[al][m].x;
            acc.y += rp * q[al][m].y;
            const T re = rget(R, a, 6 + 3 * al + oax, kx, kyp, kz, yflip);
            accE.x += re * q[(NIN > 3 ? 3 : 0) + al][m].x;
            accE.y += re * q[(NIN > 3 ? 3 : 0) + al][m].y;
          }
          acc.x += accE.y;   // -i * accE
          acc.y -= accE.x;
        }
        // output phase: conj of the half-voxel shift of the output component
        const C2<T> ph = oax == 0 ? phx[kx] : phyz;
        z[m] = cmul(acc, cconj(ph));
      }
    }
    const int msk = NIN == 3 ? (o < 3 ? 1 : 2) : 3;
    C2<T>* dst = Fout + o * a.comp_stride + rhs * a.rhs_stride;
    const uint8_t* pfl = sflag + oax * a.n1x;
    if (S == 1) {
      if (valid) {
        Dft<T, RS>::run(z, T(1));
#pragma unroll
        for (int m = 0; m < RS; ++m)
          if (colok && m < a.n1x && (pfl[m] & msk)) sto(dst, off0 + (uint32_t)m * rowb, z[Dft<T, RS>::pos(m)]);
      }
    } else {
      __syncthreads();   // the previous readers of buf are done
      if (valid) {
        // first inverse stage (radix RS, p = 1) on the held values X[i + q tl]
        Dft<T, RS>::run(z, T(1));
#pragma unroll
        for (int m = 0; m < RS; ++m) buf[(i * RS + m) * ncolp + c] = z[Dft<T, RS>::pos(m)];
      }
      __syncthreads();
      int p = RS;
      for (int s = S - 2; s >= 1; --s) {
        const int rs = srad(a, s);
        const float invp = 1.0f / (float)p;
#define VC_CALL(RR) sw_mid<T, RR>(buf, tw, L, p, invp, i, c, ncolp, T(1));
        VC_SW_SWITCH(rs, VC_CALL, RMID)
#undef VC_CALL
        p *= rs;
      }
#define VC_CALL(RR) sw_last_inv<T, RR>(buf, tw, L, i, c, ncolp, dst, off0, rowb, pfl, msk, a.n1x, colok);
      VC_SW_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
    }
  }
}
#undef VC_SW_CASE
#undef VC_SW_SWITCH

// Compiled last-stage radices per kernel variant (register budget: the thread holds
// NIN x RS transformed inputs).
template <typename T, int NIN> struct SandRS {
  static constexpr int max = sandwich_rs_max((int)sizeof(T), NIN);
};

template <typename T, int NIN, int NOUT>
hipError_t launch_sandwich_v(const void* Fin, void* Fout, const void* R, const SandArgs& a, const void* tw,
                             const void* phx, const void* phy, const void* phz, const uint8_t* pflag, int nthr,
                             size_t lds, int rs, hipStream_t st) {
  dim3 grid((a.My * a.H + (1 << a.lgc) - 1) >> a.lgc, a.nrhs);
#define VC_RS(RR)                                                                                                 \
  case RR:                                                                                                        \
    if constexpr (RR <= SandRS<T, NIN>::max) {                                                                    \
      hipLaunchKernelGGL((k_xsandwich<T, NIN, NOUT, RR>), grid, dim3(nthr), lds, st, (const C2<T>*)Fin,          \
                         (C2<T>*)Fout, (const T*)R, a, (const C2<T>*)tw, (const C2<T>*)phx, (const C2<T>*)phy,    \
                         (const C2<T>*)phz, pflag);                                                               \
      return hipGetLastError();                                                                                   \
    }                                                                                                             \
    break;
  switch (rs) {
    VC_RS(2) VC_RS(3) VC_RS(4) VC_RS(5) VC_RS(6) VC_RS(7) VC_RS(8) VC_RS(9) VC_RS(10)
    default: break;
  }
#undef VC_RS
  return hipErrorInvalidValue;
}

}  // namespace vc
