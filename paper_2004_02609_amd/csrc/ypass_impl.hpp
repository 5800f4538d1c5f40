// y pass of the FFT product of eq. (11) (Sec. II.B): the C2C transform along y of
// every stored x plane, forward (after the z pass) or inverse (before it), for one tile
// of consecutive kz columns of one (component, right-hand side, x plane) per workgroup.
//
// Same register-edge Stockham structure as the x pass (sandwich_impl.hpp), without the
// multiply: with radices f0 >= ... >= RS (RS compile-time), thread (i, c) owns
// butterfly i < L/RS of column c, columns fastest across lanes;
//   stage 0 (radix f0, p = 1):  HBM rows i + q L/f0 -> registers -> LDS
//   middle stages:              LDS -> LDS in place
//   last stage (radix RS):      LDS -> registers -> HBM rows i + m L/RS
// so each column crosses LDS once plus once per middle stage, and the HBM reads and
// writes of a row touch the tile's consecutive columns.  The inverse transform is the
// same pipeline with conjugate twiddles.  Rows are pruned by per-line flags: only
// stored input rows are read and only needed output rows are written.
#pragma once
#include "sandwich_impl.hpp"

namespace vc {

// first stage (p = 1) on staged inputs: DFT of sign sg, outputs y[i R + q] to LDS
template <typename T, int R>
__device__ __forceinline__ void yp_first(const C2<T>* __restrict__ pre, bool act, T sg, char* __restrict__ lds,
                                         uint32_t wbase, uint32_t ncolpE) {
  if (!act) return;
  C2<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = pre[q];
  Dft<T, R>::run(v, sg);
  uint32_t o = wbase;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    lds_st<T>(lds, o, v[Dft<T, R>::pos(q)]);
    o += ncolpE;
  }
}

#define VC_YP_SWITCH(RADIX, CALL, HI)                                                                     \
  switch (RADIX) {                                                                                        \
    VC_YP_CASE(2, CALL, HI) VC_YP_CASE(3, CALL, HI) VC_YP_CASE(4, CALL, HI) VC_YP_CASE(5, CALL, HI)       \
    VC_YP_CASE(6, CALL, HI) VC_YP_CASE(7, CALL, HI) VC_YP_CASE(8, CALL, HI) VC_YP_CASE(9, CALL, HI)       \
    VC_YP_CASE(10, CALL, HI)                                                                              \
    default: break;                                                                                       \
  }
#define VC_YP_CASE(RR, CALL, HI)                     \
  case RR:                                           \
    if constexpr (RR >= RS && RR <= HI) { CALL(RR) } \
    break;

// One (column tile, x plane, component x right-hand side) of the pass.  PID > 0: the plan
// of kSandFixed[PID] as compile-time constants (the kernel checks it is a's).  act: the
// right-hand sides' activity (null: all active).
template <typename T, int RS, int PID>
__device__ __forceinline__ void ypass_body(C2<T>* __restrict__ data, const YArgs& a, const C2<T>* __restrict__ twg,
                                           const uint8_t* __restrict__ lflag, const uint8_t* __restrict__ pflag,
                                           const int* __restrict__ act, int tile, int plane, int bz) {
  constexpr bool FX = PID > 0;
  constexpr SandFixedPlan PD = kSandFixed[PID];
  constexpr int RMAX = 10;
  constexpr uint32_t E = sizeof(C2<T>);
  const int cz = bz / a.nrhs, rhs = bz - cz * a.nrhs;
  if (act && !act[rhs]) return;   // uniform per workgroup
  const int comp = a.cs.comp[cz], axis = a.cs.axis[cz];
  const int min_ = a.cs.min_[cz], mout = a.cs.mout[cz];
  const int need = a.inverse ? mout : min_;
  if (pflag && need && !(pflag[axis * a.n1x + plane] & need)) return;   // uniform per workgroup
  extern __shared__ char smem_raw[];
  const int L = FX ? PD.L : a.L, tl = FX ? PD.L / RS : a.tl, S = FX ? PD.nst : a.nst, ncol = a.ncol;
  auto rad = [&](int s) -> int { return FX ? PD.r[s] : (int)((a.radpack >> (5 * s)) & 31u); };
  const T sg = a.inverse ? T(1) : T(-1);
  const uint32_t ncolpE = (uint32_t)(ncol + 1) * E;
  char* twb = smem_raw;                       // L twiddles
  char* lds = smem_raw + (size_t)L * E;       // [L][ncol + 1] tile
  const int tid = threadIdx.x;
  const int i = fdiv(tid, 1.0f / (float)ncol), c = tid - i * ncol;   // column fastest
  const bool valid = i < tl;
  const int col = tile * ncol + c;
  const bool colok = col < a.ncols;
  const int colc = colok ? col : a.ncols - 1;
  // buffer view of this (component, rhs, plane) slab: masked rows read zero / write nothing
  const Buf base = make_buf(data + comp * a.comp_stride + rhs * a.rhs_stride + plane * a.plane_stride,
                            (uint32_t)a.plane_stride * E);
  const uint8_t* lf = lflag ? lflag + ((int64_t)axis * a.n1x + plane) * a.n1y : nullptr;
  // half-voxel phase of this component along y (null: none): ph[ky] on the forward
  // outputs, conj(ph[ky]) on the inverse inputs
  const C2<T>* __restrict__ ph = (a.ph && axis == a.phax) ? static_cast<const C2<T>*>(a.ph) : nullptr;
  const uint32_t rowb = (uint32_t)a.row_stride * E;
  const int r0 = rad(0);
  const int LR0 = L / r0;
  const bool act0 = i < LR0;
  for (int t = tid; t < L; t += blockDim.x) lds_st<T>(twb, (uint32_t)t * E, twg[t]);
  // input rows i + q L/f0 that are stored (bit q), output rows i + m tl that are needed
  uint32_t inmask = 0u, outmask = 0u;
  if (colok) {
    if (act0)
      for (int q = 0; q < r0; ++q) {
        const int r = i + q * LR0;
        if (r < a.nin && (!lf || !min_ || (lf[r] & min_))) inmask |= 1u << q;
      }
    if (valid)
      for (int m = 0; m < RS; ++m) {
        const int r = i + m * tl;
        if (r < a.nout && (!lf || !mout || (lf[r] & mout))) outmask |= 1u << m;
      }
  }
  const uint32_t cE = (uint32_t)c * E;
  const uint32_t rbase = (uint32_t)i * ncolpE + cE;
  const uint32_t gbase = (uint32_t)colc * E + (uint32_t)i * rowb;
  if (S == 1) {
    // one stage of radix RS = L (tl = 1): rows m straight in and out
    __syncthreads();
    if (valid) {
      C2<T> v[RS];
      uint32_t o = gbase;
#pragma unroll
      for (int m = 0; m < RS; ++m) {
        v[m] = bld<T>(base, (inmask & (1u << m)) ? o : kOob);
        o += rowb;
      }
      if (ph && a.inverse) {
#pragma unroll
        for (int m = 0; m < RS; ++m) v[m] = cmul(v[m], cconj(ph[m]));
      }
      Dft<T, RS>::run(v, sg);
      if (ph && !a.inverse) {
#pragma unroll
        for (int m = 0; m < RS; ++m) v[Dft<T, RS>::pos(m)] = cmul(v[Dft<T, RS>::pos(m)], ph[m]);
      }
      o = gbase;
#pragma unroll
      for (int m = 0; m < RS; ++m) {
        bst<T>(base, (outmask & (1u << m)) ? o : kOob, v[Dft<T, RS>::pos(m)]);
        o += rowb;
      }
    }
    return;
  }
  C2<T> pre[RMAX];
  {
    const uint32_t gstride = (uint32_t)LR0 * rowb;
#define VC_CALL(RR) sw_load<T, RR>(pre, base, gbase, gstride, inmask, act0);
    VC_YP_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
  }
  __syncthreads();   // twiddles in LDS
  if (ph && a.inverse && act0) {
    // inputs rows i + q L/f0
#define VC_CALL(RR)                                                   \
  _Pragma("unroll") for (int q = 0; q < RR; ++q) pre[q] = cmul(pre[q], cconj(ph[i + q * LR0]));
    VC_YP_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
  }
  {
    uint32_t wbase = (uint32_t)i * (uint32_t)r0 * ncolpE + cE;
    asm volatile("" : "+v"(wbase));
#define VC_CALL(RR) yp_first<T, RR>(pre, act0, sg, lds, wbase, ncolpE);
    VC_YP_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
  }
  __syncthreads();
  int p = r0;
#pragma unroll
  for (int s = 1; s < (FX ? PD.nst : S) - 1; ++s) {
    const int rs = rad(s);
    const float invp = stage_inv(p);
#define VC_CALL(RR) sw_mid<T, RR>(lds, twb, L, p, invp, i, rbase, cE, ncolpE, sg);
    VC_YP_SWITCH(rs, VC_CALL, RMAX)
#undef VC_CALL
    p *= rs;
  }
  if (valid) {
    // last stage (radix RS, p = tl): rows i + m tl, twiddle exponent m i, outputs
    // X[i + m tl] straight to HBM
    C2<T> v[RS];
    const uint32_t st = (uint32_t)tl * ncolpE;
    uint32_t o = rbase;
#pragma unroll
    for (int m = 0; m < RS; ++m) {
      v[m] = lds_ld<T>(lds, o);
      o += st;
    }
    tw_mul<T, RS>(v, twb, (uint32_t)i * E, sg);
    Dft<T, RS>::run(v, sg);
    if (ph && !a.inverse) {
      // outputs X[i + m tl]
#pragma unroll
      for (int m = 0; m < RS; ++m) v[Dft<T, RS>::pos(m)] = cmul(v[Dft<T, RS>::pos(m)], ph[i + m * tl]);
    }
    uint32_t og = gbase;
    const uint32_t gs = (uint32_t)tl * rowb;
#pragma unroll
    for (int m = 0; m < RS; ++m) {
      bst<T>(base, (outmask & (1u << m)) ? og : kOob, v[Dft<T, RS>::pos(m)]);
      og += gs;
    }
  }
}

// Several adjacent columns per thread (FP32, compiled plans, tile widths a multiple of
// CPT): thread (i, g) owns butterfly i of columns CPT g .. CPT g + CPT - 1, so the index
// arithmetic, row flags and twiddle reads of a butterfly serve all of them and a tile
// needs 1/CPT of the waves.  Same stages, masks and phases as ypass_body.  Launched with
// CPT = 2 (four columns per thread measured slower: 80-110 VGPRs, 4-6 waves per SIMD).
template <typename T, int R, int CPT>
__device__ __forceinline__ void tw_mul_n(C2<T> (&v)[CPT][R], const char* __restrict__ twb, uint32_t tsb, T sg) {
  C2<T> w[R];
  uint32_t o = 0;
#pragma unroll
  for (int q = 1; q < R; ++q) {
    o += tsb;
    w[q] = lds_ld<T>(twb, o);
  }
#pragma unroll
  for (int q = 1; q < R; ++q) {
    w[q].y *= -sg;
#pragma unroll
    for (int j = 0; j < CPT; ++j) v[j][q] = cmul(v[j][q], w[q]);
  }
}

// a middle Stockham stage of radix R (p = product of the earlier radices) on the
// thread's columns, in place in LDS: reads, barrier, writes, barrier
template <typename T, int L, int R, int P, int CPT>
__device__ __forceinline__ void yp_mid_n(char* __restrict__ lds, const char* __restrict__ twb, int i, uint32_t rbase,
                                         uint32_t cE, uint32_t ncolpE, T sg) {
  constexpr uint32_t E = sizeof(C2<T>);
  constexpr int LR = L / R;
  asm volatile("" : "+v"(i), "+v"(rbase));   // keep this stage's address arithmetic here
  const bool act = i < LR;
  C2<T> v[CPT][R];
  uint32_t wb = 0;
  if (act) {
    const uint32_t rstride = (uint32_t)LR * ncolpE;
    uint32_t o = rbase;
#pragma unroll
    for (int q = 0; q < R; ++q) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) v[j][q] = lds_ld<T>(lds, o + j * E);
      o += rstride;
    }
    const int ip = i / P, k = i - ip * P;
    tw_mul_n<T, R, CPT>(v, twb, (uint32_t)(k * (LR / P)) * E, sg);
#pragma unroll
    for (int j = 0; j < CPT; ++j) Dft<T, R>::run(v[j], sg);
    wb = (uint32_t)(ip * P * R + k) * ncolpE + cE;
  }
  __syncthreads();
  if (act) {
    const uint32_t wstride = (uint32_t)P * ncolpE;
#pragma unroll
    for (int q = 0; q < R; ++q) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) lds_st<T>(lds, wb + j * E, v[j][Dft<T, R>::pos(q)]);
      wb += wstride;
    }
  }
  __syncthreads();
}

template <typename T, int RS, int PID, int CPT>
__device__ __forceinline__ void ypass_body_n(C2<T>* __restrict__ data, const YArgs& a, const C2<T>* __restrict__ twg,
                                             const uint8_t* __restrict__ lflag, const uint8_t* __restrict__ pflag,
                                             const int* __restrict__ act, int tile, int plane, int bz) {
  constexpr SandFixedPlan PD = kSandFixed[PID];
  constexpr int L = PD.L, TL = PD.L / RS, S = PD.nst, R0 = PD.r[0], LR0 = PD.L / PD.r[0];
  static_assert(PID > 0 && S >= 2 && S <= 4 && PD.r[S - 1] == RS, "compiled plans of 2 to 4 stages");
  constexpr uint32_t E = sizeof(C2<T>);
  const int cz = bz / a.nrhs, rhs = bz - cz * a.nrhs;
  if (act && !act[rhs]) return;   // uniform per workgroup
  const int comp = a.cs.comp[cz], axis = a.cs.axis[cz];
  const int min_ = a.cs.min_[cz], mout = a.cs.mout[cz];
  const int need = a.inverse ? mout : min_;
  if (pflag && need && !(pflag[axis * a.n1x + plane] & need)) return;   // uniform per workgroup
  extern __shared__ char smem_raw[];
  const T sg = a.inverse ? T(1) : T(-1);
  const int ncol = a.ncol, ngrp = ncol / CPT;
  const uint32_t ncolpE = (uint32_t)(ncol + 1) * E;
  char* twb = smem_raw;                       // L twiddles
  char* lds = smem_raw + (size_t)L * E;       // [L][ncol + 1] tile
  const int tid = threadIdx.x;
  const int i = fdiv(tid, 1.0f / (float)ngrp), cg = tid - i * ngrp;   // column groups fastest
  const bool valid = i < TL;
  const int c0 = CPT * cg;
  const int col0 = tile * ncol + c0;
  const int colc = col0 < a.ncols ? col0 : a.ncols - 1;
  const Buf base = make_buf(data + comp * a.comp_stride + rhs * a.rhs_stride + plane * a.plane_stride,
                            (uint32_t)a.plane_stride * E);
  const uint8_t* lf = lflag ? lflag + ((int64_t)axis * a.n1x + plane) * a.n1y : nullptr;
  const C2<T>* __restrict__ ph = (a.ph && axis == a.phax) ? static_cast<const C2<T>*>(a.ph) : nullptr;
  const uint32_t rowb = (uint32_t)a.row_stride * E;
  const bool act0 = i < LR0;
  for (int t = tid; t < L; t += blockDim.x) lds_st<T>(twb, (uint32_t)t * E, twg[t]);
  // rows of the first stage's inputs that are stored and of the last stage's outputs
  // that are needed (the same rows for every column of the thread)
  uint32_t inmask = 0u, outmask = 0u;
  if (col0 < a.ncols) {
    if (act0)
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const int r = i + q * LR0;
        if (r < a.nin && (!lf || !min_ || (lf[r] & min_))) inmask |= 1u << q;
      }
    if (valid)
#pragma unroll
      for (int m = 0; m < RS; ++m) {
        const int r = i + m * TL;
        if (r < a.nout && (!lf || !mout || (lf[r] & mout))) outmask |= 1u << m;
      }
  }
  // columns past the end read zero and store nothing
  uint32_t cin[CPT], cout[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const bool ok = col0 + j < a.ncols;
    cin[j] = ok ? inmask : 0u;
    cout[j] = ok ? outmask : 0u;
  }
  const uint32_t cE = (uint32_t)c0 * E;
  const uint32_t rbase = (uint32_t)i * ncolpE + cE;
  const uint32_t gbase = (uint32_t)colc * E + (uint32_t)i * rowb;
  // first stage (radix R0, p = 1): HBM rows i + q L/R0 -> registers -> LDS rows i R0 + q
  C2<T> u[CPT][R0];
  if (act0) {
    const uint32_t gstride = (uint32_t)LR0 * rowb;
    uint32_t o = gbase;
#pragma unroll
    for (int q = 0; q < R0; ++q) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) u[j][q] = bld<T>(base, (cin[j] & (1u << q)) ? o + j * E : kOob);
      o += gstride;
    }
  }
  __syncthreads();   // twiddles in LDS
  if (act0) {
    if (ph && a.inverse) {
#pragma unroll
      for (int q = 0; q < R0; ++q) {
        const C2<T> w = cconj(ph[i + q * LR0]);
#pragma unroll
        for (int j = 0; j < CPT; ++j) u[j][q] = cmul(u[j][q], w);
      }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) Dft<T, R0>::run(u[j], sg);
    uint32_t o = (uint32_t)i * (uint32_t)R0 * ncolpE + cE;
    asm volatile("" : "+v"(o));
#pragma unroll
    for (int q = 0; q < R0; ++q) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) lds_st<T>(lds, o + j * E, u[j][Dft<T, R0>::pos(q)]);
      o += ncolpE;
    }
  }
  __syncthreads();
  if constexpr (S >= 3) yp_mid_n<T, L, PD.r[1], PD.r[0], CPT>(lds, twb, i, rbase, cE, ncolpE, sg);
  if constexpr (S >= 4) yp_mid_n<T, L, PD.r[2], PD.r[0] * PD.r[1], CPT>(lds, twb, i, rbase, cE, ncolpE, sg);
  if (valid) {
    // last stage (radix RS, p = L/RS): rows i + m TL, twiddle exponent m i, outputs
    // X[i + m TL] straight to HBM
    C2<T> v[CPT][RS];
    const uint32_t st = (uint32_t)TL * ncolpE;
    uint32_t o = rbase;
#pragma unroll
    for (int m = 0; m < RS; ++m) {
#pragma unroll
      for (int j = 0; j < CPT; ++j) v[j][m] = lds_ld<T>(lds, o + j * E);
      o += st;
    }
    tw_mul_n<T, RS, CPT>(v, twb, (uint32_t)i * E, sg);
#pragma unroll
    for (int j = 0; j < CPT; ++j) Dft<T, RS>::run(v[j], sg);
    if (ph && !a.inverse) {
#pragma unroll
      for (int m = 0; m < RS; ++m) {
        const C2<T> w = ph[i + m * TL];
#pragma unroll
        for (int j = 0; j < CPT; ++j) v[j][Dft<T, RS>::pos(m)] = cmul(v[j][Dft<T, RS>::pos(m)], w);
      }
    }
    uint32_t og = gbase;
    const uint32_t gs = (uint32_t)TL * rowb;
#pragma unroll
    for (int m = 0; m < RS; ++m) {
#pragma unroll
      for (int j = 0; j < CPT; ++j)
        bst<T>(base, (cout[j] & (1u << m)) ? og + j * E : kOob, v[j][Dft<T, RS>::pos(m)]);
      og += gs;
    }
  }
}

// workgroup -> (tile, plane, component x rhs).  Workgroups are issued to the 8 XCDs in
// turn by linear id w; with XCD grouping (a.xg) the G consecutive tiles of a row, whose
// rows share cache lines, go to w, w + 8, ..., w + 8 (G - 1), which sit on one XCD and
// start together (a bijection on the largest multiple of 8 G; the rest keep their
// order); xg < 0: G = every tile of the row.
__device__ __forceinline__ void ypass_coords(const YArgs& a, int* tile, int* plane, int* bz) {
  *tile = blockIdx.x;
  *plane = blockIdx.y;
  *bz = blockIdx.z;
  if (a.xg > 1 || (a.xg < 0 && gridDim.x > 1)) {
    const uint32_t gx = gridDim.x, gy = gridDim.y, G = a.xg > 0 ? (uint32_t)a.xg : gx, span = 8u * G;
    const uint32_t W = gx * gy * gridDim.z;
    const uint32_t w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    uint32_t l = w;
    if (w < W / span * span) {
      const uint32_t k = w >> 3;
      l = (k / G) * span + (w & 7u) * G + k % G;
    }
    *tile = (int)(l % gx);
    const uint32_t r = l / gx;
    *plane = (int)(r % gy);
    *bz = (int)(r / gy);
  }
}

template <typename T, int RS, int PID, int CPT>
__global__ void __launch_bounds__(1024)
k_ypass_n(C2<T>* __restrict__ data, YArgs a, const C2<T>* __restrict__ twg, const uint8_t* __restrict__ lflag,
          const uint8_t* __restrict__ pflag) {
  if (a.skip && *a.skip) return;
  if (a.L != kSandFixed[PID].L || a.nst != kSandFixed[PID].nst || a.radpack != sand_fixed_pack(PID) ||
      a.tl * RS != a.L || a.ncol % CPT != 0)
    return;
  int tile, plane, bz;
  ypass_coords(a, &tile, &plane, &bz);
  ypass_body_n<T, RS, PID, CPT>(data, a, twg, lflag, pflag, a.act, tile, plane, bz);
}

template <typename T, int RS, int PID = 0>
__global__ void __launch_bounds__(1024)
k_ypass(C2<T>* __restrict__ data, YArgs a, const C2<T>* __restrict__ twg, const uint8_t* __restrict__ lflag,
        const uint8_t* __restrict__ pflag) {
  if (a.skip && *a.skip) return;
  if (PID > 0 && (a.L != kSandFixed[PID].L || a.nst != kSandFixed[PID].nst || a.radpack != sand_fixed_pack(PID) ||
                  a.tl * RS != a.L))
    return;
  int tile, plane, bz;
  ypass_coords(a, &tile, &plane, &bz);
  ypass_body<T, RS, PID>(data, a, twg, lflag, pflag, a.act, tile, plane, bz);
}

// several scenes in one launch (the members of a packed set with last radix RS):
// linear workgroup -> (scene, component x rhs, plane, tile)
template <typename T, int RS>
__global__ void __launch_bounds__(1024)
k_ypass_multi(const YScene* __restrict__ tab, int nscene, const int* __restrict__ skip, const int* __restrict__ act) {
  if (skip && *skip) return;
  const int lin = blockIdx.x;
  const YScene& sc = tab[find_scene(tab, nscene, lin)];
  const int local = lin - sc.blk0;
  const int per = sc.gx * sc.gy;
  const int bz = local / per, rem = local - bz * per;
  const int plane = rem / sc.gx, tile = rem - plane * sc.gx;
  ypass_body<T, RS, 0>(static_cast<C2<T>*>(sc.data), sc.a, static_cast<const C2<T>*>(sc.tw), sc.lflag, sc.pflag,
                       act ? act + sc.c0 : nullptr, tile, plane, bz);
}
#undef VC_YP_CASE
#undef VC_YP_SWITCH

// launch with last-stage radix RR: the fixed-plan kernel of the first table entry that
// equals the runtime plan, else the generic one
template <typename T, int RR, int ID>
hipError_t launch_ypass_rs(void* data, const YArgs& a, const void* tw, const uint8_t* lflag, const uint8_t* pflag,
                           dim3 grid, int nthr, size_t lds, int cpt, hipStream_t st) {
  if constexpr (ID < kSandNumFixed) {
    if constexpr (sand_fixed_last(ID) == RR) {
      if (a.L == kSandFixed[ID].L && a.nst == kSandFixed[ID].nst && a.radpack == sand_fixed_pack(ID) &&
          a.tl * RR == a.L) {
        if constexpr (sizeof(T) == 4 && kSandFixed[ID].nst >= 2 && kSandFixed[ID].nst <= 4) {
          auto go = [&](auto kernel) -> hipError_t {
            if (lds > kLdsBudget) {
              const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
              if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL(kernel, grid, dim3(nthr), lds, st, (C2<T>*)data, a, (const C2<T>*)tw, lflag, pflag);
            return hipGetLastError();
          };
          if (cpt == 2) return go(k_ypass_n<T, RR, ID, 2>);
        }
        if (cpt != 1) return hipErrorInvalidValue;
        if (lds > kLdsBudget) {
          const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ypass<T, RR, ID>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
          if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_ypass<T, RR, ID>), grid, dim3(nthr), lds, st, (C2<T>*)data, a, (const C2<T>*)tw,
                           lflag, pflag);
        return hipGetLastError();
      }
    }
    return launch_ypass_rs<T, RR, ID + 1>(data, a, tw, lflag, pflag, grid, nthr, lds, cpt, st);
  } else {
    if (cpt != 1) return hipErrorInvalidValue;
    if (lds > kLdsBudget) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ypass<T, RR, 0>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_ypass<T, RR, 0>), grid, dim3(nthr), lds, st, (C2<T>*)data, a, (const C2<T>*)tw, lflag,
                       pflag);
    return hipGetLastError();
  }
}

// every assumption of the kernel on its arguments, the LDS bytes it needs in *lds
template <typename T>
bool ypass_args_ok(const YArgs& a, int nthr, bool flags, size_t* lds_out, int cpt) {
  if (a.nst < 1 || a.nst > kSandMaxStages || a.ncol < 1 || a.ncol > 32 || nthr < 64 || nthr > 1024 || (nthr & 63) ||
      a.cs.n < 1 || a.cs.n > 6 || a.nrhs < 1 || !(a.xg >= -1 && a.xg <= 4 && a.xg != 3))
    return false;
  long prod = 1;
  int prev = 1 << 30;
  for (int s = 0; s < a.nst; ++s) {
    const int r = (int)((a.radpack >> (5 * s)) & 31u);
    if (r < 2 || r > 10 || r > prev) return false;
    prev = r;
    prod *= r;
  }
  if (!(cpt == 1 || cpt == 2) || a.ncol % cpt != 0) return false;
  if (prod != a.L || (long)a.tl * prev != a.L || (long)a.tl * (a.ncol / cpt) > nthr) return false;
  if (a.nin > a.L || a.nout > a.L) return false;
  if (flags)
    for (int q = 0; q < a.cs.n; ++q)
      if ((a.cs.min_[q] && a.nin > a.n1y) || (a.cs.mout[q] && a.nout > a.n1y)) return false;
  if ((uint64_t)a.plane_stride * sizeof(C2<T>) > 0xFFFFFF00ull) return false;
  const size_t lds = (size_t)sizeof(C2<T>) * ((size_t)a.L + (size_t)a.L * (a.ncol + 1));
  if (lds > lds_ext_budget()) return false;
  *lds_out = lds;
  return true;
}

template <typename T>
hipError_t launch_ypass_multi(const YScene* tab, int nscene, int nblocks, int rs, int nthr, size_t lds,
                              const int* skip, const int* act, hipStream_t st) {
  if (nscene <= 0 || nblocks <= 0) return hipSuccess;
  if (nthr < 64 || nthr > 1024 || (nthr & 63) || lds > lds_ext_budget()) return hipErrorInvalidValue;
#define VC_RS(RR)                                                                                              \
  case RR:                                                                                                     \
    if (lds > kLdsBudget) {                                                                                    \
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ypass_multi<T, RR>),            \
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);           \
      if (e != hipSuccess) return e;                                                                           \
    }                                                                                                          \
    hipLaunchKernelGGL((k_ypass_multi<T, RR>), dim3(nblocks), dim3(nthr), lds, st, tab, nscene, skip, act);     \
    return hipGetLastError();
  switch (rs) {
    VC_RS(2) VC_RS(3) VC_RS(4) VC_RS(5) VC_RS(6) VC_RS(7) VC_RS(8) VC_RS(9) VC_RS(10)
    default: break;
  }
#undef VC_RS
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_ypass(void* data, const YArgs& a, const void* tw, const uint8_t* lflag, const uint8_t* pflag,
                        int nplanes, int nthr, hipStream_t st) {
  // every assumption of the kernel (plan, tile, flag rows, 32-bit slab offsets, LDS)
  size_t lds = 0;
  const int cpt = ypass_cols_per_thread(a.L, a.nst, a.radpack, a.tl, a.ncol, (int)sizeof(T));
  if (!ypass_args_ok<T>(a, nthr, lflag != nullptr, &lds, cpt)) return hipErrorInvalidValue;
  const int rs = (int)((a.radpack >> (5 * (a.nst - 1))) & 31u);
  dim3 grid((a.ncols + a.ncol - 1) / a.ncol, nplanes, a.cs.n * a.nrhs);
#define VC_RS(RR)                                                                                \
  case RR:                                                                                       \
    return launch_ypass_rs<T, RR, 1>(data, a, tw, lflag, pflag, grid, nthr, lds, cpt, st);
  switch (rs) {
    VC_RS(2) VC_RS(3) VC_RS(4) VC_RS(5) VC_RS(6) VC_RS(7) VC_RS(8) VC_RS(9) VC_RS(10)
    default: break;
  }
#undef VC_RS
  return hipErrorInvalidValue;
}

}  // namespace vc
