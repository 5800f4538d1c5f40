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
//
// Instruction economy (the pass is bound by vector-instruction issue): every LDS and
// HBM address is a per-thread byte base computed once plus a workgroup-uniform stride
// (one add per element); the rows a thread's first / last butterfly touches are
// validated once into bit masks; the spectra offsets and fold signs of the thread's
// frequencies are computed once, so each multiply term is a load, a sign flip and two
// FMAs.
#pragma once
#include <hip/hip_ext.h>

#include "fft_core.hpp"
#include "mvp_kernels.h"

namespace vc {

// Workgroups are dispatched to the 8 XCDs round-robin by linear id; this maps linear id
// -> work index so that each XCD gets one contiguous range of work.
__device__ __forceinline__ int xcd_remap(int lin, int n) {
  const int xcd = lin & 7, idx = lin >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Loads / stores at a base plus a 32-bit byte offset (the launcher checks every array
// slab the sandwich indexes is below 4 GiB), one VGPR per address.
template <typename V>
__device__ __forceinline__ V ldo(const V* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename V>
__device__ __forceinline__ void sto(V* __restrict__ base, uint32_t byte_off, V v) {
  *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// Raw buffer views (stride 0) of one array slab: an access at a byte offset at or past
// the slab's size reads zero and a store there writes nothing (the memory unit's range
// check).  Masked row accesses pass kOob instead of branching around the access, and
// each address is a uniform resource plus one 32-bit offset.  Slabs are at most kOob
// bytes (checked by the launchers).
constexpr uint32_t kOob = 0xFFFFFFF0u;
struct Buf {
  __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ Buf make_buf(const void* p, uint32_t bytes) {
  return Buf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000)};
}
typedef unsigned int vc_u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int vc_u32x4 __attribute__((ext_vector_type(4)));
template <typename T> __device__ __forceinline__ C2<T> bld(Buf b, uint32_t off);
template <> __device__ __forceinline__ C2<float> bld<float>(Buf b, uint32_t off) {
  return __builtin_bit_cast(C2<float>, __builtin_amdgcn_raw_buffer_load_b64(b.r, off, 0, 0));
}
template <> __device__ __forceinline__ C2<double> bld<double>(Buf b, uint32_t off) {
  return __builtin_bit_cast(C2<double>, __builtin_amdgcn_raw_buffer_load_b128(b.r, off, 0, 0));
}
template <typename T> __device__ __forceinline__ void bst(Buf b, uint32_t off, C2<T> v);
template <> __device__ __forceinline__ void bst<float>(Buf b, uint32_t off, C2<float> v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(vc_u32x2, v), b.r, off, 0, 0);
}
template <> __device__ __forceinline__ void bst<double>(Buf b, uint32_t off, C2<double> v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(vc_u32x4, v), b.r, off, 0, 0);
}
template <typename T> __device__ __forceinline__ T bld1(Buf b, uint32_t off);
template <> __device__ __forceinline__ float bld1<float>(Buf b, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, off, 0, 0));
}
template <> __device__ __forceinline__ double bld1<double>(Buf b, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, off, 0, 0));
}

// LDS accesses of one complex value as one 8- (FP32) or 16-byte (FP64) access: every
// offset here is a multiple of the element size, and the wide access takes a constant
// offset in its immediate field.  (The LDS-tile FFT of the z passes keeps pairs of
// 4-byte accesses, which conflict less in its access pattern.)
template <typename T> struct LdsVec;
template <> struct LdsVec<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct LdsVec<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <typename T>
__device__ __forceinline__ C2<T> lds_ld(const char* __restrict__ lds, uint32_t off) {
  const typename LdsVec<T>::type v = *reinterpret_cast<const typename LdsVec<T>::type*>(lds + off);
  return C2<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void lds_st(char* __restrict__ lds, uint32_t off, C2<T> v) {
  typename LdsVec<T>::type w;
  w.x = v.x;
  w.y = v.y;
  *reinterpret_cast<typename LdsVec<T>::type*>(lds + off) = w;
}

// component-wise select (a select of whole structs by a runtime flag can be lowered to
// a small table in scratch memory)
template <typename T>
__device__ __forceinline__ C2<T> csel(bool f, C2<T> a, C2<T> b) {
  return C2<T>{f ? a.x : b.x, f ? a.y : b.y};
}

// flip the sign of v when bit 31 of s is set (s is 0 or 0x80000000)
__device__ __forceinline__ float flip(float v, uint32_t s) { return __uint_as_float(__float_as_uint(v) ^ s); }
__device__ __forceinline__ double flip(double v, uint32_t s) {
  const uint64_t u = (uint64_t)__double_as_longlong(v) ^ ((uint64_t)s << 32);
  return __longlong_as_double((long long)u);
}

// one complex twiddle at byte offset off: from the LDS copy of the table, or (TWG) from
// the table in global memory (the Tucker-fused pass, whose LDS holds the tile's spectra)
template <typename T, bool TWG>
__device__ __forceinline__ C2<T> tw_ld(const char* __restrict__ twb, uint32_t off) {
  if constexpr (TWG) return ldo<C2<T>>(reinterpret_cast<const C2<T>*>(twb), off);
  else return lds_ld<T>(twb, off);
}

// v[q] *= w^(q ts), w = exp(-+2 pi i / L) from the table; tsb = ts * sizeof(C2).
// All R-1 table reads are issued before the first multiply, so they are in flight
// together instead of one round trip per factor.
template <typename T, int R, bool TWG = false>
__device__ __forceinline__ void tw_mul(C2<T>* v, const char* __restrict__ twb, uint32_t tsb, T sg) {
  C2<T> w[R];
  uint32_t o = 0;
#pragma unroll
  for (int q = 1; q < R; ++q) {
    o += tsb;
    w[q] = tw_ld<T, TWG>(twb, o);
  }
#pragma unroll
  for (int q = 1; q < R; ++q) {
    w[q].y *= -sg;
    v[q] = cmul(v[q], w[q]);
  }
}

// 1/p for the butterfly split i = ip p + k of a middle stage (p <= 512, i < 512): the
// hardware reciprocal (1 ulp) keeps fdiv exact there, (i + 1/2)/p being at least
// 1/(2p) >= 1/1024 from an integer while the product errs by < 512 * 2^-22 / p
__device__ __forceinline__ float stage_inv(int p) { return __builtin_amdgcn_rcpf((float)p); }

// first-stage inputs of butterfly i: rows i + q L/R of one component from HBM into
// registers; bit q of vmask says row i + q L/R is stored (else it reads as zero)
template <typename T, int R>
__device__ __forceinline__ void sw_load(C2<T>* __restrict__ pre, Buf src, uint32_t gbase, uint32_t gstride,
                                        uint32_t vmask, bool act) {
  if (!act) return;
  uint32_t o = gbase;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    pre[q] = bld<T>(src, (vmask & (1u << q)) ? o : kOob);
    o += gstride;
  }
}

// forward stage 0 (p = 1) on the staged inputs, outputs y[i R + q] to LDS; the loads
// of the next component (if any) go into the staging registers first, so they are in
// flight during this component's transform
template <typename T, int R>
__device__ __forceinline__ void sw_first(C2<T>* __restrict__ pre, bool next, Buf nsrc,
                                         uint32_t gbase, uint32_t gstride, uint32_t nmask, bool act,
                                         char* __restrict__ lds, uint32_t wbase, uint32_t ncolpE) {
  if (!act) return;
  C2<T> v[R];
#pragma unroll
  for (int q = 0; q < R; ++q) v[q] = pre[q];
  if (next) sw_load<T, R>(pre, nsrc, gbase, gstride, nmask, true);
  Dft<T, R>::run(v, T(-1));
  uint32_t o = wbase;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    lds_st<T>(lds, o, v[Dft<T, R>::pos(q)]);
    o += ncolpE;
  }
}

// a middle Stockham stage in place in LDS (reads, barrier, writes, barrier); rbase is
// the thread's row-i byte offset (i * ncolpE + c * E)
template <typename T, int R, bool TWG = false>
__device__ __forceinline__ void sw_mid(char* __restrict__ lds, const char* __restrict__ twb, int L, int p, float invp,
                                       int i, uint32_t rbase, uint32_t cE, uint32_t ncolpE, T sg) {
  asm volatile("" : "+v"(i), "+v"(rbase));   // keep this stage's address arithmetic here (no hoisting)
  const int LR = L / R;
  const bool act = i < LR;
  C2<T> v[R];
  uint32_t wb = 0;
  if (act) {
    const uint32_t rstride = (uint32_t)LR * ncolpE;
    uint32_t o = rbase;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      v[q] = lds_ld<T>(lds, o);
      o += rstride;
    }
    const int ip = fdiv(i, invp), k = i - ip * p;
    tw_mul<T, R, TWG>(v, twb, (uint32_t)(k * (LR / p)) * (uint32_t)sizeof(C2<T>), sg);
    Dft<T, R>::run(v, sg);
    wb = (uint32_t)(ip * p * R + k) * ncolpE + cE;
  }
  __syncthreads();
  if (act) {
    const uint32_t wstride = (uint32_t)p * ncolpE;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      lds_st<T>(lds, wb, v[Dft<T, R>::pos(q)]);
      wb += wstride;
    }
  }
  __syncthreads();
}

// inverse last stage (radix R = f0, p = L/R): LDS -> butterfly -> HBM rows i + q L/R
template <typename T, int R, bool TWG = false>
__device__ __forceinline__ void sw_last_inv(const char* __restrict__ lds, const char* __restrict__ twb, int L, int i,
                                            uint32_t rbase, uint32_t ncolpE, Buf dst, uint32_t gbase,
                                            uint32_t gstride, uint32_t vmask, bool act) {
  asm volatile("" : "+v"(i), "+v"(rbase));
  if (!act) return;
  const uint32_t rstride = (uint32_t)(L / R) * ncolpE;
  C2<T> v[R];
  uint32_t o = rbase;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    v[q] = lds_ld<T>(lds, o);
    o += rstride;
  }
  tw_mul<T, R, TWG>(v, twb, (uint32_t)i * (uint32_t)sizeof(C2<T>), T(1));
  Dft<T, R>::run(v, T(1));
  o = gbase;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    bst<T>(dst, (vmask & (1u << q)) ? o : kOob, v[Dft<T, R>::pos(q)]);
    o += gstride;
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
#define VC_SW_CASE(RR, CALL, HI)                     \
  case RR:                                           \
    if constexpr (RR >= RS && RR <= HI) { CALL(RR) } \
    break;

__device__ __forceinline__ int srad(const SandArgs& a, int s) { return (int)((a.radpack >> (5 * s)) & 31u); }

// pair index of the stored spectrum multiplying input b into output o
//   forward (NIN = 3): o < 3 -> P(o,b); o >= 3 -> E(o-3,b)
//   transposed (NIN = 6): b < 3 -> P(b,o); b >= 3 -> E(b-3,o)
template <int NIN>
__device__ __forceinline__ int sw_pair(int o, int b) {
  if (NIN == 3) {
    const int al = o < 3 ? o : o - 3;
    return o < 3 ? (al == b ? al : 2 + al + b) : 6 + 3 * al + b;
  }
  const int al = b < 3 ? b : b - 3;
  return b < 3 ? (al == o ? al : 2 + al + o) : 6 + 3 * al + o;
}

// The fused form's tile spectra (eq. 13, the x-mode product): for every stored pair q
// and tile column cc, X[q][kx'][cc] = sum_r U1_q[kx'][r] T2_q[ky'][kz][r] into LDS
// (xt: [npairs][Hx][ncol]).  Column cc of tile `tile` is (ky, kz) of the flattened
// column index, and ky' = min(ky, My - ky) its folded row.  The caller synchronizes
// before reading xt.
//
// FP32 on the matrix cores: V_MFMA_F32_4X4X1_16B (16 blocks of 4 x 4 x 1 per wave).
// One wave takes one unit (pair, group of 64 kx' rows, group of 4 columns): lane l
// feeds row 64g + l of U1 as A and column 4cg + (l & 3) of T2 as B, so block b = l / 4
// forms rows 64g + 4b .. 64g + 4b + 3 of those four columns, accumulating over r (one
// r per instruction).  Lane 4b + j then holds D_b[i][j] in accumulator element i.  A
// pass covers 16 values of r: A from U1 transposed ([r][kx'], rows of hxp = Hx rounded
// up to 64, r1q = r1 rounded up to 16 rows, zero filled), so each of its 16 loads reads
// 256 contiguous bytes; B from T2 ([ky'][kz][r], rows r1p = r1 rounded up to 4, zero
// past r1) as 16-byte vectors, four columns per wave.  The next pass's operands are
// loaded while the current one runs.
// A pair's table entry with every field in scalar registers (readfirstlane): the
// buffer views built from it are then uniform, so each buffer load is one instruction
// rather than a loop over the distinct descriptors of the wave.
__device__ __forceinline__ const void* uniform_ptr(const void* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return reinterpret_cast<const void*>(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ TkPairDev tk_entry(const TkPairDev* __restrict__ tab, int q) {
  TkPairDev t = tab[q];
  t.U1 = uniform_ptr(t.U1);
  t.T2 = uniform_ptr(t.T2);
  t.U1t = uniform_ptr(t.U1t);
  t.r1 = __builtin_amdgcn_readfirstlane(t.r1);
  t.r1p = __builtin_amdgcn_readfirstlane(t.r1p);
  t.r1q = __builtin_amdgcn_readfirstlane(t.r1q);
  t.hxp = __builtin_amdgcn_readfirstlane(t.hxp);
  return t;
}

// FP32 tile spectra when every pair's r1 <= 32 (the usual ranks): the matrix-core
// product of tk_tile_spectra with few operand loads and little scalar work per unit.
// A unit is (pair q, column group cg, row group g), ordered with g fastest; each wave
// takes a contiguous range of units, so consecutive units share (q, cg) and the B
// operand (the tile's T2 columns, r < 32, eight 16-byte vectors per lane) is loaded once
// per (q, cg).  A unit's A operand is rows 0..31 of U1 transposed at its 64 kx' (32
// dword loads of 256 contiguous bytes; rows past r1q read zero), all loaded one unit
// ahead into the other of two buffers, unconditionally (the last repeats a valid unit),
// so the wait before a unit covers that unit's loads only.  The unit counters advance by
// increments (no divisions per unit), and the 8-rank chunks past r1 are skipped.
__device__ __forceinline__ void tk_tile_spectra_r32(float* __restrict__ xt, const SandArgs& a, int tile, int ncol,
                                                    int lane, int wave, int nwave, int ngr, int ncg, int units,
                                                    int Hy) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const int ncols = a.My * a.H;
  const int u_beg = (int)((int64_t)units * wave / nwave), u_end = (int)((int64_t)units * (wave + 1) / nwave);
  if (u_beg >= u_end) return;
  f32x4 bv[8];
  auto loadB = [&](const TkPairDev& tp, int cg) {
    const int colb = cg * 4 + (lane & 3);
    const int colq = tile * ncol + colb;
    const bool bok = colb < ncol && colq < ncols;
    const int jq = bok ? colq / a.H : 0, kzq = bok ? colq - jq * a.H : 0;
    // descriptors from scalar registers at the point of use (a loop-carried entry may
    // otherwise be kept in vector registers, which turns each load into a loop)
    const int r1p = __builtin_amdgcn_readfirstlane(tp.r1p);
    const Buf tb = make_buf(uniform_ptr(tp.T2), (uint32_t)__builtin_amdgcn_readfirstlane(Hy * a.H * r1p * 4));
    const uint32_t to = (uint32_t)(min(jq, a.My - jq) * a.H + kzq) * (uint32_t)r1p * 4u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool in = bok && 4 * k < r1p;
      bv[k] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(tb.r, in ? to + 16u * k : kOob, 0, 0));
    }
  };
  auto loadA = [&](const TkPairDev& tp, int g, float* av) {
    const int hxp = __builtin_amdgcn_readfirstlane(tp.hxp);
    const Buf ub = make_buf(uniform_ptr(tp.U1t), (uint32_t)__builtin_amdgcn_readfirstlane(tp.r1q * hxp * 4));
    const uint32_t ho = (uint32_t)hxp * 4u;
    uint32_t uo = ((uint32_t)__builtin_amdgcn_readfirstlane(g * 64) + (uint32_t)lane) * 4u;
    // rows of the 8-rank chunks the pair's r1 reaches (the others are never used)
    const int nch = __builtin_amdgcn_readfirstlane((tp.r1 + 7) >> 3);
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      if (cc == 0 || cc < nch) {
#pragma unroll
        for (int k = 8 * cc; k < 8 * cc + 8; ++k) {
          av[k] = bld1<float>(ub, uo);
          uo += ho;
        }
      }
    }
  };
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  int q = u_beg / (ngr * ncg);
  int cg = (u_beg - q * ngr * ncg) / ngr;
  int g = u_beg - q * ngr * ncg - cg * ngr;
  int u = u_beg;
  TkPairDev tp = tk_entry(a.tk, q);
  loadB(tp, cg);
  float A0[32], A1[32];
  loadA(tp, g, A0);
  // one unit from `cur`, the next one's A loads issued into `nx` first
  auto unit = [&](const float* cur, float* nx) -> bool {
    int q1 = q, cg1 = cg, g1 = g + 1;
    if (g1 == ngr) {
      g1 = 0;
      if (++cg1 == ncg) { cg1 = 0; ++q1; }
    }
    const bool more = u + 1 < u_end;
    const bool newq = more && q1 != q;
    const TkPairDev tn = newq ? tk_entry(a.tk, q1) : tp;
    loadA(tn, more ? g1 : g, nx);
    const int nch = __builtin_amdgcn_readfirstlane((tp.r1 + 7) >> 3);
    acc = f32x4{0.f, 0.f, 0.f, 0.f};
#define VC_TK_CHUNK(CC)                                                                                     \
  _Pragma("unroll") for (int e = 0; e < 4; ++e) acc =                                                       \
      __builtin_amdgcn_mfma_f32_4x4x1f32(cur[8 * (CC) + e], bv[2 * (CC)][e], acc, 0, 0, 0);                 \
  _Pragma("unroll") for (int e = 0; e < 4; ++e) acc =                                                       \
      __builtin_amdgcn_mfma_f32_4x4x1f32(cur[8 * (CC) + 4 + e], bv[2 * (CC) + 1][e], acc, 0, 0, 0);
    VC_TK_CHUNK(0)
    if (nch > 1) { VC_TK_CHUNK(1) }
    if (nch > 2) { VC_TK_CHUNK(2) }
    if (nch > 3) { VC_TK_CHUNK(3) }
#undef VC_TK_CHUNK
    const int b = lane >> 2, col = cg * 4 + (lane & 3);
    if (col < ncol) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rw = g * 64 + 4 * b + i;
        if (rw < a.Hx) xt[((int64_t)q * a.Hx + rw) * ncol + col] = acc[i];
      }
    }
    if (!more) return false;
    if (newq || cg1 != cg) loadB(tn, cg1);   // a new pair or column group
    q = q1;
    cg = cg1;
    g = g1;
    tp = tn;
    ++u;
    return true;
  };
  for (;;) {
    if (!unit(A0, A1)) break;
    if (!unit(A1, A0)) break;
  }
}

template <typename T>
__device__ __forceinline__ void tk_tile_spectra(T* __restrict__ xt, const SandArgs& a, int tile, int ncol) {
  const int ncols = a.My * a.H;
  if constexpr (sizeof(T) == 4) {
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    // the wave index is uniform: the unit indices below live in scalar registers and a
    // pair's table entry comes through the scalar cache
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwave = blockDim.x >> 6;
    const int ngr = (a.Hx + 63) >> 6, ncg = (ncol + 3) >> 2;
    const int units = a.npairs * ngr * ncg;
    const int Hy = a.My / 2 + 1;
    if (a.tk_r1max <= 32) {
      tk_tile_spectra_r32(xt, a, tile, ncol, lane, wave, nwave, ngr, ncg, units, Hy);
      return;
    }
    struct Ops {
      float av[16];
      f32x4 bv[4];
      int r1q;
    };
    // operands of the pass (unit u, r in [r0, r0 + 16)) through buffer views, zero past
    // r1 or outside the tile (T2 offsets past the row or for absent columns are sent out
    // of range; U1t is zero filled)
    auto load = [&](int u, int r0, Ops& o) {
      const int q = u / (ngr * ncg);
      const int rem = u - q * ngr * ncg;
      const int g = rem / ncg, cg = rem - g * ncg;
      const TkPairDev tp = tk_entry(a.tk, q);
      const int hxp = __builtin_amdgcn_readfirstlane(tp.hxp);
      const Buf ub = make_buf(uniform_ptr(tp.U1t), (uint32_t)__builtin_amdgcn_readfirstlane(tp.r1q * hxp * 4));
      const uint32_t ho = (uint32_t)hxp * 4u;
      uint32_t uo = ((uint32_t)__builtin_amdgcn_readfirstlane(r0 * hxp + g * 64) + (uint32_t)lane) * 4u;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        o.av[k] = bld1<float>(ub, uo);
        uo += ho;
      }
      const int colb = cg * 4 + (lane & 3);
      const int colq = tile * ncol + colb;
      const bool bok = colb < ncol && colq < ncols;
      const int jq = bok ? colq / a.H : 0, kzq = bok ? colq - jq * a.H : 0;
      const int r1p = __builtin_amdgcn_readfirstlane(tp.r1p);
      const Buf tb = make_buf(uniform_ptr(tp.T2), (uint32_t)__builtin_amdgcn_readfirstlane(Hy * a.H * r1p * 4));
      const uint32_t to = ((uint32_t)(min(jq, a.My - jq) * a.H + kzq) * (uint32_t)r1p + (uint32_t)r0) * 4u;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool in = bok && r0 + 4 * k < tp.r1p;
        o.bv[k] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(tb.r, in ? to + 16u * k : kOob, 0, 0));
      }
      o.r1q = tp.r1q;
    };
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    // one pass: 16 rank-one updates; the unit's block goes to LDS after its last pass
    auto run = [&](const Ops& o, int u, int r0, bool last) {
      if (r0 == 0) acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(o.av[4 * k + e], o.bv[k][e], acc, 0, 0, 0);
      }
      if (last) {
        const int q = u / (ngr * ncg);
        const int rem = u - q * ngr * ncg;
        const int g = rem / ncg, cg = rem - g * ncg;
        const int b = lane >> 2, col = cg * 4 + (lane & 3);
        if (col < ncol) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int rw = g * 64 + 4 * b + i;
            if (rw < a.Hx) xt[((int64_t)q * a.Hx + rw) * ncol + col] = acc[i];
          }
        }
      }
    };
    // passes of this wave: units wave, wave + nwave, ..., each r0 = 0, 16, ... < r1q.
    // Two operand sets in turn: the loads of the next pass are in flight while the
    // current pass runs; they are issued unconditionally (the last repeats a valid
    // pass) so the wait before each pass covers only that pass's loads.
    if (wave < units) {
      Ops A, B;
      int u = wave, r0 = 0;
      load(u, r0, A);
      for (;;) {
        int u1 = u, r1 = r0 + 16;
        if (r1 >= A.r1q) { u1 = u + nwave; r1 = 0; }
        const bool more1 = u1 < units;
        load(more1 ? u1 : u, more1 ? r1 : r0, B);
        run(A, u, r0, r1 == 0);
        if (!more1) break;
        u = u1;
        r0 = r1;
        int u2 = u, r2 = r0 + 16;
        if (r2 >= B.r1q) { u2 = u + nwave; r2 = 0; }
        const bool more2 = u2 < units;
        load(more2 ? u2 : u, more2 ? r2 : r0, A);
        run(B, u, r0, r2 == 0);
        if (!more2) break;
        u = u2;
        r0 = r2;
      }
    }
  } else {
    // FP64 (the refinement's residual products) on the vector units, 16-byte loads
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    const int per = a.Hx * ncol;
    for (int e = threadIdx.x; e < a.npairs * per; e += blockDim.x) {
      const int qp = e / per;
      const int rem = e - qp * per;
      const int kxq = rem / ncol, cc = rem - kxq * ncol;
      const int colq = tile * ncol + cc;
      T acc = T(0);
      if (colq < ncols) {
        const int jq = colq / a.H, kzq = colq - jq * a.H;
        const TkPairDev tp = a.tk[qp];
        const f64x2* __restrict__ u = reinterpret_cast<const f64x2*>(static_cast<const T*>(tp.U1) + (int64_t)kxq * tp.r1p);
        const f64x2* __restrict__ t2 = reinterpret_cast<const f64x2*>(
            static_cast<const T*>(tp.T2) + ((int64_t)min(jq, a.My - jq) * a.H + kzq) * tp.r1p);
        for (int v = 0; v < (tp.r1p >> 1); ++v) {
          const f64x2 x = u[v], y = t2[v];
          acc += x.x * y.x + x.y * y.y;
        }
      }
      xt[e] = acc;
    }
  }
}

// The staged form's tile spectra: the stored octants of the npairs pairs at the tile's
// columns copied into LDS (xt: [npairs][Hx][ncol], the fused form's layout), so every
// right-hand side reads them from LDS and HBM delivers them once per tile.  Thread t
// copies column t % ncol of the rows t / ncol, t / ncol + T, ... (T = threads / ncol)
// over (pair, kx'), eight loads in flight before their stores; columns outside the grid
// hold zero.  The caller synchronizes before reading xt.
template <typename T>
__device__ __forceinline__ void tk_stage_spectra(T* __restrict__ xt, const SandArgs& a, const T* __restrict__ R,
                                                 int tile, int ncol) {
  const int ncols = a.My * a.H;
  const int rstep = (int)blockDim.x / ncol;
  const int r0 = (int)threadIdx.x / ncol, c = (int)threadIdx.x - r0 * ncol;
  if (r0 >= rstep) return;
  const int col = tile * ncol + c;
  const bool cok = col < ncols;
  const int colc = cok ? col : 0;
  const int ky = colc / a.H, kz = colc - ky * a.H;
  const int kyp = min(ky, a.My - ky);
  const Buf rb = make_buf(R, (uint32_t)((uint64_t)a.npairs * (uint64_t)a.pair_stride * sizeof(T)));
  const uint32_t cofs = (uint32_t)(kyp * a.H + kz) * (uint32_t)sizeof(T);
  const uint32_t rowb = (uint32_t)(a.Hy * a.H) * (uint32_t)sizeof(T);        // bytes per kx' row
  const uint32_t pairb = (uint32_t)a.pair_stride * (uint32_t)sizeof(T);
  const int rows = a.npairs * a.Hx;
  int row = r0, q = r0 / a.Hx, kxp = r0 - (r0 / a.Hx) * a.Hx;
  while (row < rows) {
    T v[8];
    int dst[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = row < rows;
      v[u] = bld1<T>(rb, (in && cok) ? (uint32_t)q * pairb + (uint32_t)kxp * rowb + cofs : kOob);
      dst[u] = in ? (q * a.Hx + kxp) * ncol + c : -1;
      row += rstep;
      kxp += rstep;
      while (kxp >= a.Hx) {
        kxp -= a.Hx;
        ++q;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (dst[u] >= 0) xt[dst[u]] = v[u];
  }
}

// one column tile of the pass for right-hand sides rhs0 .. rhs0 + nrhs_loop - 1; PID > 0
// takes the plan from kSandFixed[PID] as compile-time constants (the launcher checks
// that it is a.radpack's).
// TK: the Tucker-fused form (eq. 13).  No stored spectra: the workgroup first builds its
// tile's spectra X[pair][kx'][column] = sum_r U1[kx'][r] T2[r][ky'][kz] of every pair
// into LDS (the x-mode product, from the factor U1 and the strip T2 = S x2 U2 x3 U3),
// then runs every right-hand side against them; the twiddles and x phases are read from
// their tables in global memory (the LDS holds the spectra instead).
// NC > 0: the tile width as a compile-time constant (must equal a.ncol), so the LDS and
// HBM strides derived from it fold into the instructions.
template <typename T, int NIN, int NOUT, int RS, int PID = 0, int TK = 0, int NC = 0>
__device__ __forceinline__ void sandwich_body(const C2<T>* __restrict__ Fin, C2<T>* __restrict__ Fout,
                                              const T* __restrict__ R, const SandArgs& a,
                                              const C2<T>* __restrict__ twg, const C2<T>* __restrict__ phx,
                                              const uint8_t* __restrict__ pflag, int tile, int rhs0,
                                              int nrhs_loop) {
  constexpr int RMAX = sandwich_rmax((int)sizeof(T)), RMID = sandwich_rmid((int)sizeof(T));
  constexpr uint32_t E = sizeof(C2<T>);
  extern __shared__ char smem_raw[];
  constexpr bool FX = PID > 0;
  constexpr bool FU = TK != 0;
  constexpr SandFixedPlan PD = kSandFixed[PID];
  const int L = FX ? PD.L : a.Mx, tl = FX ? PD.L / RS : a.tl, S = FX ? PD.nst : a.nst;
  auto rad = [&](int s) -> int { return FX ? PD.r[s] : srad(a, s); };
  int ncol = NC > 0 ? NC : a.ncol;
  uint32_t ncolpE = (uint32_t)ncol * E;   // unpadded rows: measured faster than a pitch of ncol + 1 or + 2
  // FP32 keeps the x half-voxel phases in LDS beside the twiddles; FP64 (whose tiles are
  // twice as large, and whose registers are full) reads them from the cached table
  constexpr bool PH_LDS = sizeof(T) == 4 && !FU;
  // fused: [npairs][Hx][ncol] spectra of the tile (16-byte aligned), then the tile
  const uint32_t pairXb = FU ? (uint32_t)(a.Hx * ncol) * (uint32_t)sizeof(T) : 0u;
  const uint32_t xtb = FU ? ((uint32_t)a.npairs * pairXb + 15u) & ~15u : 0u;
  const char* twb = FU ? reinterpret_cast<const char*>(twg) : smem_raw;   // L twiddles
  char* phb = smem_raw + (size_t)L * E;                    // L x phases (FP32)
  char* lds = FU ? smem_raw + xtb : smem_raw + (size_t)(PH_LDS ? 2 : 1) * L * E; // [L][ncol] tile
  uint8_t* sflag = reinterpret_cast<uint8_t*>(lds + (size_t)L * ncolpE);   // plane flags of the 3 axes
  const int tid = threadIdx.x;
  const int ncols = a.My * a.H;                 // flattened (ky, kz) columns
  const uint32_t rowb = (uint32_t)ncols * E;   // bytes between x rows
  const uint32_t slab = (uint32_t)a.n1x * rowb;  // bytes of one (component, rhs) slab
  const uint32_t pairb = (uint32_t)a.pair_stride * (uint32_t)sizeof(T);
  const int r0 = rad(0);
  const int LR0 = L / r0;
  if (!FU) {
    for (int t = tid; t < L; t += blockDim.x) {
      lds_st<T>(smem_raw, (uint32_t)t * E, twg[t]);
      if (PH_LDS) lds_st<T>(phb, (uint32_t)t * E, phx[t]);
    }
  }
  for (int t = tid; t < 3 * a.n1x; t += blockDim.x) sflag[t] = pflag[t];
  if (FU) {
    if (a.tk) tk_tile_spectra<T>(reinterpret_cast<T*>(smem_raw), a, tile, ncol);
    else tk_stage_spectra<T>(reinterpret_cast<T*>(smem_raw), a, R, tile, ncol);
  }
  __syncthreads();

  // right-hand sides of this workgroup (one, except in the fused form)
  const int nloop = FU ? nrhs_loop : 1;
#pragma unroll 1
  for (int kr = 0; kr < nloop; ++kr) {
    const int rhs = rhs0 + kr;
    int tidv = tid;
    if (FU) {
      if (a.act && !a.act[rhs]) continue;   // uniform over the workgroup
      __syncthreads();                      // the previous right-hand side is done with the tile
      // the thread's geometry below is derived again for each right-hand side rather
      // than held in registers across the loop (the transforms need those registers)
      asm volatile("" : "+v"(tidv));
    }
    // the tile width too, so the per-stage strides derived from it are not all computed
    // once before the loop and held in scalar registers across it
    if (FU && NC == 0) asm volatile("" : "+s"(ncol), "+s"(ncolpE));
    const int i = NC > 0 ? tidv / NC : fdiv(tidv, 1.0f / (float)ncol);
    const int c = tidv - i * ncol;   // column fastest
    const bool valid = i < tl;
    const int col = tile * ncol + c;
    const bool colok = col < ncols;
    const int colc = colok ? col : ncols - 1;
    // tiles of consecutive flattened columns: each tile's rows are 32-byte aligned
    // chunks of the planes, and the tiles sharing a cache line run side by side
    const int ky = fdiv(colc, 1.0f / (float)a.H), kz = colc - ky * a.H;
    const int mcol = colc;   // the column's position in the work array
    const int yflip = ky > a.My / 2;
    const int kyp = yflip ? a.My - ky : ky;
    const bool act0 = i < LR0;                   // owns a butterfly of the first / last stage
    // half-voxel phase along x of the thread's frequency kx = i + m tl
    auto phase_x = [&](int m) -> C2<T> { return PH_LDS ? lds_ld<T>(phb, (uint32_t)(i + m * tl) * E) : phx[i + m * tl]; };

    // per-thread geometry: LDS bases, HBM bases and strides of the first / last stage
    const uint32_t cE = (uint32_t)c * E;
    const uint32_t rbase = (uint32_t)i * ncolpE + cE;                // row i of the tile
    const uint32_t gbase = (uint32_t)mcol * E + (uint32_t)i * rowb;    // HBM row i of the column
    const uint32_t gstride = (uint32_t)LR0 * rowb;                   // HBM rows i + q L/f0
    // rows i + q L/f0 (q < f0) that are stored, per axis: bits 0..15 planes with conductor
    // panels, bits 16..31 planes with dielectric panels
    uint32_t rm0 = 0u, rm1 = 0u, rm2 = 0u;
    if (act0 && colok) {
      for (int qq = 0; qq < r0; ++qq) {
        const int r = i + qq * LR0;
        if (r >= a.n1x) break;
        const uint32_t f0 = sflag[r], f1 = sflag[a.n1x + r], f2 = sflag[2 * a.n1x + r];
        rm0 |= ((f0 & 1u) << qq) | (((f0 >> 1) & 1u) << (16 + qq));
        rm1 |= ((f1 & 1u) << qq) | (((f1 >> 1) & 1u) << (16 + qq));
        rm2 |= ((f2 & 1u) << qq) | (((f2 >> 1) & 1u) << (16 + qq));
      }
    }
    auto vm = [&](int ax, int msk) -> uint32_t {
      const uint32_t m = ax == 0 ? rm0 : (ax == 1 ? rm1 : rm2);
      return ((msk & 1) ? (m & 0xffffu) : 0u) | ((msk & 2) ? (m >> 16) : 0u);
    };

    C2<T> q[NIN][RS];
    C2<T> pre[RMAX];   // staged first-stage inputs of the component about to be transformed
    if (S > 1) {
#define VC_CALL(RR) sw_load<T, RR>(pre, make_buf(Fin + rhs * a.rhs_stride, slab), gbase, gstride, vm(0, NIN == 3 ? 3 : 1), act0);
      VC_SW_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
    }
#pragma unroll
    for (int b = 0; b < NIN; ++b) {
      const int fax = b % 3;
      const int fmsk = NIN == 3 ? 3 : (b < 3 ? 1 : 2);
      const Buf src = make_buf(Fin + b * a.comp_stride + rhs * a.rhs_stride, slab);
      C2<T> v[RS];
      if (S == 1) {
        if (valid) {
          const uint32_t msk = vm(fax, fmsk);
          uint32_t o = gbase;
#pragma unroll
          for (int m = 0; m < RS; ++m) {
            v[m] = bld<T>(src, (msk & (1u << m)) ? o : kOob);
            o += rowb;
          }
          Dft<T, RS>::run(v, T(-1));
        }
      } else {
        if (b > 0) __syncthreads();   // readers of the previous component are done with the tile
        const int bn = b + 1;
        const bool next = bn < NIN;
        const Buf nsrc = make_buf(Fin + bn * a.comp_stride + rhs * a.rhs_stride, slab);
        const uint32_t nmask = vm(bn % 3, NIN == 3 ? 3 : (bn < 3 ? 1 : 2));
        {
          uint32_t wbase = (uint32_t)i * (uint32_t)r0 * ncolpE + cE;
          asm volatile("" : "+v"(wbase));
#define VC_CALL(RR) sw_first<T, RR>(pre, next, nsrc, gbase, gstride, nmask, act0, lds, wbase, ncolpE);
          VC_SW_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
        }
        __syncthreads();
        int p = r0;
#pragma unroll
        for (int s = 1; s < (FX ? PD.nst : S) - 1; ++s) {
          const int rs = rad(s);
          const float invp = stage_inv(p);
#define VC_CALL(RR) sw_mid<T, RR, FU>(lds, twb, L, p, invp, i, rbase, cE, ncolpE, T(-1));
          VC_SW_SWITCH(rs, VC_CALL, RMID)
#undef VC_CALL
          p *= rs;
        }
        if (valid) {
          // last forward stage (radix RS, p = tl): butterfly i reads rows i + q tl,
          // twiddle exponent q i, outputs X[i + q tl]
          const uint32_t st = (uint32_t)tl * ncolpE;
          uint32_t o = rbase;
#pragma unroll
          for (int m = 0; m < RS; ++m) {
            v[m] = lds_ld<T>(lds, o);
            o += st;
          }
          tw_mul<T, RS, FU>(v, twb, (uint32_t)i * E, T(-1));
          Dft<T, RS>::run(v, T(-1));
        }
      }
      // half-voxel phase of the input component (shift to the common lattice); slot
      // pos(m) holds X[i + m tl]
      if (valid) {
        C2<T> w[RS];
#pragma unroll
        for (int m = 0; m < RS; ++m)
          w[m] = fax == 0 ? cmul(v[Dft<T, RS>::pos(m)], phase_x(m)) : v[Dft<T, RS>::pos(m)];
        // per-element selects keep q in registers (a switch of stores is merged into one
        // dynamically indexed store, which moves q to scratch memory)
#pragma unroll
        for (int bb = 0; bb < NIN; ++bb)
#pragma unroll
          for (int m = 0; m < RS; ++m)
            if (bb == b) q[bb][m] = w[m];
      }
    }

    // spectra offsets and fold signs of the thread's frequencies kx = i + m tl
    uint32_t roff[RS], xs[RS];
    const uint32_t ys = yflip ? 0x80000000u : 0u;
#pragma unroll
    for (int m = 0; m < RS; ++m) {
      const int kx = i + m * tl;
      const bool xf = kx > a.Mx / 2;
      const int kxp = xf ? a.Mx - kx : kx;
      roff[m] = !valid ? 0u
                : FU ? (uint32_t)(kxp * ncol + c) * (uint32_t)sizeof(T)
                     : (uint32_t)((kxp * a.Hy + kyp) * a.H + kz) * (uint32_t)sizeof(T);
      xs[m] = xf ? 0x80000000u : 0u;
    }
    // spectra of the block multiply, loaded one output component ahead
    constexpr int NQ = NIN == 3 ? 3 : 6;
    T rv[NQ][RS];
    auto load_spectra = [&](int o) {
#pragma unroll
      for (int b = 0; b < NQ; ++b) {
        const int qi = sw_pair<NIN>(o, b);
        const unsigned odd = (unsigned)(a.oddmask >> (3 * qi)) & 7u;
        if constexpr (FU) {
          const char* xb = smem_raw + (uint32_t)qi * pairXb;
#pragma unroll
          for (int m = 0; m < RS; ++m) {
            const uint32_t sg = ((odd & 1u) ? xs[m] : 0u) ^ ((odd & 2u) ? ys : 0u);
            rv[b][m] = flip(*reinterpret_cast<const T*>(xb + roff[m]), sg);
          }
        } else {
          const Buf base = make_buf(R + (int64_t)qi * a.pair_stride, pairb);
#pragma unroll
          for (int m = 0; m < RS; ++m) {
            const uint32_t sg = ((odd & 1u) ? xs[m] : 0u) ^ ((odd & 2u) ? ys : 0u);
            rv[b][m] = flip(bld1<T>(base, roff[m]), sg);
          }
        }
      }
    };
    // stored spectra come from HBM and are loaded one output component ahead; the fused
    // form's come from LDS and are loaded just before their use (no registers held
    // through the inverse transforms)
    if (valid && !FU) load_spectra(0);
#pragma unroll 1
    for (int o = 0; o < NOUT; ++o) {
      const int oax = NIN == 3 ? (o < 3 ? o : o - 3) : o;
      C2<T> z[RS];
      if (valid) {
        // the fused form's wide kernels load the output's half-voxel phases (x-normal
        // outputs only) from global memory together before the multiply: one memory
        // latency rather than one per frequency (the other kernels have no registers to
        // spare for them, or read them from LDS)
        constexpr bool PHO = FU && NIN == 3 && kSandFixed[PID].wide;
        C2<T> pho[RS];
        if (PHO && oax == 0) {
#pragma unroll
          for (int m = 0; m < RS; ++m) pho[m] = phase_x(m);
        }
        if (FU) load_spectra(o);
#pragma unroll
        for (int m = 0; m < RS; ++m) {
          C2<T> acc = {T(0), T(0)};
          if (NIN == 3) {
            // o < 3: C_alpha = sum_b P(alpha,b) Q'_b ; o >= 3: D_alpha = i sum_b E(alpha,b) Q'_b
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              acc.x += rv[b][m] * q[b][m].x;
              acc.y += rv[b][m] * q[b][m].y;
            }
            if (o >= 3) acc = C2<T>{-acc.y, acc.x};
          } else {
            // transposed product: out_b = sum_al P(al,b) X'C_al - i sum_al E(al,b) X'D_al
            C2<T> accE = {T(0), T(0)};
#pragma unroll
            for (int al = 0; al < 3; ++al) {
              acc.x += rv[al][m] * q[al][m].x;
              acc.y += rv[al][m] * q[al][m].y;
              accE.x += rv[3 + al][m] * q[(NIN > 3 ? 3 : 0) + al][m].x;
              accE.y += rv[3 + al][m] * q[(NIN > 3 ? 3 : 0) + al][m].y;
            }
            acc.x += accE.y;   // -i * accE
            acc.y -= accE.x;
          }
          // output phase: conj of the half-voxel shift of the output component
          z[m] = oax == 0 ? cmul(acc, cconj(PHO ? pho[m] : phase_x(m))) : acc;
        }
        if (!FU && o + 1 < NOUT) load_spectra(o + 1);
      }
      const int msk = NIN == 3 ? (o < 3 ? 1 : 2) : 3;
      const Buf dst = make_buf(Fout + o * a.comp_stride + rhs * a.rhs_stride, slab);
      const uint32_t omask = vm(oax, msk);
      if (S == 1) {
        if (valid) {
          Dft<T, RS>::run(z, T(1));
          uint32_t og = gbase;
#pragma unroll
          for (int m = 0; m < RS; ++m) {
            bst<T>(dst, (omask & (1u << m)) ? og : kOob, z[Dft<T, RS>::pos(m)]);
            og += rowb;
          }
        }
      } else {
        __syncthreads();   // the previous readers of the tile are done
        if (valid) {
          // first inverse stage (radix RS, p = 1) on the held values X[i + q tl]
          Dft<T, RS>::run(z, T(1));
          uint32_t ow = (uint32_t)i * (uint32_t)RS * ncolpE + cE;
#pragma unroll
          for (int m = 0; m < RS; ++m) {
            lds_st<T>(lds, ow, z[Dft<T, RS>::pos(m)]);
            ow += ncolpE;
          }
        }
        __syncthreads();
        int p = RS;
#pragma unroll
        for (int s = (FX ? PD.nst : S) - 2; s >= 1; --s) {
          const int rs = rad(s);
          const float invp = stage_inv(p);
#define VC_CALL(RR) sw_mid<T, RR, FU>(lds, twb, L, p, invp, i, rbase, cE, ncolpE, T(1));
          VC_SW_SWITCH(rs, VC_CALL, RMID)
#undef VC_CALL
          p *= rs;
        }
#define VC_CALL(RR) sw_last_inv<T, RR, FU>(lds, twb, L, i, rbase, ncolpE, dst, gbase, gstride, omask, act0);
        VC_SW_SWITCH(r0, VC_CALL, RMAX)
#undef VC_CALL
      }
    }
  }
}
#undef VC_SW_CASE
#undef VC_SW_SWITCH

// Right-hand sides fastest: the workgroups that read one tile's spectra run together on
// one XCD, so those spectra come from HBM once per tile rather than once per RHS.
template <typename T, int NIN, int NOUT, int RS, int PID = 0>
__global__ void __launch_bounds__(sand_max_threads_fixed(PID, (int)sizeof(T), NIN),
                                  sand_max_threads_fixed(PID, (int)sizeof(T), NIN) == 1024
                                      ? 4
                                      : ((sizeof(T) == 8 || NIN == 6) ? 2 : 3))
k_xsandwich(const C2<T>* __restrict__ Fin, C2<T>* __restrict__ Fout, const T* __restrict__ R, SandArgs a,
            const C2<T>* __restrict__ twg, const C2<T>* __restrict__ phx, const uint8_t* __restrict__ pflag) {
  if (a.skip && *a.skip) return;
  // a fixed-plan kernel never runs a plan other than its own (uniform check)
  if (PID > 0 && (a.Mx != kSandFixed[PID].L || a.nst != kSandFixed[PID].nst || a.radpack != sand_fixed_pack(PID) ||
                  a.tl * RS != a.Mx))
    return;
  const int ntiles = gridDim.x;
  const int work = xcd_remap(blockIdx.y * ntiles + blockIdx.x, ntiles * gridDim.y);
  const int tile = work / a.nrhs, rhs = work - tile * a.nrhs;
  if (a.act && !a.act[rhs]) return;
  sandwich_body<T, NIN, NOUT, RS, PID>(Fin, Fout, R, a, twg, phx, pflag, tile, rhs, 1);
}

// The Tucker-fused form: one workgroup per tile for all right-hand sides (the tile's
// spectra are built once into LDS and shared by them: the factor U1 is read once per
// tile, not once per right-hand side); tiles XCD-contiguous in the column
// order.
template <typename T, int NIN, int NOUT, int RS, int PID = 0, int NC = 0>
__global__ void __launch_bounds__(sand_max_threads_fixed(PID, (int)sizeof(T), NIN),
                                  sand_max_threads_fixed(PID, (int)sizeof(T), NIN) == 1024
                                      ? 4
                                      : ((sizeof(T) == 8 || NIN == 6) ? 2 : 3))
k_xsandwich_tk(const C2<T>* __restrict__ Fin, C2<T>* __restrict__ Fout, const T* __restrict__ R, SandArgs a,
               const C2<T>* __restrict__ twg, const C2<T>* __restrict__ phx, const uint8_t* __restrict__ pflag) {
  if (a.skip && *a.skip) return;
  if (PID > 0 && (a.Mx != kSandFixed[PID].L || a.nst != kSandFixed[PID].nst || a.radpack != sand_fixed_pack(PID) ||
                  a.tl * RS != a.Mx))
    return;
  if (NC > 0 && a.ncol != NC) return;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  sandwich_body<T, NIN, NOUT, RS, PID, 1, NC>(Fin, Fout, R, a, twg, phx, pflag, tile, 0, a.nrhs);
}

// several scenes in one launch: linear workgroup -> (scene, tile, rhs), XCD-contiguous
template <typename T, int NIN, int NOUT, int RS>
__global__ void __launch_bounds__(512, (sizeof(T) == 8 || NIN == 6) ? 2 : 3)
k_xsandwich_multi(const SandScene* __restrict__ tab, int nscene, const int* __restrict__ skip,
                  const int* __restrict__ act) {
  if (skip && *skip) return;
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const SandScene& sc = tab[find_scene(tab, nscene, lin)];
  const int work = lin - sc.blk0;
  const int tile = work / sc.a.nrhs, rhs = work - tile * sc.a.nrhs;
  if (act && !act[sc.c0 + rhs]) return;
  sandwich_body<T, NIN, NOUT, RS>(static_cast<const C2<T>*>(sc.Fin), static_cast<C2<T>*>(sc.Fout),
                                  static_cast<const T*>(sc.R), sc.a, static_cast<const C2<T>*>(sc.tw),
                                  static_cast<const C2<T>*>(sc.phx), sc.pflag, tile, rhs, 1);
}

// Compiled last-stage radices per kernel variant (register budget: the thread holds
// NIN x RS transformed inputs).
template <typename T, int NIN> struct SandRS {
  static constexpr int max = sandwich_rs_max((int)sizeof(T), NIN);
};

// launch with last-stage radix RR: the fixed-plan kernel of the first table entry that
// equals the runtime plan, else the generic one
// e0 / e1: optional events stamped by the launch itself (hipExtLaunchKernelGGL)
template <typename T, int NIN, int NOUT, int RR, int ID, int TK>
hipError_t launch_sandwich_rs(const void* Fin, void* Fout, const void* R, const SandArgs& a, const void* tw,
                              const void* phx, const uint8_t* pflag, int nthr,
                              size_t lds, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int ntiles = (a.My * a.H + a.ncol - 1) / a.ncol;
  dim3 grid = TK ? dim3(ntiles) : dim3(ntiles, a.nrhs);
  auto go = [&](auto kernel) -> hipError_t {
    // above the default 64 KiB of dynamic LDS (the fused form's spectra), declare it
    if (lds > kLdsBudget) {
      const hipError_t ea = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (ea != hipSuccess) return ea;
    }
    if (e0 || e1)
      hipExtLaunchKernelGGL(kernel, grid, dim3(nthr), (std::uint32_t)lds, st, e0, e1, 0u, (const C2<T>*)Fin,
                            (C2<T>*)Fout, (const T*)R, a, (const C2<T>*)tw, (const C2<T>*)phx, pflag);
    else
      hipLaunchKernelGGL(kernel, grid, dim3(nthr), lds, st, (const C2<T>*)Fin, (C2<T>*)Fout, (const T*)R, a,
                         (const C2<T>*)tw, (const C2<T>*)phx, pflag);
    return hipGetLastError();
  };
  if constexpr (ID < kSandNumFixed) {
    if constexpr (sand_fixed_last(ID) == RR) {
      if (a.Mx == kSandFixed[ID].L && a.nst == kSandFixed[ID].nst && a.radpack == sand_fixed_pack(ID) &&
          a.tl * RR == a.Mx) {
        if constexpr (TK) {
          // the FP32 three-input wide kernels also come with the 4-column tile compiled in
          if constexpr (sizeof(T) == 4 && NIN == 3 && kSandFixed[ID].wide)
            if (a.ncol == 4) return go(k_xsandwich_tk<T, NIN, NOUT, RR, ID, 4>);
          return go(k_xsandwich_tk<T, NIN, NOUT, RR, ID>);
        }
        else return go(k_xsandwich<T, NIN, NOUT, RR, ID>);
      }
    }
    return launch_sandwich_rs<T, NIN, NOUT, RR, ID + 1, TK>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, st,
                                                            e0, e1);
  } else {
    if constexpr (TK) return go(k_xsandwich_tk<T, NIN, NOUT, RR, 0>);
    else return go(k_xsandwich<T, NIN, NOUT, RR, 0>);
  }
}

template <typename T, int NIN, int NOUT, int TK>
hipError_t launch_sandwich_v(const void* Fin, void* Fout, const void* R, const SandArgs& a, const void* tw,
                             const void* phx, const uint8_t* pflag, int nthr,
                             size_t lds, int rs, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
#define VC_RS(RR)                                                                                                 \
  case RR:                                                                                                        \
    if constexpr (RR <= SandRS<T, NIN>::max) {                                                                    \
      return launch_sandwich_rs<T, NIN, NOUT, RR, 1, TK>(Fin, Fout, R, a, tw, phx, pflag, nthr, lds, st, \
                                                         e0, e1);                                                 \
    }                                                                                                             \
    break;
  switch (rs) {
    VC_RS(2) VC_RS(3) VC_RS(4) VC_RS(5) VC_RS(6) VC_RS(7) VC_RS(8) VC_RS(9) VC_RS(10)
    default: break;
  }
#undef VC_RS
  return hipErrorInvalidValue;
}

template <typename T, int NIN, int NOUT>
hipError_t launch_sandwich_multi_v(const SandScene* tab, int nscene, int nblocks, const int* skip, const int* act,
                                   int nthr, size_t lds, int rs, hipStream_t st) {
  if (nscene <= 0 || nblocks <= 0) return hipSuccess;
#define VC_RS(RR)                                                                                                 \
  case RR:                                                                                                        \
    if constexpr (RR <= SandRS<T, NIN>::max) {                                                                    \
      hipLaunchKernelGGL((k_xsandwich_multi<T, NIN, NOUT, RR>), dim3(nblocks), dim3(nthr), lds, st, tab, nscene, \
                         skip, act);                                                                              \
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
