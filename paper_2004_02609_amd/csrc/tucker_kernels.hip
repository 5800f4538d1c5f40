// Tucker rebuild of the stored kernel spectra (eq. 13, Sec. II.C) on the matrix cores.
//
// X = S x_1 U1 x_2 U2 x_3 U3 is three mode products, each a (batched) GEMM with small
// inner dimension r_i:
//   T1 (r1 r2 x D3)    = S (r1 r2 x r3) U3^T
//   T2[a] (D2 x D3)    = U2 (D2 x r2) T1[a] (r2 x D3),     a < r1
//   X (D1 x D2 D3)     = U1 (D1 x r1) T2 (r1 x D2 D3)      (the dominant one)
// computed by one strided batched GEMM kernel on v_mfma_*_16x16x4 (FP32 or FP64): a
// wave owns a 16 x 16 output tile and steps through K four at a time; operands come
// straight from memory (K is a Tucker rank, tens at most) with zero padding at edges.
#include <hip/hip_runtime.h>

#include "mvp_kernels.h"

namespace vc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// C[z][m][n] = sum_k A[z][m][k] B[z][k][n] with arbitrary element strides.
// 16x16x4 operand layout: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; its
// accumulator r holds C[4 (l / 16) + r][l % 16] for the FP32 instruction and
// C[l / 16 + 4 r][l % 16] for the FP64 one (measured on gfx950).
template <typename T>
__global__ void __launch_bounds__(256) k_mfma_gemm(const T* __restrict__ A, const T* __restrict__ B, T* __restrict__ C,
                                                   GemmArgs g) {
  if (g.skip && *g.skip) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 32 + (wave >> 1) * 16;
  const int n0 = blockIdx.x * 32 + (wave & 1) * 16;
  const int z = blockIdx.z;
  const T* Az = A + (int64_t)z * g.bsa;
  const T* Bz = B + (int64_t)z * g.bsb;
  T* Cz = C + (int64_t)z * g.bsc;
  const int li = lane & 15, lk = lane >> 4;
  const int am = m0 + li, bn = n0 + li;
  typename Mfma<T>::acc_t acc = {T(0), T(0), T(0), T(0)};
  for (int k0 = 0; k0 < g.K; k0 += 4) {
    const int k = k0 + lk;
    const T a = (am < g.M && k < g.K) ? Az[(int64_t)am * g.sam + (int64_t)k * g.sak] : T(0);
    const T b = (bn < g.N && k < g.K) ? Bz[(int64_t)k * g.sbk + (int64_t)bn * g.sbn] : T(0);
    acc = Mfma<T>::run(a, b, acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = sizeof(T) == 8 ? m0 + lk + 4 * r : m0 + 4 * lk + r;
    if (row < g.M && bn < g.N) Cz[(int64_t)row * g.scm + (int64_t)bn * g.scn] = acc[r];
  }
}

template <typename T>
hipError_t launch_mfma_gemm(const T* A, const T* B, T* C, const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) return hipErrorInvalidValue;
  dim3 grid((g.N + 31) / 32, (g.M + 31) / 32, g.batch);
  if (grid.y > 65535u || grid.z > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mfma_gemm<T>, grid, dim3(256), 0, st, A, B, C, g);
  return hipGetLastError();
}

template hipError_t launch_mfma_gemm<float>(const float*, const float*, float*, const GemmArgs&, hipStream_t);
template hipError_t launch_mfma_gemm<double>(const double*, const double*, double*, const GemmArgs&, hipStream_t);

// Many GEMMs in one launch (every stored pair of a rebuild step): a device table holds
// each GEMM's operands, sizes, strides, batch and first workgroup; a workgroup finds
// its GEMM by binary search.  A wave keeps its 16-row strip of A in registers (K <= 64,
// the Tucker ranks) and sweeps kGemmStrip output tiles along N, so one workgroup writes
// 32 x 32 * kGemmStrip elements.
constexpr int kGemmStrip = 8;
constexpr int kGemmKFrag = 16;   // K <= 4 * kGemmKFrag held in registers

template <typename T>
__global__ void __launch_bounds__(256) k_mfma_gemm_multi(const GemmDesc* __restrict__ tab, int ndesc,
                                                         const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lin = blockIdx.x;
  const GemmDesc& g = tab[find_scene(tab, ndesc, lin)];
  const int local = lin - g.blk0;
  const int per = g.gx * g.gy;
  const int z = local / per, rem = local - z * per;
  const int by = rem / g.gx, bx = rem - by * g.gx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int M = g.M, N = g.N, K = g.K;
  const T* Az = static_cast<const T*>(g.A) + (int64_t)z * g.bsa;
  const T* Bz = static_cast<const T*>(g.B) + (int64_t)z * g.bsb;
  T* Cz = static_cast<T*>(g.C) + (int64_t)z * g.bsc;
  const int m0 = by * 32 + (wave >> 1) * 16;
  const int am = m0 + li;
  T afrag[kGemmKFrag];
#pragma unroll
  for (int f = 0; f < kGemmKFrag; ++f) {
    const int k = 4 * f + lk;
    afrag[f] = (f * 4 < K && am < M && k < K) ? Az[(int64_t)am * g.sam + (int64_t)k * g.sak] : T(0);
  }
  for (int t = 0; t < kGemmStrip; ++t) {
    const int n0 = (bx * kGemmStrip + t) * 32 + (wave & 1) * 16;
    if (n0 >= N) break;
    const int bn = n0 + li;
    typename Mfma<T>::acc_t acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int f = 0; f < kGemmKFrag; ++f) {
      if (f * 4 >= K) break;
      const int k = 4 * f + lk;
      const T b = (bn < N && k < K) ? Bz[(int64_t)k * g.sbk + (int64_t)bn * g.sbn] : T(0);
      acc = Mfma<T>::run(afrag[f], b, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = sizeof(T) == 8 ? m0 + lk + 4 * r : m0 + 4 * lk + r;
      if (row < M && bn < N) Cz[(int64_t)row * g.scm + (int64_t)bn * g.scn] = acc[r];
    }
  }
}

// lays out the table's workgroups (gx, gy, blk0) and returns the total, or -1 when a
// GEMM does not fit the kernel (K above the register strip)
int gemm_table_layout(GemmDesc* d, int n) {
  int64_t blk = 0;
  for (int i = 0; i < n; ++i) {
    if (d[i].K < 1 || d[i].K > 4 * kGemmKFrag || d[i].M < 1 || d[i].N < 1 || d[i].batch < 1) return -1;
    d[i].gx = (d[i].N + 32 * kGemmStrip - 1) / (32 * kGemmStrip);
    d[i].gy = (d[i].M + 31) / 32;
    d[i].blk0 = (int)blk;
    blk += (int64_t)d[i].gx * d[i].gy * d[i].batch;
    if (blk > (int64_t)1 << 30) return -1;
  }
  return (int)blk;
}

template <typename T>
hipError_t launch_mfma_gemm_multi(const GemmDesc* tab, int ndesc, int nblocks, const int* skip, hipStream_t st) {
  if (ndesc <= 0 || nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mfma_gemm_multi<T>, dim3(nblocks), dim3(256), 0, st, tab, ndesc, skip);
  return hipGetLastError();
}

template hipError_t launch_mfma_gemm_multi<float>(const GemmDesc*, int, int, const int*, hipStream_t);
template hipError_t launch_mfma_gemm_multi<double>(const GemmDesc*, int, int, const int*, hipStream_t);

// FP64 -> FP32 copy of the compressed factors
__global__ void k_to_f32(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// out[b][a][c] = in[a][b][c] (the unfoldings the compression hands to the SVD)
__global__ void k_swap01(const double* __restrict__ in, double* __restrict__ out, int A, int B, int C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)A * B * C;
  if (i >= n) return;
  const int64_t c = i % C, ab = i / C;
  const int64_t b = ab % B, a = ab / B;
  out[(b * A + a) * C + c] = in[i];
}

hipError_t launch_swap01(const double* in, double* out, int A, int B, int C, hipStream_t st) {
  const int64_t n = (int64_t)A * B * C;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_swap01, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, A, B, C);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* in, float* out, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

}  // namespace vc
