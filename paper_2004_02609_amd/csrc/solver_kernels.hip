// FP64 kernels of the iterative solve: Gram-Schmidt products for GMRES (several
// right-hand sides advance together, each column with its own coefficients), the
// block-diagonal-diagonal preconditioner of eq. (14) (Sec. II.D) and the charge ->
// capacitance reduction of eq. (8).  Reductions run in a fixed order (per-block
// partials, then a serial pass) so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "mvp_kernels.h"

namespace vc {

constexpr int kRedThreads = 256;
constexpr int kChunk = 8192;   // rows per partial-sum block

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// partial[(chunk*nrhs + r)*k + i] = sum_{n in chunk} V_i[r][n] * w[r][n]
__global__ void __launch_bounds__(kRedThreads)
k_dot_partial(const double* __restrict__ V, int64_t ldv, int64_t N, int k, const double* __restrict__ w,
              int64_t ldw, int nrhs, double* __restrict__ partial, const int* __restrict__ active) {
  __shared__ double red[kRedThreads];
  const int chunk = blockIdx.x, r = blockIdx.y;
  const int64_t n0 = (int64_t)chunk * kChunk;
  const int64_t n1 = n0 + kChunk < N ? n0 + kChunk : N;
  double* out = partial + ((int64_t)chunk * nrhs + r) * k;
  if (active && !active[r]) {
    if (threadIdx.x == 0)
      for (int i = 0; i < k; ++i) out[i] = 0.0;
    return;
  }
  const double* wr = w + (int64_t)r * ldw;
  for (int i = 0; i < k; ++i) {
    const double* vi = V + (int64_t)i * ldv + (int64_t)r * N;
    double acc = 0.0;
    for (int64_t n = n0 + threadIdx.x; n < n1; n += blockDim.x) acc += vi[n] * wr[n];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[i] = acc;
  }
}

__global__ void k_dot_final(const double* __restrict__ partial, int nchunk, int nrhs, int k, double* __restrict__ h,
                            int64_t ldh) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= k * nrhs) return;
  const int r = id / k, i = id - r * k;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[((int64_t)c * nrhs + r) * k + i];
  h[(int64_t)r * ldh + i] = s;
}

// h[r*ldh + i] = <V_i[r], w[r]> for i < k (V_i[r] at V + i*ldv + r*N)
hipError_t launch_gemv_t(const double* V, int64_t ldv, int64_t N, int k, const double* w, int64_t ldw, int nrhs,
                         double* h, int64_t ldh, const int* active, double* partial, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  const int nchunk = (int)((N + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_dot_partial, dim3(nchunk, nrhs), dim3(kRedThreads), 0, st, V, ldv, N, k, w, ldw, nrhs,
                     partial, active);
  hipLaunchKernelGGL(k_dot_final, dim3((k * nrhs + 127) / 128), dim3(128), 0, st, partial, nchunk, nrhs, k, h, ldh);
  return hipGetLastError();
}

int64_t gemv_t_partial_size(int64_t N, int kmax, int nrhs) {
  return ((N + kChunk - 1) / kChunk) * (int64_t)nrhs * kmax;
}

// w[r] -= sum_{i<k} V_i[r] h[r*ldh + i]
__global__ void k_gemv_n_sub(const double* __restrict__ V, int64_t ldv, int64_t N, int k, const double* __restrict__ h,
                             int64_t ldh, double* __restrict__ w, int64_t ldw, const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += V[(int64_t)i * ldv + (int64_t)r * N + n] * h[(int64_t)r * ldh + i];
  w[(int64_t)r * ldw + n] -= acc;
}

hipError_t launch_gemv_n_sub(const double* V, int64_t ldv, int64_t N, int k, const double* h, int64_t ldh, double* w,
                             int64_t ldw, int nrhs, const int* active, int, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_n_sub, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, V, ldv, N, k, h, ldh,
                     w, ldw, active);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kRedThreads)
k_colnorm(const double* __restrict__ w, int64_t ldw, int64_t N, double* __restrict__ out) {
  __shared__ double red[kRedThreads];
  const int r = blockIdx.x;
  const double* wr = w + (int64_t)r * ldw;
  double acc = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x) acc += wr[n] * wr[n];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[r] = sqrt(acc);
}

hipError_t launch_colnorm(const double* w, int64_t ldw, int64_t N, int nrhs, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colnorm, dim3(nrhs), dim3(kRedThreads), 0, st, w, ldw, N, out);
  return hipGetLastError();
}

// mode 0: w[r] *= s[r]; mode 1: w[r] /= s[r] (w[r] = 0 when s[r] == 0)
__global__ void k_scale_cols(double* __restrict__ w, int64_t ldw, int64_t N, const double* __restrict__ s, int mode) {
  const int r = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double f = s[r];
  if (mode == 1) {
    w[(int64_t)r * ldw + n] = f != 0.0 ? w[(int64_t)r * ldw + n] / f : 0.0;
  } else {
    w[(int64_t)r * ldw + n] *= f;
  }
}

hipError_t launch_scale_cols(double* w, int64_t ldw, int64_t N, int nrhs, const double* s, int mode, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, w, ldw, N, s, mode);
  return hipGetLastError();
}

// y[r] += a[r] x[r] (sub = 0) or y[r] = x[r] - y[r] (sub = 1, a unused)
__global__ void k_axpy_cols(double* __restrict__ y, const double* __restrict__ x, int64_t N,
                            const double* __restrict__ a, int sub) {
  const int r = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t o = (int64_t)r * N + n;
  if (sub) y[o] = x[o] - y[o];
  else y[o] += a[r] * x[o];
}

hipError_t launch_axpy_cols(double* y, const double* x, int64_t N, int nrhs, const double* a, int sub,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, y, x, N, a, sub);
  return hipGetLastError();
}

// Dielectric rows of eq. (14): y = x / I_kk; conductor rows are overwritten by the block apply.
__global__ void k_diag_scale(const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ dinv,
                             int64_t N) {
  const int r = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  y[(int64_t)r * N + n] = dinv[n] * x[(int64_t)r * N + n];
}

hipError_t launch_diag_scale(const double* x, double* y, const double* dinv, int64_t N, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_scale, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, x, y, dinv, N);
  return hipGetLastError();
}

// Conductor rows of eq. (14): for each box, y_box = Binv x_box with the box's (shared,
// de-duplicated) inverse block.  One workgroup per box; x_box staged in LDS.
constexpr int kBoxThreads = 256;
constexpr int kBoxLds = 4096;   // doubles of x_box staged per pass
__global__ void __launch_bounds__(kBoxThreads)
k_block_apply(const double* __restrict__ x, double* __restrict__ y, int64_t N, int nrhs,
              const int32_t* __restrict__ box_ptr, const int32_t* __restrict__ box_panels,
              const int32_t* __restrict__ box_block, const int64_t* __restrict__ block_off,
              const int32_t* __restrict__ block_n, const double* __restrict__ blocks) {
  __shared__ double xs[kBoxLds];
  const int box = blockIdx.x;
  const int p0 = box_ptr[box];
  const int nb = box_ptr[box + 1] - p0;
  const int blk = box_block[box];
  const double* B = blocks + block_off[blk];
  const int rpp = kBoxLds / nb;   // right-hand sides per pass (nb <= kBoxLds guaranteed by the host)
  for (int r0 = 0; r0 < nrhs; r0 += rpp) {
    const int rn = (nrhs - r0) < rpp ? (nrhs - r0) : rpp;
    __syncthreads();
    for (int e = threadIdx.x; e < rn * nb; e += blockDim.x) {
      const int r = e / nb, j = e - r * nb;
      xs[e] = x[(int64_t)(r0 + r) * N + box_panels[p0 + j]];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rn * nb; e += blockDim.x) {
      const int r = e / nb, i = e - r * nb;
      const double* Bi = B + (int64_t)i * nb;
      const double* xr = xs + r * nb;
      double acc = 0.0;
      for (int j = 0; j < nb; ++j) acc += Bi[j] * xr[j];
      y[(int64_t)(r0 + r) * N + box_panels[p0 + i]] = acc;
    }
  }
  (void)block_n;
}

hipError_t launch_block_apply(const double* x, double* y, int64_t N, int nrhs, const int32_t* box_ptr,
                              const int32_t* box_panels, const int32_t* box_block, const int64_t* block_off,
                              const int32_t* block_n, const double* blocks, int nbox, hipStream_t st) {
  if (nbox == 0) return hipSuccess;
  hipLaunchKernelGGL(k_block_apply, dim3(nbox), dim3(kBoxThreads), 0, st, x, y, N, nrhs, box_ptr, box_panels,
                     box_block, block_off, block_n, blocks);
  return hipGetLastError();
}

// C[i][j] = scale * sum_{k in conductor i} weight[k] * rho[j*N + k]   (eq. 8)
__global__ void __launch_bounds__(kRedThreads)
k_cap_reduce(const double* __restrict__ rho, int64_t N, int m, const int32_t* __restrict__ cond_panels,
             const int32_t* __restrict__ cond_ptr, const double* __restrict__ weight, double scale,
             double* __restrict__ C) {
  __shared__ double red[kRedThreads];
  const int i = blockIdx.x, j = blockIdx.y;
  double acc = 0.0;
  for (int t = cond_ptr[i] + threadIdx.x; t < cond_ptr[i + 1]; t += blockDim.x) {
    const int k = cond_panels[t];
    acc += weight[k] * rho[(int64_t)j * N + k];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) C[(int64_t)i * m + j] = scale * acc;
}

hipError_t launch_cap_reduce(const double* rho, int64_t N, int m, const int32_t* cond_panels, const int32_t* cond_ptr,
                             const double* weight, double scale, double* C, hipStream_t st) {
  hipLaunchKernelGGL(k_cap_reduce, dim3(m, m), dim3(kRedThreads), 0, st, rho, N, m, cond_panels, cond_ptr, weight,
                     scale, C);
  return hipGetLastError();
}

// C = scale * W^T rho for nrhs columns (eq. 8): C[i, j] over the panels of conductor i
__global__ void __launch_bounds__(kRedThreads)
k_cap_reduce_n(const double* __restrict__ rho, int64_t N, int nrhs, const int32_t* __restrict__ cond_panels,
               const int32_t* __restrict__ cond_ptr, const double* __restrict__ weight, double scale,
               double* __restrict__ C) {
  __shared__ double red[kRedThreads];
  const int i = blockIdx.x, j = blockIdx.y;
  double acc = 0.0;
  for (int t = cond_ptr[i] + threadIdx.x; t < cond_ptr[i + 1]; t += blockDim.x) {
    const int k = cond_panels[t];
    acc += weight[k] * rho[(int64_t)j * N + k];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) C[(int64_t)i * nrhs + j] = scale * acc;
}

hipError_t launch_cap_reduce_n(const double* rho, int64_t N, int m, int nrhs, const int32_t* cond_panels,
                               const int32_t* cond_ptr, const double* weight, double scale, double* C,
                               hipStream_t st) {
  if (m <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cap_reduce_n, dim3(m, nrhs), dim3(kRedThreads), 0, st, rho, N, nrhs, cond_panels, cond_ptr,
                     weight, scale, C);
  return hipGetLastError();
}

// adjoint of the reduction: g_rho[k, j] = scale * w_k * g_C[cond_k, j] (0 on dielectric panels)
__global__ void k_cap_reduce_adj(const double* __restrict__ gC, int64_t N, int nrhs, const int32_t* __restrict__ pcond,
                                 const double* __restrict__ weight, double scale, double* __restrict__ grho) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (k >= N) return;
  const int ci = pcond[k];
  grho[(int64_t)j * N + k] = ci >= 0 ? scale * weight[k] * gC[(int64_t)ci * nrhs + j] : 0.0;
}

hipError_t launch_cap_reduce_adj(const double* gC, int64_t N, int nrhs, const int32_t* pcond, const double* weight,
                                 double scale, double* grho, hipStream_t st) {
  if (N <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cap_reduce_adj, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, gC, N, nrhs, pcond,
                     weight, scale, grho);
  return hipGetLastError();
}

// dC[b, i, j] = scale * sum over the entries e of block b of
//   cond_e >= 0 (free-charge weight term):  [i == cond_e] rho[k_e, j]
//   cond_e <  0 (jump term, eq. 7):         -coef_e lam[k_e, i] rho[k_e, j]
// one workgroup per (b, i, j); deterministic reduction order
__global__ void __launch_bounds__(kRedThreads)
k_grad_eps(const int32_t* __restrict__ bptr, const int32_t* __restrict__ ek, const int32_t* __restrict__ econd,
           const double* __restrict__ ecoef, const double* __restrict__ rho, const double* __restrict__ lam,
           int64_t N, int m, double scale, double* __restrict__ dC) {
  __shared__ double red[kRedThreads];
  const int b = blockIdx.x, i = blockIdx.y, j = blockIdx.z;
  double acc = 0.0;
  for (int t = bptr[b] + threadIdx.x; t < bptr[b + 1]; t += blockDim.x) {
    const int64_t k = ek[t];
    const int ce = econd[t];
    const double r = rho[(int64_t)j * N + k];
    if (ce >= 0) {
      if (ce == i) acc += r;
    } else {
      acc -= ecoef[t] * lam[(int64_t)i * N + k] * r;
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) dC[((int64_t)b * m + i) * m + j] = scale * acc;
}

hipError_t launch_grad_eps(const int32_t* bptr, const int32_t* ek, const int32_t* econd, const double* ecoef,
                           const double* rho, const double* lam, int64_t N, int m, int nblocks, double scale,
                           double* dC, hipStream_t st) {
  if (nblocks <= 0 || m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_eps, dim3(nblocks, m, m), dim3(kRedThreads), 0, st, bptr, ek, econd, ecoef, rho, lam, N,
                     m, scale, dC);
  return hipGetLastError();
}

}  // namespace vc
