// FP64 kernels of the iterative solve: Gram-Schmidt products for GMRES (several
// right-hand sides advance together, each column with its own coefficients), the
// block-diagonal-diagonal preconditioner of eq. (14) (Sec. II.D) and the charge ->
// capacitance reduction of eq. (8).  Reductions run in a fixed order (per-block
// partials, then a serial pass) so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "mvp_kernels.h"

namespace vc {

constexpr int kRedThreads = 256;

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

// Inner products for Gram-Schmidt.  Work is split over (row chunk, block of 8 basis
// vectors, right-hand side): each thread keeps 8 running sums over its rows (w read once
// per block), the wave sums them with shuffles and the waves through LDS, in a fixed
// order.  partial[(chunk*nrhs + r)*k + i] = sum_{n in chunk} V_i[r][n] * w[r][n].
constexpr int kDotChunk = 2048;   // rows per partial sum
constexpr int kDotBlk = 8;        // basis vectors per workgroup

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kRedThreads)
k_dot_partial(const double* __restrict__ V, int64_t ldv, int64_t N, int k, const double* __restrict__ w,
              int64_t ldw, int nrhs, double* __restrict__ partial, const int* __restrict__ active) {
  __shared__ double red[kDotBlk][kRedThreads / 64];
  const int chunk = blockIdx.x, kb = blockIdx.y, r = blockIdx.z;
  const int i0 = kb * kDotBlk;
  const int nb = k - i0 < kDotBlk ? k - i0 : kDotBlk;
  double* out = partial + ((int64_t)chunk * nrhs + r) * k + i0;
  if (active && !active[r]) {
    if ((int)threadIdx.x < nb) out[threadIdx.x] = 0.0;
    return;
  }
  const int64_t n0 = (int64_t)chunk * kDotChunk;
  const int64_t n1 = n0 + kDotChunk < N ? n0 + kDotChunk : N;
  const double* wr = w + (int64_t)r * ldw;
  const double* v0 = V + (int64_t)i0 * ldv + (int64_t)r * N;
  double acc[kDotBlk];
#pragma unroll
  for (int q = 0; q < kDotBlk; ++q) acc[q] = 0.0;
  for (int64_t n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
    const double wn = wr[n];
#pragma unroll
    for (int q = 0; q < kDotBlk; ++q)
      if (q < nb) acc[q] += v0[(int64_t)q * ldv + n] * wn;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kDotBlk; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == 0) red[q][wv] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < nb) {
    double t = 0.0;
    for (int u = 0; u < (int)(blockDim.x >> 6); ++u) t += red[threadIdx.x][u];
    out[threadIdx.x] = t;
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
  const int nchunk = (int)((N + kDotChunk - 1) / kDotChunk);
  const int nkb = (k + kDotBlk - 1) / kDotBlk;
  hipLaunchKernelGGL(k_dot_partial, dim3(nchunk, nkb, nrhs), dim3(kRedThreads), 0, st, V, ldv, N, k, w, ldw, nrhs,
                     partial, active);
  hipLaunchKernelGGL(k_dot_final, dim3((k * nrhs + 127) / 128), dim3(128), 0, st, partial, nchunk, nrhs, k, h, ldh);
  return hipGetLastError();
}

int64_t gemv_t_partial_size(int64_t N, int kmax, int nrhs) {
  return ((N + kDotChunk - 1) / kDotChunk) * (int64_t)nrhs * kmax;
}

// w[r] -= sum_{i<k_r} V_i[r] h[r*ldh + i], k_r = kcol[r] when given (basis vectors past
// a column's own count are never read: they may hold stale memory), else k
__global__ void k_gemv_n_sub(const double* __restrict__ V, int64_t ldv, int64_t N, int k, const double* __restrict__ h,
                             int64_t ldh, double* __restrict__ w, int64_t ldw, const int* __restrict__ active,
                             const int* __restrict__ kcol) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int kr = kcol ? min(kcol[r], k) : k;
  double acc = 0.0;
  for (int i = 0; i < kr; ++i) acc += V[(int64_t)i * ldv + (int64_t)r * N + n] * h[(int64_t)r * ldh + i];
  w[(int64_t)r * ldw + n] -= acc;
}

hipError_t launch_gemv_n_sub(const double* V, int64_t ldv, int64_t N, int k, const double* h, int64_t ldh, double* w,
                             int64_t ldw, int nrhs, const int* active, int, hipStream_t st, const int* kcol) {
  hipLaunchKernelGGL(k_gemv_n_sub, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, V, ldv, N, k, h, ldh,
                     w, ldw, active, kcol);
  return hipGetLastError();
}

// column 2-norms: per-chunk partial sums of squares (wave shuffles, fixed order), then
// one thread per column adds the chunks and takes the root
__global__ void __launch_bounds__(kRedThreads)
k_sumsq_partial(const double* __restrict__ w, int64_t ldw, int64_t N, int nrhs, double* __restrict__ partial,
                const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double red[kRedThreads / 64];
  const int chunk = blockIdx.x, r = blockIdx.y;
  const int64_t n0 = (int64_t)chunk * kDotChunk;
  const int64_t n1 = n0 + kDotChunk < N ? n0 + kDotChunk : N;
  const double* wr = w + (int64_t)r * ldw;
  double acc = 0.0;
  for (int64_t n = n0 + threadIdx.x; n < n1; n += blockDim.x) acc += wr[n] * wr[n];
  const double t = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double u = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) u += red[q];
    partial[(int64_t)chunk * nrhs + r] = u;
  }
}

__global__ void k_sumsq_final(const double* __restrict__ partial, int nchunk, int nrhs, double* __restrict__ out,
                              const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[(int64_t)c * nrhs + r];
  out[r] = sqrt(s);
}

// norms of nrhs columns; partial: caller workspace of colnorm_partial_size(N, nrhs)
hipError_t launch_colnorm(const double* w, int64_t ldw, int64_t N, int nrhs, double* out, double* partial,
                          hipStream_t st, const int* skip) {
  const int nchunk = (int)((N + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(k_sumsq_partial, dim3(nchunk, nrhs), dim3(kRedThreads), 0, st, w, ldw, N, nrhs, partial, skip);
  hipLaunchKernelGGL(k_sumsq_final, dim3((nrhs + 63) / 64), dim3(64), 0, st, partial, nchunk, nrhs, out, skip);
  return hipGetLastError();
}

int64_t colnorm_partial_size(int64_t N, int nrhs) { return ((N + kDotChunk - 1) / kDotChunk) * (int64_t)nrhs; }

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
                            const double* __restrict__ a, int sub, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int r = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int64_t o = (int64_t)r * N + n;
  if (sub) y[o] = x[o] - y[o];
  else y[o] += a[r] * x[o];
}

hipError_t launch_axpy_cols(double* y, const double* x, int64_t N, int nrhs, const double* a, int sub,
                            hipStream_t st, const int* skip) {
  hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, y, x, N, a, sub, skip);
  return hipGetLastError();
}

// Dielectric rows of eq. (14): y = x / I_kk; conductor rows are overwritten by the block apply.
// (dinv_ld: column stride of dinv, 0 when one diagonal serves every column)
__global__ void k_diag_scale(const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ dinv,
                             int64_t dinv_ld, int64_t N, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int r = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  y[(int64_t)r * N + n] = dinv[(int64_t)r * dinv_ld + n] * x[(int64_t)r * N + n];
}

hipError_t launch_diag_scale(const double* x, double* y, const double* dinv, int64_t N, int nrhs, const int* skip,
                             hipStream_t st, int64_t dinv_ld) {
  hipLaunchKernelGGL(k_diag_scale, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, x, y, dinv, dinv_ld, N,
                     skip);
  return hipGetLastError();
}

// Conductor rows of eq. (14): for each box, y_box = Binv x_box with the box's (shared,
// de-duplicated) inverse block, stored transposed.  One workgroup per box; x_box staged
// in LDS.  When the box has fewer panels than the workgroup has threads, G = threads / nb
// groups of threads each sum every G-th column of the block for all staged right-hand
// sides (each block entry loaded once per pass), and the groups' sums are added in a
// fixed order through LDS.  gridDim.y = S splits each box's rows into S slices, one per
// workgroup, so a few large boxes still spread over the chip (every slice stages the
// whole x_box; the columns of a row are summed by more groups).
constexpr int kBoxThreads = 512;
constexpr int kBoxLds = 4096;   // doubles of x_box staged per pass
constexpr int kBoxRB = 4;       // right-hand sides per accumulation sweep
__global__ void __launch_bounds__(kBoxThreads)
k_block_apply(const double* __restrict__ x, double* __restrict__ y, int64_t N, int nrhs,
              const int32_t* __restrict__ box_ptr, const int32_t* __restrict__ box_panels,
              const int32_t* __restrict__ box_block, const int64_t* __restrict__ block_off,
              const int32_t* __restrict__ block_n, const double* __restrict__ blocks, const int* __restrict__ skip,
              const int32_t* __restrict__ box_c0, const int32_t* __restrict__ box_nc, int trans) {
  if (skip && *skip) return;
  __shared__ double xs[kBoxLds];
  __shared__ double red[kBoxRB * kBoxThreads];
  const int box = blockIdx.x;
  if (box_c0) {   // the box belongs to one problem of a packed set: its own columns only
    const int64_t o = (int64_t)box_c0[box] * N;
    x += o;
    y += o;
    nrhs = box_nc[box];
  }
  const int p0 = box_ptr[box];
  const int nb = box_ptr[box + 1] - p0;
  // this workgroup's slice of the box's rows: [lo, lo + nr)
  const int rsl = (nb + (int)gridDim.y - 1) / (int)gridDim.y;
  const int lo = (int)blockIdx.y * rsl;
  const int nr = nb - lo < rsl ? nb - lo : rsl;
  if (nr <= 0) return;   // uniform over the workgroup, before any barrier
  const int blk = box_block[box];
  const double* B = blocks + block_off[blk];
  const int rpp = kBoxLds / nb;   // right-hand sides per pass (nb <= kBoxLds guaranteed by the host)
  const int t = threadIdx.x;
  const int G = nr < kBoxThreads ? kBoxThreads / nr : 1;
  // the block is stored transposed: B^T[j][i] = Binv[i][j] (lanes, consecutive i, read
  // consecutive addresses); the transposed apply reads B^T[i][j]
  const int64_t sj = trans ? 1 : nb, si = trans ? nb : 1;
  for (int r0 = 0; r0 < nrhs; r0 += rpp) {
    const int rn = (nrhs - r0) < rpp ? (nrhs - r0) : rpp;
    __syncthreads();
    for (int e = t; e < rn * nb; e += blockDim.x) {
      const int r = e / nb, j = e - r * nb;
      xs[e] = x[(int64_t)(r0 + r) * N + box_panels[p0 + j]];
    }
    __syncthreads();
    for (int rb = 0; rb < rn; rb += kBoxRB) {
      const int rbn = rn - rb < kBoxRB ? rn - rb : kBoxRB;
      for (int i0 = 0; i0 < nr; i0 += (G > 1 ? nr : kBoxThreads)) {
        const int g = G > 1 ? t / nr : 0;
        const int il = G > 1 ? t - g * nr : i0 + t;   // row within the slice
        const int i = lo + il;
        const bool on = G > 1 ? g < G : il < nr;
        double acc[kBoxRB];
#pragma unroll
        for (int q = 0; q < kBoxRB; ++q) acc[q] = 0.0;
        if (on) {
          const double* bi = B + (int64_t)i * si;
          const double* xr = xs + rb * nb;
#pragma unroll 4
          for (int j = g; j < nb; j += G) {
            const double bv = bi[(int64_t)j * sj];
#pragma unroll
            for (int q = 0; q < kBoxRB; ++q)
              if (q < rbn) acc[q] += bv * xr[q * nb + j];
          }
        }
        if (G == 1) {
          if (on)
#pragma unroll
            for (int q = 0; q < kBoxRB; ++q)
              if (q < rbn) y[(int64_t)(r0 + rb + q) * N + box_panels[p0 + i]] = acc[q];
        } else {
          if (on)
#pragma unroll
            for (int q = 0; q < kBoxRB; ++q) red[(q * G + g) * nr + il] = acc[q];
          __syncthreads();
          for (int e = t; e < rbn * nr; e += blockDim.x) {
            const int q = e / nr, ii = e - q * nr;
            double v = 0.0;
            for (int gg = 0; gg < G; ++gg) v += red[(q * G + gg) * nr + ii];
            y[(int64_t)(r0 + rb + q) * N + box_panels[p0 + lo + ii]] = v;
          }
          __syncthreads();
        }
      }
    }
  }
  (void)block_n;
}

hipError_t launch_block_apply(const double* x, double* y, int64_t N, int nrhs, const int32_t* box_ptr,
                              const int32_t* box_panels, const int32_t* box_block, const int64_t* block_off,
                              const int32_t* block_n, const double* blocks, int nbox, const int* skip,
                              hipStream_t st, const int32_t* box_c0, const int32_t* box_nc, int trans) {
  if (nbox == 0) return hipSuccess;
  // row slices per box: enough workgroups for the chip when there are few boxes
  int S = (512 + nbox - 1) / nbox;
  if (S > 4) S = 4;
  hipLaunchKernelGGL(k_block_apply, dim3(nbox, S), dim3(kBoxThreads), 0, st, x, y, N, nrhs, box_ptr, box_panels,
                     box_block, block_off, block_n, blocks, skip, box_c0, box_nc, trans);
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

// ------------------------------------------------------------------ device-side GMRES cycle
// The restart cycle runs without host round trips (so it can be captured as a graph):
// per-column Hessenberg columns, Givens rotations, convergence masks and the final
// triangular solve live on the device.  One workgroup, one thread per column (up to
// kCycleMax columns).
// Per-column state layout: H[c][(m+1) x m] row-major, cs/sn[c][m], g[c][m+1].

constexpr int kCycleMax = 256;
// a power of two (the block reductions halve the width) of at least one wave
static inline unsigned cycle_threads(int nrhs) { return nrhs <= 64 ? 64u : (nrhs <= 128 ? 128u : 256u); }

__device__ __forceinline__ int any_over_block(int v, int* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] |= red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// start of a cycle from the residual norms rn: relative residual, active masks,
// g = (|r|, 0, ...), scal = |r| for V_0 = r / |r| (0 = zero column), skip flags
__global__ void k_cycle_start(int nrhs, int m, const double* __restrict__ rn, const double* __restrict__ bn,
                              const double* __restrict__ rtolp, int* __restrict__ act_cycle, int* __restrict__ act_step,
                              double* __restrict__ g, double* __restrict__ scal, int* __restrict__ kd,
                              int* __restrict__ skip, double* __restrict__ rre_out) {
  if (skip[2]) return;   // problem disabled for this round (batched form): state left as is
  __shared__ int red[kCycleMax];
  const int c = threadIdx.x;
  const double rtol = *rtolp;
  int a = 0;
  if (c < nrhs) {
    const double b = bn[c], r = rn[c];
    const double rre = b > 0.0 ? r / b : 0.0;
    rre_out[c] = rre;
    a = (b > 0.0 && !(rre <= rtol)) ? 1 : 0;   // NaN stays active; the host reports it
    act_cycle[c] = a;
    act_step[c] = a;
    kd[c] = 0;
    for (int i = 0; i <= m; ++i) g[(int64_t)c * (m + 1) + i] = 0.0;
    g[(int64_t)c * (m + 1)] = r;
    scal[c] = a ? r : 0.0;
  }
  const int any = any_over_block(a, red);
  if (threadIdx.x == 0) {
    skip[0] = any ? 0 : 1;   // cycle-level: nothing to do this cycle
    skip[1] = any ? 0 : 1;   // step-level: no column still iterating
  }
}

hipError_t launch_cycle_start(int nrhs, int m, const double* rn, const double* bn, const double* rtol, int* act_cycle,
                              int* act_step, double* g, double* scal, int* kd, int* skip, double* rre_out,
                              hipStream_t st) {
  if (nrhs > kCycleMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cycle_start, dim3(1), dim3(cycle_threads(nrhs)), 0, st, nrhs, m, rn, bn, rtol, act_cycle, act_step, g, scal,
                     kd, skip, rre_out);
  return hipGetLastError();
}

// State the host reads after a segment of Arnoldi steps in the relaxed mixed form, in
// one copy: out[0] = the largest residual estimate |g(kd)| / |b| over the columns still
// iterating (0 if none), out[1] = the step-level skip flag, out[2 + c] = iters[c].
__global__ void k_relax_state(int nrhs, int m, const double* __restrict__ g, const int* __restrict__ kd,
                              const int* __restrict__ act_step, const double* __restrict__ bn,
                              const int* __restrict__ iters, const int* __restrict__ skip, double* __restrict__ out) {
  __shared__ double red[kCycleMax];
  const int c = threadIdx.x;
  double e = 0.0;
  if (c < nrhs) {
    if (act_step[c] && bn[c] > 0.0) {
      e = fabs(g[(int64_t)c * (m + 1) + kd[c]]) / bn[c];
      if (!(e == e)) e = INFINITY;   // a NaN estimate keeps FP64 products
    }
    out[2 + c] = (double)iters[c];
  }
  red[c] = e;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (c < s) red[c] = fmax(red[c], red[c + s]);
    __syncthreads();
  }
  if (c == 0) {
    out[0] = red[0];
    out[1] = (double)skip[1];
  }
}

hipError_t launch_relax_state(int nrhs, int m, const double* g, const int* kd, const int* act_step, const double* bn,
                              const int* iters, const int* skip, double* out, hipStream_t st) {
  if (nrhs > kCycleMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_relax_state, dim3(1), dim3(cycle_threads(nrhs)), 0, st, nrhs, m, g, kd, act_step, bn, iters,
                     skip, out);
  return hipGetLastError();
}

// Arnoldi step j: H(:, j) = h1 + h2 (classical Gram-Schmidt, twice), H(j+1, j) = |w|,
// previous rotations applied, new rotation from (H(j,j), H(j+1,j)), g rotated; a column
// freezes when its residual estimate |g(j+1)| / |b| <= rtol / 2, on breakdown, or at
// the end of the cycle.  scal = |w| for V_{j+1} = w / |w| (0 once frozen).
__device__ __forceinline__ void arnoldi_step(int c, int j, int nrhs, int m, const double* __restrict__ h1,
                                             const double* __restrict__ h2, int ldh, double hnc,
                                             double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                                             double* __restrict__ g, const double* __restrict__ bn, double rtol,
                                             int* __restrict__ act_step, int* __restrict__ kd, int* __restrict__ iters,
                                             double* __restrict__ scal, int* __restrict__ skip, int* __restrict__ bad,
                                             int* red) {
  int still = 0;
  if (c < nrhs) {
    if (act_step[c]) {
      double* Hc = H + (int64_t)c * (m + 1) * m;
      double* csc = cs + (int64_t)c * m;
      double* snc = sn + (int64_t)c * m;
      double* gc = g + (int64_t)c * (m + 1);
      for (int i = 0; i <= j; ++i) Hc[i * m + j] = h1[(int64_t)c * ldh + i] + h2[(int64_t)c * ldh + i];
      Hc[(j + 1) * m + j] = hnc;
      for (int i = 0; i < j; ++i) {
        const double a = Hc[i * m + j], b = Hc[(i + 1) * m + j];
        Hc[i * m + j] = csc[i] * a + snc[i] * b;
        Hc[(i + 1) * m + j] = -snc[i] * a + csc[i] * b;
      }
      const double a = Hc[j * m + j], b = Hc[(j + 1) * m + j];
      const double rr = hypot(a, b);
      const double cc = rr > 0.0 ? a / rr : 1.0, ss = rr > 0.0 ? b / rr : 0.0;
      csc[j] = cc;
      snc[j] = ss;
      Hc[j * m + j] = rr;
      Hc[(j + 1) * m + j] = 0.0;
      gc[j + 1] = -ss * gc[j];
      gc[j] = cc * gc[j];
      const double est = fabs(gc[j + 1]) / bn[c];
      if (!isfinite(est)) bad[0] = 1;
      const bool breakdown = hnc <= 1e-300 || hnc <= 1e-14 * fabs(rr);
      kd[c] = j + 1;
      iters[c] += 1;
      still = (est > 0.5 * rtol && !breakdown && j + 1 < m && isfinite(est)) ? 1 : 0;
      act_step[c] = still;
      scal[c] = still ? hnc : 0.0;
    } else {
      scal[c] = 0.0;
    }
  }
  const int any = any_over_block(still, red);
  if (threadIdx.x == 0) skip[1] = any ? 0 : 1;
}

__global__ void k_arnoldi(int j, int nrhs, int m, const double* __restrict__ h1, const double* __restrict__ h2,
                          int ldh, const double* __restrict__ hn, double* __restrict__ H, double* __restrict__ cs,
                          double* __restrict__ sn, double* __restrict__ g, const double* __restrict__ bn,
                          const double* __restrict__ rtolp, int* __restrict__ act_step, int* __restrict__ kd, int* __restrict__ iters,
                          double* __restrict__ scal, int* __restrict__ skip, int* __restrict__ bad) {
  __shared__ int red[kCycleMax];
  const int c = threadIdx.x;
  arnoldi_step(c, j, nrhs, m, h1, h2, ldh, c < nrhs ? hn[c] : 0.0, H, cs, sn, g, bn, *rtolp, act_step, kd, iters,
               scal, skip, bad, red);
}

hipError_t launch_arnoldi(int j, int nrhs, int m, const double* h1, const double* h2, int ldh, const double* hn,
                          double* H, double* cs, double* sn, double* g, const double* bn, const double* rtol,
                          int* act_step, int* kd, int* iters, double* scal, int* skip, int* bad, hipStream_t st) {
  if (nrhs > kCycleMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(cycle_threads(nrhs)), 0, st, j, nrhs, m, h1, h2, ldh, hn, H, cs, sn, g, bn, rtol,
                     act_step, kd, iters, scal, skip, bad);
  return hipGetLastError();
}

// y = -(R^{-1} g) over the kd[c] steps of the cycle (the rotated Hessenberg R is upper
// triangular), zero beyond and for columns inactive this cycle; the sign matches the
// subtracting gemv that forms V y.
__global__ void k_backsolve(int nrhs, int m, const double* __restrict__ H, const double* __restrict__ g,
                            const int* __restrict__ kd, const int* __restrict__ act_cycle, double* __restrict__ y,
                            int ldy) {
  const int c = threadIdx.x;
  if (c >= nrhs) return;
  double* yc = y + (int64_t)c * ldy;
  for (int i = 0; i < ldy; ++i) yc[i] = 0.0;
  if (!act_cycle[c]) return;
  const double* Hc = H + (int64_t)c * (m + 1) * m;
  const double* gc = g + (int64_t)c * (m + 1);
  const int k = kd[c];
  for (int i = k - 1; i >= 0; --i) {
    double t = gc[i];
    for (int l = i + 1; l < k; ++l) t -= Hc[i * m + l] * yc[l];
    yc[i] = Hc[i * m + i] != 0.0 ? t / Hc[i * m + i] : 0.0;
  }
  for (int i = 0; i < k; ++i) yc[i] = -yc[i];
}

hipError_t launch_backsolve(int nrhs, int m, const double* H, const double* g, const int* kd, const int* act_cycle,
                            double* y, int ldy, hipStream_t st) {
  if (nrhs > kCycleMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(cycle_threads(nrhs)), 0, st, nrhs, m, H, g, kd, act_cycle, y, ldy);
  return hipGetLastError();
}

// dst[r] = src[r] / s[r] (0 when s[r] == 0); skipped when *skip
__global__ void k_scale_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t N,
                             const double* __restrict__ s, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int r = blockIdx.y;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double f = s[r];
  dst[(int64_t)r * N + n] = f != 0.0 ? src[(int64_t)r * N + n] / f : 0.0;
}

hipError_t launch_scale_copy(double* dst, const double* src, int64_t N, int nrhs, const double* s, const int* skip,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, dst, src, N, s, skip);
  return hipGetLastError();
}

// fill with zeros (a kernel, so a captured graph holds no memset node)
__global__ void k_zero(double* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

__global__ void k_zero_u32(unsigned* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// unit-potential right-hand sides: grid (ceil(N / 256), m)
__global__ void k_unit_rhs(double* __restrict__ b, const int32_t* __restrict__ pcond, int64_t N) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (k < N) b[(int64_t)j * N + k] = pcond[k] == j ? 1.0 : 0.0;
}

hipError_t launch_unit_rhs(double* b, const int32_t* pcond, int64_t N, int m, hipStream_t st) {
  if (N <= 0 || m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_rhs, dim3((unsigned)((N + 255) / 256), m), dim3(256), 0, st, b, pcond, N);
  return hipGetLastError();
}

// x[r] += z[r] for the columns active this cycle; skipped when *skip
__global__ void k_add_active(double* __restrict__ x, const double* __restrict__ z, int64_t N,
                             const int* __restrict__ act, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int r = blockIdx.y;
  if (!act[r]) return;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  x[(int64_t)r * N + n] += z[(int64_t)r * N + n];
}

hipError_t launch_add_active(double* x, const double* z, int64_t N, int nrhs, const int* act, const int* skip,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_add_active, dim3((unsigned)((N + 255) / 256), nrhs), dim3(256), 0, st, x, z, N, act, skip);
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


// ------------------------------------------------------------------ fused Gram-Schmidt step
// Rows per partial sum of the three launches below: about 1024 workgroups per launch
// over all columns, at least one row per thread (so a small system still spreads over
// the chip instead of a few long per-thread loops).
// A chunk of w is staged in LDS, so chunks hold at most kCgsMaxRows rows (more chunks
// on larger systems).
constexpr int kCgsMaxRows = 4096;
static int64_t cgs_chunk(int64_t N, int nrhs) {
  int64_t c = (N * (int64_t)nrhs + 1023) / 1024;
  c = (c + kRedThreads - 1) / kRedThreads * kRedThreads;
  c = c < kCgsMaxRows ? c : kCgsMaxRows;
  return c > kRedThreads ? c : kRedThreads;
}
int64_t cgs_partial_size(int64_t N, int kmax, int nrhs) {
  return ((N + kRedThreads - 1) / kRedThreads) * (int64_t)nrhs * kmax;
}
// out[i] = sum over the chunk's rows t < rows of V_i[n0 + t] wl[t] for i < k, with the
// chunk of w in LDS (wl).  Wave v takes the basis vectors in groups of kCgsGroup:
// [G v, G v + G), then G nw further on, and so on; each lane adds the rows lane,
// lane + 128, ... and lane + 64, lane + 192, ... in two sums (two rows' loads of every
// vector in flight per iteration), then one wave reduction per vector (no cross-wave
// step).
constexpr int kCgsGroup = 4;
__device__ __forceinline__ void chunk_dots(const double* __restrict__ vr, int64_t ldv, int64_t n0, int rows, int k,
                                           const double* __restrict__ wl, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i0 = wv * kCgsGroup; i0 < k; i0 += nw * kCgsGroup) {
    double acc[kCgsGroup], acc2[kCgsGroup];
    const double* vq[kCgsGroup];
#pragma unroll
    for (int q = 0; q < kCgsGroup; ++q) {
      acc[q] = 0.0;
      acc2[q] = 0.0;
      vq[q] = vr + (int64_t)(i0 + q < k ? i0 + q : i0) * ldv + n0;   // (an absent vector reads a present one)
    }
    int t = lane;
    for (; t + 64 < rows; t += 128) {
      const double wt = wl[t], wt2 = wl[t + 64];
      double a[kCgsGroup], b[kCgsGroup];
#pragma unroll
      for (int q = 0; q < kCgsGroup; ++q) {
        a[q] = vq[q][t];
        b[q] = vq[q][t + 64];
      }
#pragma unroll
      for (int q = 0; q < kCgsGroup; ++q) {
        acc[q] += a[q] * wt;
        acc2[q] += b[q] * wt2;
      }
    }
    if (t < rows) {
      const double wt = wl[t];
#pragma unroll
      for (int q = 0; q < kCgsGroup; ++q) acc[q] += vq[q][t] * wt;
    }
#pragma unroll
    for (int q = 0; q < kCgsGroup; ++q) {
      const double sum = wave_sum(acc[q] + acc2[q]);
      if (lane == 0 && i0 + q < k) out[i0 + q] = sum;
    }
  }
}

// out[i * out_stride] = sum over c < nchunk of part[c * stride + i] for i < k: one thread
// per vector, chunks added in order (loads issued ahead of the adds)
__device__ __forceinline__ void sum_chunks_ordered(const double* __restrict__ part, int nchunk, int64_t stride, int k,
                                                   double* __restrict__ out, int64_t out_stride) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double sum = 0.0;
    int c = 0;
    for (; c + 4 <= nchunk; c += 4) {
      const double a0 = part[(int64_t)c * stride + i], a1 = part[(int64_t)(c + 1) * stride + i];
      const double a2 = part[(int64_t)(c + 2) * stride + i], a3 = part[(int64_t)(c + 3) * stride + i];
      sum += a0;
      sum += a1;
      sum += a2;
      sum += a3;
    }
    for (; c < nchunk; ++c) sum += part[(int64_t)c * stride + i];
    out[i * out_stride] = sum;
  }
}

// One Arnoldi step's classical Gram-Schmidt (applied twice) and norm in three launches:
//   A  h1 = V^T w                          (each block all k vectors on its row chunk;
//                                           the last block of each column adds the chunks)
//   B  w -= V h1; h2 = V^T w               (the last block of each column adds the chunks)
//   C  w -= V h2; |w|; Arnoldi/Givens step  (the last block of the launch does the step)
// "Last block" = the block whose increment of a device counter completes the count;
// it resets the counter for the next launch.  Partials are indexed by block and added
// in a fixed order, so results stay bitwise reproducible.

// true in every thread of the block that completes the count (after a device fence)
__device__ __forceinline__ bool last_block(unsigned* cnt, unsigned total, int* flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *flag = atomicAdd(cnt, 1u) == total - 1u ? 1 : 0;
  __syncthreads();
  const bool last = *flag != 0;
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) *cnt = 0u;
  }
  return last;
}

__global__ void __launch_bounds__(kRedThreads)
k_cgs_dot(const double* __restrict__ V, int64_t ldv, int64_t N, int64_t chunk_rows, int k,
          const double* __restrict__ w, int nrhs, double* __restrict__ h, int64_t ldh, double* __restrict__ partial,
          const int* __restrict__ active, unsigned* __restrict__ cnt) {
  __shared__ double wl[kCgsMaxRows];
  __shared__ int flag;
  const int chunk = blockIdx.x, r = blockIdx.y, nchunk = gridDim.x;
  if (active && !active[r]) return;   // every block of this column returns: its count stays 0
  const int64_t n0 = (int64_t)chunk * chunk_rows;
  const int rows = (int)((n0 + chunk_rows < N ? n0 + chunk_rows : N) - n0);
  const double* wr = w + (int64_t)r * N;
  for (int t = threadIdx.x; t < rows; t += blockDim.x) wl[t] = wr[n0 + t];
  __syncthreads();
  // all k basis vectors against this chunk of w
  chunk_dots(V + (int64_t)r * N, ldv, n0, rows, k, wl, partial + ((int64_t)chunk * nrhs + r) * k);
  if (last_block(cnt + r, (unsigned)nchunk, &flag))
    sum_chunks_ordered(partial + (int64_t)r * k, nchunk, (int64_t)nrhs * k, k, h + (int64_t)r * ldh, 1);
}

__global__ void __launch_bounds__(kRedThreads)
k_cgs_update_dot(const double* __restrict__ V, int64_t ldv, int64_t N, int64_t chunk_rows, int k,
                 const double* __restrict__ h1, int64_t ldh, double* __restrict__ w, int nrhs,
                 double* __restrict__ h2, double* __restrict__ partial, const int* __restrict__ active,
                 unsigned* __restrict__ cnt) {
  __shared__ double wl[kCgsMaxRows];
  __shared__ int flag;
  const int chunk = blockIdx.x, r = blockIdx.y, nchunk = gridDim.x;
  if (active && !active[r]) return;
  const int64_t n0 = (int64_t)chunk * chunk_rows;
  const int rows = (int)((n0 + chunk_rows < N ? n0 + chunk_rows : N) - n0);
  double* wr = w + (int64_t)r * N;
  const double* vr = V + (int64_t)r * N;
  const double* hr = h1 + (int64_t)r * ldh;
  // w -= V h1 on this chunk, kept in LDS for the dots
  for (int t = threadIdx.x; t < rows; t += blockDim.x) {
    const int64_t n = n0 + t;
    double acc = 0.0;
#pragma unroll 4
    for (int i = 0; i < k; ++i) acc += vr[(int64_t)i * ldv + n] * hr[i];
    const double wn = wr[n] - acc;
    wr[n] = wn;
    wl[t] = wn;
  }
  __syncthreads();
  chunk_dots(vr, ldv, n0, rows, k, wl, partial + ((int64_t)chunk * nrhs + r) * k);
  if (last_block(cnt + r, (unsigned)nchunk, &flag))
    sum_chunks_ordered(partial + (int64_t)r * k, nchunk, (int64_t)nrhs * k, k, h2 + (int64_t)r * ldh, 1);
}

__global__ void __launch_bounds__(kRedThreads)
k_cgs_update_norm_step(const double* __restrict__ V, int64_t ldv, int64_t N, int64_t chunk_rows, int k,
                       const double* __restrict__ h1,
                       const double* __restrict__ h2, int64_t ldh, double* __restrict__ w, int nrhs,
                       double* __restrict__ partial, unsigned* __restrict__ cnt, int j, int m, double* __restrict__ H,
                       double* __restrict__ cs, double* __restrict__ sn, double* __restrict__ g,
                       const double* __restrict__ bn, const double* __restrict__ rtolp, int* __restrict__ act_step,
                       int* __restrict__ kd, int* __restrict__ iters, double* __restrict__ scal,
                       int* __restrict__ skip, int* __restrict__ bad, double* __restrict__ nrm_out) {
  __shared__ double red[kRedThreads / 64];
  __shared__ int ired[kRedThreads];
  __shared__ int flag;
  const int chunk = blockIdx.x, r = blockIdx.y, nchunk = gridDim.x;
  if (act_step[r]) {
    const int64_t n0 = (int64_t)chunk * chunk_rows;
    const int64_t n1 = n0 + chunk_rows < N ? n0 + chunk_rows : N;
    double* wr = w + (int64_t)r * N;
    const double* vr = V + (int64_t)r * N;
    const double* hr = h2 + (int64_t)r * ldh;
    double sq = 0.0;
    for (int64_t n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
      double acc = 0.0;
#pragma unroll 4
      for (int i = 0; i < k; ++i) acc += vr[(int64_t)i * ldv + n] * hr[i];
      const double wn = wr[n] - acc;
      wr[n] = wn;
      sq += wn * wn;
    }
    const double t = wave_sum(sq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
      double u = 0.0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) u += red[q];
      partial[(int64_t)chunk * nrhs + r] = u;
    }
  }
  // every block counts (the step below also handles the inactive columns)
  if (!last_block(cnt, (unsigned)(nchunk * nrhs), &flag)) return;
  const int c = threadIdx.x;
  double hnc = 0.0;
  if (c < nrhs && act_step[c]) {
    double s2 = 0.0;
    for (int q = 0; q < nchunk; ++q) s2 += partial[(int64_t)q * nrhs + c];
    hnc = sqrt(s2);
    nrm_out[c] = hnc;
  }
  arnoldi_step(c, j, nrhs, m, h1, h2, (int)ldh, hnc, H, cs, sn, g, bn, *rtolp, act_step, kd, iters, scal, skip, bad,
               ired);
}

hipError_t launch_cgs_step(const double* V, int64_t ldv, int64_t N, int k, double* w, int nrhs, double* h1,
                           double* h2, int ldh, double* partial, unsigned* cnt, int j, int m, double* H, double* cs,
                           double* sn, double* g, const double* bn, const double* rtol, int* act_step, int* kd,
                           int* iters, double* scal, int* skip, int* bad, double* nrm_out, hipStream_t st) {
  if (nrhs > kRedThreads || k <= 0) return hipErrorInvalidValue;
  const int64_t rows = cgs_chunk(N, nrhs);
  const int nchunk = (int)((N + rows - 1) / rows);
  unsigned* cA = cnt;                                  // [nrhs]
  unsigned* cB = cnt + cgs_counter_size_a(k, nrhs);    // [nrhs]
  unsigned* cC = cB + nrhs;                            // [1]
  hipLaunchKernelGGL(k_cgs_dot, dim3(nchunk, nrhs), dim3(kRedThreads), 0, st, V, ldv, N, rows, k, w, nrhs, h1,
                     (int64_t)ldh, partial, act_step, cA);
  hipLaunchKernelGGL(k_cgs_update_dot, dim3(nchunk, nrhs), dim3(kRedThreads), 0, st, V, ldv, N, rows, k, h1,
                     (int64_t)ldh, w, nrhs, h2, partial, act_step, cB);
  hipLaunchKernelGGL(k_cgs_update_norm_step, dim3(nchunk, nrhs), dim3(kRedThreads), 0, st, V, ldv, N, rows, k, h1, h2,
                     (int64_t)ldh, w, nrhs, partial, cC, j, m, H, cs, sn, g, bn, rtol, act_step, kd, iters, scal,
                     skip, bad, nrm_out);
  return hipGetLastError();
}

int64_t cgs_counter_size_a(int kmax, int nrhs) { return (int64_t)((kmax + kDotBlk - 1) / kDotBlk) * nrhs; }
int64_t cgs_counter_size(int kmax, int nrhs) { return cgs_counter_size_a(kmax, nrhs) + nrhs + 1; }

}  // namespace vc
