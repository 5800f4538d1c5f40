// Setup kernels: the block Toeplitz tensors of App. B (Algorithm 1) embedded in
// circulants (Tab. VIII-X, generalised to any circulant length >= 2N+1), their FP64
// FFT, and the extraction of the real spectra that the product multiplies with.
//
// Panel integrals (dimensionless, voxel edge 1, Green's function 1/|r-r'|):
//   P(alpha,beta,d) = int_So int_Ss 1/|r-r'|                     eq. (5)
//   E(alpha,beta,d) = d/dd_alpha P(alpha,beta,d)                  eq. (6), along +alpha
// with d = centre(observer) - centre(source).  Touching squares use the exact 4-D
// corner sums (the route of App. A and its citation for eq. 5): for parallel squares
// sum_{a,b} w_a w_b F(d_p+a, d_q+b, d_alpha) with w = (1,-2,1) and
// d^2/du^2 d^2/dv^2 F = 1/r; for orthogonal squares (observer normal alpha, source
// normal beta, shared axis gamma) sum_{i,j} s_i s_j sum_c w_c G(d_alpha-1/2+i,
// d_beta-1/2+j, d_gamma+c) with d/du d/dv d^2/dw^2 G = 1/r; E uses dF/dw and dG/du.
// Separated squares use a 4-D Gauss-Legendre product rule whose order grows as the
// separation shrinks (error below ~1e-15 relative for every order used).
#include <hip/hip_runtime.h>
#include <math.h>

#include "fft_core.hpp"
#include "mvp_kernels.h"
#include "octant_kernels.h"

namespace vc {

__device__ __forceinline__ double Fpar(double u, double v, double w) {
  const double r = sqrt(u * u + v * v + w * w);
  const double ruw = sqrt(u * u + w * w), rvw = sqrt(v * v + w * w);
  double t = 0.0;
  if (ruw > 0.0) t += (u * u - w * w) * v * 0.5 * asinh(v / ruw);
  if (rvw > 0.0) t += (v * v - w * w) * u * 0.5 * asinh(u / rvw);
  if (w != 0.0) t -= u * v * w * atan(u * v / (w * r));
  return t - r * (u * u + v * v - 2.0 * w * w) * (1.0 / 6.0);
}

__device__ __forceinline__ double Fpar_w(double u, double v, double w) {
  const double r = sqrt(u * u + v * v + w * w);
  const double ruw = sqrt(u * u + w * w), rvw = sqrt(v * v + w * w);
  double t = w * r;
  if (w != 0.0) t -= u * v * atan(u * v / (w * r));
  if (rvw > 0.0) t -= u * w * asinh(u / rvw);
  if (ruw > 0.0) t -= v * w * asinh(v / ruw);
  return t;
}

__device__ __forceinline__ double Gorth(double u, double v, double w) {
  const double r = sqrt(u * u + v * v + w * w);
  const double rvw = sqrt(v * v + w * w), ruw = sqrt(u * u + w * w), ruv = sqrt(u * u + v * v);
  double t = 0.0;
  if (rvw > 0.0) t += (v * w * w * 0.5 - v * v * v * (1.0 / 6.0)) * asinh(u / rvw);
  if (ruw > 0.0) t += (u * w * w * 0.5 - u * u * u * (1.0 / 6.0)) * asinh(v / ruw);
  if (ruv > 0.0) t += u * v * w * asinh(w / ruv);
  if (w != 0.0) t -= w * w * w * (1.0 / 6.0) * atan(u * v / (w * r));
  if (v != 0.0) t -= v * v * w * 0.5 * atan(u * w / (v * r));
  if (u != 0.0) t -= u * u * w * 0.5 * atan(v * w / (u * r));
  return t - u * v * r * (1.0 / 3.0);
}

__device__ __forceinline__ double Gorth_u(double u, double v, double w) {
  const double r = sqrt(u * u + v * v + w * w);
  const double ruw = sqrt(u * u + w * w), ruv = sqrt(u * u + v * v);
  double t = -0.5 * v * r;
  if (ruw > 0.0) t += (w * w - u * u) * 0.5 * asinh(v / ruw);
  if (ruv > 0.0) t += v * w * asinh(w / ruv);
  if (u != 0.0) t -= u * w * atan(v * w / (u * r));
  return t;
}

// Exact 4-D integral for touching squares.
__device__ double kernel_exact(int alpha, int beta, const double d[3], int want) {
  const double w3[3] = {1.0, -2.0, 1.0};
  double s = 0.0;
  if (alpha == beta) {
    const int p = (alpha + 1) % 3, q = (alpha + 2) % 3;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const double u = d[p] + (a - 1), v = d[q] + (b - 1);
        s += w3[a] * w3[b] * (want == 0 ? Fpar(u, v, d[alpha]) : Fpar_w(u, v, d[alpha]));
      }
    return s;
  }
  const int g = 3 - alpha - beta;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const double sij = (i == j) ? 1.0 : -1.0;
      const double u = d[alpha] - 0.5 + i, v = d[beta] - 0.5 + j;
      for (int c = 0; c < 3; ++c) {
        const double w = d[g] + (c - 1);
        s += sij * w3[c] * (want == 0 ? Gorth(u, v, w) : Gorth_u(u, v, w));
      }
    }
  return s;
}

// Gauss-Legendre nodes/weights on [-1/2, 1/2]: gl[n*24 + i] nodes, gl[n*24 + 12 + i] weights.
__device__ double kernel_gauss(int alpha, int beta, const double d[3], int want, int n, const double* __restrict__ gl) {
  const int po = (alpha + 1) % 3, qo = (alpha + 2) % 3;
  const int ps = (beta + 1) % 3, qs = (beta + 2) % 3;
  const double* x = gl + n * 24;
  const double* w = gl + n * 24 + 12;
  double acc = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double o[3] = {d[0], d[1], d[2]};
      o[po] += x[a];
      o[qo] += x[b];
      const double wo = w[a] * w[b];
      double part = 0.0;
      for (int c = 0; c < n; ++c)
        for (int e = 0; e < n; ++e) {
          double t[3] = {o[0], o[1], o[2]};
          t[ps] -= x[c];
          t[qs] -= x[e];
          const double r2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
          const double ir = 1.0 / sqrt(r2);
          const double f = want == 0 ? ir : -t[alpha] * ir * ir * ir;
          part += w[c] * w[e] * f;
        }
      acc += wo * part;
    }
  return acc;
}

__device__ double panel_kernel(int alpha, int beta, const double d[3], int want, const double* __restrict__ gl) {
  // Euclidean separation of the two closed squares
  double s2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double ext = (a == alpha ? 0.0 : 0.5) + (a == beta ? 0.0 : 0.5);
    const double g = fabs(d[a]) - ext;
    if (g > 0.0) s2 += g * g;
  }
  if (want == 1 && alpha == beta && d[alpha] == 0.0) return 0.0;  // coplanar field integral
  if (s2 == 0.0) return kernel_exact(alpha, beta, d, want);
  const double sep = sqrt(s2);
  int n;
  if (sep < 2.0) n = 10;
  else if (sep < 3.0) n = 8;
  else if (sep < 5.0) n = 7;
  else if (sep < 10.0) n = 6;
  else if (sep < 20.0) n = 5;
  else if (sep < 100.0) n = 4;
  else n = 3;
  return kernel_gauss(alpha, beta, d, want, n, gl);
}

__global__ void k_fill_circulant(double* __restrict__ C, FillArgs a, const double* __restrict__ gl) {
  const int64_t total = (int64_t)a.Mx * a.My * a.Mz;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int jz = (int)(id % a.Mz);
  const int jy = (int)((id / a.Mz) % a.My);
  const int jx = (int)(id / ((int64_t)a.Mz * a.My));
  const int j[3] = {jx, jy, jz};
  const int M[3] = {a.Mx, a.My, a.Mz};
  double d[3];
  for (int ax = 0; ax < 3; ++ax) {
    int l;
    if (j[ax] <= a.no[ax] - 1) l = j[ax];
    else if (j[ax] >= M[ax] - (a.ns[ax] - 1)) l = j[ax] - M[ax];
    else { C[id] = 0.0; return; }
    d[ax] = (double)l;
  }
  if (a.alpha != a.beta) {
    d[a.alpha] -= 0.5;
    d[a.beta] += 0.5;
  }
  C[id] = a.scale * panel_kernel(a.alpha, a.beta, d, a.want, gl);
}

hipError_t launch_fill_circulant(double* C, const FillArgs& a, const double* gl, hipStream_t st) {
  const int64_t total = (int64_t)a.Mx * a.My * a.Mz;
  const int nt = 256;
  hipLaunchKernelGGL(k_fill_circulant, dim3((unsigned)((total + nt - 1) / nt)), dim3(nt), 0, st, C, a, gl);
  return hipGetLastError();
}

// Toeplitz octant of one pair (App. B): the kernel at the non-negative centre offsets
// d_a = t_a + h_a, t_a = 0..D_a-1, with h_a = 1/2 on the two normal axes of an
// orthogonal pair (their panel centres sit half a voxel apart there) and 0 elsewhere.
// Every lag of a grid with n_a <= D_a - 1 voxels maps onto one of these offsets.
__global__ void k_fill_octant(double* __restrict__ T, OctArgs a, const double* __restrict__ gl) {
  const int64_t total = (int64_t)a.D[0] * a.D[1] * a.D[2];
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  double d[3];
  d[2] = (double)(id % a.D[2]);
  d[1] = (double)((id / a.D[2]) % a.D[1]);
  d[0] = (double)(id / ((int64_t)a.D[2] * a.D[1]));
  if (a.alpha != a.beta) {
    d[a.alpha] += 0.5;
    d[a.beta] += 0.5;
  }
  T[id] = panel_kernel(a.alpha, a.beta, d, a.want, gl);
}

hipError_t launch_fill_octant(double* T, const OctArgs& a, const double* gl, hipStream_t st) {
  const int64_t total = (int64_t)a.D[0] * a.D[1] * a.D[2];
  if (total == 0) return hipSuccess;
  const int nt = 256;
  hipLaunchKernelGGL(k_fill_octant, dim3((unsigned)((total + nt - 1) / nt)), dim3(nt), 0, st, T, a, gl);
  return hipGetLastError();
}

// Circulant embedding of one pair read from its octant T (D0 x D1 x D2): the lags of
// k_fill_circulant, each taken at |d| (the kernel of eq. 5 is even in every offset
// component; its derivative of eq. 6 is odd in d_alpha and even in the other two).
// Offsets beyond the octant (the host sizes it so that none occurs) are written as NaN.
__global__ void k_embed_octant(double* __restrict__ C, const double* __restrict__ T, FillArgs a, OctArgs o) {
  const int64_t total = (int64_t)a.Mx * a.My * a.Mz;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int j[3] = {(int)(id / ((int64_t)a.Mz * a.My)), (int)((id / a.Mz) % a.My), (int)(id % a.Mz)};
  const int M[3] = {a.Mx, a.My, a.Mz};
  int t[3];
  bool neg_alpha = false;
  for (int ax = 0; ax < 3; ++ax) {
    int l;
    if (j[ax] <= a.no[ax] - 1) l = j[ax];
    else if (j[ax] >= M[ax] - (a.ns[ax] - 1)) l = j[ax] - M[ax];
    else { C[id] = 0.0; return; }
    // d = l - 1/2 on the observer normal, l + 1/2 on the source normal of an
    // orthogonal pair, l elsewhere; t = |d| - h
    int ta;
    bool neg;
    if (a.alpha != a.beta && ax == a.alpha) { neg = l <= 0; ta = neg ? -l : l - 1; }
    else if (a.alpha != a.beta && ax == a.beta) { neg = l < 0; ta = neg ? -l - 1 : l; }
    else { neg = l < 0; ta = neg ? -l : l; }
    if (ax == a.alpha) neg_alpha = neg;
    if (ta >= o.D[ax]) { C[id] = __builtin_nan(""); return; }
    t[ax] = ta;
  }
  const double v = T[((int64_t)t[0] * o.D[1] + t[1]) * o.D[2] + t[2]];
  C[id] = a.scale * ((a.want == 1 && neg_alpha) ? -v : v);
}

hipError_t launch_embed_octant(double* C, const double* T, const FillArgs& a, const OctArgs& o, hipStream_t st) {
  const int64_t total = (int64_t)a.Mx * a.My * a.Mz;
  const int nt = 256;
  hipLaunchKernelGGL(k_embed_octant, dim3((unsigned)((total + nt - 1) / nt)), dim3(nt), 0, st, C, T, a, o);
  return hipGetLastError();
}

__global__ void k_kernel_table(const double* __restrict__ dd, int n, int alpha, int beta, int want,
                               double* __restrict__ out, const double* __restrict__ gl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d[3] = {dd[3 * i], dd[3 * i + 1], dd[3 * i + 2]};
  out[i] = panel_kernel(alpha, beta, d, want, gl);
}

hipError_t launch_kernel_table(const double* d, int n, int alpha, int beta, int want, double* out, const double* gl,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kernel_table, dim3((n + 127) / 128), dim3(128), 0, st, d, n, alpha, beta, want, out, gl);
  return hipGetLastError();
}

// Real-to-complex along z of dense real lines, two lines per complex transform.
__global__ void __launch_bounds__(1024)
k_zr2c_dense(const double* __restrict__ in, C2<double>* __restrict__ out, int nlines, int H, AxisPlan pl,
             const C2<double>* __restrict__ twg, int ncol) {
  extern __shared__ char smem_raw[];
  const int L = pl.L, ncolp = ncol + 1;
  int lgc = 0;
  while ((1 << (lgc + 1)) <= ncol) ++lgc;
  C2<double>* tw = reinterpret_cast<C2<double>*>(smem_raw);
  C2<double>* buf = tw + L;
  C2<double>* buf2 = buf + L * ncolp;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int t = tid; t < L; t += nthr) tw[t] = twg[t];
  const int pair0 = blockIdx.x * ncol;
  for (int e = tid; e < L * ncol; e += nthr) {
    const int c = e / L, z = e - c * L;
    const int la = 2 * (pair0 + c), lb = la + 1;
    C2<double> v = {0.0, 0.0};
    if (la < nlines) v.x = in[(int64_t)la * L + z];
    if (lb < nlines) v.y = in[(int64_t)lb * L + z];
    buf[z * ncolp + c] = v;
  }
  __syncthreads();
  const C2<double>* res = lds_fft<double, Tune<double>::maxr>(buf, buf2, tw, pl, lgc, ncolp, false);
  for (int e = tid; e < H * ncol; e += nthr) {
    const int c = e / H, k = e - c * H;
    const int la = 2 * (pair0 + c), lb = la + 1;
    const C2<double> Z = res[k * ncolp + c];
    const C2<double> Zc = cconj(res[((L - k) % L) * ncolp + c]);
    if (la < nlines) out[(int64_t)la * H + k] = C2<double>{0.5 * (Z.x + Zc.x), 0.5 * (Z.y + Zc.y)};
    if (lb < nlines) out[(int64_t)lb * H + k] = C2<double>{0.5 * (Z.y - Zc.y), -0.5 * (Z.x - Zc.x)};
  }
}

hipError_t launch_zr2c_dense(const double* in, void* out, int nlines, int H, const AxisPlan& pl, const void* tw,
                             int ncol, int nthr, hipStream_t st) {
  const int npairs = (nlines + 1) / 2;
  const size_t lds = sizeof(C2<double>) * ((size_t)pl.L + 2 * (size_t)pl.L * (ncol + 1));
  if (lds > kLdsBudget) {   // a transform too long for the default budget declares its LDS
    if (lds > lds_ext_budget()) return hipErrorInvalidValue;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_zr2c_dense),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_zr2c_dense, dim3((npairs + ncol - 1) / ncol), dim3(nthr), lds, st, in, (C2<double>*)out,
                     nlines, H, pl, (const C2<double>*)tw, ncol);
  return hipGetLastError();
}

// Spectrum S of pair (alpha,beta) -> real tensor R on the non-negative octant:
//   P, alpha == beta : S = R
//   P, alpha != beta : S = exp(-i pi k_alpha/M_alpha) exp(+i pi k_beta/M_beta) R
//   E               : S = i * (same phase, none when alpha == beta) * R
// The discarded component (which must vanish) is reduced into *resid (max |.|).
__global__ void k_extract(const C2<double>* __restrict__ spec, double* __restrict__ R64, float* __restrict__ R32,
                          ExtractArgs a, unsigned long long* __restrict__ resid) {
  const int64_t total = (int64_t)a.Hy * a.H * a.Hx;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double bad = 0.0;
  if (id < total) {
    // stored layout [kx < Hx][ky < Hy][kz < H], kz contiguous
    const int kz = (int)(id % a.H);
    const int ky = (int)((id / a.H) % a.Hy);
    const int kx = (int)(id / ((int64_t)a.Hy * a.H));
    const C2<double> S = spec[((int64_t)kx * a.My + ky) * a.H + kz];
    const int k[3] = {kx, ky, kz};
    const int M[3] = {a.Mx, a.My, a.Mz};
    double th = 0.0;
    if (a.alpha != a.beta) th = -M_PI * k[a.alpha] / M[a.alpha] + M_PI * k[a.beta] / M[a.beta];
    double sn, cs;
    sincos(th, &sn, &cs);
    // S * exp(-i th)
    const double re = S.x * cs + S.y * sn;
    const double im = S.y * cs - S.x * sn;
    const double val = (a.kind == 2) ? im : re;
    bad = fabs((a.kind == 2) ? re : im);
    if (R64) R64[a.pair_off + id] = val;
    if (R32) R32[a.pair_off + id] = (float)val;
  }
  // block max of the discarded part
  __shared__ double red[256];
  red[threadIdx.x] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(resid, (unsigned long long)__double_as_longlong(red[0]));
}

hipError_t launch_extract(const void* spec, double* R64, float* R32, const ExtractArgs& a, double* resid,
                          hipStream_t st) {
  const int64_t total = (int64_t)a.Hy * a.H * a.Hx;
  hipLaunchKernelGGL(k_extract, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, (const C2<double>*)spec,
                     R64, R32, a, (unsigned long long*)resid);
  return hipGetLastError();
}

}  // namespace vc
