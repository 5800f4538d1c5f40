// In-LDS mixed-radix FFT engine for gfx950 (wave64), templated on float / double.
//
// A workgroup transforms `ncol` independent lines of length L held in LDS as a
// [L][ncolp] tile (element i of line c at buf[i*ncolp + c], ncolp = ncol + pad).
// Each stage of radix R is a Stockham autosort step: butterfly i in [0, L/R) of a
// line reads x[i + q*L/R] (q < R), multiplies by w^(q*k*L/(pR)) (k = i mod p, p the
// product of the earlier radices, w = exp(-+2 pi i / L) from a table), does a
// radix-R DFT and writes y[(i-k)*R + k + q*p].  Stages alternate between two LDS
// tiles (read one, write the other), so each needs a single barrier and a thread holds
// one butterfly in registers at a time.  Consecutive threads take consecutive columns,
// which keeps LDS accesses on distinct banks.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vc {

template <typename T> struct C2 { T x, y; };

template <typename T> __host__ __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __host__ __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __host__ __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __host__ __device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.x, -a.y}; }
template <typename T> __host__ __device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (fwd) or +i (inv): s = -1 for -i, +1 for +i
template <typename T> __host__ __device__ __forceinline__ C2<T> cmuli(C2<T> a, T s) { return {-s * a.y, s * a.x}; }

// Radices supported by the engine.
constexpr int kMaxStages = 10;
struct AxisPlan {
  int L;
  int nst;
  int rad[kMaxStages];
};

// cos / sin of 2*pi*k/5 and 2*pi*k/7 (k = 1, 2, 3)
#define VC_C51 0.30901699437494742410
#define VC_C52 -0.80901699437494742410
#define VC_S51 0.95105651629515357212
#define VC_S52 0.58778525229247312917
#define VC_C71 0.62348980185873353053
#define VC_C72 -0.22252093395631440429
#define VC_C73 -0.90096886790241912624
#define VC_S71 0.78183148246802980871
#define VC_S72 0.97492791218182360702
#define VC_S73 0.43388373911755812048
#define VC_S31 0.86602540378443864676

// ---- composite radices: Cooley-Tukey in registers with compile-time twiddles ----
// cos / sin of 2 pi m / n evaluated at compile time (Taylor series after reduction to
// [-pi/4, pi/4] by octant symmetry), accurate to a few ulp in double.
constexpr double ct_pi = 3.14159265358979323846264338327950288;
constexpr double ct_sin_series(double x) {
  double t = x, s = x;
  for (int k = 1; k < 14; ++k) { t *= -x * x / ((2.0 * k) * (2.0 * k + 1.0)); s += t; }
  return s;
}
constexpr double ct_cos_series(double x) {
  double t = 1.0, s = 1.0;
  for (int k = 1; k < 14; ++k) { t *= -x * x / ((2.0 * k - 1.0) * (2.0 * k)); s += t; }
  return s;
}
// angle 2 pi m / n = (pi/4) * (8m/n): octant o = floor(8m/n), remainder in [0, pi/4)
constexpr double ct_cos2pi(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long o = (8 * m) / n;
  const double r = (ct_pi / 4.0) * ((double)(8 * m - o * n) / (double)n);   // [0, pi/4)
  const double c = ct_cos_series(r), sn = ct_sin_series(r);
  const double ca = ct_cos_series(ct_pi / 4.0 - r), sa = ct_sin_series(ct_pi / 4.0 - r);
  switch (o) {
    case 0: return c;            // r
    case 1: return sa;           // pi/2 - (pi/4 - r)
    case 2: return -sn;          // pi/2 + r
    case 3: return -ca;          // pi - (pi/4 - r)
    case 4: return -c;           // pi + r
    case 5: return -sa;
    case 6: return sn;
    default: return ca;
  }
}
// sin(2 pi m / n) = cos(2 pi (4m - n) / (4n))
constexpr double ct_sin2pi(long m, long n) { return ct_cos2pi(4 * m - n, 4 * n); }

template <typename T, int R> struct Dft;

// Every Dft<T,R>::run leaves output X[k] in register slot pos(k) (identity for prime
// radices; a compile-time digit permutation for composite ones, so no copy is needed).
// R = A * B, input index n = n1 + A n2, output index k = B k1 + k2:
//   X[B k1 + k2] = sum_n1 W_A^{n1 k1} W_R^{n1 k2} sum_n2 v[n1 + A n2] W_B^{n2 k2}
// Pass 1 (per n1) leaves Y[n1][k2] in slot n1 + A k2; pass 2 (per k2) leaves
// X[B k1 + k2] in slot k1 + A k2, each inner transform in its own permuted slots.
template <typename T, int A, int B> struct DftAB {
  static constexpr int R = A * B;
  static __host__ __device__ constexpr int pos(int k) {
    return Dft<T, A>::pos(k / B) + A * (k % B);
  }
  static __host__ __device__ __forceinline__ void run(C2<T>* v, T sg) {
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      C2<T> u[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) u[n2] = v[n1 + A * n2];
      Dft<T, B>::run(u, sg);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) {
        const C2<T> y = u[Dft<T, B>::pos(k2)];
        if ((n1 * k2) % R == 0) {
          v[n1 + A * k2] = y;
        } else {
          const T c = T(ct_cos2pi(n1 * k2, R)), s = T(ct_sin2pi(n1 * k2, R));
          // exp(sg * 2 pi i n1 k2 / R) = c + i sg s
          v[n1 + A * k2] = C2<T>{y.x * c - sg * s * y.y, y.y * c + sg * s * y.x};
        }
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      C2<T> u[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) u[n1] = v[n1 + A * k2];
      Dft<T, A>::run(u, sg);
#pragma unroll
      for (int s1 = 0; s1 < A; ++s1) v[s1 + A * k2] = u[s1];   // slot pos_A(k1) holds X[B k1 + k2]
    }
  }
};

// Radix-R DFT in registers.  sg = -1 forward (exp(-2 pi i qk/R)), +1 inverse.

template <typename T> struct Dft<T, 2> {
  static __host__ __device__ constexpr int pos(int k) { return k; }
  static __host__ __device__ __forceinline__ void run(C2<T>* v, T) {
    C2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};
template <typename T> struct Dft<T, 3> {
  static __host__ __device__ constexpr int pos(int k) { return k; }
  static __host__ __device__ __forceinline__ void run(C2<T>* v, T sg) {
    C2<T> s = cadd(v[1], v[2]);
    C2<T> d = csub(v[1], v[2]);
    C2<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
    C2<T> r = cmuli(d, sg * T(VC_S31));
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};
template <typename T> struct Dft<T, 4> {
  static __host__ __device__ constexpr int pos(int k) { return k; }
  static __host__ __device__ __forceinline__ void run(C2<T>* v, T sg) {
    C2<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C2<T> c = cadd(v[1], v[3]), d = cmuli(csub(v[1], v[3]), sg);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};
template <typename T> struct Dft<T, 5> {
  static __host__ __device__ constexpr int pos(int k) { return k; }
  static __host__ __device__ __forceinline__ void run(C2<T>* v, T sg) {
    C2<T> s1 = cadd(v[1], v[4]), d1 = csub(v[1], v[4]);
    C2<T> s2 = cadd(v[2], v[3]), d2 = csub(v[2], v[3]);
    C2<T> x0 = v[0];
    C2<T> a1 = {x0.x + T(VC_C51) * s1.x + T(VC_C52) * s2.x, x0.y + T(VC_C51) * s1.y + T(VC_C52) * s2.y};
    C2<T> a2 = {x0.x + T(VC_C52) * s1.x + T(VC_C51) * s2.x, x0.y + T(VC_C52) * s1.y + T(VC_C51) * s2.y};
    C2<T> b1 = {T(VC_S51) * d1.x + T(VC_S52) * d2.x, T(VC_S51) * d1.y + T(VC_S52) * d2.y};
    C2<T> b2 = {T(VC_S52) * d1.x - T(VC_S51) * d2.x, T(VC_S52) * d1.y - T(VC_S51) * d2.y};
    b1 = cmuli(b1, sg);
    b2 = cmuli(b2, sg);
    v[0] = {x0.x + s1.x + s2.x, x0.y + s1.y + s2.y};
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};
template <typename T> struct Dft<T, 7> {
  static __host__ __device__ constexpr int pos(int k) { return k; }
  static __host__ __device__ __forceinline__ void run(C2<T>* v, T sg) {
    C2<T> s1 = cadd(v[1], v[6]), d1 = csub(v[1], v[6]);
    C2<T> s2 = cadd(v[2], v[5]), d2 = csub(v[2], v[5]);
    C2<T> s3 = cadd(v[3], v[4]), d3 = csub(v[3], v[4]);
    C2<T> x0 = v[0];
    const T c1 = T(VC_C71), c2 = T(VC_C72), c3 = T(VC_C73);
    const T n1 = T(VC_S71), n2 = T(VC_S72), n3 = T(VC_S73);
    C2<T> a1 = {x0.x + c1 * s1.x + c2 * s2.x + c3 * s3.x, x0.y + c1 * s1.y + c2 * s2.y + c3 * s3.y};
    C2<T> a2 = {x0.x + c2 * s1.x + c3 * s2.x + c1 * s3.x, x0.y + c2 * s1.y + c3 * s2.y + c1 * s3.y};
    C2<T> a3 = {x0.x + c3 * s1.x + c1 * s2.x + c2 * s3.x, x0.y + c3 * s1.y + c1 * s2.y + c2 * s3.y};
    // sin(2 pi qk/7): k=1: (n1, n2, n3); k=2: (n2, -n3, -n1); k=3: (n3, -n1, n2)
    C2<T> b1 = {n1 * d1.x + n2 * d2.x + n3 * d3.x, n1 * d1.y + n2 * d2.y + n3 * d3.y};
    C2<T> b2 = {n2 * d1.x - n3 * d2.x - n1 * d3.x, n2 * d1.y - n3 * d2.y - n1 * d3.y};
    C2<T> b3 = {n3 * d1.x - n1 * d2.x + n2 * d3.x, n3 * d1.y - n1 * d2.y + n2 * d3.y};
    b1 = cmuli(b1, sg);
    b2 = cmuli(b2, sg);
    b3 = cmuli(b3, sg);
    v[0] = {x0.x + s1.x + s2.x + s3.x, x0.y + s1.y + s2.y + s3.y};
    v[1] = cadd(a1, b1);
    v[6] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[5] = csub(a2, b2);
    v[3] = cadd(a3, b3);
    v[4] = csub(a3, b3);
  }
};


template <typename T> struct Dft<T, 6> : DftAB<T, 2, 3> {};
template <typename T> struct Dft<T, 8> : DftAB<T, 2, 4> {};
template <typename T> struct Dft<T, 9> : DftAB<T, 3, 3> {};
template <typename T> struct Dft<T, 10> : DftAB<T, 2, 5> {};
template <typename T> struct Dft<T, 12> : DftAB<T, 3, 4> {};
template <typename T> struct Dft<T, 14> : DftAB<T, 2, 7> {};
template <typename T> struct Dft<T, 15> : DftAB<T, 3, 5> {};
template <typename T> struct Dft<T, 16> : DftAB<T, 4, 4> {};
template <typename T> struct Dft<T, 18> : DftAB<T, 2, 9> {};
template <typename T> struct Dft<T, 20> : DftAB<T, 4, 5> {};
template <typename T> struct Dft<T, 21> : DftAB<T, 3, 7> {};
template <typename T> struct Dft<T, 25> : DftAB<T, 5, 5> {};
template <typename T> struct Dft<T, 27> : DftAB<T, 3, 9> {};

// The scene a workgroup of a multi-scene launch works on: the last entry whose first
// linear workgroup blk0 is <= lin (blk0 increases along the table).
template <typename S>
__device__ __forceinline__ int find_scene(const S* __restrict__ tab, int n, int lin) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].blk0 <= lin) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Exact t / d for 0 <= t < 2^22 and d >= 1 given inv = 1.0f / d: (t + 1/2) / d is at
// least 1/(2d) away from an integer, and the float product errs by < t * 2^-23 / d.
__device__ __forceinline__ int fdiv(int t, float inv) { return (int)(((float)t + 0.5f) * inv); }

// One Stockham stage of radix R over ncol = 2^lgc lines, from src to dst (ping-pong:
// no thread reads what another writes in the same stage, so one barrier per stage and
// registers for a single butterfly at a time).
template <typename T, int R>
__device__ __forceinline__ void fft_stage(const C2<T>* __restrict__ src, C2<T>* __restrict__ dst,
                                          const C2<T>* __restrict__ tw, int L, int lgc, int ncolp, int p, float invp,
                                          T sg) {
  const int nthr = blockDim.x;
  const int LR = L / R;
  const int nb = LR << lgc;
  const int cmask = (1 << lgc) - 1;
  const int tstep_base = L / (p * R);
  for (int b = threadIdx.x; b < nb; b += nthr) {
    const int col = b & cmask, i = b >> lgc;
    C2<T> v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = src[(i + q * LR) * ncolp + col];
    const int ip = fdiv(i, invp);
    const int k = i - ip * p;
    if (p > 1) {
      const int ts = k * tstep_base;
#pragma unroll
      for (int q = 1; q < R; ++q) {
        C2<T> w = tw[q * ts];
        w.y *= -sg;  // table holds exp(-2 pi i t/L); conjugated for the inverse
        v[q] = cmul(v[q], w);
      }
    }
    Dft<T, R>::run(v, sg);
    const int j = ip * p * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) dst[(j + q * p) * ncolp + col] = v[Dft<T, R>::pos(q)];
  }
  __syncthreads();
}

// Full transform of 2^lgc lines held in buf (caller synchronizes before), using buf2 as
// the second ping-pong buffer; returns the buffer that holds the result.  Only
// radices <= MAXR are compiled in (bounds per-thread registers); the host plans each
// axis within that bound.
template <typename T, int MAXR>
__device__ C2<T>* lds_fft(C2<T>* __restrict__ buf, C2<T>* __restrict__ buf2, const C2<T>* __restrict__ tw,
                          const AxisPlan& pl, int lgc, int ncolp, bool inverse) {
  const T sg = inverse ? T(1) : T(-1);
  int p = 1;
  C2<T>* src = buf;
  C2<T>* dst = buf2;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = pl.rad[s];
    const float invp = 1.0f / (float)p;
#define VC_ST(RR) \
  case RR:        \
    if constexpr (RR <= MAXR) fft_stage<T, RR>(src, dst, tw, pl.L, lgc, ncolp, p, invp, sg); \
    break;
    switch (R) {
      VC_ST(2) VC_ST(3) VC_ST(4) VC_ST(5) VC_ST(6) VC_ST(7) VC_ST(8) VC_ST(9) VC_ST(10) VC_ST(12) VC_ST(14)
      VC_ST(15) VC_ST(16) VC_ST(18) VC_ST(20) VC_ST(21) VC_ST(25) VC_ST(27)
      default: break;
    }
#undef VC_ST
    p *= R;
    C2<T>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

}  // namespace vc
