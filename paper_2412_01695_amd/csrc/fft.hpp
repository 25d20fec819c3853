// In-register mixed-radix (2, 3, 4, 5) and prime-factor complex FFT for one
// thread.
//
// The 3D transform of the paper (Sec. 4, Eqs. zfft, yfft, xfft, fwFFT) is a
// sequence of 1D transforms of length N_i along each axis.  Here every 1D
// line is held by one work-item in registers and transformed with a fully
// unrolled recursion -- Good-Thomas prime-factor splits where the length has
// coprime factors, decimation-in-time Cooley-Tukey otherwise -- whose every
// index and twiddle factor is a compile-time constant, so the data never
// leaves the VGPRs and every twiddle is an immediate/SGPR operand.  Lines are exchanged
// between axes through LDS by the calling kernel.
//
//   SIGN = +1 : X[l] = sum_m x[m] exp(+2 pi i l m / N)   (inverse, unnormalised)
//   SIGN = -1 : X[m] = sum_l x[l] exp(-2 pi i l m / N)   (forward, 1/N applied elsewhere)
//
// Twiddles come from a constexpr sine/cosine (octant reduction on the exact
// rational angle, then a Horner-evaluated Taylor series on [0, pi/4]); a host
// test compares them with the C library.  Inputs that are known zeros (the
// plane-wave sphere only fills the first W of N entries) are written as
// literal zeros: built with -fno-signed-zeros the compiler folds every
// operation on them away, which prunes the first radix stages for free.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

namespace mkpw {

template <class T>
struct cplx {
  T x, y;
};

template <class T>
__host__ __device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T>
__host__ __device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T>
__host__ __device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
template <class T>
__host__ __device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <class T>
__host__ __device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }

__host__ __device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
// c + a b as four fused multiply-adds (written out: contraction of the
// expression form leaves a product, a fused multiply-add and an add per part)
template <class T>
__host__ __device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> c) {
  return {fma_t(-a.y, b.y, fma_t(a.x, b.x, c.x)), fma_t(a.y, b.x, fma_t(a.x, b.y, c.y))};
}

// ---------------------------------------------------------------- compile-time loops

template <class F, int... Is>
__host__ __device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------- compile-time trigonometry

namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;

// sin(x), cos(x) for 0 <= x <= pi/4 by Taylor series, Horner form, 13 terms
constexpr double sin_small(double x) {
  double x2 = x * x, r = 1.0;
  for (int n = 25; n >= 3; n -= 2) r = 1.0 - x2 / double(n * (n - 1)) * r;
  return x * r;
}
constexpr double cos_small(double x) {
  double x2 = x * x, r = 1.0;
  for (int n = 24; n >= 2; n -= 2) r = 1.0 - x2 / double(n * (n - 1)) * r;
  return r;
}

constexpr double cos2pi(long p, long q);
// sin(2 pi p / q) for any integers, q > 0
constexpr double sin2pi(long p, long q) {
  p %= q;
  if (p < 0) p += q;
  if (p == 0 || 2 * p == q) return 0.0;
  if (2 * p > q) return -sin2pi(q - p, q);           // sin(2pi - a) = -sin a
  if (4 * p > q) return sin2pi(q - 2 * p, 2 * q);    // sin(pi - a) = sin a   (p/q > 1/4)
  if (4 * p == q) return 1.0;
  if (8 * p > q) return cos2pi(q - 4 * p, 4 * q);    // sin a = cos(pi/2 - a)
  return sin_small(2.0 * kPi * double(p) / double(q));
}
constexpr double cos2pi(long p, long q) {
  p %= q;
  if (p < 0) p += q;
  if (p == 0) return 1.0;
  if (2 * p == q) return -1.0;
  if (4 * p == q || 4 * p == 3 * q) return 0.0;
  if (2 * p > q) return cos2pi(q - p, q);            // cos(2pi - a) = cos a
  if (4 * p > q) return -cos2pi(q - 2 * p, 2 * q);   // cos(pi - a) = -cos a
  if (8 * p > q) return sin2pi(q - 4 * p, 4 * q);    // cos a = sin(pi/2 - a)
  return cos_small(2.0 * kPi * double(p) / double(q));
}
}  // namespace ct

// multiply v by exp(SIGN * 2 pi i J / N), trivial angles special-cased at compile time
template <class T, long J, long N, int SIGN>
__device__ __forceinline__ cplx<T> twiddle(cplx<T> v) {
  constexpr long j = ((J % N) + N) % N;
  if constexpr (j == 0) {
    return v;
  } else if constexpr (2 * j == N) {
    return {-v.x, -v.y};
  } else if constexpr (4 * j == N) {  // * (SIGN i)
    return SIGN > 0 ? cplx<T>{-v.y, v.x} : cplx<T>{v.y, -v.x};
  } else if constexpr (4 * j == 3 * N) {  // * (-SIGN i)
    return SIGN > 0 ? cplx<T>{v.y, -v.x} : cplx<T>{-v.y, v.x};
  } else {
    constexpr T c = T(ct::cos2pi(j, N));
    constexpr T s = T(SIGN * ct::sin2pi(j, N));
    return {v.x * c - v.y * s, v.x * s + v.y * c};
  }
}

// ---------------------------------------------------------------- butterflies (length R DFTs)

template <class T, int SIGN>
__device__ __forceinline__ void bfly2(cplx<T> (&a)[2]) {
  cplx<T> t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <class T, int SIGN>
__device__ __forceinline__ void bfly4(cplx<T> (&a)[4]) {
  cplx<T> s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
  cplx<T> s13 = cadd(a[1], a[3]), d13 = csub(a[1], a[3]);
  // SIGN i * d13
  cplx<T> r = SIGN > 0 ? cplx<T>{-d13.y, d13.x} : cplx<T>{d13.y, -d13.x};
  a[0] = cadd(s02, s13);
  a[2] = csub(s02, s13);
  a[1] = cadd(d02, r);
  a[3] = csub(d02, r);
}

// odd R: X_k = a0 + sum_j [(a_j + a_{R-j}) cos(2pi jk/R) + i SIGN (a_j - a_{R-j}) sin(2pi jk/R)]
template <class T, int R, int SIGN>
__device__ __forceinline__ void bfly_odd(cplx<T> (&a)[R]) {
  constexpr int H = (R - 1) / 2;
  cplx<T> s[H + 1], d[H + 1];
  sfor<H>([&](auto jj) {
    constexpr int j = decltype(jj)::value + 1;
    s[j] = cadd(a[j], a[R - j]);
    d[j] = csub(a[j], a[R - j]);
  });
  cplx<T> a0 = a[0];
  cplx<T> x0 = a0;
  sfor<H>([&](auto jj) { x0 = cadd(x0, s[decltype(jj)::value + 1]); });
  sfor<H>([&](auto kk) {
    constexpr int k = decltype(kk)::value + 1;
    cplx<T> A = a0;
    sfor<H>([&](auto jj) {
      constexpr int j = decltype(jj)::value + 1;
      constexpr T c = T(ct::cos2pi(long(j) * k, R));
      A.x += s[j].x * c;
      A.y += s[j].y * c;
    });
    // X_k = A + i B, X_{R-k} = A - i B with B = SIGN sum_j d_j sin(2 pi jk/R),
    // each output accumulated from A so that every product fuses into an FMA
    cplx<T> P = A, Q = A;
    sfor<H>([&](auto jj) {
      constexpr int j = decltype(jj)::value + 1;
      constexpr T sn = T(SIGN * ct::sin2pi(long(j) * k, R));
      P.x -= d[j].y * sn;
      P.y += d[j].x * sn;
      Q.x += d[j].y * sn;
      Q.y -= d[j].x * sn;
    });
    a[k] = P;
    a[R - k] = Q;
  });
  a[0] = x0;
}

template <class T, int N, int SIGN>
__device__ __forceinline__ void fft(cplx<T> (&x)[N]);

// a radix-R butterfly is an R-point DFT: 2 and 4 written out, odd primes by
// the symmetric form above, composite radices (8) by the recursion
template <class T, int R, int SIGN>
__device__ __forceinline__ void bfly(cplx<T> (&a)[R]) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    bfly2<T, SIGN>(a);
  } else if constexpr (R == 4) {
    bfly4<T, SIGN>(a);
  } else if constexpr (R == 3 || R == 5 || R == 7) {
    bfly_odd<T, R, SIGN>(a);
  } else {
    fft<T, R, SIGN>(a);
  }
}

// First radix of a Cooley-Tukey (decimation in time) split, for lengths that
// have no coprime factorisation (powers of 2 and 3) and for the odd primes.
template <int N>
constexpr int pick_radix() {
  if constexpr (N == 1 || N == 2 || N == 3 || N == 4 || N == 5) return N;
  else if constexpr (N % 4 == 0) return 4;
  else if constexpr (N % 2 == 0) return 2;
  else if constexpr (N % 3 == 0) return 3;
  else if constexpr (N % 5 == 0) return 5;
  else return N;  // prime: direct (odd) butterfly
}

// First factor N1 of a prime-factor (Good-Thomas) split N = N1 N2 with N1, N2
// coprime, 0 for none.  Inverse transforms here always start from a window of
// nonzero inputs and forward ones always end in a window of wanted outputs;
// the split that lets the most operations on the zeros (or on the unwanted
// outputs) fold away differs with the direction, and was chosen by counting
// the generated FP64 instructions (e.g. 24 points: 196 for 10 -> 24 inverse,
// 228 for 24 -> 10 forward, against 224 and 256 with radix-4 Cooley-Tukey).
template <int N, int SIGN>
constexpr int pfa_first() {
  if constexpr (N == 6 || N == 10 || N == 18) return 2;
  else if constexpr (N == 12) return 3;
  else if constexpr (N == 15) return SIGN > 0 ? 5 : 3;
  else if constexpr (N == 20) return SIGN > 0 ? 5 : 4;
  else if constexpr (N == 24) return SIGN > 0 ? 8 : 3;
  else if constexpr (N == 30) return SIGN > 0 ? 15 : 2;
  else if constexpr (N == 36) return 4;
  else return 0;
}

template <int A, int M>
constexpr int inv_mod() {  // A^-1 mod M for coprime A, M
  for (int q = 1; q < M; ++q)
    if ((A * q) % M == 1) return q;
  return 1;
}

// Prime-factor DFT: with n = (n1 N2 + n2 N1) mod N on the input and
// k = (k1 N2 q2 + k2 N1 q1) mod N on the output (q2 = N2^-1 mod N1,
// q1 = N1^-1 mod N2), the length-N DFT is a 2D N1 x N2 DFT with no twiddle
// factors.  All the index maps are compile-time register renamings.
template <class T, int N, int SIGN>
__device__ __forceinline__ void fft_pfa(cplx<T> (&x)[N]) {
  constexpr int N1 = pfa_first<N, SIGN>(), N2 = N / N1;
  constexpr int Q2 = inv_mod<N2 % N1, N1>(), Q1 = inv_mod<N1 % N2, N2>();
  cplx<T> a[N2][N1];
  sfor<N1>([&](auto i1) {
    sfor<N2>([&](auto i2) {
      constexpr int n1 = decltype(i1)::value, n2 = decltype(i2)::value;
      a[n2][n1] = x[(n1 * N2 + n2 * N1) % N];
    });
  });
  sfor<N2>([&](auto i2) { fft<T, N1, SIGN>(a[decltype(i2)::value]); });
  cplx<T> b[N1][N2];
  sfor<N1>([&](auto i1) {
    sfor<N2>([&](auto i2) { b[decltype(i1)::value][decltype(i2)::value] = a[decltype(i2)::value][decltype(i1)::value]; });
  });
  sfor<N1>([&](auto i1) { fft<T, N2, SIGN>(b[decltype(i1)::value]); });
  sfor<N1>([&](auto i1) {
    sfor<N2>([&](auto i2) {
      constexpr int k1 = decltype(i1)::value, k2 = decltype(i2)::value;
      x[(k1 * N2 * Q2 + k2 * N1 * Q1) % N] = b[k1][k2];
    });
  });
}

// In-place length-N DFT of x (decimation in time, fully unrolled).
template <class T, int N, int SIGN>
__device__ __forceinline__ void fft(cplx<T> (&x)[N]) {
  constexpr int R = pick_radix<N>();
  if constexpr (pfa_first<N, SIGN>() > 1) {
    fft_pfa<T, N, SIGN>(x);
  } else if constexpr (R == N) {
    bfly<T, N, SIGN>(x);
  } else {
    constexpr int M = N / R;
    cplx<T> y[R][M];
    sfor<R>([&](auto r) { sfor<M>([&](auto m) { y[r][m] = x[R * decltype(m)::value + decltype(r)::value]; }); });
    sfor<R>([&](auto r) { fft<T, M, SIGN>(y[r]); });
    sfor<M>([&](auto k1) {
      constexpr int K1 = decltype(k1)::value;
      cplx<T> t[R];
      sfor<R>([&](auto r) {
        constexpr int RR = decltype(r)::value;
        t[RR] = twiddle<T, long(RR) * K1, N, SIGN>(y[RR][K1]);
      });
      bfly<T, R, SIGN>(t);
      sfor<R>([&](auto k2) { x[K1 + M * decltype(k2)::value] = t[decltype(k2)::value]; });
    });
  }
}

// ---------------------------------------------------------------- lane-pair transforms
//
// A length-N line (N = 2M) shared by two adjacent lanes of a wavefront:
//  * pair_inverse: one radix-2 decimation-in-frequency step, after which lane p
//    holds h[j] = X[2j + p] (j < M) -- X[2j] is the M-point DFT of
//    x[m] + x[m+M], X[2j+1] that of (x[m] - x[m+M]) w^m -- so the two lanes
//    need no exchange;
//  * pair_forward: lane r holds u[j] = x[2j + r] (exactly what pair_inverse
//    leaves), each lane takes the M-point DFT, and the radix-2
//    decimation-in-time combination Y[k] = U0[k] + w^k U1[k],
//    Y[k + M] = U0[k] - w^k U1[k] needs one swap of the lanes' values
//    (DPP quad permutation 1,0,3,2).
// Both lanes run the same instructions; lane-dependent signs and twiddles are
// selected per lane.

__device__ __forceinline__ float swap_pair(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double swap_pair(double v) {
  int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// lane 1 multiplies by exp(SIGN 2 pi i J / N), lane 0 keeps v
template <class T, long J, long N, int SIGN>
__device__ __forceinline__ cplx<T> twiddle_odd(cplx<T> v, int p) {
  if constexpr (((J % N) + N) % N == 0) {
    return v;
  } else {
    cplx<T> t = twiddle<T, J, N, SIGN>(v);
    return p ? t : v;
  }
}

template <class T, int N, int WI, int SIGN, class LD>
__device__ __forceinline__ void pair_inverse(cplx<T> (&h)[N / 2], int p, LD&& ld) {
  constexpr int M = N / 2;
  const T sg = p ? T(-1) : T(1);
  sfor<M>([&](auto mm) {
    constexpr int m = decltype(mm)::value;
    if constexpr (m < WI) {
      cplx<T> a = ld(m);
      if constexpr (m + M < WI) {
        cplx<T> b = ld(m + M);
        a.x += sg * b.x;
        a.y += sg * b.y;
      }
      h[m] = twiddle_odd<T, m, N, SIGN>(a, p);
    } else {
      h[m] = {T(0), T(0)};
    }
  });
  fft<T, M, SIGN>(h);
}

// on return u[k] (k < min(M, WO)) is Y[k] on lane 0 and Y[k + M] on lane 1
template <class T, int N, int WO, int SIGN>
__device__ __forceinline__ void pair_forward(cplx<T> (&u)[N / 2], int r) {
  constexpr int M = N / 2;
  constexpr int K = WO < M ? WO : M;
  fft<T, M, SIGN>(u);
  const T sg = r ? T(-1) : T(1);
  sfor<K>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    cplx<T> own = twiddle_odd<T, k, N, SIGN>(u[k], r);
    cplx<T> oth = {swap_pair(own.x), swap_pair(own.y)};
    u[k] = {oth.x + sg * own.x, oth.y + sg * own.y};
  });
}

}  // namespace mkpw
