// Shared device helpers: complex type, compile-time trigonometry, register-resident DFTs.
//
// The register DFTs are the building block of every FFT pass: a length-P transform is split
// as P = P1 * P2 (Cooley-Tukey, one LDS exchange between the two factors) and each factor
// runs entirely in one lane's registers.  All twiddles inside a factor are compile-time
// constants; multiplications by 0 and +-1 fold away after unrolling.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ace {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T r, i;
};

template <typename T>
__host__ __device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__host__ __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) {
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ C2<T> cmul_conjb(C2<T> a, C2<T> b) {
  return {a.r * b.r + a.i * b.i, a.i * b.r - a.r * b.i};
}
template <typename T>
__host__ __device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.r * s, a.i * s}; }

// ---------------------------------------------------------------------------------------
// Compile-time cos / sin of 2*pi*m/n with exact quadrant / octant reduction (integer
// arithmetic), then a Taylor series on |x| <= pi/4.  Accurate to about 1 ulp in double.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double sin_series(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

struct CosSin {
  double c, s;
};

// cos and sin of 2*pi*m/n for integers m (any sign), n > 0.
constexpr CosSin cossin_2pi(long long m, long long n) {
  long long r = m % n;
  if (r < 0) r += n;
  // angle = 2*pi*r/n = (pi/2) * (4r/n): quadrant q, remainder rr in units of pi/(2n)
  long long q = (4 * r) / n;
  long long rr = 4 * r - q * n;  // angle within quadrant = (pi/2) * rr / n
  double c0 = 0, s0 = 0;
  if (2 * rr <= n) {
    double x = kPi * double(rr) / double(2 * n);
    c0 = cos_series(x);
    s0 = sin_series(x);
  } else {
    double x = kPi * double(n - rr) / double(2 * n);
    c0 = sin_series(x);
    s0 = cos_series(x);
  }
  if (q == 0) return {c0, s0};
  if (q == 1) return {-s0, c0};
  if (q == 2) return {-c0, -s0};
  return {s0, -c0};
}

template <int N>
struct TwTable {
  double c[N];
  double s[N];
  constexpr TwTable() : c(), s() {
    for (int m = 0; m < N; ++m) {
      CosSin v = cossin_2pi(m, N);
      c[m] = v.c;
      s[m] = v.s;
    }
  }
};
template <int N>
inline constexpr TwTable<N> kTw{};

// ---------------------------------------------------------------------------------------
// Constants of the single-precision transforms.
//
// Rounding a DFT constant (a twiddle cos / sin) to FP32 changes the transform itself, not just
// one result: the forward transform and its conjugate inverse then miss each other by a fixed
// O(2^-24) matrix, and a pair energy <rho|G (*) rho> picks up a first-order bias that does not
// average out over the grid (about 1e-7 relative in the exchange energy, measured by emulating
// the passes in NumPy).  The rounding of the data in the arithmetic itself is unbiased and
// costs about 100 times less.  Most of the bias comes from constants whose rounded magnitude
// is off (|c + i s| != 1 scales every value through them the same way); a phase error moves
// much less.  So:
//  * the 45-degree factor of radix 8 (c = +-s, for which no float pair has unit magnitude) is
//    carried as an unevaluated sum hi + lo of two floats (hi = RNE(c), lo = RNE(c - hi)), and
//    x * c is formed as fma(x, hi, x * lo): one rounding of the product with the constant
//    correct to about 2^-48;
//  * the cos / sin of radices 3, 5, 7 (the odd-radix butterflies), the in-register twiddles off
//    the multiples of 45 degrees and the inter-factor table twiddles (one complex product per
//    point and factor) are plain float pairs chosen for unit magnitude: among the floats within 3 ulps of cos and sin, the pair with the smallest
//    |c^2 + s^2 - 1| (then the smallest phase error), one instruction per constant product.
//    For the table twiddles this removes about 90 % of their share of the bias in the NumPy
//    emulation; for the butterflies the round-trip bias of the 1-D transforms is as small as
//    with hi + lo constants (a unit-magnitude 45-degree pair instead raised it fourfold).
// ACE_FFT_SPLIT_CONSTANTS = 0 rounds the hi + lo constants to plain floats (for measurement
// only).
#ifndef ACE_FFT_SPLIT_CONSTANTS
#define ACE_FFT_SPLIT_CONSTANTS 1
#endif
constexpr bool kSplitConstants = ACE_FFT_SPLIT_CONSTANTS != 0;

struct SplitF {
  float hi, lo;
};
__host__ __device__ constexpr SplitF split_f(double c) {
  return {float(c), kSplitConstants ? float(c - double(float(c))) : 0.0f};
}

// x * c for a compile-time constant c (T = double: the double product)
template <typename T>
__host__ __device__ __forceinline__ T mul_k(T x, double c) {
  if constexpr (sizeof(T) == 4) {
    const SplitF k = split_f(c);
    return k.lo == 0.0f ? x * k.hi : fmaf(x, k.hi, x * k.lo);
  } else {
    return x * T(c);
  }
}
// acc + x * c for a compile-time constant c
template <typename T>
__host__ __device__ __forceinline__ T fma_k(T x, double c, T acc) {
  if constexpr (sizeof(T) == 4) {
    const SplitF k = split_f(c);
    return k.lo == 0.0f ? fmaf(x, k.hi, acc) : fmaf(x, k.hi, fmaf(x, k.lo, acc));
  } else {
    return acc + x * T(c);
  }
}

// a * (c + i s) for compile-time constants c, s (branches fold after unrolling).
template <typename T>
__host__ __device__ __forceinline__ C2<T> cmul_k(C2<T> a, double c, double s) {
  if (s == 0.0) {
    if (c == 1.0) return a;
    if (c == -1.0) return {-a.r, -a.i};
    return {mul_k(a.r, c), mul_k(a.i, c)};
  }
  if (c == 0.0) {
    if (s == 1.0) return {-a.i, a.r};
    if (s == -1.0) return {a.i, -a.r};
    return {-mul_k(a.i, s), mul_k(a.r, s)};
  }
  if constexpr (sizeof(T) == 4) {
    const SplitF kc = split_f(c), ks = split_f(s);
    if (c == s || c == -s) {
      // (1 +- i) c: one sum and one difference, then two constant products
      const float u = a.r - (c == s ? a.i : -a.i), w = a.i + (c == s ? a.r : -a.r);
      return {mul_k(u, c), mul_k(w, c)};
    }
    if (kc.lo != 0.0f && ks.lo != 0.0f) {
      // correction terms first (products with the small parts), then the main products
      const float cr = fmaf(a.r, kc.lo, -a.i * ks.lo);
      const float ci = fmaf(a.r, ks.lo, a.i * kc.lo);
      return {fmaf(a.r, kc.hi, fmaf(-a.i, ks.hi, cr)), fmaf(a.r, ks.hi, fmaf(a.i, kc.hi, ci))};
    }
    if (kc.lo != 0.0f) {
      return {fmaf(a.r, kc.hi, fmaf(-a.i, ks.hi, a.r * kc.lo)),
              fmaf(a.r, ks.hi, fmaf(a.i, kc.hi, a.i * kc.lo))};
    }
    if (ks.lo != 0.0f) {
      return {fmaf(a.r, kc.hi, fmaf(-a.i, ks.hi, -a.i * ks.lo)),
              fmaf(a.r, ks.hi, fmaf(a.i, kc.hi, a.r * ks.lo))};
    }
  }
  return {a.r * T(c) - a.i * T(s), a.r * T(s) + a.i * T(c)};
}

// Odd-radix butterfly constants as unit-magnitude float pairs: for each angle 2 pi m / R the
// float pair within 3 ulps of (cos, sin) with the smallest |c^2 + s^2 - 1| (then the smallest
// phase error), one instruction per constant product instead of the two of the hi + lo form.
// Compile-time tables.  ACE_FFT_UNIT_CONSTANTS = 0 keeps the hi + lo form (for measurement).
#ifndef ACE_FFT_UNIT_CONSTANTS
#define ACE_FFT_UNIT_CONSTANTS 1
#endif
constexpr bool kUnitConstants = ACE_FFT_UNIT_CONSTANTS != 0;

// spacing of the floats around float(x), as a double (the spacing of its binade)
constexpr double float_ulp(double x) {
  double a = x < 0 ? -x : x;
  if (a == 0.0) return 1.0e-45;
  double p = 1.0;
  while (p > a) p *= 0.5;
  while (p * 2.0 <= a) p *= 2.0;
  return p * 1.1920928955078125e-07;  // 2^-23
}
constexpr double abs_c(double x) { return x < 0 ? -x : x; }

struct UnitF {
  float c, s;
};
constexpr UnitF unit_pair_f(double c, double s) {
  const float c0 = float(c), s0 = float(s);
  const bool exact =
      (c0 == 0.f || c0 == 1.f || c0 == -1.f) && (s0 == 0.f || s0 == 1.f || s0 == -1.f);
  if (exact) return {c0, s0};
  const double uc = float_ulp(c0), us = float_ulp(s0);
  UnitF best{c0, s0};
  double bm = 2.0, bp = 2.0;
  for (int dc = -3; dc <= 3; ++dc)
    for (int ds = -3; ds <= 3; ++ds) {
      const float fc = float(double(c0) + dc * uc), fs = float(double(s0) + ds * us);
      const double m = abs_c(double(fc) * fc + double(fs) * fs - 1.0);
      const double ph = abs_c(double(fs) * c - double(fc) * s);
      if (m < bm || (m == bm && ph < bp)) {
        bm = m;
        bp = ph;
        best = {fc, fs};
      }
    }
  return best;
}

template <int N>
struct TwTableU {
  float c[N];
  float s[N];
  constexpr TwTableU() : c(), s() {
    for (int m = 0; m < N; ++m) {
      const UnitF u = unit_pair_f(kTw<N>.c[m], kTw<N>.s[m]);
      c[m] = u.c;
      s[m] = u.s;
    }
  }
};
template <int N>
inline constexpr TwTableU<N> kTwU{};

// Twiddle table entry exp(-2 pi i m / P) of the two-factor transforms: FP64 as is (16 bytes),
// FP32 as a float pair of unit magnitude (8 bytes, unit_twiddle_f below).
template <typename T>
struct TwE;
template <>
struct alignas(16) TwE<double> {
  double c, s;
};
template <>
struct alignas(8) TwE<float> {
  float c, s;
};

// a * w and a * conj(w) for a table twiddle w
__host__ __device__ __forceinline__ C2<double> tw_mul(C2<double> a, TwE<double> w) {
  return {a.r * w.c - a.i * w.s, a.r * w.s + a.i * w.c};
}
__host__ __device__ __forceinline__ C2<double> tw_mul_conj(C2<double> a, TwE<double> w) {
  return {a.r * w.c + a.i * w.s, a.i * w.c - a.r * w.s};
}
__host__ __device__ __forceinline__ C2<float> tw_mul(C2<float> a, TwE<float> w) {
  return {fmaf(a.r, w.c, -a.i * w.s), fmaf(a.r, w.s, a.i * w.c)};
}
__host__ __device__ __forceinline__ C2<float> tw_mul_conj(C2<float> a, TwE<float> w) {
  return {fmaf(a.r, w.c, a.i * w.s), fmaf(a.i, w.c, -a.r * w.s)};
}

// The FP32 table twiddle for cos + i sin (host side, when a context is created): the float
// pair within 3 ulps of (RNE(cos), RNE(sin)) with the smallest |c^2 + s^2 - 1|, ties broken by
// the smaller phase error.  Exact values (0, +-1) come back unchanged.
inline TwE<float> unit_twiddle_f(double c, double s) {
  auto step = [](float x, int d) {
    for (int i = 0; i < (d < 0 ? -d : d); ++i)
      x = __builtin_nextafterf(x, d > 0 ? __builtin_inff() : -__builtin_inff());
    return x;
  };
  TwE<float> best = {float(c), float(s)};
  double bmag = 2.0, bph = 2.0;
  for (int dc = -3; dc <= 3; ++dc)
    for (int ds = -3; ds <= 3; ++ds) {
      const float fc = step(float(c), dc), fs = step(float(s), ds);
      const double mag = __builtin_fabs((double)fc * fc + (double)fs * fs - 1.0);
      // |sin| of the angle between (fc, fs) and (c, s): the phase error
      const double ph = __builtin_fabs((double)fs * c - (double)fc * s);
      if (mag < bmag || (mag == bmag && ph < bph)) {
        bmag = mag;
        bph = ph;
        best = {fc, fs};
      }
    }
  return best;
}

// W_N^{m} with sign DIR: exp(DIR * 2 pi i m / N); DIR = -1 forward, +1 inverse.
template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ C2<T> twk(C2<T> a, int m) {
  const int mm = m % N;
  if constexpr (sizeof(T) == 4 && kUnitConstants) {
    // angles off the multiples of 45 degrees: a unit-magnitude float pair, 4 instructions
    if ((8 * mm) % N != 0) {
      const float c = kTwU<N>.c[mm], s = DIR * kTwU<N>.s[mm];
      return {fmaf(a.r, c, -a.i * s), fmaf(a.r, s, a.i * c)};
    }
  }
  return cmul_k<T>(a, kTw<N>.c[mm], DIR * kTw<N>.s[mm]);
}

constexpr int pick_radix(int n) {
  return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : (n % 5 == 0) ? 5 : n;
}

// Odd-prime (or small) direct butterfly, natural order in/out.
template <typename T, int R, int DIR>
__host__ __device__ __forceinline__ void butterfly(C2<T>* x) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    C2<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    C2<T> s02 = cadd(x[0], x[2]), d02 = csub(x[0], x[2]);
    C2<T> s13 = cadd(x[1], x[3]), d13 = csub(x[1], x[3]);
    // DIR * i * d13
    C2<T> j13 = (DIR < 0) ? C2<T>{d13.i, -d13.r} : C2<T>{-d13.i, d13.r};
    x[0] = cadd(s02, s13);
    x[2] = csub(s02, s13);
    x[1] = cadd(d02, j13);
    x[3] = csub(d02, j13);
  } else {
    // X_k = x0 + sum_{m=1}^{(R-1)/2} [(x_m + x_{R-m}) cos(2 pi m k/R) + DIR i (x_m - x_{R-m}) sin(2 pi m k/R)]
    static_assert(R % 2 == 1, "odd radix expected");
    constexpr int Hh = (R - 1) / 2;
    C2<T> sp[Hh], sm[Hh];
#pragma unroll
    for (int m = 1; m <= Hh; ++m) {
      sp[m - 1] = cadd(x[m], x[R - m]);
      sm[m - 1] = csub(x[m], x[R - m]);
    }
    C2<T> out[R];
    C2<T> x0 = x[0];
    C2<T> tot = x0;
#pragma unroll
    for (int m = 0; m < Hh; ++m) tot = cadd(tot, sp[m]);
    out[0] = tot;
#pragma unroll
    for (int k = 1; k <= Hh; ++k) {
      C2<T> re = x0, im;
#pragma unroll
      for (int m = 1; m <= Hh; ++m) {
        const int mk = (m * k) % R;
        if constexpr (sizeof(T) == 4 && kUnitConstants) {
          const float c = kTwU<R>.c[mk], s = kTwU<R>.s[mk];
          re.r = fmaf(sp[m - 1].r, c, re.r);
          re.i = fmaf(sp[m - 1].i, c, re.i);
          im.r = m == 1 ? sm[0].r * s : fmaf(sm[m - 1].r, s, im.r);
          im.i = m == 1 ? sm[0].i * s : fmaf(sm[m - 1].i, s, im.i);
        } else {
          const double c = kTw<R>.c[mk];
          const double s = kTw<R>.s[mk];
          re.r = fma_k(sp[m - 1].r, c, re.r);
          re.i = fma_k(sp[m - 1].i, c, re.i);
          if (m == 1) {
            im.r = mul_k(sm[0].r, s);
            im.i = mul_k(sm[0].i, s);
          } else {
            im.r = fma_k(sm[m - 1].r, s, im.r);
            im.i = fma_k(sm[m - 1].i, s, im.i);
          }
        }
      }
      // DIR * i * im
      C2<T> jim = (DIR < 0) ? C2<T>{im.i, -im.r} : C2<T>{-im.i, im.r};
      out[k] = cadd(re, jim);
      out[R - k] = csub(re, jim);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = out[k];
  }
}

constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }
// multiplicative inverse of a modulo m (gcd(a, m) = 1)
constexpr int inv_mod(int a, int m) {
  for (int u = 1; u < m; ++u)
    if ((a * u) % m == 1) return u;
  return 1;
}

// In-register DFT of length N, natural order in and out, unnormalised.
// X_k = sum_n x_n exp(DIR 2 pi i n k / N).
// N = R M with gcd(R, M) = 1 goes the prime-factor (Good-Thomas) way: input n = (M n1 + R n2)
// mod N, output k = CRT(k mod R, k mod M), so W_N^{nk} = W_R^{n1 k1} W_M^{n2 k2} and no twiddle
// is multiplied between the two factors (both maps are compile-time index permutations).
// Otherwise decimation in time with twiddles W_N^{rk}.
template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dft(C2<T>* x) {
  constexpr int R = pick_radix(N);
  constexpr int M = N / R;
  if constexpr (M == 1) {
    butterfly<T, R, DIR>(x);
  } else if constexpr (gcd_c(R, M) == 1) {
    constexpr int UR = inv_mod(M % R, R);  // k = (M UR k1 + R UM k2) mod N
    constexpr int UM = inv_mod(R % M, M);
    C2<T> y[M][R];
#pragma unroll
    for (int n2 = 0; n2 < M; ++n2)
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) y[n2][n1] = x[(M * n1 + R * n2) % N];
#pragma unroll
    for (int n2 = 0; n2 < M; ++n2) butterfly<T, R, DIR>(y[n2]);
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      C2<T> t[M];
#pragma unroll
      for (int n2 = 0; n2 < M; ++n2) t[n2] = y[n2][k1];
      dft<T, M, DIR>(t);
#pragma unroll
      for (int k2 = 0; k2 < M; ++k2) x[(M * UR * k1 + R * UM * k2) % N] = t[k2];
    }
  } else {
    // decimation in time: y_r = DFT_M(x[r + R m]); X[k + M s] = sum_r W_R^{rs} W_N^{rk} y_r[k]
    C2<T> y[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int m = 0; m < M; ++m) y[r][m] = x[r + R * m];
#pragma unroll
    for (int r = 0; r < R; ++r) dft<T, M, DIR>(y[r]);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      C2<T> t[R];
#pragma unroll
      for (int r = 0; r < R; ++r) t[r] = twk<T, N, DIR>(y[r][k], r * k);
      butterfly<T, R, DIR>(t);
#pragma unroll
      for (int s = 0; s < R; ++s) x[k + M * s] = t[s];
    }
  }
}

// Length-N DFT whose inputs x[N/2 .. N) are zero (N even).  Reads x[0..N/2), writes x[0..N).
template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dft_in_half(C2<T>* x) {
  static_assert(N % 2 == 0, "even length");
  constexpr int H = N / 2;
  C2<T> e[H], o[H];
#pragma unroll
  for (int m = 0; m < H; ++m) {
    e[m] = x[m];
    o[m] = twk<T, N, DIR>(x[m], m);
  }
  dft<T, H, DIR>(e);
  dft<T, H, DIR>(o);
#pragma unroll
  for (int m = 0; m < H; ++m) {
    x[2 * m] = e[m];
    x[2 * m + 1] = o[m];
  }
}

// Length-N DFT of which only outputs x[0 .. N/2) are needed (N even).  Reads x[0..N).
template <typename T, int N, int DIR>
__host__ __device__ __forceinline__ void dft_out_half(C2<T>* x) {
  static_assert(N % 2 == 0, "even length");
  constexpr int H = N / 2;
  C2<T> e[H], o[H];
#pragma unroll
  for (int m = 0; m < H; ++m) {
    e[m] = x[2 * m];
    o[m] = x[2 * m + 1];
  }
  dft<T, H, DIR>(e);
  dft<T, H, DIR>(o);
#pragma unroll
  for (int m = 0; m < H; ++m) x[m] = cadd(e[m], twk<T, N, DIR>(o[m], m));
}

}  // namespace ace
