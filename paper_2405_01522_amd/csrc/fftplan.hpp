// Factorisation of the padded FFT length P = 2N into P = P1 * P2.
//
// Every 1-D transform of the pair-Poisson passes is done as one P1-point DFT per lane
// (stride-P2 elements), a twiddle W_P^{n2 k1}, an exchange through LDS, and one P2-point DFT
// per lane (contiguous elements).  The forward result is left in the "position" order
// q = k1 * P2 + k2 holding frequency k = k1 + P1 * k2; the inverse consumes that order and
// returns natural order, so no digit reversal pass is ever made.  P1 is even so that the
// zero-padded half of the input (n >= N) is exactly n1 >= P1/2 and the P1-point DFT can skip
// it (forward) or skip computing it (inverse, cropped output).
#pragma once

namespace ace {

constexpr bool small_primes_only(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  while (n % 7 == 0) n /= 7;
  return n == 1;
}

// ACE_PLAN_P2_EIGHT selects the transposed split P = (P/8) * 8 (larger first factor).
#ifndef ACE_PLAN_P2_EIGHT
#define ACE_PLAN_P2_EIGHT 0
#endif
constexpr int plan_p1(int P) {
  if (ACE_PLAN_P2_EIGHT && P >= 32 && P % 16 == 0 && P / 8 <= 16) return P / 8;
  if (P >= 32 && P % 8 == 0) return 8;
  for (int d = 4; d < P; d += 2)
    if (P % d == 0 && P / d >= 2) return d;
  return 2;
}

template <int N>
struct Plan {
  static constexpr int P = 2 * N;
  static constexpr int P1 = plan_p1(P);
  static constexpr int P2 = P / P1;
  static constexpr int H1 = P1 / 2;
  static constexpr int HO = P / 2 + 1;  // octant edge of the real-even kernel spectrum
  static_assert(P1 * P2 == P && P1 % 2 == 0, "bad factorisation");
  static_assert(small_primes_only(P1) && small_primes_only(P2), "radices 2,3,5,7 only");
  // frequency held at position q
  static constexpr __host__ __device__ int freq(int q) { return (q / P2) + P1 * (q % P2); }
};

}  // namespace ace
