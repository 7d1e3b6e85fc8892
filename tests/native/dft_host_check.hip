// Host-side check of the register DFTs and of the two-step P = P1 * P2 transform used by the
// pair-Poisson passes.  Compiled with hipcc and run on the CPU (no GPU needed): every routine
// under test is __host__ __device__.  Reference: naive O(P^2) DFT in long double.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2405_01522_amd/csrc/common.hpp"
#include "../../paper_2405_01522_amd/csrc/fftplan.hpp"

using namespace ace;
typedef std::complex<long double> cld;

static std::vector<cld> naive(const std::vector<cld>& x, int dir) {
  const int n = (int)x.size();
  std::vector<cld> out(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < n; ++k) {
    cld s = 0;
    for (int m = 0; m < n; ++m) {
      long long e = (long long)m * k % n;
      long double a = dir * 2.0L * pi * (long double)e / n;
      s += x[m] * cld(cosl(a), sinl(a));
    }
    out[k] = s;
  }
  return out;
}

static int failures = 0;
static void check(const char* what, int n, double err, double tol) {
  if (!(err <= tol)) {
    std::printf("FAIL %s n=%d err=%.3e tol=%.1e\n", what, n, err, tol);
    ++failures;
  }
}

template <typename T, int N>
static void test_dft(std::mt19937_64& rng, double tol) {
  std::normal_distribution<double> nd;
  for (int dir : {-1, 1}) {
    std::vector<cld> x(N);
    C2<T> v[N];
    for (int k = 0; k < N; ++k) {
      v[k] = {T(nd(rng)), T(nd(rng))};
      x[k] = cld(v[k].r, v[k].i);
    }
    std::vector<cld> ref = naive(x, dir);
    if (dir < 0) dft<T, N, -1>(v); else dft<T, N, 1>(v);
    double err = 0, mx = 0;
    for (int k = 0; k < N; ++k) {
      err = std::fmax(err, (double)std::abs(ref[k] - cld(v[k].r, v[k].i)));
      mx = std::fmax(mx, (double)std::abs(ref[k]));
    }
    check(sizeof(T) == 8 ? "dft64" : "dft32", N * dir, err / mx, tol);
  }
  if constexpr (N % 2 == 0) {
    // input-pruned forward and output-pruned inverse
    std::vector<cld> x(N, 0);
    C2<T> v[N];
    for (int k = 0; k < N / 2; ++k) {
      v[k] = {T(nd(rng)), T(nd(rng))};
      x[k] = cld(v[k].r, v[k].i);
    }
    std::vector<cld> ref = naive(x, -1);
    dft_in_half<T, N, -1>(v);
    double err = 0, mx = 0;
    for (int k = 0; k < N; ++k) {
      err = std::fmax(err, (double)std::abs(ref[k] - cld(v[k].r, v[k].i)));
      mx = std::fmax(mx, (double)std::abs(ref[k]));
    }
    check("dft_in_half", N, err / mx, tol);
    for (int k = 0; k < N; ++k) {
      v[k] = {T(nd(rng)), T(nd(rng))};
      x[k] = cld(v[k].r, v[k].i);
    }
    ref = naive(x, 1);
    dft_out_half<T, N, 1>(v);
    err = 0; mx = 0;
    for (int k = 0; k < N / 2; ++k) {
      err = std::fmax(err, (double)std::abs(ref[k] - cld(v[k].r, v[k].i)));
      mx = std::fmax(mx, (double)std::abs(ref[k]));
    }
    check("dft_out_half", N, err / mx, tol);
  }
}

// Table twiddles exp(-2 pi i m / P) as the library builds them (FP32: unit-magnitude pairs).
template <typename T, int P>
static std::vector<TwE<T>> twiddle_table() {
  std::vector<TwE<T>> tw(P);
  for (int m = 0; m < P; ++m) {
    CosSin cs = cossin_2pi(m, P);
    if constexpr (sizeof(T) == 8) {
      tw[m] = {cs.c, -cs.s};
    } else {
      tw[m] = unit_twiddle_f(cs.c, -cs.s);
    }
  }
  return tw;
}

// Two-step forward transform of a length-P signal whose upper half is zero, left in position
// order; then the two-step inverse with cropped output, exactly as the passes do it.
template <typename T, int NB>
static void test_two_step(std::mt19937_64& rng, double tol) {
  typedef Plan<NB> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1;
  std::normal_distribution<double> nd;
  std::vector<TwE<T>> tw = twiddle_table<T, P>();
  std::vector<cld> x(P, 0);
  std::vector<C2<T>> buf(P);
  for (int z = 0; z < NB; ++z) x[z] = cld(nd(rng), nd(rng));
  // step A (per n2): pruned P1-point DFT over n1, twiddle, store at k1*P2+n2
  for (int n2 = 0; n2 < P2; ++n2) {
    C2<T> v[P1];
    for (int n1 = 0; n1 < H1; ++n1) {
      cld a = x[n1 * P2 + n2];
      v[n1] = {T(a.real()), T(a.imag())};
    }
    dft_in_half<T, P1, -1>(v);
    for (int k1 = 0; k1 < P1; ++k1) buf[k1 * P2 + n2] = tw_mul(v[k1], tw[n2 * k1]);
  }
  // step B (per k1): P2-point DFT of the contiguous block
  for (int k1 = 0; k1 < P1; ++k1) {
    C2<T> v[P2];
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = buf[k1 * P2 + k2];
    dft<T, P2, -1>(v);
    for (int k2 = 0; k2 < P2; ++k2) buf[k1 * P2 + k2] = v[k2];
  }
  std::vector<cld> ref = naive(x, -1);
  double err = 0, mx = 0;
  for (int q = 0; q < P; ++q) {
    cld got(buf[q].r, buf[q].i);
    err = std::fmax(err, (double)std::abs(ref[PL::freq(q)] - got));
    mx = std::fmax(mx, (double)std::abs(ref[PL::freq(q)]));
  }
  check("two_step_fwd", P, err / mx, tol);
  // inverse: step B' per k1, step A' per n2 with conj twiddle, keep n1 < H1
  for (int k1 = 0; k1 < P1; ++k1) {
    C2<T> v[P2];
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = buf[k1 * P2 + k2];
    dft<T, P2, 1>(v);
    for (int k2 = 0; k2 < P2; ++k2) buf[k1 * P2 + k2] = v[k2];
  }
  err = 0; mx = 0;
  for (int n2 = 0; n2 < P2; ++n2) {
    C2<T> v[P1];
    for (int k1 = 0; k1 < P1; ++k1) v[k1] = tw_mul_conj(buf[k1 * P2 + n2], tw[n2 * k1]);
    dft_out_half<T, P1, 1>(v);
    for (int n1 = 0; n1 < H1; ++n1) {
      cld got(v[n1].r / T(P), v[n1].i / T(P));
      err = std::fmax(err, (double)std::abs(x[n1 * P2 + n2] - got));
      mx = std::fmax(mx, (double)std::abs(x[n1 * P2 + n2]));
    }
  }
  check("two_step_roundtrip", P, err / mx, tol);
}

// Systematic error of the single-precision round trip that the pair energies see: for smooth
// positive inputs x (Gaussians at random centres and widths, like pair densities) and a
// positive even spectral weight g (like the Coulomb kernel), E = <x | IDFT(g DFT(x))> computed
// with the FP32 two-step transforms, relative to the long-double value, averaged over many
// inputs.  Rounding of the data averages out; rounded constants do not.  Returns the mean
// relative error.
template <int NB>
static double roundtrip_energy_bias(std::mt19937_64& rng, int samples) {
  typedef Plan<NB> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1;
  std::vector<TwE<float>> tw = twiddle_table<float, P>();
  std::uniform_real_distribution<double> ud(0.0, 1.0);
  // the weights (with the 1/P of the inverse folded in) are FP32 numbers, used as such by both
  // sides, so that only the transforms differ
  std::vector<float> g(P);
  for (int k = 0; k < P; ++k) {
    const int kk = k <= P - k ? k : P - k;
    g[k] = float(1.0 / ((1.0 + 0.5 * kk * kk) * P));
  }
  double sum = 0.0;
  for (int smp = 0; smp < samples; ++smp) {
    const double c0 = NB * (0.3 + 0.4 * ud(rng)), w = NB * (0.05 + 0.1 * ud(rng));
    std::vector<float> x(NB);
    for (int z = 0; z < NB; ++z) x[z] = float(std::exp(-((z - c0) * (z - c0)) / (2 * w * w)));
    // exact energy in long double
    std::vector<cld> xl(P, 0);
    for (int z = 0; z < NB; ++z) xl[z] = cld(x[z], 0);
    std::vector<cld> xh = naive(xl, -1);
    long double e_ref = 0;
    for (int k = 0; k < P; ++k) e_ref += (long double)g[k] * std::norm(xh[k]);
    // FP32 two-step forward, weight (in position order), two-step inverse, crop
    std::vector<C2<float>> buf(P);
    for (int n2 = 0; n2 < P2; ++n2) {
      C2<float> v[P1];
      for (int n1 = 0; n1 < H1; ++n1) v[n1] = {x[n1 * P2 + n2], 0.f};
      dft_in_half<float, P1, -1>(v);
      for (int k1 = 0; k1 < P1; ++k1) buf[k1 * P2 + n2] = tw_mul(v[k1], tw[n2 * k1]);
    }
    for (int k1 = 0; k1 < P1; ++k1) {
      C2<float> v[P2];
      for (int k2 = 0; k2 < P2; ++k2) v[k2] = buf[k1 * P2 + k2];
      dft<float, P2, -1>(v);
      for (int k2 = 0; k2 < P2; ++k2) {
        const float gk = g[PL::freq(k1 * P2 + k2)];
        v[k2] = {v[k2].r * gk, v[k2].i * gk};
      }
      dft<float, P2, 1>(v);
      for (int k2 = 0; k2 < P2; ++k2) buf[k1 * P2 + k2] = v[k2];
    }
    long double e = 0;
    for (int n2 = 0; n2 < P2; ++n2) {
      C2<float> v[P1];
      for (int k1 = 0; k1 < P1; ++k1) v[k1] = tw_mul_conj(buf[k1 * P2 + n2], tw[n2 * k1]);
      dft_out_half<float, P1, 1>(v);
      for (int n1 = 0; n1 < H1; ++n1) e += (long double)x[n1 * P2 + n2] * v[n1].r;
    }
    sum += double((e - e_ref) / e_ref);
  }
  return sum / samples;
}

int main() {
  std::mt19937_64 rng(1234);
  const double t64 = 1e-14, t32 = 2e-6;
  test_dft<double, 2>(rng, t64); test_dft<double, 3>(rng, t64); test_dft<double, 4>(rng, t64);
  test_dft<double, 5>(rng, t64); test_dft<double, 6>(rng, t64); test_dft<double, 7>(rng, t64);
  test_dft<double, 8>(rng, t64); test_dft<double, 9>(rng, t64); test_dft<double, 10>(rng, t64);
  test_dft<double, 12>(rng, t64); test_dft<double, 14>(rng, t64); test_dft<double, 16>(rng, t64);
  test_dft<float, 8>(rng, t32); test_dft<float, 12>(rng, t32); test_dft<float, 16>(rng, t32);
  test_dft<float, 7>(rng, t32); test_dft<float, 10>(rng, t32);
  test_two_step<double, 8>(rng, t64); test_two_step<double, 9>(rng, t64);
  test_two_step<double, 10>(rng, t64); test_two_step<double, 12>(rng, t64);
  test_two_step<double, 16>(rng, t64); test_two_step<double, 20>(rng, t64);
  test_two_step<double, 24>(rng, t64); test_two_step<double, 32>(rng, t64);
  test_two_step<double, 40>(rng, t64); test_two_step<double, 48>(rng, t64);
  test_two_step<double, 56>(rng, t64); test_two_step<double, 64>(rng, t64);
  test_two_step<float, 48>(rng, t32); test_two_step<float, 64>(rng, t32);
  {
    // FP32 round-trip energy bias of the padded lengths of the benchmark boxes
    const double b48 = roundtrip_energy_bias<48>(rng, 400);
    const double b64 = roundtrip_energy_bias<64>(rng, 400);
    const double b40 = roundtrip_energy_bias<40>(rng, 400);
    const double b56 = roundtrip_energy_bias<56>(rng, 400);
    std::printf("fp32 round-trip energy bias: P=80 %.2e  P=96 %.2e  P=112 %.2e  P=128 %.2e\n", b40,
                b48, b56, b64);
    const double lim = kSplitConstants ? 1e-8 : 1.0;
    check("roundtrip_bias", 80, std::fabs(b40), lim);
    check("roundtrip_bias", 96, std::fabs(b48), lim);
    check("roundtrip_bias", 112, std::fabs(b56), lim);
    check("roundtrip_bias", 128, std::fabs(b64), lim);
  }
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
