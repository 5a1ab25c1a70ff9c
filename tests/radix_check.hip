// Host check of the in-register DFT butterflies of the line engine (the same
// source, compiled for the CPU): Dft<R, INV> of random complex vectors
// against a direct double-precision DFT, forward and inverse, for every radix
// the FFT plans use.  Prints the worst relative error per radix; exits 1 if
// any exceeds the bound.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include "../paper_2506_16076_amd/csrc/radix.h"

using namespace fcsd;

template <int R, bool INV>
static double check_one(std::mt19937& g) {
  std::uniform_real_distribution<float> u(-1.f, 1.f);
  double worst = 0.0;
  for (int rep = 0; rep < 50; ++rep) {
    float2 x[R];
    std::complex<double> ref[R];
    for (int t = 0; t < R; ++t) x[t] = make_float2(u(g), u(g));
    double norm = 0.0;
    for (int q = 0; q < R; ++q) {
      std::complex<double> s = 0.0;
      for (int t = 0; t < R; ++t) {
        const double a = (INV ? 2.0 : -2.0) * M_PI * (double)t * q / R;
        s += std::complex<double>(x[t].x, x[t].y) * std::polar(1.0, a);
      }
      ref[q] = s;
      norm = std::max(norm, std::abs(s));
    }
    Dft<R, INV>::run(x);
    for (int q = 0; q < R; ++q)
      worst = std::max(worst, std::abs(std::complex<double>(x[q].x, x[q].y) - ref[q]) / norm);
  }
  return worst;
}

template <int R>
static bool check(std::mt19937& g) {
  const double e = std::max(check_one<R, false>(g), check_one<R, true>(g));
  const bool ok = e <= 2e-6;
  printf("radix %2d: worst relative error %.2e %s\n", R, e, ok ? "ok" : "FAIL");
  return ok;
}

int main() {
  std::mt19937 g(7);
  bool ok = true;
  ok &= check<2>(g);
  ok &= check<3>(g);
  ok &= check<4>(g);
  ok &= check<5>(g);
  ok &= check<6>(g);
  ok &= check<7>(g);
  ok &= check<8>(g);
  ok &= check<9>(g);
  ok &= check<10>(g);
  ok &= check<11>(g);
  ok &= check<12>(g);
  ok &= check<13>(g);
  ok &= check<14>(g);
  ok &= check<15>(g);
  ok &= check<16>(g);
  return ok ? 0 : 1;
}
