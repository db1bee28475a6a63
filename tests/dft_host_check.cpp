// Host check of the register DFTs (dft.h): every compile-time length against a
// direct O(R^2) DFT in double precision on seeded complex inputs.  Prints one
// line per length and exits non-zero if any relative error exceeds 1e-6.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include "dft.h"

using namespace lddmm::dft;

template <int R>
static double check() {
  std::mt19937 gen(1000 + R);
  std::normal_distribution<float> nd;
  float2 v[R];
  std::complex<double> x[R];
  for (int i = 0; i < R; ++i) {
    v[i] = make_float2(nd(gen), nd(gen));
    x[i] = {v[i].x, v[i].y};
  }
  Dft<R>::run(v);
  double err = 0.0, mx = 0.0;
  for (int m = 0; m < R; ++m) {
    std::complex<double> s = 0.0;
    for (int p = 0; p < R; ++p) s += x[p] * std::polar(1.0, -2.0 * M_PI * p * m / R);
    err = std::fmax(err, std::abs(s - std::complex<double>(v[m].x, v[m].y)));
    mx = std::fmax(mx, std::abs(s));
  }
  std::printf("R=%2d rel err %.3e\n", R, err / mx);
  return err / mx;
}

int main() {
  const double e[] = {check<2>(),  check<3>(),  check<4>(),  check<5>(),  check<6>(),
                      check<7>(),  check<8>(),  check<9>(),  check<10>(), check<12>(),
                      check<14>(), check<15>(), check<16>(), check<20>(), check<28>(),
                      check<35>()};
  double worst = 0.0;
  for (double x : e) worst = std::fmax(worst, x);
  std::printf("worst %.3e\n", worst);
  return worst < 1e-6 ? 0 : 1;
}
