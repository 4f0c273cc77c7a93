// Checks every radix-R butterfly of the transform kernels (forward, inverse, zero-pruned) on
// the CPU against the DFT written out in double precision; prints the worst relative error.
#include <algorithm>
#include <complex>
#include <cstdio>
#include <random>

#include "fft.hpp"

using dpx::DFT;

template <int R, bool INV, bool HALF>
double check(unsigned seed) {
  std::mt19937 g(seed);
  std::normal_distribution<float> nd;
  float2 v[R];
  std::complex<double> x[R];
  for (int i = 0; i < R; ++i) {
    v[i] = make_float2(nd(g), nd(g));
    if (HALF && i >= R / 2) v[i] = make_float2(0.f, 0.f);
    x[i] = {v[i].x, v[i].y};
  }
  DFT<R, INV, HALF>::run(v);
  double err = 0.0, ref = 0.0;
  for (int k = 0; k < R; ++k) {
    std::complex<double> s = 0.0;
    for (int n = 0; n < R; ++n) s += x[n] * std::polar(1.0, (INV ? 2.0 : -2.0) * M_PI * ((n * k) % R) / R);
    err = std::max(err, std::abs(s - std::complex<double>(v[k].x, v[k].y)));
    ref = std::max(ref, std::abs(s));
  }
  return err / ref;
}

template <int R>
double all_forms() {
  double e = std::max(check<R, false, false>(R), check<R, true, false>(R + 1));
  if constexpr (R % 2 == 0) e = std::max({e, check<R, false, true>(R + 2), check<R, true, true>(R + 3)});
  return e;
}

int main() {
  const double e[] = {all_forms<2>(), all_forms<3>(), all_forms<4>(),  all_forms<5>(),
                      all_forms<6>(), all_forms<8>(), all_forms<10>(), all_forms<12>(),
                      all_forms<16>(), all_forms<20>()};
  double worst = 0.0;
  for (double x : e) worst = std::max(worst, x);
  std::printf("%.3e\n", worst);
  return 0;
}
