// The register DFTs of dft.hpp (every radix the line transforms use, forward
// and inverse) against the O(N^2) definition in double precision, with the
// constants rounded to nearest.  Host build against the emulation header.
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdio>
#include <random>

#include "dft.hpp"

namespace {

brahms::DftConsts nearest_consts() {
  brahms::DftConsts k{};
  k.h = float(std::sqrt(0.5));
  k.c8 = float(std::cos(M_PI / 8));
  k.s8 = float(std::sin(M_PI / 8));
  k.r3 = float(std::sqrt(3.0) / 2);
  k.c12 = float(std::cos(M_PI / 12));
  k.s12 = float(std::sin(M_PI / 12));
  k.t8 = float(std::tan(M_PI / 8));
  k.c36 = float(std::cos(M_PI / 18));
  k.s36 = float(std::sin(M_PI / 18));
  k.c18 = float(std::cos(M_PI / 9));
  k.s18 = float(std::sin(M_PI / 9));
  k.c9 = float(std::cos(2 * M_PI / 9));
  k.s9 = float(std::sin(2 * M_PI / 9));
  return k;
}

template <int N, bool INV>
double rel_error(const brahms::DftConsts& K, unsigned seed) {
  std::mt19937 rng(seed);
  std::uniform_real_distribution<float> uni(-1.f, 1.f);
  float2 v[N];
  std::complex<double> x[N];
  for (int n = 0; n < N; ++n) {
    v[n] = make_float2(uni(rng), uni(rng));
    x[n] = {v[n].x, v[n].y};
  }
  brahms::dft<N, INV>(v, K);
  double num = 0, den = 0;
  for (int k = 0; k < N; ++k) {
    std::complex<double> s = 0;
    for (int n = 0; n < N; ++n) s += x[n] * std::polar(1.0, (INV ? 2 : -2) * M_PI * double(n) * k / N);
    num += std::norm(std::complex<double>(v[k].x, v[k].y) - s);
    den += std::norm(s);
  }
  return std::sqrt(num / den);
}

template <int N>
bool check(const brahms::DftConsts& K) {
  double worst = 0;
  for (unsigned seed = 0; seed < 50; ++seed) {
    worst = std::max(worst, rel_error<N, false>(K, seed));
    worst = std::max(worst, rel_error<N, true>(K, 1000 + seed));
  }
  // a few FP32 roundings per output: far below 1e-6; a wrong sign, index or
  // twiddle gives O(1)
  const bool ok = worst < 1e-6;
  std::printf("N = %2d: worst relative L2 error %.3g %s\n", N, worst, ok ? "ok" : "FAIL");
  return ok;
}

}  // namespace

int main() {
  const brahms::DftConsts K = nearest_consts();
  bool ok = true;
  ok &= check<1>(K);
  ok &= check<2>(K);
  ok &= check<3>(K);
  ok &= check<4>(K);
  ok &= check<6>(K);
  ok &= check<8>(K);
  ok &= check<12>(K);
  ok &= check<16>(K);
  ok &= check<24>(K);
  ok &= check<9>(K);
  ok &= check<18>(K);
  ok &= check<36>(K);
  return ok ? 0 : 1;
}
