#pragma once
// The twiddle table of the block FFT, W_4096^k = exp(-2 pi i k / 4096) for
// k < 2048, computed at compile time. Plain C++ (no HIP), so that a host
// program can check the table.
//
// Compile-time cos and sin of 2 pi k / n: a double-precision Taylor series on
// [0, pi / 4] after reduction by the quadrant and octant symmetries, rounded
// once to float (the table matches correctly rounded values to within one
// float rounding of a tie).
namespace pwbf {
namespace fft {
namespace detail {
constexpr double kTwoPi = 6.28318530717958647692528676655900577;
constexpr double sin_series(double x) {
  double t = x, s = x;
  for (int i = 1; i < 13; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double cos_series(double x) {
  double t = 1.0, s = 1.0;
  for (int i = 1; i < 13; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
struct Tw {
  float c, s;
};
constexpr Tw w_of(int k, int n) {  // exp(-2 pi i k / n), 0 <= k < n, 8 | n
  const int q4 = n / 4, q = k / q4, kr = k % q4;
  double cr = 0.0, sr = 0.0;
  if (2 * kr <= q4) {
    const double x = kTwoPi * kr / n;
    cr = cos_series(x);
    sr = sin_series(x);
  } else {
    const double x = kTwoPi * (q4 - kr) / n;
    cr = sin_series(x);
    sr = cos_series(x);
  }
  double c = 0.0, s = 0.0;
  switch (q) {
    case 0: c = cr; s = sr; break;
    case 1: c = -sr; s = cr; break;
    case 2: c = -cr; s = -sr; break;
    default: c = sr; s = -cr; break;
  }
  return {(float)c, (float)-s};
}
constexpr int kTwN = 4096;  // the largest transform
struct alignas(8) TwTable {
  Tw v[kTwN / 2];
  constexpr TwTable() : v() {
    for (int k = 0; k < kTwN / 2; ++k) v[k] = w_of(k, kTwN);
  }
};
}  // namespace detail
}  // namespace fft
}  // namespace pwbf
