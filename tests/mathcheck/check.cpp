// check.cpp -- the integrand headers' mathematical functions (atan_rr, tan_halfpi,
// sincos_2pi) compiled for the host in binary64 and compared with the C library's long
// double versions over the ranges the integrands use.  Prints the largest error of each
// in units in the last place of the reference (of the larger of |sin|, |cos| for the
// pair), as JSON.  TEST INFRASTRUCTURE: built and run by tests/test_math_functions.py.
#include "hip/hip_runtime.h"
#include "device_common.hpp"
#include "integrands.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>

static double ulp_of(long double r) {
  const double d = std::fabs(static_cast<double>(r));
  return std::nextafter(d, INFINITY) - d;
}

int main(int argc, char** argv) {
  const long n = argc > 1 ? std::atol(argv[1]) : 1000000;
  std::mt19937_64 g(11);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  double e_atan = 0, e_tan = 0, e_sin = 0, e_cos = 0;
  auto atan_at = [&](double x) {
    const long double r = atanl(static_cast<long double>(x));
    e_atan = std::max(e_atan, static_cast<double>(fabsl(vg::atan_rr(x) - r)) / ulp_of(r));
  };
  auto tan_at = [&](double x) {
    const long double r = tanl(static_cast<long double>(x));
    e_tan = std::max(e_tan, static_cast<double>(fabsl(vg::tan_halfpi(x) - r)) / ulp_of(r));
  };
  auto sincos_at = [&](double x) {
    double s, c;
    vg::sincos_2pi(x, s, c);
    const long double a = 2.0L * 3.141592653589793238462643383279502884L * static_cast<long double>(x);
    const long double rs = sinl(a), rc = cosl(a);
    const double m = ulp_of(std::max(fabsl(rs), fabsl(rc)));
    e_sin = std::max(e_sin, static_cast<double>(fabsl(s - rs)) / m);
    e_cos = std::max(e_cos, static_cast<double>(fabsl(c - rc)) / m);
  };
  const double pio2 = 1.5707963267948966;
  for (long i = 0; i < n; ++i) {
    const double sgn = u(g) < 0.5 ? -1.0 : 1.0;
    atan_at(sgn * std::pow(10.0, -13.0 + 26.0 * u(g)));  // magnitudes 1e-13 .. 1e13
    atan_at((2.0 * u(g) - 1.0) * 4.0);                     // around the folds
    tan_at((2.0 * u(g) - 1.0) * pio2 * 0.9999999);
    tan_at(sgn * pio2 * (1.0 - std::pow(10.0, -12.0 * u(g))));  // towards the pole
    tan_at(sgn * std::pow(10.0, -15.0 * u(g)));                 // towards zero
    sincos_at(u(g));
  }
  for (double x : {0.0, 0.66, 0.6600000000000001, 2.414213562373095, 2.4142135623730954, 1.0, 1e300})
    atan_at(x);
  for (double x : {0.7853981633974483, 0.7853981633974484, 1e-300}) tan_at(x);
  for (double x : {0.0, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 1.0}) sincos_at(x);
  std::printf("{\"atan\": %.4f, \"tan\": %.4f, \"sin\": %.4f, \"cos\": %.4f}\n", e_atan, e_tan, e_sin, e_cos);
  return 0;
}
