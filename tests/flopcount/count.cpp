// count.cpp -- FLOPs per event of the kernels' formulation, counted on the host.
//
// The integrand headers of the GPU library (integrands.hpp, device_common.hpp) are
// compiled for the host with binary64 replaced by a counting scalar: every addition,
// subtraction and multiplication counts 1, every fused multiply-add 2, each hardware
// reciprocal / inverse-square-root estimate outside a priced routine 1 (the rocprof
// counter's convention).  Each evaluation of a mathematical function -- a division or
// reciprocal, a square root, tan, the sine and cosine of one angle, atan, log, exp,
// expm1 -- counts what one call of the library's version of it costs in FP64 FLOPs on
// gfx950 (measured with ocml_price.hip, given on the command line), whatever the kernel
// uses to evaluate it: the routines the headers mark with VG_PRICED are priced so and
// their own operations are not counted, and so is every '/' on per-event values.  The
// count is therefore the method's arithmetic with the amplitudes as the kernels state
// them, independent of how the kernels evaluate the functions.  Operations whose
// operands are all uniform (literals, the configuration's constants) are not counted:
// the GPU computes them once per thread, outside the event loop.  Comparisons, selects,
// sign changes, truncations and integer work count nothing.  The event's point comes
// from the same counter-based generator and a grid map written with the same
// arithmetic as the kernel's, through a grid read from a file (the uniforms come from a
// host generator, each counted as the one subtraction the kernel's construction of a
// uniform from its Philox words costs); the weight's product
// J f and the accumulation (S1 += w, w^2, S2 += w^2, one addition per dimension for the
// grid histogram) are added as 4 + D FLOPs.
//
// TEST INFRASTRUCTURE: built and run by tests/test_flop_count.py; not part of the library.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

namespace fc {
struct Tally {
  double flop = 0.0;
  double trans = 0.0;   // hardware estimates (rcp, rsq)
  double lib = 0.0;     // FLOPs of library-function calls
};
inline Tally g;
inline double price_atan = 0, price_log = 0, price_exp = 0, price_expm1 = 0, price_tan = 0, price_sincos = 0,
              price_sqrt = 0, price_div = 0, price_sqrt_div = 0;
// > 0 inside a priced routine: its own operations are not counted
inline int suspend = 0;

struct F64 {
  double v;
  bool u;  // uniform: derived only from literals and configuration constants
  constexpr F64() : v(0.0), u(true) {}
  constexpr F64(double x) : v(x), u(true) {}
  constexpr F64(double x, bool uni) : v(x), u(uni) {}
  template <class T, std::enable_if_t<std::is_integral_v<T>, int> = 0>
  constexpr F64(T x) : v(static_cast<double>(x)), u(false) {}
  template <class T, std::enable_if_t<std::is_arithmetic_v<T>, int> = 0>
  constexpr explicit operator T() const { return static_cast<T>(v); }
};

constexpr void count(double n, bool uniform) {
  if (!std::is_constant_evaluated() && !uniform && suspend == 0) g.flop += n;
}
inline void priced(double price, bool uniform) {
  if (!uniform && suspend == 0) g.lib += price, g.flop += price;
}
// a routine that evaluates a mathematical function: priced once, its body not counted
struct Priced {
  Priced(double price, bool uniform) {
    priced(price, uniform);
    ++suspend;
  }
  ~Priced() { --suspend; }
};
constexpr F64 operator+(F64 a, F64 b) { count(1, a.u && b.u); return {a.v + b.v, a.u && b.u}; }
constexpr F64 operator-(F64 a, F64 b) { count(1, a.u && b.u); return {a.v - b.v, a.u && b.u}; }
constexpr F64 operator*(F64 a, F64 b) { count(1, a.u && b.u); return {a.v * b.v, a.u && b.u}; }
constexpr F64 operator/(F64 a, F64 b) {
  if (!std::is_constant_evaluated()) priced(price_div, a.u && b.u);
  return {a.v / b.v, a.u && b.u};
}
constexpr F64 operator-(F64 a) { return {-a.v, a.u}; }
inline F64& operator+=(F64& a, F64 b) { return a = a + b; }
inline F64& operator-=(F64& a, F64 b) { return a = a - b; }
inline F64& operator*=(F64& a, F64 b) { return a = a * b; }
inline F64& operator/=(F64& a, F64 b) { return a = a / b; }
constexpr bool operator<(F64 a, F64 b) { return a.v < b.v; }
constexpr bool operator>(F64 a, F64 b) { return a.v > b.v; }
constexpr bool operator<=(F64 a, F64 b) { return a.v <= b.v; }
constexpr bool operator>=(F64 a, F64 b) { return a.v >= b.v; }
constexpr bool operator==(F64 a, F64 b) { return a.v == b.v; }
constexpr bool operator!=(F64 a, F64 b) { return a.v != b.v; }

inline F64 fma_c(F64 a, F64 b, F64 c) {
  const bool uni = a.u && b.u && c.u;
  count(2, uni);
  return {std::fma(a.v, b.v, c.v), uni};
}
inline F64 hw_est(double v, bool uni) {
  if (!uni && suspend == 0) g.trans += 1, g.flop += 1;
  return {v, uni};
}
inline F64 lib_call(double v, bool uni, double price) {
  priced(price, uni);
  return {v, uni};
}
}  // namespace fc

using fc::F64;
inline F64 fc_rcp(F64 x) { return fc::hw_est(1.0 / x.v, x.u); }
inline F64 fc_rsq(F64 x) { return fc::hw_est(1.0 / std::sqrt(x.v), x.u); }
inline uint32_t fc_xor3(uint32_t a, uint32_t b, uint32_t c) { return a ^ b ^ c; }
inline F64 __fma_rn(F64 a, F64 b, F64 c) { return fc::fma_c(a, b, c); }
inline F64 __hiloint2double(int hi, int lo) {
  const uint64_t b = (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
  double d;
  std::memcpy(&d, &b, 8);
  return {d, false};
}
inline F64 fabs(F64 x) { return {std::fabs(x.v), x.u}; }
inline F64 fmin(F64 a, F64 b) { return {std::fmin(a.v, b.v), a.u && b.u}; }
inline F64 fmax(F64 a, F64 b) { return {std::fmax(a.v, b.v), a.u && b.u}; }
inline F64 trunc(F64 x) { return {std::trunc(x.v), x.u}; }
inline F64 rint(F64 x) { return {std::rint(x.v), x.u}; }
inline F64 floor(F64 x) { return {std::floor(x.v), x.u}; }
inline F64 ldexp(F64 x, int e) { return {std::ldexp(x.v, e), x.u}; }
inline F64 copysign(F64 a, F64 b) { return {std::copysign(a.v, b.v), a.u && b.u}; }
inline bool signbit(F64 x) { return std::signbit(x.v); }
inline bool isfinite(F64 x) { return std::isfinite(x.v); }
inline F64 atan(F64 x) { return fc::lib_call(std::atan(x.v), x.u, fc::price_atan); }
inline F64 log(F64 x) { return fc::lib_call(std::log(x.v), x.u, fc::price_log); }
inline F64 exp(F64 x) { return fc::lib_call(std::exp(x.v), x.u, fc::price_exp); }
inline F64 expm1(F64 x) { return fc::lib_call(std::expm1(x.v), x.u, fc::price_expm1); }
// used only by the test integrands and the binary32 forms, which are not counted here
inline F64 cos(F64 x) { return {std::cos(x.v), x.u}; }
inline F64 pow(F64 a, F64 b) { return {std::pow(a.v, b.v), a.u && b.u}; }
inline void sincospif(float x, float* s, float* c) {
  *s = std::sin(3.14159265f * x);
  *c = std::cos(3.14159265f * x);
}
template <class T> inline T __shfl_xor(T v, int, int) { return v; }

#define double F64
#include "integrands.hpp"
#undef double

namespace {
// vg::PhysConst of a W+W- configuration, with the host-side formulas of the library
// (the values only steer which branches the events take)
vg::PhysConst ww_const(bool had) {
  vg::PhysConst k{};
  const double alpha = 1.0 / 128.0, MZ = 91.1876, GZ = 2.4952, MW = 80.4, GW = 2.1;
  const double sw2 = 1.0 - (MW / MZ) * (MW / MZ), sw = std::sqrt(sw2), cw = std::sqrt(1.0 - sw2);
  const double rs = had ? 13000.0 : 500.0, e2 = 4.0 * vg::kPi.v * alpha, g2 = e2 / sw2;
  k.conv = 0.3893794e9;
  k.pdfA = 1.0;
  k.pdfa = -0.5;
  k.pdfb = 3.0;
  k.pdf_pow = 1;
  k.pdf_a2 = -1;
  k.pdf_b = 3;
  k.M2 = MW * MW;
  k.MG = MW * GW;
  k.rs = rs;
  k.shat = rs * rs;
  k.m2lo = 0.0;
  k.invMG = 1.0 / (MW * GW);
  k.tlo = (0.0 - MW * MW) / (MW * GW);
  k.rho_lo = std::atan(k.tlo.v);
  k.rho_rng = std::atan((rs * rs - MW * MW) / (MW * GW)) - k.rho_lo.v;
  k.gs = std::sqrt(g2) / std::sqrt(2.0);
  k.ct = -0.5 * g2;
  const double dr = rs * rs - MZ * MZ, di = MZ * GZ, dd = dr * dr + di * di;
  double csr2 = 0.0;
  for (int q = 0; q < 2; ++q) {
    const double Q = q == 0 ? 2.0 / 3.0 : -1.0 / 3.0, T3 = q == 0 ? 0.5 : -0.5;
    for (int h = 0; h < 2; ++h) {
      const double gz = h == 0 ? (T3 - Q * sw2) / (sw * cw) : -Q * sw / cw, f = gz * cw / sw;
      k.cs_re[q][h] = e2 * (Q / (rs * rs) + f * dr / dd);
      k.cs_im[q][h] = e2 * (-f * di / dd);
      if (had) {
        k.csq[q] = e2 * Q;
        k.csf[q][h] = e2 * f;
      }
    }
    csr2 += k.cs_re[q][1].v * k.cs_re[q][1].v + k.cs_im[q][1].v * k.cs_im[q][1].v;
  }
  k.csR2 = csr2;
  if (had) {
    const double S = rs * rs, Llo = std::log(150.0 * 150.0 / S), Lhi = 0.0;
    k.S = S;
    k.Lhi = Lhi;
    k.Lrng = Llo - Lhi;
    k.Ldiff = Lhi - Llo;
    k.mz2 = MZ * MZ;
    k.mzgz = MZ * GZ;
  }
  k.MG2 = k.MG.v * k.MG.v;
  k.MGt = k.MG.v * (1.0 + k.tlo.v * k.tlo.v);
  k.mzgz2 = k.mzgz.v * k.mzgz.v;
  return k;
}
// vg::PhysConst of the W+ configuration (13 TeV, window from 40 GeV, pT > 20 GeV, |eta| < 2.5)
vg::PhysConst wplus_const() {
  vg::PhysConst k{};
  const double alpha = 1.0 / 128.0, MZ = 91.1876, MW = 80.4, GW = 2.1;
  const double sw2 = 1.0 - (MW / MZ) * (MW / MZ), rs = 13000.0, e2 = 4.0 * vg::kPi.v * alpha, g2 = e2 / sw2;
  k.conv = 0.3893794e9;
  k.pdfA = 1.0;
  k.pdfa = -0.5;
  k.pdfb = 3.0;
  k.pdf_pow = 1;
  k.pdf_a2 = -1;
  k.pdf_b = 3;
  k.invS = 1.0 / (rs * rs);
  k.M2 = MW * MW;
  k.MG = MW * GW;
  k.m2lo = 40.0 * 40.0;
  k.invMG = 1.0 / (MW * GW);
  k.tlo = (40.0 * 40.0 - MW * MW) / (MW * GW);
  k.rho_lo = std::atan(k.tlo.v);
  k.rho_rng = std::atan((rs * rs - MW * MW) / (MW * GW)) - k.rho_lo.v;
  k.g4v2_24 = g2 * g2 / 24.0;
  k.ptmin2 = 400.0;
  const double th = std::tanh(2.5);
  k.th2 = th * th;
  k.MG2 = k.MG.v * k.MG.v;
  k.MGt = k.MG.v * (1.0 + k.tlo.v * k.tlo.v);
  return k;
}
}  // namespace

// usage: count <process: ww_4l | ww_had | w_plus> <grid file: D lines of n + 1 edges> <events>
//              <atan> <log> <exp> <expm1> <tan> <sincos> <sqrt> <div>   (FP64 FLOPs per call)
int main(int argc, char** argv) {
  if (argc != 12) {
    std::fprintf(stderr, "usage: count process gridfile events atan log exp expm1 tan sincos sqrt div\n");
    return 2;
  }
  const std::string proc = argv[1];
  const bool had = proc == "ww_had", wp = proc == "w_plus";
  if (!had && !wp && proc != "ww_4l") return 2;
  const int D = had ? 10 : wp ? 4 : 8;
  std::vector<double> e;
  {
    FILE* fh = std::fopen(argv[2], "r");
    if (!fh) return 2;
    double v;
    while (std::fscanf(fh, "%lf", &v) == 1) e.push_back(v);
    std::fclose(fh);
  }
  const int n = static_cast<int>(e.size()) / D - 1;
  if (n < 2 || static_cast<int>(e.size()) != D * (n + 1)) return 2;
  const long nev = std::atol(argv[3]);
  fc::price_atan = std::atof(argv[4]);
  fc::price_log = std::atof(argv[5]);
  fc::price_exp = std::atof(argv[6]);
  fc::price_expm1 = std::atof(argv[7]);
  fc::price_tan = std::atof(argv[8]);
  fc::price_sincos = std::atof(argv[9]);
  fc::price_sqrt = std::atof(argv[10]);
  fc::price_div = std::atof(argv[11]);
  fc::price_sqrt_div = fc::price_sqrt + fc::price_div;  // a square root and its reciprocal
  const vg::PhysConst c = wp ? wplus_const() : ww_const(had);
  double per[4] = {0, 0, 0, 0};  // uniforms + grid map, integrand, weight + accumulation
  long nonzero = 0;
  std::mt19937_64 rng(1);
  for (long i = 0; i < nev; ++i) {
    F64 u[16], x[16];
    const double f0 = fc::g.flop;
    for (int d = 0; d < D; ++d) {
      u[d] = F64((static_cast<double>(rng() >> 12) + 0.5) * 0x1p-52, false);
      fc::g.flop += 1;  // (1 + w 2^-52) - (1 - 2^-53)
    }
    // the grid map as the kernel writes it: t = u n, k = floor(t) (at most n - 1),
    // delta = t - k, x = fma(delta, h, e_k), J = prod n h
    F64 J = 1.0;
    for (int d = 0; d < D; ++d) {
      const F64 t = u[d] * F64(static_cast<double>(n));
      int k = static_cast<int>(t.v);
      k = k > n - 1 ? n - 1 : k;
      const F64 delta = t - F64(k);
      const F64 lo = F64(e[d * (n + 1) + k], false), hi = F64(e[d * (n + 1) + k + 1], false);
      const F64 h = hi - lo;
      x[d] = __fma_rn(delta, h, lo);
      J = J * (F64(static_cast<double>(n)) * h);
    }
    const double f1 = fc::g.flop;
    F64 q;
    const F64 f = had ? vg::f_ww<F64, true>(c, x, q) : wp ? vg::f_w(c, x, q) : vg::f_ww<F64, false>(c, x, q);
    const double f2 = fc::g.flop;
    per[0] += f1 - f0;
    per[1] += f2 - f1;
    per[2] += 4 + D;  // w = J f; S1 += w; w^2; S2 += w^2; the D histogram additions
    if (f.v != 0.0) ++nonzero;
  }
  const double N = static_cast<double>(nev);
  std::printf("{\"process\": \"%s\", \"events\": %ld, \"nonzero\": %ld, \"uniforms_and_map\": %.4f, "
              "\"integrand\": %.4f, \"weight_and_sums\": %.4f, \"total\": %.4f, \"hw_estimates\": %.4f, "
              "\"library_calls\": %.4f}\n",
              proc.c_str(), nev, nonzero, per[0] / N, per[1] / N, per[2] / N, (per[0] + per[1] + per[2]) / N,
              fc::g.trans / N, fc::g.lib / N);
  return 0;
}
