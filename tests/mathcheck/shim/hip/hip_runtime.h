// Host stand-in for <hip/hip_runtime.h>, used only by the host accuracy check of the
// integrand headers' mathematical functions (tests/mathcheck/check.cpp): the device
// qualifiers become plain inline functions, binary64 stays binary64, and the hardware
// reciprocal / inverse-square-root estimates become the exact operations (the kernels
// refine the estimates by Newton steps to the same place).  Cross-lane builtins, which
// the checked functions do not use, act on one lane.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))
#define __builtin_amdgcn_bitop3_b32(a, b, c, imm) ((a) ^ (b) ^ (c))
#define __builtin_amdgcn_update_dpp(old, v, ctrl, rmask, bmask, bound) (v)
#define VG_OPAQUE_SGPR(x) (void)(x)
#define VG_PRICED(kind, x)
using std::copysign;
using std::exp;
using std::expm1;
using std::fabs;
using std::floor;
using std::fma;
using std::isfinite;
using std::ldexp;
using std::log;
using std::pow;
using std::rint;
using std::signbit;
using std::sqrt;
using std::trunc;
inline double __fma_rn(double a, double b, double c) { return std::fma(a, b, c); }
inline double __hiloint2double(int hi, int lo) {
  const uint64_t b = (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}
inline long long __double_as_longlong(double d) {
  long long b;
  std::memcpy(&b, &d, 8);
  return b;
}
inline double __longlong_as_double(long long b) {
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}
template <class T>
inline T __shfl_xor(T v, int, int) {
  return v;
}
inline void sincospif(float, float*, float*) {}
inline int __builtin_amdgcn_readlane(int v, int) { return v; }
