// device_common.hpp -- counter-based random numbers and exact fixed-point
// accumulation for the gfx950 VEGAS kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vg {

// a value held in a scalar register that the compiler must treat as rewritten at this
// point (so it is not hoisted across it); a host build of these headers that only
// counts arithmetic defines it away
#ifndef VG_OPAQUE_SGPR
#define VG_OPAQUE_SGPR(x) asm volatile("" : "+s"(x))
#endif

// marks a routine that evaluates a mathematical function (division, square root, tan,
// ...): nothing in the GPU build; the host build that counts the kernels' FLOPs prices
// the call at what the library's version of that function costs and does not count
// the routine's own operations
#ifndef VG_PRICED
#define VG_PRICED(kind, x)
#endif

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Every event owns its
// counter (event index, iteration, call), so the set of events of an iteration
// does not depend on how the launch splits the work -- the GPU form of handing
// each thread a fixed group of random numbers (paper Sec. 2.2).
// ---------------------------------------------------------------------------
struct u32x4 {
  uint32_t x, y, z, w;
};

// a ^ b ^ c in one instruction (v_bitop3_b32 with the truth table of a three-input xor)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return static_cast<uint32_t>(__builtin_amdgcn_bitop3_b32(a, b, c, 0x96));
}

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32 gives both halves)
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
    const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
    c = u32x4{xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// (hi:lo) -> odd multiple of 2^-53 in (0,1): top 52 bits w, value (2w+1) 2^-53.  The 52
// bits become the mantissa of 1 + w 2^-52 in [1, 2); subtracting 1 - 2^-53 (a binary64
// number) leaves (2w + 1) 2^-53 exactly, which is representable, so the one rounding is
// exact
__device__ __forceinline__ double words_to_unit(uint32_t hi, uint32_t lo) {
  const uint32_t mhi = 0x3ff00000u | (hi >> 12);
  const uint32_t mlo = (hi << 20) | (lo >> 12);
  const double one_w = __hiloint2double(static_cast<int>(mhi), static_cast<int>(mlo));
  return one_w - (1.0 - 0x1p-53);
}

// ndim uniforms of event `ev` in iteration `it`; call k fills u[2k], u[2k+1]
template <int D>
__device__ __forceinline__ void event_uniforms(uint64_t seed, uint32_t it, uint64_t ev, int ndim,
                                               double* u) {
  uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  // the key is the same for every event: an empty asm that claims to rewrite it keeps
  // the compiler from hoisting the ten round keys out of the event loop (twenty scalar
  // registers held across the integrand, spilled and read back lane by lane); formed
  // here they cost eighteen scalar additions per event, off the vector pipeline
  VG_OPAQUE_SGPR(k0);
  VG_OPAQUE_SGPR(k1);
  const int nd = D > 0 ? D : ndim;
#pragma unroll
  for (int k = 0; k < (D > 0 ? (D + 1) / 2 : 8); ++k) {
    if (D == 0 && 2 * k >= nd) break;
    const u32x4 o = philox4x32_10(
        u32x4{static_cast<uint32_t>(ev), static_cast<uint32_t>(ev >> 32), it, static_cast<uint32_t>(k)},
        k0, k1);
    u[2 * k] = words_to_unit(o.y, o.x);
    if (2 * k + 1 < nd) u[2 * k + 1] = words_to_unit(o.w, o.z);
  }
}

// ---------------------------------------------------------------------------
// binary64 reciprocal, square root and inverse square root from the hardware
// estimates (v_rcp_f64, v_rsq_f64) refined by Newton / Goldschmidt steps, without
// the scaling that the IEEE-exact library forms spend on subnormal, infinite and
// zero arguments (the callers' arguments are normal positive numbers, or zero where
// stated).  Each step squares the relative error of the estimate, so two steps
// from the hardware's estimate reach the binary64 rounding level; the results are
// within a few units in the last place of the correctly rounded ones (the event
// weights need 1e-12, not bit equality).
// ---------------------------------------------------------------------------
// 1 / d for normal d (either sign)
__device__ __forceinline__ double rcp_nr(double d) {
  VG_PRICED(div, d);
  double r = __builtin_amdgcn_rcp(d);
  double e = __fma_rn(-d, r, 1.0);
  r = __fma_rn(r, e, r);
  e = __fma_rn(-d, r, 1.0);
  return __fma_rn(r, e, r);
}

// n / d for normal d: n times the reciprocal, then one residual correction
__device__ __forceinline__ double div_nr(double n, double d) {
  VG_PRICED(div, d);
  const double r = rcp_nr(d);
  const double q = n * r;
  return __fma_rn(__fma_rn(-d, q, n), r, q);
}

// sqrt(a) and 1 / sqrt(a) for normal a > 0 (Goldschmidt: g -> sqrt(a), h -> 1/(2 sqrt(a)))
__device__ __forceinline__ void sqrt_rsqrt_nr(double a, double& g, double& inv) {
  VG_PRICED(sqrt_div, a);
  const double y = __builtin_amdgcn_rsq(a);
  g = a * y;
  double h = 0.5 * y;
  double r = __fma_rn(-h, g, 0.5);
  g = __fma_rn(g, r, g);
  h = __fma_rn(h, r, h);
  r = __fma_rn(-h, g, 0.5);
  g = __fma_rn(g, r, g);
  h = __fma_rn(h, r, h);
  const double d = __fma_rn(-g, g, a);
  g = __fma_rn(d, h, g);
  inv = h + h;
}

// sqrt(a) for a >= 0 (0 for a == 0)
__device__ __forceinline__ double sqrt_nr(double a) {
  VG_PRICED(sqrt, a);
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y;
  double h = 0.5 * y;
  const double r = __fma_rn(-h, g, 0.5);
  g = __fma_rn(g, r, g);
  h = __fma_rn(h, r, h);
  double d = __fma_rn(-g, g, a);
  g = __fma_rn(d, h, g);
  d = __fma_rn(-g, g, a);
  g = __fma_rn(d, h, g);
  return a > 0.0 ? g : 0.0;
}

// binary32: the hardware's single-precision forms
__device__ __forceinline__ float rcp_nr(float d) { return 1.0f / d; }
__device__ __forceinline__ float div_nr(float n, float d) { return n / d; }
__device__ __forceinline__ void sqrt_rsqrt_nr(float a, float& g, float& inv) {
  g = sqrtf(a);
  inv = 1.0f / g;
}
__device__ __forceinline__ float sqrt_nr(float a) { return sqrtf(a); }

// ---------------------------------------------------------------------------
// Exact fixed-point accumulation.  A value v with |v| < 2^E is represented as
// X = trunc(|v| 2^(94-E)) < 2^94, split into three 32-bit digits that are summed
// in int64 (signed digits for negative v).  Integer addition is associative,
// so any order of accumulation -- any block size, grid size or atomic order --
// gives the same bits.  For N < 2^31 addends no digit sum can overflow.
// ---------------------------------------------------------------------------
constexpr int FX_BITS = 94;

// exponent E with |v| < 2^E for the largest magnitude `vmax` (finite, >= 0)
__host__ __device__ __forceinline__ int fx_exponent(double vmax) {
  if (!(vmax > 0.0)) return 0;
  uint64_t b;
  __builtin_memcpy(&b, &vmax, sizeof(b));
  const int ex = static_cast<int>((b >> 52) & 0x7ff);
  if (ex == 0) return -1022;  // subnormal: below 2^-1022
  return ex - 1022;           // v < 2^(ex-1023+1)
}

// digits of v at scale 2^(94 - E) (|v| < 2^E): X = |v| 2^(94-E) is exact (a change
// of exponent), then X = d2 2^64 + d1 2^32 + d0 with every step exact in binary64
// (trunc, and fma of a product that is exactly representable); the magnitude's
// digits carry the sign of v.  Equal, digit for digit, to shifting the integer
// mantissa (and truncating the bits below 2^0).  Values at or above 2^E only occur
// at a scale the caller discards; X is clamped so the conversions stay defined.
__device__ __forceinline__ void fx_digits(double v, int E, long long& d0, long long& d1, long long& d2) {
  const double X = fmin(ldexp(fabs(v), FX_BITS - E), 0x1p95);
  const double h = trunc(X * 0x1p-64);
  const double r = __fma_rn(-h, 0x1p64, X);
  const double m = trunc(r * 0x1p-32);
  const double l = trunc(__fma_rn(-m, 0x1p32, r));
  long long a2 = static_cast<long long>(static_cast<uint32_t>(h));
  long long a1 = static_cast<long long>(static_cast<uint32_t>(m));
  long long a0 = static_cast<long long>(static_cast<uint32_t>(l));
  if (signbit(v)) {
    a0 = -a0;
    a1 = -a1;
    a2 = -a2;
  }
  d0 = a0;
  d1 = a1;
  d2 = a2;
}

// the same digits for a value known to be >= 0 (w^2 of a finite weight): no sign
__device__ __forceinline__ void fx_digits_pos(double v, int E, long long& d0, long long& d1, long long& d2) {
  const double X = fmin(ldexp(v, FX_BITS - E), 0x1p95);
  const double h = trunc(X * 0x1p-64);
  const double r = __fma_rn(-h, 0x1p64, X);
  const double m = trunc(r * 0x1p-32);
  const double l = trunc(__fma_rn(-m, 0x1p32, r));
  d2 = static_cast<long long>(static_cast<uint32_t>(h));
  d1 = static_cast<long long>(static_cast<uint32_t>(m));
  d0 = static_cast<long long>(static_cast<uint32_t>(l));
}

// w^2 takes four digits: Y = trunc(v 2^(126 - E)) < 2^126 (v < 2^E), the same exact
// splitting one digit further, so each event's w^2 is resolved to 2^-126 of 2^E -- 2^-94
// of the iteration's largest w^2 when the scale sits 2^32 above it -- and the totals of
// grid bins far below the largest keep their relative precision
constexpr int FX2_BITS = 126;

__device__ __forceinline__ void fx2_digits(double v, int E, long long h[4]) {
  const double X = fmin(ldexp(v, FX2_BITS - E), 0x1p127);
  const double t3 = trunc(X * 0x1p-96);
  const double r2 = __fma_rn(-t3, 0x1p96, X);
  const double t2 = trunc(r2 * 0x1p-64);
  const double r1 = __fma_rn(-t2, 0x1p64, r2);
  const double t1 = trunc(r1 * 0x1p-32);
  const double t0 = trunc(__fma_rn(-t1, 0x1p32, r1));
  h[3] = static_cast<long long>(static_cast<uint32_t>(t3));
  h[2] = static_cast<long long>(static_cast<uint32_t>(t2));
  h[1] = static_cast<long long>(static_cast<uint32_t>(t1));
  h[0] = static_cast<long long>(static_cast<uint32_t>(t0));
}

// digit sums -> double, (D2 2^64 + D1 2^32 + D0) 2^(E-94), after carry normalisation
__host__ __device__ __forceinline__ double fx_value(long long D0, long long D1, long long D2, int E) {
  long long c = D0 >> 32;  // arithmetic shift: floor division by 2^32
  D0 -= c * 4294967296LL;
  D1 += c;
  c = D1 >> 32;
  D1 -= c * 4294967296LL;
  D2 += c;
  const double low = static_cast<double>(D1) * 4294967296.0 + static_cast<double>(D0);
  const double v = static_cast<double>(D2) * 18446744073709551616.0 + low;
  return ldexp(v, E - FX_BITS);
}

// four digit sums -> double, (D3 2^96 + D2 2^64 + D1 2^32 + D0) 2^(E-126)
__host__ __device__ __forceinline__ double fx2_value(long long D0, long long D1, long long D2, long long D3, int E) {
  long long c = D0 >> 32;
  D0 -= c * 4294967296LL;
  D1 += c;
  c = D1 >> 32;
  D1 -= c * 4294967296LL;
  D2 += c;
  c = D2 >> 32;
  D2 -= c * 4294967296LL;
  D3 += c;
  const double low = static_cast<double>(D1) * 4294967296.0 + static_cast<double>(D0);
  const double high = static_cast<double>(D3) * 4294967296.0 + static_cast<double>(D2);
  return ldexp(high * 18446744073709551616.0 + low, E - FX2_BITS);
}

// ---------------------------------------------------------------------------
// wave64 reductions by DPP (row shifts 1, 2, 4, 8 within each row of 16 lanes, then
// row 0 into row 1 and row 2 into row 3, then rows 0-1 into rows 2-3): the moves stay in
// the VALU, where a butterfly's cross-lane permutes go through the LDS unit and wait
// for it.  Lane 63 ends with the total, which is read out for every lane (call with
// all 64 lanes active; integer sums and maxima are exact, so the order is free)
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROW_MASK, 0xf, BOUND);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(v >> 32), CTRL, ROW_MASK, 0xf, BOUND);
  return (static_cast<unsigned long long>(static_cast<unsigned int>(hi)) << 32) | static_cast<unsigned int>(lo);
}

__device__ __forceinline__ unsigned long long read_lane63_u64(unsigned long long v) {
  const unsigned int lo = __builtin_amdgcn_readlane(static_cast<int>(v), 63);
  const unsigned int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), 63);
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ long long wave_sum_i64(long long x) {
  unsigned long long v = static_cast<unsigned long long>(x);  // two's complement: wrap-around sums
  v += dpp_u64<0x111, 0xf, true>(v);
  v += dpp_u64<0x112, 0xf, true>(v);
  v += dpp_u64<0x114, 0xf, true>(v);
  v += dpp_u64<0x118, 0xf, true>(v);
  v += dpp_u64<0x142, 0xa, false>(v);
  v += dpp_u64<0x143, 0xc, false>(v);
  return static_cast<long long>(read_lane63_u64(v));
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  unsigned long long o;
  o = dpp_u64<0x111, 0xf, true>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x112, 0xf, true>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x114, 0xf, true>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x118, 0xf, true>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x142, 0xa, false>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x143, 0xc, false>(v);
  v = o > v ? o : v;
  return read_lane63_u64(v);
}

}  // namespace vg
