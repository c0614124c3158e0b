// device_common.hpp -- counter-based random numbers and exact fixed-point
// accumulation for the gfx950 VEGAS kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vg {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Every event owns its
// counter (event index, iteration, call), so the set of events of an iteration
// does not depend on how the launch splits the work -- the GPU form of handing
// each thread a fixed group of random numbers (paper Sec. 2.2).
// ---------------------------------------------------------------------------
struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32 gives both halves)
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c.z;
    const uint32_t lo0 = static_cast<uint32_t>(p0), hi0 = static_cast<uint32_t>(p0 >> 32);
    const uint32_t lo1 = static_cast<uint32_t>(p1), hi1 = static_cast<uint32_t>(p1 >> 32);
    c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// (hi:lo) -> odd multiple of 2^-53 in (0,1): top 52 bits w, value (2w+1) 2^-53, formed
// as hi 2^-32 + (lo >> 12) 2^-52 + 2^-53 -- disjoint bit ranges, so both fmas are exact
__device__ __forceinline__ double words_to_unit(uint32_t hi, uint32_t lo) {
  return __fma_rn(static_cast<double>(hi), 0x1p-32, __fma_rn(static_cast<double>(lo >> 12), 0x1p-52, 0x1p-53));
}

// ndim uniforms of event `ev` in iteration `it`; call k fills u[2k], u[2k+1]
template <int D>
__device__ __forceinline__ void event_uniforms(uint64_t seed, uint32_t it, uint64_t ev, int ndim,
                                               double* u) {
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
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

// ---------------------------------------------------------------------------
// wave64 reductions (butterfly over all 64 lanes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long wave_sum_i64(long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

}  // namespace vg
