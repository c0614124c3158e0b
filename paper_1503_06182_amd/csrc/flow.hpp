// flow.hpp -- learned proposal on the VEGAS y-space: a coupling-layer
// rational-quadratic spline flow (Durkan et al., Neural Spline Flows, 2019)
// with BF16 MFMA MLPs (FP32 accumulate) and FP32 splines, for gfx950.
//
// Layer l leaves its four conditioning coordinates unchanged and maps each of
// the four others by a monotone 16-bin rational-quadratic spline on [0,1]
// whose 47 parameters come from an MLP 4 -> 128 -> 128 -> 188 (ReLU) of the
// conditioning coordinates.  Density direction y -> z: layers 0..5, forward
// splines, log q(y) = sum log s'.  Sampling direction z -> y: layers 5..0,
// inverse splines.  Base density uniform on [0,1]^8.
//
// The forward kernels give each block (256 threads = 4 waves) tiles of 64
// events: the first layer of the MLP on v_mfma_f32_16x16x4_f32 (K = 4), the two
// 128-wide contractions on v_mfma_f32_16x16x32_bf16 (activations from LDS, the
// layer's weights held in each wave's registers for the whole launch; the density
// direction takes the activations as the A operand, the sampling direction the
// weights), the spline parameters rounded to binary16 in LDS, then one thread per
// (event, transformed coordinate) for the spline.  The backward kernel recomputes
// the density direction's MLP (tiles of 32, weights from global memory, the same
// MFMA sequence, so the same bits).
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vg {

constexpr int FL_NDIM = 8, FL_NB = 16, FL_NPAR = 47, FL_HID = 128, FL_NOUT = 188, FL_NOUTP = 192;
constexpr int FL_NLAYER = 6, FL_TILE = 32;
constexpr int FL_LAYER = 4 * FL_HID + FL_HID + FL_HID * FL_HID + FL_HID + FL_HID * FL_NOUT + FL_NOUT;  // 41404
constexpr int FL_NPARAMS = FL_NLAYER * FL_LAYER;                                                   // 248424
// offsets inside one layer of the FP32 master vector: W1 [4][128], b1, W2 [128][128], b2, W3 [128][188], b3
constexpr int FO_W1 = 0, FO_B1 = 512, FO_W2 = 640, FO_B2 = 17024, FO_W3 = 17152, FO_B3 = 41216;
// BF16 copies per layer: transposed (for the forward) W2t [128 out][128 in], W3t [192 out][128 in];
// natural (for the backward) W2n [128 in][128 out], W3n [128 in][192 out]; padded columns zero
constexpr int FB_W2T = 0, FB_W3T = 16384, FB_W2N = 16384 + 24576, FB_W3N = 2 * 16384 + 24576;
constexpr int FB_LAYER = 2 * 16384 + 2 * 24576;  // 81920 bf16 per layer
constexpr float FL_EPS = 1e-3f;
// LDS row strides: whole 16-byte units (the matrix-core operands are 16-byte loads),
// offset from a power of two against bank conflicts.  The activation tiles' stride is
// 72 four-byte words: on gfx950 the 16-byte fragment loads of 16 rows are free of bank
// conflicts when the stride in words is 8 modulo 16 (measured: two-way conflicts at
// 68, 76 or 84 words, eight-way at 64)
constexpr int FL_LDA = FL_HID + 16;  // bf16 activation tiles
constexpr int FL_LDP = FL_NOUTP + 8; // fp32 spline-parameter tile of the backward (and its bf16 gradient)
// spline-parameter tile of the forward kernels (binary16): coordinate c's 47 parameters at
// [56 c, 56 c + 47) of a 248-element row, so every spline's parameters start on a 16-byte
// boundary (a 16-byte LDS load that is not 16-byte aligned costs about 16 aligned ones on
// gfx950).  The row of 124 words keeps both the third layer's 8-byte stores and the
// splines' 16-byte loads at two-way bank conflicts at most (measured).
constexpr int FL_SPS = 56, FL_LDQ = 248;
constexpr int FL_TILE_F = 64;        // events per tile of the forward kernels
constexpr float FL_DSHIFT = 0.53974242f;  // log(expm1(1 - eps)) for eps = 1e-3: raw 0 gives derivative 1

// transformed coordinates of each layer (the conditioning coordinates are the rest, in order)
__device__ __constant__ const int kFlowX[FL_NLAYER][4] = {{4, 5, 6, 7}, {0, 1, 2, 3}, {1, 3, 5, 7},
                                                           {0, 2, 4, 6}, {2, 3, 6, 7}, {0, 1, 4, 5}};
__device__ __constant__ const int kFlowC[FL_NLAYER][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 2, 4, 6},
                                                           {1, 3, 5, 7}, {0, 1, 4, 5}, {2, 3, 6, 7}};

typedef __bf16 __attribute__((ext_vector_type(8))) bf16x8_t;
typedef float __attribute__((ext_vector_type(4))) f32x4_t;

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even (v_cvt_pk_bf16_f32 on gfx950)
  const __hip_bfloat16 b = __float2bfloat16(f);
  return *reinterpret_cast<const uint16_t*>(&b);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }
// spline parameters are rounded to binary16 (round to nearest even) in both directions
__device__ __forceinline__ float round_h(float x) { return static_cast<float>(static_cast<_Float16>(x)); }

// Output slots of a wave's two 16-unit tiles t = 0, 1 over its 32 units [32 w, 32 w + 32):
// slot s of tile t is unit 32 w + 8 (s / 4) + 4 t + s % 4, so the lanes of group
// g = l / 16, which receive slots 4 g .. 4 g + 3 of both tiles, hold the 8 consecutive
// units 32 w + 8 g .. + 7 of their event and store them in one 16-byte write.
__device__ __forceinline__ int pair_unit(int wave, int t, int s) { return 32 * wave + 8 * (s >> 2) + 4 * t + (s & 3); }

// first MLP layer on the matrix cores, binary32 (K = the 4 conditioning inputs), by a
// block of 4 waves: wave w computes hidden units [32 w, 32 w + 32) as two 16-unit tiles.
// Tile (t, event rows r0 .. r0+15): h1^T = W1^T cond^T + b1 on v_mfma_f32_16x16x4_f32 --
// lane l supplies W1[l/16][unit of slot l%16] (A) and cond[r0 + l%16][l/16] (B), starts
// from the biases of its four slots and receives those four units of event r0 + l%16.
struct H1Frag {
  float w[2], b[2][4];
};

__device__ __forceinline__ H1Frag load_h1_frag(const float* __restrict__ m, int wave, int lane) {
  H1Frag f;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    f.w[t] = m[FO_W1 + (lane >> 4) * FL_HID + pair_unit(wave, t, lane & 15)];
#pragma unroll
    for (int j = 0; j < 4; ++j) f.b[t][j] = m[FO_B1 + pair_unit(wave, t, 4 * (lane >> 4) + j)];
  }
  return f;
}

typedef float __attribute__((ext_vector_type(2))) f32x2_t;
typedef __bf16 __attribute__((ext_vector_type(2))) bf16x2_t;
typedef _Float16 __attribute__((ext_vector_type(2))) f16x2_t;
typedef short __attribute__((ext_vector_type(2))) i16x2_t;

// max(round_bf16(a), 0), max(round_bf16(b), 0) in one word (v_cvt_pk_bf16_f32, then
// v_pk_max_i16 on the bit patterns: a bfloat16 with the sign bit set is a negative
// 16-bit integer, so the integer maximum with 0 is the ReLU).  Rounding to nearest
// keeps the sign and ReLU(x) is 0 or x, so this equals the rounding of max(x, 0)
// bit for bit for every x but a NaN (a negative x gives +0 either way).
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
  const f32x2_t v = {a, b};
  const i16x2_t r = __builtin_bit_cast(i16x2_t, __builtin_convertvector(v, bf16x2_t));
  const i16x2_t z = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(r, z));
}

// the ReLU of the four values of a0, then of a1, as eight bf16 in one 16-byte word
__device__ __forceinline__ uint4 pack_relu_bf16x8(f32x4_t a0, f32x4_t a1) {
  return make_uint4(relu_bf16x2(a0[0], a0[1]), relu_bf16x2(a0[2], a0[3]), relu_bf16x2(a1[0], a1[1]),
                    relu_bf16x2(a1[2], a1[3]));
}

// two binary32 values -> two binary16 (round to nearest even, v_cvt_pk_f16_f32) in one word
__device__ __forceinline__ uint32_t pack_f16x2(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2_t));
}

// h1 of `rows` events (a multiple of 16; cond [rows][4] in LDS) -> bf16 in LDS (stride
// FL_LDA); every kernel runs this same sequence, so h1 has the same bits everywhere
__device__ __forceinline__ void mlp_h1(const H1Frag& f, const float (*cond)[4], uint16_t* h1, int rows) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r0 = 0; r0 < rows; r0 += 16) {
    const float c = cond[r0 + (lane & 15)][lane >> 4];
    f32x4_t a0 = {f.b[0][0], f.b[0][1], f.b[0][2], f.b[0][3]};
    f32x4_t a1 = {f.b[1][0], f.b[1][1], f.b[1][2], f.b[1][3]};
    a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(f.w[0], c, a0, 0, 0, 0);
    a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(f.w[1], c, a1, 0, 0, 0);
    *reinterpret_cast<uint4*>(h1 + (r0 + (lane & 15)) * FL_LDA + 32 * wave + 8 * (lane >> 4)) =
        pack_relu_bf16x8(a0, a1);
  }
}

// One 16x16x32 step: lane l supplies A[r0 + l%16][k0 + 8(l/16) .. +7] and
// Bt[c0 + l%16][k0 + 8(l/16) .. +7] (one 16-byte load each) and receives
// acc[j] = C[r0 + 4(l/16) + j][c0 + l%16].  The instruction sums over all 32 k of
// the step; A and B supply them in the same lane order, so which k the hardware
// pairs inside a lane group is immaterial.
__device__ __forceinline__ bf16x8_t load_bfrag(const uint16_t* __restrict__ Bt, int ldb, int c0, int k0, int lane) {
  return *reinterpret_cast<const bf16x8_t*>(Bt + static_cast<int64_t>(c0 + (lane & 15)) * ldb + k0 + 8 * (lane >> 4));
}

__device__ __forceinline__ f32x4_t mfma_step(bf16x8_t a, bf16x8_t b, f32x4_t acc) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

// C(16x16 at r0, c0) = sum_k A[r][k] Bt[c][k] over K (a multiple of 32): A rows in LDS
// (stride lda, bf16), Bt rows in global memory (stride ldb, bf16); strides and k
// offsets are multiples of 8 elements (16-byte loads).
__device__ __forceinline__ f32x4_t mfma_rowcol(const uint16_t* A, int lda, const uint16_t* __restrict__ Bt, int ldb,
                                               int r0, int c0, int K, int lane) {
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  const int ri = lane & 15, kq = 8 * (lane >> 4);
  const uint16_t* ap = A + (r0 + ri) * lda + kq;
  const uint16_t* bp = Bt + static_cast<int64_t>(c0 + ri) * ldb + kq;
  for (int k0 = 0; k0 < K; k0 += 32) {
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(ap + k0);
    const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(bp + k0);
    acc = mfma_step(a, b, acc);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// rational-quadratic spline on [0,1], 16 bins, boundary derivatives 1.
// Fast single-precision exp / log / reciprocal throughout; the forward and
// inverse evaluations and the knot construction of the backward use the same
// operations in the same order, so the backward differentiates exactly the
// function the forward evaluated.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fexp(float x) { return __expf(x); }
__device__ __forceinline__ float flog(float x) { return __logf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float softplus_f(float z) { return z > 20.f ? z : flog(1.f + fexp(z)); }
// knot i (0 < i < 16) of the partition whose bins are eps + (1 - 16 eps) softmax(r):
// i eps + (1 - 16 eps) S_i / S_16, S_i = e_0 + ... + e_{i-1} the partial sums of the
// softmax numerators, with c = (1 - 16 eps) / S_16 (the same function as the running
// sum of the bin widths, one rounding per knot); knots 0 and 16 are 0 and 1 exactly
constexpr float FL_KSCALE = 1.f - FL_NB * FL_EPS;
__device__ __forceinline__ float knot_at(float S, float c, int i) { return __fmaf_rn(S, c, static_cast<float>(i) * FL_EPS); }

// the four numbers of the rational-quadratic map on one bin, and its evaluation
struct Bin {
  float x0, x1, y0, y1, d0, d1;
};

__device__ __forceinline__ float rq_forward(const Bin& q, float x, float& ld) {
  const float w = q.x1 - q.x0, h = q.y1 - q.y0;
  const float iw = frcp(w);
  const float s = h * iw;
  const float xi = (x - q.x0) * iw, t = xi * (1.f - xi);
  const float den = s + (q.d1 + q.d0 - 2.f * s) * t;
  const float iden = frcp(den);
  const float y = q.y0 + h * (s * xi * xi + q.d0 * t) * iden;
  const float P = q.d1 * xi * xi + 2.f * s * t + q.d0 * (1.f - xi) * (1.f - xi);
  ld = flog(s * s * P * iden * iden);
  return y;
}

__device__ __forceinline__ float rq_inverse(const Bin& q, float y, float& ld) {
  const float w = q.x1 - q.x0, h = q.y1 - q.y0;
  const float s = h * frcp(w);
  const float dy = y - q.y0;
  const float g = q.d1 + q.d0 - 2.f * s;
  const float a = h * (s - q.d0) + dy * g;
  const float b = h * q.d0 - dy * g;
  const float c = -s * dy;
  const float disc = fmaxf(b * b - 4.f * a * c, 0.f);
  float xi = 2.f * c * frcp(-b - sqrtf(disc));
  xi = fminf(fmaxf(xi, 0.f), 1.f);
  const float x = q.x0 + xi * w;
  const float t = xi * (1.f - xi);
  const float iden = frcp(s + g * t);
  const float P = q.d1 * xi * xi + 2.f * s * t + q.d0 * (1.f - xi) * (1.f - xi);
  ld = flog(s * s * P * iden * iden);
  return x;
}

// largest of 16 logits (binary16 in LDS: packed three-operand maxima, v_pk_maximum3_f16, exact)
__device__ __forceinline__ float max16(const _Float16* r) {
  f16x2_t m[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const f16x2_t a = {r[4 * i], r[4 * i + 1]}, b = {r[4 * i + 2], r[4 * i + 3]};
    m[i] = __builtin_elementwise_maximum(a, b);
  }
  const f16x2_t t = __builtin_elementwise_maximum(__builtin_elementwise_maximum(m[0], m[1]),
                                                  __builtin_elementwise_maximum(m[2], m[3]));
  return static_cast<float>(__builtin_elementwise_maximum(t.x, t.y));
}
__device__ __forceinline__ float max16(const float* r) {
  float m = r[0];
#pragma unroll
  for (int i = 1; i < FL_NB; ++i) m = fmaxf(m, r[i]);
  return m;
}

// softmax numerators e_i = exp(r_i - max r) of 16 logits, as exp2(r_i log2 e - max r log2 e)
// (one fused multiply-add per logit: the common rounding of max r log2 e scales every
// numerator alike and cancels in the ratios), and their partial sums S[i] = e_0 + ... +
// e_{i-1}, accumulated left to right (S[16] the sum)
template <typename T>
__device__ __forceinline__ void softmax16(const T* r, float* e, float* S) {
  constexpr float kLog2e = 1.44269504088896341f;
  const float nm = -max16(r) * kLog2e;
  S[0] = 0.f;
#pragma unroll
  for (int i = 0; i < FL_NB; ++i) {
    e[i] = __builtin_amdgcn_exp2f(__fmaf_rn(static_cast<float>(r[i]), kLog2e, nm));
    S[i + 1] = S[i] + e[i];
  }
}

// spline of one coordinate from its 47 parameters (forward: x -> y; INV: y -> x) and
// log s' of the forward map; the bin k is the number of interior knots below v (of the
// x knots forward, of the y knots inverse).  The knots below v form a prefix of 1..15,
// so the last one below v is knot k and the one after it knot k + 1.
template <bool INV, typename T>
__device__ __forceinline__ float spline_eval(const T* p, float v, float& ld) {
  float ew[FL_NB], eh[FL_NB], Sw[FL_NB + 1], Sh[FL_NB + 1];
  softmax16(p, ew, Sw);
  softmax16(p + FL_NB, eh, Sh);
  const float cw = FL_KSCALE * frcp(Sw[FL_NB]), ch = FL_KSCALE * frcp(Sh[FL_NB]);
  float xk[FL_NB + 1], yk[FL_NB + 1];
  xk[0] = yk[0] = 0.f;
  xk[FL_NB] = yk[FL_NB] = 1.f;
#pragma unroll
  for (int i = 1; i < FL_NB; ++i) {
    xk[i] = knot_at(Sw[i], cw, i);
    yk[i] = knot_at(Sh[i], ch, i);
  }
  Bin q{0.f, xk[1], 0.f, yk[1], 1.f, 1.f};
  int k = 0;
#pragma unroll
  for (int i = 1; i < FL_NB; ++i) {
    const bool below = (INV ? yk[i] : xk[i]) < v;
    q.x0 = below ? xk[i] : q.x0;
    q.x1 = below ? xk[i + 1] : q.x1;
    q.y0 = below ? yk[i] : q.y0;
    q.y1 = below ? yk[i + 1] : q.y1;
    k = below ? i : k;
  }
  q.d0 = k == 0 ? 1.f : FL_EPS + softplus_f(static_cast<float>(p[2 * FL_NB + k - 1]) + FL_DSHIFT);
  q.d1 = k == FL_NB - 1 ? 1.f : FL_EPS + softplus_f(static_cast<float>(p[2 * FL_NB + k]) + FL_DSHIFT);
  return INV ? rq_inverse(q, v, ld) : rq_forward(q, v, ld);
}

// knots of the backward (all 17 of each kind and the softmax outputs)
struct Knots {
  float xk[FL_NB + 1], yk[FL_NB + 1], dk[FL_NB + 1];
  float pw[FL_NB], ph[FL_NB];  // softmax outputs
};

__device__ __forceinline__ void make_knots(const float* raw, Knots& K) {
  float ew[FL_NB], eh[FL_NB], Sw[FL_NB + 1], Sh[FL_NB + 1];
  softmax16(raw, ew, Sw);
  softmax16(raw + FL_NB, eh, Sh);
  const float iw = frcp(Sw[FL_NB]), ih = frcp(Sh[FL_NB]);
  const float cw = FL_KSCALE * iw, ch = FL_KSCALE * ih;
  K.xk[0] = 0.f;
  K.yk[0] = 0.f;
  K.xk[FL_NB] = 1.f;
  K.yk[FL_NB] = 1.f;
#pragma unroll
  for (int i = 0; i < FL_NB; ++i) {
    K.pw[i] = ew[i] * iw;
    K.ph[i] = eh[i] * ih;
  }
#pragma unroll
  for (int i = 1; i < FL_NB; ++i) {
    K.xk[i] = knot_at(Sw[i], cw, i);
    K.yk[i] = knot_at(Sh[i], ch, i);
  }
  K.dk[0] = 1.f;
  K.dk[FL_NB] = 1.f;
#pragma unroll
  for (int i = 1; i < FL_NB; ++i) K.dk[i] = FL_EPS + softplus_f(raw[2 * FL_NB + i - 1] + FL_DSHIFT);
}

// bin of x among the x knots 1..15 (number of them below x), and its numbers
__device__ __forceinline__ int knot_bin(const float* t, float v) {
  int k = 0;
#pragma unroll
  for (int i = 1; i < FL_NB; ++i) k += (t[i] < v) ? 1 : 0;
  return k;
}

__device__ __forceinline__ Bin pick_bin(const Knots& K, int k) {
  Bin b{K.xk[0], K.xk[1], K.yk[0], K.yk[1], K.dk[0], K.dk[1]};
#pragma unroll
  for (int i = 1; i < FL_NB; ++i)
    if (i == k) b = Bin{K.xk[i], K.xk[i + 1], K.yk[i], K.yk[i + 1], K.dk[i], K.dk[i + 1]};
  return b;
}

// reverse sweep of (y, log s') = spline(x; raw): given ybar and ldbar, returns xbar and
// writes rawbar[47]
__device__ __forceinline__ float rqs_bwd(const float* raw, const Knots& K, float x, float ybar, float ldbar,
                                         float* rawbar) {
  const int k = knot_bin(K.xk, x);
  const Bin q = pick_bin(K, k);
  const float w = q.x1 - q.x0, h = q.y1 - q.y0;
  const float s = h / w, d0 = q.d0, d1 = q.d1;
  const float xi = (x - q.x0) / w, t = xi * (1.f - xi);
  const float g = d1 + d0 - 2.f * s;
  const float den = s + g * t;
  const float num = s * xi * xi + d0 * t;
  const float omx = 1.f - xi;
  const float P = d1 * xi * xi + 2.f * s * t + d0 * omx * omx;
  float sb = 0.f, tb = 0.f, xib = 0.f, d0b = 0.f, d1b = 0.f, denb = 0.f, hb = 0.f, wb = 0.f, ykb = 0.f, xkb = 0.f;
  // ld = 2 log s + log P - 2 log den
  sb += ldbar * 2.f / s;
  const float Pb = ldbar / P;
  denb += -2.f * ldbar / den;
  d1b += Pb * xi * xi;
  sb += Pb * 2.f * t;
  tb += Pb * 2.f * s;
  d0b += Pb * omx * omx;
  xib += Pb * (2.f * d1 * xi - 2.f * d0 * omx);
  // y = y_k + h num / den
  ykb += ybar;
  hb += ybar * num / den;
  const float numb = ybar * h / den;
  denb += -ybar * h * num / (den * den);
  sb += numb * xi * xi;
  xib += numb * 2.f * s * xi;
  d0b += numb * t;
  tb += numb * d0;
  // den = s + (d1 + d0 - 2 s) t
  sb += denb * (1.f - 2.f * t);
  d1b += denb * t;
  d0b += denb * t;
  tb += denb * g;
  // t = xi (1 - xi)
  xib += tb * (1.f - 2.f * xi);
  // xi = (x - x_k) / w
  const float xbar = xib / w;
  xkb += -xib / w;
  wb += -xib * xi / w;
  // s = h / w
  hb += sb / w;
  wb += -sb * h / (w * w);
  // w = x_{k+1} - x_k, h = y_{k+1} - y_k; x_j = sum_{i<j} width_i for j <= 15 (x_16 = 1 fixed)
  const float xk1b = (k + 1 < FL_NB) ? wb : 0.f, yk1b = (k + 1 < FL_NB) ? hb : 0.f;
  xkb -= wb;
  ykb -= hb;
  // widths_i = eps + (1 - 16 eps) softmax_i: raw bar_j = p_j (pbar_j - sum_i p_i pbar_i)
  const float scale = 1.f - FL_NB * FL_EPS;
  float wib[FL_NB], hib[FL_NB];
  float dotw = 0.f, doth = 0.f;
#pragma unroll
  for (int i = 0; i < FL_NB; ++i) {
    wib[i] = scale * ((i < k ? xkb : 0.f) + (i < k + 1 ? xk1b : 0.f));
    hib[i] = scale * ((i < k ? ykb : 0.f) + (i < k + 1 ? yk1b : 0.f));
    dotw += K.pw[i] * wib[i];
    doth += K.ph[i] * hib[i];
  }
#pragma unroll
  for (int i = 0; i < FL_NB; ++i) {
    rawbar[i] = K.pw[i] * (wib[i] - dotw);
    rawbar[FL_NB + i] = K.ph[i] * (hib[i] - doth);
  }
  // interior derivatives d_j = eps + softplus(raw_{32 + j - 1} + shift), j = 1..15
#pragma unroll
  for (int j = 1; j < FL_NB; ++j) {
    const float z = raw[2 * FL_NB + j - 1] + FL_DSHIFT;
    const float sig = z > 20.f ? 1.f : frcp(1.f + fexp(-z));  // d softplus / dz (softplus_f is z above 20)
    const float db = (j == k ? d0b : 0.f) + (j == k + 1 ? d1b : 0.f);
    rawbar[2 * FL_NB + j - 1] = db * sig;
  }
  return xbar;
}

}  // namespace vg
