// flow.hip -- kernels and C ABI of the learned proposal (see flow.hpp).
//
// Training step on a batch of VEGAS-weighted events (y_i, w_i), loss
// L = -sum_i w_i log q(y_i) / sum_i w_i (importance-weighted forward KL):
//   gather (a per-step bijection of the data indices), per-layer forward in the
//   density direction (activations of every layer kept), the per-event loss
//   seeds dL/dlog q_i = -w_i / sum w, per-layer backward (spline reverse sweep,
//   MLP backward on MFMA), weight gradients as MFMA contractions over the
//   batch, Adam on the FP32 master weights, BF16 copies refreshed.
// Sampling: z uniform (Philox) -> inverse layers 5..0 -> y, log q(y).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "device_common.hpp"
#include "flow.hpp"
#include "vegas.h"

namespace vg {

// ---------------------------------------------------------------------------
// FP32 master -> BF16 copies (transposed and natural), padded columns zero
// ---------------------------------------------------------------------------
__global__ void k_flow_prep(const float* __restrict__ master, uint16_t* __restrict__ wb) {
  const int l = blockIdx.y;
  const float* m = master + l * FL_LAYER;
  uint16_t* o = wb + static_cast<int64_t>(l) * FB_LAYER;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < FB_LAYER; i += gridDim.x * blockDim.x) {
    float v;
    if (i < FB_W3T) {  // W2t[out][in]
      const int out = i / FL_HID, in = i % FL_HID;
      v = m[FO_W2 + in * FL_HID + out];
    } else if (i < FB_W2N) {  // W3t[out][in], out < 192
      const int j = i - FB_W3T, out = j / FL_HID, in = j % FL_HID;
      v = out < FL_NOUT ? m[FO_W3 + in * FL_NOUT + out] : 0.f;
    } else if (i < FB_W3N) {  // W2n[in][out]
      v = m[FO_W2 + (i - FB_W2N)];
    } else {  // W3n[in][out], out < 192
      const int j = i - FB_W3N, in = j / FL_NOUTP, out = j % FL_NOUTP;
      v = out < FL_NOUT ? m[FO_W3 + in * FL_NOUT + out] : 0.f;
    }
    o[i] = f2bf(v);
  }
}

// He-uniform hidden layers from a Philox stream keyed by (seed, parameter index),
// zero output layer and biases: the initial flow is the identity (q = 1)
__global__ void k_flow_init(float* master, uint64_t seed) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < FL_NPARAMS; i += gridDim.x * blockDim.x) {
    const int off = i % FL_LAYER;
    float v = 0.f;
    if (off < FO_B1 || (off >= FO_W2 && off < FO_B2)) {
      const u32x4 r = philox4x32_10(u32x4{static_cast<uint32_t>(i), 0u, 0xF10Fu, 0u}, static_cast<uint32_t>(seed),
                                    static_cast<uint32_t>(seed >> 32));
      const float u = (static_cast<float>(r.x >> 8) + 0.5f) * (1.f / 16777216.f);
      const float bound = off < FO_B1 ? sqrtf(6.f / 4.f) : sqrtf(6.f / FL_HID);
      v = (2.f * u - 1.f) * bound;
    }
    master[i] = v;
  }
}

// ---------------------------------------------------------------------------
// MLP of one 32-event tile for the backward: cond (LDS [32][4]) -> h1, h2 (LDS bf16)
// -> spline parameters (LDS, binary32 holding the binary16-rounded values).  B comes
// from global memory; the MFMA sequence per output tile is the forward kernel's, so
// every value equals the forward's bit for bit.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mlp_tile32(const float* __restrict__ m, const uint16_t* __restrict__ w,
                                           const float (*cond)[4], uint16_t* h1, uint16_t* h2, float* par) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  mlp_h1(load_h1_frag(m, wave, lane), cond, h1, FL_TILE);
  __syncthreads();
  // h2: 2 row blocks x 8 column blocks; wave w owns column blocks 2w, 2w+1
  for (int rb = 0; rb < 2; ++rb)
    for (int cc = 0; cc < 2; ++cc) {
      const int cb = 2 * wave + cc;
      const f32x4_t acc = mfma_rowcol(h1, FL_LDA, w + FB_W2T, FL_HID, rb * 16, cb * 16, FL_HID, lane);
      const int col = cb * 16 + (lane & 15);
      const float bias = m[FO_B2 + col];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + 4 * (lane >> 4) + j;
        h2[row * FL_LDA + col] = f2bf(fmaxf(acc[j] + bias, 0.f));
      }
    }
  __syncthreads();
  // spline parameters: 2 row blocks x 12 column blocks; wave w owns column blocks 3w..3w+2
  for (int rb = 0; rb < 2; ++rb)
    for (int cc = 0; cc < 3; ++cc) {
      const int cb = 3 * wave + cc;
      const f32x4_t acc = mfma_rowcol(h2, FL_LDA, w + FB_W3T, FL_HID, rb * 16, cb * 16, FL_HID, lane);
      const int col = cb * 16 + (lane & 15);
      const float bias = col < FL_NOUT ? m[FO_B3 + col] : 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + 4 * (lane >> 4) + j;
        par[row * FL_LDP + col] = round_h(acc[j] + bias);
      }
    }
  __syncthreads();
}

// x of lane i ^ 1 (CTRL 0xB1) or i ^ 2 (0x4E) within each group of four lanes (DPP quad_perm)
template <int CTRL>
__device__ __forceinline__ float quad_xor(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

// one coupling layer over a batch; SAMPLE: inverse splines (z -> y), else forward (y -> z).
// vout may alias vin.  logq[i] += sum of log s' of the four transformed coordinates.
// Tiles of 64 events; each wave keeps the weight fragments of its output units (W2: 2
// blocks of 16, W3: 3) for all eight k-steps in registers for the whole launch.
template <bool SAMPLE>
__global__ __launch_bounds__(256, 3) void k_flow_layer(const float* __restrict__ master,
                                                        const uint16_t* __restrict__ wb, int l, const float* vin,
                                                        float* vout, float* logq, int64_t B) {
  // h1 is dead once the second layer has run (a barrier follows it), so the spline
  // parameters the third layer writes share its space: 52 KB per block, 3 blocks per CU
  static_assert(FL_TILE_F * FL_LDQ * sizeof(_Float16) >= FL_TILE_F * FL_LDA * sizeof(uint16_t), "h1 / par union");
  __shared__ float cond[FL_TILE_F][4];
  __shared__ __align__(16) _Float16 h1_par[FL_TILE_F * FL_LDQ];
  __shared__ __align__(16) uint16_t h2[FL_TILE_F * FL_LDA];
  uint16_t* const h1 = reinterpret_cast<uint16_t*>(h1_par);
  _Float16* const par = h1_par;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float* m = master + l * FL_LAYER;
  const uint16_t* w = wb + static_cast<int64_t>(l) * FB_LAYER;
  bf16x8_t b2[2][FL_HID / 32], b3[3][FL_HID / 32];
  // second layer: forward, output columns (2 w + cc) 16 + lane % 16; sampling, the units
  // of the paired-tile order (the lanes of a group receive 8 consecutive units of an event)
#pragma unroll
  for (int cc = 0; cc < 2; ++cc) {
    const int row = SAMPLE ? pair_unit(wave, cc, lane & 15) : (2 * wave + cc) * 16 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < FL_HID / 32; ++ks)
      b2[cc][ks] = *reinterpret_cast<const bf16x8_t*>(w + FB_W2T + row * FL_HID + ks * 32 + 8 * (lane >> 4));
  }
  // third layer: forward, output columns 48 w .. 48 w + 47 in the parameters' order;
  // sampling, the 47 parameters of coordinate w (the 48th slot takes zero row 188 of the
  // padded copy), so that wave w's outputs are exactly the parameters of the spline of
  // coordinate w: tiles 0 and 1 give parameters 0 .. 31 in the paired-tile order,
  // tile 2 parameters 32 .. 47 in order
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const int s = lane & 15;
    const int slot = cc < 2 ? 8 * (s >> 2) + 4 * cc + (s & 3) : 32 + s;
    const int row = SAMPLE ? (slot < FL_NPAR ? wave * FL_NPAR + slot : FL_NOUT) : 48 * wave + 16 * cc + s;
#pragma unroll
    for (int ks = 0; ks < FL_HID / 32; ++ks)
      b3[cc][ks] = *reinterpret_cast<const bf16x8_t*>(w + FB_W3T + row * FL_HID + ks * 32 + 8 * (lane >> 4));
  }
  // biases: forward, of the lane's output column (C = A Bt with the activations as A),
  // in registers; sampling, of the lane's four output rows (C^T = Bt^T A^T: the
  // weights are the A operand, so a lane receives four consecutive outputs of one
  // event, eight over a pair of tiles, stored in one 16-byte write), read from LDS as
  // the accumulators' initial values (registers held through the splines would spill)
  __shared__ __align__(16) float bias_s[SAMPLE ? FL_HID + FL_NOUTP : 1];
  float bias2[2], bias3[3];
  if constexpr (SAMPLE) {
    for (int i = tid; i < FL_HID + FL_NOUTP; i += blockDim.x) {
      const int c = (i - FL_HID) / 48, slot = (i - FL_HID) % 48;
      bias_s[i] = i < FL_HID ? m[FO_B2 + i] : (slot < FL_NPAR ? m[FO_B3 + c * FL_NPAR + slot] : 0.f);
    }
  } else {
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) bias2[cc] = m[FO_B2 + (2 * wave + cc) * 16 + (lane & 15)];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const int col = (3 * wave + cc) * 16 + (lane & 15);
      bias3[cc] = col < FL_NOUT ? m[FO_B3 + col] : 0.f;
    }
  }
  const H1Frag u1 = load_h1_frag(m, wave, lane);
  const int ri = lane & 15, kq = 4 * (lane >> 4), kq8 = 8 * (lane >> 4);
  // thread (event e, slot c) of a tile: its conditioning input c goes to LDS, and it
  // transforms coordinate kFlowX[l][c] after the MLP.  Both inputs of the next tile are
  // loaded while the current one runs (tiles hold disjoint events, so an in-place
  // layer's stores never touch them).
  const int e = tid >> 2, c = tid & 3;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * FL_TILE_F;
  const int xc = kFlowX[l][c], cc_in = kFlowC[l][c];
  int64_t e0 = static_cast<int64_t>(blockIdx.x) * FL_TILE_F;
  float cn = 0.5f, vn = 0.f;
  if (e0 + e < B) {
    cn = vin[(e0 + e) * FL_NDIM + cc_in];
    vn = vin[(e0 + e) * FL_NDIM + xc];
  }
  for (; e0 < B; e0 += stride) {
    const int64_t ev = e0 + e;
    cond[e][c] = cn;
    const float vx = vn;
    if (ev + stride < B) {
      cn = vin[(ev + stride) * FL_NDIM + cc_in];
      vn = vin[(ev + stride) * FL_NDIM + xc];
    }
    __syncthreads();
    // the three products run at a raised wave priority and the splines at the base one:
    // a SIMD then issues the products of one block's waves ahead of another block's
    // spline work, which keeps the co-resident blocks in different phases, the matrix
    // cores busy beside the vector ALUs (measured 9 % faster than equal priorities, and
    // 5 % faster than the reverse order)
    __builtin_amdgcn_s_setprio(2);
    mlp_h1(u1, cond, h1, FL_TILE_F);
    __syncthreads();
    if constexpr (SAMPLE) {
      // the bias is the accumulators' initial value (the lane's slots' biases, read
      // once per layer and tile); ReLU and the bfloat16 rounding on pairs
      // (v_cvt_pk_bf16_f32, v_pk_max_i16)
      const f32x4_t bb2[2] = {*reinterpret_cast<const f32x4_t*>(bias_s + 32 * wave + 2 * kq),
                              *reinterpret_cast<const f32x4_t*>(bias_s + 32 * wave + 2 * kq + 4)};
#pragma unroll
      for (int rb = 0; rb < FL_TILE_F / 16; ++rb) {
        f32x4_t acc[2];
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          acc[cc] = bb2[cc];
#pragma unroll
          for (int ks = 0; ks < FL_HID / 32; ++ks) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(h1 + (rb * 16 + ri) * FL_LDA + ks * 32 + kq8);
            acc[cc] = mfma_step(b2[cc][ks], a, acc[cc]);
          }
        }
        *reinterpret_cast<uint4*>(h2 + (rb * 16 + ri) * FL_LDA + 32 * wave + 2 * kq) = pack_relu_bf16x8(acc[0], acc[1]);
      }
      __syncthreads();
      const f32x4_t bb3[3] = {*reinterpret_cast<const f32x4_t*>(bias_s + FL_HID + 48 * wave + 2 * kq),
                              *reinterpret_cast<const f32x4_t*>(bias_s + FL_HID + 48 * wave + 2 * kq + 4),
                              *reinterpret_cast<const f32x4_t*>(bias_s + FL_HID + 48 * wave + 32 + kq)};
#pragma unroll
      for (int rb = 0; rb < FL_TILE_F / 16; ++rb) {
        f32x4_t acc[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          acc[cc] = bb3[cc];
#pragma unroll
          for (int ks = 0; ks < FL_HID / 32; ++ks) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(h2 + (rb * 16 + ri) * FL_LDA + ks * 32 + kq8);
            acc[cc] = mfma_step(b3[cc][ks], a, acc[cc]);
          }
        }
        _Float16* const q = par + (rb * 16 + ri) * FL_LDQ + wave * FL_SPS;
        *reinterpret_cast<uint4*>(q + 2 * kq) = make_uint4(pack_f16x2(acc[0][0], acc[0][1]), pack_f16x2(acc[0][2], acc[0][3]),
                                                           pack_f16x2(acc[1][0], acc[1][1]), pack_f16x2(acc[1][2], acc[1][3]));
        *reinterpret_cast<uint2*>(q + 32 + kq) = make_uint2(pack_f16x2(acc[2][0], acc[2][1]), pack_f16x2(acc[2][2], acc[2][3]));
      }
    } else {
      // the forward adds the bias after the products, as the backward's recomputation
      // of the MLP does, so that the two agree bit for bit
#pragma unroll
      for (int rb = 0; rb < FL_TILE_F / 16; ++rb)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ks = 0; ks < FL_HID / 32; ++ks) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(h1 + (rb * 16 + ri) * FL_LDA + ks * 32 + kq8);
            acc = mfma_step(a, b2[cc][ks], acc);
          }
          const int col = (2 * wave + cc) * 16 + ri;
#pragma unroll
          for (int j = 0; j < 4; ++j) h2[(rb * 16 + kq + j) * FL_LDA + col] = f2bf(fmaxf(acc[j] + bias2[cc], 0.f));
        }
      __syncthreads();
#pragma unroll
      for (int rb = 0; rb < FL_TILE_F / 16; ++rb)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int ks = 0; ks < FL_HID / 32; ++ks) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(h2 + (rb * 16 + ri) * FL_LDA + ks * 32 + kq8);
            acc = mfma_step(a, b3[cc][ks], acc);
          }
          const int col = (3 * wave + cc) * 16 + ri;  // parameter col % 47 of coordinate col / 47
          if (col < FL_NOUT) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              par[(rb * 16 + kq + j) * FL_LDQ + (col / FL_NPAR) * FL_SPS + col % FL_NPAR] =
                  static_cast<_Float16>(acc[j] + bias3[cc]);
          }
        }
    }
    __syncthreads();
    {
      __builtin_amdgcn_s_setprio(0);
      float ld = 0.f;
      if (ev < B) {
        const float o = spline_eval<SAMPLE>(par + e * FL_LDQ + c * FL_SPS, vx, ld);
        vout[ev * FL_NDIM + xc] = o;
        if (vout != vin) vout[ev * FL_NDIM + cc_in] = cond[e][c];
      }
      // the event's four log s' (lanes 4e .. 4e+3): sums over lane pairs, then pairs of pairs
      ld += quad_xor<0xB1>(ld);
      ld += quad_xor<0x4E>(ld);
      if (c == 0 && ev < B) logq[ev] += ld;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// backward of one layer over a batch (one 32-event tile per block iteration)
//   gout = dL/d(layer output) [B][8], glq = dL/d log q [B]  ->  gin = dL/d(layer input);
//   stores H1, H2, DR (bf16 and fp32), DH2 (bf16 and fp32), DH1 (fp32), COND for the weight
//   gradients, feature-major ([feature][ld], ld = the batch capacity rounded up to 32) so
//   the contractions over events read contiguous runs; every row of the last tile is
//   written, and the rows past the batch carry zero gradients
// ---------------------------------------------------------------------------
struct FlowBwdBufs {
  uint16_t *H1, *H2, *DRb, *DH2b;
  float *DRf, *DH2f, *DH1f, *COND;
  int64_t ld;
};

__global__ __launch_bounds__(256) void k_flow_layer_bwd(const float* __restrict__ master,
                                                         const uint16_t* __restrict__ wb, int l,
                                                         const float* __restrict__ vin, const float* __restrict__ gout,
                                                         float* __restrict__ gin, const float* __restrict__ glq,
                                                         int64_t B, FlowBwdBufs s) {
  __shared__ float cond[FL_TILE][4];
  __shared__ __align__(16) uint16_t h1[FL_TILE * FL_LDA];
  __shared__ __align__(16) uint16_t h2[FL_TILE * FL_LDA];
  __shared__ __align__(16) float par[FL_TILE * FL_LDP];    // spline parameters, then their gradients, then dh1
  __shared__ __align__(16) uint16_t dpb[FL_TILE * FL_LDP];  // gradients of the spline parameters (bf16), then dh2 (bf16)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float* m = master + l * FL_LAYER;
  const uint16_t* w = wb + static_cast<int64_t>(l) * FB_LAYER;
  for (int64_t e0 = static_cast<int64_t>(blockIdx.x) * FL_TILE; e0 < B; e0 += static_cast<int64_t>(gridDim.x) * FL_TILE) {
    if (tid < FL_TILE * 4) {
      const int e = tid >> 2, c = tid & 3;
      const int64_t ev = e0 + e;
      const float v = ev < B ? vin[ev * FL_NDIM + kFlowC[l][c]] : 0.5f;
      cond[e][c] = v;
      s.COND[c * s.ld + ev] = v;
    }
    __syncthreads();
    mlp_tile32(m, w, cond, h1, h2, par);
    // activations of the tile for the weight gradients
    for (int i = tid; i < FL_TILE * FL_HID; i += blockDim.x) {
      const int e = i % FL_TILE, j = i / FL_TILE;
      s.H1[j * s.ld + e0 + e] = h1[e * FL_LDA + j];
      s.H2[j * s.ld + e0 + e] = h2[e * FL_LDA + j];
    }
    // spline reverse sweep: thread (event, transformed coordinate)
    if (tid < FL_TILE * 4) {
      const int e = tid >> 2, j = tid & 3;
      const int64_t ev = e0 + e;
      float* p = &par[e * FL_LDP + j * FL_NPAR];
      float raw[FL_NPAR], rb[FL_NPAR];
#pragma unroll
      for (int i = 0; i < FL_NPAR; ++i) raw[i] = p[i];
      if (ev < B) {
        Knots K;
        make_knots(raw, K);
        const int d = kFlowX[l][j];
        const float xb = rqs_bwd(raw, K, vin[ev * FL_NDIM + d], gout[ev * FL_NDIM + d], glq[ev], rb);
        gin[ev * FL_NDIM + d] = xb;
      } else {
#pragma unroll
        for (int i = 0; i < FL_NPAR; ++i) rb[i] = 0.f;
      }
#pragma unroll
      for (int i = 0; i < FL_NPAR; ++i) p[i] = rb[i];  // each thread owns its 47 entries
      if (j == 3) {  // the 4 padded columns (188..191) of the event's row
#pragma unroll
        for (int i = 0; i < FL_NOUTP - FL_NOUT; ++i) p[FL_NPAR + i] = 0.f;
      }
    }
    __syncthreads();
    for (int i = tid; i < FL_TILE * FL_NOUTP; i += blockDim.x) {
      const int e = i % FL_TILE, c = i / FL_TILE;
      const float g = par[e * FL_LDP + c];
      dpb[e * FL_LDP + c] = f2bf(g);
      s.DRb[c * s.ld + e0 + e] = f2bf(g);
      s.DRf[c * s.ld + e0 + e] = g;
    }
    __syncthreads();
    // dh2 = dp W3^T (mask h2 > 0): A = dpb [32][192], Bt = W3n [128 in][192 out]
    float dh2v[2][2][4];
    for (int rb = 0; rb < 2; ++rb)
      for (int cc = 0; cc < 2; ++cc) {
        const int cb = 2 * wave + cc;
        const f32x4_t acc = mfma_rowcol(dpb, FL_LDP, w + FB_W3N, FL_NOUTP, rb * 16, cb * 16, FL_NOUTP, lane);
        const int col = cb * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = rb * 16 + 4 * (lane >> 4) + j;
          dh2v[rb][cc][j] = bf2f(h2[row * FL_LDA + col]) > 0.f ? acc[j] : 0.f;
        }
      }
    __syncthreads();  // dpb is read by every wave above; reuse it for dh2 (bf16) below
    for (int rb = 0; rb < 2; ++rb)
      for (int cc = 0; cc < 2; ++cc) {
        const int col = (2 * wave + cc) * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = rb * 16 + 4 * (lane >> 4) + j;
          const float g = dh2v[rb][cc][j];
          dpb[row * FL_LDA + col] = f2bf(g);
          s.DH2b[col * s.ld + e0 + row] = f2bf(g);
          s.DH2f[col * s.ld + e0 + row] = g;
        }
      }
    __syncthreads();
    // dh1 = dh2 W2^T (mask h1 > 0): A = dh2 [32][128] (in dpb, stride FL_LDA), Bt = W2n [128 in][128 out]
    for (int rb = 0; rb < 2; ++rb)
      for (int cc = 0; cc < 2; ++cc) {
        const int cb = 2 * wave + cc;
        const f32x4_t acc = mfma_rowcol(dpb, FL_LDA, w + FB_W2N, FL_HID, rb * 16, cb * 16, FL_HID, lane);
        const int col = cb * 16 + (lane & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = rb * 16 + 4 * (lane >> 4) + j;
          const float g = bf2f(h1[row * FL_LDA + col]) > 0.f ? acc[j] : 0.f;
          par[row * FL_LDP + col] = g;
          s.DH1f[col * s.ld + e0 + row] = g;
        }
      }
    __syncthreads();
    // dcond = dh1 W1^T; gin of the conditioning coordinates = gout + dcond
    if (tid < FL_TILE * 4) {
      const int e = tid >> 2, c = tid & 3;
      const int64_t ev = e0 + e;
      if (ev < B) {
        float a = 0.f;
        for (int k = 0; k < FL_HID; ++k) a += par[e * FL_LDP + k] * m[FO_W1 + c * FL_HID + k];
        const int d = kFlowC[l][c];
        gin[ev * FL_NDIM + d] = gout[ev * FL_NDIM + d] + a;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// weight gradients of one layer, split over the batch (split-K): split sp sums the
// events [sp kc, (sp + 1) kc) into its own partial row; a second kernel adds the
// rows in split order (deterministic) and writes the layer's slice of grad.
//   dW3 = H2^T DR, dW2 = H1^T DH2 on MFMA (16 events per step);
//   dW1 = COND^T DH1, db1..db3 = column sums, on the VALU
// ---------------------------------------------------------------------------
constexpr int kWgTiles = 96 + 64;                  // 16x16 output tiles: dW3 (8 x 12), dW2 (8 x 8)
constexpr int kWgValu = 512 + 128 + 128 + FL_NOUT;  // dW1, db1, db2, db3
constexpr int kWgPart = kWgTiles * 256 + kWgValu;   // floats per split
constexpr int kWgMaxSplit = 64;
constexpr int kWgBlocksX = (kWgTiles + (kWgValu + 63) / 64 + 3) / 4;

// C(16x16 at m0, n0) = sum_k A[m][k] B[k][n] with A = Ht (feature-major [m][ld]) and
// B = Dt ([n][ld]) over k in [k_lo, k_hi) (multiples of 32): lane l supplies
// Ht[m0 + l%16][k0 + 8(l/16) .. +7] and Dt[n0 + l%16][k0 + 8(l/16) .. +7], one
// 16-byte load each
__device__ __forceinline__ f32x4_t mfma_tn(const uint16_t* __restrict__ Ht, const uint16_t* __restrict__ Dt,
                                           int64_t ld, int m0, int n0, int64_t k_lo, int64_t k_hi, int lane) {
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  const uint16_t* ap = Ht + (m0 + (lane & 15)) * ld + 8 * (lane >> 4);
  const uint16_t* bp = Dt + (n0 + (lane & 15)) * ld + 8 * (lane >> 4);
#pragma unroll 4
  for (int64_t k0 = k_lo; k0 < k_hi; k0 += 32) {
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(ap + k0);
    const bf16x8_t b = *reinterpret_cast<const bf16x8_t*>(bp + k0);
    acc = mfma_step(a, b, acc);
  }
  return acc;
}

// sum over k in [k_lo, k_hi) (multiples of 4) of x[k] (y == nullptr) or x[k] y[k]
__device__ __forceinline__ float dot_run(const float* __restrict__ x, const float* __restrict__ y, int64_t k_lo,
                                         int64_t k_hi) {
  float a = 0.f;
#pragma unroll 4
  for (int64_t k = k_lo; k < k_hi; k += 4) {
    const float4 u = *reinterpret_cast<const float4*>(x + k);
    if (y) {
      const float4 v = *reinterpret_cast<const float4*>(y + k);
      a += u.x * v.x + u.y * v.y + u.z * v.z + u.w * v.w;
    } else {
      a += u.x + u.y + u.z + u.w;
    }
  }
  return a;
}

// k_hi is the batch rounded up to 32 (the padded rows hold zero gradients)
__global__ __launch_bounds__(256) void k_flow_wgrad_part(int64_t Bp, int kc, FlowBwdBufs s, float* part) {
  const int lane = threadIdx.x & 63;
  const int wave_g = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t k_lo = static_cast<int64_t>(blockIdx.y) * kc;
  const int64_t k_hi = k_lo + kc < Bp ? k_lo + kc : Bp;
  float* out = part + static_cast<int64_t>(blockIdx.y) * kWgPart;
  if (wave_g < 96) {
    const int mb = wave_g / 12, nb = wave_g % 12;
    const f32x4_t acc = mfma_tn(s.H2, s.DRb, s.ld, mb * 16, nb * 16, k_lo, k_hi, lane);
#pragma unroll
    for (int j = 0; j < 4; ++j) out[wave_g * 256 + lane * 4 + j] = acc[j];
  } else if (wave_g < kWgTiles) {
    const int t = wave_g - 96, mb = t / 8, nb = t % 8;
    const f32x4_t acc = mfma_tn(s.H1, s.DH2b, s.ld, mb * 16, nb * 16, k_lo, k_hi, lane);
#pragma unroll
    for (int j = 0; j < 4; ++j) out[wave_g * 256 + lane * 4 + j] = acc[j];
  } else {
    const int t = (wave_g - kWgTiles) * 64 + lane;
    float a = 0.f;
    if (t < 512) a = dot_run(s.COND + (t / FL_HID) * s.ld, s.DH1f + (t % FL_HID) * s.ld, k_lo, k_hi);
    else if (t < 640) a = dot_run(s.DH1f + (t - 512) * s.ld, nullptr, k_lo, k_hi);
    else if (t < 768) a = dot_run(s.DH2f + (t - 640) * s.ld, nullptr, k_lo, k_hi);
    else if (t < kWgValu) a = dot_run(s.DRf + (t - 768) * s.ld, nullptr, k_lo, k_hi);
    if (t < kWgValu) out[kWgTiles * 256 + t] = a;
  }
}

__global__ void k_flow_wgrad_sum(int nsplit, const float* __restrict__ part, float* grad_layer) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kWgPart) return;
  float a = 0.f;
  for (int sp = 0; sp < nsplit; ++sp) a += part[static_cast<int64_t>(sp) * kWgPart + idx];
  if (idx < kWgTiles * 256) {
    const int tile = idx / 256, r = idx % 256, lane = r / 4, j = r % 4;
    const int row16 = 4 * (lane >> 4) + j, col16 = lane & 15;
    if (tile < 96) {
      const int row = (tile / 12) * 16 + row16, col = (tile % 12) * 16 + col16;
      if (col < FL_NOUT) grad_layer[FO_W3 + row * FL_NOUT + col] = a;
    } else {
      const int t = tile - 96;
      grad_layer[FO_W2 + ((t / 8) * 16 + row16) * FL_HID + (t % 8) * 16 + col16] = a;
    }
  } else {
    const int t = idx - kWgTiles * 256;
    if (t < 512) grad_layer[FO_W1 + t] = a;  // [c][n] with c = t / 128
    else if (t < 640) grad_layer[FO_B1 + t - 512] = a;
    else if (t < 768) grad_layer[FO_B2 + t - 640] = a;
    else grad_layer[FO_B3 + t - 768] = a;
  }
}

// ---------------------------------------------------------------------------
// loss terms: W = sum w (one block, fixed order), glq_i = -w_i / W; loss = -sum w log q / W
// ---------------------------------------------------------------------------
__global__ void k_flow_seed(const double* __restrict__ w, int64_t B, float* glq, double* scal) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < B; i += blockDim.x) s += w[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double W = red[0];
  for (int64_t i = threadIdx.x; i < B; i += blockDim.x) glq[i] = static_cast<float>(-w[i] / W);
  if (threadIdx.x == 0) scal[0] = W;
}

__global__ void k_flow_loss(const double* __restrict__ w, const float* __restrict__ logq, int64_t B, double* scal) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < B; i += blockDim.x) s += w[i] * static_cast<double>(logq[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) scal[1] = -red[0] / scal[0];
}

// Adam on the FP32 master weights (bias-corrected), step t >= 1
__global__ void k_flow_adam(float* master, const float* grad, float* m1, float* m2, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < FL_NPARAMS; i += gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float a = b1 * m1[i] + (1.f - b1) * g;
    const float v = b2 * m2[i] + (1.f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    master[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

// batch gather through the bijection i -> (a i + c) mod n (a odd and coprime to n)
__global__ void k_flow_gather(const float* __restrict__ y, const double* __restrict__ w, int64_t n, uint64_t a,
                              uint64_t c, int64_t start, int64_t B, float* yb, double* wb) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < B;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const uint64_t j = static_cast<uint64_t>(start + i) % static_cast<uint64_t>(n);
    const uint64_t idx = (a * j + c) % static_cast<uint64_t>(n);  // a, j, c < n < 2^31: no overflow
    for (int d = 0; d < FL_NDIM; ++d) yb[i * FL_NDIM + d] = y[idx * FL_NDIM + d];
    wb[i] = w[idx];
  }
}

__global__ void k_flow_zero(float* p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.f;
}

// base points of a flow-proposal iteration: z_i = the event's Philox uniforms (binary32)
__global__ void k_flow_zinit(uint64_t seed, uint32_t iter, int64_t n, float* z, float* logq) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double u[FL_NDIM];
    event_uniforms<FL_NDIM>(seed, iter, static_cast<uint64_t>(i), FL_NDIM, u);
#pragma unroll
    for (int d = 0; d < FL_NDIM; ++d) z[i * FL_NDIM + d] = static_cast<float>(u[d]);
    logq[i] = 0.f;
  }
}

}  // namespace vg

// ===========================================================================
// host
// ===========================================================================
using namespace vg;

namespace vg {
void record_hip_error(const char* what, hipError_t e);  // the message vegas_strerror(VEGAS_EHIP) returns
}

struct vegas_flow_state {
  hipStream_t stream;
  int32_t max_batch;
  int64_t max_sample;
  void* mem;
  float *master, *grad, *m1, *m2;
  uint16_t* wb;
  float *V;     // [7][max_batch][8] activations of the density direction
  float *G;     // [2][max_batch][8] gradients w.r.t. layer outputs / inputs
  float *logq;  // [max_batch]
  float *glq;   // [max_batch]
  float *yb;    // [max_batch][8] gathered batch
  double *wbat; // [max_batch]
  double *scal; // [4] sum w, loss
  FlowBwdBufs bw;
  float *zs, *lqs;  // sampling buffers [max_sample][8], [max_sample]
  float* wpart;     // [kWgMaxSplit][kWgPart] split-K partials of the weight gradients
  uint64_t adam_t;
  hipEvent_t ev_ready, ev_used;  // cross-stream ordering with a VEGAS handle's stream
};

#define VF_HIP(call)                                                       \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      record_hip_error(#call, e_);                                          \
      return VEGAS_EHIP;                                                   \
    }                                                                      \
  } while (0)

namespace {

size_t al(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int flow_prep(vegas_flow_state* f) {
  hipLaunchKernelGGL(k_flow_prep, dim3(80, FL_NLAYER), dim3(256), 0, f->stream, f->master, f->wb);
  VF_HIP(hipGetLastError());
  return VEGAS_OK;
}

// forward-kernel blocks: three resident per CU (LDS 44 KB, at most 168 VGPRs); more tiles
// per block amortise the per-launch load of the weights into registers
constexpr int kFwdBlocks = 3 * 256;

int64_t grid_for(int64_t n, int per_block, int cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g > cap) g = cap;
  return g < 1 ? 1 : g;
}

// density direction over B events of y: V[0] = y, V[l+1] = layer l (V[l]); logq
int flow_forward(vegas_flow_state* f, const float* y, int64_t B) {
  VF_HIP(hipMemcpyAsync(f->V, y, sizeof(float) * FL_NDIM * B, hipMemcpyDeviceToDevice, f->stream));
  hipLaunchKernelGGL(k_flow_zero, dim3(grid_for(B, 256, 1024)), dim3(256), 0, f->stream, f->logq, B);
  VF_HIP(hipGetLastError());
  const int64_t stride = static_cast<int64_t>(f->max_batch) * FL_NDIM;
  for (int l = 0; l < FL_NLAYER; ++l) {
    hipLaunchKernelGGL(k_flow_layer<false>, dim3(grid_for(B, FL_TILE_F, kFwdBlocks)), dim3(256), 0, f->stream, f->master,
                       f->wb, l, f->V + l * stride, f->V + (l + 1) * stride, f->logq, B);
    VF_HIP(hipGetLastError());
  }
  return VEGAS_OK;
}

// gradient of L = -sum w log q / sum w over the batch (f->yb, f->wbat) into f->grad
int flow_backward(vegas_flow_state* f, const double* w, int64_t B, double* loss_host) {
  hipLaunchKernelGGL(k_flow_seed, dim3(1), dim3(256), 0, f->stream, w, B, f->glq, f->scal);
  VF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_flow_loss, dim3(1), dim3(256), 0, f->stream, w, f->logq, B, f->scal);
  VF_HIP(hipGetLastError());
  const int64_t stride = static_cast<int64_t>(f->max_batch) * FL_NDIM;
  float* gout = f->G;           // dL/d z = 0 (uniform base density)
  float* gin = f->G + stride;
  hipLaunchKernelGGL(k_flow_zero, dim3(grid_for(B * FL_NDIM, 256, 1024)), dim3(256), 0, f->stream, gout,
                     B * FL_NDIM);
  VF_HIP(hipGetLastError());
  for (int l = FL_NLAYER - 1; l >= 0; --l) {
    hipLaunchKernelGGL(k_flow_layer_bwd, dim3(grid_for(B, FL_TILE, 4096)), dim3(256), 0, f->stream, f->master, f->wb,
                       l, f->V + l * stride, gout, gin, f->glq, B, f->bw);
    VF_HIP(hipGetLastError());
    const int64_t Bp = (B + 31) / 32 * 32;  // rows past B (written by the backward) hold zero gradients
    int kc = 256;
    if ((Bp + kc - 1) / kc > kWgMaxSplit) kc = static_cast<int>(((Bp + kWgMaxSplit - 1) / kWgMaxSplit + 31) / 32 * 32);
    const int nsplit = static_cast<int>((Bp + kc - 1) / kc);
    hipLaunchKernelGGL(k_flow_wgrad_part, dim3(kWgBlocksX, nsplit), dim3(256), 0, f->stream, Bp, kc, f->bw, f->wpart);
    VF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_flow_wgrad_sum, dim3((kWgPart + 255) / 256), dim3(256), 0, f->stream, nsplit, f->wpart,
                       f->grad + l * FL_LAYER);
    VF_HIP(hipGetLastError());
    float* t = gout;
    gout = gin;
    gin = t;
  }
  if (loss_host) {
    double sc[2];
    VF_HIP(hipMemcpyAsync(sc, f->scal, sizeof(sc), hipMemcpyDeviceToHost, f->stream));
    VF_HIP(hipStreamSynchronize(f->stream));
    *loss_host = sc[1];
  }
  return VEGAS_OK;
}

}  // namespace

extern "C" {

int vegas_flow_create(int32_t max_batch, int64_t max_sample, uint64_t seed, void* stream, vegas_flow* out) {
  if (!out || max_batch < 1 || max_batch > (1 << 22) || max_sample < 0 || max_sample >= (int64_t(1) << 31))
    return VEGAS_EINVAL;
  *out = nullptr;
  vegas_flow_state* f = new (std::nothrow) vegas_flow_state();
  if (!f) return VEGAS_ENOMEM;
  f->stream = static_cast<hipStream_t>(stream);
  f->max_batch = max_batch;
  f->max_sample = max_sample;
  const size_t P = FL_NPARAMS, Bm = static_cast<size_t>(max_batch), S = static_cast<size_t>(max_sample);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = al(off + bytes);
    return o;
  };
  const size_t o_master = take(4 * P), o_grad = take(4 * P), o_m1 = take(4 * P), o_m2 = take(4 * P);
  const size_t o_wb = take(2 * static_cast<size_t>(FB_LAYER) * FL_NLAYER);
  const size_t o_V = take(4 * 7 * Bm * FL_NDIM), o_G = take(4 * 2 * Bm * FL_NDIM);
  const size_t o_logq = take(4 * Bm), o_glq = take(4 * Bm), o_yb = take(4 * Bm * FL_NDIM), o_wbat = take(8 * Bm);
  const size_t o_scal = take(8 * 4);
  const size_t Bl = (Bm + FL_TILE - 1) / FL_TILE * FL_TILE;  // row stride of the feature-major buffers
  const size_t o_H1 = take(2 * Bl * FL_HID), o_H2 = take(2 * Bl * FL_HID), o_DRb = take(2 * Bl * FL_NOUTP);
  const size_t o_DH2b = take(2 * Bl * FL_HID), o_DRf = take(4 * Bl * FL_NOUTP), o_DH2f = take(4 * Bl * FL_HID);
  const size_t o_DH1f = take(4 * Bl * FL_HID), o_COND = take(4 * Bl * 4);
  const size_t o_zs = take(4 * S * FL_NDIM), o_lqs = take(4 * S);
  const size_t o_wpart = take(4 * static_cast<size_t>(kWgMaxSplit) * kWgPart);
  if (hipMalloc(&f->mem, off) != hipSuccess) {
    delete f;
    return VEGAS_ENOMEM;
  }
  char* b = static_cast<char*>(f->mem);
  f->master = reinterpret_cast<float*>(b + o_master);
  f->grad = reinterpret_cast<float*>(b + o_grad);
  f->m1 = reinterpret_cast<float*>(b + o_m1);
  f->m2 = reinterpret_cast<float*>(b + o_m2);
  f->wb = reinterpret_cast<uint16_t*>(b + o_wb);
  f->V = reinterpret_cast<float*>(b + o_V);
  f->G = reinterpret_cast<float*>(b + o_G);
  f->logq = reinterpret_cast<float*>(b + o_logq);
  f->glq = reinterpret_cast<float*>(b + o_glq);
  f->yb = reinterpret_cast<float*>(b + o_yb);
  f->wbat = reinterpret_cast<double*>(b + o_wbat);
  f->scal = reinterpret_cast<double*>(b + o_scal);
  f->bw.H1 = reinterpret_cast<uint16_t*>(b + o_H1);
  f->bw.H2 = reinterpret_cast<uint16_t*>(b + o_H2);
  f->bw.DRb = reinterpret_cast<uint16_t*>(b + o_DRb);
  f->bw.DH2b = reinterpret_cast<uint16_t*>(b + o_DH2b);
  f->bw.DRf = reinterpret_cast<float*>(b + o_DRf);
  f->bw.DH2f = reinterpret_cast<float*>(b + o_DH2f);
  f->bw.DH1f = reinterpret_cast<float*>(b + o_DH1f);
  f->bw.COND = reinterpret_cast<float*>(b + o_COND);
  f->bw.ld = static_cast<int64_t>(Bl);
  f->zs = reinterpret_cast<float*>(b + o_zs);
  f->lqs = reinterpret_cast<float*>(b + o_lqs);
  f->wpart = reinterpret_cast<float*>(b + o_wpart);
  if (hipEventCreateWithFlags(&f->ev_ready, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&f->ev_used, hipEventDisableTiming) != hipSuccess) {
    (void)hipFree(f->mem);
    delete f;
    return VEGAS_EHIP;
  }
  hipLaunchKernelGGL(k_flow_init, dim3(256), dim3(256), 0, f->stream, f->master, seed);
  hipLaunchKernelGGL(k_flow_zero, dim3(256), dim3(256), 0, f->stream, f->m1, static_cast<int64_t>(P));
  hipLaunchKernelGGL(k_flow_zero, dim3(256), dim3(256), 0, f->stream, f->m2, static_cast<int64_t>(P));
  if (hipGetLastError() != hipSuccess || flow_prep(f) != VEGAS_OK || hipStreamSynchronize(f->stream) != hipSuccess) {
    (void)hipFree(f->mem);
    (void)hipEventDestroy(f->ev_ready);
    (void)hipEventDestroy(f->ev_used);
    delete f;
    return VEGAS_EHIP;
  }
  *out = f;
  return VEGAS_OK;
}

int vegas_flow_destroy(vegas_flow f) {
  if (!f) return VEGAS_EINVAL;
  int rc = VEGAS_OK;
  if (hipStreamSynchronize(f->stream) != hipSuccess) rc = VEGAS_EHIP;
  if (hipFree(f->mem) != hipSuccess) rc = VEGAS_EHIP;
  (void)hipEventDestroy(f->ev_ready);
  (void)hipEventDestroy(f->ev_used);
  delete f;
  return rc;
}

int vegas_flow_get_params(vegas_flow f, float* dst_dev) {
  if (!f || !dst_dev) return VEGAS_EINVAL;
  VF_HIP(hipMemcpyAsync(dst_dev, f->master, sizeof(float) * FL_NPARAMS, hipMemcpyDeviceToDevice, f->stream));
  return VEGAS_OK;
}

int vegas_flow_set_params(vegas_flow f, const float* src_dev) {
  if (!f || !src_dev) return VEGAS_EINVAL;
  VF_HIP(hipMemcpyAsync(f->master, src_dev, sizeof(float) * FL_NPARAMS, hipMemcpyDeviceToDevice, f->stream));
  hipLaunchKernelGGL(k_flow_zero, dim3(256), dim3(256), 0, f->stream, f->m1, static_cast<int64_t>(FL_NPARAMS));
  hipLaunchKernelGGL(k_flow_zero, dim3(256), dim3(256), 0, f->stream, f->m2, static_cast<int64_t>(FL_NPARAMS));
  VF_HIP(hipGetLastError());
  f->adam_t = 0;
  return flow_prep(f);
}

int vegas_flow_density(vegas_flow f, const float* y_dev, int64_t B, float* logq_dev) {
  if (!f || !y_dev || !logq_dev || B < 1 || B > f->max_batch) return VEGAS_EINVAL;
  const int rc = flow_forward(f, y_dev, B);
  if (rc != VEGAS_OK) return rc;
  VF_HIP(hipMemcpyAsync(logq_dev, f->logq, sizeof(float) * B, hipMemcpyDeviceToDevice, f->stream));
  return VEGAS_OK;
}

int vegas_flow_loss_grad(vegas_flow f, const float* y_dev, const double* w_dev, int64_t B, float* grad_dev,
                         double* loss_host) {
  if (!f || !y_dev || !w_dev || B < 1 || B > f->max_batch) return VEGAS_EINVAL;
  int rc = flow_forward(f, y_dev, B);
  if (rc != VEGAS_OK) return rc;
  rc = flow_backward(f, w_dev, B, loss_host);
  if (rc != VEGAS_OK) return rc;
  if (grad_dev) VF_HIP(hipMemcpyAsync(grad_dev, f->grad, sizeof(float) * FL_NPARAMS, hipMemcpyDeviceToDevice, f->stream));
  return VEGAS_OK;
}

int vegas_flow_train_step(vegas_flow f, const float* y_dev, const double* w_dev, int64_t n_data, int32_t batch,
                          uint64_t step, float lr, double* loss_host) {
  if (!f || !y_dev || !w_dev || n_data < 1 || n_data >= (int64_t(1) << 31) || batch < 1 || batch > f->max_batch ||
      !(lr > 0.f))
    return VEGAS_EINVAL;
  // per-epoch bijection i -> (a i + c) mod n with a coprime to n, from a Philox draw keyed by the epoch
  const uint64_t per_epoch = (static_cast<uint64_t>(n_data) + batch - 1) / batch;
  const uint64_t epoch = step / per_epoch;
  const int64_t start = static_cast<int64_t>((step % per_epoch) * batch);
  uint64_t a = 1, c = 0;
  {
    uint32_t s0 = static_cast<uint32_t>(epoch) * 0x9E3779B9u + 0x7F4A7C15u;
    uint32_t s1 = static_cast<uint32_t>(epoch >> 32) ^ 0x85EBCA6Bu;
    for (int r = 0; r < 3; ++r) {
      s0 ^= s1 * 0xC2B2AE35u + static_cast<uint32_t>(r);
      s1 ^= (s0 << 13) | (s0 >> 19);
    }
    const uint64_t n = static_cast<uint64_t>(n_data);
    a = (static_cast<uint64_t>(s0) | 1u) % n;
    if (a == 0) a = 1;
    auto gcd = [](uint64_t x, uint64_t y) {
      while (y) {
        const uint64_t t = x % y;
        x = y;
        y = t;
      }
      return x;
    };
    while (gcd(a, n) != 1) a = (a + 2) % n ? (a + 2) % n : 1;
    c = static_cast<uint64_t>(s1) % n;
  }
  const int64_t B = batch;
  hipLaunchKernelGGL(k_flow_gather, dim3(grid_for(B, 256, 1024)), dim3(256), 0, f->stream, y_dev, w_dev, n_data, a, c,
                     start, B, f->yb, f->wbat);
  VF_HIP(hipGetLastError());
  int rc = flow_forward(f, f->yb, B);
  if (rc != VEGAS_OK) return rc;
  rc = flow_backward(f, f->wbat, B, loss_host);
  if (rc != VEGAS_OK) return rc;
  f->adam_t++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, static_cast<float>(f->adam_t));
  const float c2 = 1.f - std::pow(b2, static_cast<float>(f->adam_t));
  hipLaunchKernelGGL(k_flow_adam, dim3(512), dim3(256), 0, f->stream, f->master, f->grad, f->m1, f->m2, lr, b1, b2,
                     1e-8f, c1, c2);
  VF_HIP(hipGetLastError());
  return flow_prep(f);
}

int vegas_flow_sample(vegas_flow f, const float* z_dev, int64_t n, float* y_dev, float* logq_dev) {
  if (!f || !z_dev || !y_dev || !logq_dev || n < 1) return VEGAS_EINVAL;
  if (y_dev != z_dev) VF_HIP(hipMemcpyAsync(y_dev, z_dev, sizeof(float) * FL_NDIM * n, hipMemcpyDeviceToDevice, f->stream));
  hipLaunchKernelGGL(k_flow_zero, dim3(grid_for(n, 256, 1024)), dim3(256), 0, f->stream, logq_dev, n);
  VF_HIP(hipGetLastError());
  for (int l = FL_NLAYER - 1; l >= 0; --l) {
    hipLaunchKernelGGL(k_flow_layer<true>, dim3(grid_for(n, FL_TILE_F, kFwdBlocks)), dim3(256), 0, f->stream, f->master,
                       f->wb, l, y_dev, y_dev, logq_dev, n);
    VF_HIP(hipGetLastError());
  }
  return VEGAS_OK;
}

}  // extern "C"

namespace vg {

// proposal points of a flow iteration on stream s (a VEGAS handle's): z from the
// stream keyed by (seed, iter, i), y = F^{-1}(z), log q(y); the flow's own stream
// is ordered before, and (via finish) after, the use on s
int flow_sample_events(vegas_flow f, hipStream_t s, uint64_t seed, uint32_t iter, int64_t n, const float** y,
                       const float** lq) {
  if (!f || n < 1 || n > f->max_sample) return VEGAS_EINVAL;
  if (s != f->stream) {
    VF_HIP(hipEventRecord(f->ev_ready, f->stream));
    VF_HIP(hipStreamWaitEvent(s, f->ev_ready, 0));
  }
  hipLaunchKernelGGL(k_flow_zinit, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, seed, iter, n, f->zs, f->lqs);
  VF_HIP(hipGetLastError());
  for (int l = FL_NLAYER - 1; l >= 0; --l) {
    hipLaunchKernelGGL(k_flow_layer<true>, dim3(grid_for(n, FL_TILE_F, kFwdBlocks)), dim3(256), 0, s, f->master, f->wb, l,
                       f->zs, f->zs, f->lqs, n);
    VF_HIP(hipGetLastError());
  }
  *y = f->zs;
  *lq = f->lqs;
  return VEGAS_OK;
}

int flow_sample_finish(vegas_flow f, hipStream_t s) {
  if (s != f->stream) {
    VF_HIP(hipEventRecord(f->ev_used, s));
    VF_HIP(hipStreamWaitEvent(f->stream, f->ev_used, 0));
  }
  return VEGAS_OK;
}

}  // namespace vg
