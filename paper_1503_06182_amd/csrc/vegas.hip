// vegas.hip -- gfx950 kernels and the C-ABI host library for the per-event
// VEGAS iteration (Campbell, Ellis, Giele, "A Multi-Threaded Version of MCFM",
// Sec. 2.1-2.2).
//
// One iteration is three or four launches on the handle's stream:
//   k_event     one event per lane (grid-stride): Philox point -> grid map ->
//               phase space -> PDFs x |M|^2 -> weight; writes the event record
//               (w, packed bin indices) and the exact max |w|.  From the second
//               iteration on it also adds each event's exact digits of w, w^2
//               (S1, S2 per lane; d[dim][bin] in LDS) at the scales the previous
//               iteration fixed, one row of partials per block.
//   k_accum     first iteration only (or digits too large for LDS): the same
//               digits from the records, at this iteration's own scales.
//   k_accsum    column sums of the partial rows (integer atomics).
//   k_finalize  one block: totals -> d, S1, S2 as doubles, I_j and var_j; re-folds
//               from the records if this iteration's max |w| left the window of
//               the previous scale, and fixes the next iteration's scales.
//   k_refine    (vegas_refine) one 64-lane block per dimension: smoothing,
//               damping, equal-importance rebinning.
// Integer accumulation is associative, so every launch configuration gives
// byte-identical results (the paper's independence from the thread count,
// Sec. 2.2, made structural).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vegas.h"
#include "device_common.hpp"
#include "integrands.hpp"
#include "adjoint.hpp"

namespace vg {

constexpr int kWave = 64;

constexpr int kMaxRowsEvent = 1 << 16;  // cap on event-kernel blocks
constexpr int kMaxRowsAcc = 1024;       // cap on accumulation blocks (rows of the digit partials)

// digit columns of an iteration's exact sums: S1 = sum w in kD1 digits, then S2 = sum
// w^2 in kD2 digits, then the grid histogram (dimension d, bin b: slot d n + b of nslot)
// digit-major -- digit k of slot s in column kColHist + k nslot + s -- so that the LDS
// atomics of lanes in different bins fall on different banks (slot-major, the four
// digits of a slot span 32 bytes and every slot's digit k met one of a few banks)
constexpr int kD1 = 3, kD2 = 4;
constexpr int kColS2 = kD1;             // first column of S2
constexpr int kColHist = kD1 + kD2;     // first column of the grid histogram
__host__ __device__ constexpr int hist_col(int slot) { return kColHist + slot; }  // digit 0; digit k: + k nslot
__host__ __device__ constexpr int hist_cols(int nslot) { return kColHist + kD2 * nslot; }
// row stride of the digit partials: the ncol = 7 + 4 D n columns padded to a whole
// number of 32-column (256-byte) tiles, so that every tile the column reduction reads
// is aligned to the 128-byte lines it is fetched in
__host__ __device__ constexpr int part_ld(int ncol) { return (ncol + 31) & ~31; }
constexpr int kFusedLdsMax = 64 * 1024; // LDS of an event block (grid + digits) that allows the fused fold
// observable histogram: bins 1..nobs uniform on [lo, hi), 0 = underflow, nobs + 1 = overflow
constexpr int kObsLd = VEGAS_MAX_OBS_BINS + 2;
constexpr int kStrataBlocks = 1024;  // blocks of the hypercube fold (rows of its partials)
constexpr int kDirectRowsMax = 64;   // up to this many partial rows the finalisation sums them itself
constexpr int kFinThreads = 1024;    // finalisation block when it folds or refines (else 256)

// n / d for n < 2^31 by multiply and shift: with l = ceil(log2 d), M = floor(2^(32+l) / d)
// + 1 < 2^33 gives floor(n M / 2^(32+l)) = floor(n / d) exactly, and n M < 2^64
struct UDiv {
  unsigned long long M;
  int s;
};
inline UDiv udiv_magic(uint32_t d) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  return {(1ull << (32 + l)) / d + 1ull, 32 + l};
}
__device__ __forceinline__ uint32_t udiv(uint32_t n, UDiv q) {
  return static_cast<uint32_t>((static_cast<unsigned long long>(n) * q.M) >> q.s);
}
// observable bin k: the digits of sum w at column 7 k, those of sum w^2 at 7 k + 3
constexpr int kObsW = kD1 + kD2;
__host__ __device__ constexpr int obs_cols(int nobs) { return nobs > 0 ? kObsW * (nobs + 2) : 0; }

struct DevBufs {
  double* edges;                 // [D][n+1] current grid
  double* edges_alt;             // [D][n+1] the grid refined speculatively by k_finalize
  double* rec_w;                 // [maxN]
  uint32_t* rec_bins;            // [ceil(D/4)][maxN], 4 bins of 8 bits per word
  // per-iteration values in two slots, "this iteration" and "the next": the host swaps the
  // pointers after each iteration, so the finalisation reads this iteration's slot while
  // it clears (maxw, cnt) or writes (fxs) the next one, and its blocks never race
  unsigned long long* maxw;      // [1] bits of max |w| (device-wide atomic max)
  unsigned long long* cnt;       // [2] n_nonzero, n_nonfinite (atomic)
  int* fxs;                      // [4] valid, E1, E2 of the fused fold at this iteration's scales
  unsigned long long* maxw_next;  // the next iteration's slots (cleared / set by k_finalize)
  unsigned long long* cnt_next;
  int* fxs_next;
  long long* part_acc;           // [rows][part_ld(3*(2+D*n))] per-block digit sums: S1, S2, d[...]
  long long* acc_tot;            // [3*(2+D*n)] digit sums over all blocks
  double* hist;                  // [D*n + 2] d, S1, S2 of the last iteration
  uint8_t* rec_obs;              // [maxN] observable bin of each event (with an observable set)
  double* obs_acc;               // [3 kObsLd + 2] combination: sum w_j H, sum w_j^2 var, sum H (zero-variance
                                 //   iterations), then sum w_j and the count of zero-variance iterations
  double* obs_out;               // [4][kObsLd] last H, its error, the combination, its error
  long long* strat_part;         // [kStrataBlocks][4] per-block digits of V = sum_h sum_{i in h}
                                 //   (w_i - mean_h)^2 (stratified sampling; summed by the finalisation)
  double* history;               // [VEGAS_MAX_ITER][2] I_j, var_j
  double* iter_out;              // [8] I_j, var_j, nz, nnf, N
  double* result;                // [4] I, sigma, chi2/dof, n_iter
};

// ---------------------------------------------------------------------------
// grid map: k = floor(u n) clamped, delta = u n - k, x = fma(delta, h, e_k),
// J = prod n h (plain roundings, no contraction)
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ double grid_map(const double* __restrict__ e_lds, int n, int ndim,
                                           const double* u, double* x, int* bins) {
#pragma clang fp contract(off)
  const int nd = D > 0 ? D : ndim;
  const double dn = static_cast<double>(n);
  double J = 1.0;
#pragma unroll
  for (int d = 0; d < (D > 0 ? D : VEGAS_MAX_DIM); ++d) {
    if (d >= nd) break;
    const double t = u[d] * dn;
    int k = static_cast<int>(t);
    k = k > n - 1 ? n - 1 : k;
    const double delta = t - static_cast<double>(k);
    const double* e = e_lds + d * (n + 1);
    const double lo = e[k];
    const double h = e[k + 1] - lo;
    x[d] = __fma_rn(delta, h, lo);
    J *= dn * h;
    bins[d] = k;
  }
  return J;
}

// q: the process's observable (x_0, cos(theta) of the mu-), or its square (m_ll,
// the e+ p_T, the e+ nu mass), see obs_is_square
template <int PROC, int PREC, int D>
__device__ __forceinline__ double integrand(const PhysConst& c, const double* x, double& q) {
  if constexpr (PROC == VEGAS_GAUSS) {
    q = x[0];
    return f_gauss<D>(c, x);
  } else if constexpr (PROC == VEGAS_GENZ) {
    q = x[0];
    return f_genz<D>(c, x);
  } else if constexpr (PROC == VEGAS_EEMUMU) {
    q = 2.0 * x[0] - 1.0;
    return f_eemumu(c, x);
  } else if constexpr (PROC == VEGAS_DY_Z) {
    return f_dy(c, x, q);
  } else if constexpr (PROC == VEGAS_W_PLUS) {
    return f_w(c, x, q);
  } else if constexpr (PROC == VEGAS_WW_HAD) {
    if constexpr (PREC == VEGAS_FP32_ME) return f_ww<float, true>(c, x, q);
    else return f_ww<double, true>(c, x, q);
  } else if constexpr (PREC == VEGAS_FP32_ME) {
    return f_ww<float>(c, x, q);
  } else {
    return f_ww<double>(c, x, q);
  }
}

template <int PROC>
constexpr bool obs_is_square() {
  return PROC == VEGAS_DY_Z || PROC == VEGAS_W_PLUS || PROC == VEGAS_WW_4L || PROC == VEGAS_WW_HAD;
}

// bin of an observable value o: 0 below lo, nobs + 1 at or above hi (and for a NaN),
// else floor((o - lo) nobs / (hi - lo)) + 1 with scale = nobs / (hi - lo) rounded once,
// at most nobs (the clamp is taken in binary64, so the index stays in 0 .. nobs + 1
// whatever the product)
__device__ __forceinline__ int obs_bin(double o, double lo, double hi, double scale, int nobs) {
  if (o < lo) return 0;
  if (!(o < hi)) return nobs + 1;
  const double t = floor((o - lo) * scale);
  return t < static_cast<double>(nobs) ? static_cast<int>(t) + 1 : nobs;
}

// ---------------------------------------------------------------------------
// exact accumulation of one event: S1 = sum w and S2 = sum w^2 in per-lane
// registers, d[dim][bin] = sum w^2 in LDS (4 integer digits per slot); the
// digits are taken at scales fixed for the whole iteration, so every partition
// of the events gives the same integer totals
// ---------------------------------------------------------------------------
constexpr int kLane = kD1 + kD2;  // per-lane digit sums: S1, then S2
struct LaneSums {
  long long v[kLane];
};

__device__ __forceinline__ void lane_sums_zero(LaneSums& ls) {
#pragma unroll
  for (int k = 0; k < kLane; ++k) ls.v[k] = 0;
}

// the digits of one event: w (d, kD1) and w^2 (h, kD2)
struct EvDigits {
  long long d[kD1], h[kD2];
};

// S1, S2 digits of w; returns the digits of w and of w^2 for the histograms.
// NONNEG: the process's weights are never negative (cross sections, the Gaussian), so the
// digits of w need no sign handling
template <bool NONNEG>
__device__ __forceinline__ void acc_sums(double w, int E1, int E2, LaneSums& ls, EvDigits& g) {
  if constexpr (NONNEG) fx_digits_pos(w, E1, g.d[0], g.d[1], g.d[2]);
  else fx_digits(w, E1, g.d[0], g.d[1], g.d[2]);
  fx2_digits(w * w, E2, g.h);  // w^2 of a finite weight: >= 0
#pragma unroll
  for (int k = 0; k < kD1; ++k) ls.v[k] += g.d[k];
#pragma unroll
  for (int k = 0; k < kD2; ++k) ls.v[kD1 + k] += g.h[k];
}

// the top digit of w^2 is zero unless this iteration's w^2 came within 2^-32 of the
// scale (the scale sits 2^32 above the previous iteration's largest): the histogram
// adds it only when some active lane of the wave has it (a wave-uniform test; adding
// zero changes nothing, so the totals are the same either way)
__device__ __forceinline__ bool top_digit_needed(const EvDigits& g) { return __ballot(g.h[3] != 0) != 0ull; }

// the digits are added whether or not they are zero (but the top digit, see
// top_digit_needed): a branch around each atomic cost more (2 % of the W+ and W+W- event
// kernels) than the atomics it saved.  The LDS byte offset is formed in 32 bits
__device__ __forceinline__ unsigned long long* lds_col(long long* acc, int col) {
  return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(acc) + static_cast<uint32_t>(col) * 8u);
}

// the digits of w^2 to columns col, col + stride, col + 2 stride, col + 3 stride
__device__ __forceinline__ void acc_hist(long long* acc, int col, int stride, const EvDigits& g, bool top) {
  unsigned long long* p = lds_col(acc, col);
  atomicAdd(p, static_cast<unsigned long long>(g.h[0]));
  atomicAdd(p + stride, static_cast<unsigned long long>(g.h[1]));
  atomicAdd(p + 2 * stride, static_cast<unsigned long long>(g.h[2]));
  if (top) atomicAdd(p + 3 * stride, static_cast<unsigned long long>(g.h[3]));
}

// observable bin (seven consecutive columns): the digits of w, then those of w^2
__device__ __forceinline__ void acc_obs(long long* acc, int col, const EvDigits& g, bool top) {
  unsigned long long* p = lds_col(acc, col);
#pragma unroll
  for (int k = 0; k < kD1; ++k) atomicAdd(p + k, static_cast<unsigned long long>(g.d[k]));
  acc_hist(acc, col + kD1, 1, g, top);
}

// per-lane S1, S2 -> wave butterfly -> LDS columns 0 .. kLane - 1 (call with the whole block)
__device__ __forceinline__ void acc_sums_to_lds(LaneSums& ls, long long* acc) {
#pragma unroll
  for (int k = 0; k < kLane; ++k) ls.v[k] = wave_sum_i64(ls.v[k]);
  if ((threadIdx.x & 63) == 0) {
    unsigned long long* p = reinterpret_cast<unsigned long long*>(acc);
#pragma unroll
    for (int k = 0; k < kLane; ++k) atomicAdd(p + k, static_cast<unsigned long long>(ls.v[k]));
  }
}

struct EventArgs {
  PhysConst pc;
  DevBufs b;
  uint64_t seed;
  int64_t nev;
  int64_t stride_rec;  // maxN (record plane stride)
  uint32_t iter;
  int ndim, nbins;
  const float* ext_y;   // learned proposal: points y [nev][8] and log q(y) [nev] (EXT kernels only)
  const float* ext_lq;
  int nobs;             // observable bins (OBS kernels only)
  double obs_lo, obs_hi, obs_scale;
  int strata_m, strata_npc;  // STRAT kernels: strata per axis, events per hypercube
  double strata_md;          // strata_m as binary64
  UDiv div_m, div_npc;       // division by strata_m and by strata_npc
  // adaptive allocation (STRAT kernels, s_cube non-null): the hypercube of each event
  // and the counts; each weight is scaled by N / (H n_h)
  const int32_t* s_cube;
  const int32_t* s_cnt;
  double s_N, s_Hd;
};

// ---------------------------------------------------------------------------
// K1: events
// ---------------------------------------------------------------------------
// waves per SIMD the register allocation must allow with 256-thread blocks
constexpr double kExtLo = 0x1p-40, kExtHi = 1.0 - 0x1p-40;

template <int PROC>
constexpr int event_min_waves() {
  return PROC == VEGAS_WW_HAD ? 2 : (PROC == VEGAS_WW_4L ? 3 : 4);
}

// EXT: the point is the learned proposal's y (binary32, kept inside the open unit
// cube) instead of the event's uniforms, and the weight is divided by q(y).
// FUSED: the event also adds its exact digits at the scales fixed by the
// previous iteration (b.fxs) and the block writes one row of partials; the
// finalisation re-folds from the records if the scales turn out not to fit.
// OBS: the event's observable bin is recorded (and, fused, its w and w^2 digits
// go to that bin's six columns after the grid histogram's).
// STRAT: stratified sampling (Lepage's stratified + importance mode): event i lies in
// hypercube floor(i / npc) of the m^D equal ones, u = (c + r) / m with c the base-m
// digits of the hypercube (dimension 0 the least significant).
template <int PROC, int PREC, int D, int MAXT, bool EXT = false, bool FUSED = false, bool OBS = false,
          bool STRAT = false>
__global__ __launch_bounds__(MAXT, (MAXT == 256 ? event_min_waves<PROC>() : 1)) void k_event(EventArgs a) {
  extern __shared__ unsigned char smem[];
  const int n = a.nbins, nd = D > 0 ? D : a.ndim;
  const int ncol_h = hist_cols(nd * n);
  const int ncol = ncol_h + (OBS ? obs_cols(a.nobs) : 0);
  double* e_lds = reinterpret_cast<double*>(smem);
  long long* acc = reinterpret_cast<long long*>(e_lds + nd * (n + 1));  // FUSED: [ncol]
  for (int i = threadIdx.x; i < nd * (n + 1); i += blockDim.x) e_lds[i] = a.b.edges[i];
  if constexpr (FUSED)
    for (int i = threadIdx.x; i < ncol; i += blockDim.x) acc[i] = 0;
  // with 10 or more dimensions the register budget of 2 waves per SIMD is spent on the
  // integrand, so the lane's S1, S2 digit sums live in LDS, one private slot per lane
  // and digit (no atomics: no other lane touches it) instead of 12 registers
  constexpr bool kLdsSums = FUSED && D >= 10 && MAXT == 256;
  long long* lsum = acc + ncol;  // kLdsSums: [kLane][256]
  if constexpr (kLdsSums)
#pragma unroll
    for (int k = 0; k < kLane; ++k) lsum[k * 256 + threadIdx.x] = 0;
  if (blockIdx.x == 0) {
    // clear this iteration's digit totals (the previous iteration's were consumed
    // by its finalisation, earlier on the stream)
    for (int i = threadIdx.x; i < ncol; i += blockDim.x) a.b.acc_tot[i] = 0;

  }
  int E1 = 0, E2 = 0;
  if constexpr (FUSED) {
    E1 = a.b.fxs[1];
    E2 = a.b.fxs[2];
  }
  __syncthreads();

  LaneSums ls;
  lane_sums_zero(ls);
  // per-lane counts fit 32 bits (fewer than 2^31 events per launch), and so does the
  // event index: both keep registers free for the integrand
  unsigned long long wmax = 0ull;
  uint32_t nz = 0u, nnf = 0u;
  const int32_t step = static_cast<int32_t>(gridDim.x * blockDim.x);
  const int32_t nev32 = static_cast<int32_t>(a.nev);
  for (int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x); i < nev32; i += step) {
    double u[D > 0 ? D : VEGAS_MAX_DIM], x[D > 0 ? D : VEGAS_MAX_DIM];
    // wave priorities: the uniforms (integer work) at the base priority, the grid map
    // (the grid's LDS loads) one step up, the integrand at the top, so that a SIMD
    // issues the floating-point work of waves already past their loads first and the
    // waves of a block drift apart in phase (W+W- 340 against 366 us per 1e7-event
    // launch, hadronic W+W- 490 against 532, with the fold there back at the base
    // priority; the light W+ kernel is unchanged)
    __builtin_amdgcn_s_setprio(0);
    int bins[D > 0 ? D : VEGAS_MAX_DIM];
    if constexpr (EXT) {
#pragma unroll
      for (int d = 0; d < (D > 0 ? D : VEGAS_MAX_DIM); ++d) {
        if (d >= nd) break;
        const double v = static_cast<double>(a.ext_y[static_cast<int64_t>(i) * nd + d]);
        u[d] = fmin(fmax(v, kExtLo), kExtHi);
      }
    } else {
      event_uniforms<D>(a.seed, a.iter, static_cast<uint64_t>(i), nd, u);
      if constexpr (STRAT) {
        uint32_t hc = a.s_cube ? static_cast<uint32_t>(a.s_cube[i]) : udiv(static_cast<uint32_t>(i), a.div_npc);
        const uint32_t m = static_cast<uint32_t>(a.strata_m);
#pragma unroll
        for (int d = 0; d < (D > 0 ? D : VEGAS_MAX_DIM); ++d) {
          if (d >= nd) break;
          const uint32_t q = udiv(hc, a.div_m);
          u[d] = (static_cast<double>(hc - q * m) + u[d]) / a.strata_md;
          hc = q;
        }
      }
    }
    __builtin_amdgcn_s_setprio(1);
    const double J = grid_map<D>(e_lds, n, nd, u, x, bins);
    __builtin_amdgcn_s_setprio(3);
    // the bins, 4 of 8 bits per word.  With 10 or more fixed dimensions they are
    // recorded before the integrand, so that only the packed words stay live across
    // it (the fused fold takes the bins back out of them); with fewer, or a run-time
    // dimension, keeping the bins themselves allocates better
    constexpr int kWords = D > 0 ? (D + 3) / 4 : 4;
    constexpr bool kEarlyBins = D >= 10;
    uint32_t bw[kWords];
    if constexpr (kEarlyBins) {
#pragma unroll
      for (int g = 0; g < kWords; ++g) {
        bw[g] = 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * g + j < nd) bw[g] |= static_cast<uint32_t>(bins[4 * g + j]) << (8 * j);
        a.b.rec_bins[g * a.stride_rec + i] = bw[g];
      }
    }
    double q;
    const double f = integrand<PROC, PREC, D>(a.pc, x, q);
    double w = J * f;
    if constexpr (STRAT && !EXT)
      if (a.s_cube) w *= a.s_N / (a.s_Hd * static_cast<double>(a.s_cnt[a.s_cube[i]]));
    int obin = 0;
    if constexpr (OBS) {
      obin = obs_bin(obs_is_square<PROC>() ? sqrt(q) : q, a.obs_lo, a.obs_hi, a.obs_scale, a.nobs);
      a.b.rec_obs[i] = static_cast<uint8_t>(obin);
    }
    if constexpr (EXT) w *= exp(-static_cast<double>(a.ext_lq[i]));
    if (!isfinite(w * w)) {
      ++nnf;
      w = 0.0;
    } else if (w != 0.0) {
      ++nz;
    }
    a.b.rec_w[i] = w;
    if constexpr (!kEarlyBins) {
#pragma unroll
      for (int g = 0; g < kWords; ++g) {
        if (4 * g >= nd) break;
        uint32_t word = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (4 * g + j < nd) word |= static_cast<uint32_t>(bins[4 * g + j]) << (8 * j);
        a.b.rec_bins[g * a.stride_rec + i] = word;
      }
    }
    if constexpr (PROC == VEGAS_WW_HAD) __builtin_amdgcn_s_setprio(0);
    const unsigned long long wb = static_cast<unsigned long long>(__double_as_longlong(fabs(w)));
    wmax = wb > wmax ? wb : wmax;
    if constexpr (FUSED) {
      if (w != 0.0) {
        EvDigits g;
        if constexpr (kLdsSums) {
          LaneSums t;
          lane_sums_zero(t);
          acc_sums<PROC != VEGAS_GENZ>(w, E1, E2, t, g);
#pragma unroll
          for (int k = 0; k < kLane; ++k) lsum[k * 256 + threadIdx.x] += t.v[k];
        } else {
          acc_sums<PROC != VEGAS_GENZ>(w, E1, E2, ls, g);
        }
        const bool top = top_digit_needed(g);
#pragma unroll
        for (int d = 0; d < (D > 0 ? D : VEGAS_MAX_DIM); ++d) {
          if (d >= nd) break;
          const int bin = kEarlyBins ? static_cast<int>((bw[d >> 2] >> (8 * (d & 3))) & 0xffu) : bins[d];
          acc_hist(acc, hist_col(d * n + bin), nd * n, g, top);
        }
        if constexpr (OBS) acc_obs(acc, ncol_h + kObsW * obin, g, top);
      }
    }
  }
  // block totals (LDS) -> one device-wide atomic per block and quantity
  __shared__ unsigned long long blk[3];
  if (threadIdx.x < 3) blk[threadIdx.x] = 0ull;
  __syncthreads();
  wmax = wave_max_u64(wmax);
  const long long snz = wave_sum_i64(static_cast<long long>(nz));
  const long long snf = wave_sum_i64(static_cast<long long>(nnf));
  if ((threadIdx.x & (kWave - 1)) == 0) {
    atomicMax(&blk[0], wmax);
    atomicAdd(&blk[1], static_cast<unsigned long long>(snz));
    atomicAdd(&blk[2], static_cast<unsigned long long>(snf));
  }
  if constexpr (kLdsSums)
#pragma unroll
    for (int k = 0; k < kLane; ++k) ls.v[k] = lsum[k * 256 + threadIdx.x];
  if constexpr (FUSED) acc_sums_to_lds(ls, acc);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (blk[0]) atomicMax(&a.b.maxw[0], blk[0]);
    if (blk[1]) atomicAdd(&a.b.cnt[0], blk[1]);
    if (blk[2]) atomicAdd(&a.b.cnt[1], blk[2]);
  }
  if constexpr (FUSED) {
    long long* row = a.b.part_acc + static_cast<int64_t>(blockIdx.x) * part_ld(ncol);
    for (int i = threadIdx.x; i < ncol; i += blockDim.x) row[i] = acc[i];
  }
}

// ---------------------------------------------------------------------------
// column reduction of the per-block partials: block (x, y) covers 32 columns and
// rows [32 y, 32 y + 32) with 8 row groups, then one device-wide integer atomic
// per column (max and sum are exact and order-free)
// ---------------------------------------------------------------------------
constexpr int kColTile = 32, kRowTile = 32;

// ---------------------------------------------------------------------------
// stratified sampling: per hypercube (its npc events are consecutive records) the
// mean and then the sum of squared deviations V_h, in binary64 in record order, one
// thread per hypercube; V = sum_h V_h folded exactly (order-free integer digits) at
// the scale of npc max w^2, which bounds every V_h.  Each block writes one row of
// digit sums (no same-address atomics); the finalisation adds the rows.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int strata_exponent(double wmax, int npc) {
  return fx_exponent(wmax * wmax * static_cast<double>(npc));
}

// the block's digit sums -> its row of the partials (call with the whole block)
__device__ __forceinline__ void strata_row(DevBufs& b, long long s0, long long s1, long long s2) {
  __shared__ long long red[3];
  if (threadIdx.x < 3) red[threadIdx.x] = 0;
  __syncthreads();
  s0 = wave_sum_i64(s0);
  s1 = wave_sum_i64(s1);
  s2 = wave_sum_i64(s2);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    unsigned long long* p = reinterpret_cast<unsigned long long*>(red);
    atomicAdd(p + 0, static_cast<unsigned long long>(s0));
    atomicAdd(p + 1, static_cast<unsigned long long>(s1));
    atomicAdd(p + 2, static_cast<unsigned long long>(s2));
  }
  __syncthreads();
  if (threadIdx.x < 3) b.strat_part[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x];
}

__global__ void k_strata(DevBufs b, int64_t H, int npc) {
  const double wmx = __longlong_as_double(static_cast<long long>(b.maxw[0]));
  const int EV = strata_exponent(wmx, npc);
  long long s0 = 0, s1 = 0, s2 = 0;
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t h = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; h < H; h += step) {
    const double* w = b.rec_w + h * npc;
    double sum = 0.0;
#pragma unroll 8
    for (int k = 0; k < npc; ++k) sum += w[k];
    const double mh = sum / static_cast<double>(npc);
    double V = 0.0;
#pragma unroll 8
    for (int k = 0; k < npc; ++k) {
      const double dv = w[k] - mh;
      V = __fma_rn(dv, dv, V);
    }
    long long d0, d1, d2;
    fx_digits_pos(V, EV, d0, d1, d2);
    s0 += d0;
    s1 += d1;
    s2 += d2;
  }
  strata_row(b, s0, s1, s2);
}

// ---------------------------------------------------------------------------
// adaptive allocation: hypercube h holds records off[h] .. off[h] + cnt[h] - 1 of the
// scaled weights w_s = c_h w, c_h = N / (H n_h); the folded term is
// n_h sum (w_s - mean)^2 / (n_h - 1) (var_j = V / N^2, bounded by 2 N max w_s^2), and
// sigma_h of the unscaled weight is kept in sig for the next allocation.
// The counts span two orders of magnitude, so a thread per hypercube alone would leave
// most lanes idle behind the largest: small hypercubes are folded by their own lane,
// large ones by the whole wave.  The order of every sum depends on the counts alone,
// never on the launch shape.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int strata_exponent_adapt(double wmax, double N) {
  return fx_exponent(2.0 * N * wmax * wmax);
}

// a DPP move of a binary64 value (both halves with the same control); lanes without a
// source, or in rows the mask leaves out, receive 0
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROW_MASK, 0xf, BOUND);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROW_MASK, 0xf, BOUND);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// sum over the wave in a fixed order: scans within each row of 16 lanes (row_shr 1, 2,
// 4, 8), then row 0 into row 1 and row 2 into row 3 (row_bcast:15), then rows 0-1 into
// rows 2-3 (row_bcast:31); lane 63 holds the total, read out for every lane.  DPP moves
// stay in the VALU, where the butterfly's cross-lane permutes go through the LDS unit.
__device__ __forceinline__ double wave_total_f64(double v) {
  v += dpp_f64<0x111, 0xf, true>(v);
  v += dpp_f64<0x112, 0xf, true>(v);
  v += dpp_f64<0x114, 0xf, true>(v);
  v += dpp_f64<0x118, 0xf, true>(v);
  v += dpp_f64<0x142, 0xa, false>(v);
  v += dpp_f64<0x143, 0xc, false>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), kWave - 1);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), kWave - 1);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// counts up to this are folded by the hypercube's own lane; larger ones by the whole
// wave, one after another (fixed by the counts, so is every summation order)
constexpr int kStrataLaneMax = 64;

__global__ __launch_bounds__(256) void k_strata_adapt(DevBufs b, int64_t H, const int32_t* cnt, const int32_t* off,
                                                      double* sig, double N) {
  const double wmx = __longlong_as_double(static_cast<long long>(b.maxw[0]));
  const int EV = strata_exponent_adapt(wmx, N);
  const double Hd = static_cast<double>(H);
  const double* __restrict__ rw = b.rec_w;
  long long s0 = 0, s1 = 0, s2 = 0;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  // the loop runs per wave (base uniform), lane l taking hypercube base + l
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * blockDim.x + (threadIdx.x - lane); base < H;
       base += step) {
    const int64_t h = base + lane;
    const bool valid = h < H;
    const int c = valid ? cnt[h] : 0;
    const int64_t o = valid ? off[h] : 0;
    double V = 0.0;
    if (valid && c <= kStrataLaneMax) {
      // unrolled so that eight loads are in flight at once (each lane walks its own
      // cache lines); the additions keep their order
      const double* w = rw + o;
      double sum = 0.0;
#pragma unroll 8
      for (int k = 0; k < c; ++k) sum += w[k];
      const double mh = sum / static_cast<double>(c);
#pragma unroll 8
      for (int k = 0; k < c; ++k) {
        const double dv = w[k] - mh;
        V = __fma_rn(dv, dv, V);
      }
    }
    unsigned long long big = __ballot(valid && c > kStrataLaneMax);
    while (big) {
      const int l = __ffsll(static_cast<long long>(big)) - 1;
      big &= big - 1;
      const int cl = __shfl(c, l, kWave);
      const double* w = rw + __shfl(o, l, kWave);
      double sum = 0.0;
      for (int k = lane; k < cl; k += kWave) sum += w[k];
      const double mh = wave_total_f64(sum) / static_cast<double>(cl);
      double v = 0.0;
      for (int k = lane; k < cl; k += kWave) {
        const double dv = w[k] - mh;
        v = __fma_rn(dv, dv, v);
      }
      v = wave_total_f64(v);
      if (lane == l) V = v;
    }
    if (valid) {
      const double cd = static_cast<double>(c);
      const double ch = N / (Hd * cd);
      sig[h] = sqrt(V / (cd - 1.0)) / ch;
      V = cd * V / (cd - 1.0);
      long long d0, d1, d2;
      fx_digits_pos(V, EV, d0, d1, d2);
      s0 += d0;
      s1 += d1;
      s2 += d2;
    }
  }
  strata_row(b, s0, s1, s2);
}

// ---------------------------------------------------------------------------
// adaptive allocation over G blocks of kAllocThreads, block b owning the contiguous
// hypercubes [b C, (b + 1) C) (G and C depend on H only, so every sum below has a
// fixed order): p_h = sigma_h^beta (1 before any stratified iteration), n_h = 2 +
// floor((n - 2H) p_h / sum p) with the remaining R events one each to hypercubes
// 0 .. R - 1 (equal counts if sum p is not positive or the floors overshoot), and
// the exclusive prefix sum of the counts as offsets
// ---------------------------------------------------------------------------
constexpr int kAllocThreads = 256;
constexpr int kAllocBlocksMax = 1024;

__device__ double block_sum_fixed(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = kAllocThreads / 2; st > 0; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ long long block_sum_int(long long v, long long* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int st = kAllocThreads / 2; st > 0; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const long long r = red[0];
  __syncthreads();
  return r;
}

// sum of p over all blocks' partials, in the same order in every block
__device__ double alloc_total(const double* part, int G, double* red) {
  double a = 0.0;
  for (int k = threadIdx.x; k < G; k += kAllocThreads) a += part[k];
  return block_sum_fixed(a, red);
}

__global__ __launch_bounds__(kAllocThreads) void k_strata_alloc_p(const double* sig, double* p, double* part,
                                                                   int64_t H, int64_t C, double beta, int have_sig) {
  __shared__ double red[kAllocThreads];
  const int64_t h0 = static_cast<int64_t>(blockIdx.x) * C, h1 = min(H, h0 + C);
  double acc = 0.0;
  for (int64_t h = h0 + threadIdx.x; h < h1; h += kAllocThreads) {
    const double v = have_sig ? pow(sig[h], beta) : 1.0;
    p[h] = v;
    acc += v;
  }
  const double tot = block_sum_fixed(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kAllocThreads) void k_strata_alloc_f(const double* p, int32_t* cnt, const double* part,
                                                                   long long* partf, int64_t H, int64_t C, int G,
                                                                   int64_t freev) {
  __shared__ double red[kAllocThreads];
  __shared__ long long lred[kAllocThreads];
  const double A = alloc_total(part, G, red);
  const int64_t h0 = static_cast<int64_t>(blockIdx.x) * C, h1 = min(H, h0 + C);
  long long loc = 0;
  if (A > 0.0)
    for (int64_t h = h0 + threadIdx.x; h < h1; h += kAllocThreads) {
      const int32_t f = static_cast<int32_t>(floor(static_cast<double>(freev) * p[h] / A));
      cnt[h] = f;
      loc += f;
    }
  const long long tot = block_sum_int(loc, lred);
  if (threadIdx.x == 0) partf[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kAllocThreads) void k_strata_alloc_c(int32_t* cnt, int32_t* off, const double* part,
                                                                   const long long* partf, int64_t H, int64_t C,
                                                                   int G, int64_t freev) {
  __shared__ double red[kAllocThreads];
  __shared__ long long lred[kAllocThreads];
  const double A = alloc_total(part, G, red);
  long long F = 0;
  for (int k = threadIdx.x; k < G; k += kAllocThreads) F += partf[k];
  F = block_sum_int(F, lred);
  const bool equal = !(A > 0.0) || F > freev;
  const long long q = freev / H;
  const long long R = freev - (equal ? q * H : F);
  // events before this block: 2 per hypercube, the floors, and the remainder's ones
  long long start = 0;
  for (int k = threadIdx.x; k < static_cast<int>(blockIdx.x); k += kAllocThreads) {
    const int64_t a0 = static_cast<int64_t>(k) * C, a1 = min(H, a0 + C);
    start += 2 * (a1 - a0) + (equal ? q * (a1 - a0) : partf[k]) + max<int64_t>(0, min<int64_t>(a1, R) - a0);
  }
  start = block_sum_int(start, lred);
  // final counts and offsets of this block's hypercubes: contiguous sub-chunks per
  // thread, their sums scanned in thread order
  const int64_t h0 = static_cast<int64_t>(blockIdx.x) * C, h1 = min(H, h0 + C);
  const int64_t sub = (h1 - h0 + kAllocThreads - 1) / kAllocThreads;
  const int64_t s0 = min(h1, h0 + static_cast<int64_t>(threadIdx.x) * sub), s1 = min(h1, s0 + sub);
  long long loc = 0;
  for (int64_t h = s0; h < s1; ++h) {
    const int32_t c = static_cast<int32_t>(2 + (equal ? q : cnt[h]) + (h < R ? 1 : 0));
    cnt[h] = c;
    loc += c;
  }
  lred[threadIdx.x] = loc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long run = start;
    for (int k = 0; k < kAllocThreads; ++k) {
      const long long v = lred[k];
      lred[k] = run;
      run += v;
    }
  }
  __syncthreads();
  long long o = lred[threadIdx.x];
  for (int64_t h = s0; h < s1; ++h) {
    off[h] = static_cast<int32_t>(o);
    o += cnt[h];
  }
}

// groups of 64 consecutive hypercubes, lane l of a wave owning hypercube 64 g + l; the
// group's records are contiguous
constexpr int32_t kNoRecord = 0x7fffffff;

struct StrataGroup {
  int32_t o, c;  // this lane's hypercube: first record and count (kNoRecord, 0 past H)
  int64_t B, E;  // the group's records [B, E)
};

// call with the whole wave (g uniform)
__device__ __forceinline__ StrataGroup strata_group(const int32_t* cnt, const int32_t* off, int64_t H, int64_t g) {
  const int64_t h = g * kWave + (threadIdx.x & (kWave - 1));
  StrataGroup s;
  s.o = h < H ? off[h] : kNoRecord;
  s.c = h < H ? cnt[h] : 0;
  const int last = static_cast<int>(min<int64_t>(H - g * kWave, kWave)) - 1;
  s.B = __shfl(s.o, 0, kWave);
  s.E = static_cast<int64_t>(__shfl(s.o + s.c, last, kWave));
  return s;
}

// the lane of the group whose hypercube holds record p, B <= p < E: the last lane whose
// first record is <= p (first records increase strictly, every count being >= 2; past
// H they are kNoRecord).  Call with the whole wave.
__device__ __forceinline__ int strata_lane_of(int32_t p, int32_t o) {
  int j = 0;
#pragma unroll
  for (int st = kWave / 2; st > 0; st >>= 1) {
    const int32_t oc = __shfl(o, j + st, kWave);
    if (oc <= p) j += st;
  }
  return j;
}

// the hypercube index of every event: cube[off[h] .. off[h] + cnt[h] - 1] = h, one
// wave per group of 64 hypercubes writing its records 64 at a time
__global__ __launch_bounds__(256) void k_strata_expand(const int32_t* cnt, const int32_t* off, int32_t* cube,
                                                       int64_t H) {
  const int lane = threadIdx.x & (kWave - 1), wpb = blockDim.x / kWave;
  const int64_t ngroups = (H + kWave - 1) / kWave, gstep = static_cast<int64_t>(gridDim.x) * wpb;
  for (int64_t g = static_cast<int64_t>(blockIdx.x) * wpb + threadIdx.x / kWave; g < ngroups; g += gstep) {
    const StrataGroup s = strata_group(cnt, off, H, g);
    for (int64_t cb = s.B; cb < s.E; cb += kWave) {
      const int64_t p = cb + lane;
      const int j = strata_lane_of(static_cast<int32_t>(p < s.E ? p : s.E - 1), s.o);
      if (p < s.E) cube[p] = static_cast<int32_t>(g * kWave + j);
    }
  }
}

// ---------------------------------------------------------------------------
// K2 (two-pass fold): exact accumulation of S1, S2 and d from the records at the
// scales of this iteration's own max |w|.  Block (x, y) holds the histogram of
// dimensions [y dpg, (y + 1) dpg) in LDS (and S1, S2 when y == 0) and writes its
// part of row x of the partials.
// ---------------------------------------------------------------------------
struct AccArgs {
  DevBufs b;
  int64_t nev;
  int64_t stride_rec;
  int ndim, nbins;
  int dims_per_group;
  int nobs;  // observable bins (the y == 0 blocks fold them with S1, S2)
};

__global__ void k_accum(AccArgs a) {
  extern __shared__ unsigned char smem[];
  const int n = a.nbins, nd = a.ndim, ncol_h = hist_cols(nd * n);
  const int ncol = ncol_h + obs_cols(a.nobs);
  const int dlo = blockIdx.y * a.dims_per_group;
  const int dhi = min(nd, dlo + a.dims_per_group);
  const int lslots = (dhi - dlo) * n, lcol = hist_cols(lslots);
  const int ocol = blockIdx.y == 0 ? obs_cols(a.nobs) : 0;  // block-uniform
  // [lcol]: S1, S2, d of the group's dimensions; then [ocol]: the observable's bins
  long long* acc = reinterpret_cast<long long*>(smem);
  for (int i = threadIdx.x; i < lcol + ocol; i += blockDim.x) acc[i] = 0;
  // one scale per quantity: 2^(94 - E1) for w and 2^(126 - E2) for w^2, with |w| < 2^E1
  // and w^2 < 2^E2 for every event
  const double wmax = __longlong_as_double(static_cast<long long>(a.b.maxw[0]));
  const int E1 = fx_exponent(wmax);
  const int E2 = fx_exponent(wmax * wmax);
  __syncthreads();

  LaneSums ls;
  lane_sums_zero(ls);
  const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < a.nev; i += step) {
    const double w = a.b.rec_w[i];
    if (w == 0.0) continue;
    EvDigits g;
    acc_sums<false>(w, E1, E2, ls, g);
    // the same digits of w^2 go to the event's bin in every dimension
    for (int d = dlo; d < dhi; ++d) {
      const uint32_t word = a.b.rec_bins[(d >> 2) * a.stride_rec + i];
      const int bin = static_cast<int>((word >> (8 * (d & 3))) & 0xffu);
      acc_hist(acc, hist_col((d - dlo) * n + bin), lslots, g, true);
    }
    if (ocol) acc_obs(acc, lcol + kObsW * static_cast<int>(a.b.rec_obs[i]), g, true);
  }
  acc_sums_to_lds(ls, acc);
  __syncthreads();
  long long* row = a.b.part_acc + static_cast<int64_t>(blockIdx.x) * part_ld(ncol);
  if (blockIdx.y == 0)
    for (int i = threadIdx.x; i < kColHist; i += blockDim.x) row[i] = acc[i];
  // local column kColHist + k lslots + ls -> global kColHist + k nd n + dlo n + ls
  for (int i = threadIdx.x; i < lcol - kColHist; i += blockDim.x) {
    const int k = i / lslots, ls = i - k * lslots;
    row[hist_col(dlo * n + ls) + k * (nd * n)] = acc[kColHist + i];
  }
  for (int i = threadIdx.x; i < ocol; i += blockDim.x) row[ncol_h + i] = acc[lcol + i];
}

// ---------------------------------------------------------------------------
// K3: digit totals -> doubles (d, S1, S2), then I_j and var_j.  One block.
// After a fused fold, the scales of the previous iteration are kept only while
// this iteration's max |w| lies in [2^(E1 - kFxLow), 2^E1) and its max w^2 in
// [2^(E2 - kFxLow), 2^E2); otherwise the block
// re-folds every record at this iteration's own scales (same totals as the
// two-pass fold).  It then fixes the next iteration's scales and clears the
// iteration's max |w| and counters.
// ---------------------------------------------------------------------------
constexpr int kFxHead = 16;  // next scale: 2^16 above this iteration's max |w|
constexpr int kFxLow = 40;   // the fused scales are kept down to 2^-40 of themselves (>= 54 bits per event)

struct FinArgs {
  DevBufs b;
  int64_t nev, stride_rec;
  int ndim, nbins;
  uint32_t iter;
  int fused;
  int spec;      // also refine the grid into b.edges_alt (waves 0..D-1, one dimension each)
  int fold_lds;  // bytes of dynamic LDS before the refinement scratch (the re-fold's digits)
  int obs_lds;   // byte offset of the observable scratch [2 (nobs + 2)] doubles
  int nobs, obs_first;
  int64_t strata_H;  // > 0: stratified, var_j from the hypercubes' V
  int strata_npc;
  int strata_blocks;  // rows of the hypercube fold's partials
  int strata_adapt;   // unequal counts: var_j = V / N^2
  double alpha;
  int direct_rows;    // > 0: no column-sum launch ran; sum rows [0, direct_rows) of the
                      // partials here, each block only the columns it converts
};

// var_j: the plain (S2 / N - I^2) / (N - 1), or, stratified, sum_h (1/H)^2 sigma_h^2 / npc
// = V / (H^2 npc (npc - 1)) with V from the hypercube fold, whose row sums the block
// left per wave in sv (wmax: this iteration's max |w|, read by every thread before
// the finalisation clears it)
__device__ __forceinline__ double iteration_variance(const FinArgs& f, double S1, double S2, double wmax,
                                                     const long long (*sv)[3]) {
  const double N = static_cast<double>(f.nev);
  if (f.strata_H > 0) {
    long long t[3] = {0, 0, 0};
    for (int w = 0; w < static_cast<int>(blockDim.x) / kWave; ++w)
      for (int k = 0; k < 3; ++k) t[k] += sv[w][k];
    if (f.strata_adapt) return fx_value(t[0], t[1], t[2], strata_exponent_adapt(wmax, N)) / (N * N);
    const double V = fx_value(t[0], t[1], t[2], strata_exponent(wmax, f.strata_npc));
    const double H = static_cast<double>(f.strata_H), c = static_cast<double>(f.strata_npc);
    return V / (H * H * c * (c - 1.0));
  }
  const double I = S1 / N;
  return fma(-I, I, S2 / N) / (N - 1.0);
}

__device__ __forceinline__ void refine_dim(bool active, bool preloaded, int n, double alpha, const double* hist,
                                           const double* e_in, double* e_out, double* sm);

// OBS: an observable histogram is set (f.nobs > 0); the plain variant carries none of its code
template <bool OBS>
__device__ __forceinline__ void finalize_block(const FinArgs& f, unsigned char* smem) {
  __shared__ double s12[2];
  const DevBufs& b = f.b;
  const int n = f.nbins, nd = f.ndim, nslot = nd * n, ncol_h = hist_cols(nslot);
  const int ncol = ncol_h + (OBS ? obs_cols(f.nobs) : 0);
  // few partial rows (small iterations, no column-sum launch): this block sums the
  // columns it converts -- digit k of its dimensions' slots, and in block 0 S1, S2 and
  // the observable's -- over rows g, g + R, ... (up to 32 per item, item = (column, g)).
  // The loads of each thread's first item are issued here, before anything waits on
  // memory, assuming the per-dimension split; a re-fold discards them.
  const int dr = f.direct_rows, dsplit = gridDim.x > 1;
  const int dlo = dsplit ? static_cast<int>(blockIdx.x) : 0, dnh = (dsplit ? 1 : nd) * n;
  const int dncb = dr > 0 ? kD2 * dnh + (blockIdx.x == 0 ? kColHist + (OBS ? obs_cols(f.nobs) : 0) : 0) : 0;
  const int dR = (dr + 31) / 32;
  const int64_t dld = part_ld(ncol);
  auto dcol_of = [&](int qc) {
    if (qc < kD2 * dnh) {
      const int k = qc / dnh;
      return hist_col(dlo * n + (qc - k * dnh)) + k * nslot;
    }
    const int e = qc - kD2 * dnh;
    return e < kColHist ? e : ncol_h + (e - kColHist);
  };
  auto dsum_item = [&](int q, int& col) {
    const int qc = q % dncb, g = q / dncb;
    col = dcol_of(qc);
    long long v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int r = g + dR * k;
      v[k] = r < dr ? b.part_acc[r * dld + col] : 0;
    }
    long long t = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) t += v[k];
    return t;
  };
  // this iteration's max |w|, counters and fold scales (read before the row loads wait)
  const double wmax = __longlong_as_double(static_cast<long long>(b.maxw[0]));
  const unsigned long long nz = b.cnt[0], nnf = b.cnt[1];
  const int Ef = b.fxs[1], E2f = b.fxs[2];
  // the grid edges the block refines, likewise loaded early (same split assumption)
  const int ne_early = (dsplit ? 1 : nd) * (n + 1);
  const bool e_fast = f.spec && ne_early <= kFinThreads;  // a refining finalisation has kFinThreads
  double e_early = 0.0;
  if (e_fast && static_cast<int>(threadIdx.x) < ne_early) e_early = b.edges[dlo * (n + 1) + threadIdx.x];
  long long dsum = 0;
  int dcol = -1;
  if (static_cast<int>(threadIdx.x) < dncb * dR) dsum = dsum_item(threadIdx.x, dcol);
  const int Ec1 = fx_exponent(wmax), Ec2 = fx_exponent(wmax * wmax);
  int E1 = Ec1, E2 = Ec2, fold = 0;
  if (f.fused) {
    // the scales are kept while this iteration's max |w| is below 2^Ef and neither w nor
    // w^2 lost more than kFxLow bits of headroom: w^2 is folded at 2 Ef, so its headroom
    // shrinks twice as fast as that of w
    if (Ec1 > Ef || Ec1 < Ef - kFxLow || Ec2 < E2f - kFxLow) {
      fold = 2;
    } else {
      fold = 1;
      E1 = Ef;
      E2 = E2f;
    }
  }
  // one block per dimension (launched so when the refinement is computed here): block d
  // converts and refines dimension d, block 0 also forms the iteration's results.  A
  // re-fold needs every record in one block, so then block 0 does everything alone.
  const bool split = gridDim.x > 1 && fold != 2;  // grid-uniform
  if (blockIdx.x > 0 && !split) return;
  const int d_lo = split ? static_cast<int>(blockIdx.x) : 0, d_hi = split ? d_lo + 1 : nd;
  const bool lead = blockIdx.x == 0;
  double* rsm = reinterpret_cast<double*>(smem + f.fold_lds);  // refinement scratch [dims][4 (n + 1)]
  if (f.spec) {  // the grid the refinement starts from
    if (e_fast && split == (dsplit != 0)) {  // the early loads cover this block's dimensions
      const int i = threadIdx.x;
      if (i < ne_early) rsm[(i / (n + 1)) * 4 * (n + 1) + 3 * (n + 1) + i % (n + 1)] = e_early;
    } else {
      for (int i = threadIdx.x; i < (d_hi - d_lo) * (n + 1); i += blockDim.x)
        rsm[(i / (n + 1)) * 4 * (n + 1) + 3 * (n + 1) + i % (n + 1)] = b.edges[d_lo * (n + 1) + i];
    }
  }
  const long long* tot = b.acc_tot;
  if (dr > 0 && fold != 2) {  // block-uniform (fold != 2: the split the loads assumed)
    long long* acc = reinterpret_cast<long long*>(smem);
    for (int q = threadIdx.x; q < dncb; q += blockDim.x) acc[dcol_of(q)] = 0;
    __syncthreads();
    if (dcol >= 0) atomicAdd(reinterpret_cast<unsigned long long*>(&acc[dcol]), static_cast<unsigned long long>(dsum));
    for (int q = threadIdx.x + blockDim.x; q < dncb * dR; q += blockDim.x) {
      int col;
      const long long t = dsum_item(q, col);
      atomicAdd(reinterpret_cast<unsigned long long*>(&acc[col]), static_cast<unsigned long long>(t));
    }
    __syncthreads();
    tot = acc;
  }
  if (fold == 2) {  // block-uniform
    long long* acc = reinterpret_cast<long long*>(smem);
    for (int i = threadIdx.x; i < ncol; i += blockDim.x) acc[i] = 0;
    __syncthreads();
    LaneSums ls;
    lane_sums_zero(ls);
    for (int64_t i = threadIdx.x; i < f.nev; i += blockDim.x) {
      const double w = b.rec_w[i];
      if (w == 0.0) continue;
      EvDigits g;
      acc_sums<false>(w, E1, E2, ls, g);
      for (int d = 0; d < nd; ++d) {
        const uint32_t word = b.rec_bins[(d >> 2) * f.stride_rec + i];
        acc_hist(acc, hist_col(d * n + static_cast<int>((word >> (8 * (d & 3))) & 0xffu)), nslot, g, true);
      }
      if constexpr (OBS) acc_obs(acc, ncol_h + kObsW * static_cast<int>(b.rec_obs[i]), g, true);
    }
    acc_sums_to_lds(ls, acc);
    __syncthreads();
    tot = acc;
  }
  // observable bins: value nslot + 2 + 2k is sum w of bin k (scale E1), the next one
  // sum w^2 (scale E2); their values go to osm
  double* osm = reinterpret_cast<double*>(smem + f.obs_lds);
  const int nslot_all = nslot + 2 + (OBS ? 2 * (f.nobs + 2) : 0);
  // stratified: the hypercube fold's row sums, per wave (rows strided over the block)
  __shared__ long long sv[16][3];
  if (lead && f.strata_H > 0) {  // block-uniform
    long long t0 = 0, t1 = 0, t2 = 0;
    for (int r = threadIdx.x; r < f.strata_blocks; r += blockDim.x) {
      t0 += b.strat_part[r * 4 + 0];
      t1 += b.strat_part[r * 4 + 1];
      t2 += b.strat_part[r * 4 + 2];
    }
    t0 = wave_sum_i64(t0);
    t1 = wave_sum_i64(t1);
    t2 = wave_sum_i64(t2);
    if ((threadIdx.x & (kWave - 1)) == 0) {
      sv[threadIdx.x / kWave][0] = t0;
      sv[threadIdx.x / kWave][1] = t1;
      sv[threadIdx.x / kWave][2] = t2;
    }
  }
  // the combination so far, one bin per thread (nobs + 2 <= 256 <= blockDim.x), read
  // before the barrier that precedes its update
  double ws_old = 0.0, zc_old = 0.0, aw = 0.0, av = 0.0, az = 0.0;
  const int kb = threadIdx.x;
  if constexpr (OBS) {
    ws_old = b.obs_acc[3 * kObsLd];
    zc_old = b.obs_acc[3 * kObsLd + 1];
    if (kb < f.nobs + 2) {
      aw = b.obs_acc[kb];
      av = b.obs_acc[kObsLd + kb];
      az = b.obs_acc[2 * kObsLd + kb];
    }
  }
  // the values this block converts: S1, S2 and the observable's (block 0), and the
  // histogram slots of its dimensions
  const int h_lo = d_lo * n, h_hi = d_hi * n;
  for (int q = threadIdx.x; q < nslot_all; q += blockDim.x) {
    int slot = q;
    if (split) {
      if (q < 2 || q >= nslot + 2) {
        if (!lead) continue;
      } else if (q - 2 >= h_hi - h_lo) {
        continue;
      } else {
        slot = 2 + h_lo + (q - 2);
      }
    }
    if (OBS && slot >= nslot + 2) {
      const int so = slot - (nslot + 2);
      const long long* t = tot + ncol_h + kObsW * (so >> 1);
      osm[so] = (so & 1) ? fx2_value(t[kD1], t[kD1 + 1], t[kD1 + 2], t[kD1 + 3], E2) : fx_value(t[0], t[1], t[2], E1);
      continue;
    }
    // S1, S2: consecutive digits; a histogram slot: its digits nslot columns apart
    const long long* t = tot + (slot == 0 ? 0 : slot == 1 ? kColS2 : hist_col(slot - 2));
    const int ds = slot < 2 ? 1 : nslot;
    const double v = slot == 0 ? fx_value(t[0], t[1], t[2], E1) : fx2_value(t[0], t[ds], t[2 * ds], t[3 * ds], E2);
    const int h = slot < 2 ? nslot + slot : slot - 2;
    b.hist[h] = v;
    if (slot < 2) s12[slot] = v;
    else if (f.spec) rsm[(h / n - d_lo) * 4 * (n + 1) + h % n] = v;
  }
  __syncthreads();
  if (lead && threadIdx.x == 0) {
    const double S1 = s12[0], S2 = s12[1];
    const double N = static_cast<double>(f.nev);
    const double I = S1 / N;
    const double var = iteration_variance(f, S1, S2, wmax, sv);
    b.history[2 * f.iter] = I;
    b.history[2 * f.iter + 1] = var;
    b.iter_out[0] = I;
    b.iter_out[1] = var;
    b.iter_out[2] = static_cast<double>(nz);
    b.iter_out[3] = static_cast<double>(nnf);
    b.iter_out[4] = N;
    b.iter_out[5] = static_cast<double>(fold);
    // the next iteration's slots: its scales, and its max |w| and counters from zero
    b.fxs_next[0] = 1;
    b.fxs_next[1] = Ec1 + kFxHead;
    b.fxs_next[2] = 2 * (Ec1 + kFxHead);
    b.maxw_next[0] = 0ull;
    b.cnt_next[0] = 0ull;
    b.cnt_next[1] = 0ull;
  }
  if (OBS && lead) {
    // per bin: H = S1_b / N and var_b = (S2_b / N - H^2) / (N - 1), as for the
    // integral; iterations from obs_first on are combined with the integral's
    // weights 1 / var_j (the plain mean once an iteration has zero variance)
    const double N = static_cast<double>(f.nev);
    const double var = iteration_variance(f, s12[0], s12[1], wmax, sv);
    const bool on = f.iter >= static_cast<uint32_t>(f.obs_first);
    const bool pos = var > 0.0;
    const double wj = pos ? 1.0 / var : 0.0;
    const double ws = on && pos ? ws_old + wj : ws_old;
    const double zc = on && !pos ? zc_old + 1.0 : zc_old;
    if (kb < f.nobs + 2) {
      const int k = kb;
      const double h = osm[2 * k] / N;
      const double v = fma(-h, h, osm[2 * k + 1] / N) / (N - 1.0);
      if (on) {
        if (pos) {
          aw += wj * h;
          av += wj * wj * v;
          b.obs_acc[k] = aw;
          b.obs_acc[kObsLd + k] = av;
        } else {
          az += h;
          b.obs_acc[2 * kObsLd + k] = az;
        }
      }
      double c = 0.0, e = 0.0;
      if (zc > 0.0) {
        c = az / zc;
      } else if (ws > 0.0) {
        c = aw / ws;
        e = sqrt(av) / ws;
      }
      b.obs_out[k] = h;
      b.obs_out[kObsLd + k] = sqrt(v > 0.0 ? v : 0.0);
      b.obs_out[2 * kObsLd + k] = c;
      b.obs_out[3 * kObsLd + k] = e;
    }
    if (threadIdx.x == 0) {
      b.obs_acc[3 * kObsLd] = ws;
      b.obs_acc[3 * kObsLd + 1] = zc;
    }
  }
  if (f.spec) {
    // the refinement vegas_refine would compute from this histogram, so that it only
    // has to swap the grid buffers (the same routine as k_refine: the same bits)
    // (the histogram and the old grid are already in the scratch; refine_dim's first
    // barrier orders those LDS writes before its reads)
    const int d = d_lo + (threadIdx.x >> 6);
    const bool active = d < d_hi;
    refine_dim(active, true, n, f.alpha, nullptr, nullptr, b.edges_alt + (active ? d : 0) * (n + 1),
               rsm + (active ? d - d_lo : 0) * 4 * (n + 1));
  }
}

// column sums of the per-block partial rows: block (x, y) covers 32 columns and rows
// [32 y, 32 y + 32) with 8 row groups, then one device-wide integer atomic per
// column (sums of integers: exact and order-free)
__global__ void k_accsum(DevBufs b, int ncol, int rows) {
  __shared__ long long red[8][kColTile];
  const int c = threadIdx.x & 31, rg = threadIdx.x >> 5;
  const int col = blockIdx.x * kColTile + c;
  const int64_t ld = part_ld(ncol);
  // the rows rg, rg + 8, ... of this tile: all loads issued before the first add
  long long v[kRowTile / 8];
#pragma unroll
  for (int k = 0; k < kRowTile / 8; ++k) {
    const int r = blockIdx.y * kRowTile + rg + 8 * k;
    v[k] = (col < ncol && r < rows) ? b.part_acc[r * ld + col] : 0;
  }
  long long sum = 0;
#pragma unroll
  for (int k = 0; k < kRowTile / 8; ++k) sum += v[k];
  red[rg][c] = sum;
  __syncthreads();
  if (rg == 0 && col < ncol) {
    for (int g = 1; g < 8; ++g) sum += red[g][c];
    if (sum) atomicAdd(reinterpret_cast<unsigned long long*>(&b.acc_tot[col]), static_cast<unsigned long long>(sum));
  }
}

// one block (a separate launch: a grid-wide "last block" hand-off would need a
// device-scope fence in every block, which costs far more than the launch)
template <bool OBS>
__global__ void k_finalize(FinArgs f) {
  extern __shared__ unsigned char smem[];  // fused: the digit columns, for a re-fold; the refinement scratch
  finalize_block<OBS>(f, smem);
}

// ---------------------------------------------------------------------------
// K4: grid refinement, one single-wave block per dimension
// ---------------------------------------------------------------------------

// Refinement of dimension d by one wave (lane = threadIdx.x % 64) with LDS scratch
// sm[4 (n + 1)]; every wave of the block calls it (its one barrier is block-wide);
// active == false only keeps the barrier.  Reads the histogram hist[n] and edges
// e_in[n + 1] (or finds them already in sm[0..n) and sm[3 (n + 1) ..] when preloaded),
// writes e_out[n + 1] (may equal e_in).  An empty histogram keeps the dimension's grid.
// Lane l owns the bins [c l, c l + c), c = ceil(n / 64) <= 4: after the barrier the
// smoothing, the damping, the cumulative importance and the new edges stay in its
// registers, with wave sums and one wave scan by DPP; each lane places the new edges
// that fall into its own bins (edge k lies in the old bin j with cm[j] < k stp <= cm[j+1],
// the same bin a search over cm finds), so no cross-lane search is needed.
__device__ __forceinline__ double wave_scan_f64(double v) {  // inclusive, lanes 0..63
  v += dpp_f64<0x111, 0xf, true>(v);
  v += dpp_f64<0x112, 0xf, true>(v);
  v += dpp_f64<0x114, 0xf, true>(v);
  v += dpp_f64<0x118, 0xf, true>(v);
  v += dpp_f64<0x142, 0xa, false>(v);
  v += dpp_f64<0x143, 0xc, false>(v);
  return v;
}

__device__ __forceinline__ double wave_scan_max_f64(double v) {  // inclusive, for v >= 0
  v = fmax(v, dpp_f64<0x111, 0xf, true>(v));
  v = fmax(v, dpp_f64<0x112, 0xf, true>(v));
  v = fmax(v, dpp_f64<0x114, 0xf, true>(v));
  v = fmax(v, dpp_f64<0x118, 0xf, true>(v));
  v = fmax(v, dpp_f64<0x142, 0xa, false>(v));
  v = fmax(v, dpp_f64<0x143, 0xc, false>(v));
  return v;
}

__device__ __forceinline__ double read_lane_f64(double v, int lane) {  // lane wave-uniform
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), lane);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

__device__ __forceinline__ void refine_dim(bool active, bool preloaded, int n, double alpha, const double* hist,
                                           const double* e_in, double* e_out, double* sm) {
  double* hs = sm;                // histogram of this dimension
  double* eo = sm + 3 * (n + 1);  // old edges
  const int lane = threadIdx.x & 63;
  if (active && !preloaded) {
    for (int k = lane; k < n; k += kWave) hs[k] = hist[k];
    for (int k = lane; k <= n; k += kWave) eo[k] = e_in[k];
  }
  __syncthreads();
  const int c = (n + kWave - 1) / kWave, j0 = c * lane;
  // smoothed histogram of the lane's bins, and the sums of the raw and smoothed ones
  double v[4];
  double s = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int k = j0 + i;
    v[i] = 0.0;
    if (active && i < c && k < n) {
      double t;
      if (k == 0) t = (hs[0] + hs[1]) / 2.0;
      else if (k == n - 1) t = (hs[n - 2] + hs[n - 1]) / 2.0;
      else t = (hs[k - 1] + hs[k] + hs[k + 1]) / 3.0;
      v[i] = t;
      s += hs[k];
      sb += t;
    }
  }
  s = wave_total_f64(s);
  sb = wave_total_f64(sb);
  const bool work = active && s > 0.0;  // wave-uniform
  if (work) {
    // damped importance m of each bin (the usual damping exponent 1.5 without pow)
    const double isb = 1.0 / sb;
    double m[4];
    double part = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      m[i] = 0.0;
      if (i < c && j0 + i < n) {
        const double r = v[i] * isb;
        if (r == 1.0) {
          m[i] = 1.0;
        } else if (r != 0.0) {
          const double y = (r - 1.0) / log(r);
          m[i] = alpha == 1.5 ? y * sqrt(y) : pow(y, alpha);
        }
        part += m[i];
      }
    }
    // cumulative importance at the lane's bin edges, cm[j0 + i] = cb[i]: the lane's sums
    // r from the scan's exclusive value, raised to the largest chunk end of the lanes
    // before it (a maximum is exact, so the lane after this one sees this lane's top
    // cb[c] as its cb[0], bit for bit): cm is non-decreasing across lanes, and the
    // bins' intervals (cm[j], cm[j+1]] tile (0, cm[n]] whatever the sums' rounding
    double r[5];
    r[0] = wave_scan_f64(part) - part;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i + 1] = (i < c && j0 + i < n) ? r[i] + m[i] : r[i];
    const double carry = wave_scan_max_f64(dpp_f64<0x138, 0xf, true>(r[4]));  // lanes before (wave_shr:1)
    double cb[5];
    cb[0] = carry;
#pragma unroll
    for (int i = 1; i < 5; ++i) cb[i] = fmax(r[i], carry);
    const double stp = read_lane_f64(cb[4], (n - 1) / c) / n;  // cm[n] / n
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = j0 + i;
      if (i >= c || j >= n) break;
      const double lo = cb[i], hi = cb[i + 1];
      // the first interior edge above lo
      int k = static_cast<int>(lo / stp);
      k = k < 1 ? 1 : k;
      while (k > 1 && (k - 1) * stp > lo) --k;
      while (k < n && k * stp <= lo) ++k;
      if (k >= n) continue;
      const double e0 = eo[j], e1 = eo[j + 1];
      for (; k < n; ++k) {
        const double target = k * stp;
        if (j < n - 1 && target > hi) break;  // the last bin takes every remaining edge
        double frac = m[i] > 0.0 ? (target - lo) / m[i] : 0.0;
        frac = frac < 0.0 ? 0.0 : (frac > 1.0 ? 1.0 : frac);
        e_out[k] = e0 + frac * (e1 - e0);
      }
    }
    if (lane == 0) {
      e_out[0] = 0.0;
      e_out[n] = 1.0;
    }
  } else if (active && e_out != e_in) {
    for (int k = lane; k <= n; k += kWave) e_out[k] = eo[k];
  }
}

// one 64-lane block per dimension, in place
__global__ void k_refine(DevBufs b, int nbins, double alpha) {
  extern __shared__ unsigned char smem[];
  const int d = blockIdx.x, n = nbins;
  double* e = b.edges + d * (n + 1);
  refine_dim(true, false, n, alpha, b.hist + d * n, e, e, reinterpret_cast<double*>(smem));
}

// ---------------------------------------------------------------------------
// K5: inverse-variance combination over the iterations
// ---------------------------------------------------------------------------
__global__ void k_result(DevBufs b, int first, int n_iter) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int nzero = 0;
  double zsum = 0.0, ws = 0.0, iws = 0.0;
  for (int j = first; j < n_iter; ++j) {
    const double I = b.history[2 * j], v = b.history[2 * j + 1];
    if (v <= 0.0) {
      ++nzero;
      zsum += I;
    } else {
      ws += 1.0 / v;
      iws += I / v;
    }
  }
  const int n = n_iter - first;
  if (nzero) {
    b.result[0] = zsum / nzero;
    b.result[1] = 0.0;
    b.result[2] = 0.0;
  } else {
    const double I = iws / ws;
    double chi = 0.0;
    for (int j = first; j < n_iter; ++j) {
      const double dI = b.history[2 * j] - I;
      chi += dI * dI / b.history[2 * j + 1];
    }
    b.result[0] = I;
    b.result[1] = sqrt(1.0 / ws);
    b.result[2] = n > 1 ? chi / (n - 1) : 0.0;
  }
  b.result[3] = n;
}

// training data for the learned proposal: the uniform points (binary32) and weights
// of events [first, first+n) of iteration iter (8 dimensions)
__global__ void k_export(const double* __restrict__ rec_w, uint64_t seed, uint32_t iter, int64_t first, int64_t n,
                         float* y, double* w) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double u[8];
    event_uniforms<8>(seed, iter, static_cast<uint64_t>(first + i), 8, u);
#pragma unroll
    for (int d = 0; d < 8; ++d) y[i * 8 + d] = static_cast<float>(u[d]);
    w[i] = rec_w[first + i];
  }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_uniform_grid(double* edges, int ndim, int nbins) {
  for (int i = threadIdx.x; i < ndim * (nbins + 1); i += blockDim.x) {
    const int k = i % (nbins + 1);
    edges[i] = static_cast<double>(k) / nbins;
  }
}

}  // namespace vg

// ===========================================================================
// host library
// ===========================================================================
using namespace vg;

namespace {

thread_local std::string g_last_hip_error;

struct Layout {
  size_t edges, edges_alt, rec_w, rec_bins, rec_obs, maxw, cnt, fxs, part_acc, acc_tot, hist, obs_acc, obs_out,
      strat_acc, history, iter_out, result, total;
};

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

Layout make_layout(int D, int n, int64_t maxN) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const int words = (D + 3) / 4;
  L.edges = take(sizeof(double) * D * (n + 1));
  L.edges_alt = take(sizeof(double) * D * (n + 1));
  L.rec_w = take(sizeof(double) * maxN);
  L.rec_bins = take(sizeof(uint32_t) * words * maxN);
  L.rec_obs = take(maxN);
  L.maxw = take(sizeof(unsigned long long) * 4);
  L.cnt = take(sizeof(unsigned long long) * 4);
  L.fxs = take(sizeof(int) * 8);
  // digit columns for the largest observable histogram
  const int ncol_max = hist_cols(D * n) + obs_cols(VEGAS_MAX_OBS_BINS);
  L.part_acc = take(sizeof(long long) * kMaxRowsAcc * part_ld(ncol_max));
  L.acc_tot = take(sizeof(long long) * ncol_max);
  L.hist = take(sizeof(double) * (D * n + 2));
  L.obs_acc = take(sizeof(double) * (3 * kObsLd + 2));
  L.obs_out = take(sizeof(double) * 4 * kObsLd);
  L.strat_acc = take(sizeof(long long) * 4 * kStrataBlocks);
  L.history = take(sizeof(double) * 2 * VEGAS_MAX_ITER);
  L.iter_out = take(sizeof(double) * 8);
  L.result = take(sizeof(double) * 4);
  L.total = off;
  return L;
}

int process_ndim(int process, int requested) {
  switch (process) {
    case VEGAS_GAUSS:
    case VEGAS_GENZ: return requested;
    case VEGAS_EEMUMU: return 2;
    case VEGAS_DY_Z: return 3;
    case VEGAS_W_PLUS: return 4;
    case VEGAS_WW_4L: return 8;
    case VEGAS_WW_HAD: return 10;
    default: return -1;
  }
}

int validate(const vegas_config* c, int64_t max_events) {
  if (!c) return VEGAS_EINVAL;
  if (c->process < VEGAS_GAUSS || c->process > VEGAS_WW_HAD) return VEGAS_EINVAL;
  const int D = process_ndim(c->process, c->ndim);
  if (D < 1 || D > VEGAS_MAX_DIM || D != c->ndim) return VEGAS_EINVAL;
  if (c->nbins < 2 || c->nbins > VEGAS_MAX_BINS) return VEGAS_EINVAL;
  if (!(c->alpha >= 0.0) || !std::isfinite(c->alpha)) return VEGAS_EINVAL;
  if (c->nparams < 0 || c->nparams > VEGAS_MAX_PARAMS) return VEGAS_EINVAL;
  if (c->nparams > 0 && !c->params) return VEGAS_EINVAL;
  if (c->precision != VEGAS_FP64 && c->precision != VEGAS_FP32_ME) return VEGAS_EINVAL;
  // binary32 amplitudes only at the partonic W+W- energy: in the hadronic process
  // sqrt(shat) reaches sqrt(S), where the diagrams cancel by (shat / M_W^2)^2
  if (c->precision == VEGAS_FP32_ME && c->process != VEGAS_WW_4L) return VEGAS_EINVAL;
  const int w = c->waves_per_block;
  if (!(w == 0 || w == 1 || w == 2 || w == 4 || w == 8 || w == 16)) return VEGAS_EINVAL;
  if (c->max_blocks < 0) return VEGAS_EINVAL;
  if (max_events < 2 || max_events >= (int64_t(1) << 31)) return VEGAS_EINVAL;
  switch (c->process) {
    case VEGAS_GAUSS:
      if (c->nparams < 2 || !(c->params[1] > 0.0)) return VEGAS_EINVAL;
      break;
    case VEGAS_GENZ:
      if (c->nparams < 1 + 2 * D) return VEGAS_EINVAL;
      break;
    default:
      if (c->nparams < VEGAS_NPHYS) return VEGAS_EINVAL;
  }
  if (c->process == VEGAS_WW_HAD) {  // the sqrt(shat) window: 0 < MLO < MHI <= sqrt(S)
    const double rs = c->params[VEGAS_P_SQRTS], lo = c->params[VEGAS_P_MLO];
    const double hi = c->params[VEGAS_P_MHI] > 0 ? c->params[VEGAS_P_MHI] : rs;
    if (!(lo > 0.0 && lo < hi && hi <= rs && std::isfinite(rs))) return VEGAS_EINVAL;
  }
  return VEGAS_OK;
}

// configuration-wide constants, computed once on the host
PhysConst make_consts(const vegas_config* c, const double* p) {
  PhysConst k;
  std::memset(&k, 0, sizeof(k));
  k.process = c->process;
  k.ndim = c->ndim;
  k.nbins = c->nbins;
  if (c->process == VEGAS_GAUSS) {
    const double mu = p[0], sg = p[1];
    k.mu = mu;
    k.inv2s2 = 1.0 / (2.0 * sg * sg);
    k.gnorm = 1.0 / (sg * std::sqrt(2.0 * kPi));
    return k;
  }
  if (c->process == VEGAS_GENZ) {
    k.family = static_cast<int>(p[0]);
    for (int d = 0; d < c->ndim; ++d) {
      k.ga[d] = p[1 + d];
      k.gw[d] = p[1 + c->ndim + d];
    }
    return k;
  }
  const double alpha = p[VEGAS_P_ALPHA], sw2 = p[VEGAS_P_SW2];
  const double MZ = p[VEGAS_P_MZ], GZ = p[VEGAS_P_GZ], MW = p[VEGAS_P_MW], GW = p[VEGAS_P_GW];
  const double rs = p[VEGAS_P_SQRTS];
  const double sw = std::sqrt(sw2), cw = std::sqrt(1.0 - sw2);
  const double e2 = 4.0 * kPi * alpha;
  const double g2 = e2 / sw2;
  k.conv = p[VEGAS_P_CONV];
  k.pdfA = p[VEGAS_P_PDF_A];
  k.pdfa = p[VEGAS_P_PDF_a];
  k.pdfb = p[VEGAS_P_PDF_b];
  {
    const double a2 = 2.0 * k.pdfa;
    const bool a_ok = a2 == std::floor(a2) && std::fabs(a2) <= 8.0;
    const bool b_ok = k.pdfb == std::floor(k.pdfb) && k.pdfb >= 0.0 && k.pdfb <= 16.0;
    k.pdf_pow = a_ok && b_ok ? 1 : 0;
    k.pdf_a2 = a_ok ? static_cast<int>(a2) : 0;
    k.pdf_b = b_ok ? static_cast<int>(k.pdfb) : 0;
  }
  k.invS = 1.0 / (rs * rs);
  k.e4 = e2 * e2;
  k.s_ee = rs * rs;
  if (c->process == VEGAS_DY_Z) {
    k.M2 = MZ * MZ;
    k.MG = MZ * GZ;
    const double lo = p[VEGAS_P_MLO], hi = p[VEGAS_P_MHI] > 0 ? p[VEGAS_P_MHI] : rs;
    k.m2lo = lo * lo;
    k.invMG = 1.0 / k.MG;
    k.tlo = (k.m2lo - MZ * MZ) / k.MG;
    k.rho_lo = std::atan(k.tlo);
    k.rho_rng = std::atan((hi * hi - MZ * MZ) / k.MG) - k.rho_lo;
    k.mz2 = MZ * MZ;
    k.mzgz = MZ * GZ;
    k.e4_12 = e2 * e2 / 12.0;
    const double gl[2] = {(-0.5 + sw2) / (sw * cw), sw / cw};
    for (int q = 0; q < 2; ++q) {
      const double Q = q == 0 ? 2.0 / 3.0 : -1.0 / 3.0, T3 = q == 0 ? 0.5 : -0.5;
      const double gq[2] = {(T3 - Q * sw2) / (sw * cw), -Q * sw / cw};
      k.qql[q] = -Q;
      for (int h = 0; h < 2; ++h)
        for (int hp = 0; hp < 2; ++hp) k.gg[q][2 * h + hp] = gq[h] * gl[hp];
    }
  } else if (c->process == VEGAS_W_PLUS) {
    k.M2 = MW * MW;
    k.MG = MW * GW;
    const double lo = p[VEGAS_P_MLO], hi = p[VEGAS_P_MHI] > 0 ? p[VEGAS_P_MHI] : rs;
    k.m2lo = lo * lo;
    k.invMG = 1.0 / k.MG;
    k.tlo = (k.m2lo - MW * MW) / k.MG;
    k.rho_lo = std::atan(k.tlo);
    k.rho_rng = std::atan((hi * hi - MW * MW) / k.MG) - k.rho_lo;
    const double v = p[VEGAS_P_VUD];
    k.g4v2_24 = g2 * g2 * v * v / 24.0;
    k.ptmin2 = p[VEGAS_P_PTMIN] * p[VEGAS_P_PTMIN];
    const double th = std::tanh(p[VEGAS_P_ETAMAX]);
    k.th2 = th * th;
  } else if (c->process == VEGAS_WW_4L || c->process == VEGAS_WW_HAD) {
    k.M2 = MW * MW;
    k.MG = MW * GW;
    k.rs = rs;
    k.shat = rs * rs;
    k.m2lo = 0.0;
    k.invMG = 1.0 / k.MG;
    k.tlo = (0.0 - MW * MW) / k.MG;
    k.rho_lo = std::atan(k.tlo);
    k.rho_rng = std::atan((k.shat - MW * MW) / k.MG) - k.rho_lo;
    k.gs = std::sqrt(g2) / std::sqrt(2.0);
    k.ct = -0.5 * g2;
    // Cs = e^2 (Q/shat + gZ (cw/sw) / (shat - MZ^2 + i MZ GZ))
    const double dr = k.shat - MZ * MZ, di = MZ * GZ, dd = dr * dr + di * di;
    double csr2 = 0.0;
    for (int q = 0; q < 2; ++q) {
      const double Q = q == 0 ? 2.0 / 3.0 : -1.0 / 3.0, T3 = q == 0 ? 0.5 : -0.5;
      for (int h = 0; h < 2; ++h) {
        const double gz = h == 0 ? (T3 - Q * sw2) / (sw * cw) : -Q * sw / cw;
        const double f = gz * cw / sw;
        k.cs_re[q][h] = e2 * (Q / k.shat + f * dr / dd);
        k.cs_im[q][h] = e2 * (-f * di / dd);
      }
      csr2 += k.cs_re[q][1] * k.cs_re[q][1] + k.cs_im[q][1] * k.cs_im[q][1];
    }
    k.csR2 = csr2;
    if (c->process == VEGAS_WW_HAD) {
      const double S = rs * rs, lo = p[VEGAS_P_MLO], hi = p[VEGAS_P_MHI] > 0 ? p[VEGAS_P_MHI] : rs;
      const double Llo = std::log(lo * lo / S), Lhi = std::log(hi * hi / S);
      k.S = S;
      k.Lhi = Lhi;
      k.Lrng = Llo - Lhi;
      k.Ldiff = Lhi - Llo;
      k.mz2 = MZ * MZ;
      k.mzgz = MZ * GZ;
      for (int q = 0; q < 2; ++q) {
        const double Q = q == 0 ? 2.0 / 3.0 : -1.0 / 3.0, T3 = q == 0 ? 0.5 : -0.5;
        k.csq[q] = e2 * Q;
        for (int h = 0; h < 2; ++h) {
          const double gz = h == 0 ? (T3 - Q * sw2) / (sw * cw) : -Q * sw / cw;
          k.csf[q][h] = e2 * (gz * cw / sw);
        }
      }
    }
  }
  // uniform products, with the kernels' roundings (one product each)
  k.MG2 = k.MG * k.MG;
  k.MGt = k.MG * (1.0 + k.tlo * k.tlo);
  k.mzgz2 = k.mzgz * k.mzgz;
  return k;
}

}  // namespace

// Scratch for the allocation-free adjoint (vegas_grad_noalloc): static device memory,
// one copy per GPU that loads this library, held until the process ends.  Host code
// never passes this name to a kernel (on the host it is only a stand-in for the
// symbol): each device's address is taken once with hipGetSymbolAddress and kept.
static __device__ __align__(256) double scratch[VEGAS_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

// the current device's address of the scratch array (taken on its first use)
hipError_t scratch_address(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}
}  // namespace

struct vegas_state {
  vegas_config cfg;
  double params[VEGAS_MAX_PARAMS];
  int D, n;
  int64_t maxN;
  hipStream_t stream;
  int device;
  void* base;
  bool owns;
  Layout L;
  DevBufs b;
  PhysConst pc;
  uint32_t iter;      // next iteration index
  bool have_hist;     // an iteration ran since init / the last refine
  bool any_iter;
  bool last_flow;     // the last iteration used the learned proposal
  int64_t last_n;
  int wpb, max_blocks;
  int event_lds, acc_lds, fused_lds, fin_lds;
  int acc_dpg, acc_groups;      // histogram dimensions per k_accum block, and blocks along y
  bool fused_ok;                // the fused fold fits in LDS for this configuration
  bool spec_ok;                 // the finalisation can also refine (scratch fits, D <= 16)
  bool spec_ready;              // b.edges_alt holds the refinement of the current grid and histogram
  int nobs, obs_first;          // observable histogram: bins (0 = off) and first combined iteration
  double obs_lo, obs_hi;
  bool obs_have;                // an iteration ran since the observable was set
  int strata_m;                 // stratified sampling: strata per axis (0 = off)
  double strata_beta;           // > 0: adaptive allocation n_h ~ sigma_h^beta
  // adaptive allocation scratch (library-allocated on first use): sigma_h, p_h, counts
  // and offsets per hypercube (capacity s_capH), per-block partial sums, the
  // hypercube of each event [maxN]
  double* s_sig;
  double* s_p;
  double* s_part;
  long long* s_partf;
  int32_t *s_cnt, *s_off, *s_cube;
  int64_t s_capH;
  bool s_have_sig;              // s_sig holds the last stratified iteration's sigma_h
  int64_t last_strata_npc;      // last iteration: events per hypercube (equal counts), -1 adaptive,
                                //   0 not stratified
  size_t smem_max;              // LDS per block the launches may use
  int refine_lds;               // LDS of the refinement scratch: D * 4 (n + 1) doubles
  bool scale_valid;             // the device holds scales from a previous iteration (b.fxs)
  int ncu, occ_event, occ_event_fused, occ_acc;  // CUs, and resident 256-thread blocks per CU
  // optional per-stage kernel timing with HIP events on the handle's stream:
  // bit s set = the kernels of stage s are timed
  uint32_t timing;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;  // (stage, start/stop)
  double stage_ms[4];
  int64_t stage_n[4];
  int64_t last_launch[4];  // event blocks, threads per block, fold rows, fold columns of the last iteration
  // adjoint scratch (library-allocated on first use, grown on demand)
  double* gbuf;
  size_t gbuf_doubles;
  double* scratch;            // this device's copy of the static scratch array (vegas_grad_noalloc)
  std::string scratch_error;  // why its address could not be taken, if it could not
  // a recorded schedule (vegas_run_schedule): its event counts, the host state it starts
  // from and the one it leaves, and the instantiated graph of its launches
  hipGraphExec_t sched_exec = nullptr;
  hipStream_t cap_stream = nullptr;  // the recording's own stream (the caller's may be the null stream)
  std::vector<int64_t> sched_n;
  int sched_refine = 0;
  unsigned char sched_pre[256], sched_post[256];
};

#define VG_HIP(call)                                                  \
  do {                                                                \
    hipError_t e_ = (call);                                           \
    if (e_ != hipSuccess) {                                           \
      g_last_hip_error = std::string(#call) + ": " + hipGetErrorString(e_); \
      return VEGAS_EHIP;                                              \
    }                                                                 \
  } while (0)

namespace {

int pick_threads(const vegas_state* h) { return kWave * (h->wpb > 0 ? h->wpb : 4); }

// grid-stride launches: enough blocks to fill every CU at the kernel's occupancy
// (one resident wave of blocks), capped by the partial-buffer rows and the knob.  Past
// one block per CU, whole rounds of blocks (a multiple of the CU count) and at least
// kMinPasses grid-stride passes per lane: each block also clears and writes a row of
// digit sums, which few passes do not repay (W+ at 3e5 events: 15.6 us with 256 blocks,
// 21.0 us with 1024; Drell-Yan at 1e5: 9.2 us with 256, 10.7 us with 391)
constexpr int64_t kMinPasses = 4;
int pick_blocks(const vegas_state* h, int64_t nev, int threads, int occ, int rows_cap) {
  int64_t nb = (nev + threads - 1) / threads;
  int64_t fill = static_cast<int64_t>(h->ncu) * (occ > 0 ? occ : 1) * 256 / threads;
  if (fill < 1) fill = 1;
  const int64_t ncu = h->ncu > 0 ? h->ncu : 1;
  if (h->max_blocks <= 0 && nb > ncu && fill >= ncu) {
    int64_t rounds = nev / (ncu * threads * kMinPasses);
    rounds = rounds < 1 ? 1 : rounds;
    nb = ncu * rounds;
  }
  if (nb > fill) nb = fill;
  if (h->max_blocks > 0 && nb > h->max_blocks) nb = h->max_blocks;
  if (nb > rows_cap) nb = rows_cap;
  if (nb < 1) nb = 1;
  return static_cast<int>(nb);
}

// two instantiations per integrand: up to 4 waves per block (the register budget of a
// 256-thread block, the performance path) and up to 16 waves (for the launch knob)
hipEvent_t pool_event(vegas_state* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// launch on the handle's stream; with timing on, the start and stop events are
// bound to the kernel's own dispatch (no marker packets between kernels)
struct TimedLaunch {
  vegas_state* h;
  int stage;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TimedLaunch(vegas_state* hh, int st) : h(hh), stage(st) {
    if (!((h->timing >> stage) & 1u)) return;
    e0 = pool_event(h);
    e1 = e0 ? pool_event(h) : nullptr;
    if (e0 && !e1) {
      h->ev_pool.push_back(e0);
      e0 = nullptr;
    }
  }
  hipError_t done() {
    const hipError_t err = hipGetLastError();
    if (e0 && e1) {
      if (err == hipSuccess) {
        h->ev_pending.push_back({stage, {e0, e1}});
      } else {
        h->ev_pool.push_back(e0);
        h->ev_pool.push_back(e1);
      }
    }
    return err;
  }
};

// fold finished event pairs into the per-stage totals (the stream must be idle)
void stage_collect(vegas_state* h) {
  for (auto& p : h->ev_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
      h->stage_ms[p.first] += ms;
      h->stage_n[p.first] += 1;
    }
    h->ev_pool.push_back(p.second.first);
    h->ev_pool.push_back(p.second.second);
  }
  h->ev_pending.clear();
}

template <int PROC, int PREC, int D, bool EXT, bool FUSED, bool OBS, bool STRAT>
hipError_t launch_event_tfo(vegas_state* h, const EventArgs& a, int blocks, int threads) {
  TimedLaunch t(h, 0);
  const int lds = FUSED ? h->fused_lds : h->event_lds;
  if (EXT || threads <= 256)
    hipExtLaunchKernelGGL((k_event<PROC, PREC, D, 256, EXT, FUSED, OBS, STRAT>), dim3(blocks),
                          dim3(EXT ? 256 : threads), lds, h->stream, t.e0, t.e1, 0, a);
  else
    hipExtLaunchKernelGGL((k_event<PROC, PREC, D, 1024, false, FUSED, OBS, STRAT>), dim3(blocks), dim3(threads), lds,
                          h->stream, t.e0, t.e1, 0, a);
  return t.done();
}

// the learned proposal replaces the stratified placement, so EXT kernels have no STRAT variant
template <int PROC, int PREC, int D, bool EXT, bool FUSED, bool OBS>
hipError_t launch_event_tfs(vegas_state* h, const EventArgs& a, int blocks, int threads) {
  if constexpr (!EXT)
    if (a.strata_m > 0) return launch_event_tfo<PROC, PREC, D, EXT, FUSED, OBS, true>(h, a, blocks, threads);
  return launch_event_tfo<PROC, PREC, D, EXT, FUSED, OBS, false>(h, a, blocks, threads);
}

template <int PROC, int PREC, int D, bool EXT, bool FUSED>
hipError_t launch_event_tf(vegas_state* h, const EventArgs& a, int blocks, int threads) {
  return a.nobs > 0 ? launch_event_tfs<PROC, PREC, D, EXT, FUSED, true>(h, a, blocks, threads)
                    : launch_event_tfs<PROC, PREC, D, EXT, FUSED, false>(h, a, blocks, threads);
}

template <int PROC, int PREC, int D, bool EXT = false>
hipError_t launch_event_t(vegas_state* h, const EventArgs& a, int blocks, int threads, bool fused) {
  return fused ? launch_event_tf<PROC, PREC, D, EXT, true>(h, a, blocks, threads)
               : launch_event_tf<PROC, PREC, D, EXT, false>(h, a, blocks, threads);
}

hipError_t launch_event(vegas_state* h, const EventArgs& a, int blocks, int threads, bool fused) {
  switch (h->cfg.process) {
    case VEGAS_GAUSS: return launch_event_t<VEGAS_GAUSS, VEGAS_FP64, 0>(h, a, blocks, threads, fused);
    case VEGAS_GENZ: return launch_event_t<VEGAS_GENZ, VEGAS_FP64, 0>(h, a, blocks, threads, fused);
    case VEGAS_EEMUMU: return launch_event_t<VEGAS_EEMUMU, VEGAS_FP64, 2>(h, a, blocks, threads, fused);
    case VEGAS_DY_Z: return launch_event_t<VEGAS_DY_Z, VEGAS_FP64, 3>(h, a, blocks, threads, fused);
    case VEGAS_W_PLUS: return launch_event_t<VEGAS_W_PLUS, VEGAS_FP64, 4>(h, a, blocks, threads, fused);
    case VEGAS_WW_4L:
      if (h->cfg.precision == VEGAS_FP32_ME)
        return launch_event_t<VEGAS_WW_4L, VEGAS_FP32_ME, 8>(h, a, blocks, threads, fused);
      return launch_event_t<VEGAS_WW_4L, VEGAS_FP64, 8>(h, a, blocks, threads, fused);
    case VEGAS_WW_HAD:
      return launch_event_t<VEGAS_WW_HAD, VEGAS_FP64, 10>(h, a, blocks, threads, fused);
  }
  return hipErrorInvalidValue;
}

// learned-proposal variants (8-dimensional integrands only, 256-thread blocks)
hipError_t launch_event_ext(vegas_state* h, const EventArgs& a, int blocks, bool fused) {
  switch (h->cfg.process) {
    case VEGAS_GAUSS: return launch_event_t<VEGAS_GAUSS, VEGAS_FP64, 0, true>(h, a, blocks, 256, fused);
    case VEGAS_GENZ: return launch_event_t<VEGAS_GENZ, VEGAS_FP64, 0, true>(h, a, blocks, 256, fused);
    case VEGAS_WW_4L:
      if (h->cfg.precision == VEGAS_FP32_ME)
        return launch_event_t<VEGAS_WW_4L, VEGAS_FP32_ME, 8, true>(h, a, blocks, 256, fused);
      return launch_event_t<VEGAS_WW_4L, VEGAS_FP64, 8, true>(h, a, blocks, 256, fused);
    default: return hipErrorInvalidValue;
  }
}

bool ext_supported(const vegas_state* h) {
  const int p = h->cfg.process;
  return h->D == 8 && (p == VEGAS_GAUSS || p == VEGAS_GENZ || p == VEGAS_WW_4L);
}

template <int PROC, int PREC, int D, bool FUSED, bool OBS>
const void* event_kernel_ptr(bool strat) {
  return strat ? reinterpret_cast<const void*>(&k_event<PROC, PREC, D, 256, false, FUSED, OBS, true>)
               : reinterpret_cast<const void*>(&k_event<PROC, PREC, D, 256, false, FUSED, OBS, false>);
}

template <int PROC, int PREC, int D>
int occupancy_event_t(int lds, bool fused, bool obs, bool strat) {
  int nb = 0;
  const void* k = fused ? (obs ? event_kernel_ptr<PROC, PREC, D, true, true>(strat)
                               : event_kernel_ptr<PROC, PREC, D, true, false>(strat))
                        : (obs ? event_kernel_ptr<PROC, PREC, D, false, true>(strat)
                               : event_kernel_ptr<PROC, PREC, D, false, false>(strat));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int occupancy_event(const vegas_state* h, bool fused) {
  const int lds = fused ? h->fused_lds : h->event_lds;
  const bool o = h->nobs > 0, st = h->strata_m > 0;
  switch (h->cfg.process) {
    case VEGAS_GAUSS: return occupancy_event_t<VEGAS_GAUSS, VEGAS_FP64, 0>(lds, fused, o, st);
    case VEGAS_GENZ: return occupancy_event_t<VEGAS_GENZ, VEGAS_FP64, 0>(lds, fused, o, st);
    case VEGAS_EEMUMU: return occupancy_event_t<VEGAS_EEMUMU, VEGAS_FP64, 2>(lds, fused, o, st);
    case VEGAS_DY_Z: return occupancy_event_t<VEGAS_DY_Z, VEGAS_FP64, 3>(lds, fused, o, st);
    case VEGAS_W_PLUS: return occupancy_event_t<VEGAS_W_PLUS, VEGAS_FP64, 4>(lds, fused, o, st);
    case VEGAS_WW_4L:
      if (h->cfg.precision == VEGAS_FP32_ME)
        return occupancy_event_t<VEGAS_WW_4L, VEGAS_FP32_ME, 8>(lds, fused, o, st);
      return occupancy_event_t<VEGAS_WW_4L, VEGAS_FP64, 8>(lds, fused, o, st);
    case VEGAS_WW_HAD:
      return occupancy_event_t<VEGAS_WW_HAD, VEGAS_FP64, 10>(lds, fused, o, st);
  }
  return 1;
}

// LDS sizes, the fused-fold and speculative-refinement switches and the occupancies
// for the current digit columns (grid histogram plus the observable's bins)
void configure_lds(vegas_state* h) {
  const int D = h->D, n = h->n;
  const size_t smem = h->smem_max;
  const int ocol = obs_cols(h->nobs);
  // histogram dimensions per k_accum block: as many as fit in the block's LDS
  // (the y == 0 blocks also hold S1, S2 and the observable's bins)
  const size_t per_dim = sizeof(long long) * kD2 * n;
  int dpg = static_cast<int>((smem - sizeof(long long) * (kColHist + ocol)) / per_dim);
  dpg = dpg < 1 ? 1 : (dpg > D ? D : dpg);
  h->acc_dpg = dpg;
  h->acc_groups = (D + dpg - 1) / dpg;
  h->acc_lds = static_cast<int>(sizeof(long long) * (hist_cols(dpg * n) + ocol));
  const int full = static_cast<int>(sizeof(long long) * (hist_cols(D * n) + ocol));
  // 10 or more dimensions: the lanes' S1, S2 digit sums also live in LDS ([7][256])
  h->fused_lds = h->event_lds + full + (D >= 10 ? static_cast<int>(sizeof(long long) * kLane * 256) : 0);
  h->fused_ok = h->fused_lds <= kFusedLdsMax;
  h->fin_lds = h->fused_ok ? full : 0;
  h->refine_lds = static_cast<int>(sizeof(double) * 4 * D * (n + 1));
  const int obs_lds = h->nobs ? static_cast<int>(sizeof(double) * 2 * (h->nobs + 2)) : 0;
  h->spec_ok = D <= 16 && h->fin_lds + h->refine_lds + obs_lds <= static_cast<int>(smem);
  h->occ_event = occupancy_event(h, false);
  h->occ_event_fused = h->fused_ok ? occupancy_event(h, true) : 1;
  int nb = 0;
  h->occ_acc = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_accum), 256,
                                                            h->acc_lds) == hipSuccess && nb > 0
                   ? nb
                   : 1;
}

}  // namespace

extern "C" {

const char* vegas_strerror(int status) {
  switch (status) {
    case VEGAS_OK: return "ok";
    case VEGAS_EINVAL: return "invalid configuration or argument";
    case VEGAS_ESTATE: return "call out of order";
    case VEGAS_ENOMEM: return "workspace too small or device allocation failed";
    case VEGAS_EHIP: return g_last_hip_error.empty() ? "HIP runtime error" : g_last_hip_error.c_str();
    case VEGAS_ETOOBIG: return "request larger than the allocation-free scratch (VEGAS_SCRATCH_DOUBLES)";
    default: return "unknown status";
  }
}

int vegas_workspace_size(const vegas_config* cfg, int64_t max_events, size_t* bytes) {
  const int v = validate(cfg, max_events);
  if (v != VEGAS_OK) return v;
  if (!bytes) return VEGAS_EINVAL;
  *bytes = make_layout(cfg->ndim, cfg->nbins, max_events).total;
  return VEGAS_OK;
}

int vegas_init(const vegas_config* cfg, int64_t max_events, void* workspace, size_t ws_bytes,
               void* stream, vegas_handle* out) {
  if (!out) return VEGAS_EINVAL;
  *out = nullptr;
  const int v = validate(cfg, max_events);
  if (v != VEGAS_OK) return v;
  const int D = cfg->ndim, n = cfg->nbins;
  Layout L = make_layout(D, n, max_events);
  if (workspace && (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) & 255)))
    return VEGAS_ENOMEM;
  vegas_state* h = new (std::nothrow) vegas_state();
  if (!h) return VEGAS_ENOMEM;
  h->cfg = *cfg;
  std::memset(h->params, 0, sizeof(h->params));
  if (cfg->nparams) std::memcpy(h->params, cfg->params, sizeof(double) * cfg->nparams);
  h->cfg.params = h->params;
  h->D = D;
  h->n = n;
  h->maxN = max_events;
  h->stream = static_cast<hipStream_t>(stream);
  h->L = L;
  h->wpb = cfg->waves_per_block;
  h->max_blocks = cfg->max_blocks;
  h->event_lds = static_cast<int>(sizeof(double) * D * (n + 1));
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return VEGAS_EHIP;
  }
  // this device's scratch array for the allocation-free adjoint; a failure here only
  // disables that call (it then reports the error)
  {
    const hipError_t e = scratch_address(h->device, &h->scratch);
    if (e != hipSuccess) {
      h->scratch = nullptr;
      h->scratch_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    }
  }
  if (workspace) {
    h->base = workspace;
    h->owns = false;
  } else {
    if (hipMalloc(&h->base, L.total) != hipSuccess) {
      delete h;
      return VEGAS_ENOMEM;
    }
    h->owns = true;
  }
  char* B = static_cast<char*>(h->base);
  h->b.edges = reinterpret_cast<double*>(B + L.edges);
  h->b.edges_alt = reinterpret_cast<double*>(B + L.edges_alt);
  h->b.rec_w = reinterpret_cast<double*>(B + L.rec_w);
  h->b.rec_bins = reinterpret_cast<uint32_t*>(B + L.rec_bins);
  h->b.maxw = reinterpret_cast<unsigned long long*>(B + L.maxw);
  h->b.cnt = reinterpret_cast<unsigned long long*>(B + L.cnt);
  h->b.fxs = reinterpret_cast<int*>(B + L.fxs);
  h->b.maxw_next = h->b.maxw + 2;
  h->b.cnt_next = h->b.cnt + 2;
  h->b.fxs_next = h->b.fxs + 4;
  h->b.part_acc = reinterpret_cast<long long*>(B + L.part_acc);
  h->b.acc_tot = reinterpret_cast<long long*>(B + L.acc_tot);
  h->b.hist = reinterpret_cast<double*>(B + L.hist);
  h->b.rec_obs = reinterpret_cast<uint8_t*>(B + L.rec_obs);
  h->b.obs_acc = reinterpret_cast<double*>(B + L.obs_acc);
  h->b.obs_out = reinterpret_cast<double*>(B + L.obs_out);
  h->b.strat_part = reinterpret_cast<long long*>(B + L.strat_acc);
  h->b.history = reinterpret_cast<double*>(B + L.history);
  h->b.iter_out = reinterpret_cast<double*>(B + L.iter_out);
  h->b.result = reinterpret_cast<double*>(B + L.result);
  h->pc = make_consts(&h->cfg, h->params);
  {
    hipDeviceProp_t prop;
    const bool have_prop = hipGetDeviceProperties(&prop, h->device) == hipSuccess;
    h->ncu = have_prop ? prop.multiProcessorCount : 256;
    if (h->ncu < 1) h->ncu = 1;
    size_t smem = have_prop ? prop.sharedMemPerBlock : 65536;
    h->smem_max = smem > 65536 ? 65536 : smem;
    configure_lds(h);
  }
  // zero the device-wide atomics and every buffer after the partials with a fill kernel
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, h->stream,
                     reinterpret_cast<unsigned long long*>(B + L.maxw),
                     static_cast<int64_t>((L.part_acc - L.maxw) / 8));
  hipLaunchKernelGGL(k_fill_u64, dim3(64), dim3(256), 0, h->stream,
                     reinterpret_cast<unsigned long long*>(B + L.hist),
                     static_cast<int64_t>((L.total - L.hist) / 8));
  hipLaunchKernelGGL(k_uniform_grid, dim3(1), dim3(256), 0, h->stream, h->b.edges, D, n);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    g_last_hip_error = "vegas_init: initial fill failed";
    if (h->owns) (void)hipFree(h->base);
    delete h;
    return VEGAS_EHIP;
  }
  *out = h;
  return VEGAS_OK;
}

int vegas_destroy(vegas_handle h) {
  if (!h) return VEGAS_EINVAL;
  int rc = VEGAS_OK;
  if (hipStreamSynchronize(h->stream) != hipSuccess) rc = VEGAS_EHIP;
  for (auto& p : h->ev_pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->sched_exec) (void)hipGraphExecDestroy(h->sched_exec);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->gbuf) (void)hipFree(h->gbuf);
  if (h->s_sig) (void)hipFree(h->s_sig);
  if (h->s_cnt) (void)hipFree(h->s_cnt);
  if (h->s_off) (void)hipFree(h->s_off);
  if (h->s_cube) (void)hipFree(h->s_cube);
  if (h->s_p) (void)hipFree(h->s_p);
  if (h->s_part) (void)hipFree(h->s_part);
  if (h->s_partf) (void)hipFree(h->s_partf);
  if (h->owns) {
    if (hipStreamSynchronize(h->stream) != hipSuccess) rc = VEGAS_EHIP;
    if (hipFree(h->base) != hipSuccess) rc = VEGAS_EHIP;
  }
  delete h;
  return rc;
}

int vegas_last_launch(vegas_handle h, int64_t* info) {
  if (!h || !info) return VEGAS_EINVAL;
  if (!h->any_iter) return VEGAS_ESTATE;
  for (int i = 0; i < 4; ++i) info[i] = h->last_launch[i];
  return VEGAS_OK;
}

int vegas_set_timing(vegas_handle h, int32_t stages) {
  if (!h || stages < 0 || stages > VEGAS_TIME_ALL) return VEGAS_EINVAL;
  h->timing = static_cast<uint32_t>(stages);
  return VEGAS_OK;
}

int vegas_stage_times(vegas_handle h, double* ms, int64_t* launches, int32_t reset) {
  if (!h) return VEGAS_EINVAL;
  VG_HIP(hipStreamSynchronize(h->stream));
  stage_collect(h);
  for (int i = 0; i < 4; ++i) {
    if (ms) ms[i] = h->stage_ms[i];
    if (launches) launches[i] = h->stage_n[i];
  }
  if (reset)
    for (int i = 0; i < 4; ++i) {
      h->stage_ms[i] = 0.0;
      h->stage_n[i] = 0;
    }
  return VEGAS_OK;
}

int vegas_set_launch(vegas_handle h, int32_t waves_per_block, int32_t max_blocks) {
  if (!h) return VEGAS_EINVAL;
  const int w = waves_per_block;
  if (!(w == 0 || w == 1 || w == 2 || w == 4 || w == 8 || w == 16) || max_blocks < 0) return VEGAS_EINVAL;
  h->wpb = w;
  h->max_blocks = max_blocks;
  return VEGAS_OK;
}

}  // extern "C"

namespace vg {
int flow_sample_events(vegas_flow f, hipStream_t s, uint64_t seed, uint32_t iter, int64_t n, const float** y,
                       const float** lq);
int flow_sample_finish(vegas_flow f, hipStream_t s);

void record_hip_error(const char* what, hipError_t e) {
  g_last_hip_error = std::string(what) + ": " + hipGetErrorString(e);
}
}  // namespace vg

namespace {

// one iteration: events (from the counter stream, or from the learned proposal's
// points when ext_y is given), then the exact accumulation and the combination
// hypercubes of the stratified sampling (0: off; < 0: more than 2^31 - 1)
int64_t strata_cubes(const vegas_state* h) {
  if (h->strata_m <= 0) return 0;
  int64_t H = 1;
  for (int d = 0; d < h->D; ++d) {
    H *= h->strata_m;
    if (H > 2147483647LL) return -1;
  }
  return H;
}

int run_iteration(vegas_handle h, int64_t n_req, const float* ext_y, const float* ext_lq,
                  vegas_iter_result* out) {
  // stratified: npc = floor(n / H) events in each of the H hypercubes, n = H npc used
  const int64_t H = ext_y ? 0 : strata_cubes(h);
  const int64_t npc = H > 0 ? n_req / H : 0;
  if (H < 0 || (H > 0 && npc < 2)) return VEGAS_EINVAL;
  // adaptive: every requested event is used, n_h from the last iteration's sigma_h
  const bool adapt = H > 0 && h->strata_beta > 0.0;
  const int64_t n_events = H > 0 && !adapt ? H * npc : n_req;
  if (adapt) {
    if (h->s_capH < H) {  // scratch for the allocation (first use, or more hypercubes)
      VG_HIP(hipStreamSynchronize(h->stream));
      if (h->s_sig) VG_HIP(hipFree(h->s_sig));
      if (h->s_p) VG_HIP(hipFree(h->s_p));
      if (h->s_cnt) VG_HIP(hipFree(h->s_cnt));
      if (h->s_off) VG_HIP(hipFree(h->s_off));
      h->s_sig = h->s_p = nullptr;
      h->s_cnt = h->s_off = nullptr;
      h->s_capH = 0;
      VG_HIP(hipMalloc(&h->s_sig, sizeof(double) * H));
      VG_HIP(hipMalloc(&h->s_p, sizeof(double) * H));
      VG_HIP(hipMalloc(&h->s_cnt, sizeof(int32_t) * H));
      VG_HIP(hipMalloc(&h->s_off, sizeof(int32_t) * H));
      h->s_capH = H;
      h->s_have_sig = false;
    }
    if (!h->s_cube) VG_HIP(hipMalloc(&h->s_cube, sizeof(int32_t) * h->maxN));
    if (!h->s_part) VG_HIP(hipMalloc(&h->s_part, sizeof(double) * kAllocBlocksMax));
    if (!h->s_partf) VG_HIP(hipMalloc(&h->s_partf, sizeof(long long) * kAllocBlocksMax));
    // G blocks of C hypercubes each (from H alone: the sums' order is fixed)
    const int G = static_cast<int>(std::min<int64_t>((H + 1023) / 1024, kAllocBlocksMax));
    const int64_t C = (H + G - 1) / G;
    const int64_t freev = n_events - 2 * H;
    hipLaunchKernelGGL(k_strata_alloc_p, dim3(G), dim3(kAllocThreads), 0, h->stream, h->s_sig, h->s_p, h->s_part, H,
                       C, h->strata_beta, h->s_have_sig ? 1 : 0);
    hipLaunchKernelGGL(k_strata_alloc_f, dim3(G), dim3(kAllocThreads), 0, h->stream, h->s_p, h->s_cnt, h->s_part,
                       h->s_partf, H, C, G, freev);
    hipLaunchKernelGGL(k_strata_alloc_c, dim3(G), dim3(kAllocThreads), 0, h->stream, h->s_cnt, h->s_off, h->s_part,
                       h->s_partf, H, C, G, freev);
    VG_HIP(hipGetLastError());
    const int64_t xb = std::min<int64_t>((H + 255) / 256, 4096);
    hipLaunchKernelGGL(k_strata_expand, dim3(static_cast<unsigned>(xb)), dim3(256), 0, h->stream, h->s_cnt,
                       h->s_off, h->s_cube, H);
    VG_HIP(hipGetLastError());
  }
  const int threads = ext_y ? 256 : pick_threads(h);
  const int nslot = h->D * h->n;
  EventArgs ea;
  ea.pc = h->pc;
  ea.b = h->b;
  ea.seed = h->cfg.seed;
  ea.nev = n_events;
  ea.stride_rec = h->maxN;
  ea.iter = h->iter;
  ea.ndim = h->D;
  ea.nbins = h->n;
  ea.ext_y = ext_y;
  ea.ext_lq = ext_lq;
  ea.nobs = h->nobs;
  ea.obs_lo = h->obs_lo;
  ea.obs_hi = h->obs_hi;
  ea.obs_scale = h->nobs ? static_cast<double>(h->nobs) / (h->obs_hi - h->obs_lo) : 0.0;
  ea.strata_m = H > 0 ? h->strata_m : 0;
  ea.strata_npc = static_cast<int>(npc);
  ea.strata_md = static_cast<double>(h->strata_m);
  ea.div_m = udiv_magic(static_cast<uint32_t>(h->strata_m > 0 ? h->strata_m : 1));
  ea.div_npc = udiv_magic(static_cast<uint32_t>(npc > 0 ? npc : 1));
  ea.s_cube = adapt ? h->s_cube : nullptr;
  ea.s_cnt = adapt ? h->s_cnt : nullptr;
  ea.s_N = static_cast<double>(n_events);
  ea.s_Hd = static_cast<double>(H);
  // fused fold (digits added by the event kernel at the previous iteration's scales)
  // whenever such scales exist and the digits fit in LDS; the choice depends on
  // the history and the configuration only, never on the launch shape
  const bool fused = h->fused_ok && h->scale_valid;
  const int ev_blocks = fused ? pick_blocks(h, n_events, threads, h->occ_event_fused, kMaxRowsAcc)
                              : pick_blocks(h, n_events, threads, h->occ_event, kMaxRowsEvent);
  if (ext_y)
    VG_HIP(launch_event_ext(h, ea, ev_blocks, fused));
  else
    VG_HIP(launch_event(h, ea, ev_blocks, threads, fused));
  int rows = ev_blocks;
  if (!fused) {
    AccArgs aa;
    aa.b = h->b;
    aa.nev = n_events;
    aa.stride_rec = h->maxN;
    aa.ndim = h->D;
    aa.nbins = h->n;
    aa.dims_per_group = h->acc_dpg;
    aa.nobs = h->nobs;
    rows = pick_blocks(h, n_events, threads, h->occ_acc, kMaxRowsAcc);
    TimedLaunch t(h, 1);
    hipExtLaunchKernelGGL(k_accum, dim3(rows, h->acc_groups), dim3(threads), h->acc_lds, h->stream, t.e0, t.e1, 0,
                          aa);
    VG_HIP(t.done());
  }
  const int ncol = hist_cols(nslot) + obs_cols(h->nobs);
  // few partial rows of a fused fold whose finalisation refines the grid (one block per
  // dimension): those blocks sum the rows they need themselves, and the column-sum
  // launch, a fixed cost of several microseconds, is skipped
  const bool spec = h->spec_ok && !ext_y;
  const int direct_rows = (fused && spec && rows <= kDirectRowsMax) ? rows : 0;
  if (!direct_rows) {
    TimedLaunch t(h, 1);
    hipExtLaunchKernelGGL(k_accsum, dim3((ncol + kColTile - 1) / kColTile, (rows + kRowTile - 1) / kRowTile),
                          dim3(256), 0, h->stream, t.e0, t.e1, 0, h->b, ncol, rows);
    VG_HIP(t.done());
  }
  const int strata_blocks = H > 0 ? static_cast<int>(std::min<int64_t>((H + 255) / 256, kStrataBlocks)) : 0;
  if (H > 0) {
    TimedLaunch t(h, 1);
    if (adapt)
      hipExtLaunchKernelGGL(k_strata_adapt, dim3(strata_blocks), dim3(256), 0, h->stream, t.e0, t.e1, 0, h->b, H,
                            h->s_cnt, h->s_off, h->s_sig, static_cast<double>(n_events));
    else
      hipExtLaunchKernelGGL(k_strata, dim3(strata_blocks), dim3(256), 0, h->stream, t.e0, t.e1, 0, h->b, H,
                            static_cast<int>(npc));
    VG_HIP(t.done());
    if (adapt) h->s_have_sig = true;
  }
  h->last_launch[0] = ev_blocks;
  h->last_launch[1] = threads;
  h->last_launch[2] = rows;
  h->last_launch[3] = ncol;
  {
    FinArgs fa;
    fa.b = h->b;
    fa.nev = n_events;
    fa.stride_rec = h->maxN;
    fa.ndim = h->D;
    fa.nbins = h->n;
    fa.iter = h->iter;
    fa.fused = fused ? 1 : 0;
    fa.spec = spec ? 1 : 0;
    fa.fold_lds = fused ? h->fin_lds : 0;
    fa.obs_lds = fa.fold_lds + (fa.spec ? h->refine_lds : 0);
    fa.nobs = h->nobs;
    fa.obs_first = h->obs_first;
    fa.strata_H = H;
    fa.strata_npc = static_cast<int>(npc);
    fa.strata_blocks = strata_blocks;
    fa.strata_adapt = adapt ? 1 : 0;
    fa.alpha = h->cfg.alpha;
    fa.direct_rows = direct_rows;
    const int lds = fa.obs_lds + (h->nobs ? static_cast<int>(sizeof(double) * 2 * (h->nobs + 2)) : 0);
    // with the refinement done here, one block per dimension (block 0 also forms the
    // results; a re-fold falls back to block 0 alone)
    const unsigned fblocks = fa.spec ? static_cast<unsigned>(h->D) : 1u;
    TimedLaunch t(h, 2);
    if (h->nobs)
      hipExtLaunchKernelGGL(k_finalize<true>, dim3(fblocks), dim3(fused || fa.spec ? kFinThreads : 256), lds, h->stream,
                            t.e0, t.e1, 0, fa);
    else
      hipExtLaunchKernelGGL(k_finalize<false>, dim3(fblocks), dim3(fused || fa.spec ? kFinThreads : 256), lds, h->stream,
                            t.e0, t.e1, 0, fa);
    VG_HIP(t.done());
    h->spec_ready = fa.spec != 0;
  }
  // the next iteration's slots become the current ones
  std::swap(h->b.maxw, h->b.maxw_next);
  std::swap(h->b.cnt, h->b.cnt_next);
  std::swap(h->b.fxs, h->b.fxs_next);
  h->scale_valid = true;
  const uint32_t j = h->iter;
  h->iter++;
  h->have_hist = ext_y == nullptr;  // the grid stays frozen under the learned proposal
  h->last_flow = ext_y != nullptr;
  h->any_iter = true;
  h->obs_have = h->nobs > 0;
  h->last_strata_npc = H > 0 ? (adapt ? -1 : npc) : 0;
  h->last_n = n_events;
  if (out) {
    double o[6];
    VG_HIP(hipMemcpyAsync(o, h->b.iter_out, sizeof(o), hipMemcpyDeviceToHost, h->stream));
    VG_HIP(hipStreamSynchronize(h->stream));
    out->integral = o[0];
    out->variance = o[1];
    out->n_nonzero = static_cast<int64_t>(o[2]);
    out->n_nonfinite = static_cast<int64_t>(o[3]);
    out->n_events = n_events;
    out->iteration = j;
    out->fold = static_cast<int32_t>(o[5]);
  }
  return VEGAS_OK;
}

}  // namespace

extern "C" {

int vegas_iterate(vegas_handle h, int64_t n_events, vegas_iter_result* out) {
  if (!h) return VEGAS_EINVAL;
  if (n_events < 2 || n_events > h->maxN) return VEGAS_EINVAL;
  if (h->iter >= VEGAS_MAX_ITER) return VEGAS_ESTATE;
  return run_iteration(h, n_events, nullptr, nullptr, out);
}

int vegas_iterate_flow(vegas_handle h, vegas_flow f, int64_t n_events, vegas_iter_result* out) {
  if (!h || !f) return VEGAS_EINVAL;
  if (!ext_supported(h) || n_events < 2 || n_events > h->maxN || h->strata_m > 0) return VEGAS_EINVAL;
  if (h->iter >= VEGAS_MAX_ITER) return VEGAS_ESTATE;
  const float *y = nullptr, *lq = nullptr;
  int rc = flow_sample_events(f, h->stream, h->cfg.seed, h->iter, n_events, &y, &lq);
  if (rc != VEGAS_OK) return rc;
  rc = run_iteration(h, n_events, y, lq, out);
  const int rc2 = flow_sample_finish(f, h->stream);
  return rc != VEGAS_OK ? rc : rc2;
}

int vegas_export(vegas_handle h, int64_t first, int64_t n, float* y_dev, double* w_dev) {
  if (!h || !y_dev || !w_dev || h->D != 8) return VEGAS_EINVAL;
  if (!h->any_iter || h->last_flow) return VEGAS_ESTATE;
  if (first < 0 || n < 1 || first + n > h->last_n) return VEGAS_EINVAL;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_export, dim3(blocks), dim3(256), 0, h->stream, h->b.rec_w, h->cfg.seed, h->iter - 1, first, n,
                     y_dev, w_dev);
  VG_HIP(hipGetLastError());
  return VEGAS_OK;
}

int vegas_refine(vegas_handle h) {
  if (!h) return VEGAS_EINVAL;
  if (!h->have_hist) return VEGAS_ESTATE;
  if (h->spec_ready) {
    // the finalisation already refined this grid from this histogram: swap buffers
    std::swap(h->b.edges, h->b.edges_alt);
  } else {
    TimedLaunch t(h, 3);
    hipExtLaunchKernelGGL(k_refine, dim3(h->D), dim3(kWave), sizeof(double) * 4 * (h->n + 1), h->stream, t.e0,
                          t.e1, 0, h->b, h->n, h->cfg.alpha);
    VG_HIP(t.done());
  }
  h->spec_ready = false;
  h->have_hist = false;
  return VEGAS_OK;
}

}  // extern "C"

namespace {

// the host state that iterations and refinements read and leave behind, packed
// field by field (no padding bytes) so that two states compare by their bytes
struct HostIter {
  unsigned char bytes[256];
  size_t n = 0;
  template <class T>
  void put(const T& v) {
    std::memcpy(bytes + n, &v, sizeof(T));
    n += sizeof(T);
  }
};
static_assert(sizeof(DevBufs) + 64 <= 256, "host iteration state exceeds its buffer");

HostIter host_iter(const vegas_state* h) {
  HostIter s;
  s.put(h->b);
  s.put(h->iter);
  s.put(h->last_n);
  s.put(h->last_strata_npc);
  const unsigned char f[8] = {h->have_hist, h->any_iter, h->last_flow, h->spec_ready,
                              h->obs_have,  h->scale_valid, h->s_have_sig, 0};
  s.put(f);
  // the configuration a launch sequence depends on
  s.put(h->wpb);
  s.put(h->max_blocks);
  s.put(h->nobs);
  s.put(h->obs_first);
  return s;
}

void set_host_iter(vegas_state* h, const unsigned char* p) {
  size_t n = 0;
  auto get = [&](auto& v) {
    std::memcpy(&v, p + n, sizeof(v));
    n += sizeof(v);
  };
  get(h->b);
  get(h->iter);
  get(h->last_n);
  get(h->last_strata_npc);
  unsigned char f[8];
  get(f);
  h->have_hist = f[0];
  h->any_iter = f[1];
  h->last_flow = f[2];
  h->spec_ready = f[3];
  h->obs_have = f[4];
  h->scale_valid = f[5];
  h->s_have_sig = f[6];
}

int run_schedule_eager(vegas_handle h, const int64_t* n_events, int32_t count, int32_t refine) {
  for (int32_t j = 0; j < count; ++j) {
    const int rc = run_iteration(h, n_events[j], nullptr, nullptr, nullptr);
    if (rc != VEGAS_OK) return rc;
    if (refine) {
      const int rr = vegas_refine(h);
      if (rr != VEGAS_OK) return rr;
    }
  }
  return VEGAS_OK;
}

}  // namespace

extern "C" {

int vegas_run_schedule(vegas_handle h, const int64_t* n_events, int32_t count, int32_t refine) {
  if (!h || !n_events || count < 1 || count > VEGAS_MAX_ITER) return VEGAS_EINVAL;
  for (int32_t j = 0; j < count; ++j)
    if (n_events[j] < 2 || n_events[j] > h->maxN) return VEGAS_EINVAL;
  if (static_cast<int64_t>(h->iter) + count > VEGAS_MAX_ITER) return VEGAS_ESTATE;
  // stratified runs may allocate and synchronise on the way, and timed runs bind events
  // to each launch: both run as plain calls
  if (h->strata_m > 0 || h->timing != 0) return run_schedule_eager(h, n_events, count, refine);
  const HostIter pre = host_iter(h);
  const std::vector<int64_t> ns(n_events, n_events + count);
  if (h->sched_exec && h->sched_refine == refine && h->sched_n == ns &&
      std::memcmp(h->sched_pre, pre.bytes, pre.n) == 0) {
    VG_HIP(hipGraphLaunch(h->sched_exec, h->stream));
    set_host_iter(h, h->sched_post);
    return VEGAS_OK;
  }
  if (h->sched_exec) {
    VG_HIP(hipGraphExecDestroy(h->sched_exec));
    h->sched_exec = nullptr;
  }
  // record: the same calls, captured instead of executed -- on a stream of the
  // library's own (a capture cannot begin on the null stream), which stands in for the
  // handle's stream while the calls are made; the graph then runs on the handle's stream
  if (!h->cap_stream) VG_HIP(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  const hipStream_t user_stream = h->stream;
  h->stream = h->cap_stream;
  hipError_t eb = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
  int rc = VEGAS_OK;
  hipGraph_t g = nullptr;
  hipError_t ec = hipSuccess;
  if (eb == hipSuccess) {
    rc = run_schedule_eager(h, n_events, count, refine);
    ec = hipStreamEndCapture(h->stream, &g);
  }
  h->stream = user_stream;
  if (eb != hipSuccess) {
    set_host_iter(h, pre.bytes);
    g_last_hip_error = std::string("hipStreamBeginCapture: ") + hipGetErrorString(eb);
    return VEGAS_EHIP;
  }
  if (rc != VEGAS_OK || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    set_host_iter(h, pre.bytes);
    if (rc != VEGAS_OK) return rc;
    g_last_hip_error = std::string("hipStreamEndCapture: ") + hipGetErrorString(ec);
    return VEGAS_EHIP;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    set_host_iter(h, pre.bytes);
    g_last_hip_error = std::string("hipGraphInstantiate: ") + hipGetErrorString(ei);
    return VEGAS_EHIP;
  }
  const HostIter post = host_iter(h);
  h->sched_exec = x;
  h->sched_n = ns;
  h->sched_refine = refine;
  std::memcpy(h->sched_pre, pre.bytes, pre.n);
  std::memcpy(h->sched_post, post.bytes, post.n);
  VG_HIP(hipGraphLaunch(h->sched_exec, h->stream));
  return VEGAS_OK;
}

int vegas_result_from(vegas_handle h, int32_t first, double* integral, double* error, double* chi2_dof,
                      int32_t* n_iter) {
  if (!h) return VEGAS_EINVAL;
  if (!h->any_iter || h->iter == 0) return VEGAS_ESTATE;
  if (first < 0 || static_cast<uint64_t>(first) >= h->iter) return VEGAS_EINVAL;
  hipLaunchKernelGGL(k_result, dim3(1), dim3(64), 0, h->stream, h->b, static_cast<int>(first),
                     static_cast<int>(h->iter));
  VG_HIP(hipGetLastError());
  double r[4];
  VG_HIP(hipMemcpyAsync(r, h->b.result, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  if (integral) *integral = r[0];
  if (error) *error = r[1];
  if (chi2_dof) *chi2_dof = r[2];
  if (n_iter) *n_iter = static_cast<int32_t>(r[3]);
  return VEGAS_OK;
}

int vegas_result(vegas_handle h, double* integral, double* error, double* chi2_dof, int32_t* n_iter) {
  return vegas_result_from(h, 0, integral, error, chi2_dof, n_iter);
}

int vegas_set_observable(vegas_handle h, int32_t nbins, double lo, double hi, int32_t first_iteration) {
  if (!h || nbins < 0 || nbins > VEGAS_MAX_OBS_BINS || first_iteration < 0) return VEGAS_EINVAL;
  if (nbins > 0 && !(std::isfinite(lo) && std::isfinite(hi) && lo < hi &&
                    std::isfinite(static_cast<double>(nbins) / (hi - lo))))
    return VEGAS_EINVAL;
  h->nobs = nbins;
  h->obs_lo = nbins ? lo : 0.0;
  h->obs_hi = nbins ? hi : 0.0;
  h->obs_first = first_iteration;
  h->obs_have = false;
  configure_lds(h);
  // clear the combination (a fill kernel on the handle's stream)
  hipLaunchKernelGGL(k_fill_u64, dim3(4), dim3(256), 0, h->stream,
                     reinterpret_cast<unsigned long long*>(h->b.obs_acc), static_cast<int64_t>(3 * kObsLd + 2));
  VG_HIP(hipGetLastError());
  return VEGAS_OK;
}

int vegas_set_strata(vegas_handle h, int32_t strata_per_axis) {
  if (!h || strata_per_axis < 0) return VEGAS_EINVAL;
  const int old = h->strata_m;
  h->strata_m = strata_per_axis;
  if (strata_cubes(h) < 0) {
    h->strata_m = old;
    return VEGAS_EINVAL;
  }
  h->s_have_sig = false;
  h->last_strata_npc = 0;
  configure_lds(h);  // occupancy of the stratified event kernels
  return VEGAS_OK;
}

int vegas_set_strata_beta(vegas_handle h, double beta) {
  if (!h || !(beta >= 0.0) || !std::isfinite(beta)) return VEGAS_EINVAL;
  h->strata_beta = beta;
  h->s_have_sig = false;
  return VEGAS_OK;
}

int vegas_get_strata_counts(vegas_handle h, int32_t* counts) {
  if (!h || !counts) return VEGAS_EINVAL;
  const int64_t H = strata_cubes(h);
  if (H <= 0 || h->last_strata_npc == 0) return VEGAS_ESTATE;
  if (h->last_strata_npc > 0) {  // equal counts
    for (int64_t k = 0; k < H; ++k) counts[k] = static_cast<int32_t>(h->last_strata_npc);
    return VEGAS_OK;
  }
  VG_HIP(hipMemcpyAsync(counts, h->s_cnt, sizeof(int32_t) * H, hipMemcpyDeviceToHost, h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  return VEGAS_OK;
}

int vegas_get_observable(vegas_handle h, double* last, double* last_err, double* comb, double* comb_err) {
  if (!h) return VEGAS_EINVAL;
  if (!h->nobs || !h->obs_have) return VEGAS_ESTATE;
  const int k = h->nobs + 2;
  std::vector<double> buf(4 * static_cast<size_t>(kObsLd));
  VG_HIP(hipMemcpyAsync(buf.data(), h->b.obs_out, sizeof(double) * buf.size(), hipMemcpyDeviceToHost, h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  double* outs[4] = {last, last_err, comb, comb_err};
  for (int q = 0; q < 4; ++q)
    if (outs[q]) std::memcpy(outs[q], buf.data() + q * kObsLd, sizeof(double) * k);
  return VEGAS_OK;
}

int vegas_get_grid(vegas_handle h, double* edges) {
  if (!h || !edges) return VEGAS_EINVAL;
  VG_HIP(hipMemcpyAsync(edges, h->b.edges, sizeof(double) * h->D * (h->n + 1), hipMemcpyDeviceToHost,
                        h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  return VEGAS_OK;
}

int vegas_set_grid(vegas_handle h, const double* edges) {
  if (!h || !edges) return VEGAS_EINVAL;
  const int n = h->n;
  for (int d = 0; d < h->D; ++d) {
    const double* e = edges + d * (n + 1);
    if (e[0] != 0.0 || e[n] != 1.0) return VEGAS_EINVAL;
    for (int k = 0; k < n; ++k)
      if (!(e[k + 1] >= e[k])) return VEGAS_EINVAL;
  }
  VG_HIP(hipMemcpyAsync(h->b.edges, edges, sizeof(double) * h->D * (n + 1), hipMemcpyHostToDevice,
                        h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  h->spec_ready = false;  // a refinement must start from the new grid
  return VEGAS_OK;
}

int vegas_get_hist(vegas_handle h, double* d, double* sums) {
  if (!h) return VEGAS_EINVAL;
  if (!h->any_iter) return VEGAS_ESTATE;
  const int ns = h->D * h->n;
  std::vector<double> buf(ns + 2);
  VG_HIP(hipMemcpyAsync(buf.data(), h->b.hist, sizeof(double) * (ns + 2), hipMemcpyDeviceToHost, h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  if (d) std::memcpy(d, buf.data(), sizeof(double) * ns);
  if (sums) {
    sums[0] = buf[ns];
    sums[1] = buf[ns + 1];
  }
  return VEGAS_OK;
}

int vegas_get_weights(vegas_handle h, int64_t first, int64_t n, double* w, uint8_t* bins) {
  if (!h || !w || first < 0 || n < 0) return VEGAS_EINVAL;
  if (!h->any_iter) return VEGAS_ESTATE;
  if (first + n > h->last_n) return VEGAS_EINVAL;
  if (n == 0) return VEGAS_OK;
  VG_HIP(hipMemcpyAsync(w, h->b.rec_w + first, sizeof(double) * n, hipMemcpyDeviceToHost, h->stream));
  std::vector<uint32_t> words;
  const int nw = (h->D + 3) / 4;
  if (bins) {
    words.resize(static_cast<size_t>(nw) * n);
    for (int g = 0; g < nw; ++g)
      VG_HIP(hipMemcpyAsync(words.data() + g * n, h->b.rec_bins + g * h->maxN + first, sizeof(uint32_t) * n,
                            hipMemcpyDeviceToHost, h->stream));
  }
  VG_HIP(hipStreamSynchronize(h->stream));
  if (bins)
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < h->D; ++d) bins[i * h->D + d] = static_cast<uint8_t>(words[(d / 4) * n + i] >> (8 * (d % 4)));
  return VEGAS_OK;
}

namespace {
// doubles of adjoint scratch a call needs: the per-tile partials ([ceil(n/64)][6][B]) and
// the first level of the fixed tree over them
size_t grad_scratch_doubles(int32_t B, int64_t n_events) {
  const int64_t ntiles = (n_events + 63) / 64;
  const int64_t lvl1 = (ntiles + kTreeRows - 1) / kTreeRows;
  return static_cast<size_t>((ntiles + lvl1) * kGradVals * B);
}

int grad_check(vegas_handle h, const double* params_dev, int32_t B, int64_t n_events, double* sigma_dev,
               double* dsigma_dev) {
  if (!h || !params_dev || !sigma_dev || !dsigma_dev) return VEGAS_EINVAL;
  if (h->cfg.process != VEGAS_DY_Z) return VEGAS_EINVAL;
  if (B < 1 || B > kGradMaxPoints || n_events < 1 || n_events >= (int64_t(1) << 31)) return VEGAS_EINVAL;
  return VEGAS_OK;
}

// the adjoint's launches with the scratch at buf (>= grad_scratch_doubles(B, n) doubles)
int grad_launch(vegas_handle h, const double* params_dev, int32_t B, int64_t n_events, uint32_t iteration,
                double* sigma_dev, double* dsigma_dev, double* buf) {
  const int64_t ntiles = (n_events + 63) / 64;
  const int cols = kGradVals * B;
  double* tiles = buf;
  double* lvl = buf + ntiles * cols;
  GradArgs ga;
  ga.pc = h->pc;
  ga.edges = h->b.edges;
  ga.theta = params_dev;
  ga.tiles = tiles;
  ga.seed = h->cfg.seed;
  ga.nev = n_events;
  ga.ntiles = ntiles;
  ga.iter = iteration;
  ga.nbins = h->n;
  ga.B = B;
  {
    const double e2 = 4.0 * kPi * h->params[VEGAS_P_ALPHA];
    ga.e4_12 = e2 * e2 / 12.0;
  }
  const int lds = static_cast<int>(sizeof(double) * (3 * (h->n + 1) + 4 * 64 * 5));
  const int64_t groups = (ntiles + 3) / 4;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(&k_dy_grad), 256, lds) !=
          hipSuccess || occ < 1)
    occ = 1;
  int64_t blocks = static_cast<int64_t>(h->ncu) * occ;
  if (blocks > groups) blocks = groups;
  {
    TimedLaunch t(h, 0);  // timed as the events stage
    hipExtLaunchKernelGGL(k_dy_grad, dim3(static_cast<unsigned>(blocks)), dim3(256), lds, h->stream, t.e0, t.e1, 0,
                          ga);
    VG_HIP(t.done());
  }
  // fixed tree over tiles: 256-row chunks, level by level, ping-pong between the buffers
  const double* in = tiles;
  double* out = lvl;
  int64_t rows = ntiles;
  while (rows > 1) {
    const int64_t rout = (rows + kTreeRows - 1) / kTreeRows;
    const int tiles_c = (cols + kTreeCols - 1) / kTreeCols, gy = tiles_c < 64 ? tiles_c : 64;
    TimedLaunch t(h, 1);  // timed as the fold stage
    hipExtLaunchKernelGGL(k_tree_level, dim3(static_cast<unsigned>(rout), gy), dim3(kTreeRows), 0, h->stream, t.e0,
                          t.e1, 0, in, out, rows, cols);
    VG_HIP(t.done());
    rows = rout;
    in = out;
    out = (out == lvl) ? tiles : lvl;
  }
  {
    TimedLaunch t(h, 2);  // timed as the finalisation stage
    hipExtLaunchKernelGGL(k_grad_out, dim3(1), dim3(64), 0, h->stream, t.e0, t.e1, 0, in, B, n_events, sigma_dev,
                          dsigma_dev);
    VG_HIP(t.done());
  }
  return VEGAS_OK;
}
}  // namespace

int vegas_grad(vegas_handle h, const double* params_dev, int32_t B, int64_t n_events, uint32_t iteration,
               double* sigma_dev, double* dsigma_dev) {
  const int v = grad_check(h, params_dev, B, n_events, sigma_dev, dsigma_dev);
  if (v != VEGAS_OK) return v;
  const size_t need = grad_scratch_doubles(B, n_events);
  if (h->gbuf_doubles < need) {
    VG_HIP(hipStreamSynchronize(h->stream));
    if (h->gbuf) VG_HIP(hipFree(h->gbuf));
    h->gbuf = nullptr;
    h->gbuf_doubles = 0;
    if (hipMalloc(&h->gbuf, need * sizeof(double)) != hipSuccess) {
      h->gbuf = nullptr;
      return VEGAS_ENOMEM;
    }
    h->gbuf_doubles = need;
  }
  return grad_launch(h, params_dev, B, n_events, iteration, sigma_dev, dsigma_dev, h->gbuf);
}

int vegas_grad_noalloc(vegas_handle h, const double* params_dev, int32_t B, int64_t n_events, uint32_t iteration,
                       double* sigma_dev, double* dsigma_dev) {
  const int v = grad_check(h, params_dev, B, n_events, sigma_dev, dsigma_dev);
  if (v != VEGAS_OK) return v;
  if (grad_scratch_doubles(B, n_events) > VEGAS_SCRATCH_DOUBLES) return VEGAS_ETOOBIG;
  if (!h->scratch) {
    g_last_hip_error = h->scratch_error;
    return VEGAS_EHIP;
  }
  return grad_launch(h, params_dev, B, n_events, iteration, sigma_dev, dsigma_dev, h->scratch);
}

// checkpoint layout: header {magic, process, ndim, nbins, iter, seed} then edges, history
namespace {
struct CkptHeader {
  uint64_t magic;
  int32_t process, ndim, nbins;
  uint32_t iter;
  uint64_t seed;
  int32_t fxs[4];  // fused-fold scales for the next iteration (valid, E1, E2, unused)
};
constexpr uint64_t kMagic = 0x5645474153434b32ull;  // "VEGASCK2"
}  // namespace

int vegas_get_state(vegas_handle h, void* buf, size_t* bytes) {
  if (!h || !bytes) return VEGAS_EINVAL;
  const size_t ne = static_cast<size_t>(h->D) * (h->n + 1), nh = 2 * static_cast<size_t>(h->iter);
  const size_t need = sizeof(CkptHeader) + sizeof(double) * (ne + nh);
  if (!buf) {
    *bytes = need;
    return VEGAS_OK;
  }
  if (*bytes < need) return VEGAS_EINVAL;
  CkptHeader hd{kMagic, h->cfg.process, h->D, h->n, h->iter, h->cfg.seed, {0, 0, 0, 0}};
  char* p = static_cast<char*>(buf);
  double* e = reinterpret_cast<double*>(p + sizeof(hd));
  VG_HIP(hipMemcpyAsync(hd.fxs, h->b.fxs, sizeof(hd.fxs), hipMemcpyDeviceToHost, h->stream));
  VG_HIP(hipMemcpyAsync(e, h->b.edges, sizeof(double) * ne, hipMemcpyDeviceToHost, h->stream));
  if (nh) VG_HIP(hipMemcpyAsync(e + ne, h->b.history, sizeof(double) * nh, hipMemcpyDeviceToHost, h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  std::memcpy(p, &hd, sizeof(hd));
  *bytes = need;
  return VEGAS_OK;
}

int vegas_set_state(vegas_handle h, const void* buf, size_t bytes) {
  if (!h || !buf || bytes < sizeof(CkptHeader)) return VEGAS_EINVAL;
  CkptHeader hd;
  std::memcpy(&hd, buf, sizeof(hd));
  if (hd.magic != kMagic || hd.process != h->cfg.process || hd.ndim != h->D || hd.nbins != h->n ||
      hd.seed != h->cfg.seed || hd.iter > VEGAS_MAX_ITER)
    return VEGAS_EINVAL;
  const size_t ne = static_cast<size_t>(h->D) * (h->n + 1), nh = 2 * static_cast<size_t>(hd.iter);
  if (bytes != sizeof(CkptHeader) + sizeof(double) * (ne + nh)) return VEGAS_EINVAL;
  const double* e = reinterpret_cast<const double*>(static_cast<const char*>(buf) + sizeof(hd));
  if (hd.fxs[0] != 0 && hd.fxs[0] != 1) return VEGAS_EINVAL;
  // the scale of w^2 is always twice that of w (a stored pair that disagrees is refused)
  if (hd.fxs[0] == 1 && hd.fxs[2] != 2 * hd.fxs[1]) return VEGAS_EINVAL;
  VG_HIP(hipMemcpyAsync(h->b.edges, e, sizeof(double) * ne, hipMemcpyHostToDevice, h->stream));
  if (nh) VG_HIP(hipMemcpyAsync(h->b.history, e + ne, sizeof(double) * nh, hipMemcpyHostToDevice, h->stream));
  VG_HIP(hipMemcpyAsync(h->b.fxs, hd.fxs, sizeof(hd.fxs), hipMemcpyHostToDevice, h->stream));
  VG_HIP(hipStreamSynchronize(h->stream));
  h->scale_valid = hd.fxs[0] == 1;
  h->spec_ready = false;
  // the observable histogram keeps its binning; its combination starts afresh
  if (h->nobs) {
    hipLaunchKernelGGL(k_fill_u64, dim3(4), dim3(256), 0, h->stream,
                       reinterpret_cast<unsigned long long*>(h->b.obs_acc), static_cast<int64_t>(3 * kObsLd + 2));
    VG_HIP(hipGetLastError());
  }
  h->obs_have = false;
  h->s_have_sig = false;  // the adaptive allocation restarts from equal counts
  h->last_strata_npc = 0;
  h->iter = hd.iter;
  h->any_iter = hd.iter > 0;
  h->have_hist = false;
  h->last_n = 0;
  return VEGAS_OK;
}

}  // extern "C"
