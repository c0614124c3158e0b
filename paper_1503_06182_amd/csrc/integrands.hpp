// integrands.hpp -- per-event integrands f(x) on [0,1]^D for the gfx950 kernels.
//
// The paper evaluates a phase-space point and a matrix element times parton
// densities per event (Sec. 2.1); it prints neither.  The readings implemented
// here: Breit-Wigner mapping of resonant masses, the (tau, ln x1) mapping of the
// parton fractions, massless two-body decays with Lorentz boosts, chiral
// couplings, parametric PDFs A x^a (1-x)^b, and 3n-4 phase-space dimensions
// for n final-state particles (Sec. 3.2).  Every configuration-wide constant
// (couplings, mapping ranges) is computed once on the host into PhysConst and
// reaches the kernel as a by-value argument (constant/scalar memory).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace vg {

constexpr double kPi = 3.14159265358979323846;

struct PhysConst {
  int process, ndim, nbins, family;
  double conv;                // (hbar c)^2 in pb GeV^2
  // Breit-Wigner mapping of the first resonance: m^2 = M2 + MG tan(rho_lo + x rho_rng)
  double M2, MG, invMG, rho_lo, rho_rng, m2lo, tlo;
  // uniform products formed once on the host (the same roundings as in the kernels'
  // expressions), so that no per-thread copy of them takes vector registers: MG^2,
  // MG (1 + tlo^2), (MZ GZ)^2
  double MG2, MGt, mzgz2;
  double invS;                // 1 / S (hadronic)
  double pdfA, pdfa, pdfb;
  int pdf_pow;                // 1: a = a2/2 with integer a2 in [-8, 8] and integer b in [0, 16]
  int pdf_a2, pdf_b;
  // Drell-Yan: Q_q Q_l and chiral Z couplings g[q][h] * g_l[h'] products
  double qql[2];              // Q_q * Q_l for q = u, d
  double gg[2][4];            // g_q,h g_l,h' for (h,h') = LL, LR, RL, RR
  double e4_12;               // e^4 / 12
  double mzgz, mz2;
  // W+
  double g4v2_24;             // g^4 |V|^2 / 24
  double ptmin2, th2;         // pT^2 cut, tanh(eta_max)^2
  // WW
  double rs, shat, gs;        // sqrt(shat), shat, g / sqrt(2)
  double cs_re[2][2], cs_im[2][2];  // s-channel photon+Z coefficient, [q][h]
  double ct;                  // exchange-diagram coefficient: -g^2 / 2
  double csR2;                // |Cs[u][R]|^2 + |Cs[d][R]|^2
  // hadronic WW: ln tau = Lhi + x8 * Lrng on [ln tau_lo, ln tau_hi] (Lrng = Llo - Lhi),
  // shat = tau S; per event the s-channel coefficients e^2 Q / shat + e^2 f (shat - MZ^2
  // - i MZ GZ) / |shat - MZ^2 + i MZ GZ|^2 from csq[q] = e^2 Q and csf[q][h] = e^2 f
  double S, Lhi, Lrng, Ldiff; // Ldiff = Lhi - Llo
  double csq[2], csf[2][2];
  // e+e- -> mu+mu-
  double s_ee, e4;
  // Gaussian test integrand
  double mu, inv2s2, gnorm;   // exp(-(x-mu)^2 inv2s2) * gnorm per dimension
  // Genz families
  double ga[16], gw[16];
};

// a polynomial coefficient materialised in a scalar register pair where it is used: an
// FMA then takes it as its SGPR operand, instead of a copy of a loop-invariant vector
// register into the accumulating FMA's destination before each step
__device__ __forceinline__ double poly_coef(double c) {
  VG_OPAQUE_SGPR(c);
  return c;
}

// ---------------------------------------------------------------------------
// atan(v) by the method of Moshier's Cephes library (atan.c): fold |v| to
// |x| <= 0.66 with atan(|v|) = pi/2 + atan(-1/|v|) above tan(3 pi/8) and
// pi/4 + atan((|v| - 1)/(|v| + 1)) above 0.66, then atan(x) = x + x z P(z)/Q(z),
// z = x^2, with its degree-4 / 5 rational fit; the low part of pi/2 (resp. half of
// it) is added last.  Branch-free here: the fold is one division (n / d with d = 1 on
// the low range), and P/Q the second; the coefficients are scalar-register operands.
// Relative error about 2 units in the last place (checked on the CPU against atanl).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double atan_rr(double v) {
  VG_PRICED(atan, v);
  constexpr double kT3p8 = 2.41421356237309504880, kPio2 = 1.57079632679489661923,
                   kPio4 = 0.78539816339744830962, kMoreBits = 6.123233995736765886130e-17;
  const double a = fabs(v);
  const bool hi = a > kT3p8, mid = !hi && a > 0.66;
  const double x = div_nr(hi ? -1.0 : (mid ? a - 1.0 : a), hi ? a : (mid ? a + 1.0 : 1.0));
  const double z = x * x;
  double p = poly_coef(-8.750608600031904122785e-1);
  p = __fma_rn(p, z, poly_coef(-1.615753718733365076637e1));
  p = __fma_rn(p, z, poly_coef(-7.500855792314704667340e1));
  p = __fma_rn(p, z, poly_coef(-1.228866684490136173410e2));
  p = __fma_rn(p, z, poly_coef(-6.485021904942025371773e1));
  double q = z + poly_coef(2.485846490142306297962e1);
  q = __fma_rn(q, z, poly_coef(1.650270098316988542046e2));
  q = __fma_rn(q, z, poly_coef(4.328810604912902668951e2));
  q = __fma_rn(q, z, poly_coef(4.853903996359136964868e2));
  q = __fma_rn(q, z, poly_coef(1.945506571482613964425e2));
  const double r = __fma_rn(x, z * div_nr(p, q), x);
  const double y = hi ? kPio2 + (r + kMoreBits) : (mid ? kPio4 + (r + 0.5 * kMoreBits) : r);
  return copysign(y, v);
}

// ---------------------------------------------------------------------------
// tan(x) for |x| < pi/2 (the Breit-Wigner map's arguments): |x| > pi/4 is folded to
// y = pi/2 - |x| (pi/2 as the sum of two binary64 numbers; the first difference is
// exact, both being within a factor 2), and tan y = y + y z P(z)/Q(z), z = y^2, with the
// degree-2 / 4 rational fit of Moshier's Cephes library (tan.c) on |y| <= pi/4, taken
// here as N/Q with N = y (Q + z P): one division gives tan y = N/Q or cot y = Q/N.  A
// few units in the last place (checked on the CPU against tanl).
// ---------------------------------------------------------------------------
// sin y and cos y for |y| <= pi/4 by the minimax polynomials of the fdlibm / FreeBSD msun
// kernels (k_sin.c, k_cos.c; Sun Microsystems): sin y = y + y^3 (S1 + z R(z)), z = y^2,
// and cos y = 1 - z/2 + z^2 C(z), the leading 1 - z/2 carried with its rounding error.
// About one unit in the last place (checked on the CPU against sinl and cosl).
__device__ __forceinline__ void sincos_pio4(double y, double& sn, double& cs) {
  const double z = y * y, w = z * z;
  const double rs = __fma_rn(z, __fma_rn(z, poly_coef(2.75573137070700676789e-06), poly_coef(-1.98412698298579493134e-04)),
                             poly_coef(8.33333333332248946124e-03)) +
                    z * w * __fma_rn(z, poly_coef(1.58969099521155010221e-10), poly_coef(-2.50507602534068634195e-08));
  sn = __fma_rn(z * y, __fma_rn(z, rs, poly_coef(-1.66666666666666324348e-01)), y);
  const double rc = z * __fma_rn(z, __fma_rn(z, poly_coef(2.48015872894767294178e-05), poly_coef(-1.38888888888741095749e-03)),
                                 poly_coef(4.16666666666666019037e-02)) +
                    w * w * __fma_rn(z, __fma_rn(z, poly_coef(-1.13596475577881948265e-11), poly_coef(2.08757232129817482790e-09)),
                                     poly_coef(-2.75573143513906633035e-07));
  const double hz = 0.5 * z, v = 1.0 - hz;
  cs = v + (((1.0 - v) - hz) + z * rc);
}

// tan y = nm / q on |y| <= pi/4 (the rational fit above)
__device__ __forceinline__ void tan_nq(double y, double& nm, double& q) {
  const double z = y * y;
  double p = poly_coef(-1.30936939181383777646e4);
  p = __fma_rn(p, z, poly_coef(1.15351664838587416140e6));
  p = __fma_rn(p, z, poly_coef(-1.79565251976484877988e7));
  q = z + poly_coef(1.36812963470692954678e4);
  q = __fma_rn(q, z, poly_coef(-1.32089234440210967447e6));
  q = __fma_rn(q, z, poly_coef(2.50083801823357915839e7));
  q = __fma_rn(q, z, poly_coef(-5.38695755929454629881e7));
  nm = y * __fma_rn(z, p, q);
}

__device__ __forceinline__ double tan_halfpi(double x) {
  VG_PRICED(tan, x);
  constexpr double kPio4 = 0.78539816339744830962, kPio2Hi = 1.5707963267948966,
                   kPio2Lo = 6.123233995736766e-17;
  const double a = fabs(x);
  const bool big = a > kPio4;
  const double y = big ? (kPio2Hi - a) + kPio2Lo : a;
  double nm, q;
  tan_nq(y, nm, q);
  const double t = big ? div_nr(q, nm) : div_nr(nm, q);
  return copysign(t, x);
}

// ---------------------------------------------------------------------------
// mappings (rounding kept as in their plain definitions: no contraction)
// ---------------------------------------------------------------------------
// m^2 = M^2 + M G tan(rho_lo + r rrng) on the process's window (lower edge m2lo,
// rho_lo = atan(tlo)); jac = dm^2/dr = rrng ((m^2 - M^2)^2 + (M G)^2) / (M G)
__device__ __forceinline__ double bw_mass(const PhysConst& c, double r, double rrng) {
#pragma clang fp contract(off)
  const double rho = c.rho_lo + r * rrng;
  // below the pole the mass is measured from the window's lower edge (tangent
  // addition theorem), free of the cancellation in M^2 + M G tan(rho) as m^2 -> m2lo;
  // one tangent per event either way (no divergent second call)
  const bool below = rho < 0.0;
  const double t = tan_halfpi(below ? r * rrng : rho);
  return below ? c.m2lo + c.MGt * t * rcp_nr(1.0 - c.tlo * t) : c.M2 + c.MG * t;
}

__device__ __forceinline__ double bw_map(const PhysConst& c, double r, double rrng, double& jac) {
#pragma clang fp contract(off)
  const double m2 = bw_mass(c, r, rrng);
  const double dm = m2 - c.M2;
  jac = rrng * (dm * dm + c.MG2) * c.invMG;
  return m2;
}

// ---------------------------------------------------------------------------
// product of the two parton densities, f(x1) f(x2) = A^2 tau^a ((1-x1)(1-x2))^b with
// tau = x1 x2, L = ln tau and P = (1-x1)(1-x2) (> 0).  For half-integer a and integer
// b (the usual parametrisations) the powers are products, square roots and one
// reciprocal; otherwise exp(a L + b ln P).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ipow_pos(double v, int k) {  // v^k, 0 <= k <= 16
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= v;
  return r;
}

__device__ __forceinline__ double pdf_pair(const PhysConst& c, double tau, double L, double P) {
  if (c.pdf_pow) {
    const int a2 = c.pdf_a2;
    const int ka = (a2 >= 0 ? a2 : -a2) >> 1;   // |a| rounded down
    double ta = ipow_pos(tau, ka);
    if (a2 & 1) ta *= sqrt_nr(tau);
    if (a2 < 0) ta = rcp_nr(ta);
    return c.pdfA * c.pdfA * ta * ipow_pos(P, c.pdf_b);
  }
  return c.pdfA * c.pdfA * exp(c.pdfa * L + c.pdfb * log(P));
}

// ---------------------------------------------------------------------------
// test integrands
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ double f_gauss(const PhysConst& c, const double* x) {
  const int nd = D > 0 ? D : c.ndim;
  double s = 0.0, norm = 1.0;
#pragma unroll
  for (int d = 0; d < (D > 0 ? D : 16); ++d) {
    if (d >= nd) break;
    const double z = x[d] - c.mu;
    s += z * z;
    norm *= c.gnorm;
  }
  return norm * exp(-s * c.inv2s2);
}

template <int D>
__device__ __forceinline__ double f_genz(const PhysConst& c, const double* x) {
  const int nd = D > 0 ? D : c.ndim;
  double s = 0.0, f = 1.0;
  switch (c.family) {
    case 1:
      for (int d = 0; d < nd; ++d) s += c.ga[d] * x[d];
      return cos(2.0 * kPi * c.gw[0] + s);
    case 2:
      for (int d = 0; d < nd; ++d) {
        const double z = x[d] - c.gw[d];
        f *= 1.0 / (1.0 / (c.ga[d] * c.ga[d]) + z * z);
      }
      return f;
    case 3:
      for (int d = 0; d < nd; ++d) s += c.ga[d] * x[d];
      return pow(1.0 + s, -static_cast<double>(nd + 1));
    case 4:
      for (int d = 0; d < nd; ++d) {
        const double z = x[d] - c.gw[d];
        s += c.ga[d] * c.ga[d] * z * z;
      }
      return exp(-s);
    case 5:
      for (int d = 0; d < nd; ++d) s += c.ga[d] * fabs(x[d] - c.gw[d]);
      return exp(-s);
    case 6:
      if (x[0] > c.gw[0]) return 0.0;
      if (nd > 1 && x[1] > c.gw[1]) return 0.0;
      for (int d = 0; d < nd; ++d) s += c.ga[d] * x[d];
      return exp(s);
    default:
      return __builtin_nan("");
  }
}

// e+e- -> mu+mu-: <|M|^2> = e^4 (1 + c^2); flux 1/(2s), dPhi_2 = dOmega/(32 pi^2),
// solid-angle Jacobian 4 pi -> f = conv e^4 (1 + c^2) / (16 pi s)
__device__ __forceinline__ double f_eemumu(const PhysConst& c, const double* x) {
  const double cs = 2.0 * x[0] - 1.0;
  return c.conv * c.e4 * (1.0 + cs * cs) / (16.0 * kPi * c.s_ee);
}

// ---------------------------------------------------------------------------
// q qbar -> photon/Z -> l- l+ (both beam orderings).  With one PDF for all
// four flavours the two orderings sum to sum_{hh'} |A_hh'|^2 * 2 (1 + c^2).
// ---------------------------------------------------------------------------
// obs_sq: the square of the observable, the lepton-pair mass m_ll^2
__device__ __forceinline__ double f_dy(const PhysConst& c, const double* x, double& obs_sq) {
  double jbw;
  const double m2 = bw_map(c, x[0], c.rho_rng, jbw);
  obs_sq = m2;
  double L, l1, l2;
  {
#pragma clang fp contract(off)
    L = log(m2 * c.invS);
    l1 = x[1] * L;
    l2 = L - l1;
  }
  const double jtau = -L * c.invS;
  // f(x1) f(x2) with tau = x1 x2 = m2 / S and 1 - x = -expm1(ln x)
  const double ff = pdf_pair(c, m2 * c.invS, L, expm1(l1) * expm1(l2));
  const double cs = 2.0 * x[2] - 1.0;
  // 1 / (shat - MZ^2 + i MZ GZ)
  const double ds = m2 - c.mz2;
  const double den = rcp_nr(ds * ds + c.mzgz2);
  const double pre = ds * den, pim = -c.mzgz * den;
  const double inv_s = rcp_nr(m2);
  double sum = 0.0;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int hh = 0; hh < 4; ++hh) {
      const double re = c.qql[q] * inv_s + c.gg[q][hh] * pre;
      const double im = c.gg[q][hh] * pim;
      sum += re * re + im * im;
    }
  const double me = c.e4_12 * m2 * m2 * sum * 2.0 * (1.0 + cs * cs);
  // conv * J_bw * J_tau * J_cos(2) * flux 1/(2 shat) * 2 pi / (32 pi^2)
  return c.conv * jbw * jtau * 2.0 * (0.5 * inv_s) * (1.0 / (16.0 * kPi)) * ff * me;
}

// ---------------------------------------------------------------------------
// u dbar -> W+ -> e+ nu (both orderings) with e+ cuts pT > ptmin, |eta| < etamax.
// Orderings sum to g^4 |V|^2 shat^2 (1 + c^2) / (24 |D|^2); the cuts use the
// boost-invariant pT^2 = (shat/4)(1 - c^2) and the lab polar cosine
// (c + beta)/(1 + beta c), beta = (x1 - x2)/(x1 + x2).
// ---------------------------------------------------------------------------
// obs_sq: the square of the observable, the e+ transverse momentum (taken before the cuts)
__device__ __forceinline__ double f_w(const PhysConst& c, const double* x, double& obs_sq) {
  double jbw;
  const double m2 = bw_map(c, x[0], c.rho_rng, jbw);
  double L, l1, l2;
  {
#pragma clang fp contract(off)
    L = log(m2 * c.invS);
    l1 = x[1] * L;
    l2 = L - l1;
  }
  const double jtau = -L * c.invS;
  const double cs = 2.0 * x[2] - 1.0;
  // x = 1 + expm1(ln x): beta = (x1 - x2)/(x1 + x2) and 1 - x from the same two values
  const double em1 = expm1(l1), em2 = expm1(l2);
  const double pt2 = 0.25 * m2 * (1.0 - cs) * (1.0 + cs);
  obs_sq = pt2;
  const double beta = div_nr(em1 - em2, 2.0 + em1 + em2);
  const double num = cs + beta, dnm = 1.0 + beta * cs;
  const bool pass = (pt2 > c.ptmin2) && (num * num < c.th2 * dnm * dnm);
  if (!pass) return 0.0;
  const double ds = m2 - c.M2;
  const double den = ds * ds + c.MG2;
  // |M|^2 / (2 shat) = g^4 |V|^2 / 24 * shat^2 (1 + cos^2) / den / (2 shat): one division
  const double me_flux = c.g4v2_24 * (0.5 * m2) * (1.0 + cs * cs) * rcp_nr(den);
  const double ff = pdf_pair(c, m2 * c.invS, L, em1 * em2);
  // conv * J_bw * J_tau * |M|^2 / (2 shat) * (2 * 2 pi)/(32 pi^2)
  return c.conv * jbw * jtau * (1.0 / (8.0 * kPi)) * ff * me_flux;
}

// ---------------------------------------------------------------------------
// q qbar -> W+ W- -> e+ nu mu- nubar: helicity amplitudes in two-component
// (Weyl) form.  Quarks along +-z; lepton helicities fixed by V-A; the quark-pair
// currents are then j_L = rs (0, 1, -i, 0) and j_R = rs (0, 1, i, 0).
// ---------------------------------------------------------------------------
template <typename R>
struct cx {
  R re, im;
};
template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <typename R>
__device__ __forceinline__ cx<R> cconjmul(cx<R> a, cx<R> b) {  // conj(a) * b
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__device__ __forceinline__ R cabs2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// helicity-minus massless 2-spinor (left-chiral), phase chosen per hemisphere: with
// r = sqrt(p0 + |p3|), (-(p1 - i p2) / r, r) for p3 >= 0 and (-r, (p1 + i p2) / r) below
// (the two differ by a phase, so |M|^2 does not depend on the choice; dividing by the
// larger of p0 +- p3 avoids the cancellation).  One square root and its reciprocal from
// the same estimate, and selects instead of branches (a wave holds both hemispheres).
template <typename R>
__device__ __forceinline__ void spinor_m(const R p[4], cx<R>& s0, cx<R>& s1) {
  const bool up = p[3] >= R(0);
  R r, ir;
  sqrt_rsqrt_nr(p[0] + fabs(p[3]), r, ir);
  const R a = p[1] * ir, b = p[2] * ir;
  s0 = {up ? -a : -r, up ? b : R(0)};
  s1 = {up ? r : a, up ? R(0) : b};
}

// J^mu = a^dagger sigma-bar^mu b (contravariant components)
template <typename R>
__device__ __forceinline__ void current(cx<R> a0, cx<R> a1, cx<R> b0, cx<R> b1, cx<R> J[4]) {
  const cx<R> t00 = cconjmul(a0, b0), t11 = cconjmul(a1, b1);
  const cx<R> t01 = cconjmul(a0, b1), t10 = cconjmul(a1, b0);
  J[0] = cadd(t00, t11);
  J[1] = {-(t01.re + t10.re), -(t01.im + t10.im)};
  const cx<R> d = csub(t01, t10);
  J[2] = {-d.im, d.re};  // i * d
  J[3] = csub(t11, t00);
}

template <typename R>
__device__ __forceinline__ cx<R> mdot(const cx<R> a[4], const cx<R> b[4]) {
  cx<R> s = cmul(a[0], b[0]);
  s = csub(s, cmul(a[1], b[1]));
  s = csub(s, cmul(a[2], b[2]));
  return csub(s, cmul(a[3], b[3]));
}

template <typename R>
__device__ __forceinline__ cx<R> mdot_r(const R a[4], const cx<R> b[4]) {
  return {a[0] * b[0].re - a[1] * b[1].re - a[2] * b[2].re - a[3] * b[3].re,
          a[0] * b[0].im - a[1] * b[1].im - a[2] * b[2].im - a[3] * b[3].im};
}

// [ (sigma-bar.e2)(sigma.k)(sigma-bar.e1) ]_{01}; sigma-bar.e = e^0 + sigma.e,
// sigma.k = k^0 - sigma.k (k real)
template <typename R>
__device__ __forceinline__ cx<R> chain01(const cx<R> e2[4], const R k[4], R B00, R B11, const cx<R> e1[4]) {
  const cx<R> A00 = cadd(e2[0], e2[3]);
  const cx<R> A01 = {e2[1].re + e2[2].im, e2[1].im - e2[2].re};  // e2^1 - i e2^2
  const cx<R> C01 = {e1[1].re + e1[2].im, e1[1].im - e1[2].re};  // e1^1 - i e1^2
  const cx<R> C11 = csub(e1[0], e1[3]);
  const cx<R> B01 = {-k[1], k[2]};   // -(k1 - i k2)
  const cx<R> B10 = {-k[1], -k[2]};  // -(k1 + i k2)
  const cx<R> y0 = cadd(cscale(C01, B00), cmul(B01, C11));
  const cx<R> y1 = cadd(cmul(B10, C01), cscale(C11, B11));
  return cadd(cmul(A00, y0), cmul(A01, y1));
}

// exchange-propagator invariants: t = k^2 and k^0 -+ k^3 for k = p1 - q(W+) (u quark)
// and k = p1 - q(W-) (d quark); given when they were formed in binary64 from the
// mapped masses (used by the binary32 amplitude), else taken from the momenta
template <typename R>
struct ExchInv {
  R tu, td, b00u, b11u, b00d, b11d;
};

// the energy of one hadronic event (the s-channel coefficients are formed from it
// where the amplitude needs them, so that only two values stay live)
struct WWHad {
  double rs, sh;
};

// the lepton current of one W decay, J = a^dagger sigma-bar b with a, b the
// helicity-minus spinors of pa, pb (formed as soon as the decay momenta are, so that
// only the current stays live)
template <typename R>
__device__ __forceinline__ void lepton_current(const double pa[4], const double pb[4], cx<R> J[4]) {
  R a[4], b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a[i] = static_cast<R>(pa[i]);
    b[i] = static_cast<R>(pb[i]);
  }
  cx<R> a0, a1, b0, b1;
  spinor_m(a, a0, a1);
  spinor_m(b, b0, b1);
  current(a0, a1, b0, b1, J);
}

// sum over q in {u, d} and quark helicity of |M|^2 (no averages) WITHOUT the two W
// propagators and couplings g/sqrt2 / (m^2 - MW^2 + i MW GW): every diagram is linear
// in each W's polarisation current, so they factor out of every amplitude as one complex
// number, and |.|^2 of it, g^4/4 / ((m+^2 - MW^2)^2 + (MW GW)^2) / ((m-^2 - MW^2)^2 +
// (MW GW)^2), cancels against the Breit-Wigner maps' Jacobians (the caller multiplies
// the remainder, (g^2/2)^2 / (MW GW)^2 times the maps' ranges, into the weight).  From the
// lepton currents Jp = ubar(nu) gamma P_L v(e+), Jm = ubar(mu-) gamma P_L v(nubar) (the
// polarisations ep, em up to those factors) and the W momenta qp, qm
template <typename R, bool HAD = false>
__device__ __forceinline__ R ww_me2(const PhysConst& c, const WWHad& hd, const cx<R> ep[4], const cx<R> em[4],
                                    const R qp[4], const R qm[4], const ExchInv<R>* inv) {
  R Ppq[4], Pmq[4], dq[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const R PP = qp[mu] + qm[mu];
    Ppq[mu] = PP + qp[mu];
    Pmq[mu] = PP + qm[mu];
    dq[mu] = qm[mu] - qp[mu];
  }
  // triple-gauge vertex contracted with ep, em
  const cx<R> a1 = mdot_r(Ppq, em), a2 = mdot(ep, em), a3 = mdot_r(Pmq, ep);
  cx<R> V1, V2;
  V1 = csub(cadd(cmul(ep[1], a1), cscale(a2, dq[1])), cmul(em[1], a3));
  V2 = csub(cadd(cmul(ep[2], a1), cscale(a2, dq[2])), cmul(em[2], a3));
  const R rs = static_cast<R>(HAD ? hd.rs : c.rs);
  // j_L.V = -rs (V1 - i V2), j_R.V = -rs (V1 + i V2)
  const cx<R> AL = {-rs * (V1.re + V2.im), -rs * (V1.im - V2.re)};
  const cx<R> AR = {-rs * (V1.re - V2.im), -rs * (V1.im + V2.re)};
  // exchange diagrams: u quark emits W+ first (k = p1 - qp), d quark emits W- first (k = p1 - qm);
  // p1 = (rs/2, 0, 0, rs/2); vbar(p2) ... u(p1) picks -rs * [..]_{01}
  const R half = rs * R(0.5);
  R ku[4] = {half - qp[0], -qp[1], -qp[2], half - qp[3]};
  R kd[4] = {half - qm[0], -qm[1], -qm[2], half - qm[3]};
  R tu, td, b00u, b11u, b00d, b11d;
  if (inv) {
    tu = inv->tu;
    td = inv->td;
    b00u = inv->b00u;
    b11u = inv->b11u;
    b00d = inv->b00d;
    b11d = inv->b11d;
  } else {
    tu = ku[0] * ku[0] - ku[1] * ku[1] - ku[2] * ku[2] - ku[3] * ku[3];
    td = kd[0] * kd[0] - kd[1] * kd[1] - kd[2] * kd[2] - kd[3] * kd[3];
    b00u = ku[0] - ku[3];
    b11u = ku[0] + ku[3];
    b00d = kd[0] - kd[3];
    b11d = kd[0] + kd[3];
  }
  const cx<R> Tu = chain01(em, ku, b00u, b11u, ep);
  const cx<R> Td = chain01(ep, kd, b00d, b11d, em);
  const R ct = static_cast<R>(c.ct);
  const R rsct = -rs * ct;
  const R fu = rsct * rcp_nr(tu), fd = rsct * rcp_nr(td);
  double cre[2], cim[2], csR2 = c.csR2;  // s-channel photon + Z, left-handed quark, [q]
  if constexpr (HAD) {
    // e^2 Q / shat + e^2 f (shat - MZ^2 - i MZ GZ) / |shat - MZ^2 + i MZ GZ|^2
    const double dr = hd.sh - c.mz2, idd = rcp_nr(dr * dr + c.mzgz2), ish = rcp_nr(hd.sh);
    csR2 = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      cre[q] = c.csq[q] * ish + c.csf[q][0] * dr * idd;
      cim[q] = -c.csf[q][0] * c.mzgz * idd;
      const double rr = c.csq[q] * ish + c.csf[q][1] * dr * idd, ri = -c.csf[q][1] * c.mzgz * idd;
      csR2 += rr * rr + ri * ri;
    }
  } else {
    cre[0] = c.cs_re[0][0];
    cim[0] = c.cs_im[0][0];
    cre[1] = c.cs_re[1][0];
    cim[1] = c.cs_im[1][0];
  }
  const cx<R> csuL = {static_cast<R>(cre[0]), static_cast<R>(cim[0])};
  const cx<R> csdL = {static_cast<R>(cre[1]), static_cast<R>(cim[1])};
  const cx<R> MuL = cadd(cmul(csuL, AL), cscale(Tu, fu));
  const cx<R> MdL = cadd(cmul(csdL, AL), cscale(Td, fd));
  return cabs2(MuL) + cabs2(MdL) + static_cast<R>(csR2) * cabs2(AR);
}

// rest frame of Q (mass m, im = 1 / m) -> frame of Q, for k and its back-to-back partner
template <typename R>
__device__ __forceinline__ void boost_pair(const R Q[4], R m, R im, const R k[4], R a[4], R b[4]) {
  const R qk = Q[1] * k[1] + Q[2] * k[2] + Q[3] * k[3];
  const R iqm = rcp_nr(Q[0] + m);
  const R Ea = (Q[0] * k[0] + qk) * im;
  const R Eb = (Q[0] * k[0] - qk) * im;
  const R fa = (k[0] + Ea) * iqm, fb = (k[0] + Eb) * iqm;
  a[0] = Ea;
  b[0] = Eb;
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    a[i] = k[i] + fa * Q[i];
    b[i] = -k[i] + fb * Q[i];
  }
}

// sin and cos of 2 pi x for 0 <= x <= 1: x = q/4 + r with q = rint(4 x) and |r| <= 1/8
// (r exact: x and q/4 are within a factor 2 of each other when q > 0), y = 2 pi r, then
// the rotation by q quarter turns
__device__ __forceinline__ void sincos_2pi(double x, double& s, double& c) {
  VG_PRICED(sincos, x);
  const double q = rint(4.0 * x);
  const double y = (x - 0.25 * q) * 6.283185307179586477;
  double sn, cs;
  sincos_pio4(y, sn, cs);
  const int qi = static_cast<int>(q) & 3;
  const double a = (qi & 1) ? cs : sn, b = (qi & 1) ? sn : cs;
  s = qi >= 2 ? -a : a;
  c = (qi == 1 || qi == 2) ? -b : b;
}
__device__ __forceinline__ void sincos_2pi(float x, float& s, float& c) { sincospif(2.0f * x, &s, &c); }

// WW_4L: x0 -> m+^2 (BW on [0, shat]), x1 -> m-^2 (BW on [0, (rs - m+)^2]),
// x2, x3 -> W+ direction, x4..x7 -> lepton directions in the W rest frames.
// Phase space (masses, momenta, lambda, Jacobian) is binary64; only the
// amplitude (spinors, currents, diagrams) is evaluated in R.
// obs_sq: the square of the observable, the e+ nu mass m_+^2 (0 where the map gives none)
// HAD: the hadronic integrand (10 dims): x8 -> ln tau, x9 -> ln x1, the partonic weight
// at shat = tau S times the luminosity 2 |dtau/dx8| (-ln tau) f(x1) f(x2) (the two beam
// orderings give the same integral)
template <typename R, bool HAD = false>
__device__ __forceinline__ double f_ww(const PhysConst& c, const double* x, double& obs_sq) {
  double rs = c.rs, sh = c.shat, rho_rng = c.rho_rng, lum = 1.0;
  WWHad hd;
  if constexpr (HAD) {
    double L, l1, l2;
    {
#pragma clang fp contract(off)
      L = c.Lhi + x[8] * c.Lrng;
      l1 = x[9] * L;
      l2 = L - l1;
    }
    const double tau = exp(L);
    sh = tau * c.S;
    rs = sqrt_nr(sh);
    rho_rng = atan_rr((sh - c.M2) * c.invMG) - c.rho_lo;
    lum = 2.0 * (tau * c.Ldiff) * (-L) * pdf_pair(c, tau, L, expm1(l1) * expm1(l2));
    hd.rs = rs;
    hd.sh = sh;
  }
  // the masses from the Breit-Wigner maps; their Jacobians' resonance factors cancel
  // the W propagators (see ww_me2): only the maps' ranges enter the weight
  const double mp2 = bw_mass(c, x[0], rho_rng);
  obs_sq = mp2 > 0.0 ? mp2 : 0.0;
  if (!(mp2 > 0.0)) return 0.0;
  double mp, imp;
  sqrt_rsqrt_nr(mp2, mp, imp);
  const double up = (rs - mp) * (rs - mp);
  const double rrng2 = atan_rr((up - c.M2) * c.invMG) - c.rho_lo;
  const double mm2 = bw_mass(c, x[1], rrng2);
  if (!(mm2 > 0.0)) return 0.0;
  double mm, imm;
  sqrt_rsqrt_nr(mm2, mm, imm);
  const double lam = (sh - mp2 - mm2) * (sh - mp2 - mm2) - 4.0 * mp2 * mm2;
  if (!(lam > 0.0)) return 0.0;
  const double sl = sqrt_nr(lam);
  const double i2rs = HAD ? 0.5 * rcp_nr(rs) : 1.0 / (2.0 * rs);
  const double q = sl * i2rs;
  const double Ep = (sh + mp2 - mm2) * i2rs, Em = (sh - mp2 + mm2) * i2rs;
  const double ct = 2.0 * x[2] - 1.0, st = sqrt_nr((1.0 - ct) * (1.0 + ct));
  double sf, cf;
  sincos_2pi(x[3], sf, cf);
  const double qp[4] = {Ep, q * st * cf, q * st * sf, q * ct};
  const double qm[4] = {Em, -qp[1], -qp[2], -qp[3]};
  // each W's decay leptons in the CM frame, turned into its lepton current at once
  cx<R> Jp[4], Jm[4];
  {
    const double c3 = 2.0 * x[4] - 1.0, s3 = sqrt_nr((1.0 - c3) * (1.0 + c3));
    double s, cc;
    sincos_2pi(x[5], s, cc);
    const double h = 0.5 * mp;
    const double k[4] = {h, h * s3 * cc, h * s3 * s, h * c3};
    double d3[4], d4[4];
    boost_pair<double>(qp, mp, imp, k, d3, d4);
    lepton_current<R>(d4, d3, Jp);
  }
  {
    const double c5 = 2.0 * x[6] - 1.0, s5 = sqrt_nr((1.0 - c5) * (1.0 + c5));
    double s, cc;
    sincos_2pi(x[7], s, cc);
    const double h = 0.5 * mm;
    const double k[4] = {h, h * s5 * cc, h * s5 * s, h * c5};
    double d5[4], d6[4];
    boost_pair<double>(qm, mm, imm, k, d5, d6);
    lepton_current<R>(d5, d6, Jm);
  }
  R qpr[4], qmr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    qpr[i] = static_cast<R>(qp[i]);
    qmr[i] = static_cast<R>(qm[i]);
  }
  const double two = 2.0;
  (void)two;
  double me;
  if constexpr (sizeof(R) < sizeof(double)) {
    // binary32 amplitude: the exchange invariants cancel for forward W bosons, so
    // they are formed here in binary64 without cancellation,
    // E -+ q cos = m^2 / (E + q) + q (1 -+ cos) for the W+ (and with cos -> -cos for the W-)
    const double qd = sl * i2rs, Epd = (sh + mp2 - mm2) * i2rs, Emd = (sh - mp2 + mm2) * i2rs;
    const double cd = 2.0 * x[2] - 1.0;
    const double epm = div_nr(mp2, Epd + qd) + qd * (1.0 - cd);  // Ep - q cos
    const double emm = div_nr(mm2, Emd + qd) + qd * (1.0 + cd);  // Em + q cos
    ExchInv<R> iv;
    iv.tu = static_cast<R>(mp2 - rs * epm);
    iv.td = static_cast<R>(mm2 - rs * emm);
    iv.b00u = static_cast<R>(-epm);
    iv.b11u = static_cast<R>(rs - (Epd + qd * cd));
    iv.b00d = static_cast<R>(-emm);
    iv.b11d = static_cast<R>(rs - (Emd - qd * cd));
    me = static_cast<double>(
        ww_me2<R, HAD>(c, hd, Jp, Jm, qpr, qmr, &iv));
  } else {
    me = static_cast<double>(
        ww_me2<R, HAD>(c, hd, Jp, Jm, qpr, qmr, nullptr));
  }
  // dPhi_2(P) (4 pi) = sl / (8 pi shat), dm+^2/(2 pi), dm-^2/(2 pi), [dPhi_2(W) (4 pi)]^2 =
  // 1 / (64 pi^2), flux 1 / (2 shat), colour and spin average 1/12: one constant over shat^2;
  // each Breit-Wigner Jacobian times its propagator's |g/sqrt2 / (m^2 - MW^2 + i MW GW)|^2
  // is (g^2/2) / (MW GW) times the map's range
  constexpr double kPS = 0.5 / (12.0 * 8.0 * kPi * 4.0 * kPi * kPi * 64.0 * kPi * kPi);
  const double gbw = (c.gs * c.gs) * c.invMG;
  const double ish = HAD ? rcp_nr(sh) : 1.0 / sh;
  const double w = (c.conv * kPS) * (gbw * gbw) * (ish * ish) * (sl * me) * (rho_rng * rrng2);
  if constexpr (HAD) return w * lum;
  return w;
}

}  // namespace vg
