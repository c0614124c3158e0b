/*
 * vegas_oracle.c -- CPU ORACLE for the per-event VEGAS iteration.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, by the smoke check and by the
 * CPU-baseline leg of bench.py; never by the product path.  Plain, serial,
 * FP64 with long-double accumulation; no blocking, no fusion, no reordering.
 * Independent of the HIP library: nothing here is shared with csrc/.
 *
 * Citations are to Campbell, Ellis, Giele, "A Multi-Threaded Version of MCFM"
 * (EPJC 2015): Sec. 2.1 (VEGAS iterations, serial grid optimisation, events
 * independent), Sec. 2.2 (per-event groups of random numbers; accurate sums),
 * Sec. 3.2 (3n-4 phase-space dimensions).  The paper gives no formula for any
 * step; the readings used are listed in the design notes and restated in the
 * comment of each function.
 *
 * Pins: the random-number generator (Philox4x32-10) reproduces the published
 * known-answer vectors of its authors (tests/golden/philox4x32_10_kat.txt), and
 * the uniform construction is checked against the first of them; everything
 * else is pinned by closed forms, invariants or brute-force quadrature in
 * tests/test_oracle_*.py.
 */
#include "vegas_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PI 3.14159265358979323846

/* ======================================================================
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): a 10-round keyed
 * bijection on 128-bit counters.  Each round multiplies words 0 and 2 by the
 * published constants, swaps the high/low halves across the word pairs and
 * xors in the round key; the key is bumped by the Weyl constants between rounds.
 * ====================================================================== */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Two 32-bit words (hi:lo) -> uniform in (0,1): keep the top 52 bits w and
 * return (w + 1/2) * 2^-52, which is exact in binary64 and never 0 or 1. */
static double words_to_uniform(uint32_t hi, uint32_t lo) {
  uint64_t w = (((uint64_t)hi << 32) | (uint64_t)lo) >> 12;
  return ((double)(2 * w + 1)) * 0x1p-53;
}

/* Counter (event_lo, event_hi, iteration, call k), key (seed_lo, seed_hi);
 * call k yields u[2k] from words (1:0) and u[2k+1] from words (3:2). */
void ora_uniforms(uint64_t seed, uint32_t iter, uint64_t event, int ndim, double *u) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int k = 0; 2 * k < ndim; ++k) {
    uint32_t ctr[4] = {(uint32_t)event, (uint32_t)(event >> 32), iter, (uint32_t)k};
    uint32_t out[4];
    ora_philox4x32_10(ctr, key, out);
    u[2 * k] = words_to_uniform(out[1], out[0]);
    if (2 * k + 1 < ndim) u[2 * k + 1] = words_to_uniform(out[3], out[2]);
  }
}

/* ======================================================================
 * Test integrands
 * ====================================================================== */
static double f_gauss(int ndim, const double *par, const double *x, double *obs) {
  if (obs) *obs = x[0];
  double mu = par[0], sg = par[1];
  double f = 1.0;
  for (int d = 0; d < ndim; ++d) {
    double z = (x[d] - mu) / sg;
    f *= exp(-0.5 * z * z) / (sg * sqrt(2.0 * PI));
  }
  return f;
}

/* Genz (1984) families; par = {family, a[ndim], w[ndim]} */
static double f_genz(int ndim, const double *par, const double *x, double *obs) {
  if (obs) *obs = x[0];
  int fam = (int)par[0];
  const double *a = par + 1, *w = par + 1 + ndim;
  double s = 0.0, f = 1.0;
  switch (fam) {
    case 1: /* oscillatory */
      for (int d = 0; d < ndim; ++d) s += a[d] * x[d];
      return cos(2.0 * PI * w[0] + s);
    case 2: /* product peak */
      for (int d = 0; d < ndim; ++d) f *= 1.0 / (1.0 / (a[d] * a[d]) + (x[d] - w[d]) * (x[d] - w[d]));
      return f;
    case 3: /* corner peak */
      for (int d = 0; d < ndim; ++d) s += a[d] * x[d];
      return pow(1.0 + s, -(double)(ndim + 1));
    case 4: /* gaussian */
      for (int d = 0; d < ndim; ++d) s += a[d] * a[d] * (x[d] - w[d]) * (x[d] - w[d]);
      return exp(-s);
    case 5: /* continuous */
      for (int d = 0; d < ndim; ++d) s += a[d] * fabs(x[d] - w[d]);
      return exp(-s);
    case 6: /* discontinuous */
      if (x[0] > w[0]) return 0.0;
      if (ndim > 1 && x[1] > w[1]) return 0.0;
      for (int d = 0; d < ndim; ++d) s += a[d] * x[d];
      return exp(s);
    default:
      return NAN;
  }
}

/* ======================================================================
 * Physics helpers
 * ====================================================================== */
typedef struct {
  double alpha, sw2, mz, gz, mw, gw, sqrts, A, a, b, mlo, mhi, ptmin, etamax, vud, conv;
} phys;

static phys unpack(const double *p) {
  phys q;
  q.alpha = p[ORA_P_ALPHA]; q.sw2 = p[ORA_P_SW2]; q.mz = p[ORA_P_MZ]; q.gz = p[ORA_P_GZ];
  q.mw = p[ORA_P_MW]; q.gw = p[ORA_P_GW]; q.sqrts = p[ORA_P_SQRTS];
  q.A = p[ORA_P_PDF_A]; q.a = p[ORA_P_PDF_a]; q.b = p[ORA_P_PDF_b];
  q.mlo = p[ORA_P_MLO]; q.mhi = p[ORA_P_MHI]; q.ptmin = p[ORA_P_PTMIN];
  q.etamax = p[ORA_P_ETAMAX]; q.vud = p[ORA_P_VUD]; q.conv = p[ORA_P_CONV];
  return q;
}

/* Breit-Wigner mapping of r in [0,1] onto m^2 in [m2lo, m2hi]:
 * rho uniform between rho_lo = atan(t_lo), t_lo = (m2lo-M^2)/(M G), and
 * rho_hi = atan((m2hi-M^2)/(M G)); m^2 = M^2 + M G tan(rho); jac = dm^2/dr.
 * Below the pole (rho < 0) the same m^2 is taken from the lower edge by the
 * tangent addition theorem, m^2 = m2lo + M G (1 + t_lo^2) tan(d) / (1 - t_lo tan(d)),
 * d = rho - rho_lo, which avoids the cancellation of M^2 + M G tan(rho) as m^2 -> 0. */
static void bw_map(double M, double G, double m2lo, double m2hi, double r, double *m2,
                   double *jac) {
  double MG = M * G;
  double tlo = (m2lo - M * M) / MG;
  double rlo = atan(tlo);
  double rhi = atan((m2hi - M * M) / MG);
  double rho = rlo + r * (rhi - rlo);
  if (rho < 0.0) {
    double td = tan(r * (rhi - rlo));
    *m2 = m2lo + MG * (1.0 + tlo * tlo) * td / (1.0 - tlo * td);
  } else {
    *m2 = M * M + MG * tan(rho);
  }
  double dm = *m2 - M * M;
  *jac = (rhi - rlo) * (dm * dm + MG * MG) / MG;
}

/* parametric parton density A x^a (1-x)^b, taking ln x and 1-x */
static double pdf(const phys *P, double lnx, double omx) {
  return P->A * exp(P->a * lnx) * pow(omx, P->b);
}

/* ---- Drell-Yan: q qbar -> photon/Z -> l- l+ ----
 * <|M|^2>(c) = (1/4)(1/3) sum_{h,h'} e^4 shat^2 |A_hh'|^2 (1 +- c)^2, with
 * A_hh' = Q_q Q_l / shat + g_q,h g_l,h' / (shat - M_Z^2 + i M_Z G_Z), '+' for h = h',
 * c = cosine of the angle between the quark and the l-.
 * Z couplings g_f,L = (T3 - Q sw^2)/(sw cw), g_f,R = -Q sw/cw. */
static void dy_couplings(const phys *P, int flavour, double *Qq, double gq[2], double gl[2]) {
  double sw = sqrt(P->sw2), cw = sqrt(1.0 - P->sw2);
  double T3 = flavour == 0 ? 0.5 : -0.5;
  *Qq = flavour == 0 ? 2.0 / 3.0 : -1.0 / 3.0;
  gq[0] = (T3 - *Qq * P->sw2) / (sw * cw);
  gq[1] = -*Qq * sw / cw;
  double Ql = -1.0, T3l = -0.5;
  gl[0] = (T3l - Ql * P->sw2) / (sw * cw);
  gl[1] = -Ql * sw / cw;
}

double ora_me_dy(const double *params, double shat, double c, int flavour) {
  phys P = unpack(params);
  double Qq, gq[2], gl[2];
  dy_couplings(&P, flavour, &Qq, gq, gl);
  double e2 = 4.0 * PI * P.alpha;
  double complex propz = 1.0 / (shat - P.mz * P.mz + I * P.mz * P.gz);
  double sum = 0.0;
  for (int h = 0; h < 2; ++h)
    for (int hp = 0; hp < 2; ++hp) {
      double complex A = Qq * (-1.0) / shat + gq[h] * gl[hp] * propz;
      double ang = (h == hp) ? (1.0 + c) * (1.0 + c) : (1.0 - c) * (1.0 - c);
      sum += creal(A * conj(A)) * ang;
    }
  return e2 * e2 * shat * shat * sum / 12.0;
}

/* integral over c of <|M|^2>/(32 pi shat): (pi alpha^2 shat / 9) sum |A|^2 */
double ora_sigmahat_dy(const double *params, double shat, int flavour) {
  phys P = unpack(params);
  double Qq, gq[2], gl[2];
  dy_couplings(&P, flavour, &Qq, gq, gl);
  double complex propz = 1.0 / (shat - P.mz * P.mz + I * P.mz * P.gz);
  double sum = 0.0;
  for (int h = 0; h < 2; ++h)
    for (int hp = 0; hp < 2; ++hp) {
      double complex A = Qq * (-1.0) / shat + gq[h] * gl[hp] * propz;
      sum += creal(A * conj(A));
    }
  return PI * P.alpha * P.alpha * shat * sum / 9.0;
}

/* C0 reading: x0 -> m^2 by Breit-Wigner(M_Z, G_Z) on [mlo^2, mhi^2];
 * x1 -> ln x1 = x1 * ln tau, x2 = tau / x1, Jacobian |ln tau| / S;
 * x2 -> cos(theta) of the l- along beam 1 = 2 x2 - 1.  Both beam orderings. */
static double f_dy(const double *par, const double *x, double *obs) {
  phys P = unpack(par);
  double S = P.sqrts * P.sqrts;
  double m2, jbw;
  bw_map(P.mz, P.gz, P.mlo * P.mlo, P.mhi * P.mhi, x[0], &m2, &jbw);
  if (obs) *obs = sqrt(m2); /* the lepton-pair mass */
  double tau = m2 / S;
  double L = log(tau);
  double l1 = x[1] * L, l2 = L - l1;
  double jtau = -L / S;
  double f1 = pdf(&P, l1, -expm1(l1)), f2 = pdf(&P, l2, -expm1(l2));
  double c = 2.0 * x[2] - 1.0, jc = 2.0;
  double me = 0.0;
  for (int q = 0; q < 2; ++q) me += ora_me_dy(par, m2, c, q) + ora_me_dy(par, m2, -c, q);
  double flux = 1.0 / (2.0 * m2);
  double dphi2 = 2.0 * PI / (32.0 * PI * PI); /* phi integrated, d cos(theta) left */
  return P.conv * jbw * jtau * jc * flux * dphi2 * f1 * f2 * me;
}

/* C1 reading: x0 -> m^2 by Breit-Wigner(M_W, G_W) on [mlo^2, mhi^2] (mhi <= 0 -> sqrt S);
 * x1 -> ln x1 as in f_dy; x2 -> cos(theta*) of the e+ along beam 1; x3 -> phi*.
 * <|M|^2> = g^4 |V|^2 uhat^2 / (12 |shat - M_W^2 + i M_W G_W|^2),
 * uhat = (p_u - p_e+)^2 = -shat (1 - cos(u, e+)) / 2.
 * Cuts on the e+ in the lab: pT > ptmin and |eta| < etamax. */
static double f_w(const double *par, const double *x, double *obs) {
  phys P = unpack(par);
  double S = P.sqrts * P.sqrts;
  double mhi = P.mhi > 0 ? P.mhi : P.sqrts;
  double m2, jbw;
  bw_map(P.mw, P.gw, P.mlo * P.mlo, mhi * mhi, x[0], &m2, &jbw);
  double tau = m2 / S;
  double L = log(tau);
  double l1 = x[1] * L, l2 = L - l1;
  double jtau = -L / S;
  double x1 = exp(l1), x2 = exp(l2);
  double c = 2.0 * x[2] - 1.0, phi = 2.0 * PI * x[3];
  /* e+ momentum in the partonic rest frame, then boost along z */
  double E = 0.5 * sqrt(m2);
  double s = sqrt((1.0 - c) * (1.0 + c));
  double p[4] = {E, E * s * cos(phi), E * s * sin(phi), E * c};
  double beta = (x1 - x2) / (x1 + x2);
  double gam = 1.0 / sqrt((1.0 - beta) * (1.0 + beta));
  double Elab = gam * (p[0] + beta * p[3]);
  double pzlab = gam * (p[3] + beta * p[0]);
  double pt = sqrt(p[1] * p[1] + p[2] * p[2]);
  if (obs) *obs = pt; /* the e+ transverse momentum (boost-invariant along z) */
  double eta = atanh(pzlab / Elab);
  if (!(pt > P.ptmin && fabs(eta) < P.etamax)) return 0.0;
  double g2 = 4.0 * PI * P.alpha / P.sw2;
  double den = (m2 - P.mw * P.mw) * (m2 - P.mw * P.mw) + P.mw * P.mw * P.gw * P.gw;
  double me = 0.0;
  for (int ord = 0; ord < 2; ++ord) {
    double cu = ord == 0 ? c : -c; /* u from beam 1, or from beam 2 */
    double uhat = -m2 * (1.0 - cu) / 2.0;
    me += g2 * g2 * P.vud * P.vud * uhat * uhat / (12.0 * den);
  }
  double f1 = pdf(&P, l1, -expm1(l1)), f2 = pdf(&P, l2, -expm1(l2));
  double flux = 1.0 / (2.0 * m2);
  double dphi2 = (2.0 * 2.0 * PI) / (32.0 * PI * PI);
  return P.conv * jbw * jtau * flux * dphi2 * f1 * f2 * me;
}

/* ======================================================================
 * Dirac algebra (chiral basis) for the four-fermion and WW amplitudes.
 *   gamma^0 = [[0,1],[1,0]], gamma^k = [[0, sigma^k], [-sigma^k, 0]],
 *   P_L = diag(1,1,0,0), P_R = diag(0,0,1,1).  Metric (+,-,-,-).
 * ====================================================================== */
typedef double complex cx;
typedef struct { cx m[4][4]; } mat4;

static mat4 GAM[4], PL, PR;
static int gamma_ready = 0;

static void init_gamma(void) {
  if (gamma_ready) return;
  memset(GAM, 0, sizeof(GAM));
  memset(&PL, 0, sizeof(PL));
  memset(&PR, 0, sizeof(PR));
  /* Pauli matrices */
  cx sig[4][2][2] = {{{1, 0}, {0, 1}}, {{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      GAM[0].m[i][j + 2] = sig[0][i][j];
      GAM[0].m[i + 2][j] = sig[0][i][j];
      for (int k = 1; k < 4; ++k) {
        GAM[k].m[i][j + 2] = sig[k][i][j];
        GAM[k].m[i + 2][j] = -sig[k][i][j];
      }
    }
  PL.m[0][0] = PL.m[1][1] = 1;
  PR.m[2][2] = PR.m[3][3] = 1;
  gamma_ready = 1;
}

static mat4 mmul(const mat4 *A, const mat4 *B) {
  mat4 C;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cx s = 0;
      for (int k = 0; k < 4; ++k) s += A->m[i][k] * B->m[k][j];
      C.m[i][j] = s;
    }
  return C;
}

/* a-slash = gamma^mu a_mu for a contravariant complex 4-vector a^mu */
static mat4 slash(const cx a[4]) {
  mat4 S;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      S.m[i][j] = GAM[0].m[i][j] * a[0] - GAM[1].m[i][j] * a[1] - GAM[2].m[i][j] * a[2] -
                  GAM[3].m[i][j] * a[3];
  return S;
}

static mat4 slash_real(const double a[4]) {
  cx c[4] = {a[0], a[1], a[2], a[3]};
  return slash(c);
}

/* abar M b = a^dagger gamma^0 M b */
static cx sandwich(const cx a[4], const mat4 *M, const cx b[4]) {
  mat4 G0M = mmul(&GAM[0], M);
  cx s = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) s += conj(a[i]) * G0M.m[i][j] * b[j];
  return s;
}

/* Massless helicity spinors u(p, -) (upper, left-chiral) and u(p, +) (lower,
 * right-chiral), normalised to u^dagger u = 2E.  The two forms of each differ by
 * a phase; the one that avoids dividing by a small E +- pz is used.  For a
 * massless antifermion of helicity +/- the same functions with the opposite
 * label serve as v(p, +/-). */
static void spinor_minus(const double p[4], cx u[4]) {
  double E = p[0], px = p[1], py = p[2], pz = p[3];
  if (pz >= 0) {
    double r = sqrt(E + pz);
    u[0] = -(px - I * py) / r;
    u[1] = r;
  } else {
    double r = sqrt(E - pz);
    u[0] = -r;
    u[1] = (px + I * py) / r;
  }
  u[2] = 0;
  u[3] = 0;
}

static void spinor_plus(const double p[4], cx u[4]) {
  double E = p[0], px = p[1], py = p[2], pz = p[3];
  u[0] = 0;
  u[1] = 0;
  if (pz >= 0) {
    double r = sqrt(E + pz);
    u[2] = r;
    u[3] = (px + I * py) / r;
  } else {
    double r = sqrt(E - pz);
    u[2] = (px - I * py) / r;
    u[3] = r;
  }
}

/* current J^mu = abar gamma^mu P b */
static void current(const cx a[4], const mat4 *P, const cx b[4], cx J[4]) {
  for (int mu = 0; mu < 4; ++mu) {
    mat4 GP = mmul(&GAM[mu], P);
    J[mu] = sandwich(a, &GP, b);
  }
}

static cx cdot(const cx a[4], const cx b[4]) { return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]; }
static double rdot(const double a[4], const double b[4]) {
  return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* residuals of the massless Dirac equation and of ubar gamma^mu u = 2 p^mu */
int ora_spinor_check(const double p[4], double *max_dirac_residual, double *max_current_err) {
  init_gamma();
  mat4 ps = slash_real(p);
  double rd = 0.0, rc = 0.0;
  for (int hel = 0; hel < 2; ++hel) {
    cx u[4];
    if (hel == 0) spinor_minus(p, u); else spinor_plus(p, u);
    for (int i = 0; i < 4; ++i) {
      cx s = 0;
      for (int j = 0; j < 4; ++j) s += ps.m[i][j] * u[j];
      if (cabs(s) > rd) rd = cabs(s);
    }
    mat4 one;
    memset(&one, 0, sizeof(one));
    for (int i = 0; i < 4; ++i) one.m[i][i] = 1;
    cx J[4];
    current(u, &one, u, J);
    for (int mu = 0; mu < 4; ++mu) {
      double e = cabs(J[mu] - 2.0 * p[mu]);
      if (e > rc) rc = e;
    }
  }
  *max_dirac_residual = rd;
  *max_current_err = rc;
  return 0;
}

/* e+e- -> mu+mu- through a photon, from explicit currents:
 * M = e^2 [vbar(p2) gamma^mu P_h u(p1)] [ubar(p3) gamma_mu P_h' v(p4)] / s, averaged
 * over the 4 initial helicity states.  e- along +z, mu- at (theta, phi). */
double ora_me_eemumu_dirac(const double *params, double s, double c, double phi) {
  init_gamma();
  phys P = unpack(params);
  double e2 = 4.0 * PI * P.alpha;
  double E = 0.5 * sqrt(s), sn = sqrt((1.0 - c) * (1.0 + c));
  double p1[4] = {E, 0, 0, E}, p2[4] = {E, 0, 0, -E};
  double p3[4] = {E, E * sn * cos(phi), E * sn * sin(phi), E * c};
  double p4[4] = {E, -p3[1], -p3[2], -p3[3]};
  double sum = 0.0;
  for (int h = 0; h < 2; ++h)
    for (int hp = 0; hp < 2; ++hp) {
      cx u1[4], v2[4], u3[4], v4[4], j[4], J[4];
      const mat4 *Ph = h == 0 ? &PL : &PR, *Php = hp == 0 ? &PL : &PR;
      if (h == 0) { spinor_minus(p1, u1); spinor_minus(p2, v2); }
      else { spinor_plus(p1, u1); spinor_plus(p2, v2); }
      if (hp == 0) { spinor_minus(p3, u3); spinor_minus(p4, v4); }
      else { spinor_plus(p3, u3); spinor_plus(p4, v4); }
      current(v2, Ph, u1, j);
      current(u3, Php, v4, J);
      cx M = e2 * cdot(j, J) / s;
      sum += creal(M * conj(M));
    }
  return sum / 4.0;
}

/* ---- q qbar -> W+ W- amplitude, doubly resonant (s-channel gamma and Z,
 * t-channel d exchange for q = u, u-channel u exchange for q = d).
 * ep, em: W+ and W- "polarisation" vectors (lepton currents times couplings over
 * propagators, or on-shell polarisation vectors); qp, qm: W momenta.
 * The sign between the s-channel and the exchange diagram is the one for which
 * the longitudinal amplitude stays bounded at high energy (gauge cancellation);
 * the tests check that the other sign grows. */
#define WW_SIGN_T_U (-1.0)
#define WW_SIGN_T_D (-1.0)

static cx ww_amplitude(const phys *P, double shat, const double p1[4], const double p2[4],
                       const cx ep[4], const cx em[4], const double qp[4], const double qm[4],
                       int flavour, int helicity, double sign_t) {
  init_gamma();
  double e2 = 4.0 * PI * P->alpha;
  double sw = sqrt(P->sw2), cw = sqrt(1.0 - P->sw2);
  double g2 = e2 / P->sw2;
  double Qq = flavour == 0 ? 2.0 / 3.0 : -1.0 / 3.0;
  double T3 = flavour == 0 ? 0.5 : -0.5;
  double gz = helicity == 0 ? (T3 - Qq * P->sw2) / (sw * cw) : -Qq * sw / cw;
  cx u1[4], v2[4];
  const mat4 *Proj = helicity == 0 ? &PL : &PR;
  if (helicity == 0) { spinor_minus(p1, u1); spinor_minus(p2, v2); }
  else { spinor_plus(p1, u1); spinor_plus(p2, v2); }

  /* triple gauge vertex contracted with ep, em (all-incoming cyclic form with
   * V(P) in, W+(qp) and W-(qm) out) */
  double PP[4], Ppq[4], Pmq[4], dq[4];
  for (int mu = 0; mu < 4; ++mu) {
    PP[mu] = qp[mu] + qm[mu];
    Ppq[mu] = PP[mu] + qp[mu];
    Pmq[mu] = PP[mu] + qm[mu];
    dq[mu] = qm[mu] - qp[mu];
  }
  cx Ppq_c[4], Pmq_c[4];
  for (int mu = 0; mu < 4; ++mu) { Ppq_c[mu] = Ppq[mu]; Pmq_c[mu] = Pmq[mu]; }
  cx a1 = cdot(Ppq_c, em), a2 = cdot(ep, em), a3 = cdot(Pmq_c, ep);
  cx V[4];
  for (int mu = 0; mu < 4; ++mu) V[mu] = ep[mu] * a1 + a2 * dq[mu] - em[mu] * a3;
  cx Cs = e2 * (Qq / shat + gz * (cw / sw) / (shat - P->mz * P->mz + I * P->mz * P->gz));
  mat4 Vs = slash(V);
  mat4 VsP = mmul(&Vs, Proj);
  cx amp = Cs * sandwich(v2, &VsP, u1);
  if (helicity == 0) {
    double k[4];
    const cx *first = flavour == 0 ? ep : em; /* boson emitted next to u(p1) */
    const cx *second = flavour == 0 ? em : ep;
    const double *qfirst = flavour == 0 ? qp : qm;
    for (int mu = 0; mu < 4; ++mu) k[mu] = p1[mu] - qfirst[mu];
    mat4 S2 = slash(second), Sk = slash_real(k), S1 = slash(first);
    mat4 T = mmul(&S2, &Sk);
    T = mmul(&T, &S1);
    T = mmul(&T, &PL);
    amp += sign_t * 0.5 * g2 * sandwich(v2, &T, u1) / rdot(k, k);
  }
  return amp;
}

/* Lorentz boost of k (given in the rest frame of Q, mass m) to the frame of Q */
static void boost_from_rest(const double Q[4], double m, const double k[4], double out[4]) {
  double qk = Q[1] * k[1] + Q[2] * k[2] + Q[3] * k[3];
  double E = (Q[0] * k[0] + qk) / m;
  double f = (k[0] + E) / (Q[0] + m);
  out[0] = E;
  for (int i = 1; i < 4; ++i) out[i] = k[i] + f * Q[i];
}

/* C2 reading (partonic, fixed sqrt(shat) = params[SQRTS]):
 * x0 -> m+^2 by BW(M_W, G_W) on [0, shat]; x1 -> m-^2 by BW on [0, (sqrt(shat)-m+)^2];
 * x2, x3 -> (cos, phi) of the W+ in the CM frame; x4, x5 -> e+ angles in the W+
 * rest frame; x6, x7 -> mu- angles in the W- rest frame.
 * mom = {e+, nu_e, mu-, nubar_mu, q, qbar}; jac = dPhi_4 / d^8x. */
void ora_ww_momenta(const double *params, const double *x, double mom[6][4], double *m2p,
                    double *m2m, double *jac) {
  phys P = unpack(params);
  double rs = P.sqrts, shat = rs * rs;
  double mp2, jp, mm2, jm;
  bw_map(P.mw, P.gw, 0.0, shat, x[0], &mp2, &jp);
  memset(mom, 0, sizeof(double) * 24);
  *m2p = mp2;
  *m2m = 0.0;
  *jac = 0.0;
  if (!(mp2 > 0.0)) return;
  double mp = sqrt(mp2);
  double up = (rs - mp) * (rs - mp);
  bw_map(P.mw, P.gw, 0.0, up, x[1], &mm2, &jm);
  *m2m = mm2;
  if (!(mm2 > 0.0)) return;
  double mm = sqrt(mm2);
  double lam = (shat - mp2 - mm2) * (shat - mp2 - mm2) - 4.0 * mp2 * mm2;
  if (!(lam > 0.0)) return;
  double q = sqrt(lam) / (2.0 * rs);
  double Ep = (shat + mp2 - mm2) / (2.0 * rs), Em = (shat - mp2 + mm2) / (2.0 * rs);
  double c = 2.0 * x[2] - 1.0, phi = 2.0 * PI * x[3], s = sqrt((1.0 - c) * (1.0 + c));
  double n[3] = {s * cos(phi), s * sin(phi), c};
  double qp[4] = {Ep, q * n[0], q * n[1], q * n[2]};
  double qm[4] = {Em, -q * n[0], -q * n[1], -q * n[2]};
  /* W+ -> e+ nu */
  double c3 = 2.0 * x[4] - 1.0, f3 = 2.0 * PI * x[5], s3 = sqrt((1.0 - c3) * (1.0 + c3));
  double k3[4] = {0.5 * mp, 0.5 * mp * s3 * cos(f3), 0.5 * mp * s3 * sin(f3), 0.5 * mp * c3};
  double k4[4] = {0.5 * mp, -k3[1], -k3[2], -k3[3]};
  boost_from_rest(qp, mp, k3, mom[0]);
  boost_from_rest(qp, mp, k4, mom[1]);
  /* W- -> mu- nubar */
  double c5 = 2.0 * x[6] - 1.0, f5 = 2.0 * PI * x[7], s5 = sqrt((1.0 - c5) * (1.0 + c5));
  double k5[4] = {0.5 * mm, 0.5 * mm * s5 * cos(f5), 0.5 * mm * s5 * sin(f5), 0.5 * mm * c5};
  double k6[4] = {0.5 * mm, -k5[1], -k5[2], -k5[3]};
  boost_from_rest(qm, mm, k5, mom[2]);
  boost_from_rest(qm, mm, k6, mom[3]);
  double E = 0.5 * rs;
  double p1[4] = {E, 0, 0, E}, p2[4] = {E, 0, 0, -E};
  memcpy(mom[4], p1, sizeof(p1));
  memcpy(mom[5], p2, sizeof(p2));
  /* dPhi_2(P; q+, q-) (dm+^2/2pi)(dm-^2/2pi) dPhi_2(q+) dPhi_2(q-), solid angles 4 pi each */
  double dphi_prod = sqrt(lam) / (32.0 * PI * PI * shat) * 4.0 * PI;
  double dphi_dec = 1.0 / (32.0 * PI * PI) * 4.0 * PI;
  *jac = dphi_prod * (jp / (2.0 * PI)) * (jm / (2.0 * PI)) * dphi_dec * dphi_dec;
}

/* |M|^2 of q qbar -> e+ nu mu- nubar for one quark flavour (0 = u, 1 = d) and
 * quark helicity (0 = L, 1 = R); no spin or colour average.  The W propagators
 * use the mapped virtualities m2p, m2m. */
double ora_ww_me2(const double *params, const double mom[6][4], double m2p, double m2m,
                  int flavour, int helicity) {
  init_gamma();
  phys P = unpack(params);
  double g = sqrt(4.0 * PI * P.alpha / P.sw2);
  cx u4[4], v3[4], u5[4], v6[4], Jp[4], Jm[4], ep[4], em[4];
  spinor_minus(mom[1], u4);
  spinor_minus(mom[0], v3);
  spinor_minus(mom[2], u5);
  spinor_minus(mom[3], v6);
  current(u4, &PL, v3, Jp);
  current(u5, &PL, v6, Jm);
  cx Dp = m2p - P.mw * P.mw + I * P.mw * P.gw;
  cx Dm = m2m - P.mw * P.mw + I * P.mw * P.gw;
  double qp[4], qm[4];
  for (int mu = 0; mu < 4; ++mu) {
    ep[mu] = g / sqrt(2.0) * Jp[mu] / Dp;
    em[mu] = g / sqrt(2.0) * Jm[mu] / Dm;
    qp[mu] = mom[0][mu] + mom[1][mu];
    qm[mu] = mom[2][mu] + mom[3][mu];
  }
  double shat = P.sqrts * P.sqrts;
  double sgn = flavour == 0 ? WW_SIGN_T_U : WW_SIGN_T_D;
  cx M = ww_amplitude(&P, shat, mom[4], mom[5], ep, em, qp, qm, flavour, helicity, sgn);
  return creal(M * conj(M));
}

static double f_ww(const double *par, const double *x, double *obs) {
  phys P = unpack(par);
  double mom[6][4], m2p, m2m, jac;
  ora_ww_momenta(par, x, mom, &m2p, &m2m, &jac);
  if (obs) *obs = m2p > 0.0 ? sqrt(m2p) : 0.0; /* the e+ nu mass */
  if (!(jac > 0.0)) return 0.0;
  double shat = P.sqrts * P.sqrts;
  double me = 0.0;
  for (int q = 0; q < 2; ++q)
    for (int h = 0; h < 2; ++h) me += ora_ww_me2(par, (const double(*)[4])mom, m2p, m2m, q, h);
  double avg = 1.0 / 4.0 * 1.0 / 3.0; /* spin and colour average */
  return P.conv * (1.0 / (2.0 * shat)) * avg * me * jac;
}

/* Hadronic W+W- (10 dims): the partonic integrand above at sqrt(shat) = sqrt(tau S),
 * folded with the parton luminosity.  x_8 -> ln tau uniform on [ln tau_lo, ln tau_hi]
 * (sqrt(shat) between MLO and MHI, MHI <= 0 meaning sqrt(S)), x_9 -> ln x1 = x_9 ln tau,
 * x2 = tau / x1.  sigma = sum over beams of int dx1 dx2 f(x1) f(x2) sigmahat: with one
 * density for quarks and antiquarks the quark comes from either beam with the same
 * weight, and the orderings give the same integral (they differ by a rotation of the
 * whole final state), so the weight is twice the quark-from-beam-1 term:
 *   w = 2 |d tau/d x_8| (-ln tau) f(x1) f(x2) f_ww(x_0..7; tau S). */
static double f_ww_had(const double *par, const double *x, double *obs) {
  phys P = unpack(par);
  double S = P.sqrts * P.sqrts;
  double rlo = P.mlo, rhi = P.mhi > 0 ? P.mhi : P.sqrts;
  double Llo = log(rlo * rlo / S), Lhi = log(rhi * rhi / S);
  double L = Lhi + x[8] * (Llo - Lhi);
  double tau = exp(L);
  double l1 = x[9] * L, l2 = L - l1;
  double jtau = tau * (Lhi - Llo);
  double lum = 2.0 * jtau * (-L) * pdf(&P, l1, -expm1(l1)) * pdf(&P, l2, -expm1(l2));
  double pp[ORA_NPHYS];
  memcpy(pp, par, sizeof(pp));
  pp[ORA_P_SQRTS] = sqrt(tau * S);
  return lum * f_ww(pp, x, obs);
}

/* On-shell q qbar -> W+ W- with explicit polarisation vectors, for the gauge
 * cancellation and narrow-width tests.  pol: 0 = longitudinal, 1 = +, 2 = -.
 * W+ at (theta, phi) in the CM frame; outgoing bosons take eps*. */
static void polvec(const double q[4], double M, int pol, cx eps[4]) {
  double qq = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double ct = q[3] / qq, st = sqrt(q[1] * q[1] + q[2] * q[2]) / qq;
  double cp = 1.0, sp = 0.0;
  if (st > 0) { cp = q[1] / (qq * st); sp = q[2] / (qq * st); }
  if (pol == 0) {
    eps[0] = qq / M;
    for (int i = 1; i < 4; ++i) eps[i] = q[0] * q[i] / (qq * M);
    return;
  }
  double th[3] = {ct * cp, ct * sp, -st}, ph[3] = {-sp, cp, 0.0};
  double lam = pol == 1 ? 1.0 : -1.0;
  eps[0] = 0;
  for (int i = 0; i < 3; ++i) eps[i + 1] = -lam * (th[i] + lam * I * ph[i]) / sqrt(2.0);
}

double ora_ww_onshell_me2(const double *params, double shat, double cth, double phi,
                          int flavour, int helicity, int pol_p, int pol_m, int sign_t) {
  init_gamma();
  phys P = unpack(params);
  double rs = sqrt(shat), M = P.mw;
  double q = sqrt(shat / 4.0 - M * M);
  double st = sqrt(1.0 - cth * cth);
  double n[3] = {st * cos(phi), st * sin(phi), cth};
  double qp[4] = {0.5 * rs, q * n[0], q * n[1], q * n[2]};
  double qm[4] = {0.5 * rs, -q * n[0], -q * n[1], -q * n[2]};
  double p1[4] = {0.5 * rs, 0, 0, 0.5 * rs}, p2[4] = {0.5 * rs, 0, 0, -0.5 * rs};
  cx ep[4], em[4];
  polvec(qp, M, pol_p, ep);
  polvec(qm, M, pol_m, em);
  for (int mu = 0; mu < 4; ++mu) { ep[mu] = conj(ep[mu]); em[mu] = conj(em[mu]); }
  double sgn = (double)sign_t;
  if (sign_t == 0) sgn = flavour == 0 ? WW_SIGN_T_U : WW_SIGN_T_D;
  cx A = ww_amplitude(&P, shat, p1, p2, ep, em, qp, qm, flavour, helicity, sgn);
  return creal(A * conj(A));
}

/* ======================================================================
 * Integrand dispatch
 * ====================================================================== */
int ora_ndim(int process, int ndim_requested) {
  switch (process) {
    case ORA_GAUSS:
    case ORA_GENZ: return ndim_requested;
    case ORA_EEMUMU: return 2;
    case ORA_DY_Z: return 3;
    case ORA_W_PLUS: return 4;
    case ORA_WW_4L: return 8;
    case ORA_WW_HAD: return 10;
    default: return -1;
  }
}

/* e+e- -> mu+mu-: x0 -> cos(theta) = 2 x0 - 1, x1 -> phi = 2 pi x1; <|M|^2> from
 * explicit Dirac currents; flux 1/(2s), dPhi_2 = dOmega / (32 pi^2). */
static double f_eemumu(const double *par, const double *x, double *obs) {
  phys P = unpack(par);
  double s = P.sqrts * P.sqrts;
  double c = 2.0 * x[0] - 1.0, phi = 2.0 * PI * x[1];
  if (obs) *obs = c; /* cos(theta) of the mu- */
  double me = ora_me_eemumu_dirac(par, s, c, phi);
  return P.conv * (1.0 / (2.0 * s)) * me * (4.0 * PI) / (32.0 * PI * PI);
}

/* The integrand at x; obs (nullable) receives the process's observable: x_0
 * (test integrands), cos(theta) of the mu- (e+e-), the lepton-pair mass (Drell-Yan),
 * the e+ transverse momentum (W+), the e+ nu mass (W+W-). */
static double integrand_obs(int process, int ndim, const double *params, const double *x, double *obs) {
  switch (process) {
    case ORA_GAUSS: return f_gauss(ndim, params, x, obs);
    case ORA_GENZ: return f_genz(ndim, params, x, obs);
    case ORA_EEMUMU: return f_eemumu(params, x, obs);
    case ORA_DY_Z: return f_dy(params, x, obs);
    case ORA_W_PLUS: return f_w(params, x, obs);
    case ORA_WW_4L: return f_ww(params, x, obs);
    case ORA_WW_HAD: return f_ww_had(params, x, obs);
    default: return NAN;
  }
}

double ora_integrand(int process, int ndim, const double *params, int nparams,
                     const double *x) {
  (void)nparams;
  return integrand_obs(process, ndim, params, x, NULL);
}

double ora_observable(int process, int ndim, const double *params, const double *x) {
  double o = NAN;
  integrand_obs(process, ndim, params, x, &o);
  return o;
}

/* ======================================================================
 * VEGAS state: grid, one iteration, refinement, combination
 * ====================================================================== */
struct ora_state {
  int process, ndim, nbins;
  uint64_t seed;
  double alpha;
  double params[64];
  int nparams;
  double *edges;   /* [ndim][nbins+1] */
  long double *d;  /* [ndim][nbins], last iteration */
  long double s1, s2;
  int have_hist;
  uint32_t iter;
  int n_iter, cap;
  double *Ij, *varj;
  /* observable histogram: nobs uniform bins on [lo, hi) plus under- and overflow */
  int nobs, obs_first, obs_have;
  double obs_lo, obs_hi;
  long double obs_s1[ORA_MAX_OBS + 2], obs_s2[ORA_MAX_OBS + 2];
  double obs_last[ORA_MAX_OBS + 2], obs_last_err[ORA_MAX_OBS + 2];
  long double obs_acc_w[ORA_MAX_OBS + 2], obs_acc_v[ORA_MAX_OBS + 2], obs_zacc[ORA_MAX_OBS + 2];
  long double obs_wsum;
  int obs_zcount;
  /* stratified sampling: m strata per axis (0 = off), npc events per hypercube in the
   * current (last) iteration */
  int strata_m;
  int64_t strata_npc;
  /* adaptive allocation (beta > 0): counts and offsets of the current (last)
   * iteration, the within-hypercube deviation sigma_h of the weight from the last
   * stratified iteration (have_sig), and counts injected for the next iteration */
  double strata_beta;
  int64_t *scount, *soff;
  double *ssig;
  int have_sig, have_inject;
  int64_t *sinject;
};

ora_state *ora_create(int process, int ndim, int nbins, uint64_t seed, double alpha,
                      const double *params, int nparams) {
  int D = ora_ndim(process, ndim);
  if (D < 1 || D > 16 || nbins < 2 || nbins > 255 || nparams > 64 || nparams < 0) return NULL;
  ora_state *s = (ora_state *)calloc(1, sizeof(ora_state));
  s->process = process;
  s->ndim = D;
  s->nbins = nbins;
  s->seed = seed;
  s->alpha = alpha;
  s->nparams = nparams;
  if (nparams) memcpy(s->params, params, sizeof(double) * nparams);
  s->edges = (double *)malloc(sizeof(double) * D * (nbins + 1));
  s->d = (long double *)calloc((size_t)D * nbins, sizeof(long double));
  /* uniform start: e_k = k / n */
  for (int d = 0; d < D; ++d)
    for (int k = 0; k <= nbins; ++k) s->edges[d * (nbins + 1) + k] = (double)k / nbins;
  s->cap = 64;
  s->Ij = (double *)malloc(sizeof(double) * s->cap);
  s->varj = (double *)malloc(sizeof(double) * s->cap);
  return s;
}

static void strata_free(ora_state *s);

void ora_destroy(ora_state *s) {
  if (!s) return;
  strata_free(s);
  free(s->edges);
  free(s->d);
  free(s->Ij);
  free(s->varj);
  free(s);
}

/* grid map: k = floor(u n) (clamped to n-1), delta = u n - k,
 * x = e_k + delta (e_{k+1} - e_k) (fused multiply-add), J = prod_d n (e_{k+1} - e_k) */
static void grid_map(const ora_state *s, const double *u, double *x, double *jac, int *bins) {
  int n = s->nbins;
  double J = 1.0;
  for (int d = 0; d < s->ndim; ++d) {
    double t = u[d] * (double)n;
    int k = (int)floor(t);
    if (k > n - 1) k = n - 1;
    double delta = t - (double)k;
    const double *e = s->edges + d * (n + 1);
    double h = e[k + 1] - e[k];
    x[d] = fma(delta, h, e[k]);
    J *= (double)n * h;
    bins[d] = k;
  }
  *jac = J;
}

int ora_grid_map(const ora_state *s, const double *u, double *x, double *jac, int *bins) {
  grid_map(s, u, x, jac, bins);
  return 0;
}

/* Stratified sampling (Lepage's stratified + importance mode): the unit cube is cut
 * into m^D equal hypercubes and hypercube h gets events h npc .. (h + 1) npc - 1;
 * event i lies in h = floor(i / npc), whose coordinates are the base-m digits of h
 * (dimension 0 the least significant), and its uniforms r are placed inside it:
 * u_d = (c_d + r_d) / m. */
/* hypercube of event i: floor(i / npc) with equal counts, else the one whose
 * offset range holds i (binary search over the offsets) */
static uint64_t strata_cube(const ora_state *s, uint64_t i) {
  if (s->strata_beta <= 0.0) return i / (uint64_t)s->strata_npc;
  int64_t lo = 0, hi = ora_strata_cubes(s) - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if ((uint64_t)s->soff[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return (uint64_t)lo;
}

static void strata_place(const ora_state *s, uint64_t i, double *u) {
  uint64_t h = strata_cube(s, i);
  for (int d = 0; d < s->ndim; ++d) {
    uint64_t c = h % (uint64_t)s->strata_m;
    h /= (uint64_t)s->strata_m;
    u[d] = ((double)c + u[d]) / (double)s->strata_m;
  }
}

static double event_weight_obs(const ora_state *s, uint32_t iter, uint64_t i, int *bins, double *obs) {
  double u[16], x[16], J;
  ora_uniforms(s->seed, iter, i, s->ndim, u);
  if (s->strata_m > 0 && s->strata_npc > 0) strata_place(s, i, u);
  grid_map(s, u, x, &J, bins);
  double f = integrand_obs(s->process, s->ndim, s->params, x, obs);
  if (s->strata_m > 0 && s->strata_npc > 0 && s->strata_beta > 0.0) {
    /* unequal counts: each event stands for volume 1 / (H n_h) instead of 1 / N, so
     * its weight is scaled by c_h = N / (H n_h); the estimate stays sum w / N */
    int64_t H = ora_strata_cubes(s), h = (int64_t)strata_cube(s, i);
    double N = (double)(s->soff[H - 1] + s->scount[H - 1]);
    double c = N / ((double)H * (double)s->scount[h]);
    return J * f * c;
  }
  return J * f;
}

static double event_weight(const ora_state *s, uint32_t iter, uint64_t i, int *bins) {
  return event_weight_obs(s, iter, i, bins, NULL);
}

/* bin of observable value o: 1 .. nobs for lo <= o < hi (uniform width), 0 below,
 * nobs + 1 at or above hi (and for a value that is not a number) */
static int obs_bin(const ora_state *s, double o) {
  if (o < s->obs_lo) return 0;
  if (!(o < s->obs_hi)) return s->nobs + 1;
  double t = floor((o - s->obs_lo) * ((double)s->nobs / (s->obs_hi - s->obs_lo)));
  return t < (double)s->nobs ? (int)t + 1 : s->nobs; /* the last bin holds [hi - width, hi) */
}

int ora_event_weights(const ora_state *s, uint32_t iter, int64_t first, int64_t n,
                      double *w, uint8_t *bins) {
  int b[16];
  for (int64_t i = 0; i < n; ++i) {
    w[i] = event_weight(s, iter, (uint64_t)(first + i), b);
    if (bins)
      for (int d = 0; d < s->ndim; ++d) bins[i * s->ndim + d] = (uint8_t)b[d];
  }
  return 0;
}

/* One iteration: all n events at the current grid; S1 = sum w, S2 = sum w^2 and
 * d[dim][bin] = sum of w^2 over events in that bin, in long double.
 * Non-finite weights are counted and contribute nothing.
 * I_j = S1 / n, var_j = (S2 / n - I_j^2) / (n - 1). */
int64_t ora_strata_cubes(const ora_state *s) {
  if (s->strata_m <= 0) return 0;
  int64_t H = 1;
  for (int d = 0; d < s->ndim; ++d) {
    H *= s->strata_m;
    if (H > 2147483647LL) return -1;
  }
  return H;
}

static void strata_free(ora_state *s) {
  free(s->scount);
  free(s->soff);
  free(s->ssig);
  free(s->sinject);
  s->scount = s->soff = s->sinject = NULL;
  s->ssig = NULL;
  s->have_sig = s->have_inject = 0;
}

int ora_set_strata(ora_state *s, int m) {
  if (m < 0) return -1;
  int old = s->strata_m;
  s->strata_m = m;
  if (ora_strata_cubes(s) < 0) {
    s->strata_m = old;
    return -1;
  }
  s->strata_npc = 0;
  strata_free(s);
  return 0;
}

/* beta > 0: adaptive allocation (VEGAS+ reading): iteration j + 1 gives hypercube h
 * n_h = 2 + floor((n - 2H) p_h / sum p) events with p_h = sigma_h^beta, sigma_h the
 * standard deviation of the (unscaled) weight in h in iteration j, the remaining
 * R = n - 2H - sum floor(...) events one each to hypercubes 0 .. R - 1 (equal counts
 * before any stratified iteration, if every p_h is 0, or if R came out negative);
 * beta = 0: equal counts floor(n / H), the rest of n unused. */
int ora_set_strata_beta(ora_state *s, double beta) {
  if (!(beta >= 0.0) || !isfinite(beta)) return -1;
  s->strata_beta = beta;
  s->have_sig = 0;
  return 0;
}

/* counts of the last iteration's hypercubes (H of them) */
int ora_get_strata_counts(const ora_state *s, int64_t *counts) {
  int64_t H = ora_strata_cubes(s);
  if (H <= 0 || s->strata_npc <= 0) return -2;
  if (s->strata_beta <= 0.0 || !s->scount) {
    for (int64_t h = 0; h < H; ++h) counts[h] = s->strata_npc;
    return 0;
  }
  memcpy(counts, s->scount, sizeof(int64_t) * (size_t)H);
  return 0;
}

/* counts the next (adaptive) iteration uses instead of its own allocation; they
 * must sum to that iteration's n, each >= 2 */
int ora_inject_strata_counts(ora_state *s, const int64_t *counts) {
  int64_t H = ora_strata_cubes(s);
  if (H <= 0 || s->strata_beta <= 0.0) return -1;
  free(s->sinject);
  s->sinject = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
  memcpy(s->sinject, counts, sizeof(int64_t) * (size_t)H);
  s->have_inject = 1;
  return 0;
}

/* the counts the allocation rule gives for n events over H hypercubes */
static void strata_rule(const ora_state *s, int64_t H, int64_t n, int64_t *cnt) {
  int64_t free_ev = n - 2 * H;
  int have = s->have_sig && s->ssig;
  long double A = 0.0L;
  for (int64_t h = 0; h < H; ++h) A += have ? (long double)pow(s->ssig[h], s->strata_beta) : 1.0L;
  double Ad = (double)A;
  int64_t F = 0;
  int equal = !(Ad > 0.0);
  if (!equal) {
    for (int64_t h = 0; h < H; ++h) {
      double p = have ? pow(s->ssig[h], s->strata_beta) : 1.0;
      cnt[h] = (int64_t)floor((double)free_ev * p / Ad);
      F += cnt[h];
    }
    if (F > free_ev) equal = 1;
  }
  if (equal) {
    F = 0;
    for (int64_t h = 0; h < H; ++h) {
      cnt[h] = free_ev / H;
      F += cnt[h];
    }
  }
  int64_t R = free_ev - F;
  for (int64_t h = 0; h < H; ++h) cnt[h] += 2 + (h < R ? 1 : 0);
}

/* the counts the next adaptive iteration of n events would use (no state change) */
int ora_strata_next_counts(const ora_state *s, int64_t n, int64_t *counts) {
  int64_t H = ora_strata_cubes(s);
  if (H <= 0 || s->strata_beta <= 0.0 || n < 2 * H) return -1;
  strata_rule(s, H, n, counts);
  return 0;
}

/* the allocation of an adaptive iteration of n events over H hypercubes */
static int strata_allocate(ora_state *s, int64_t H, int64_t n) {
  if (!s->scount) {
    s->scount = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
    s->soff = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
    s->ssig = (double *)calloc((size_t)H, sizeof(double));
  }
  if (s->have_inject) {
    int64_t tot = 0;
    for (int64_t h = 0; h < H; ++h) {
      if (s->sinject[h] < 2) return -1;
      tot += s->sinject[h];
    }
    if (tot != n) return -1;
    memcpy(s->scount, s->sinject, sizeof(int64_t) * (size_t)H);
    s->have_inject = 0;
  } else {
    strata_rule(s, H, n, s->scount);
  }
  int64_t o = 0;
  for (int64_t h = 0; h < H; ++h) {
    s->soff[h] = o;
    o += s->scount[h];
  }
  return 0;
}

int64_t ora_strata_npc(const ora_state *s) { return s->strata_npc; }

int ora_iterate(ora_state *s, int64_t n_req, double out[4]) {
  if (n_req < 2) return -1;
  /* stratified: npc = floor(n / m^D) >= 2 events in each hypercube, n = m^D npc used */
  int64_t H = ora_strata_cubes(s), n = n_req;
  if (H > 0) {
    if (n_req / H < 2) return -1;
    s->strata_npc = n_req / H;
    n = H * s->strata_npc;
    if (s->strata_beta > 0.0) {
      n = n_req;
      if (strata_allocate(s, H, n) != 0) return -1;
    }
  }
  double *wrec = H > 0 ? (double *)malloc(sizeof(double) * (size_t)n) : NULL;
  int D = s->ndim, nb = s->nbins;
  for (int i = 0; i < D * nb; ++i) s->d[i] = 0.0L;
  long double s1 = 0.0L, s2 = 0.0L;
  int64_t nz = 0, nnf = 0;
  int b[16];
  const int nob = s->nobs ? s->nobs + 2 : 0;
  for (int k = 0; k < nob; ++k) s->obs_s1[k] = s->obs_s2[k] = 0.0L;
  for (int64_t i = 0; i < n; ++i) {
    double o = 0.0;
    double w = event_weight_obs(s, s->iter, (uint64_t)i, b, s->nobs ? &o : NULL);
    if (wrec) wrec[i] = isfinite(w) ? w : 0.0;
    if (!isfinite(w)) { ++nnf; continue; }
    if (w != 0.0) ++nz;
    double w2 = w * w;
    s1 += w;
    s2 += w2;
    for (int d = 0; d < D; ++d) s->d[d * nb + b[d]] += w2;
    if (s->nobs) {
      int k = obs_bin(s, o);
      s->obs_s1[k] += w;
      s->obs_s2[k] += w2;
    }
  }
  s->s1 = s1;
  s->s2 = s2;
  s->have_hist = 1;
  double mean = (double)(s1 / (long double)n);
  double var = (double)((s2 / (long double)n - (long double)mean * (long double)mean) / (long double)(n - 1));
  if (H > 0) {
    /* stratified estimate: I = sum_h (1/H) mean_h = S1 / n (equal counts), and
     * var = sum_h (1/H)^2 sigma_h^2 / npc with the within-hypercube sample variance
     * sigma_h^2 = sum_{i in h} (w_i - mean_h)^2 / (npc - 1) */
    if (s->strata_beta <= 0.0) {
      int64_t c = s->strata_npc;
      long double V = 0.0L;
      for (int64_t h = 0; h < H; ++h) {
        long double sh = 0.0L;
        for (int64_t k = 0; k < c; ++k) sh += wrec[h * c + k];
        long double mh = sh / (long double)c;
        for (int64_t k = 0; k < c; ++k) {
          long double dv = (long double)wrec[h * c + k] - mh;
          V += dv * dv;
        }
      }
      var = (double)(V / ((long double)H * (long double)H * (long double)c * (long double)(c - 1)));
    } else {
      /* unequal counts: with scaled weights w_s = c_h w, sum_h (1/H)^2 sigma_h^2(w) / n_h
       * = sum_h n_h sigma_h^2(w_s) / N^2; sigma_h(w) = sigma_h(w_s) / c_h is kept for
       * the next allocation */
      long double V = 0.0L;
      for (int64_t h = 0; h < H; ++h) {
        int64_t c = s->scount[h], o = s->soff[h];
        long double sh = 0.0L;
        for (int64_t k = 0; k < c; ++k) sh += wrec[o + k];
        long double mh = sh / (long double)c, q = 0.0L;
        for (int64_t k = 0; k < c; ++k) {
          long double dv = (long double)wrec[o + k] - mh;
          q += dv * dv;
        }
        V += (long double)c * q / (long double)(c - 1);
        long double ch = (long double)n / ((long double)H * (long double)c);
        s->ssig[h] = (double)(sqrtl(q / (long double)(c - 1)) / ch);
      }
      var = (double)(V / ((long double)n * (long double)n));
      s->have_sig = 1;
    }
    free(wrec);
  }
  if (s->n_iter == s->cap) {
    s->cap *= 2;
    s->Ij = (double *)realloc(s->Ij, sizeof(double) * s->cap);
    s->varj = (double *)realloc(s->varj, sizeof(double) * s->cap);
  }
  s->Ij[s->n_iter] = mean;
  s->varj[s->n_iter] = var;
  if (s->nobs) {
    /* this iteration's histogram (sum of w / n per bin) and its error; iterations
     * from obs_first on enter the combination with the weights of the integral
     * (1 / var_j), or as a plain mean if some iteration has zero variance */
    for (int k = 0; k < nob; ++k) {
      long double h = s->obs_s1[k] / (long double)n;
      long double v = (s->obs_s2[k] / (long double)n - h * h) / (long double)(n - 1);
      s->obs_last[k] = (double)h;
      s->obs_last_err[k] = (double)sqrtl(v > 0.0L ? v : 0.0L);
      if ((int)s->iter >= s->obs_first) {
        if (var > 0.0) {
          long double wj = 1.0L / (long double)var;
          s->obs_acc_w[k] += wj * h;
          s->obs_acc_v[k] += wj * wj * v;
        } else {
          s->obs_zacc[k] += h;
        }
      }
    }
    if ((int)s->iter >= s->obs_first) {
      if (var > 0.0) s->obs_wsum += 1.0L / (long double)var;
      else s->obs_zcount++;
    }
    s->obs_have = 1;
  }
  s->n_iter++;
  s->iter++;
  out[0] = mean;
  out[1] = var;
  out[2] = (double)nz;
  out[3] = (double)nnf;
  return 0;
}

/* The CPU scheme of the paper, for the all-core baseline beside the serial
 * oracle (Sec. 2.2): the event loop split over nthreads threads, thread t
 * taking the fixed chunk of events [t n / T, (t + 1) n / T) and accumulating
 * its own long-double S1, S2 and d; the chunks' partials are then added in
 * chunk order, so the result depends on T only through that fixed split, never
 * on the scheduling.  Plain importance sampling only (no strata, no observable).
 * Updates the state exactly as ora_iterate does. */
int ora_iterate_threads(ora_state *s, int64_t n, int nthreads, double out[4]) {
  if (n < 2 || nthreads < 1 || s->strata_m > 0 || s->nobs) return -1;
  const int D = s->ndim, nb = s->nbins, T = nthreads;
  const size_t row = 2 + (size_t)D * nb;
  long double *part = (long double *)calloc((size_t)T * row, sizeof(long double));
  int64_t *cnt = (int64_t *)calloc((size_t)T * 2, sizeof(int64_t));
  if (!part || !cnt) {
    free(part);
    free(cnt);
    return -1;
  }
#pragma omp parallel for schedule(static, 1) num_threads(T)
  for (int t = 0; t < T; ++t) {
    long double *p = part + (size_t)t * row;
    int b[16];
    const int64_t lo = n * t / T, hi = n * (t + 1) / T;
    for (int64_t i = lo; i < hi; ++i) {
      double w = event_weight(s, s->iter, (uint64_t)i, b);
      if (!isfinite(w)) { ++cnt[2 * t + 1]; continue; }
      if (w != 0.0) ++cnt[2 * t];
      double w2 = w * w;
      p[0] += w;
      p[1] += w2;
      for (int d = 0; d < D; ++d) p[2 + d * nb + b[d]] += w2;
    }
  }
  long double s1 = 0.0L, s2 = 0.0L;
  int64_t nz = 0, nnf = 0;
  for (int i = 0; i < D * nb; ++i) s->d[i] = 0.0L;
  for (int t = 0; t < T; ++t) {
    const long double *p = part + (size_t)t * row;
    s1 += p[0];
    s2 += p[1];
    for (int i = 0; i < D * nb; ++i) s->d[i] += p[2 + i];
    nz += cnt[2 * t];
    nnf += cnt[2 * t + 1];
  }
  free(part);
  free(cnt);
  s->s1 = s1;
  s->s2 = s2;
  s->have_hist = 1;
  double mean = (double)(s1 / (long double)n);
  double var = (double)((s2 / (long double)n - (long double)mean * (long double)mean) / (long double)(n - 1));
  if (s->n_iter == s->cap) {
    s->cap *= 2;
    s->Ij = (double *)realloc(s->Ij, sizeof(double) * s->cap);
    s->varj = (double *)realloc(s->varj, sizeof(double) * s->cap);
  }
  s->Ij[s->n_iter] = mean;
  s->varj[s->n_iter] = var;
  s->n_iter++;
  s->iter++;
  out[0] = mean;
  out[1] = var;
  out[2] = (double)nz;
  out[3] = (double)nnf;
  return 0;
}

/* Refinement of one dimension (edges e[0..n], histogram d[0..n-1]):
 * smooth with neighbours, normalise to r_k, damp m_k = ((r_k - 1) / ln r_k)^alpha,
 * then place the new interior edges where the cumulative m of the old bins
 * reaches k * sum(m) / n, linearly inside the old bin. */
/* Smoothed, normalised and damped importance of each old bin:
 * dbar_k = mean of d over k and its neighbours, r_k = dbar_k / sum(dbar),
 * m_k = ((r_k - 1) / ln r_k)^alpha with the limits m = 0 at r = 0, m = 1 at r = 1.
 * Returns 0 when the histogram is empty (the grid then stays). */
int ora_refine_weights(int n, double alpha, const double *d, double *m) {
  double dsum = 0.0;
  for (int k = 0; k < n; ++k) dsum += d[k];
  if (!(dsum > 0.0)) return 0;
  double *db = (double *)malloc(sizeof(double) * n);
  db[0] = (d[0] + d[1]) / 2.0;
  db[n - 1] = (d[n - 2] + d[n - 1]) / 2.0;
  for (int k = 1; k < n - 1; ++k) db[k] = (d[k - 1] + d[k] + d[k + 1]) / 3.0;
  double dbsum = 0.0;
  for (int k = 0; k < n; ++k) dbsum += db[k];
  for (int k = 0; k < n; ++k) {
    double r = db[k] / dbsum;
    if (r == 0.0) m[k] = 0.0;
    else if (r == 1.0) m[k] = 1.0;
    else m[k] = pow((r - 1.0) / log(r), alpha);
  }
  free(db);
  return 1;
}

/* Refinement of one dimension (edges e[0..n], histogram d[0..n-1]): place the
 * new interior edges where the cumulative m of the old bins reaches
 * k * sum(m) / n, linearly inside the old bin. */
static void refine_dim(int n, double alpha, const double *d, double *e) {
  double *m = (double *)malloc(sizeof(double) * n);
  double *enew = (double *)malloc(sizeof(double) * (n + 1));
  if (!ora_refine_weights(n, alpha, d, m)) {
    free(m);
    free(enew);
    return;
  }
  double msum = 0.0;
  for (int k = 0; k < n; ++k) msum += m[k];
  double step = msum / n;
  enew[0] = 0.0;
  enew[n] = 1.0;
  int j = 0;
  double cum = 0.0; /* cumulative m of old bins 0..j-1 */
  for (int k = 1; k < n; ++k) {
    double target = k * step;
    while (j < n - 1 && cum + m[j] < target) {
      cum += m[j];
      ++j;
    }
    double frac = m[j] > 0.0 ? (target - cum) / m[j] : 0.0;
    if (frac < 0.0) frac = 0.0;
    if (frac > 1.0) frac = 1.0;
    enew[k] = e[j] + frac * (e[j + 1] - e[j]);
  }
  memcpy(e, enew, sizeof(double) * (n + 1));
  free(m);
  free(enew);
}

int ora_refine_grid(int ndim, int nbins, double alpha, const double *d, double *edges) {
  for (int dd = 0; dd < ndim; ++dd) refine_dim(nbins, alpha, d + dd * nbins, edges + dd * (nbins + 1));
  return 0;
}

int ora_refine(ora_state *s) {
  if (!s->have_hist) return -2;
  int D = s->ndim, nb = s->nbins;
  double *d = (double *)malloc(sizeof(double) * D * nb);
  for (int i = 0; i < D * nb; ++i) d[i] = (double)s->d[i];
  ora_refine_grid(D, nb, s->alpha, d, s->edges);
  free(d);
  return 0;
}

/* Inverse-variance combination over iterations first .. n_iter-1; chi^2 per
 * degree of freedom about the combined value.  Iterations with zero variance
 * (a constant integrand) are exact: their plain mean is returned with sigma 0.
 * first > 0 drops the warm-up stage of a two-stage schedule such as the one of
 * the timing runs in Sec. 3.2. */
int ora_result_from(const ora_state *s, int first, double out[4]) {
  int n = s->n_iter;
  out[0] = out[1] = out[2] = 0.0;
  out[3] = 0.0;
  if (n == 0) return -2;
  if (first < 0 || first >= n) return -1;
  out[3] = n - first;
  int nzero = 0;
  long double zsum = 0.0L;
  for (int j = first; j < n; ++j)
    if (s->varj[j] <= 0.0) { ++nzero; zsum += s->Ij[j]; }
  if (nzero) {
    out[0] = (double)(zsum / nzero);
    return 0;
  }
  long double wsum = 0.0L, iwsum = 0.0L;
  for (int j = first; j < n; ++j) {
    wsum += 1.0L / s->varj[j];
    iwsum += (long double)s->Ij[j] / s->varj[j];
  }
  long double comb = iwsum / wsum;
  out[0] = (double)comb;
  out[1] = (double)sqrtl(1.0L / wsum);
  if (n - first > 1) {
    long double chi = 0.0L;
    for (int j = first; j < n; ++j) chi += (s->Ij[j] - comb) * (s->Ij[j] - comb) / s->varj[j];
    out[2] = (double)(chi / (n - first - 1));
  }
  return 0;
}

/* All iterations so far. */
int ora_result(const ora_state *s, double out[4]) { return ora_result_from(s, 0, out); }

/* Observable histogram: nbins uniform bins on [lo, hi) plus under- and overflow
 * (nbins = 0 turns it off); iterations from `first` (the iteration counter) on are
 * combined.  Clears the combination. */
int ora_set_observable(ora_state *s, int nbins, double lo, double hi, int first) {
  if (nbins < 0 || nbins > ORA_MAX_OBS || first < 0) return -1;
  if (nbins > 0 && !(isfinite(lo) && isfinite(hi) && lo < hi && isfinite((double)nbins / (hi - lo))))
    return -1;
  s->nobs = nbins;
  s->obs_lo = lo;
  s->obs_hi = hi;
  s->obs_first = first;
  s->obs_have = 0;
  for (int k = 0; k < ORA_MAX_OBS + 2; ++k) s->obs_acc_w[k] = s->obs_acc_v[k] = s->obs_zacc[k] = 0.0L;
  s->obs_wsum = 0.0L;
  s->obs_zcount = 0;
  return 0;
}

/* last iteration's histogram and error, and the combination and its error
 * (arrays of nbins + 2, each nullable); -2 before any iteration with it on */
int ora_get_observable(const ora_state *s, double *last, double *last_err, double *comb, double *comb_err) {
  if (!s->nobs || !s->obs_have) return -2;
  for (int k = 0; k < s->nobs + 2; ++k) {
    if (last) last[k] = s->obs_last[k];
    if (last_err) last_err[k] = s->obs_last_err[k];
    double c = 0.0, e = 0.0;
    if (s->obs_zcount) {
      c = (double)(s->obs_zacc[k] / s->obs_zcount);
    } else if (s->obs_wsum > 0.0L) {
      c = (double)(s->obs_acc_w[k] / s->obs_wsum);
      e = (double)(sqrtl(s->obs_acc_v[k]) / s->obs_wsum);
    }
    if (comb) comb[k] = c;
    if (comb_err) comb_err[k] = e;
  }
  return 0;
}

int ora_get_grid(const ora_state *s, double *edges) {
  memcpy(edges, s->edges, sizeof(double) * s->ndim * (s->nbins + 1));
  return 0;
}

int ora_set_grid(ora_state *s, const double *edges) {
  memcpy(s->edges, edges, sizeof(double) * s->ndim * (s->nbins + 1));
  return 0;
}

int ora_get_hist(const ora_state *s, double *d, double sums[2]) {
  for (int i = 0; i < s->ndim * s->nbins; ++i) d[i] = (double)s->d[i];
  sums[0] = (double)s->s1;
  sums[1] = (double)s->s2;
  return s->have_hist ? 0 : -2;
}

int ora_set_iteration(ora_state *s, uint32_t iter) {
  s->iter = iter;
  return 0;
}

uint32_t ora_get_iteration(const ora_state *s) { return s->iter; }

/* ======================================================================
 * Adjoint oracle for the Drell-Yan integrand: forward-mode dual numbers with
 * five tangent directions theta = (M_Z, G_Z, sw^2, a, b).  The event's mapped
 * point (and so the grid, Breit-Wigner and tau Jacobians) stays at the nominal
 * parameters stored in the state; |M|^2 and the PDFs take theta.
 * ====================================================================== */
typedef struct { double v, d[5]; } dual;

static dual dconst(double v) { dual r; r.v = v; for (int i = 0; i < 5; ++i) r.d[i] = 0.0; return r; }
static dual dvar(double v, int k) { dual r = dconst(v); r.d[k] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
static dual ddiv(dual a, dual b) { dual r; r.v = a.v / b.v; for (int i = 0; i < 5; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v); return r; }
static dual dsqrt(dual a) { dual r; r.v = sqrt(a.v); for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] / (2.0 * r.v); return r; }
static dual dexp(dual a) { dual r; r.v = exp(a.v); for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] * r.v; return r; }
static dual dscale(dual a, double c) { dual r; r.v = a.v * c; for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] * c; return r; }

/* <|M|^2>(c) of ora_me_dy with dual parameters; A = Re + i Im written out */
static dual me_dy_dual(double alpha, dual sw2, dual mz, dual gz, double shat, double c, int flavour) {
  dual sw = dsqrt(sw2), cw = dsqrt(dsub(dconst(1.0), sw2));
  dual swcw = dmul(sw, cw);
  double Qq = flavour == 0 ? 2.0 / 3.0 : -1.0 / 3.0, T3 = flavour == 0 ? 0.5 : -0.5;
  dual gq[2], gl[2];
  gq[0] = ddiv(dsub(dconst(T3), dscale(sw2, Qq)), swcw);
  gq[1] = ddiv(dscale(sw, -Qq), cw);
  gl[0] = ddiv(dsub(dconst(-0.5), dscale(sw2, -1.0)), swcw);
  gl[1] = ddiv(sw, cw);
  dual mz2 = dmul(mz, mz);
  dual ds = dsub(dconst(shat), mz2);
  dual mg = dmul(mz, gz);
  dual den = dadd(dmul(ds, ds), dmul(mg, mg));
  dual pre = ddiv(ds, den), pim = ddiv(dscale(mg, -1.0), den); /* 1/(s - M^2 + i M G) */
  double e2 = 4.0 * PI * alpha;
  dual sum = dconst(0.0);
  for (int h = 0; h < 2; ++h)
    for (int hp = 0; hp < 2; ++hp) {
      dual gg = dmul(gq[h], gl[hp]);
      dual re = dadd(dconst(-Qq / shat), dmul(gg, pre));
      dual im = dmul(gg, pim);
      dual a2 = dadd(dmul(re, re), dmul(im, im));
      double ang = (h == hp) ? (1.0 + c) * (1.0 + c) : (1.0 - c) * (1.0 - c);
      sum = dadd(sum, dscale(a2, ang));
    }
  return dscale(sum, e2 * e2 * shat * shat / 12.0);
}

static dual dy_weight_dual(const ora_state *s, uint32_t iter, uint64_t i, const double *theta) {
  double u[16], x[16], J;
  int b[16];
  ora_uniforms(s->seed, iter, i, s->ndim, u);
  grid_map(s, u, x, &J, b);
  phys P = unpack(s->params);
  double S = P.sqrts * P.sqrts;
  double m2, jbw;
  bw_map(P.mz, P.gz, P.mlo * P.mlo, P.mhi * P.mhi, x[0], &m2, &jbw);
  double tau = m2 / S, L = log(tau), l1 = x[1] * L, l2 = L - l1, jtau = -L / S;
  double c = 2.0 * x[2] - 1.0;
  dual mz = dvar(theta[0], 0), gz = dvar(theta[1], 1), sw2 = dvar(theta[2], 2);
  dual a = dvar(theta[3], 3), bb = dvar(theta[4], 4);
  /* f(x) = A exp(a ln x + b ln(1-x)) */
  dual f1 = dscale(dexp(dadd(dscale(a, l1), dscale(bb, log(-expm1(l1))))), P.A);
  dual f2 = dscale(dexp(dadd(dscale(a, l2), dscale(bb, log(-expm1(l2))))), P.A);
  dual me = dconst(0.0);
  for (int q = 0; q < 2; ++q) {
    me = dadd(me, me_dy_dual(P.alpha, sw2, mz, gz, m2, c, q));
    me = dadd(me, me_dy_dual(P.alpha, sw2, mz, gz, m2, -c, q));
  }
  double pre = P.conv * jbw * jtau * 2.0 * (1.0 / (2.0 * m2)) * (2.0 * PI / (32.0 * PI * PI)) * J;
  return dscale(dmul(dmul(f1, f2), me), pre);
}

double ora_dy_weight_theta(const ora_state *s, uint32_t iter, int64_t event, const double *theta) {
  return dy_weight_dual(s, iter, (uint64_t)event, theta).v;
}

int ora_dy_grad(const ora_state *s, uint32_t iter, int64_t n, const double *theta,
                double *sigma, double dsigma[5]) {
  if (s->process != ORA_DY_Z || n < 1) return -1;
  long double sv = 0.0L, sd[5] = {0, 0, 0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    dual w = dy_weight_dual(s, iter, (uint64_t)i, theta);
    sv += w.v;
    for (int k = 0; k < 5; ++k) sd[k] += w.d[k];
  }
  *sigma = (double)(sv / n);
  for (int k = 0; k < 5; ++k) dsigma[k] = (double)(sd[k] / n);
  return 0;
}
