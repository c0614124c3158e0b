"""Pins for the oracle's integrands against closed forms and quadrature (CPU only).

The paper prints no matrix element or phase space (its process code lives in
MCFM, Sec. 2.1); the integrands are the readings listed in the design notes.
Each is pinned here by something other than itself: textbook cross sections,
resonance widths and asymmetries, Lorentz invariance, gauge cancellation, the
narrow-width limit and brute-force quadrature.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

ALPHA = 1 / 128
E2 = 4 * math.pi * ALPHA
GL = {n: np.polynomial.legendre.leggauss(n) for n in (4, 16, 24, 40, 64, 128)}


def gl01(n):
    x, w = GL[n]
    return 0.5 * (x + 1), 0.5 * w


def composite(f, a, b, panels, n=16):
    x, w = GL[n]
    edges = np.linspace(a, b, panels + 1)
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        xm, xr = 0.5 * (hi + lo), 0.5 * (hi - lo)
        tot += xr * sum(wi * f(xm + xr * xi) for xi, wi in zip(x, w))
    return tot


# ------------------------------------------------------------ e+e- -> mu+mu-
def test_eemumu_pointwise_textbook():
    """<|M|^2> = 2 e^4 (t^2 + u^2)/s^2 from the explicit Dirac currents."""
    p = W.phys_params(91.0)
    s = 91.0 ** 2
    for c in np.linspace(-0.99, 0.99, 9):
        t, u = -s * (1 - c) / 2, -s * (1 + c) / 2
        me = oracle.me_eemumu_dirac(p, s, c, 0.37)
        assert abs(me / (2 * E2 ** 2 * (t * t + u * u) / s ** 2) - 1) < 1e-13


def test_eemumu_total_cross_section():
    """sigma = 4 pi alpha^2 / (3 s), by quadrature of the 2-D integrand."""
    p = W.phys_params(91.0)
    s = 91.0 ** 2
    xa, wa = gl01(4)
    xb, wb = gl01(4)
    tot = sum(wi * wj * oracle.integrand(W.EEMUMU, p, [x, y])
              for x, wi in zip(xa, wa) for y, wj in zip(xb, wb))
    exact = 4 * math.pi * ALPHA ** 2 / (3 * s) * p[15]
    assert abs(tot / exact - 1) < 1e-13


def test_spinors_solve_dirac_equation():
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = rng.normal(size=3) * rng.uniform(0.1, 100)
        r1, r2 = oracle.spinor_check(np.array([np.linalg.norm(v), *v]))
        assert r1 < 1e-12 * np.linalg.norm(v) and r2 < 1e-12 * np.linalg.norm(v)
    for p in ([5.0, 0, 0, 5.0], [5.0, 0, 0, -5.0]):   # along the beams (branch ends)
        r1, r2 = oracle.spinor_check(np.array(p))
        assert r1 < 1e-14 and r2 < 1e-13


# ------------------------------------------------------------ Drell-Yan ----
def dy_couplings(sw2, flavour):
    sw, cw = math.sqrt(sw2), math.sqrt(1 - sw2)
    Q, T3 = (2 / 3, 0.5) if flavour == 0 else (-1 / 3, -0.5)
    gq = ((T3 - Q * sw2) / (sw * cw), -Q * sw / cw)
    gl = ((-0.5 + sw2) / (sw * cw), sw / cw)
    return Q, gq, gl


def test_dy_photon_only_limit():
    """With the Z pushed far away, sigmahat(q qbar -> gamma* -> l l) =
    4 pi alpha^2 Q_q^2 / (9 shat) (textbook, with the 1/N_c colour average)."""
    p = W.phys_params(mz=1.0e9)
    for fl, Q in ((0, 2 / 3), (1, -1 / 3)):
        for shat in (50.0 ** 2, 200.0 ** 2):
            exact = 4 * math.pi * ALPHA ** 2 * Q * Q / (9 * shat)
            assert abs(oracle.sigmahat_dy(p, shat, fl) / exact - 1) < 1e-12


def test_dy_angular_integral_matches_sigmahat():
    """int dc <|M|^2>(c) / (32 pi shat) = sigmahat (4-point GL is exact for (1 +- c)^2)."""
    p = W.phys_params()
    x, w = GL[4]
    for fl in (0, 1):
        for shat in (60.0 ** 2, 91.0 ** 2, 150.0 ** 2):
            tot = sum(wi * oracle.me_dy(p, shat, xi, fl) for xi, wi in zip(x, w))
            assert abs(tot / (32 * math.pi * shat) / oracle.sigmahat_dy(p, shat, fl) - 1) < 1e-13


def test_dy_z_peak_and_asymmetry():
    """At shat = M_Z^2 the photon and the (imaginary) Z amplitude do not interfere:
    sigmahat = photon part + (12 pi / M^2) G_qq G_ll / (N_c^2 G_Z^2), with the
    textbook widths G_ff = N_c alpha M (g_L^2 + g_R^2) / 6; and the forward-backward
    asymmetry is (3/4) A_q A_l times the Z fraction, A_f = (gL^2 - gR^2)/(gL^2 + gR^2)."""
    p = W.phys_params()
    sw2, MZ, GZ = p[1], p[2], p[3]
    s = MZ * MZ
    x, w = GL[16]
    for fl in (0, 1):
        Q, gq, gl = dy_couplings(sw2, fl)
        sq, sl = gq[0] ** 2 + gq[1] ** 2, gl[0] ** 2 + gl[1] ** 2
        Gqq, Gll = 3 * ALPHA * MZ * sq / 6, ALPHA * MZ * sl / 6
        photon = 4 * math.pi * ALPHA ** 2 * Q * Q / (9 * s)
        zpeak = 12 * math.pi / s * Gqq * Gll / (9 * GZ * GZ)
        assert abs(oracle.sigmahat_dy(p, s, fl) / (photon + zpeak) - 1) < 1e-12
        F = sum(0.5 * wi * oracle.me_dy(p, s, 0.5 * (xi + 1), fl) for xi, wi in zip(x, w))
        B = sum(0.5 * wi * oracle.me_dy(p, s, 0.5 * (xi - 1), fl) for xi, wi in zip(x, w))
        Aq = (gq[0] ** 2 - gq[1] ** 2) / sq
        Al = (gl[0] ** 2 - gl[1] ** 2) / sl
        zfrac = sq * sl / (MZ * GZ) ** 2 / (sq * sl / (MZ * GZ) ** 2 + 4 * (Q / s) ** 2)
        assert abs((F - B) / (F + B) / (0.75 * Aq * Al * zfrac) - 1) < 1e-12


def pdf(x, A=1.0, a=-0.5, b=3.0):
    return A * x ** a * (1 - x) ** b


def test_dy_hadronic_integrand_by_quadrature():
    """The 3-D C0 integrand (Breit-Wigner and ln-x mappings, both beam orderings)
    integrated by Gauss-Legendre equals the 2-D hadronic formula
    2 sum_q int dm^2/S int d ln x1 f(x1) f(tau/x1) sigmahat_q, done in plain m^2."""
    cfg = W.config("dy_z")
    p = cfg["params"]
    S = p[6] ** 2
    x0, w0 = gl01(64)
    x1, w1 = gl01(24)
    x2, w2 = GL[4]
    tot = 0.0
    for a, wa in zip(x0, w0):
        for b, wb in zip(x1, w1):
            for c, wc in zip(x2, w2):
                tot += wa * wb * 0.5 * wc * oracle.integrand(W.DY_Z, p, [a, b, 0.5 * (c + 1)])

    def inner(m2):
        tau = m2 / S
        L = math.log(tau)
        ys, ws = gl01(24)
        lum = sum(wy * (-L) * pdf(math.exp(y * L)) * pdf(tau / math.exp(y * L))
                  for y, wy in zip(ys, ws))
        return 2 * lum / S * (oracle.sigmahat_dy(p, m2, 0) + oracle.sigmahat_dy(p, m2, 1))

    ref = composite(inner, 81.0 ** 2, 101.0 ** 2, 200) * p[15]
    assert abs(tot / ref - 1) < 1e-9


# ------------------------------------------------------------ W+ -----------
def sigmahat_w(p, shat):
    g2 = 4 * math.pi * p[0] / p[1]
    D = (shat - p[4] ** 2) ** 2 + (p[4] * p[5]) ** 2
    return g2 * g2 * p[14] ** 2 * shat / (576 * math.pi * D)


def test_w_partonic_narrow_width_textbook():
    """int dshat sigmahat(u dbar -> W -> e nu) -> (pi/3) sqrt2 G_F M^2 |V|^2 BR as
    G -> 0, with sqrt2 G_F M^2 = g^2/4 and BR = g^2 M / (48 pi G)."""
    p = W.phys_params(gw=0.0021)
    M, G = p[4], p[5]
    g2 = 4 * math.pi * p[0] / p[1]
    rho = lambda r: M * M + M * G * math.tan(r)
    lo, hi = math.atan((10.0 ** 2 - M * M) / (M * G)), math.atan((1000.0 ** 2 - M * M) / (M * G))
    val = composite(lambda r: sigmahat_w(p, rho(r)) * M * G / math.cos(r) ** 2, lo, hi, 400)
    exact = math.pi / 3 * g2 / 4 * (g2 * M / (48 * math.pi * G))
    assert abs(val / exact - 1) < 2e-4     # O(G/M) finite-width corrections


def test_w_hadronic_no_cuts_by_quadrature():
    """The 4-D C1 integrand without cuts, integrated by Gauss-Legendre, equals the
    2-D hadronic formula with the textbook-pinned sigmahat above.  The mass window
    is closed at 200 GeV so that both quadratures converge to 1e-9."""
    p = W.phys_params(13000.0, mlo=40.0, mhi=200.0, ptmin=0.0, etamax=1e300)
    S = p[6] ** 2
    x0, w0 = gl01(128)
    x1, w1 = gl01(24)
    x2, w2 = GL[4]
    tot = 0.0
    for a, wa in zip(x0, w0):
        for b, wb in zip(x1, w1):
            for c, wc in zip(x2, w2):
                tot += wa * wb * 0.5 * wc * oracle.integrand(W.W_PLUS, p, [a, b, 0.5 * (c + 1), 0.3])
    M, G = p[4], p[5]

    def inner(m2):
        tau = m2 / S
        L = math.log(tau)
        ys, ws = gl01(24)
        lum = sum(wy * (-L) * pdf(math.exp(y * L)) * pdf(tau / math.exp(y * L))
                  for y, wy in zip(ys, ws))
        return 2 * lum / S * sigmahat_w(p, m2)

    lo, hi = math.atan((40.0 ** 2 - M * M) / (M * G)), math.atan((200.0 ** 2 - M * M) / (M * G))
    ref = composite(lambda r: inner(M * M + M * G * math.tan(r)) * M * G / math.cos(r) ** 2,
                    lo, hi, 100) * p[15]
    assert abs(tot / ref - 1) < 1e-9


def w_with_cuts_reference(p):
    """2-D quadrature with the lepton cuts integrated analytically in cos(theta*):
    the accepted region is pT^2 = (m^2/4)(1 - c^2) > ptmin^2 and
    tanh(-eta - y) < c < tanh(eta - y), y = ln(x1/x2)/2."""
    S = p[6] ** 2
    M, G = p[4], p[5]
    g2 = 4 * math.pi * p[0] / p[1]
    th = lambda c: c + c ** 3 / 3

    def inner(m2):
        tau = m2 / S
        L = math.log(tau)
        if m2 <= 4 * p[12] ** 2:
            return 0.0
        cpt = math.sqrt(1 - 4 * p[12] ** 2 / m2)
        ys, ws = gl01(40)
        D = (m2 - M * M) ** 2 + (M * G) ** 2
        tot = 0.0
        for yy, wy in zip(ys, ws):
            l1 = yy * L
            x1, x2 = math.exp(l1), math.exp(L - l1)
            rap = 0.5 * math.log(x1 / x2)
            lo = max(-cpt, math.tanh(-p[13] - rap))
            hi = min(cpt, math.tanh(p[13] - rap))
            if hi <= lo:
                continue
            dsig = g2 * g2 * m2 * m2 / (48 * D) / (32 * math.pi * m2) * 2 * (th(hi) - th(lo))
            tot += wy * (-L) * pdf(x1) * pdf(x2) * dsig
        return tot / S

    lo, hi = math.atan((p[10] ** 2 - M * M) / (M * G)), math.atan((S - M * M) / (M * G))
    return composite(lambda r: inner(M * M + M * G * math.tan(r)) * M * G / math.cos(r) ** 2,
                     lo, hi, 300) * p[15]


def test_w_with_cuts_vegas_matches_analytic_cut_quadrature():
    cfg = W.config("w_plus")
    p = cfg["params"]
    ref = w_with_cuts_reference(p)
    v = oracle.Vegas(W.W_PLUS, 4, 100, 1, 1.5, p)
    for _ in range(8):
        v.iterate(100_000)
        v.refine()
    r = v.result()
    assert abs(r["I"] - ref) < 4 * r["sigma"], (r, ref)
    assert r["sigma"] / r["I"] < 2e-3


# ------------------------------------------------------------ W+ W- ---------
def test_ww_gauge_cancellation():
    """q qbar -> W_L W_L at fixed angle: the chosen relative sign of the s-channel
    and exchange diagrams keeps |M|^2 bounded as shat grows; the other sign grows
    like shat^2 (unitarity violation).  Right-handed quarks: photon and Z cancel."""
    p = W.phys_params(500.0)
    for fl in (0, 1):
        good = [oracle.ww_onshell_me2(p, rs * rs, 0.3, 0.7, fl, 0, 0, 0) for rs in (1e3, 1e4, 1e5)]
        bad = [oracle.ww_onshell_me2(p, rs * rs, 0.3, 0.7, fl, 0, 0, 0, -(-1)) for rs in (1e3, 1e4, 1e5)]
        assert good[2] / good[1] < 1.01 and good[1] / good[0] < 1.1
        assert bad[2] / bad[1] > 5e3
        r = [oracle.ww_onshell_me2(p, rs * rs, 0.3, 0.7, fl, 1, 0, 0) for rs in (1e3, 1e4, 1e5)]
        assert r[2] / r[1] < 1.01


def boost_matrix(beta):
    b2 = beta @ beta
    g = 1 / math.sqrt(1 - b2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * beta
    L[1:, 1:] += (g - 1) * np.outer(beta, beta) / b2
    return L


def test_ww_lorentz_invariance():
    p = W.phys_params(500.0)
    rng = np.random.default_rng(4)
    for _ in range(10):
        x = rng.uniform(0.05, 0.95, 8)
        mom, m2p, m2m, jac = oracle.ww_momenta(p, x)
        Lb = boost_matrix(rng.uniform(-0.5, 0.5, 3))
        mom2 = mom @ Lb.T
        for fl in (0, 1):
            for h in (0, 1):
                a = oracle.ww_me2(p, mom, m2p, m2m, fl, h)
                b = oracle.ww_me2(p, mom2, m2p, m2m, fl, h)
                assert abs(a / b - 1) < 1e-10


def test_ww_momenta_conserve_and_are_massless():
    p = W.phys_params(500.0)
    rng = np.random.default_rng(5)
    for _ in range(20):
        mom, m2p, m2m, jac = oracle.ww_momenta(p, rng.uniform(0, 1, 8))
        tot = mom[0] + mom[1] + mom[2] + mom[3]
        assert np.allclose(tot, [500.0, 0, 0, 0], atol=1e-9)
        for k in range(4):
            assert abs(mom[k, 0] ** 2 - mom[k, 1:] @ mom[k, 1:]) < 1e-8 * mom[k, 0] ** 2 + 1e-9
        q = mom[0] + mom[1]
        assert abs((q[0] ** 2 - q[1:] @ q[1:]) / m2p - 1) < 1e-10


@pytest.mark.slow
def test_ww_narrow_width_limit():
    """sigma(q qbar -> e+ nu mu- nubar) -> sigma(q qbar -> W+W-) * BR^2 for G_W -> 0,
    with the on-shell sigma from the polarisation-summed amplitude by 1-D
    quadrature and BR = g^2 M / (48 pi G) (textbook W -> e nu width)."""
    G = 0.0021
    p = W.phys_params(500.0, gw=G)
    shat, M = 500.0 ** 2, p[4]
    x, w = GL[64]
    tot = 0.0
    for c, wc in zip(x, w):
        tot += wc * sum(oracle.ww_onshell_me2(p, shat, c, 0.0, fl, h, a, b)
                        for fl in (0, 1) for h in (0, 1) for a in range(3) for b in range(3))
    lam = (shat - 2 * M * M) ** 2 - 4 * M ** 4
    sig_ww = p[15] / (2 * shat) / 12 * math.sqrt(lam) / (32 * math.pi ** 2 * shat) * 2 * math.pi * tot
    g2 = 4 * math.pi * p[0] / p[1]
    BR = g2 * M / (48 * math.pi * G)
    v = oracle.Vegas(W.WW_4L, 8, 50, 1, 1.5, p)
    for _ in range(7):
        v.iterate(60_000)
        v.refine()
    r = v.result()
    pred = sig_ww * BR ** 2
    assert abs(r["I"] / pred - 1) < 4 * r["sigma"] / r["I"] + 2e-3, (r, pred)


# ------------------------------------------------------------ hadronic W+ W- -
def sigma_ww_onshell(p, shat, nodes=48):
    """sigma(q qbar -> W+W-), summed over u and d, from the polarisation-summed
    on-shell amplitude by Gauss-Legendre in cos(theta) (two panels)."""
    M = p[4]
    x, w = np.polynomial.legendre.leggauss(nodes)
    tot = 0.0
    for lo, hi in ((-1.0, 0.0), (0.0, 1.0)):
        for c, wc in zip(0.5 * (x + 1) * (hi - lo) + lo, 0.5 * w * (hi - lo)):
            tot += wc * sum(oracle.ww_onshell_me2(p, shat, c, 0.0, fl, h, a, b)
                            for fl in (0, 1) for h in (0, 1) for a in range(3) for b in range(3))
    lam = (shat - 2 * M * M) ** 2 - 4 * M ** 4
    return p[15] / (2 * shat) / 12 * math.sqrt(lam) / (32 * math.pi ** 2 * shat) * 2 * math.pi * tot


def test_ww_hadronic_narrow_width_limit():
    """The 10-dim hadronic integrand for G_W -> 0 against
    int dtau 2 L(tau) sigma_WW(tau S) BR^2, L(tau) = int dx1/x1 f(x1) f(tau/x1):
    the on-shell partonic cross section (the partonic narrow-width pin's) folded
    by quadrature with the luminosity, over a sqrt(shat) window [150, 400] GeV
    that contains the W-pair threshold (below it the on-shell term vanishes)."""
    G = 0.0021
    p = W.phys_params(13000.0, gw=G, mlo=150.0, mhi=400.0)
    M, S = p[4], p[6] ** 2
    lth, lhi = math.log(4 * M * M / S), math.log(400.0 ** 2 / S)
    xs, ws = gl01(24)

    def lum(L):
        return sum(wy * (-L) * pdf(math.exp(y * L)) * pdf(math.exp((1 - y) * L)) for y, wy in zip(xs, ws))

    # ln tau = lth + t^2 takes out the square-root threshold of the phase space
    tmax = math.sqrt(lhi - lth)
    xg, wg = GL[16]
    pred = 0.0
    for a, b in ((0.0, 0.5 * tmax), (0.5 * tmax, tmax)):
        for t, wt in zip(0.5 * (xg + 1) * (b - a) + a, 0.5 * wg * (b - a)):
            L = lth + t * t
            tau = math.exp(L)
            pred += wt * 2 * t * tau * 2 * lum(L) * sigma_ww_onshell(p, tau * S)
    g2 = 4 * math.pi * p[0] / p[1]
    pred *= (g2 * M / (48 * math.pi * G)) ** 2
    v = oracle.Vegas(W.WW_HAD, 10, 50, 1, 1.5, p)
    for _ in range(7):
        v.iterate(60_000)
        v.refine()
    r = v.result()
    assert abs(r["I"] / pred - 1) < 4 * r["sigma"] / r["I"] + 5e-4, (r, pred)


def test_ww_hadronic_is_the_partonic_integrand_at_tau_s():
    """Pointwise: the hadronic weight is the partonic one at sqrt(shat) = sqrt(tau S)
    times 2 |dtau/dx_8| (-ln tau) f(x1) f(x2), with ln tau on [ln tau_lo, ln tau_hi]
    and ln x1 = x_9 ln tau; the observable is the partonic one."""
    p = W.config("ww_had")["params"]
    S = p[6] ** 2
    rng = np.random.default_rng(5)
    for _ in range(20):
        x = rng.uniform(0.02, 0.98, 10)
        Llo, Lhi = math.log(150.0 ** 2 / S), 0.0
        L = Lhi + x[8] * (Llo - Lhi)
        tau = math.exp(L)
        x1 = math.exp(x[9] * L)
        pp = p.copy()
        pp[6] = math.sqrt(tau * S)
        part = oracle.integrand(W.WW_4L, pp, x[:8])
        ref = 2 * tau * (Lhi - Llo) * (-L) * pdf(x1) * pdf(tau / x1) * part
        assert abs(oracle.integrand(W.WW_HAD, p, x) / ref - 1) < 1e-12
        assert oracle.observable(W.WW_HAD, p, x) == oracle.observable(W.WW_4L, pp, x[:8])
