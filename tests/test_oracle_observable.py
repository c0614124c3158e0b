"""Pins for the oracle's observable histograms (CPU only).

A histogram bin of an observable is the integral of the same weight restricted
to the events whose observable falls in the bin, so every bin is estimated by
the same events and the same weights as the total (Sec. 2.1: the integrator
yields cross sections and distributions of kinematic variables; Sec. 3.2 shows
a di-jet mass distribution).  The pins: the bins add up to the integral and
their variances to its variance (exact identities), brute-force counting on a
constant integrand, closed forms for the e+e- angular distribution and the
Gaussian marginal, and quadrature for the Drell-Yan mass and W+ lepton p_T
spectra (the Jacobian peak, with the cuts integrated analytically).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

GL = {n: np.polynomial.legendre.leggauss(n) for n in (16, 24, 40)}


def gl01(n):
    x, w = GL[n]
    return 0.5 * (x + 1), 0.5 * w


def composite_vec(f, a, b, panels, n=16):
    x, w = GL[n]
    edges = np.linspace(a, b, panels + 1)
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        xm, xr = 0.5 * (hi + lo), 0.5 * (hi - lo)
        for xi, wi in zip(x, w):
            tot = tot + xr * wi * f(xm + xr * xi)
    return tot


def pdf(x, A=1.0, a=-0.5, b=3.0):
    return A * x ** a * (1 - x) ** b


def run(v, n_iter, n, refine=True):
    rs = []
    for _ in range(n_iter):
        rs.append(v.iterate(n))
        if refine:
            v.refine()
    return rs


def edges_of(nbins, lo, hi):
    return lo + (hi - lo) * np.arange(nbins + 1) / nbins


# ------------------------------------------------------------ identities ----
@pytest.mark.parametrize("name,nb,lo,hi", [("dy_z", 10, 81.0, 101.0),
                                          ("w_plus", 12, 10.0, 70.0),
                                          ("eemumu", 8, -1.0, 1.0),
                                          ("gauss4", 7, 0.2, 0.8)])
def test_bins_add_up_to_the_integral_and_its_variance(name, nb, lo, hi):
    """sum_b H_b = I_j, and, since an event lies in one bin only,
    var_j = sum_b var_b - (I_j^2 - sum_b H_b^2) / (N - 1) exactly."""
    c = W.config(name)
    v = oracle.Vegas(c["process"], c["ndim"], c["nbins"], c["seed"], c["alpha"], c["params"])
    v.set_observable(nb, lo, hi)
    N = 20_000
    for r in run(v, 3, N):
        pass
    last, err, _, _ = v.get_observable()
    I, var = r["I"], r["var"]
    assert abs(last.sum() - I) <= 1e-14 * abs(I)
    d, sums = v.get_hist()
    s2n = sums[1] / N / (N - 1)
    rhs = (err ** 2).sum() - (I * I - (last ** 2).sum()) / (N - 1)
    assert abs(var - rhs) <= 1e-10 * s2n


def test_counting_on_a_constant_integrand():
    """Genz corner peak with a = 0 is 1 everywhere and the uniform grid with 8 bins
    maps u to x exactly, so bin b holds (number of events with x_0 in b) / N,
    counted here from the random numbers alone; the integral's variance is 0, so
    the combination is the plain mean of the iterations and carries no error."""
    par = np.concatenate([[3.0], np.zeros(2), np.full(2, 0.5)])
    v = oracle.Vegas(W.GENZ, 2, 8, 5, 1.5, par)
    nb, lo, hi, N = 5, 0.1, 0.85, 3000
    v.set_observable(nb, lo, hi)
    hs = []
    for it in range(2):
        r = v.iterate(N)
        assert r["var"] == 0.0
        last, err, comb, cerr = v.get_observable()
        x0 = np.array([oracle.uniforms(5, it, i, 2)[0] for i in range(N)])
        k = np.where(x0 < lo, 0, np.where(x0 >= hi, nb + 1,
                     np.minimum(np.floor((x0 - lo) * (nb / (hi - lo))).astype(int) + 1, nb)))
        cnt = np.bincount(k, minlength=nb + 2)
        assert np.allclose(last * N, cnt, rtol=0, atol=1e-9)
        p = cnt / N
        assert np.allclose(err, np.sqrt(np.maximum(p - p * p, 0) / (N - 1)), rtol=1e-12, atol=1e-300)
        hs.append(last)
    assert np.allclose(comb, 0.5 * (hs[0] + hs[1]), rtol=1e-15, atol=0)
    assert np.all(cerr == 0.0)


def test_combination_uses_the_integral_weights_from_first():
    """Iterations before `first` are left out; the rest enter with the weights
    1 / var_j of the integral's combination, the errors in quadrature."""
    c = W.config("gauss4")
    v = oracle.Vegas(c["process"], c["ndim"], c["nbins"], c["seed"], c["alpha"], c["params"])
    v.set_observable(6, 0.3, 0.7, first=2)
    H, E, V = [], [], []
    for _ in range(5):
        r = v.iterate(4000)
        v.refine()
        last, err, comb, cerr = v.get_observable()
        H.append(last), E.append(err), V.append(r["var"])
    wj = 1 / np.array(V[2:])
    ref = (wj[:, None] * np.array(H[2:])).sum(0) / wj.sum()
    rerr = np.sqrt((wj[:, None] ** 2 * np.array(E[2:]) ** 2).sum(0)) / wj.sum()
    assert np.allclose(comb, ref, rtol=1e-13, atol=0)
    assert np.allclose(cerr, rerr, rtol=1e-12, atol=0)
    # the integral's own combination from the same iteration on
    assert abs(comb.sum() - v.result(first=2)["I"]) < 1e-13 * abs(comb.sum())


def test_set_observable_clears_and_validates():
    c = W.config("gauss4")
    v = oracle.Vegas(c["process"], c["ndim"], c["nbins"], c["seed"], c["alpha"], c["params"])
    with pytest.raises(RuntimeError):
        v.get_observable()                     # off
    for bad in [(-1, 0.0, 1.0), (255, 0.0, 1.0), (4, 1.0, 1.0), (4, 1.0, 0.0),
                (4, 0.0, math.inf), (4, math.nan, 1.0), (4, 0.0, 1e-310)]:
        with pytest.raises(ValueError):
            v.set_observable(*bad)
    v.set_observable(4, 0.0, 1.0)
    with pytest.raises(RuntimeError):
        v.get_observable()                     # no iteration yet
    v.iterate(1000)
    a = v.get_observable()
    v.set_observable(4, 0.0, 1.0)              # clears the combination
    with pytest.raises(RuntimeError):
        v.get_observable()
    v.iteration = 0
    v.iterate(1000)
    b = v.get_observable()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_nonfinite_events_enter_no_bin():
    par = np.concatenate([[9.0], np.ones(2), np.full(2, 0.5)])   # unknown family -> NaN
    v = oracle.Vegas(W.GENZ, 2, 10, 1, 1.5, par)
    v.set_observable(4, 0.0, 1.0)
    assert v.iterate(500)["n_nonfinite"] == 500
    last, err, _, _ = v.get_observable()
    assert np.all(last == 0) and np.all(err == 0)


# ------------------------------------------------------------ observables ---
def test_observable_definitions_pointwise():
    """x_0; cos(theta) = 2 x_1 - 1 of the e+e- map; the W+W- e+ nu mass equals the
    invariant mass of the e+ and nu momenta; the W+ lepton p_T at a fixed mass m
    (closed window) is (m/2) sin(theta*), theta* = arccos(2 x_2 - 1)."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        x = rng.uniform(0.01, 0.99, 8)
        assert oracle.observable(W.GAUSS, [0.5, 0.1], x[:3]) == x[0]
        assert oracle.observable(W.EEMUMU, W.phys_params(91.0), x[:2]) == 2 * x[0] - 1
        p = W.phys_params(500.0)
        mom, m2p, m2m, jac = oracle.ww_momenta(p, x)
        q = mom[0] + mom[1]
        mq = math.sqrt(q[0] ** 2 - q[1] ** 2 - q[2] ** 2 - q[3] ** 2)
        assert abs(oracle.observable(W.WW_4L, p, x) / mq - 1) < 1e-12
        pw = W.phys_params(13000.0, mlo=79.0, mhi=79.0)
        c = 2 * x[2] - 1
        ref = 39.5 * math.sqrt((1 - c) * (1 + c))
        assert abs(oracle.observable(W.W_PLUS, pw, x[:4]) - ref) <= 1e-13 * 39.5
        pd = W.config("dy_z")["params"]
        m = oracle.observable(W.DY_Z, pd, x[:3])
        assert 81.0 <= m <= 101.0


def test_eemumu_angular_bins_match_closed_form():
    """d sigma / d cos(theta) = (pi alpha^2 / 2s)(1 + c^2): bin [c1, c2) holds
    (3/8) [c + c^3/3] of the total 4 pi alpha^2 / (3 s)."""
    c = W.config("eemumu")
    p = c["params"]
    v = oracle.Vegas(c["process"], c["ndim"], c["nbins"], c["seed"], c["alpha"], p)
    nb = 8
    v.set_observable(nb, -1.0, 1.0, first=2)
    run(v, 6, 50_000)
    _, _, comb, cerr = v.get_observable()
    s = 91.0 ** 2
    tot = 4 * math.pi * (1 / 128) ** 2 / (3 * s) * p[15]
    e = edges_of(nb, -1.0, 1.0)
    F = lambda t: 0.375 * (t + t ** 3 / 3)
    ref = tot * (F(e[1:]) - F(e[:-1]))
    assert comb[0] == 0 and comb[-1] == 0
    assert np.all(np.abs(comb[1:-1] - ref) < 4 * cerr[1:-1]), (comb[1:-1] / ref - 1)
    assert np.all(cerr[1:-1] / ref < 1.5e-2)


def test_gaussian_marginal_bins_match_closed_form():
    """For the separable normalised Gaussian the x_0 bin [a, b) holds
    [Phi(b) - Phi(a)] times the other dimensions' integrals over [0, 1]."""
    c = W.config("gauss4")
    mu, sg = c["params"]
    v = oracle.Vegas(c["process"], c["ndim"], c["nbins"], c["seed"], c["alpha"], c["params"])
    nb, lo, hi = 6, 0.3, 0.75
    v.set_observable(nb, lo, hi, first=3)
    run(v, 8, 20_000)
    _, _, comb, cerr = v.get_observable()
    Phi = np.vectorize(lambda t: 0.5 * (1 + math.erf((t - mu) / (sg * math.sqrt(2)))))
    one = Phi(1.0) - Phi(0.0)
    e = np.concatenate([[0.0], edges_of(nb, lo, hi), [1.0]])
    ref = (Phi(e[1:]) - Phi(e[:-1])) * one ** 3
    assert np.all(np.abs(comb - ref) < 4 * cerr), (comb / ref - 1)
    assert np.all(cerr[1:-1] / ref[1:-1] < 3e-2)


def test_drell_yan_mass_bins_match_quadrature():
    """Bins of m_ll against 2 sum_q int dm^2/S int d ln x1 f(x1) f(tau/x1)
    sigmahat_q over each bin's m^2 range (sigmahat is pinned to the textbook
    photon and Z-peak forms elsewhere); the window 81 < m_ll < 101 leaves the
    under- and overflow bins empty."""
    c = W.config("dy_z")
    p = c["params"]
    S = p[6] ** 2
    v = oracle.Vegas(c["process"], c["ndim"], c["nbins"], c["seed"], c["alpha"], p)
    nb = 10
    v.set_observable(nb, 81.0, 101.0, first=2)
    run(v, 8, 300_000)
    _, _, comb, cerr = v.get_observable()
    assert comb[0] == 0 and comb[-1] == 0

    def inner(m2):
        tau = m2 / S
        L = math.log(tau)
        ys, ws = gl01(24)
        lum = sum(wy * (-L) * pdf(math.exp(y * L)) * pdf(tau / math.exp(y * L))
                  for y, wy in zip(ys, ws))
        return 2 * lum / S * (oracle.sigmahat_dy(p, m2, 0) + oracle.sigmahat_dy(p, m2, 1))

    e = edges_of(nb, 81.0, 101.0)
    ref = np.array([composite_vec(inner, a * a, b * b, 6) for a, b in zip(e[:-1], e[1:])]) * p[15]
    assert np.all(np.abs(comb[1:-1] - ref) < 4 * cerr[1:-1]), (comb[1:-1] / ref - 1)
    assert np.all(cerr[1:-1] / ref < 1e-2)


def w_pt_bins_reference(p, e):
    """Per-bin W+ cross section in lepton p_T bins [e_k, e_k+1) (last bin open),
    with the |eta| cut integrated analytically in c = cos(theta*):
    p_T^2 = (m^2/4)(1 - c^2), so p_T in [a, b) is c_b < |c| <= c_a with
    c_a = sqrt(1 - 4a^2/m^2) and c_b = sqrt(1 - 4b^2/m^2) (0 if 2b > m);
    the pseudorapidity cut is tanh(-eta - y) < c < tanh(eta - y)."""
    S = p[6] ** 2
    M, G = p[4], p[5]
    g2 = 4 * math.pi * p[0] / p[1]
    th = lambda c: c + c ** 3 / 3
    ys, ws = gl01(40)
    nb = len(e)

    def inner(m2):
        out = np.zeros(nb)
        tau = m2 / S
        L = math.log(tau)
        ca = [math.sqrt(1 - 4 * a * a / m2) if 4 * a * a < m2 else 0.0 for a in e] + [0.0]
        D = (m2 - M * M) ** 2 + (M * G) ** 2
        pref = g2 * g2 * m2 * m2 / (48 * D) / (32 * math.pi * m2) * 2
        for yy, wy in zip(ys, ws):
            l1 = yy * L
            x1, x2 = math.exp(l1), math.exp(L - l1)
            rap = 0.5 * math.log(x1 / x2)
            elo, ehi = math.tanh(-p[13] - rap), math.tanh(p[13] - rap)
            f = wy * (-L) * pdf(x1) * pdf(x2) * pref
            for k in range(nb):
                hi_c, lo_c = ca[k], ca[k + 1]
                for a, b in ((lo_c, hi_c), (-hi_c, -lo_c)):
                    lo, hi = max(a, elo), min(b, ehi)
                    if hi > lo:
                        out[k] += f * (th(hi) - th(lo))
        return out / S

    lo, hi = math.atan((p[10] ** 2 - M * M) / (M * G)), math.atan((S - M * M) / (M * G))
    return composite_vec(lambda r: inner(M * M + M * G * math.tan(r)) * M * G / math.cos(r) ** 2,
                         lo, hi, 200) * p[15]


def test_w_lepton_pt_bins_match_quadrature():
    """The p_T spectrum with its Jacobian peak at M_W / 2, against the
    quadrature above; below the 20 GeV cut the underflow bin is empty."""
    c = W.config("w_plus")
    p = c["params"]
    v = oracle.Vegas(c["process"], c["ndim"], c["nbins"], c["seed"], c["alpha"], p)
    nb, lo, hi = 8, 20.0, 52.0
    v.set_observable(nb, lo, hi, first=2)
    run(v, 8, 100_000)
    _, _, comb, cerr = v.get_observable()
    assert comb[0] == 0.0
    ref = w_pt_bins_reference(p, edges_of(nb, lo, hi))
    assert np.all(np.abs(comb[1:] - ref) < 4 * cerr[1:]), (comb[1:] / ref - 1)
    assert np.all(cerr[1:] / ref < 3e-2)
    # the peak: [36, 40), just below M_W / 2 = 40.2, where p_T -> m/2 piles up the
    # half of the resonance below M_W; the next bin needs m > 80 GeV
    assert np.argmax(comb[1:-1]) == 4 and comb[5] / comb[6] > 2.5
