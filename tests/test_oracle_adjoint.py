"""Pins for the oracle's Drell-Yan parameter gradient (dual numbers), CPU only.

theta = (M_Z, Gamma_Z, sin^2 theta_W, pdf a, pdf b).  The estimator is the
VEGAS mean at a fixed grid and fixed random stream; the proposal (grid,
Breit-Wigner and tau mappings) stays at the nominal parameters, so only |M|^2
and the PDFs depend on theta.
"""
import numpy as np

import oracle
import workloads as W


def _state():
    cfg = W.config("dy_z")
    v = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    for _ in range(2):
        v.iterate(5000)
        v.refine()
    return v


def test_dual_value_equals_plain_weight_at_nominal():
    v = _state()
    theta = np.array([W.MZ, W.GZ, W.SW2_ONSHELL, -0.5, 3.0])
    w, _ = v.event_weights(7, 0, 200)
    wd = np.array([v.dy_weight_theta(7, i, theta) for i in range(200)])
    assert np.allclose(wd, w, rtol=1e-12, atol=0)


def test_dual_gradient_matches_central_differences():
    v = _state()
    theta = np.array([W.MZ, W.GZ, W.SW2_ONSHELL, -0.5, 3.0]) * np.array([1.01, 0.98, 1.03, 1.02, 0.97])
    n = 2000
    sig, ds = v.dy_grad(9, n, theta)
    def central(k, h):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fp = np.mean([v.dy_weight_theta(9, i, tp) for i in range(n)])
        fm = np.mean([v.dy_weight_theta(9, i, tm) for i in range(n)])
        return (fp - fm) / (2 * h)

    for k in range(5):
        h = 1e-5 * abs(theta[k])
        # Richardson combination of steps h and 2h removes the O(h^2) truncation
        fd = (4 * central(k, h) - central(k, 2 * h)) / 3
        scale = abs(sig) / abs(theta[k])
        assert abs(fd - ds[k]) < 1e-7 * abs(ds[k]) + 1e-9 * scale, (k, fd, ds[k])


def test_gradient_of_pdf_exponent_is_log_moment():
    """d/da of A x^a (1-x)^b is ln(x) times the PDF, so d sigma/d a is the
    weight-averaged ln(x1 x2) = ln(tau): a closed form for each event."""
    v = _state()
    theta = np.array([W.MZ, W.GZ, W.SW2_ONSHELL, -0.5, 3.0])
    n = 300
    w, _ = v.event_weights(3, 0, n)
    sig, ds = v.dy_grad(3, n, theta)
    # ln(x1 x2) = ln(m^2 / S); m^2 from the first mapped coordinate via the oracle's grid map
    p = W.config("dy_z")["params"]
    S = p[6] ** 2
    acc = 0.0
    for i in range(n):
        u = oracle.uniforms(1, 3, i, 3)
        x, J, b = v.grid_map(u)
        MG = W.MZ * W.GZ
        rlo = np.arctan((81.0 ** 2 - W.MZ ** 2) / MG)
        rhi = np.arctan((101.0 ** 2 - W.MZ ** 2) / MG)
        m2 = W.MZ ** 2 + MG * np.tan(rlo + x[0] * (rhi - rlo))
        acc += w[i] * np.log(m2 / S)
    assert abs(ds[3] / (acc / n) - 1) < 1e-11


def test_gradient_expectation_is_derivative_of_true_cross_section():
    """Averaged over independent random streams, the estimator's gradient is the
    derivative of the true cross section sigma(theta) (the proposal does not
    depend on theta, so the pathwise gradient is unbiased).  sigma(theta) here is
    the 2-D hadronic form int dm^2/S int d ln x1 f(x1) f(tau/x1) sigmahat, done by
    Gauss-Legendre in the Breit-Wigner variable, and its derivative by central
    differences; the agreement must hold within 4 standard errors.  The test is
    required to resolve each component to 5 % of max(|d sigma/d theta|,
    sigma/|theta|): the mass window is nearly symmetric about the Z peak, so
    d sigma/d M_Z nearly cancels and is resolved on the second scale only."""
    v = _state()
    p0 = W.config("dy_z")["params"]
    S = p0[6] ** 2
    theta = np.array([W.MZ, W.GZ, W.SW2_ONSHELL, -0.5, 3.0])
    slots = [2, 3, 1, 8, 9]          # positions of theta in the parameter vector
    x24, w24 = np.polynomial.legendre.leggauss(24)
    y24, v24 = 0.5 * (x24 + 1), 0.5 * w24
    x16, w16 = np.polynomial.legendre.leggauss(16)
    MG = W.MZ * W.GZ
    rlo = np.arctan((81.0 ** 2 - W.MZ ** 2) / MG)
    rhi = np.arctan((101.0 ** 2 - W.MZ ** 2) / MG)

    def sigma(th):
        p = p0.copy()
        p[slots] = th
        a, b = p[8], p[9]
        tot = 0.0
        edges = np.linspace(rlo, rhi, 25)
        for lo, hi in zip(edges[:-1], edges[1:]):
            for xi, wi in zip(x16, w16):
                r = 0.5 * (hi + lo) + 0.5 * (hi - lo) * xi
                m2 = W.MZ ** 2 + MG * np.tan(r)
                jac = MG / np.cos(r) ** 2 * 0.5 * (hi - lo) * wi
                tau = m2 / S
                L = np.log(tau)
                x1 = np.exp(y24 * L)
                x2 = tau / x1
                lum = np.sum(v24 * (-L) * x1 ** a * (1 - x1) ** b * x2 ** a * (1 - x2) ** b)
                tot += jac * 2 * lum / S * (oracle.sigmahat_dy(p, m2, 0) + oracle.sigmahat_dy(p, m2, 1))
        return tot * p[15]

    batches = [v.dy_grad(100 + k, 20_000, theta) for k in range(64)]
    sig = np.array([s for s, _ in batches])
    ds = np.array([d for _, d in batches])
    assert abs(sig.mean() - sigma(theta)) < 4 * sig.std(ddof=1) / np.sqrt(len(sig))
    mean, err = ds.mean(0), ds.std(0, ddof=1) / np.sqrt(len(ds))
    for k in range(5):
        h = 1e-4 * abs(theta[k])
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (sigma(tp) - sigma(tm)) / (2 * h)
        assert err[k] < 0.05 * max(abs(fd), sig.mean() / abs(theta[k])), (k, err[k], fd)
        assert abs(mean[k] - fd) < 4 * err[k], (k, mean[k], fd, err[k])
