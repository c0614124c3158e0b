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
