"""Pins for the flow oracle (CPU): spline identities, invertibility, the
log-determinant against a finite-difference Jacobian, normalisation of q, and
autograd gradients against central differences."""
import math

import numpy as np
import pytest
import torch

from oracle import flow as F


def test_zero_parameters_give_identity_spline():
    raw = torch.zeros(5, F.NPAR, dtype=torch.float64)
    x = torch.rand(5, dtype=torch.float64)
    y, ld = F.rqs_forward(x, raw)
    assert torch.allclose(y, x, atol=1e-15, rtol=0) and torch.allclose(ld, torch.zeros(5, dtype=torch.float64), atol=1e-14)


def test_spline_inverse_and_endpoints():
    g = torch.Generator().manual_seed(1)
    raw = torch.randn(2000, F.NPAR, generator=g, dtype=torch.float64) * 2
    x = torch.rand(2000, generator=g, dtype=torch.float64)
    y, ld = F.rqs_forward(x, raw)
    xb, ldb = F.rqs_inverse(y, raw)
    assert torch.max(torch.abs(xb - x)) < 1e-10
    assert torch.max(torch.abs(ldb - ld)) < 1e-8
    e0, _ = F.rqs_forward(torch.zeros(2000, dtype=torch.float64), raw)
    e1, _ = F.rqs_forward(torch.ones(2000, dtype=torch.float64), raw)
    assert torch.max(torch.abs(e0)) < 1e-15 and torch.max(torch.abs(e1 - 1)) < 1e-14
    # monotone, derivative = d/dx by central differences
    h = 1e-6
    xs = torch.clamp(x, 2 * h, 1 - 2 * h)
    yp, _ = F.rqs_forward(xs + h, raw)
    ym, _ = F.rqs_forward(xs - h, raw)
    _, ldx = F.rqs_forward(xs, raw)
    fd = (yp - ym) / (2 * h)
    same_bin = torch.abs(fd / torch.exp(ldx) - 1) < 1e-5
    assert same_bin.float().mean() > 0.99 and torch.all(fd > 0)


def test_flow_logdet_matches_jacobian_and_inverse():
    theta = F.init_params(3)
    g = torch.Generator().manual_seed(4)
    theta[:] += 0.05 * torch.randn(F.NPARAMS, generator=g, dtype=torch.float64)
    y = 0.1 + 0.8 * torch.rand(20, 8, generator=g, dtype=torch.float64)
    logq, z = F.log_density(y, theta)
    yb, logq_s = F.sample(z, theta)
    assert torch.max(torch.abs(yb - y)) < 1e-10
    assert torch.max(torch.abs(logq_s - logq)) < 1e-9
    for i in range(5):
        J = torch.autograd.functional.jacobian(lambda t: F.log_density(t[None], theta)[1][0], y[i])
        # central-difference Jacobian as an independent check of autograd's
        h = 1e-6
        Jfd = torch.zeros(8, 8, dtype=torch.float64)
        for d in range(8):
            e = torch.zeros(8, dtype=torch.float64)
            e[d] = h
            Jfd[:, d] = (F.log_density((y[i] + e)[None], theta)[1][0]
                         - F.log_density((y[i] - e)[None], theta)[1][0]) / (2 * h)
        assert torch.allclose(J, Jfd, atol=1e-6, rtol=1e-5)
        sign, lad = torch.linalg.slogdet(Jfd)
        assert sign > 0 and abs(lad - logq[i]) < 1e-6


def test_density_is_normalised():
    """E_uniform[q(y)] = 1 (q is a density on the unit cube), by Monte Carlo."""
    theta = F.init_params(5)
    g = torch.Generator().manual_seed(6)
    theta[:] += 0.01 * torch.randn(F.NPARAMS, generator=g, dtype=torch.float64)
    y = torch.rand(100_000, 8, generator=g, dtype=torch.float64)
    q = torch.exp(F.log_density(y, theta)[0])
    m, s = q.mean().item(), q.std().item() / math.sqrt(len(q))
    assert abs(m - 1) < 5 * s and s < 0.01


def test_loss_gradient_matches_central_differences():
    theta = F.init_params(7)
    g = torch.Generator().manual_seed(8)
    theta[:] += 0.05 * torch.randn(F.NPARAMS, generator=g, dtype=torch.float64)
    y = torch.rand(64, 8, generator=g, dtype=torch.float64)
    w = torch.rand(64, generator=g, dtype=torch.float64) ** 3
    L, grad = F.loss_and_grad(y, w, theta)
    idx = [0, 700, 5000, 20000, F.LAYER_SIZE - 1, 3 * F.LAYER_SIZE + 17000, F.NPARAMS - 5]
    for i in idx:
        h = 1e-6
        tp, tm = theta.clone(), theta.clone()
        tp[i] += h
        tm[i] -= h
        fd = (F.loss(y, w, tp) - F.loss(y, w, tm)) / (2 * h)
        assert abs(fd - grad[i]) < 1e-6 * max(1e-3, abs(grad[i])), (i, fd, grad[i])


def _gauss_exact(mu, sg, ndim):
    one = 0.5 * (math.erf((1 - mu) / (sg * math.sqrt(2))) - math.erf(-mu / (sg * math.sqrt(2))))
    return one ** ndim


def test_flow_iteration_unbiased_pulls_over_seeds():
    """A flow iteration estimates the integral without bias for any parameters:
    points z uniform from the oracle's counter stream, y = F^-1(z), weight f(y)/q(y)
    on the uniform grid (x = y), for a random flow (output scale 0.1) and the 8-dim
    Gaussian (mu 0.5, sigma 0.2, normalised per dimension on the real line).  Over
    24 seeds of 4,000 events the pulls against the erf closed form have mean within
    3/sqrt(24) of 0 and a spread between 0.6 and 1.5."""
    import oracle
    th = F.init_params(8)
    g = torch.Generator().manual_seed(108)
    for l in range(F.NLAYER):
        W1, b1, W2, b2, W3, b3 = F.unpack(th, l)
        W3.copy_(torch.randn(W3.shape, generator=g, dtype=torch.float64) * 0.1 / math.sqrt(F.HID))
        b3.copy_(torch.randn(b3.shape, generator=g, dtype=torch.float64) * 0.1)
    mu, sg, n = 0.5, 0.2, 4000
    exact = _gauss_exact(mu, sg, 8)
    pulls = []
    for seed in range(1, 25):
        z = torch.tensor(np.array([oracle.uniforms(seed, 0, i, 8) for i in range(n)]))
        y, lq = F.sample(z, th)
        f = torch.exp(-((y - mu) ** 2).sum(1) / (2 * sg * sg)) / (sg * math.sqrt(2 * math.pi)) ** 8
        w = (f * torch.exp(-lq)).numpy()
        I, var = w.mean(), w.var(ddof=1) / n
        pulls.append((I - exact) / math.sqrt(var))
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 3 / math.sqrt(len(pulls)), pulls
    assert 0.6 < pulls.std(ddof=1) < 1.5, pulls
