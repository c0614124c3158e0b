"""GPU adjoint of the Drell-Yan estimator against the oracle and finite differences.

theta = (M_Z, Gamma_Z, sin^2 theta_W, pdf a, pdf b); 64 points nominal * (1 + 0.05 v),
v uniform in [-1,1]^5 (seed 2).  The grid is the Drell-Yan workload's grid after
its 5 iterations; the random stream is iteration 5's.  Bars: sigma within 1e-10
relative of the oracle; gradient within 1e-9 of the oracle's dual-number
gradient (relative, with a floor of 1e-12 sigma/|theta|); the adjoint within
1e-6 of Richardson-extrapolated central differences (h = 1e-5 relative) of the
same GPU estimator.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_06182_amd as P
    cfg = W.config("dy_z")
    g = P.Integrator(cfg["process"], 3, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"],
                     max_events=cfg["n_events"])
    for _ in range(cfg["n_iter"]):
        g.iterate(cfg["n_events"])
        g.refine()
    o = oracle.Vegas(cfg["process"], 3, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
    o.set_grid(g.get_grid())
    return P, g, o, torch


def test_sigma_and_gradient_match_oracle(setup):
    P, g, o, torch = setup
    theta = W.adjoint_points(64)
    n = 20011
    sig, ds = g.grad(torch.tensor(theta), n, 5)
    sig, ds = sig.cpu().numpy(), ds.cpu().numpy()
    for b in (0, 7, 31, 63):
        so, dso = o.dy_grad(5, n, theta[b])
        assert abs(sig[b] / so - 1) < 1e-10, (b, sig[b], so)
        floor = 1e-12 * so / np.abs(theta[b])
        assert np.all(np.abs(ds[b] - dso) <= 1e-9 * np.abs(dso) + floor), (b, ds[b], dso)


def test_nominal_point_equals_vegas_iteration(setup):
    """At the nominal parameters the adjoint's sigma is the iteration estimate I_j of
    the same stream and grid (the same events through the forward path)."""
    P, g, o, torch = setup
    nominal = np.array([[W.MZ, W.GZ, W.SW2_ONSHELL, -0.5, 3.0]])
    n = 10_000
    sig, _ = g.grad(torch.tensor(nominal), n, 5)
    o.iteration = 5
    ro = o.iterate(n)
    assert abs(sig.item() / ro["I"] - 1) < 1e-10


def test_adjoint_matches_central_differences(setup):
    P, g, o, torch = setup
    theta = W.adjoint_points(4, seed=11)
    n = 50_000
    _, ds = g.grad(torch.tensor(theta), n, 5)
    ds = ds.cpu().numpy()
    for k in range(5):
        def central(h):
            tp, tm = theta.copy(), theta.copy()
            tp[:, k] += h[:]
            tm[:, k] -= h[:]
            sp, _ = g.grad(torch.tensor(tp), n, 5)
            sm, _ = g.grad(torch.tensor(tm), n, 5)
            return (sp.cpu().numpy() - sm.cpu().numpy()) / (2 * h)
        h = 1e-5 * np.abs(theta[:, k])
        fd = (4 * central(h) - central(2 * h)) / 3
        sig, _ = g.grad(torch.tensor(theta), n, 5)
        scale = sig.cpu().numpy() / np.abs(theta[:, k])
        assert np.all(np.abs(fd - ds[:, k]) <= 1e-6 * np.abs(ds[:, k]) + 1e-9 * scale), (k, fd, ds[:, k])


def test_autograd_function(setup):
    P, g, o, torch = setup
    theta = torch.tensor(W.adjoint_points(64), device="cuda", requires_grad=True)
    n = 8192
    sigma = P.vegas_sigma(theta, g, n, 5)
    wts = torch.linspace(0.5, 1.5, 64, dtype=torch.float64, device="cuda")
    (sigma * wts).sum().backward()
    _, ds = g.grad(theta.detach(), n, 5)
    expect = (wts[:, None] * ds).cpu()
    assert torch.allclose(theta.grad.cpu(), expect, rtol=1e-15, atol=0)


def test_gradient_full_size_sampled(setup):
    """The C3 size: 64 points x 1e6 events; two points checked against the oracle."""
    P, g, o, torch = setup
    theta = W.adjoint_points(64)
    n = 1_000_000
    sig, ds = g.grad(torch.tensor(theta), n, 5)
    sig, ds = sig.cpu().numpy(), ds.cpu().numpy()
    assert np.all(np.isfinite(sig)) and np.all(np.isfinite(ds))
    for b in (3, 50):
        so, dso = o.dy_grad(5, n, theta[b])
        assert abs(sig[b] / so - 1) < 1e-10
        floor = 1e-12 * so / np.abs(theta[b])
        assert np.all(np.abs(ds[b] - dso) <= 1e-9 * np.abs(dso) + floor)


def test_invalid_arguments(setup):
    P, g, o, torch = setup
    with pytest.raises(P.VegasError):
        g.grad(torch.zeros(65, 5, dtype=torch.float64), 1000, 5)     # more than 64 points
    cfg = W.config("w_plus")
    gw = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=100)
    with pytest.raises(P.VegasError):
        gw.grad(torch.zeros(2, 5, dtype=torch.float64), 1000, 0)      # not Drell-Yan
