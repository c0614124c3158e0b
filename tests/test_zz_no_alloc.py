"""The allocation-free adjoint (vegas_grad_noalloc) against vegas_grad, through the
C ABI: the same kernels with the partials in the library's static scratch instead
of memory it allocates, so the results must be the same bits.  Two calls in a row,
the second with a smaller input (fewer points and events), each checked against
vegas_grad on the same inputs; a request beyond the scratch is refused with
VEGAS_ETOOBIG, and the device memory in use does not change across the calls."""
import numpy as np
import pytest

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
    return P, g, torch


def test_noalloc_equals_grad_twice_then_smaller(setup):
    P, g, torch = setup
    theta_all = torch.tensor(W.adjoint_points(64), device="cuda")
    # the largest inputs the scratch holds at B = 64, then a smaller call reusing it
    for B, n in ((64, 300_001), (17, 40_003)):
        theta = theta_all[:B].contiguous()
        sig = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
        dsig = torch.full((B, 5), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        g.grad_noalloc(theta, sig, dsig, n, 5)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        ref_s, ref_d = g.grad(theta, n, 5)
        torch.cuda.synchronize()
        assert torch.equal(sig, ref_s), (B, n)
        assert torch.equal(dsig, ref_d), (B, n)
        assert torch.isfinite(sig).all() and torch.isfinite(dsig).all()


def test_noalloc_refuses_beyond_scratch(setup):
    P, g, torch = setup
    B = 64
    theta = torch.tensor(W.adjoint_points(B), device="cuda")
    sig = torch.empty(B, dtype=torch.float64, device="cuda")
    dsig = torch.empty(B, 5, dtype=torch.float64, device="cuda")
    # T + ceil(T / 256) tiles of 6 B doubles must fit: 3.6e5 events at B = 64 do not
    with pytest.raises(P.VegasError) as e:
        g.grad_noalloc(theta, sig, dsig, 360_000, 5)
    assert e.value.status == P.vegas.ETOOBIG
    with pytest.raises(P.VegasError):
        g.grad_noalloc(theta, sig, dsig, 0, 5)       # the same argument checks as vegas_grad
