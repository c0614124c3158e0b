"""Learned proposal on the GPU against the flow oracle, and as a VEGAS proposal.

Parameters are drawn in float64 and rounded to binary32 before both sides see
them, so the two sides start from identical parameters.  The oracle is run
with bfloat16 emulation (the operands of the two 128-wide products rounded as
the matrix-core path rounds them) and without; the bars are stated per test.
"""
import math

import numpy as np
import pytest

import oracle.flow as OF
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_06182_amd as P
    return P, torch


def random_theta(torch, seed, out_scale=0.3):
    """A non-identity flow: He-uniform hidden layers and an output layer of scale out_scale."""
    th = OF.init_params(seed)
    g = torch.Generator().manual_seed(seed + 100)
    for l in range(OF.NLAYER):
        W1, b1, W2, b2, W3, b3 = OF.unpack(th, l)
        W3.copy_(torch.randn(W3.shape, generator=g, dtype=torch.float64) * out_scale / math.sqrt(OF.HID))
        b3.copy_(torch.randn(b3.shape, generator=g, dtype=torch.float64) * out_scale)
        b1.copy_(torch.randn(b1.shape, generator=g, dtype=torch.float64) * 0.1)
        b2.copy_(torch.randn(b2.shape, generator=g, dtype=torch.float64) * 0.1)
    return th.to(torch.float32).to(torch.float64)


def points(torch, n, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.rand(n, 8, generator=g, dtype=torch.float64).to(torch.float32)


def assert_rounding_noise(d, what):
    """Bars for |library - emulating oracle| on log q or y.  The library accumulates
    in binary32 (relative error ~1e-6 on each pre-activation), which now and then
    sends a value to the other neighbour when it is rounded (bfloat16 activations,
    2^-8 relative; binary16 spline parameters, 2^-11) and so moves the output by far
    more than the accumulation error itself.  Pushing relative noise of 1e-6 through
    the emulating oracle with the test's parameters (output scale 0.3) gives median
    1.1e-5 to 1.4e-5, 90th percentile 5e-4 to 7e-4, mean 3e-4 and maximum 1.4e-2
    over 1000 points; the bars leave room above those (and for the fast
    single-precision exp and log of the splines).  A wrong operand layout or index
    moves the median to O(1)."""
    q50, q90 = np.quantile(d, [0.5, 0.9])
    assert q50 <= 5e-5 and q90 <= 2e-3 and d.mean() <= 1e-3 and d.max() <= 5e-2, \
        (what, q50, q90, d.mean(), d.max())


def test_identity_initialisation(env):
    """Zero output layer: every spline is the identity (equal bins, unit derivatives)."""
    P, torch = env
    f = P.Flow(max_batch=1000, seed=5)
    y = points(torch, 1000, 1)
    lq = f.density(y.cuda()).cpu()
    assert lq.abs().max().item() <= 1e-5
    ys, lqs = f.sample(y.cuda())
    assert (ys.cpu() - y).abs().max().item() <= 1e-6
    assert lqs.abs().max().item() <= 1e-5
    theta = f.get_params().cpu()
    assert theta.shape[0] == OF.NPARAMS
    for l in range(OF.NLAYER):
        W1, b1, W2, b2, W3, b3 = OF.unpack(theta, l)
        assert W3.abs().max() == 0 and b3.abs().max() == 0
        assert 0 < W1.abs().max() <= math.sqrt(6 / 4) and 0 < W2.abs().max() <= math.sqrt(6 / 128)


def test_density_matches_oracle(env, capsys):
    """log q over 1000 points (31 full tiles of 32 and a ragged one) against the
    bf16-emulating oracle (bars of assert_rounding_noise); against the unrounded
    oracle, bfloat16 operands (2^-9 relative each, 128-term sums) leave mean |d| <= 2e-2."""
    P, torch = env
    theta = random_theta(torch, 3)
    f = P.Flow(max_batch=1000)
    f.set_params(theta)
    y = points(torch, 1000, 2)
    lq = f.density(y.cuda()).cpu().to(torch.float64)
    lo_e, _ = OF.log_density(y.to(torch.float64), theta, bf16_emulation=True)
    lo, _ = OF.log_density(y.to(torch.float64), theta)
    d_e = (lq - lo_e).abs()
    d = (lq - lo).abs()
    with capsys.disabled():
        print(f"\n  flow log q: |gpu - oracle(bf16)| mean {d_e.mean():.2e} max {d_e.max():.2e}; "
              f"|gpu - oracle(fp64)| mean {d.mean():.2e} max {d.max():.2e}; spread of log q {lo.std():.2f}")
    assert lo.std() > 1.0           # the flow is far from the identity
    assert_rounding_noise(d_e.numpy(), "log q")
    assert d.mean() <= 2e-2


def test_sampling_inverts_density(env):
    """z -> (y, log q) then log q(y) by the density direction (the conditioning
    inputs of the two directions differ by the binary32 inversion, so the same
    rounding-noise bars apply); and y, log q against the oracle's sampling
    direction (bf16 emulation)."""
    P, torch = env
    theta = random_theta(torch, 4)
    f = P.Flow(max_batch=777)
    f.set_params(theta)
    z = points(torch, 777, 3)
    y, lqs = f.sample(z.cuda())
    lqd = f.density(y)
    assert torch.all((y >= 0) & (y <= 1))
    assert_rounding_noise((lqs - lqd).abs().cpu().numpy(), "round trip")
    yo, lqo = OF.sample(z.to(torch.float64), theta, bf16_emulation=True)
    assert_rounding_noise((y.cpu().to(torch.float64) - yo).abs().numpy().ravel(), "y")
    assert_rounding_noise((lqs.cpu().to(torch.float64) - lqo).abs().numpy(), "sample log q")


def test_batch_and_position_invariance(env):
    """Every event's sampling and density are computed on their own: the first k events
    of a batch give the same bits alone (k = 1, 3, 63, 64, 65, 130: a lone event,
    partial, whole and ragged 64-event tiles), and a permuted batch the permuted bits,
    so neither the tile an event lands in nor its row there, nor the padding rows of a
    ragged tile, changes anything."""
    P, torch = env
    theta = random_theta(torch, 12)
    f = P.Flow(max_batch=1000)
    f.set_params(theta)
    z = points(torch, 1000, 13).cuda()
    y, lq = f.sample(z)
    for k in (1, 3, 63, 64, 65, 130):
        yk, lqk = f.sample(z[:k])
        assert torch.equal(yk, y[:k]) and torch.equal(lqk, lq[:k]), k
    perm = torch.randperm(1000, generator=torch.Generator().manual_seed(3)).cuda()
    yp, lqp = f.sample(z[perm])
    assert torch.equal(yp, y[perm]) and torch.equal(lqp, lq[perm])
    d = f.density(y)
    for k in (1, 65):
        assert torch.equal(f.density(y[:k]), d[:k]), k
    assert torch.equal(f.density(y[perm]), d[perm])


def test_loss_and_gradient_match_oracle(env, capsys):
    """Loss and all 248424 gradient entries on 600 weighted points.  The backward
    path rounds the gradients of the spline parameters and of h2 to bfloat16 before
    the two transposed products (as the forward rounds activations), so each
    parameter tensor's gradient is compared by relative L2 error (<= 2e-2) and the
    loss to 1e-4 relative, against the bf16-emulating oracle (autograd, float64)."""
    P, torch = env
    theta = random_theta(torch, 6)
    f = P.Flow(max_batch=600)
    f.set_params(theta)
    y = points(torch, 600, 4)
    g = torch.Generator().manual_seed(9)
    w = torch.exp(torch.randn(600, generator=g, dtype=torch.float64))
    loss, grad = f.loss_grad(y.cuda(), w.cuda())
    grad = grad.cpu().to(torch.float64)
    lo, go = OF.loss_and_grad(y.to(torch.float64), w, theta, bf16_emulation=True)
    assert abs(loss / lo.item() - 1) <= 1e-4, (loss, lo.item())
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    worst = 0.0
    for l in range(OF.NLAYER):
        gg, gr = OF.unpack(grad, l), OF.unpack(go, l)
        for nm, a, b in zip(names, gg, gr):
            rel = ((a - b).norm() / b.norm()).item()
            worst = max(worst, rel)
            assert rel <= 2e-2, (l, nm, rel)
    with capsys.disabled():
        print(f"\n  flow gradient: worst per-tensor relative L2 error {worst:.2e}; loss {loss:.6f} vs {lo.item():.6f}")


def test_loss_and_gradient_match_plain_fp64_oracle(env, capsys):
    """Loss and gradient against the plain float64 oracle (no rounding emulation).
    The matrix-core products take bfloat16 operands (8 significant bits), and on
    this case those roundings alone move the gradient by 4-7 % in relative L2 per
    tensor (the oracle with its bfloat16 emulation against itself without:
    2.4e-2 to 6.8e-2; the binary16 storage of the spline parameters adds 0.3 %),
    so the bar on each tensor is 0.12 relative L2, the whole gradient must point the
    same way (cosine >= 0.995), and the library's distance to the plain oracle may
    not exceed 1.25 x that of the emulating oracle (the library is as close to
    exact arithmetic as bfloat16 operands allow).  The loss to 1e-3 relative."""
    P, torch = env
    theta = random_theta(torch, 6)
    f = P.Flow(max_batch=600)
    f.set_params(theta)
    y = points(torch, 600, 4)
    g = torch.Generator().manual_seed(9)
    w = torch.exp(torch.randn(600, generator=g, dtype=torch.float64))
    loss, grad = f.loss_grad(y.cuda(), w.cuda())
    grad = grad.cpu().to(torch.float64)
    lp, gp = OF.loss_and_grad(y.to(torch.float64), w, theta, bf16_emulation=False)
    _, ge = OF.loss_and_grad(y.to(torch.float64), w, theta, bf16_emulation=True)
    assert abs(loss / lp.item() - 1) <= 1e-3, (loss, lp.item())
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    worst = 0.0
    for l in range(OF.NLAYER):
        for nm, a, b in zip(names, OF.unpack(grad, l), OF.unpack(gp, l)):
            rel = ((a - b).norm() / b.norm()).item()
            worst = max(worst, rel)
            assert rel <= 0.12, (l, nm, rel)
    cos = (grad @ gp / (grad.norm() * gp.norm())).item()
    d_lib = ((grad - gp).norm() / gp.norm()).item()
    d_emu = ((ge - gp).norm() / gp.norm()).item()
    with capsys.disabled():
        print(f"\n  flow gradient vs plain fp64 oracle: worst per-tensor relative L2 {worst:.2e}, whole "
              f"{d_lib:.2e} (emulating oracle {d_emu:.2e}), cosine {cos:.6f}; loss {loss:.6f} vs {lp.item():.6f}")
    assert cos >= 0.995
    assert d_lib <= 1.25 * d_emu, (d_lib, d_emu)


def test_gradient_descends_loss(env):
    """A step against the library's gradient lowers the oracle's loss (first order)."""
    P, torch = env
    theta = random_theta(torch, 7)
    f = P.Flow(max_batch=512)
    f.set_params(theta)
    y = points(torch, 512, 5)
    w = torch.ones(512, dtype=torch.float64)
    _, grad = f.loss_grad(y.cuda(), w.cuda())
    grad = grad.cpu().to(torch.float64)
    l0 = OF.loss(y.to(torch.float64), w, theta).item()
    eta = 1e-3 / grad.norm().item()
    l1 = OF.loss(y.to(torch.float64), w, theta - eta * grad).item()
    assert l1 < l0
    assert abs((l0 - l1) / (eta * grad.norm().item() ** 2) - 1) < 0.05


def _gauss_exact(mu, sg, ndim):
    one = 0.5 * (math.erf((1 - mu) / (sg * math.sqrt(2))) - math.erf(-mu / (sg * math.sqrt(2))))
    return one ** ndim


def test_export_is_the_iterations_points(env):
    import oracle
    P, torch = env
    g = P.Integrator(W.GAUSS, 8, 20, 11, 1.5, [0.5, 0.2], max_events=5000)
    g.iterate(5000)
    y, w = g.export(0, 5000)
    u = np.stack([oracle.uniforms(11, 0, i, 8) for i in (0, 1, 2, 1234, 4999)])
    assert np.array_equal(y.cpu().numpy()[[0, 1, 2, 1234, 4999]], u.astype(np.float32))
    assert np.array_equal(w.cpu().numpy(), g.get_weights(0, 5000, with_bins=False))
    y2, _ = g.export(4000, 1000)
    assert torch.equal(y2, y[4000:])


def test_identity_flow_iteration_equals_vegas(env):
    """The identity flow proposes the event's own point (rounded to binary32):
    the estimate differs from the VEGAS iteration of the same stream only by that rounding."""
    P, torch = env
    n = 100_000
    ga = P.Integrator(W.GAUSS, 8, 20, 21, 1.5, [0.5, 0.2], max_events=n)
    gb = P.Integrator(W.GAUSS, 8, 20, 21, 1.5, [0.5, 0.2], max_events=n)
    f = P.Flow(max_batch=16, max_sample=n)
    ra = ga.iterate(n)
    rb = gb.iterate_flow(f, n)
    assert rb["iteration"] == ra["iteration"] == 0
    assert abs(rb["I"] / ra["I"] - 1) < 1e-5
    assert abs(rb["var"] / ra["var"] - 1) < 1e-4


def test_flow_iteration_unbiased_gauss(env):
    """Any flow gives an unbiased estimate: a random (untrained) flow on the 8-dim
    Gaussian, 8 iterations of 2e5 events, combined pull against the closed form.
    The flow's output scale is 0.1 (log q spread 0.8, E[1/q] - 1 = 1.1 under the
    uniform density): a flow with a far wider log q (output scale 0.5 reaches
    log q = -27) has weights so heavy-tailed that variance estimates from 2e5
    events are meaningless, whatever the implementation."""
    P, torch = env
    n = 200_000
    g = P.Integrator(W.GAUSS, 8, 20, 31, 1.5, [0.5, 0.2], max_events=n)
    f = P.Flow(max_batch=16, max_sample=n)
    f.set_params(random_theta(torch, 8, out_scale=0.1))
    pulls = []
    for _ in range(8):
        r = g.iterate_flow(f, n)
        pulls.append((r["I"] - _gauss_exact(0.5, 0.2, 8)) / math.sqrt(r["var"]))
    res = g.result()
    assert res["n_iter"] == 8
    assert abs(res["I"] - _gauss_exact(0.5, 0.2, 8)) < 5 * res["sigma"], (res, pulls)
    assert max(abs(p) for p in pulls) < 5


def test_flow_errors(env):
    P, torch = env
    f = P.Flow(max_batch=64, max_sample=1000)
    g4 = P.Integrator(W.GAUSS, 4, 20, 1, 1.5, [0.5, 0.2], max_events=1000)
    with pytest.raises(P.VegasError):
        g4.iterate_flow(f, 1000)            # not 8-dimensional
    g8 = P.Integrator(W.GAUSS, 8, 20, 1, 1.5, [0.5, 0.2], max_events=2000)
    with pytest.raises(P.VegasError):
        g8.export(0, 10)                    # no iteration yet
    with pytest.raises(P.VegasError):
        g8.iterate_flow(f, 2000)            # above the flow's max_sample
    g8.iterate_flow(f, 1000)
    with pytest.raises(P.VegasError):
        g8.refine()                         # grid frozen under the flow
    with pytest.raises(P.VegasError):
        g8.export(0, 10)                    # last iteration used the flow
    with pytest.raises(P.VegasError):
        f.density(torch.zeros(65, 8, device="cuda"))   # above max_batch


def test_training_gain_on_ww(env, capsys):
    """The trained flow against plain VEGAS on the W+W- integrand: VEGAS grid
    converged (5 x 2e5), the flow trained on 2e5 of its weighted events (Adam,
    lr 1e-3, batch 4096, 10 epochs), then one iteration of 2e5 with each proposal
    on fresh streams.  Both estimates agree within errors; the flow lowers the
    per-event relative variance (the gain printed is the variance ratio)."""
    P, torch = env
    cfg = W.config("ww_4l")
    n = 200_000
    g = P.Integrator(cfg["process"], 8, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"], max_events=n)
    for _ in range(5):
        g.iterate(n)
        g.refine()
    rv = g.iterate(n)
    y, w = g.export(0, n)
    f = P.Flow(max_batch=4096, max_sample=n, seed=3)
    losses = P.train(f, y, w, epochs=10, batch=4096, lr=1e-3, log_every=50)
    rf = g.iterate_flow(f, n)
    rel_v = n * rv["var"] / rv["I"] ** 2
    rel_f = n * rf["var"] / rf["I"] ** 2
    diff = abs(rf["I"] - rv["I"]) / math.sqrt(rf["var"] + rv["var"])
    with capsys.disabled():
        print(f"\n  flow training: loss {losses[0][1]:.4f} -> {losses[-1][1]:.4f} over {losses[-1][0] + 1} steps; "
              f"per-event rel. variance VEGAS {rel_v:.4f} flow {rel_f:.4f} (gain {rel_v / rel_f:.2f}); "
              f"estimates differ by {diff:.2f} sigma")
    assert losses[-1][1] < losses[0][1]
    assert diff < 5
    assert rel_f < rel_v


def test_full_size_sampled_flow_iteration(env):
    """A flow iteration at its measured size (1e7 W+W- events, the benchmark's
    launch): for every 99991st event and the last 100, z is the binary32 of the
    counter-stream uniforms of (seed, iteration, event); Flow.sample(z) gives the
    y and log q the iteration used, and the oracle's grid map and integrand at
    that y give w = J f / q to 1e-12 (so the stream, the map and the weight are
    the oracle's); log q against the bf16-emulating flow oracle within the
    rounding-noise bars; I equal to the mean of all 1e7 weights."""
    import oracle
    P, torch = env
    cfg = W.config("ww_4l")
    n = cfg["n_events"]
    g = P.Integrator(cfg["process"], 8, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"], max_events=n)
    for _ in range(2):
        g.iterate(n)
        g.refine()
    theta = random_theta(torch, 5)
    f = P.Flow(max_batch=4096, max_sample=n, seed=1)
    f.set_params(theta)
    r = g.iterate_flow(f, n)
    it = r["iteration"]
    wg = g.get_weights(0, n, with_bins=False)
    idx = np.concatenate([np.arange(0, n - 100, 99_991), np.arange(n - 100, n)])
    z = torch.tensor(np.array([oracle.uniforms(cfg["seed"], it, int(i), 8) for i in idx])).to(torch.float32)
    y, lq = f.sample(z.cuda())
    y64, lq64 = y.cpu().to(torch.float64).numpy(), lq.cpu().to(torch.float64).numpy()
    o = oracle.Vegas(cfg["process"], 8, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
    o.set_grid(g.get_grid())
    wo = np.empty(len(idx))
    for k in range(len(idx)):
        x, J, _ = o.grid_map(np.clip(y64[k], 2.0 ** -40, 1.0 - 2.0 ** -40))
        wo[k] = J * oracle.integrand(W.WW_4L, cfg["params"], x) * math.exp(-lq64[k])
    assert np.all(wo > 0)
    rel = np.abs(wg[idx] - wo) / wo
    assert rel.max() <= 1e-12, rel.max()
    _, lqo = OF.sample(z.to(torch.float64), theta, bf16_emulation=True)
    assert_rounding_noise(np.abs(lq64 - lqo.numpy()), "log q at full size")
    assert abs(r["I"] - wg.sum() / n) <= 1e-12 * abs(r["I"])


def test_identity_flow_iteration_fills_the_observable(env):
    """The flow's event kernels with the observable histogram: with the identity flow
    the bins equal the VEGAS iteration's up to the binary32 rounding of the points,
    they add up to the flow iteration's estimate, and stratified sampling (which
    would place the points itself) is refused for flow iterations."""
    P, torch = env
    n = 100_000
    ga = P.Integrator(W.GAUSS, 8, 20, 21, 1.5, [0.5, 0.2], max_events=n)
    gb = P.Integrator(W.GAUSS, 8, 20, 21, 1.5, [0.5, 0.2], max_events=n)
    for g in (ga, gb):
        g.set_observable(10, 0.2, 0.8, first=0)
    f = P.Flow(max_batch=16, max_sample=n)
    ra = ga.iterate(n)
    rb = gb.iterate_flow(f, n)
    A, B = ga.get_observable()[0], gb.get_observable()[0]
    assert abs(B.sum() - rb["I"]) <= 1e-13 * np.sum(np.abs(B))
    assert np.all(np.abs(B - A) <= 1e-4 * np.abs(A) + 1e-12 * np.max(A)), (A, B)
    gb.set_strata(2)
    with pytest.raises(P.VegasError):
        gb.iterate_flow(f, n)


def gaussian_spline_theta(torch, mu, sg):
    """A flow set by hand (no training): layers 0 and 1 map each of their four
    coordinates by one fixed spline (zero weights W3, the spline in the bias b3) whose
    bins are equally wide and whose heights are the truncated Gaussian's probability
    per bin (floored at twice the minimum height), interior derivatives the mean of
    the neighbouring slopes; layers 2-5 are the identity.  Together they transform
    all eight coordinates, so q approximates the Gaussian's density."""
    th = OF.init_params(5)
    for l in range(OF.NLAYER):
        W1, b1, W2, b2, W3, b3 = OF.unpack(th, l)
        W3.zero_()
        b3.zero_()
    cdf = [0.5 * (1 + math.erf((k / OF.NB - mu) / (sg * math.sqrt(2)))) for k in range(OF.NB + 1)]
    H = np.diff(cdf)
    H = np.maximum(H / H.sum(), 2 * OF.EPS)
    H /= H.sum()
    hl = np.log((H - OF.EPS) / (1 - OF.NB * OF.EPS))
    slope = H * OF.NB
    d = 0.5 * (slope[:-1] + slope[1:])
    raw_d = np.log(np.expm1(d - OF.EPS)) - OF.DSHIFT
    raw = np.concatenate([np.zeros(OF.NB), hl, raw_d])
    for l in (0, 1):
        b3 = OF.unpack(th, l)[5]
        for j in range(4):
            b3[j * OF.NPAR:(j + 1) * OF.NPAR] = torch.tensor(raw)
    return th.to(torch.float32).to(torch.float64)


def test_choose_proposal_keeps_vegas_for_identity_flow(env, capsys):
    """Fallback rule: an untrained (identity) flow proposes the same points as the
    grid, so the per-event variances agree, while each flow event also runs the
    six-layer network: the rule keeps plain VEGAS (W+W-, grid adapted 4 x 2e5,
    pilot iterations of 2e5)."""
    P, torch = env
    cfg = W.config("ww_4l")
    n = 200_000
    g = P.Integrator(cfg["process"], 8, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"], max_events=n)
    for _ in range(4):
        g.iterate(n)
        g.refine()
    f = P.Flow(max_batch=16, max_sample=n, seed=3)
    c = P.choose_proposal(g, f, n)
    rv, rf = c["vegas"], c["flow"]
    relv = n * rv["var"] / rv["I"] ** 2
    relf = n * rf["var"] / rf["I"] ** 2
    with capsys.disabled():
        print(f"\n  choose_proposal (identity flow, W+W-): rel. variance VEGAS {relv:.4f} flow {relf:.4f}; "
              f"seconds VEGAS {c['vegas_s']:.2e} flow {c['flow_s']:.2e} -> use_flow={c['use_flow']}")
    assert abs(relf / relv - 1) < 0.2
    assert c["flow_s"] > c["vegas_s"]
    assert not c["use_flow"]


def test_choose_proposal_takes_flow_that_wins(env, capsys):
    """Fallback rule, the other way: on the 8-dim Gaussian (sigma 0.1) with the grid
    kept uniform, a flow whose splines follow the Gaussian (set by hand,
    gaussian_spline_theta) lowers the per-event relative variance by orders of
    magnitude, far more than its extra cost per event: the rule takes the flow.
    Both pilot estimates agree with the closed form (the flow's is unbiased)."""
    P, torch = env
    n = 200_000
    mu, sg = 0.5, 0.1
    g = P.Integrator(W.GAUSS, 8, 20, 41, 1.5, [mu, sg], max_events=n)
    f = P.Flow(max_batch=16, max_sample=n, seed=3)
    f.set_params(gaussian_spline_theta(torch, mu, sg))
    c = P.choose_proposal(g, f, n)
    rv, rf = c["vegas"], c["flow"]
    exact = _gauss_exact(mu, sg, 8)
    relv = n * rv["var"] / rv["I"] ** 2
    relf = n * rf["var"] / rf["I"] ** 2
    with capsys.disabled():
        print(f"\n  choose_proposal (Gaussian flow): rel. variance VEGAS {relv:.3g} flow {relf:.3g}; "
              f"cost VEGAS {c['vegas_cost']:.3g} flow {c['flow_cost']:.3g} -> use_flow={c['use_flow']}")
    assert relf * 100 < relv
    assert c["use_flow"]
    assert abs(rf["I"] - exact) < 5 * math.sqrt(rf["var"])
    assert abs(rv["I"] - exact) < 5 * math.sqrt(rv["var"])


def test_flow_iteration_pulls_over_seeds(env):
    """Unbiasedness over seeds: a random flow (output scale 0.1) on the 8-dim Gaussian,
    one iteration of 1e5 events for each of 24 seeds of the counter stream; the pulls
    (I - exact)/sigma have mean within 3/sqrt(24) of 0 and spread in [0.6, 1.5]."""
    P, torch = env
    n = 100_000
    theta = random_theta(torch, 8, out_scale=0.1)
    exact = _gauss_exact(0.5, 0.2, 8)
    f = P.Flow(max_batch=16, max_sample=n)
    f.set_params(theta)
    pulls = []
    for seed in range(101, 125):
        g = P.Integrator(W.GAUSS, 8, 20, seed, 1.5, [0.5, 0.2], max_events=n)
        r = g.iterate_flow(f, n)
        pulls.append((r["I"] - exact) / math.sqrt(r["var"]))
        g.close()
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 3 / math.sqrt(len(pulls)), pulls
    assert 0.6 < pulls.std(ddof=1) < 1.5, pulls
