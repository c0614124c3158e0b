"""GPU parity of the observable histograms against the oracle, through the C ABI.

Bars: per bin, the iteration's value and error within 1e-10 relative of the
oracle's (with a floor of 1e-12 of the largest bin, for bins that cancel), the
same empty bins, and the combination likewise; byte-identical histograms for
every launch configuration and every fold (two-pass, fused, re-fold).
"""
import struct

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-10

GAUSS_MAX = dict(process=W.GAUSS, ndim=16, nbins=255, seed=5, alpha=1.5, params=[0.5, 0.3])


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_06182_amd as P
    P.load()
    return P


def genz(fam):
    return dict(process=W.GENZ, ndim=5, nbins=40, seed=9, alpha=1.5,
                params=W.genz_params(fam, 5, seed=fam, difficulty=6.0))


# (name, config, (bins, lo, hi)): ranges that leave the under- and overflow bins in use
CASES = [("gauss4", W.config("gauss4"), (20, 0.3, 0.8)),
         ("eemumu", W.config("eemumu"), (16, -0.9, 0.95)),
         ("dy_z", W.config("dy_z"), (40, 85.0, 97.0)),
         ("w_plus", W.config("w_plus"), (50, 20.0, 70.0)),
         ("ww_4l", W.config("ww_4l"), (60, 60.0, 100.0)),
         ("genz1", genz(1), (10, 0.1, 0.9)),
         ("genz6", genz(6), (7, 0.05, 0.6)),
         ("gauss16x255", GAUSS_MAX, (254, 0.0, 1.0))]


def close(a, b, tag):
    a, b = np.asarray(a), np.asarray(b)
    assert np.array_equal(a == 0, b == 0), f"{tag}: empty bins differ"
    floor = 1e-12 * np.max(np.abs(b))
    bad = np.abs(a - b) > REL * np.abs(b) + floor
    assert not bad.any(), f"{tag}: {int(bad.sum())} bins off, e.g. {a[bad][:3]} vs {b[bad][:3]}"


def pair(P, cfg, n, obs, first):
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"], max_events=n)
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    g.set_observable(*obs, first=first)
    o.set_observable(*obs, first=first)
    return g, o


@pytest.mark.parametrize("name,cfg,obs", CASES, ids=[c[0] for c in CASES])
def test_observable_matches_oracle(P, name, cfg, obs):
    """Three iterations (two-pass fold, then fused where the digits fit one block's
    LDS) at a size spanning many blocks and a ragged tail, the grid injected into
    the oracle; the combination starts at iteration 1."""
    n = 6007 if cfg["process"] != W.WW_4L else 4099
    g, o = pair(P, cfg, n, obs, first=1)
    for it in range(3):
        o.set_grid(g.get_grid())
        o.iteration = it
        rg = g.iterate(n)
        o.iterate(n)
        G, O = g.get_observable(), o.get_observable()
        for k, what in enumerate(("value", "error", "combination", "combined error")):
            close(G[k], O[k], f"{name} it{it} {what}")
        # the bins add up to the iteration's estimate
        assert abs(G[0].sum() - rg["I"]) <= 1e-13 * np.sum(np.abs(G[0]))
        g.refine()
        o.refine()
    res = g.result(first=1)
    assert abs(G[2].sum() - res["I"]) <= 1e-12 * np.sum(np.abs(G[2]))


def run_schedule(P, cfg, n, iters, obs, **kw):
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"], max_events=n, **kw)
    g.set_observable(*obs, first=1)
    blobs = []
    for _ in range(iters):
        g.iterate(n)
        blobs.append(b"".join(x.tobytes() for x in g.get_observable()))
        g.refine()
    return b"".join(blobs)


@pytest.mark.parametrize("name", ["w_plus", "ww_4l", "gauss16x255"])
def test_observable_bit_identical_across_launch_configurations(P, name):
    cfg = GAUSS_MAX if name == "gauss16x255" else W.config(name)
    obs = [c[2] for c in CASES if c[0] == name][0]
    n = 50_021 if name != "ww_4l" else 20_011
    ref = run_schedule(P, cfg, n, 3, obs)
    for wpb, mb in ((1, 0), (2, 3), (8, 0), (16, 5), (4, 97)):
        assert run_schedule(P, cfg, n, 3, obs, waves_per_block=wpb, max_blocks=mb) == ref, (wpb, mb)


def _with_scale(blob, valid, e1):
    off = struct.calcsize("<Q3iIQ")
    return blob[:off] + struct.pack("<4i", valid, e1, 2 * e1, 0) + blob[off + 16:]


def test_observable_identical_for_every_fold(P):
    """Iteration 1 of the same run folded three ways: two-pass (no stored scale), and
    the re-fold forced by a stored scale the weights overflow or lie 2^100 below:
    the same integers, so the same bits; the fused fold agrees to the truncation of
    each event's digits."""
    cfg = W.config("w_plus")
    n = 50_000
    obs = (50, 20.0, 70.0)

    def mk():
        g = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
        g.set_observable(*obs, first=0)
        return g

    a = mk()
    a.iterate(n)
    a.refine()
    blob = a.get_state()
    e1 = struct.unpack_from("<2i", blob, struct.calcsize("<Q3iIQ"))[1]
    a.set_state(blob)                      # clears the combination, keeps the binning
    with pytest.raises(P.VegasError):
        a.get_observable()
    assert a.iterate(n)["fold"] == 1
    fused = a.get_observable()
    runs = {}
    for tag, v, e in (("two-pass", 0, 0), ("overflow", 1, e1 - 30), ("far above", 1, e1 + 100)):
        b = mk()
        b.set_state(_with_scale(blob, v, e))
        assert b.iterate(n)["fold"] == (0 if v == 0 else 2), tag
        runs[tag] = b.get_observable()
    for tag in ("overflow", "far above"):
        for x, y in zip(runs[tag], runs["two-pass"]):
            assert np.array_equal(x, y), tag
    m = runs["two-pass"][0] != 0
    assert np.max(np.abs(fused[0][m] / runs["two-pass"][0][m] - 1)) < 1e-13


def test_full_size_w_plus_against_oracle(P):
    """The bench workload's size (10^6 events, 100 bins per dimension) with a 50-bin
    p_T histogram: every bin against the oracle, grid injected, both folds."""
    cfg = W.config("w_plus")
    n = cfg["n_events"]
    g, o = pair(P, cfg, n, (50, 20.0, 70.0), first=0)
    for it in range(2):
        o.set_grid(g.get_grid())
        o.iteration = it
        g.iterate(n)
        o.iterate(n)
        G, O = g.get_observable(), o.get_observable()
        for k in range(4):
            close(G[k], O[k], f"w_plus 1e6 it{it} output {k}")
        g.refine()
        o.refine()


def test_full_size_ww_properties(P):
    """10^7 W+W- events (beyond what the oracle redoes in a test): the bins add up
    to the integral, their variances to its variance, and the result does not
    depend on the launch configuration."""
    cfg = W.config("ww_4l")
    n = cfg["n_events"]
    outs = []
    for kw in ({}, dict(waves_per_block=2, max_blocks=300)):
        g = P.Integrator(cfg["process"], 8, 100, 1, 1.5, cfg["params"], max_events=n, **kw)
        g.set_observable(60, 60.0, 100.0, first=0)
        for it in range(2):
            r = g.iterate(n)
            g.refine()
        H, E, C, CE = g.get_observable()
        d, sums = g.get_hist()
        assert abs(H.sum() - r["I"]) <= 1e-13 * r["I"]
        s2n = sums[1] / n / (n - 1)
        rhs = (E ** 2).sum() - (r["I"] ** 2 - (H ** 2).sum()) / (n - 1)
        assert abs(r["var"] - rhs) <= 1e-9 * s2n
        outs.append(b"".join(x.tobytes() for x in (H, E, C, CE)))
        g.close()
    assert outs[0] == outs[1]


def test_observable_api_errors(P):
    cfg = W.config("dy_z")
    g = P.Integrator(cfg["process"], 3, 50, 1, 1.5, cfg["params"], max_events=1000)
    with pytest.raises(P.VegasError):
        g.get_observable()                             # off
    for bad in [(-1, 0.0, 1.0), (255, 0.0, 1.0), (4, 1.0, 1.0), (4, 2.0, 1.0),
                (4, 0.0, float("inf")), (4, float("nan"), 1.0), (4, 0.0, 1e-310)]:
        with pytest.raises(P.VegasError):
            g.set_observable(*bad)
    with pytest.raises(P.VegasError):
        g.set_observable(4, 0.0, 1.0, first=-1)
    g.set_observable(4, 81.0, 101.0)
    with pytest.raises(P.VegasError):
        g.get_observable()                             # no iteration yet
    g.iterate(1000)
    H = g.get_observable()[0]
    assert H[0] == 0 and H[-1] == 0 and np.all(H[1:-1] > 0)
    g.set_observable(0)                                # off again
    with pytest.raises(P.VegasError):
        g.get_observable()
    r = g.iterate(1000)                                # the plain path still runs
    assert r["n_events"] == 1000
