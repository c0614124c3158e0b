"""GPU parity of the stratified sampling (Lepage's stratified + importance mode)
against the oracle, through the C ABI.

Bars as for the plain iteration: per-event weights within 1e-12, bins exact, the
iteration's integral and stratified variance within 1e-10 with the grid injected
into the oracle, the same event count, byte-identical results for every launch
configuration and for every fold.
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


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# (name, config, strata per axis, events asked for)
CASES = [("gauss4", W.config("gauss4"), 4, 6007),
         ("eemumu", W.config("eemumu"), 8, 6007),
         ("dy_z", W.config("dy_z"), 6, 6007),
         ("w_plus", W.config("w_plus"), 5, 6007),
         ("ww_4l", W.config("ww_4l"), 2, 4099),
         ("ww_had", W.config("ww_had"), 2, 4099),
         ("gauss16x255", GAUSS_MAX, 2, 131_101)]


def pair(P, cfg, n, m):
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"], max_events=n)
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
    g.set_strata(m)
    o.set_strata(m)
    return g, o


@pytest.mark.parametrize("name,cfg,m,n", CASES, ids=[c[0] for c in CASES])
def test_stratified_iterations_match_oracle(P, name, cfg, m, n):
    g, o = pair(P, cfg, n, m)
    H = m ** cfg["ndim"]
    used = H * (n // H)
    for it in range(3):
        o.set_grid(g.get_grid())
        o.iteration = it
        rg, ro = g.iterate(n), o.iterate(n)
        assert rg["n_events"] == ro["n_events"] == used
        wg, bg = g.get_weights(0, used)
        wo, bo = o.event_weights(it, 0, used)
        assert np.array_equal(bg, bo), f"{name} it{it}: bins"
        nz = wo != 0
        assert np.array_equal(wg != 0, nz), f"{name} it{it}: cut flips"
        assert np.all(np.abs(wg - wo) <= 1e-12 * np.abs(wo) + 1e-14 * np.mean(np.abs(wo))), name
        assert rel(rg["I"], ro["I"]) < REL, (name, it, rg, ro)
        assert rel(rg["var"], ro["var"]) < REL, (name, it, rg, ro)
        g.refine()
        o.refine()


def test_one_stratum_is_the_plain_iteration(P):
    cfg = W.config("w_plus")
    n = 50_000
    a = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
    b = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
    b.set_strata(1)
    for _ in range(3):
        ra, rb = a.iterate(n), b.iterate(n)
        assert ra["I"] == rb["I"] and rel(rb["var"], ra["var"]) < 1e-12
        a.refine()
        b.refine()


def run_schedule(P, cfg, n, m, **kw):
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"], max_events=n, **kw)
    g.set_strata(m)
    out = []
    for _ in range(3):
        r = g.iterate(n)
        out.append(np.array([r["I"], r["var"]]).tobytes() + g.get_grid().tobytes())
        g.refine()
    return b"".join(out)


@pytest.mark.parametrize("name,m", [("w_plus", 6), ("gauss16x255", 2)])
def test_stratified_bit_identical_across_launch_configurations(P, name, m):
    cfg = GAUSS_MAX if name == "gauss16x255" else W.config(name)
    n = 200_003 if name == "gauss16x255" else 50_021
    ref = run_schedule(P, cfg, n, m)
    for wpb, mb in ((1, 0), (2, 3), (8, 0), (16, 5), (4, 97)):
        assert run_schedule(P, cfg, n, m, waves_per_block=wpb, max_blocks=mb) == ref, (wpb, mb)


def test_stratified_variance_is_the_same_for_every_fold(P):
    """The hypercube fold reads the records, so the two-pass fold, the fused fold and
    both forced re-folds give the same variance bits."""
    cfg = W.config("w_plus")
    n = 50_000

    def mk():
        g = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
        g.set_strata(5)
        return g

    a = mk()
    a.iterate(n)
    a.refine()
    blob = a.get_state()
    off = struct.calcsize("<Q3iIQ")
    e1 = struct.unpack_from("<2i", blob, off)[1]
    r1 = a.iterate(n)
    assert r1["fold"] == 1
    for v, e in ((0, 0), (1, e1 - 30), (1, e1 + 100)):
        b = mk()
        b.set_state(blob[:off] + struct.pack("<4i", v, e, 2 * e, 0) + blob[off + 16:])
        r = b.iterate(n)
        assert r["fold"] == (0 if v == 0 else 2)
        assert r["var"] == r1["var"] and abs(r["I"] / r1["I"] - 1) < 1e-15


def test_full_size_w_plus_against_oracle(P):
    """10^6 events in 10^4 hypercubes (10 strata per axis, 100 events each), the
    bench workload's size: integral and stratified variance against the oracle."""
    cfg = W.config("w_plus")
    n = cfg["n_events"]
    g, o = pair(P, cfg, n, 10)
    for it in range(2):
        o.set_grid(g.get_grid())
        o.iteration = it
        rg, ro = g.iterate(n), o.iterate(n)
        assert rg["n_events"] == ro["n_events"] == n
        assert rel(rg["I"], ro["I"]) < REL and rel(rg["var"], ro["var"]) < REL, (it, rg, ro)
        g.refine()
        o.refine()


def test_strata_refusals(P):
    cfg = W.config("gauss4")
    g = P.Integrator(cfg["process"], 4, 50, 7, 1.5, cfg["params"], max_events=2000)
    with pytest.raises(P.VegasError):
        g.set_strata(-1)
    with pytest.raises(P.VegasError):
        g.set_strata(300)                    # 300^4 hypercubes
    g.set_strata(5)                          # 625 hypercubes
    with pytest.raises(P.VegasError):
        g.iterate(1249)
    assert g.iterate(1250)["n_events"] == 1250
    assert g.iterate(1999)["n_events"] == 1875
    g.set_strata(0)
    assert g.iterate(1249)["n_events"] == 1249


@pytest.mark.parametrize("name,m,obs", [("w_plus", 5, (50, 20.0, 70.0)), ("ww_4l", 2, (60, 60.0, 100.0))])
def test_stratified_with_observable_matches_oracle(P, name, m, obs):
    """Both switches at once (the event kernels with the observable and the stratified
    placement): weights, integral, stratified variance and every observable bin
    against the oracle; the bins combine with the stratified var_j's weights."""
    cfg = W.config(name)
    n = 6007 if name == "w_plus" else 4099
    g, o = pair(P, cfg, n, m)
    g.set_observable(*obs, first=1)
    o.set_observable(*obs, first=1)
    used = m ** cfg["ndim"] * (n // m ** cfg["ndim"])
    for it in range(3):
        o.set_grid(g.get_grid())
        o.iteration = it
        rg, ro = g.iterate(n), o.iterate(n)
        assert rg["n_events"] == ro["n_events"] == used
        assert rel(rg["I"], ro["I"]) < REL and rel(rg["var"], ro["var"]) < REL, (it, rg, ro)
        G, O = g.get_observable(), o.get_observable()
        for k in range(4):
            a, b = G[k], O[k]
            assert np.array_equal(a == 0, b == 0)
            assert np.all(np.abs(a - b) <= REL * np.abs(b) + 1e-12 * np.max(np.abs(b))), (it, k)
        g.refine()
        o.refine()


def test_stratified_checkpoint_resume_is_bit_identical(P):
    cfg = W.config("w_plus")
    n = 40_000
    mk = lambda: P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
    a = mk()
    a.set_strata(6)
    for _ in range(2):
        a.iterate(n)
        a.refine()
    blob = a.get_state()
    for _ in range(2):
        a.iterate(n)
        a.refine()
    b = mk()
    b.set_strata(6)
    b.set_state(blob)
    for _ in range(2):
        b.iterate(n)
        b.refine()
    assert a.result() == b.result()
    assert np.array_equal(a.get_grid(), b.get_grid())


ADAPT = [("gauss4", W.config("gauss4"), 4, 6007), ("w_plus", W.config("w_plus"), 5, 6007),
         ("ww_4l", W.config("ww_4l"), 2, 4099)]


@pytest.mark.parametrize("name,cfg,m,n", ADAPT, ids=[c[0] for c in ADAPT])
def test_adaptive_strata_match_oracle(P, name, cfg, m, n):
    """beta = 1: each iteration the GPU's counts agree with the oracle's own rule
    (from the oracle's sigma_h of the same events; a count may differ by one where
    binary64 rounding puts (n - 2H) p_h / sum p at an integer), then, with those
    counts injected into the oracle and the grid injected, the scaled weights,
    the integral and the variance agree to the usual bars."""
    g, o = pair(P, cfg, n, m)
    g.set_strata_beta(1.0)
    o.set_strata_beta(1.0)
    for it in range(4):
        o.set_grid(g.get_grid())
        o.iteration = it
        pred = o.strata_next_counts(n)
        rg = g.iterate(n)
        cg = g.strata_counts().astype(np.int64)
        assert cg.sum() == n and cg.min() >= 2 and rg["n_events"] == n
        diff = np.abs(cg - pred)
        assert diff.max() <= 1 and np.mean(diff > 0) <= 1e-3, (name, it, diff.max(), np.mean(diff > 0))
        o.inject_strata_counts(cg)
        ro = o.iterate(n)
        wg, bg = g.get_weights(0, n)
        wo, bo = o.event_weights(it, 0, n)
        assert np.array_equal(bg, bo)
        assert np.all(np.abs(wg - wo) <= 1e-12 * np.abs(wo) + 1e-14 * np.mean(np.abs(wo))), name
        assert rel(rg["I"], ro["I"]) < REL and rel(rg["var"], ro["var"]) < REL, (name, it, rg, ro)
        g.refine()
        o.refine()


def test_adaptive_strata_bit_identical_across_launch_configurations(P):
    cfg = W.config("w_plus")
    n = 50_021

    def run(**kw):
        g = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n, **kw)
        g.set_strata(6)
        g.set_strata_beta(0.75)
        out = []
        for _ in range(3):
            r = g.iterate(n)
            out.append(np.array([r["I"], r["var"]]).tobytes() + g.strata_counts().tobytes())
            g.refine()
        return b"".join(out)

    ref = run()
    for wpb, mb in ((1, 0), (8, 0), (16, 5), (4, 97)):
        assert run(waves_per_block=wpb, max_blocks=mb) == ref, (wpb, mb)


def test_adaptive_strata_full_size_w_plus(P):
    """10^6 events over 10^4 hypercubes with beta = 1: counts against the oracle's
    rule, then integral and variance against the oracle with the counts injected.
    From the second iteration on the counts straddle 64, so hypercubes are folded both
    by their own lane (up to 64 events) and by a whole wave (more)."""
    cfg = W.config("w_plus")
    n = cfg["n_events"]
    g, o = pair(P, cfg, n, 10)
    g.set_strata_beta(1.0)
    o.set_strata_beta(1.0)
    for it in range(3):
        o.set_grid(g.get_grid())
        o.iteration = it
        pred = o.strata_next_counts(n)
        rg = g.iterate(n)
        cg = g.strata_counts().astype(np.int64)
        diff = np.abs(cg - pred)
        assert diff.max() <= 1 and np.mean(diff > 0) <= 1e-3
        if it > 0:
            assert cg.min() <= 64 < cg.max(), (cg.min(), cg.max())
        o.inject_strata_counts(cg)
        ro = o.iterate(n)
        assert rel(rg["I"], ro["I"]) < REL and rel(rg["var"], ro["var"]) < REL, (it, rg, ro)
        g.refine()
        o.refine()
