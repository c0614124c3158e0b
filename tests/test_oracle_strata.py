"""Pins for the oracle's stratified sampling (CPU only).

Lepage's stratified + importance mode: m strata per axis cut the unit cube into
H = m^D equal hypercubes, each with the same number n of events, placed by the
grid map like any other; the estimate is sum_h (1/H) mean_h and its variance
sum_h (1/H)^2 sigma_h^2 / n.  The pins: m = 1 is the plain iteration; the
placement of each event in its hypercube (read back through the grid bins);
the closed-form variance of the stratified estimator for a 1-D Gaussian on the
uniform grid, matched both by the mean of the per-iteration variance estimates
and by the spread of the estimates themselves; pulls over seeds.  Adaptive
allocation (VEGAS+ reading, n_h following sigma_h^beta): the unequal-count
variance against its closed form with an injected allocation, and beta = 1
reaching Neyman's optimum allocation.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def phi(t):
    return 0.5 * (1 + math.erf(t / math.sqrt(2)))


def test_one_stratum_is_the_plain_iteration():
    c = W.config("gauss4")
    a = oracle.Vegas(c["process"], 4, 50, 7, 1.5, c["params"])
    b = oracle.Vegas(c["process"], 4, 50, 7, 1.5, c["params"])
    b.set_strata(1)
    for _ in range(3):
        ra, rb = a.iterate(5000), b.iterate(5000)
        assert ra["I"] == rb["I"] and rb["n_events"] == 5000
        assert abs(ra["var"] / rb["var"] - 1) < 1e-13
        a.refine()
        b.refine()
        assert np.array_equal(a.get_grid(), b.get_grid())


def test_events_lie_in_their_hypercubes():
    """On the uniform grid with k bins per stratum the grid bin of each coordinate
    gives its stratum; event i must lie in hypercube floor(i / n), whose base-m
    digits (dimension 0 the least significant) are its strata."""
    m, D, k = 3, 3, 4
    par = np.concatenate([[4.0], np.full(D, 2.0), np.full(D, 0.5)])
    v = oracle.Vegas(W.GENZ, D, m * k, 3, 1.5, par)
    v.set_strata(m)
    N = 2 * m ** D + 5                       # 2 per hypercube, 5 left over
    r = v.iterate(N)
    assert r["n_events"] == 2 * m ** D and v.strata_npc == 2
    _, bins = v.event_weights(0, 0, 2 * m ** D)
    for i in range(2 * m ** D):
        h = i // 2
        for d in range(D):
            assert bins[i, d] // k == h % m, (i, d)
            h //= m


def stratified_variance_1d(mu, sg, m, n):
    """Var of the stratified estimator of int_0^1 N(x; mu, sg) dx on the uniform
    grid: sum_h (1/m)^2 Var_h(f) / n with Var_h = m int_h f^2 - (m int_h f)^2,
    int f^2 = (1 / (2 sg sqrt(pi))) int N(x; mu, sg / sqrt2)."""
    tot = 0.0
    for h in range(m):
        a, b = h / m, (h + 1) / m
        i1 = phi((b - mu) / sg) - phi((a - mu) / sg)
        s2 = sg / math.sqrt(2)
        i2 = (phi((b - mu) / s2) - phi((a - mu) / s2)) / (2 * sg * math.sqrt(math.pi))
        tot += (m * i2 - (m * i1) ** 2) / m ** 2 / n
    return tot


def test_stratified_variance_matches_closed_form():
    """K independent iterations (fresh random numbers each, grid left uniform): the
    mean of the per-iteration variance estimates and the sample variance of the
    estimates both match the closed form, and stratification beats the plain
    estimator's (1/N)(int f^2 - I^2) by far."""
    mu, sg, m, n, K = 0.4, 0.15, 8, 6, 400
    v = oracle.Vegas(W.GAUSS, 1, 16, 11, 1.5, [mu, sg])
    v.set_strata(m)
    Is, vs = [], []
    for _ in range(K):
        r = v.iterate(m * n)
        Is.append(r["I"])
        vs.append(r["var"])
    true = stratified_variance_1d(mu, sg, m, n)
    assert abs(np.mean(vs) / true - 1) < 0.03, (np.mean(vs), true)
    assert abs(np.var(Is, ddof=1) / true - 1) < 0.2, (np.var(Is, ddof=1), true)
    exact = phi((1 - mu) / sg) - phi(-mu / sg)
    s2 = sg / math.sqrt(2)
    f2 = (phi((1 - mu) / s2) - phi(-mu / s2)) / (2 * sg * math.sqrt(math.pi))
    plain = (f2 - exact ** 2) / (m * n)
    assert true < plain / 10
    assert abs(np.mean(Is) - exact) < 4 * math.sqrt(true / K)


def test_pulls_over_seeds_with_refinement():
    c = W.config("gauss4")
    mu, sg = c["params"]
    one = phi((1 - mu) / sg) - phi(-mu / sg)
    exact = one ** 4
    pulls = []
    for seed in range(40):
        v = oracle.Vegas(W.GAUSS, 4, 30, 100 + seed, 1.5, c["params"])
        v.set_strata(3)
        for _ in range(4):
            v.iterate(3000)
            v.refine()
        r = v.result()
        pulls.append((r["I"] - exact) / r["sigma"])
    assert 0.7 < np.std(pulls) < 1.3 and abs(np.mean(pulls)) < 0.5, (np.mean(pulls), np.std(pulls))


def test_strata_refusals():
    c = W.config("gauss4")
    v = oracle.Vegas(c["process"], 4, 50, 7, 1.5, c["params"])
    with pytest.raises(ValueError):
        v.set_strata(-1)
    with pytest.raises(ValueError):
        v.set_strata(300)                    # 300^4 hypercubes overflow
    v.set_strata(5)                          # 625 hypercubes
    with pytest.raises(ValueError):
        v.iterate(1249)                      # fewer than 2 per hypercube
    assert v.iterate(1250)["n_events"] == 1250
    v.set_strata(0)
    assert v.iterate(1249)["n_events"] == 1249


def stratum_moments_1d(mu, sg, m):
    """Per stratum h of [0, 1] (width 1/m): Var_h(f) = m int_h f^2 - (m int_h f)^2 for
    the normal density f (closed forms with erf)."""
    out = []
    s2 = sg / math.sqrt(2)
    for h in range(m):
        a, b = h / m, (h + 1) / m
        i1 = phi((b - mu) / sg) - phi((a - mu) / sg)
        i2 = (phi((b - mu) / s2) - phi((a - mu) / s2)) / (2 * sg * math.sqrt(math.pi))
        out.append(m * i2 - (m * i1) ** 2)
    return np.array(out)


def test_unequal_counts_variance_matches_closed_form():
    """Adaptive mode with a fixed, injected allocation n_h: the weights are scaled by
    N / (H n_h), the estimate stays unbiased and the variance estimate matches
    sum_h (1/m)^2 Var_h(f) / n_h, both on average and as the spread of the estimates."""
    mu, sg, m, K = 0.4, 0.15, 8, 400
    counts = np.array([3, 5, 9, 14, 12, 7, 4, 2], dtype=np.int64)
    n = int(counts.sum())
    v = oracle.Vegas(W.GAUSS, 1, 16, 13, 1.5, [mu, sg])
    v.set_strata(m)
    v.set_strata_beta(1.0)
    Is, vs = [], []
    for _ in range(K):
        v.inject_strata_counts(counts)
        r = v.iterate(n)
        assert np.array_equal(v.strata_counts(), counts)
        Is.append(r["I"])
        vs.append(r["var"])
    true = float(np.sum(stratum_moments_1d(mu, sg, m) / m ** 2 / counts))
    assert abs(np.mean(vs) / true - 1) < 0.05, (np.mean(vs), true)
    assert abs(np.var(Is, ddof=1) / true - 1) < 0.2, (np.var(Is, ddof=1), true)
    exact = phi((1 - mu) / sg) - phi(-mu / sg)
    assert abs(np.mean(Is) - exact) < 4 * math.sqrt(true / K)


def test_adaptive_allocation_approaches_neyman():
    """beta = 1 gives n_h proportional to sigma_h (Neyman's optimum
    (sum_h sigma_h / m)^2 / n); the achieved variance beats equal counts and is
    close to the optimum, and every allocation keeps sum n_h = n, n_h >= 2."""
    mu, sg, m, n, K = 0.4, 0.1, 10, 400, 60
    sig = np.sqrt(stratum_moments_1d(mu, sg, m))
    neyman = float((sig / m).sum() ** 2 / n)
    equal = float(np.sum(sig ** 2 / m ** 2 / (n // m)))
    v = oracle.Vegas(W.GAUSS, 1, 20, 17, 1.5, [mu, sg])
    v.set_strata(m)
    v.set_strata_beta(1.0)
    vs = []
    for it in range(K):
        r = v.iterate(n)
        c = v.strata_counts()
        assert c.sum() == n and c.min() >= 2
        if it >= 2:
            vs.append(r["var"])
    got = np.mean(vs)
    assert got < 0.6 * equal, (got, equal)          # here Neyman is 0.51 x equal counts
    assert got < 1.1 * neyman, (got, neyman)        # measured 1.015 x


def test_adaptive_first_iteration_and_counts_invariants():
    c = W.config("gauss4")
    v = oracle.Vegas(c["process"], 4, 30, 7, 1.5, c["params"])
    v.set_strata(4)
    v.set_strata_beta(0.75)
    r = v.iterate(20_003)                      # first: equal counts, remainder to the first cubes
    cnt = v.strata_counts()
    assert r["n_events"] == 20_003 and cnt.sum() == 20_003
    q, R = divmod(20_003 - 2 * 256, 256)
    assert np.array_equal(cnt, 2 + q + (np.arange(256) < R))
    v.iterate(20_003)
    cnt = v.strata_counts()
    assert cnt.sum() == 20_003 and cnt.min() >= 2 and cnt.max() > cnt.min()
    with pytest.raises(ValueError):
        v.set_strata_beta(-1.0)
