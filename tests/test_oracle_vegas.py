"""Pins for the oracle's VEGAS loop on analytic integrands (CPU only).

Sec. 2.1 of the paper: iterations of event sets with a grid re-optimised after
each iteration.  The estimator I_j = S1/N, var_j = (S2/N - I_j^2)/(N-1) and the
inverse-variance combination are the reading used (paper silent); they are
pinned by closed-form integrals and by the pull distribution over seeds.
"""
import math
from itertools import combinations

import numpy as np
import pytest

import oracle
import workloads as W


def run(v, n_iter, n):
    for _ in range(n_iter):
        v.iterate(n)
        v.refine()
    return v.result()


def gauss_exact(mu, sg, ndim):
    one = 0.5 * (math.erf((1 - mu) / (sg * math.sqrt(2))) + math.erf(mu / (sg * math.sqrt(2))))
    return one ** ndim


def genz_exact(par, ndim):
    fam = int(par[0])
    a, w = par[1:1 + ndim], par[1 + ndim:1 + 2 * ndim]
    if fam == 1:
        z = np.exp(2j * np.pi * w[0]) * np.prod((np.exp(1j * a) - 1) / (1j * a))
        return z.real
    if fam == 2:
        return np.prod(a * (np.arctan(a * (1 - w)) + np.arctan(a * w)))
    if fam == 3:
        tot = 0.0
        for k in range(ndim + 1):
            for S in combinations(range(ndim), k):
                tot += (-1) ** k / (1 + sum(a[i] for i in S))
        return tot / (math.factorial(ndim) * np.prod(a))
    if fam == 4:
        erf = np.vectorize(math.erf)
        return np.prod(np.sqrt(np.pi) / (2 * a) * (erf(a * (1 - w)) + erf(a * w)))
    if fam == 5:
        return np.prod((2 - np.exp(-a * w) - np.exp(-a * (1 - w))) / a)
    if fam == 6:
        r = 1.0
        for i in range(ndim):
            r *= (np.exp(a[i] * w[i]) - 1) / a[i] if i < 2 else (np.exp(a[i]) - 1) / a[i]
        return r
    raise ValueError


def test_gaussian_4d_within_errors():
    cfg = W.config("gauss4")
    v = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    r = run(v, cfg["n_iter"], cfg["n_events"])
    exact = gauss_exact(0.5, 0.1, 4)
    assert abs(r["I"] - exact) < 4 * r["sigma"]
    assert r["sigma"] / exact < 5e-3
    assert r["chi2_dof"] < 4


@pytest.mark.parametrize("family", [1, 2, 3, 4, 5, 6])
def test_genz_families_within_errors(family):
    ndim = 3
    par = W.genz_params(family, ndim, seed=10 + family, difficulty=4.0)
    v = oracle.Vegas(W.GENZ, ndim, 30, 3, 1.5, par)
    r = run(v, 6, 20000)
    exact = genz_exact(par, ndim)
    assert abs(r["I"] - exact) < 4.5 * r["sigma"] + 1e-14, (r, exact)


def test_closed_forms_by_quadrature():
    """The Genz closed forms used above agree with tensor Gauss-Legendre
    quadrature of the oracle integrand (smooth families, 2-D)."""
    xs, ws = np.polynomial.legendre.leggauss(60)
    x01, w01 = 0.5 * (xs + 1), 0.5 * ws
    for fam in (1, 2, 3, 4):
        par = W.genz_params(fam, 2, seed=1, difficulty=3.0)
        tot = sum(wa * wb * oracle.integrand(W.GENZ, par, [xa, xb])
                  for xa, wa in zip(x01, w01) for xb, wb in zip(x01, w01))
        assert abs(tot - genz_exact(par, 2)) < 1e-10 * max(1, abs(tot))


def test_pull_distribution_over_seeds():
    """(I - exact)/sigma over 100 seeds has mean ~0 and width ~1."""
    pulls = []
    for seed in range(100):
        v = oracle.Vegas(W.GAUSS, 2, 20, 1000 + seed, 1.5, [0.4, 0.15])
        r = run(v, 4, 4000)
        pulls.append((r["I"] - gauss_exact(0.4, 0.15, 2)) / r["sigma"])
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.35
    assert 0.75 < pulls.std() < 1.3


def test_constant_integrand_has_zero_variance():
    """Genz corner peak with a = 0 is exactly 1: on the uniform grid with a
    power-of-two bin count every Jacobian is exactly 1, so the variance is 0
    and the result is exact."""
    par = np.concatenate([[3.0], np.zeros(2), np.full(2, 0.5)])
    v = oracle.Vegas(W.GENZ, 2, 8, 1, 1.5, par)
    r1 = v.iterate(1000)
    assert r1["I"] == 1.0 and r1["var"] == 0.0
    res = v.result()
    assert res["I"] == 1.0 and res["sigma"] == 0.0


def test_nonfinite_weights_are_counted_and_dropped():
    par = np.concatenate([[9.0], np.ones(2), np.full(2, 0.5)])   # unknown family -> NaN
    v = oracle.Vegas(W.GENZ, 2, 10, 1, 1.5, par)
    r = v.iterate(500)
    assert r["n_nonfinite"] == 500 and r["I"] == 0.0


def test_refine_before_iterate_is_an_error():
    v = oracle.Vegas(W.GAUSS, 2, 10, 1, 1.5, [0.5, 0.1])
    with pytest.raises(RuntimeError):
        v.refine()


def test_histogram_sums_to_s2_in_every_dimension():
    cfg = W.config("gauss4")
    v = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    v.iterate(5000)
    d, sums = v.get_hist()
    assert np.allclose(d.sum(axis=1), sums[1], rtol=1e-12)
    w, b = v.event_weights(0, 0, 5000)
    assert np.isclose(w.sum(), sums[0], rtol=1e-12)
    assert np.isclose((w * w).sum(), sums[1], rtol=1e-12)
    for dim in range(4):
        assert np.allclose(np.bincount(b[:, dim], weights=w * w, minlength=50), d[dim],
                           rtol=1e-11)


def test_iteration_counter_keys_the_stream():
    """Events of iteration j are a function of (seed, j, i) only: recomputing
    iteration 0's weights after later iterations (same grid) gives the same values."""
    v = oracle.Vegas(W.GAUSS, 3, 10, 5, 1.5, [0.5, 0.2])
    w0, _ = v.event_weights(0, 0, 100)
    v.iterate(1000)
    v.iterate(1000)
    w0b, _ = v.event_weights(0, 0, 100)
    assert np.array_equal(w0, w0b)
    w1, _ = v.event_weights(1, 0, 100)
    assert not np.array_equal(w0, w1)


def test_result_from_last_iteration_is_that_iteration():
    """Combining only the last iteration returns that iteration's own estimate
    (I_j, sqrt(var_j)) as iterate() reported it, with one iteration counted."""
    cfg = W.config("gauss4")
    v = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    for _ in range(2):
        v.iterate(3000)
        v.refine()
    last = v.iterate(5000)
    r = v.result(first=2)
    assert r["n_iter"] == 1 and r["chi2_dof"] == 0.0
    assert abs(r["I"] - last["I"]) <= 1e-15 * abs(last["I"])
    assert abs(r["sigma"] - math.sqrt(last["var"])) <= 1e-15 * math.sqrt(last["var"])
    assert v.result()["n_iter"] == 3


def test_result_from_out_of_range_is_an_error():
    v = oracle.Vegas(W.GAUSS, 2, 10, 1, 1.5, [0.5, 0.1])
    with pytest.raises(ValueError):
        v.result()
    v.iterate(100)
    for first in (-1, 1, 5):
        with pytest.raises(ValueError):
            v.result(first=first)


def test_two_stage_schedule_pulls_after_dropping_warm_up():
    """The timing schedule of Sec. 3.2 (4 small iterations, then 10 ten times
    larger), with the warm-up iterations dropped: the pulls against the exact
    Gaussian integral over seeds have mean 0 and width 1, and the error of the
    second stage alone is larger than that of all iterations together."""
    pulls = []
    for seed in range(1, 41):
        v = oracle.Vegas(W.GAUSS, 2, 20, seed, 1.5, [0.4, 0.15])
        for n in [300] * 4 + [3000] * 10:
            v.iterate(n)
            v.refine()
        r, rall = v.result(first=4), v.result()
        assert r["n_iter"] == 10 and rall["n_iter"] == 14
        assert r["sigma"] > rall["sigma"]
        pulls.append((r["I"] - gauss_exact(0.4, 0.15, 2)) / r["sigma"])
    pulls = np.array(pulls)
    assert abs(pulls.mean()) < 0.5
    assert 0.7 < pulls.std() < 1.35


def test_threaded_iteration_matches_serial():
    """The all-core CPU baseline (the paper's scheme of Sec. 2.2: fixed per-thread
    chunks, partials added in a fixed order) computes the same iteration as the
    serial oracle: bit for bit with one thread, to the rounding of the long-double
    partial sums with several; the refined grids agree likewise."""
    cfg = W.config("w_plus")

    def mk():
        return oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                            cfg["params"])

    a, b, c = mk(), mk(), mk()
    for _ in range(3):
        ra, rb, rc = a.iterate(30_000), b.iterate_threads(30_000, 1), c.iterate_threads(30_000, 5)
        assert ra["I"] == rb["I"] and ra["var"] == rb["var"]
        assert ra["n_nonzero"] == rc["n_nonzero"] and ra["n_nonfinite"] == rc["n_nonfinite"]
        assert abs(rc["I"] - ra["I"]) <= 1e-15 * abs(ra["I"])
        assert abs(rc["var"] - ra["var"]) <= 1e-13 * ra["var"]
        a.refine(), b.refine(), c.refine()
    assert np.array_equal(a.get_grid(), b.get_grid())
    assert np.abs(a.get_grid() - c.get_grid()).max() < 1e-13
    assert a.result()["I"] == b.result()["I"]
