"""Pins for the oracle's random numbers, grid map and grid refinement (CPU only).

The paper (Sec. 2.1) fixes the structure -- iterations of event sets, a grid
re-optimised after each iteration from all events -- but prints no formula; the
pins below are invariants and closed forms of the VEGAS mathematics.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _philox_kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                v = [int(t, 16) for t in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


# ---------------------------------------------------------------- RNG -------
def test_philox_known_answer_vectors():
    """The generator against the published Philox4x32-10 known-answer vectors
    (Salmon et al., SC'11; the replacement of the paper's per-thread groups of
    random numbers, Sec. 2.2)."""
    rows = _philox_kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = [int(x) for x in oracle.philox(ctr, key)]
        assert got == want, (ctr, key, [hex(x) for x in got])


def test_uniform_construction_from_known_answer():
    """Event 0 of iteration 0 under seed 0 is counter (0, 0, 0, 0), key (0, 0): its
    two uniforms are the top 52 bits of output words (1:0) and (3:2) of the first
    known-answer vector, as (2w + 1) 2^-53, formed here with Python integers."""
    ctr, key, out = _philox_kat()[0]
    assert ctr == [0, 0, 0, 0] and key == [0, 0]
    want = []
    for hi, lo in ((out[1], out[0]), (out[3], out[2])):
        w = ((hi << 32) | lo) >> 12
        want.append((2 * w + 1) / 2.0 ** 53)
    u = oracle.uniforms(0, 0, 0, 2)
    assert list(u) == want


def test_uniforms_deterministic_and_open_interval():
    a = np.array([oracle.uniforms(1, 3, i, 8) for i in range(2000)])
    b = np.array([oracle.uniforms(1, 3, i, 8) for i in range(2000)])
    assert np.array_equal(a, b)
    assert a.min() > 0.0 and a.max() < 1.0
    # the construction (w + 1/2) 2^-52 puts every value on the odd multiples of 2^-53
    k = a * 2.0 ** 53
    assert np.all(k == np.round(k)) and np.all(np.round(k) % 2 == 1)


def test_uniforms_statistics():
    n = 40000
    u = np.array([oracle.uniforms(5, 0, i, 6) for i in range(n)])
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / (n * 6))
    assert abs(u.var() - 1 / 12) < 0.003
    # chi^2 of 20-bin occupancy per dimension
    for d in range(6):
        h, _ = np.histogram(u[:, d], bins=20, range=(0, 1))
        chi2 = ((h - n / 20) ** 2 / (n / 20)).sum()
        assert chi2 < 50  # 19 dof, p ~ 1e-4
    # cross-dimension and lag-1 (event index) correlations
    c = np.corrcoef(u.T)
    assert np.abs(c - np.eye(6)).max() < 0.03
    assert abs(np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]) < 0.03


def test_streams_differ_by_iteration_seed_and_event():
    base = oracle.uniforms(1, 0, 10, 4)
    assert not np.array_equal(base, oracle.uniforms(1, 1, 10, 4))
    assert not np.array_equal(base, oracle.uniforms(2, 0, 10, 4))
    assert not np.array_equal(base, oracle.uniforms(1, 0, 11, 4))
    # high word of the event index is part of the counter
    assert not np.array_equal(base, oracle.uniforms(1, 0, 10 + (1 << 32), 4))


def test_philox_avalanche():
    """Flipping one counter bit flips about half of the 128 output bits."""
    rng = np.random.default_rng(0)
    flips = []
    for _ in range(200):
        ctr = rng.integers(0, 2 ** 32, 4, dtype=np.uint64).astype(np.uint32)
        key = rng.integers(0, 2 ** 32, 2, dtype=np.uint64).astype(np.uint32)
        bit = rng.integers(0, 128)
        c2 = ctr.copy()
        c2[bit // 32] ^= np.uint32(1 << (bit % 32))
        o1, o2 = oracle.philox(ctr, key), oracle.philox(c2, key)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(o1, o2)))
    assert abs(np.mean(flips) - 64) < 2.5


# ---------------------------------------------------------------- grid ------
def _random_grid(ndim, nbins, rng):
    e = np.zeros((ndim, nbins + 1))
    for d in range(ndim):
        h = rng.uniform(0.2, 5.0, nbins)
        e[d, 1:] = np.cumsum(h) / h.sum()
        e[d, -1] = 1.0
    return e


def test_grid_map_invariants():
    rng = np.random.default_rng(1)
    v = oracle.Vegas(W.GAUSS, 3, 17, 1, 1.5, [0.5, 0.2])
    e = _random_grid(3, 17, rng)
    v.set_grid(e)
    # stratified integral of the Jacobian over y is exactly sum of bin widths = 1
    m = 17 * 40
    ys = (np.arange(m) + 0.5) / m
    for d in range(3):
        tot = 0.0
        xs = []
        for y in ys:
            u = np.full(3, 0.5)
            u[d] = y
            x, J, b = v.grid_map(u)
            # J factorises; divide out the other two dimensions at u = 0.5
            xs.append(x[d])
            assert b[d] == int(np.floor(y * 17))
        # monotone in y and inside the bin's edges
        assert np.all(np.diff(xs) > 0)
    for _ in range(200):
        u = rng.uniform(0, 1, 3)
        x, J, b = v.grid_map(u)
        for d in range(3):
            assert e[d, b[d]] <= x[d] <= e[d, b[d] + 1]
        assert np.isclose(J, np.prod([17 * (e[d, b[d] + 1] - e[d, b[d]]) for d in range(3)]),
                          rtol=1e-15)
    # integral of J over the unit cube (midpoint rule per bin is exact) = 1
    tot = 0.0
    for k in range(17):
        u = np.array([(k + 0.5) / 17, 0.5, 0.5])
        x, J, b = v.grid_map(u)
        tot += J / (17 * (e[1, b[1] + 1] - e[1, b[1]])) / (17 * (e[2, b[2] + 1] - e[2, b[2]])) / 17
    assert abs(tot - 1.0) < 1e-14


def test_grid_map_end_points():
    v = oracle.Vegas(W.GAUSS, 1, 10, 1, 1.5, [0.5, 0.2])
    rng = np.random.default_rng(2)
    e = _random_grid(1, 10, rng)
    v.set_grid(e)
    x0, _, b0 = v.grid_map(np.array([0.0]))
    x1, _, b1 = v.grid_map(np.array([1.0]))
    assert x0[0] == 0.0 and b0[0] == 0
    assert x1[0] == 1.0 and b1[0] == 9   # u = 1 is clamped into the last bin


def test_refine_uniform_histogram_is_a_fixed_point():
    rng = np.random.default_rng(3)
    for nb in (2, 5, 50, 255):
        e = np.tile(np.linspace(0, 1, nb + 1), (2, 1))
        d = np.full((2, nb), 3.7)
        e2 = oracle.refine_grid(2, nb, 1.5, d, e)
        assert np.allclose(e2.reshape(2, -1), e, atol=1e-14, rtol=0)
    # any grid with a flat histogram stays put
    e = _random_grid(2, 30, rng)
    e2 = oracle.refine_grid(2, 30, 1.5, np.ones((2, 30)), e)
    assert np.allclose(e2.reshape(2, -1), e, atol=1e-14, rtol=0)


def test_refine_zero_histogram_and_alpha_zero_leave_grid():
    rng = np.random.default_rng(4)
    e = _random_grid(3, 20, rng)
    assert np.array_equal(oracle.refine_grid(3, 20, 1.5, np.zeros((3, 20)), e).reshape(3, -1), e)
    d = rng.uniform(0.1, 10, (3, 20))
    e2 = oracle.refine_grid(3, 20, 0.0, d, e)   # alpha = 0: every m_k = 1
    assert np.allclose(e2.reshape(3, -1), e, atol=1e-14, rtol=0)


def test_refine_keeps_edges_ordered_and_pinned():
    rng = np.random.default_rng(5)
    for _ in range(50):
        nb = int(rng.integers(2, 120))
        e = _random_grid(1, nb, rng)
        d = rng.exponential(1.0, (1, nb)) * (rng.uniform(size=(1, nb)) < 0.7)
        d[0, rng.integers(0, nb)] = 1.0
        e2 = oracle.refine_grid(1, nb, 1.5, d, e).reshape(1, -1)
        assert e2[0, 0] == 0.0 and e2[0, -1] == 1.0
        assert np.all(np.diff(e2[0]) >= 0)


def _exact_hist_power(e, p):
    """Infinite-statistics histogram for f = (p+1) x^p: bin k holds
    n^2 h_k * integral of f^2 over the bin (up to the common factor N/n)."""
    n = len(e) - 1
    F = (p + 1) ** 2 / (2 * p + 1) * e ** (2 * p + 1)
    h = np.diff(e)
    return n * n * h * np.diff(F)


def test_refine_places_equal_importance_per_new_bin():
    """Exact property of the rebinning: with the damped importance m_k spread
    uniformly over old bin k, every new bin carries sum(m)/n of it."""
    rng = np.random.default_rng(6)
    for _ in range(30):
        nb = int(rng.integers(3, 100))
        e = _random_grid(1, nb, rng)[0]
        d = rng.exponential(1.0, nb)
        m = oracle.refine_weights(nb, 1.5, d)
        e2 = oracle.refine_grid(1, nb, 1.5, d[None, :], e[None, :]).reshape(-1)
        cm = np.concatenate([[0.0], np.cumsum(m)])
        mass = np.diff(np.interp(e2, e, cm))   # cumulative importance at the new edges
        assert np.allclose(mass, m.sum() / nb, rtol=1e-11, atol=0)


def test_refine_weights_properties():
    """m(r) = ((r-1)/ln r)^alpha: equal for equal r, increasing in r, limits at 0 and 1."""
    m = oracle.refine_weights(5, 1.5, np.full(5, 2.0))
    assert np.allclose(m, m[0], rtol=1e-15)
    d = np.array([0.0, 0.0, 0.0, 1.0, 2.0, 4.0, 8.0, 16.0, 0.0, 0.0])
    m = oracle.refine_weights(10, 1.5, d)
    assert m[0] == 0.0                                 # r = 0 -> m = 0
    dbar = np.array([0, 0, 1 / 3, 1, 7 / 3, 14 / 3, 28 / 3, 8, 16 / 3, 0])
    order = np.argsort(dbar, kind="stable")
    assert np.all(np.diff(m[order]) >= 0)             # monotone in the smoothed value
    assert oracle.refine_weights(4, 1.5, np.zeros(4)) is None
    # one populated bin after smoothing holds r = 1 only if n = 1; with two equal bins r = 1/2
    m2 = oracle.refine_weights(2, 1.0, np.array([1.0, 1.0]))
    assert np.allclose(m2, 0.5 / np.log(2.0), rtol=1e-15)   # (1/2 - 1)/ln(1/2)


def test_refine_converges_to_importance_density():
    """Deterministic VEGAS (infinite statistics) on the Genz corner peak
    f = (1 + 2x)^-2 in 1-D: after a realistic number of iterations the edges
    sit at the equal-|f| quantiles.  (Over many tens of iterations the
    period-2 mode, which neighbour smoothing cannot damp, grows; this test stays
    within the iteration counts the method is used with.)"""
    a, n = 2.0, 20

    def hist(e):   # n^2 h_k * int_bin f^2
        F = -(1 + a * e) ** -3 / (3 * a)
        return n * n * np.diff(e) * np.diff(F)

    q = np.arange(n + 1) / n
    c = 1 - 1 / (1 + a)
    target = (1 / (1 - q * c) - 1) / a
    e = np.linspace(0, 1, n + 1)
    for _ in range(6):
        e = oracle.refine_grid(1, n, 1.5, hist(e)[None, :], e[None, :]).reshape(-1)
    assert np.abs(e - target).max() < 5e-3
    assert np.abs(np.linspace(0, 1, n + 1) - target).max() > 0.1   # it did move


def test_vegas_mc_grid_follows_deterministic_fixed_point():
    """The same fixed point reached by Monte Carlo with the oracle's own loop:
    Genz corner peak in 1-D with a = 2 is (1 + 2x)^-2 = f; compare edges with
    the exact equal-importance edges of |f| within MC noise."""
    a = 2.0
    v = oracle.Vegas(W.GENZ, 1, 20, 11, 1.5, [3.0, a, 0.5])
    for _ in range(12):
        v.iterate(50000)
        v.refine()
    e = v.get_grid()[0]
    # |f| CDF: (1 - 1/(1+a x)) / (1 - 1/(1+a)) ; inverse at k/n
    q = np.arange(21) / 20
    c = 1 - 1 / (1 + a)
    target = (1 / (1 - q * c) - 1) / a
    assert np.abs(e - target).max() < 0.02
