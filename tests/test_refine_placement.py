"""The refinement kernel's edge placement, restated in Python (CPU only).

The kernel gives each lane of a wave c = ceil(n/64) consecutive bins.  It forms the
cumulative importance at the lane's bin boundaries from a wave scan, raises them to the
running maximum of the chunk ends of the lanes before it, and lets every lane place the
new edges k (target k * stp, stp = cm[n] / n) that fall into its own bins:
cm[j] < k stp <= cm[j+1], the last bin taking every remaining edge.  These tests check,
on exact binary64 arithmetic, that this placement equals a binary search over a
sequential cm (the oracle's order), and that with arbitrarily rounded scan values the
bins' intervals still tile the range: every interior edge is written exactly once, by the
bin the search rule names.
"""
import random


def search(cm, m, eo, n):
    stp = cm[n] / n
    out = {}
    for k in range(1, n):
        t = k * stp
        lo, hi = 0, n - 1  # largest j in [0, n-1] with cm[j] < t
        while lo < hi:
            mid = (lo + hi + 1) >> 1
            if cm[mid] < t:
                lo = mid
            else:
                hi = mid - 1
        j = lo
        frac = (t - cm[j]) / m[j] if m[j] > 0 else 0.0
        frac = min(max(frac, 0.0), 1.0)
        out[k] = eo[j] + frac * (eo[j + 1] - eo[j])
    return out


def place(bounds, m, eo, n, stp):
    """bounds[j] = (lo, hi) of bin j as the kernel's lanes see them"""
    out = {}
    for j in range(n):
        lo, hi = bounds[j]
        k = max(int(lo / stp), 1)
        while k > 1 and (k - 1) * stp > lo:
            k -= 1
        while k < n and k * stp <= lo:
            k += 1
        while k < n:
            t = k * stp
            if j < n - 1 and t > hi:
                break
            assert k not in out, "edge placed twice"
            frac = (t - lo) / m[j] if m[j] > 0 else 0.0
            frac = min(max(frac, 0.0), 1.0)
            out[k] = (j, eo[j] + frac * (eo[j + 1] - eo[j]))
            k += 1
    assert sorted(out) == list(range(1, n)), "edge missing"
    return out


def importance(rng, n, kind):
    if kind == 0:
        m = [rng.random() for _ in range(n)]
    elif kind == 1:
        m = [rng.random() if rng.random() < 0.25 else 0.0 for _ in range(n)]
    elif kind == 2:
        m = [10.0 ** rng.uniform(-25, 5) for _ in range(n)]
    else:
        m = [0.0] * n
        m[rng.randrange(n)] = 1.0
    if sum(m) == 0.0:
        m[rng.randrange(n)] = 0.5
    return m


def test_placement_by_bin_equals_search():
    rng = random.Random(11)
    for trial in range(3000):
        n = rng.choice([2, 3, 50, 100, 255, rng.randint(2, 255)])
        m = importance(rng, n, trial % 4)
        cm = [0.0]
        for x in m:
            cm.append(cm[-1] + x)
        eo = [0.0] + sorted(rng.random() for _ in range(n - 1)) + [1.0]
        stp = cm[n] / n
        got = place([(cm[j], cm[j + 1]) for j in range(n)], m, eo, n, stp)
        want = search(cm, m, eo, n)
        assert {k: v for k, (j, v) in got.items()} == want, (trial, n)


def test_lane_boundaries_tile_the_range_under_any_rounding():
    rng = random.Random(5)
    for trial in range(1500):
        n = rng.choice([2, 3, 63, 64, 65, 100, 128, 129, 255, rng.randint(2, 255)])
        m = importance(rng, n, trial % 4)
        c = (n + 63) // 64
        part = [sum(m[j] for j in range(c * l, min(c * l + c, n))) for l in range(64)]
        # the scan's exclusive values, each off by a few ulps in either direction
        excl, acc = [], 0.0
        for l in range(64):
            excl.append(acc * (1 + rng.choice([-1, 0, 1]) * 2.2e-16 * rng.randint(0, 4)))
            acc += part[l]
        r = []
        for l in range(64):
            rr = [excl[l]]
            for i in range(4):
                j = c * l + i
                rr.append(rr[-1] + m[j] if (i < c and j < n) else rr[-1])
            r.append(rr)
        carry, top = [], 0.0
        for l in range(64):
            carry.append(top)
            top = max(top, r[l][4])
        cb = [[carry[l]] + [max(r[l][i], carry[l]) for i in range(1, 5)] for l in range(64)]
        bounds = [(cb[j // c][j % c], cb[j // c][j % c + 1]) for j in range(n)]
        stp = cb[(n - 1) // c][4] / n
        eo = [0.0] + sorted(rng.random() for _ in range(n - 1)) + [1.0]
        got = place(bounds, m, eo, n, stp)
        cm = [bounds[j][0] for j in range(n)]
        for k, (j, _) in got.items():  # the search rule on the kernel's own (monotone) cm
            t = k * stp
            assert cm[j] < t and all(cm[i] >= t for i in range(j + 1, n)), (trial, k, j)
