"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bars (stated in the design notes): per-event weights within 1e-12 relative in
FP64; per-iteration integral, variance, S1, S2 and histogram within 1e-10
relative with the grid injected into the oracle; bin indices bit-exact; cut
decisions identical (flips counted, none allowed); byte-identical results for
every launch configuration (the GPU form of the paper's thread-count
independence, Sec. 2.2).
"""
import struct

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

REL_EVENT = 1e-12
REL_ITER = 1e-10


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_06182_amd as P
    P.load()
    return P


def make_pair(P, cfg, max_events, **kw):
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"], max_events=max_events, **kw)
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    return g, o


def cases():
    out = []
    for name in ("gauss4", "eemumu", "dy_z", "w_plus", "ww_4l", "ww_had"):
        out.append((name, W.config(name)))
    for fam in (1, 2, 3, 4, 5, 6):
        out.append((f"genz{fam}", dict(process=W.GENZ, ndim=5, nbins=40, seed=9, alpha=1.5,
                                       params=W.genz_params(fam, 5, seed=fam, difficulty=6.0))))
    out.append(("gauss16x255", GAUSS_MAX))
    return out


# the largest grid (16 dimensions x 255 bins): its digit histogram (98 KB) exceeds one
# block's LDS, so every iteration folds from the records with the dimensions split
# over blocks
GAUSS_MAX = dict(process=W.GAUSS, ndim=16, nbins=255, seed=5, alpha=1.5, params=[0.5, 0.3])


def compare_weights(wg, wo, tag):
    """|w_gpu - w_oracle| <= 1e-12 |w_oracle| + 1e-14 mean|w_oracle|.  The absolute
    floor only matters for integrands that pass through zero (the oscillatory
    Genz family), where a relative bar is ill-conditioned."""
    assert wg.shape == wo.shape
    zg, zo = wg == 0.0, wo == 0.0
    flips = int(np.count_nonzero(zg != zo))
    assert flips == 0, f"{tag}: {flips} cut flips"
    floor = 1e-14 * np.mean(np.abs(wo))
    bad = np.abs(wg - wo) > REL_EVENT * np.abs(wo) + floor
    nz = ~zo
    rel = np.abs(wg[nz] - wo[nz]) / np.abs(wo[nz])
    assert not bad.any(), f"{tag}: {int(bad.sum())} events off, max rel {rel.max():.3e}"


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    den = np.maximum(np.abs(b), 1e-300)
    return np.max(np.abs(a - b) / den)


@pytest.mark.parametrize("name,cfg", cases(), ids=[c[0] for c in cases()])
def test_iterations_match_oracle(P, name, cfg):
    """Three iterations (with refinement) at a size that spans many blocks and a
    ragged tail; grid injected into the oracle before each iteration."""
    n = 6007 if cfg["process"] not in (W.WW_4L, W.WW_HAD) else 4099
    g, o = make_pair(P, cfg, n)
    for it in range(3):
        o.set_grid(g.get_grid())
        o.iteration = it
        rg = g.iterate(n)
        ro = o.iterate(n)
        wg, bg = g.get_weights(0, n)
        wo, bo = o.event_weights(it, 0, n)
        assert np.array_equal(bg, bo), f"{name} it{it}: bin indices differ"
        compare_weights(wg, wo, f"{name} it{it}")
        assert rg["n_nonzero"] == ro["n_nonzero"] and rg["n_nonfinite"] == ro["n_nonfinite"]
        assert rel(rg["I"], ro["I"]) < REL_ITER, (name, it, rg, ro)
        assert rel(rg["var"], ro["var"]) < REL_ITER, (name, it, rg, ro)
        dg, sg = g.get_hist()
        do, so = o.get_hist()
        assert rel(sg, so) < REL_ITER
        # the exact digit sums resolve each event's w^2 to 2^-94 of the largest (four
        # digits; the fused fold's scale sits 2^32 above the previous iteration's max
        # w^2, the two-pass fold's at this iteration's), so a bin carries at most
        # N 2^-94 max w^2 <= N 2^-94 S2 of truncation: the relative bar plus that floor
        floor = n * 2.0 ** -94 * so[1]
        assert np.array_equal(dg[do > floor] > 0, np.ones(int(np.sum(do > floor)), bool))
        assert np.all(np.abs(dg - do) <= REL_ITER * np.abs(do) + floor), \
            (name, it, float(np.max(np.abs(dg - do) / np.maximum(np.abs(do), floor))))
        g.refine()
        o.refine()
        assert np.max(np.abs(g.get_grid() - o.get_grid())) < 1e-12, f"{name} it{it}: grids"


@pytest.mark.parametrize("name", ["dy_z", "gauss4"])
def test_full_schedule_end_to_end(P, name):
    """The whole schedule without grid injection: the grids drift only by
    rounding, so the combined integral and error agree with the oracle's."""
    cfg = W.config(name)
    n = cfg["n_events"]
    g, o = make_pair(P, cfg, n)
    for _ in range(cfg["n_iter"]):
        g.iterate(n)
        g.refine()
        o.iterate(n)
        o.refine()
    rg, ro = g.result(), o.result()
    assert rel(rg["I"], ro["I"]) < REL_ITER
    assert rel(rg["sigma"], ro["sigma"]) < 1e-8
    assert abs(rg["chi2_dof"] - ro["chi2_dof"]) < 1e-6 * max(1.0, ro["chi2_dof"])
    assert rg["n_iter"] == ro["n_iter"] == cfg["n_iter"]


def test_hadronic_schedule_end_to_end(P, capsys):
    """The hadronic W+W- integrand (10 dims, weights spanning tens of decades) over
    six iterations of 1e5 events with refinement and no grid injection: whatever the
    fixed-point digits do to grid bins far below the largest, the combined integral
    stays within 1e-10 and its error within 1e-8 of the oracle's."""
    cfg = W.config("ww_had")
    n = 100_000
    g, o = make_pair(P, cfg, n)
    for _ in range(6):
        g.iterate(n)
        g.refine()
        o.iterate(n)
        o.refine()
    rg, ro = g.result(), o.result()
    dgrid = float(np.max(np.abs(g.get_grid() - o.get_grid())))
    with capsys.disabled():
        print(f"\n  ww_had schedule: rel I {rel(rg['I'], ro['I']):.2e} rel sigma {rel(rg['sigma'], ro['sigma']):.2e} "
              f"max grid difference {dgrid:.2e}")
    assert rg["n_iter"] == ro["n_iter"] == 6
    assert rel(rg["I"], ro["I"]) < REL_ITER
    assert rel(rg["sigma"], ro["sigma"]) < 1e-8


def test_paper_schedule_with_and_without_warm_up(P):
    """The two-stage schedule of the timing runs in Sec. 3.2 (4 x 1,000 then
    10 x 10,000 events) on the W+W- integrand, no grid injection: the combination
    of all iterations and that of the second stage only agree with the oracle's."""
    cfg = W.config("ww_4l")
    g, o = make_pair(P, cfg, 10_000)
    for n in [1000] * 4 + [10_000] * 10:
        g.iterate(n)
        g.refine()
        o.iterate(n)
        o.refine()
    for first, n_iter in ((0, 14), (4, 10), (13, 1)):
        rg, ro = g.result(first=first), o.result(first=first)
        assert rg["n_iter"] == ro["n_iter"] == n_iter
        assert rel(rg["I"], ro["I"]) < REL_ITER, first
        assert rel(rg["sigma"], ro["sigma"]) < 1e-8, first
        assert abs(rg["chi2_dof"] - ro["chi2_dof"]) < 1e-6 * max(1.0, ro["chi2_dof"]), first
    with pytest.raises(P.VegasError):
        g.result(first=14)


def run_schedule(P, cfg, n, n_iter, **launch):
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"], max_events=n, **launch)
    blobs = []
    for _ in range(n_iter):
        r = g.iterate(n)
        d, s = g.get_hist()
        g.refine()
        blobs.append(np.array([r["I"], r["var"]]).tobytes() + d.tobytes() + s.tobytes()
                     + g.get_grid().tobytes())
    res = g.result()
    blobs.append(np.array([res["I"], res["sigma"], res["chi2_dof"]]).tobytes())
    return b"".join(blobs)


@pytest.mark.parametrize("name", ["w_plus", "ww_4l", "ww_had", "genz2", "gauss16x255"])
def test_bit_identical_across_launch_configurations(P, name):
    if name == "genz2":
        cfg = dict(process=W.GENZ, ndim=5, nbins=40, seed=9, alpha=1.5,
                   params=W.genz_params(2, 5, seed=2, difficulty=6.0))
    elif name == "gauss16x255":
        cfg = GAUSS_MAX
    else:
        cfg = W.config(name)
    n = 50_021 if name not in ("ww_4l", "ww_had") else 20_011
    ref = run_schedule(P, cfg, n, 3)
    for wpb, mb in ((1, 0), (2, 3), (4, 1), (8, 0), (16, 5), (4, 97)):
        assert run_schedule(P, cfg, n, 3, waves_per_block=wpb, max_blocks=mb) == ref, (wpb, mb)


def test_checkpoint_resume_is_bit_identical(P):
    cfg = W.config("w_plus")
    n = 40_000
    a = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
    for _ in range(3):
        a.iterate(n)
        a.refine()
    blob = a.get_state()
    for _ in range(3):
        a.iterate(n)
        a.refine()
    ra = a.result()
    b = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
    b.set_state(blob)
    for _ in range(3):
        b.iterate(n)
        b.refine()
    rb = b.result()
    assert ra == rb
    assert np.array_equal(a.get_grid(), b.get_grid())


def _with_scale(blob, valid, e1):
    """The checkpoint with its stored fused-fold scale replaced (header: magic,
    process, ndim, nbins, iteration, seed, then valid, E1, E2, unused)."""
    off = struct.calcsize("<Q3iIQ")
    return blob[:off] + struct.pack("<4i", valid, e1, 2 * e1, 0) + blob[off + 16:]


def test_fold_modes(P):
    """The first iteration folds the sums from the records at its own scale (fold 0);
    later ones fold inside the event kernel at the scale the previous iteration fixed
    (fold 1).  A stored scale that this iteration's max |w| overflows, or one 2^100
    above it, forces the re-fold (fold 2): the same integers as a two-pass fold of the
    iteration, so bit-identical estimates and histogram.  The fused fold differs from
    them only in the truncation of each event's digits (below 2^-54 of it)."""
    cfg = W.config("w_plus")
    n = 50_000
    mk = lambda: P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=n)
    a = mk()
    assert a.iterate(n)["fold"] == 0
    a.refine()
    blob = a.get_state()
    valid, e1 = struct.unpack_from("<2i", blob, struct.calcsize("<Q3iIQ"))
    assert valid == 1
    r1 = a.iterate(n)
    d1, s1 = a.get_hist()
    assert r1["fold"] == 1
    runs = {}
    for tag, v, e in (("two-pass", 0, 0), ("overflow", 1, e1 - 30), ("far above", 1, e1 + 100)):
        b = mk()
        b.set_state(_with_scale(blob, v, e))
        r = b.iterate(n)
        assert r["fold"] == (0 if v == 0 else 2), tag
        assert r["iteration"] == 1
        runs[tag] = (r, b.get_hist())
    r0, (d0, s0) = runs["two-pass"]
    for tag in ("overflow", "far above"):
        r, (d, s) = runs[tag]
        assert r["I"] == r0["I"] and r["var"] == r0["var"], tag
        assert np.array_equal(d, d0) and np.array_equal(s, s0), tag
    assert abs(r1["I"] / r0["I"] - 1) < 1e-15 and abs(r1["var"] / r0["var"] - 1) < 1e-14
    m = d0 > 0
    assert np.max(np.abs(d1[m] / d0[m] - 1)) < 1e-13
    # a stored scale 2^k above this iteration's max |w|: w^2 is folded at twice the
    # exponent, so its headroom is 2^2k; once that exceeds 2^40 (k > 20 here) the sums
    # are re-folded (bit-identical to the two-pass fold), below it the fused digits keep
    # at least 2^-88 of the largest w^2 and agree with the two-pass fold to rounding
    bt = mk()
    bt.set_state(_with_scale(blob, 0, 0))
    bt.iterate(n)
    wmax = float(np.max(np.abs(bt.get_weights(0, n, with_bins=False))))
    ec1, ec2 = int(np.frexp(wmax)[1]), int(np.frexp(wmax * wmax)[1])
    for k in (12, 18, 20, 21, 24, 30):
        b = mk()
        b.set_state(_with_scale(blob, 1, ec1 + k))
        r = b.iterate(n)
        d, s = b.get_hist()
        refold = ec2 < 2 * (ec1 + k) - 40
        assert r["fold"] == (2 if refold else 1), (k, r["fold"])
        if refold:
            assert r["I"] == r0["I"] and r["var"] == r0["var"], k
            assert np.array_equal(d, d0) and np.array_equal(s, s0), k
        else:
            assert abs(r["I"] / r0["I"] - 1) < 1e-15 and abs(r["var"] / r0["var"] - 1) < 1e-14, k
            assert np.max(np.abs(d[m] / d0[m] - 1)) < 1e-13, k
    # the scale of w^2 is twice that of w; a checkpoint whose pair disagrees is refused
    off = struct.calcsize("<Q3iIQ")
    bad = blob[:off] + struct.pack("<4i", 1, e1, 2 * e1 + 1, 0) + blob[off + 16:]
    with pytest.raises(P.VegasError):
        mk().set_state(bad)


@pytest.mark.parametrize("name", ["w_plus", "ww_4l", "gauss16x255"])
def test_refinement_in_finalisation_equals_refine_kernel(P, name):
    """The finalisation refines the grid from the histogram it just formed (when
    the scratch fits), and vegas_refine then only swaps grid buffers; after
    set_grid the refinement runs as its own kernel.  Both give the same bytes."""
    cfg = GAUSS_MAX if name == "gauss16x255" else W.config(name)
    n = 30_011
    mk = lambda: P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                              cfg["params"], max_events=n)
    a, b = mk(), mk()
    for it in range(3):
        a.iterate(n)
        b.iterate(n)
        b.set_grid(b.get_grid())   # same grid, but forces the separate refinement kernel
        a.refine()
        b.refine()
        assert np.array_equal(a.get_grid(), b.get_grid()), (name, it)


def test_histogram_sums_and_zero_weight_edge_cases(P):
    cfg = W.config("w_plus")
    g = P.Integrator(cfg["process"], 4, 100, 1, 1.5, cfg["params"], max_events=1000)
    r = g.iterate(2)                       # minimum event count
    assert r["n_events"] == 2
    r = g.iterate(1000)
    d, s = g.get_hist()
    assert np.allclose(d.sum(axis=1), s[1], rtol=1e-14)
    w = g.get_weights(0, 1000, with_bins=False)
    assert np.isclose(w.sum(), s[0], rtol=1e-14) and np.isclose((w * w).sum(), s[1], rtol=1e-14)
    r = g.iterate(2)                       # minimum event count, fused fold
    assert r["n_events"] == 2 and r["fold"] in (1, 2)
    w = g.get_weights(0, 2, with_bins=False)
    assert np.isclose(r["I"], w.mean(), rtol=1e-14)


def test_nonfinite_weights_counted(P):
    par = np.concatenate([[9.0], np.ones(3), np.full(3, 0.5)])  # unknown Genz family -> NaN
    g = P.Integrator(W.GENZ, 3, 10, 1, 1.5, par, max_events=500)
    for it in range(3):  # the two-pass fold, then the fused fold with a max |w| of zero
        r = g.iterate(500)
        assert r["n_nonfinite"] == 500 and r["n_nonzero"] == 0 and r["I"] == 0.0 and r["var"] == 0.0
        assert r["fold"] == (0 if it == 0 else 1)
    d, s = g.get_hist()
    assert not d.any() and not s.any()


def test_errors_and_call_order(P):
    cfg = W.config("dy_z")
    g = P.Integrator(cfg["process"], 3, 50, 1, 1.5, cfg["params"], max_events=100)
    with pytest.raises(P.VegasError) as e:
        g.refine()
    assert e.value.status == -2
    with pytest.raises(P.VegasError):
        g.iterate(101)
    with pytest.raises(P.VegasError):
        g.iterate(1)
    with pytest.raises(P.VegasError):
        g.result()
    with pytest.raises(P.VegasError):
        g.set_grid(np.zeros((3, 51)))
    g.iterate(100)
    g.refine()
    with pytest.raises(P.VegasError):
        g.refine()                      # one refine per iteration


def test_full_size_sampled_parity_bench_workload(P):
    """The measured workload (W+ at 1e6 events, default launch): sampled events
    recomputed one by one by the oracle at the same grid."""
    cfg = W.config("w_plus")
    n = cfg["n_events"]
    g, o = make_pair(P, cfg, n)
    for it in range(3):
        g.iterate(n)
        g.refine()
    o.set_grid(g.get_grid())
    g.iterate(n)
    wg = g.get_weights(0, n, with_bins=False)
    idx = np.arange(0, n, 997)
    wo = np.array([o.event_weights(3, int(i), 1)[0][0] for i in idx])
    compare_weights(wg[idx], wo, "w_plus full size")
    # the tail of the launch
    wt, _ = o.event_weights(3, n - 300, 300)
    compare_weights(wg[n - 300:], wt, "w_plus tail")


@pytest.mark.parametrize("name,prec", [("ww_4l", "fp64"), ("ww_4l", "fp32me"), ("ww_had", "fp64")])
def test_full_size_sampled_parity_ww(P, name, prec):
    """W+W- (partonic, and hadronic in 10 dims) at the measured size (1e7 events per
    iteration, default launch): every 9973rd event and the launch's last 300
    recomputed one by one by the oracle at the same grid (bins bit-exact; weights
    to 1e-12 in FP64, to the binary32 bars max 2e-4 / mean 2e-6 in FP32-ME), and
    the iteration's I and var equal to the mean and variance of all 1e7 weights."""
    cfg = W.config(name)
    n = cfg["n_events"]
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"],
                     precision=P.FP32_ME if prec == "fp32me" else P.FP64, max_events=n)
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
    for _ in range(2):
        g.iterate(n)
        g.refine()
    o.set_grid(g.get_grid())
    r = g.iterate(n)
    wg, bg = g.get_weights(0, n)
    idx = np.concatenate([np.arange(0, n - 300, 9973), np.arange(n - 300, n)])
    wo = np.empty(len(idx))
    bo = np.empty((len(idx), cfg["ndim"]), dtype=bg.dtype)
    for k, i in enumerate(idx):
        w1, b1 = o.event_weights(2, int(i), 1)
        wo[k], bo[k] = w1[0], b1[0]
    assert np.array_equal(bg[idx], bo), "bin indices differ"
    if prec == "fp64":
        compare_weights(wg[idx], wo, f"{name} full size")
    else:
        m = wo != 0
        e = np.abs(wg[idx][m] - wo[m]) / np.abs(wo[m])
        assert e.max() <= 2e-4 and e.mean() <= 2e-6, (e.max(), e.mean())
    mean = np.sum(wg) / n
    var = (np.sum(wg * wg) / n - mean * mean) / (n - 1)
    assert rel(r["I"], mean) < 1e-12
    assert rel(r["var"], var) < 1e-9
    assert r["n_events"] == n and r["n_nonzero"] == int(np.count_nonzero(wg))


def test_stage_timing_and_launch_shape(P):
    """Kernel timing per stage: only the selected stages are timed (one event-kernel,
    one column-sum and one finalisation launch per iteration after the first), the
    times are positive, timing changes no result, and the reported launch shape is
    the one the iteration used."""
    cfg = W.config("w_plus")
    n = 100_000
    g, _ = make_pair(P, cfg, n)
    h = make_pair(P, cfg, n)[0]
    for x in (g, h):
        x.iterate(n)
        x.refine()
    g.set_timing(True, stages=("event",))
    g.stage_times(reset=True)
    ra = [g.iterate(n) for _ in range(2)]
    st = g.stage_times(reset=True)
    assert st["event"][1] == 2 and st["event"][0] > 0
    assert st["fold"][1] == st["finalize"][1] == st["refine"][1] == 0
    g.set_timing(True)
    g.iterate(n)
    st = g.stage_times(reset=True)
    assert st["event"][1] == st["fold"][1] == st["finalize"][1] == 1
    g.set_timing(False)
    g.iterate(n)
    assert sum(v[1] for v in g.stage_times().values()) == 0
    rb = [h.iterate(n) for _ in range(2)]
    assert [r["I"] for r in ra] == [r["I"] for r in rb] and [r["var"] for r in ra] == [r["var"] for r in rb]
    shape = g.last_launch()
    assert shape["threads"] % 64 == 0 and shape["event_blocks"] >= 1
    assert shape["fold_cols"] == 7 + 4 * cfg["ndim"] * cfg["nbins"]
    assert 1 <= shape["fold_rows"] <= 1024
    from paper_1503_06182_amd import vegas as V
    assert g._L.vegas_set_timing(g._h, 16) == V.EINVAL     # a stage mask outside 0..15
    assert g._L.vegas_set_timing(g._h, -1) == V.EINVAL


def test_empty_iteration_and_iteration_cap(P):
    """n_events 0 or negative is an error; VEGAS_MAX_ITER iterations are allowed and
    the next is refused (ESTATE), while the combination over all of them, a
    checkpoint and its restore still work."""
    from paper_1503_06182_amd import vegas as V
    g = P.Integrator(W.GAUSS, 2, 10, 3, 1.5, [0.5, 0.2], max_events=256)
    for bad in (0, -5):
        with pytest.raises(P.VegasError) as e:
            g.iterate(bad)
        assert e.value.status == V.EINVAL
    for _ in range(V.MAX_ITER):
        g.iterate(64, sync=False)
    with pytest.raises(P.VegasError) as e:
        g.iterate(64)
    assert e.value.status == V.ESTATE
    r = g.result()
    assert r["n_iter"] == V.MAX_ITER and r["sigma"] > 0
    assert g.result(first=V.MAX_ITER - 1)["n_iter"] == 1
    blob = g.get_state()
    h = P.Integrator(W.GAUSS, 2, 10, 3, 1.5, [0.5, 0.2], max_events=256)
    h.set_state(blob)
    assert h.result() == r
    with pytest.raises(P.VegasError):
        h.iterate(64)
