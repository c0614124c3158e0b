"""vegas_run_schedule: a whole schedule recorded once as a HIP graph and replayed.

The recorded form must give the same bits as the same calls made one by one (the
two-stage schedule of the timing runs in Sec. 3.2: 4 x 1,000 then 10 x 10,000 events,
refined after each iteration): on the first call (recording), on every replay from the
same state (restored with vegas_set_state, other handles' plain work and stream
synchronisations between the replays), after a change of schedule (a new recording),
and when the iteration index differs from the recorded one (recorded anew, not
replayed).  The combination is also checked against the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

SCHED = [1000] * 4 + [10_000] * 10


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1503_06182_amd as P
    P.load()
    return P


def make(P, cfg, n):
    return P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                        cfg["params"], max_events=n)


def snapshot(g, first=0):
    r = g.result(first=first)
    d, s = g.get_hist()
    return (np.array([r["I"], r["sigma"], r["chi2_dof"], r["n_iter"]]).tobytes() + g.get_grid().tobytes()
            + d.tobytes() + s.tobytes() + g.get_state())


def eager(P, cfg, sched, start=None):
    g = make(P, cfg, max(SCHED))
    if start is not None:
        g.set_state(start)
    for n in sched:
        g.iterate(n, sync=False)
        g.refine()
    return g


def test_recorded_schedule_equals_plain_calls_on_every_replay(P):
    cfg = W.config("ww_4l")
    ref = snapshot(eager(P, cfg, SCHED))
    g = make(P, cfg, max(SCHED))
    s0 = g.get_state()
    g.run_schedule(SCHED)  # records, then launches the graph
    assert snapshot(g) == ref, "recording"
    other = make(P, W.config("dy_z"), 10_000)
    for k in range(4):
        g.set_state(s0)
        g.run_schedule(SCHED)  # replays
        assert snapshot(g) == ref, f"replay {k}"
        other.iterate(10_000)  # plain work on another handle between the replays
        other.refine()


def test_new_schedule_and_other_start_record_anew(P):
    cfg = W.config("ww_4l")
    g = make(P, cfg, max(SCHED))
    s0 = g.get_state()
    g.run_schedule(SCHED)
    # another schedule from the same state: recorded anew
    short = [2000] * 3
    g.set_state(s0)
    g.run_schedule(short)
    assert snapshot(g) == snapshot(eager(P, cfg, short))
    # the first schedule again, now from the state after it (iteration 14): not the
    # recorded start, so recorded anew -- the plain continuation's bits
    g.set_state(s0)
    g.run_schedule(SCHED)
    mid = g.get_state()
    g.run_schedule(SCHED[:3])
    assert snapshot(g) == snapshot(eager(P, cfg, SCHED[:3], start=mid))
    # and without refinement
    g.set_state(s0)
    g.run_schedule(short, refine=False)
    h = make(P, cfg, max(SCHED))
    for n in short:
        h.iterate(n, sync=False)
    assert g.get_state() == h.get_state()


def test_recorded_schedule_against_the_oracle(P):
    cfg = W.config("ww_4l")
    g = make(P, cfg, max(SCHED))
    g.run_schedule(SCHED)
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
    for n in SCHED:
        o.iterate(n)
        o.refine()
    for first in (0, 4):
        rg, ro = g.result(first=first), o.result(first=first)
        assert rg["n_iter"] == ro["n_iter"]
        assert abs(rg["I"] - ro["I"]) <= 1e-10 * abs(ro["I"])
        assert abs(rg["sigma"] - ro["sigma"]) <= 1e-8 * ro["sigma"]


def test_schedule_arguments_are_checked(P):
    cfg = W.config("ww_4l")
    g = make(P, cfg, 10_000)
    with pytest.raises(P.VegasError):
        g.run_schedule([])
    with pytest.raises(P.VegasError):
        g.run_schedule([1000, 20_000])  # above max_events
    with pytest.raises(P.VegasError):
        g.run_schedule([1])
    # a rejected call leaves the handle as it was
    g.run_schedule([1000])
    assert g.result()["n_iter"] == 1
