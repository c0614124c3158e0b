"""Benchmark of the per-event VEGAS iteration on one MI355X.

Workload (default): q qbar -> W+W- -> e+ nu mu- nubar at sqrt(shat) = 500 GeV,
tree-level helicity amplitudes, 8 dimensions (two Breit-Wigner masses and the
sequential two-body decays), 100 bins per dimension, 1e7 events per iteration,
binary64, seed 1.  One step = one full VEGAS iteration: events -> exact
accumulation -> finalisation (vegas_iterate) -> grid refinement (vegas_refine;
the grid adapts over the configuration's 10 iterations and is kept afterwards,
the same kernels running every step).

Warm-up: 0.2 s of the same steps on a throwaway handle (the clocks settle over the
first tens of milliseconds of sustained load), then --warmup W (default 2) untimed
steps on the measured handle and K = --steps (default 10) timed steps.

Prints one JSON line: events/s over the timed steps, the variance-weighted
effective events/s 1/(eps^2 T) of the timed iterations' combined estimate, the
roofline of the dominant kernel (timed with HIP events on the library's own
stream), the same measurement with the matrix element in binary32 (fp32_me) and
with the learned proposal (flow), each with its ratio of effective events/s to
plain binary64 VEGAS, the serial CPU oracle timed on a bounded sample on this
host (cpu_baseline) and the paper's threaded CPU scheme on all of this host's
cores (cpu_baseline_all_cores).
"""
from __future__ import annotations

import argparse
import json
import os
import struct
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Work per event of the event kernel (the dominant kernel).
#  algorithmic_f64: the FP64 FLOPs of the method per event with the amplitudes as the
#    kernels state them, counted on the host by tests/flopcount/count.cpp (the integrand
#    headers compiled with a counting scalar: add, sub, mul = 1, fma = 2; each evaluation
#    of a mathematical function -- division or reciprocal, square root, tan, sine and
#    cosine of an angle, atan, log, exp, expm1 -- at what one call of the library's
#    version costs, OCML_FLOP_PER_CALL, however the kernel evaluates it; work on uniform
#    values not counted), through a grid the oracle adapted for five iterations; plus the
#    grid map, the uniforms and the accumulation (S1, w^2, S2, one addition per
#    dimension).  tests/test_flop_count.py recounts it.  This is the roofline's numerator.
#  f64 / f32: the FLOPs the kernel as built executes per event, from the rocprofv3
#    counter SQ_INSTS_VALU_FLOPS_FP64 (FP32) x 64 lanes / events (add, mul,
#    transcendental instruction = 1, fma = 2), reported beside it as the VALU
#    utilisation; it includes the fixed-point fold's digit split and both sides of
#    selects.
#  traffic: HBM bytes of one launch at the workload's default event count (FETCH_SIZE
#    x 2 + WRITE_SIZE x 1 KiB, the factors read from a plain 1 GiB device copy).
# The counter summaries are under profiles/.
EVENT_KERNEL_WORK = {
    ("w_plus", "fp64"): {"algorithmic_f64": 373.5, "f64": 325.2, "f32": 0.0, "traffic": 22_169_771,
                         "events": 1_000_000},
    ("ww_4l", "fp64"): {"algorithmic_f64": 1262.7, "f64": 1033.7, "f32": 0.0, "traffic": 180_107_630,
                        "events": 10_000_000},
    ("ww_4l", "fp32me"): {"algorithmic_f64": None, "f64": 636.7, "f32": 418.0, "traffic": None,
                          "events": 10_000_000},
    ("ww_had", "fp64"): {"algorithmic_f64": 1589.8, "f64": 1319.1, "f32": 0.0, "traffic": 216_902_407,
                         "events": 10_000_000},
}
# FP64 FLOPs of one call of the library's version of each mathematical function the
# integrands evaluate, measured on gfx950 with tests/flopcount/ocml_price.hip under
# rocprofv3 (SQ_INSTS_VALU_FLOPS_FP64 x 64 / calls, arguments spread over the ranges the
# integrands pass; div is 1.0 / x, sincos one sincos() call)
OCML_FLOP_PER_CALL = {"atan": 58.0, "log": 79.0, "exp": 27.0, "expm1": 32.0, "tan": 88.0, "sincos": 57.0,
                      "sqrt": 17.0, "div": 14.0}
# HBM bytes of one histogram-stage launch (k_accsum), from the same counters, at the
# workload's default event count
HIST_STAGE_TRAFFIC = {("w_plus", 1_000_000): 10_180_818, ("ww_4l", 10_000_000): 20_433_037}
# FP64 FLOPs of the adjoint's event kernel per (event, parameter point), and its HBM
# bytes per call at 64 points x 1e6 events, from the same kind of counter runs
ADJOINT_KERNEL_WORK = {"f64": 264.1, "traffic": 48_201_677, "events": 1_000_000}
# matrix-core FLOPs of one coupling layer per event: the algorithmic work of the two
# 128-wide products, 2 x (128 x 128 + 128 x 188) per event (the kernel pads the 188
# spline parameters to 192 columns; the padding is not counted as work)
FLOW_LAYER_MFMA_FLOP = 2 * (128 * 128 + 128 * 188)
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP64_VALU_TFLOPS = 78.6
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def roofline(workload, precision, n_events, avg_launch_s):
    """The event kernel against the VALU peak: achieved = algorithmic FLOPs per launch /
    average launch time.  Beside it, the FLOPs the kernel executed (rocprof counters) as
    the VALU utilisation; for the mixed FP64/FP32 kernel (no algorithmic count) the
    executed FLOPs are the numerator and frac is the sum of the two pipes' fractions."""
    work = EVENT_KERNEL_WORK.get((workload, precision))
    roof = {"kernel": "k_event", "bound": "alu", "achieved": None, "peak": PEAK_FP64_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": None, "traffic": None, "avg_launch_ms": avg_launch_s * 1e3}
    if work is None or avg_launch_s <= 0:
        return roof
    f64 = work["f64"] * n_events / avg_launch_s / 1e12
    f32 = work["f32"] * n_events / avg_launch_s / 1e12
    util = f64 / PEAK_FP64_VALU_TFLOPS + f32 / PEAK_FP32_VALU_TFLOPS
    if work["algorithmic_f64"] is not None:
        alg = work["algorithmic_f64"] * n_events / avg_launch_s / 1e12
        roof.update(achieved=alg, frac=alg / PEAK_FP64_VALU_TFLOPS,
                    flop_per_event={"algorithmic_f64": work["algorithmic_f64"]})
    else:
        roof.update(achieved=f64 + f32, frac=util, flop_per_event={})
    roof["flop_per_event"].update(executed_f64=work["f64"], executed_f32=work["f32"])
    roof.update(executed_tflops_f64=f64, executed_tflops_f32=f32, valu_flop_utilisation=util)
    if work.get("events") == n_events:
        roof["traffic"] = work["traffic"]
    return roof


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default: 2 for the VEGAS iteration, whose grid they adapt; "
                         "as many as fill 0.2 s for the other workloads)")
    ap.add_argument("--workload", default="ww_4l",
                    choices=["w_plus", "dy_z", "ww_4l", "ww_had", "ww_4l_paper", "adjoint", "flow"])
    ap.add_argument("--clock-warmup", type=float, default=0.2, metavar="SECONDS",
                    help="seconds of steps on a throwaway handle before the VEGAS-iteration schedule")
    ap.add_argument("--train-events", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--events", type=int, default=0, help="events per iteration (0: workload's)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32me"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="only the headline measurement (no fp32_me, flow, observable or strata legs)")
    ap.add_argument("--strata", type=int, default=-1,
                    help="strata per axis of the stratified leg (-1: floor((N/2)^(1/D)), Lepage's choice; 0: skip)")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle iterations (0: the workload's sample)")
    ap.add_argument("--cpu-events", type=int, default=0,
                    help="events per oracle iteration (0: the workload's sample, 10-30 s of host time)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration)")
    return ap.parse_args()


def warm_up(args, step, min_s=0.2, cap=2000):
    """Untimed steps before the timed region: exactly --warmup if given, else steps
    until 0.2 s of them have run (at least 2, at most cap) -- under sustained load the
    clocks settle over the first tens of milliseconds.  Only for steps that leave the
    state unchanged (the VEGAS iteration refines its grid: see clock_warm_up).
    Returns the count."""
    import torch
    if args.warmup is not None:
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        return args.warmup
    n = 0
    t0 = time.perf_counter()
    while n < 2 or (n < cap and time.perf_counter() - t0 < min_s):
        step()
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return n


def clock_warm_up(make, step, seconds=0.2, cap=2000):
    """The same steps on a throwaway handle for `seconds`, so that the measured handle
    starts at settled clocks without running more iterations than its schedule:
    continued refinement at a fixed event count lets the grid's bin widths start to
    alternate after a few tens of iterations, and the timed iterations are meant to
    be those of the configuration's schedule."""
    import torch
    h = make()
    n = 0
    t0 = time.perf_counter()
    while n < 2 or (n < cap and time.perf_counter() - t0 < seconds):
        step(h)
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    h.close()
    return time.perf_counter() - t0


def copy_calibration(nbytes):
    """A plain device-to-device copy of known size, for scaling the HBM byte counters."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "read": nbytes, "written": nbytes}))


def combine(history):
    """Inverse-variance combination of (I_j, var_j) pairs (for the report)."""
    ws = sum(1.0 / v for _, v in history)
    I = sum(i / v for i, v in history) / ws
    return I, (1.0 / ws) ** 0.5


def history_from_state(blob, ndim, nbins):
    head = struct.calcsize("<Q4iQ4i")
    _magic, _proc, _nd, _nb, it, _seed = struct.unpack_from("<Q3iIQ", blob, 0)
    off = head + 8 * ndim * (nbins + 1)
    vals = struct.unpack_from(f"<{2 * it}d", blob, off)
    return [(vals[2 * j], vals[2 * j + 1]) for j in range(it)]


def host_info():
    """The host CPU the baselines ran on: model name, logical CPUs, CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_threads():
    """Threads for the all-core baseline: the CPUs this process may use, at most the
    OMP_NUM_THREADS the environment grants (the GPU host's share)."""
    n = host_info()["usable_cpus"] or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def cpu_baseline(cfg, iters, events):
    import oracle
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    t0 = time.perf_counter()
    for _ in range(iters):
        o.iterate(events)
        o.refine()
    dt = time.perf_counter() - t0
    return {"value": iters * events / dt, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} iterations x {events} events of the same workload, serial "
                      f"FP64 C oracle on one host core, {dt:.1f} s", **host_info()}


def cpu_baseline_all_cores(cfg, iters, events):
    """The paper's CPU scheme (Sec. 2.2) on all usable host cores: the oracle's event
    loop split into fixed per-thread chunks, the partial sums added in chunk order."""
    import oracle
    T = cpu_threads()
    o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"])
    t0 = time.perf_counter()
    for _ in range(iters):
        o.iterate_threads(events, T)
        o.refine()
    dt = time.perf_counter() - t0
    return {"value": iters * events / dt, "unit": "events/s", "cores": T,
            "kind": "oracle, threaded (fixed chunks, fixed-order combine)",
            "sample": f"{iters} iterations x {events} events of the same workload, FP64 C oracle "
                      f"on {T} threads (OpenMP), {dt:.1f} s", **host_info()}


# the paper's own timings, as context (other hardware, another integrand: MCFM's
# pp -> H(-> b bbar) + 2 jets, 104,000 events of the 4 x 1,000 + 10 x 10,000 schedule)
PAPER_CONTEXT = {
    "note": "Sec. 3.2, Tables 1-8: H+2 jets, 10 (LO) / 13 (NLO) dims, 104,000 events per run",
    "lo_best_events_per_s": {"value": 104000 / 0.26, "hardware": "2x Xeon X5650, 12 threads (Table 2)"},
    "lo_i7_8_threads_events_per_s": {"value": 104000 / 0.32, "hardware": "Core i7-4770, 8 threads (Table 1)"},
    "lo_phi_best_events_per_s": {"value": 104000 / 1.39, "hardware": "Xeon Phi 5110P, 32 threads (Table 4)"},
    "nlo_best_events_per_s": {"value": 104000 / 25.36, "hardware": "4x Opteron 6128 HE, 32 threads (Table 7)"},
}


def bench_paper_schedule(args):
    """The W+W- integrand on the two-stage schedule of the paper's timing runs
    (4 x 1,000 + 10 x 10,000 events, grid refined after every iteration, the warm-up
    stage dropped from the result).  One step = the whole schedule from the uniform
    grid (the state is restored between steps, outside the timed region); at these
    sizes the iteration is bound by launch and synchronisation latency."""
    import torch

    import paper_1503_06182_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    cfg = W.config("ww_4l_paper")
    sched, first = cfg["schedule"], cfg["discard_first"]
    g = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                     cfg["params"], max_events=max(sched))
    s0 = g.get_state()

    def one_by_one():
        g.set_state(s0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in sched:
            g.iterate(n, sync=False)
            g.refine()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    def recorded():
        # the same schedule through vegas_run_schedule: recorded as a HIP graph on the
        # first call, replayed from the restored state on every later one
        g.set_state(s0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.run_schedule(sched)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    Wn = warm_up(args, one_by_one)
    times_calls = [one_by_one() for _ in range(args.steps)]
    r_calls = g.result(first=first)
    warm_up(args, recorded)
    times = [recorded() for _ in range(args.steps)]
    T = sum(times)
    r, rall = g.result(first=first), g.result()
    assert r == r_calls, "the recorded schedule must give the plain calls' result"
    eps = r["sigma"] / abs(r["I"])
    one = one_by_one  # the timing pass binds HIP events to each dispatch: calls one by one
    # event-kernel time per schedule from a pass with HIP events bound to each dispatch
    g.set_timing(True)
    g.stage_times(reset=True)
    one()
    st = g.stage_times()
    g.set_timing(False)
    ms_ev = st["event"][0]
    flop = EVENT_KERNEL_WORK[("ww_4l", "fp64")]["algorithmic_f64"] * sum(sched)
    roof = {"kernel": "k_event", "bound": "alu", "achieved": flop / (ms_ev * 1e-3) / 1e12,
            "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": flop / (ms_ev * 1e-3) / 1e12 / PEAK_FP64_VALU_TFLOPS, "traffic": None,
            "avg_launch_ms": ms_ev / st["event"][1],
            "note": "14 launches of 1e3 and 1e4 events: launch-latency bound"}
    n_step = sum(sched)
    line = {
        "metric": "events/s and effective events/s (1/var) at 1e-3 rel. error, 1 MI355X",
        "value": args.steps * n_step / T, "unit": "events/s", "n_gpus": 1,
        "steps": args.steps, "warmup": Wn, "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (counter-based Philox stream, seed 1)",
        "config": {"workload": "ww_4l_paper", "schedule": "4x1000+10x10000", "ndim": cfg["ndim"],
                   "nbins": cfg["nbins"], "discard_first": first},
        "effective_events_per_s": 1.0 / (eps * eps * (T / args.steps)),
        "ms_per_step_min_avg_max": [min(times) * 1e3, T / args.steps * 1e3, max(times) * 1e3],
        "ms_per_iteration": T / args.steps / len(sched) * 1e3,
        "integral_pb": r["I"], "rel_error": eps, "chi2_dof": r["chi2_dof"],
        "integral_all_iterations_pb": rall["I"],
        "kernel_ms_per_step": {k: v[0] for k, v in st.items()},
        "roofline": roof,
        "calls_one_by_one": {"ms_per_step": sum(times_calls) / args.steps * 1e3,
                             "ms_per_step_min_avg_max": [min(times_calls) * 1e3,
                                                         sum(times_calls) / args.steps * 1e3,
                                                         max(times_calls) * 1e3],
                             "ms_per_iteration": sum(times_calls) / args.steps / len(sched) * 1e3,
                             "events_per_s": args.steps * sum(sched) / sum(times_calls)},
        "path": "vegas_run_schedule (the schedule's launches recorded once as a HIP graph, replayed)",
    }
    if not args.no_cpu_baseline:
        import oracle
        reps = 20                              # about 12 s of one host core
        o_t = 0.0
        for _ in range(reps):
            o = oracle.Vegas(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                             cfg["params"])
            t0 = time.perf_counter()
            for n in sched:
                o.iterate(n)
                o.refine()
            o_t += time.perf_counter() - t0
        line["cpu_baseline"] = {"value": reps * n_step / o_t, "unit": "events/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"{reps} runs of the whole schedule, serial FP64 C oracle on "
                                          f"one host core, {o_t:.1f} s"}
    g.close()
    print(json.dumps(line), flush=True)


def bench_adjoint(args):
    """Drell-Yan adjoint: 64 parameter points x 1e6 events, FP64, at the grid reached
    after the workload's 5 iterations; one step = one vegas_grad call."""
    import torch

    import paper_1503_06182_amd as P
    import workloads as W
    torch.cuda.set_device(0)
    cfg = W.config("dy_z")
    g = P.Integrator(cfg["process"], 3, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"],
                     max_events=cfg["n_events"])
    for _ in range(cfg["n_iter"]):
        g.iterate(cfg["n_events"])
        g.refine()
    theta = torch.tensor(W.adjoint_points(64), device="cuda")
    N = args.events or 1_000_000
    Wn = warm_up(args, lambda: g.grad(theta, N, 5))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sig, ds = g.grad(theta, N, 5)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    # kernel durations: K more calls with HIP events bound to each dispatch (the
    # adjoint's event kernel is timed as the events stage, its tree as the fold)
    g.set_timing(True)
    g.stage_times(reset=True)
    for _ in range(args.steps):
        g.grad(theta, N, 5)
    torch.cuda.synchronize()
    st = g.stage_times()
    g.set_timing(False)
    avg = st["event"][0] / max(st["event"][1], 1) * 1e-3
    work = ADJOINT_KERNEL_WORK
    f64 = work["f64"] * N * 64 / avg / 1e12 if avg > 0 and work["f64"] else None
    roof = {"kernel": "k_dy_grad", "bound": "alu", "achieved": f64, "peak": PEAK_FP64_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": f64 / PEAK_FP64_VALU_TFLOPS if f64 else None,
            "traffic": work["traffic"] if N == work["events"] else None, "avg_launch_ms": avg * 1e3,
            "flop_per_point_event": work["f64"]}
    line = {"metric": "adjoint point-events/s (sigma and 5 derivatives per point and event)",
            "value": args.steps * N * 64 / T, "unit": "point-events/s", "n_gpus": 1,
            "steps": args.steps, "warmup": Wn, "ms_per_step": T / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "adjoint", "points": 64, "events": N},
            "sigma_mean_pb": float(sig.mean()),
            "kernel_ms_per_step": {k: v[0] / args.steps for k, v in st.items() if k != "refine"},
            "roofline": roof}
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.Vegas(cfg["process"], 3, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
        for _ in range(cfg["n_iter"]):
            o.iterate(cfg["n_events"])
            o.refine()
        pts, ns = W.adjoint_points(64)[::4], 600_000        # about 10 s of one host core
        t0 = time.perf_counter()
        for th in pts:
            o.dy_grad(5, ns, th)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": len(pts) * ns / dt, "unit": "point-events/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"{len(pts)} of the 64 points x {ns} events, dual-number FP64 C "
                                          f"oracle on one host core, {dt:.1f} s"}
    print(json.dumps(line), flush=True)


def bench_flow(args, emit=True):
    """Learned proposal on the W+W- integrand: the VEGAS grid converged (10 x 1e7),
    the flow trained on 1e6 events of one more VEGAS iteration (Adam, lr 1e-3, batch
    4096, 20 epochs), then K iterations of 1e7 events with the flow and K with plain
    VEGAS on the same frozen grid.  One step = one flow iteration.  emit=False: no
    CPU baseline, nothing printed, the line returned (the flow leg of the default
    benchmark)."""
    import torch

    import paper_1503_06182_amd as P
    import workloads as W
    torch.cuda.set_device(0)
    cfg = W.config("ww_4l")
    N = args.events or cfg["n_events"]
    g = P.Integrator(cfg["process"], 8, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"], max_events=N)
    for _ in range(cfg["n_iter"]):
        g.iterate(N, sync=False)
        g.refine()
    g.iterate(args.train_events)
    y, w = g.export(0, args.train_events)
    f = P.Flow(max_batch=4096, max_sample=N, seed=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = P.train(f, y, w, epochs=args.epochs, batch=4096, lr=1e-3, log_every=1000)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps_train = f.steps

    def run(kind, k):
        rs = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            rs.append(g.iterate_flow(f, N) if kind == "flow" else g.iterate(N))
        torch.cuda.synchronize()
        return rs, time.perf_counter() - t

    Wn = warm_up(args, lambda: (g.iterate_flow(f, N), g.iterate(N)))
    rf, tf = run("flow", args.steps)
    rv, tv = run("vegas", args.steps)
    If, sf = combine([(r["I"], r["var"]) for r in rf])
    Iv, sv = combine([(r["I"], r["var"]) for r in rv])
    eff_f = 1.0 / ((sf / If) ** 2 * tf)
    eff_v = 1.0 / ((sv / Iv) ** 2 * tv)
    relvar_f = sum(r["var"] * N / r["I"] ** 2 for r in rf) / len(rf)
    relvar_v = sum(r["var"] * N / r["I"] ** 2 for r in rv) / len(rv)
    # the matrix-core roofline of the sampling layers: Flow.sample of N points (the six
    # k_flow_layer<true> launches a flow iteration runs), HIP events on the flow's stream
    zs = torch.rand(N, 8, device="cuda", dtype=torch.float32)
    f.sample(zs)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        f.sample(zs)
    e1.record()
    torch.cuda.synchronize()
    t_layer = e0.elapsed_time(e1) * 1e-3 / reps / 6
    mfma = FLOW_LAYER_MFMA_FLOP * N / t_layer / 1e12
    roof = {"kernel": "k_flow_layer<true> (one coupling layer, sampling)", "bound": "mfma", "achieved": mfma,
            "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s", "frac": mfma / PEAK_BF16_MFMA_TFLOPS,
            "traffic": None, "avg_launch_ms": t_layer * 1e3, "flop_per_event": FLOW_LAYER_MFMA_FLOP}
    del zs
    line = {"metric": "events/s and effective events/s (1/var) at 1e-3 rel. error, 1 MI355X",
            "value": args.steps * N / tf, "unit": "events/s", "n_gpus": 1, "steps": args.steps,
            "warmup": Wn, "ms_per_step": tf / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "bf16-mlp/f32-spline/f64-weight",
            "data": "synthetic (counter-based Philox stream, seed 1; parametric PDFs)",
            "config": {"workload": "flow", "integrand": "ww_4l", "events_per_iteration": N,
                       "train_events": args.train_events, "epochs": args.epochs, "batch": 4096},
            "effective_events_per_s": eff_f, "vegas_events_per_s": args.steps * N / tv,
            "vegas_effective_events_per_s": eff_v, "effective_gain_vs_vegas": eff_f / eff_v,
            "per_event_rel_variance": {"flow": relvar_f, "vegas": relvar_v},
            "flow_uses": "flow" if eff_f > eff_v else "vegas (fallback)",
            "integral_pb": {"flow": If, "flow_sigma": sf, "vegas": Iv, "vegas_sigma": sv},
            "training": {"seconds": t_train, "steps": steps_train, "loss_first": losses[0][1],
                         "loss_last": losses[-1][1]},
            "roofline": roof}
    if not emit:
        g.close()
        f.close()
        return line
    if not args.no_cpu_baseline:
        # the oracle's flow iteration on a bounded sample: z from the counter stream,
        # y = F^-1(z) by the float64 flow oracle, w = J f / q by the C oracle
        import math

        import numpy as np

        import oracle
        import oracle.flow as OF
        theta = f.get_params().cpu().to(torch.float64)
        o = oracle.Vegas(cfg["process"], 8, cfg["nbins"], cfg["seed"], cfg["alpha"], cfg["params"])
        o.set_grid(g.get_grid())
        ns, chunk, it = 400_000, 20_000, rf[0]["iteration"]      # about 10 s
        t0 = time.perf_counter()
        for c0 in range(0, ns, chunk):
            z = torch.tensor(np.array([oracle.uniforms(cfg["seed"], it, i, 8)
                                       for i in range(c0, c0 + chunk)]))
            yo, lqo = OF.sample(z, theta)
            yo, lqo = yo.numpy(), lqo.numpy()
            for k in range(chunk):
                x, J, _ = o.grid_map(np.clip(yo[k], 2.0 ** -40, 1.0 - 2.0 ** -40))
                J * oracle.integrand(cfg["process"], cfg["params"], x) * math.exp(-lqo[k])
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": ns / dt, "unit": "events/s", "cores": torch.get_num_threads(),
                                "kind": "oracle",
                                "sample": f"{ns} events of a flow iteration: float64 PyTorch flow oracle "
                                          f"(up to {torch.get_num_threads()} threads) and the FP64 C oracle's "
                                          f"map and integrand, {dt:.1f} s"}
    print(json.dumps(line), flush=True)


# the observable histogram of each measured workload: (bins, lo, hi) -- the lepton-pair
# mass over the Drell-Yan window, the e+ p_T over its Jacobian peak, the e+ nu mass
OBS_BINNING = {"dy_z": (40, 81.0, 101.0), "w_plus": (50, 20.0, 70.0), "ww_4l": (60, 60.0, 100.0),
               "ww_had": (60, 60.0, 100.0)}
# the CPU baseline's sample per workload, (iterations, events per iteration), about
# 10-30 s of one host core: iterations of the workload's own size where it is small
CPU_SAMPLE = {"w_plus": (6, 10_000_000), "dy_z": (2000, 10_000), "ww_4l": (5, 400_000),
              "ww_had": (5, 500_000)}
# the all-core baseline's sample, about 10 s on 16 threads
CPU_SAMPLE_ALL_CORES = {"w_plus": (10, 10_000_000), "dy_z": (2000, 10_000), "ww_4l": (4, 2_500_000),
                        "ww_had": (4, 2_000_000)}


def observable_leg(args, make, Wn, N, plain_ms_min, plain_event):
    """The same steps with the observable histogram filled: ms per step (min over 10
    blocks of K steps, like the plain path's) and the event kernel's average, so the
    cost of the histogram is read against the plain path measured just before."""
    import torch
    nb, lo, hi = OBS_BINNING[args.workload]
    g = make()
    g.set_observable(nb, lo, hi, first=Wn)
    for _ in range(Wn):
        g.iterate(N, sync=False)
        g.refine()
    reps = []
    for _ in range(10):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            g.iterate(N, sync=False)
            g.refine()
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - t1) / args.steps * 1e3)
    g.set_timing(True)
    g.stage_times(reset=True)
    for _ in range(args.steps):
        g.iterate(N, sync=False)
        g.refine()
    torch.cuda.synchronize()
    st = g.stage_times()
    shape = g.last_launch()
    g.close()
    ev = st["event"][0] / max(st["event"][1], 1)
    ev_plain = plain_event[0] / max(plain_event[1], 1)
    return {"bins": nb, "range": [lo, hi], "first_combined": Wn,
            "ms_per_step_min": min(reps), "ms_per_step_min_plain": plain_ms_min,
            "step_overhead": min(reps) / plain_ms_min - 1.0,
            "event_kernel_ms": ev, "event_kernel_ms_plain": ev_plain,
            "event_kernel_overhead": ev / ev_plain - 1.0 if ev_plain > 0 else None,
            "kernel_ms_per_step": {k: v[0] / args.steps for k, v in st.items()},
            "fold_cols": shape["fold_cols"]}


def strata_run(args, make, Wn, N, m, beta, plain_ms_min, plain_hist):
    """The same steps with stratified sampling (m strata per axis; beta > 0: adaptive
    counts): ms per step (min over 10 blocks of K steps), and the timed iterations'
    combined relative error against the plain path's over the same iteration
    numbers, as effective events/s 1 / (eps^2 T)."""
    import torch
    g = make()
    g.set_strata(m)
    if beta > 0:
        g.set_strata_beta(beta)
    H = m ** g.ndim
    for _ in range(Wn):
        g.iterate(N, sync=False)
        g.refine()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.iterate(N, sync=False)
        g.refine()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    hist = history_from_state(g.get_state(), g.ndim, g.nbins)[Wn:Wn + args.steps]
    reps = []
    for _ in range(10):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            g.iterate(N, sync=False)
            g.refine()
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - t1) / args.steps * 1e3)
    g.set_timing(True)
    g.stage_times(reset=True)
    for _ in range(args.steps):
        g.iterate(N, sync=False)
        g.refine()
    torch.cuda.synchronize()
    st = g.stage_times()
    counts = g.strata_counts()
    g.close()
    I, sig = combine(hist)
    Ip, sigp = combine(plain_hist)
    return {"strata_per_axis": m, "beta": beta, "hypercubes": H,
            "events_per_hypercube": {"min": int(counts.min()), "max": int(counts.max()),
                                     "mean": float(counts.mean())},
            "events_used": int(counts.sum()),
            "ms_per_step_min": min(reps), "ms_per_step_min_plain": plain_ms_min,
            "step_overhead": min(reps) / plain_ms_min - 1.0,
            "rel_error": sig / abs(I), "rel_error_plain": sigp / abs(Ip),
            "effective_events_per_s": 1.0 / ((sig / abs(I)) ** 2 * T) if sig > 0 else None,
            "kernel_ms_per_step": {k: v[0] / args.steps for k, v in st.items()}}


def strata_leg(args, make, Wn, N, D, plain_ms_min, plain_hist):
    """Lepage's stratified + importance mode with his m = floor((N/2)^(1/D)) (two
    events per hypercube), and the adaptive allocation with beta = 0.75 over
    m = floor((N/8)^(1/D)) strata per axis (about eight events per hypercube, room
    for the counts to follow sigma_h)."""
    m = args.strata if args.strata > 0 else int((N / 2) ** (1.0 / D) + 1e-9)
    ma = args.strata if args.strata > 0 else int((N / 8) ** (1.0 / D) + 1e-9)
    return {"classic": strata_run(args, make, Wn, N, m, 0.0, plain_ms_min, plain_hist),
            "adaptive": strata_run(args, make, Wn, N, ma, 0.75, plain_ms_min, plain_hist)}


def measure_vegas(args, cfg, prec, N):
    """The VEGAS iteration of one workload at one precision: clock warm-up on a
    throwaway handle, W untimed and K timed steps on a fresh one (events/s, the timed
    iterations' combined error), K more with HIP events bound to each kernel (kernel
    durations), and 10 more blocks of K steps (min / avg / max per step).  The grid is
    refined after each of the configuration's n_iter iterations and kept afterwards."""
    import torch

    import paper_1503_06182_amd as P
    n_adapt = cfg["n_iter"]

    def make():
        h = P.Integrator(cfg["process"], cfg["ndim"], cfg["nbins"], cfg["seed"], cfg["alpha"],
                         cfg["params"], precision=prec, max_events=N)
        h.bench_iters = 0
        return h

    def step(h):
        h.iterate(N, sync=False)
        h.bench_iters += 1
        if h.bench_iters <= n_adapt:
            h.refine()

    clock_s = clock_warm_up(make, step, args.clock_warmup) if args.clock_warmup > 0 else 0.0
    g = make()
    Wn = 2 if args.warmup is None else args.warmup
    for _ in range(Wn):
        step(g)
    torch.cuda.synchronize()
    # throughput: K steps with nothing between the kernels
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(g)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    hist = history_from_state(g.get_state(), cfg["ndim"], cfg["nbins"])
    timed = hist[Wn:Wn + args.steps]
    # kernel durations: K more steps with HIP start/stop events bound to each kernel's
    # dispatch on the library's stream.  The events cost host time per launch: inside
    # the throughput pass, even on the event kernel alone, they slowed the W+ step by
    # 16 % (the host could no longer run ahead of the GPU), so this identical pass
    # follows the timed region instead
    g.set_timing(True)
    g.stage_times(reset=True)
    for _ in range(args.steps):
        step(g)
    torch.cuda.synchronize()
    st = g.stage_times()
    g.set_timing(False)
    # spread over repetitions: 10 more blocks of K steps (ms per step, min / avg / max)
    reps = []
    for _ in range(10):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step(g)
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - t1) / args.steps * 1e3)
    shape = g.last_launch()
    g.close()
    I, sig = combine(timed)
    eps = sig / abs(I)
    # Kish effective sample size of each timed iteration, (sum w)^2 / sum w^2 =
    # N I^2 / (I^2 + (N - 1) var), per second of the timed region
    kish = sum(N * i * i / (i * i + (N - 1) * v) if (i * i + v) > 0 else 0.0 for i, v in timed)
    return {"make": make, "Wn": Wn, "T": T, "timed": timed, "st": st, "reps": reps, "shape": shape,
            "clock_s": clock_s, "I": I, "eps": eps, "events_per_s": args.steps * N / T,
            "eff": 1.0 / (eps * eps * T), "kish": kish / T}


def progress(msg):
    """one line on stderr per finished phase (the JSON line stays alone on stdout)"""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path in this library "
              "(how it would shard is described in the design notes); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "adjoint":
        bench_adjoint(args)
        return
    if args.workload == "flow":
        bench_flow(args)
        return
    if args.workload == "ww_4l_paper":
        bench_paper_schedule(args)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    import torch

    import paper_1503_06182_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    cfg = W.config(args.workload)
    N = args.events or cfg["n_events"]
    prec = P.FP32_ME if args.precision == "fp32me" else P.FP64
    m = measure_vegas(args, cfg, prec, N)
    make, Wn, st, reps, timed, shape = m["make"], m["Wn"], m["st"], m["reps"], m["timed"], m["shape"]
    progress(f"{args.workload}: headline measured ({m['T'] / args.steps * 1e3:.3f} ms per step)")

    legs = not args.no_legs
    obs_leg = observable_leg(args, make, Wn, N, min(reps), st["event"]) \
        if legs and args.workload in OBS_BINNING else None
    if obs_leg is not None:
        progress("observable leg done")
    strata = strata_leg(args, make, Wn, N, cfg["ndim"], min(reps), timed) \
        if legs and args.strata != 0 else None
    if strata is not None:
        progress("stratified legs done")

    ms_ev, n_ev = st["event"]
    avg_ev = ms_ev / max(n_ev, 1) * 1e-3
    roof = roofline(args.workload, args.precision, N, avg_ev)
    # histogram stage: the column sums of the per-block partial rows (S1, S2 and the
    # per-bin d digits) -- HBM-bound; algorithmic bytes = rows x columns x 8 read
    ms_fold, n_fold = st["fold"]
    hist_bytes = shape["fold_rows"] * shape["fold_cols"] * 8
    avg_fold = ms_fold / max(n_fold, 1) * 1e-3
    hist_stage = {"kernel": "k_accsum", "bound": "hbm", "bytes_per_launch": hist_bytes,
                  "avg_launch_ms": avg_fold * 1e3,
                  "achieved_gbs": hist_bytes / avg_fold / 1e9 if avg_fold > 0 else None,
                  "peak_gbs": PEAK_HBM_GBS,
                  "frac": hist_bytes / avg_fold / 1e9 / PEAK_HBM_GBS if avg_fold > 0 else None,
                  "traffic": HIST_STAGE_TRAFFIC.get((args.workload, N)) if prec == P.FP64 else None,
                  "launch": shape}
    if avg_fold <= 0:
        # few partial rows: the finalisation's blocks sum them (no column-sum launch)
        hist_stage.update(kernel="k_finalize (row sums)", bytes_per_launch=hist_bytes,
                          note="no separate launch at this size; timed within the finalisation")
    line = {
        "metric": "events/s and effective events/s (1/var) at 1e-3 rel. error, 1 MI355X",
        "value": m["events_per_s"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": Wn,
        "gpu_clock_warmup_s": round(m["clock_s"], 3),
        "ms_per_step": m["T"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == P.FP64 else "f32-me/f64",
        "data": "synthetic (counter-based Philox stream, seed 1; parametric PDFs)",
        "config": {"workload": args.workload, "events_per_iteration": N, "ndim": cfg["ndim"],
                   "nbins": cfg["nbins"], "iterations_timed": args.steps,
                   "grid_adapted_iterations": cfg["n_iter"]},
        "effective_events_per_s": m["eff"],
        "time_to_1e-3_s": 1e6 / m["eff"],
        "kish_ess_per_s": m["kish"],
        "ms_per_step_10_repeats": {"min": min(reps), "avg": sum(reps) / len(reps), "max": max(reps)},
        "integral_pb": m["I"],
        "rel_error": m["eps"],
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in st.items()},
        "roofline": roof,
        "histogram_stage": hist_stage,
    }
    # the binary32 matrix element on the same workload (W+W- only), and the learned
    # proposal: their effective events/s against this line's plain binary64 VEGAS
    if legs and args.workload == "ww_4l" and prec == P.FP64:
        m32 = measure_vegas(args, cfg, P.FP32_ME, N)
        ms32, n32 = m32["st"]["event"]
        roof32 = roofline(args.workload, "fp32me", N, ms32 / max(n32, 1) * 1e-3)
        line["fp32_me"] = {
            "events_per_s": m32["events_per_s"], "effective_events_per_s": m32["eff"],
            "ms_per_step": m32["T"] / args.steps * 1e3,
            "ms_per_step_10_repeats": {"min": min(m32["reps"]), "avg": sum(m32["reps"]) / 10,
                                       "max": max(m32["reps"])},
            "rel_error": m32["eps"], "integral_pb": m32["I"],
            "speedup_events_per_s_vs_fp64": m32["events_per_s"] / m["events_per_s"],
            "speedup_effective_vs_fp64": m32["eff"] / m["eff"],
            "speedup_min_ms_per_step_vs_fp64": min(reps) / min(m32["reps"]),
            "kernel_ms_per_step": {k: v[0] / args.steps for k, v in m32["st"].items()},
            "roofline": roof32}
        progress("binary32 matrix-element leg done")
        fl = bench_flow(args, emit=False)
        progress("learned-proposal leg done")
        line["flow"] = {
            "events_per_s": fl["value"], "effective_events_per_s": fl["effective_events_per_s"],
            "ms_per_step": fl["ms_per_step"],
            "vegas_same_grid_effective_events_per_s": fl["vegas_effective_events_per_s"],
            "effective_gain_vs_vegas_same_grid": fl["effective_gain_vs_vegas"],
            "effective_gain_vs_fp64_line": fl["effective_events_per_s"] / m["eff"],
            "per_event_rel_variance": fl["per_event_rel_variance"], "flow_uses": fl["flow_uses"],
            "integral_pb": fl["integral_pb"], "training": fl["training"], "config": fl["config"],
            "roofline": fl["roofline"]}
    line["observable"] = obs_leg
    line["strata"] = strata
    if not args.no_cpu_baseline:
        it_s, ev_s = CPU_SAMPLE[args.workload]
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_iters or it_s, min(args.cpu_events or ev_s, 10 * N))
        progress("oracle on one core timed")
        it_a, ev_a = CPU_SAMPLE_ALL_CORES[args.workload]
        line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(cfg, it_a, min(ev_a, 10 * N))
        progress("oracle on all cores timed")
        line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
