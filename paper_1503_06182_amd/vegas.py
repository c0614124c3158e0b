"""ctypes binding of the gfx950 VEGAS library (libvegas.so, C ABI in include/vegas.h).

Argument marshalling only: every step of an iteration runs in the library's
HIP kernels.  PyTorch supplies the device workspace and the stream.  If the
library is not built, importing works but every call raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvegas.so")

GAUSS, GENZ, EEMUMU, DY_Z, W_PLUS, WW_4L, WW_HAD = range(7)
FP64, FP32_ME = 0, 1
OK, EINVAL, ESTATE, ENOMEM, EHIP = 0, -1, -2, -3, -4
NPHYS = 16
MAX_ITER = 4096
MAX_OBS_BINS = 254
SCRATCH_DOUBLES = 1 << 21          # static scratch of the allocation-free calls
ETOOBIG = -5                       # request larger than that scratch

EXPORTS = ["vegas_workspace_size", "vegas_init", "vegas_iterate", "vegas_refine", "vegas_run_schedule",
           "vegas_result",
           "vegas_result_from", "vegas_set_observable", "vegas_get_observable", "vegas_set_strata",
           "vegas_set_strata_beta", "vegas_get_strata_counts",
           "vegas_get_grid", "vegas_set_grid", "vegas_get_hist", "vegas_get_weights",
           "vegas_get_state", "vegas_set_state", "vegas_set_launch", "vegas_destroy",
           "vegas_strerror", "vegas_set_timing", "vegas_stage_times", "vegas_grad", "vegas_grad_noalloc", "vegas_last_launch",
           "vegas_export", "vegas_iterate_flow", "vegas_flow_create", "vegas_flow_destroy",
           "vegas_flow_get_params", "vegas_flow_set_params", "vegas_flow_density",
           "vegas_flow_loss_grad", "vegas_flow_train_step", "vegas_flow_sample"]


class VegasError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.vegas_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} (status {status})")


class Config(C.Structure):
    _fields_ = [("process", C.c_int32), ("ndim", C.c_int32), ("nbins", C.c_int32),
                ("precision", C.c_int32), ("seed", C.c_uint64), ("alpha", C.c_double),
                ("params", C.POINTER(C.c_double)), ("nparams", C.c_int32),
                ("waves_per_block", C.c_int32), ("max_blocks", C.c_int32)]


class IterResult(C.Structure):
    _fields_ = [("integral", C.c_double), ("variance", C.c_double), ("n_events", C.c_int64),
                ("n_nonzero", C.c_int64), ("n_nonfinite", C.c_int64), ("iteration", C.c_uint32),
                ("fold", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libvegas.so; raises if it is not built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.vegas_workspace_size.argtypes = [C.POINTER(Config), i64, C.POINTER(C.c_size_t)]
    L.vegas_init.argtypes = [C.POINTER(Config), i64, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.vegas_iterate.argtypes = [vp, i64, C.POINTER(IterResult)]
    L.vegas_refine.argtypes = [vp]
    L.vegas_run_schedule.argtypes = [vp, C.POINTER(i64), i32, i32]
    L.vegas_result.argtypes = [vp, dp, dp, dp, C.POINTER(i32)]
    L.vegas_result_from.argtypes = [vp, i32, dp, dp, dp, C.POINTER(i32)]
    L.vegas_set_observable.argtypes = [vp, i32, C.c_double, C.c_double, i32]
    L.vegas_set_strata.argtypes = [vp, i32]
    L.vegas_set_strata_beta.argtypes = [vp, C.c_double]
    L.vegas_get_strata_counts.argtypes = [vp, vp]
    L.vegas_get_observable.argtypes = [vp, vp, vp, vp, vp]
    L.vegas_get_grid.argtypes = [vp, vp]
    L.vegas_set_grid.argtypes = [vp, vp]
    L.vegas_get_hist.argtypes = [vp, vp, vp]
    L.vegas_get_weights.argtypes = [vp, i64, i64, vp, vp]
    L.vegas_get_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
    L.vegas_set_state.argtypes = [vp, vp, C.c_size_t]
    L.vegas_set_launch.argtypes = [vp, i32, i32]
    L.vegas_destroy.argtypes = [vp]
    L.vegas_set_timing.argtypes = [vp, i32]
    L.vegas_stage_times.argtypes = [vp, vp, vp, i32]
    L.vegas_last_launch.argtypes = [vp, vp]
    L.vegas_strerror.argtypes = [C.c_int]
    L.vegas_strerror.restype = C.c_char_p
    L.vegas_grad.argtypes = [vp, vp, i32, i64, C.c_uint32, vp, vp]
    L.vegas_grad_noalloc.argtypes = [vp, vp, i32, i64, C.c_uint32, vp, vp]
    L.vegas_export.argtypes = [vp, i64, i64, vp, vp]
    L.vegas_iterate_flow.argtypes = [vp, vp, i64, C.POINTER(IterResult)]
    L.vegas_flow_create.argtypes = [i32, i64, C.c_uint64, vp, C.POINTER(vp)]
    L.vegas_flow_destroy.argtypes = [vp]
    L.vegas_flow_get_params.argtypes = [vp, vp]
    L.vegas_flow_set_params.argtypes = [vp, vp]
    L.vegas_flow_density.argtypes = [vp, vp, i64, vp]
    L.vegas_flow_loss_grad.argtypes = [vp, vp, vp, i64, vp, dp]
    L.vegas_flow_train_step.argtypes = [vp, vp, vp, i64, i32, C.c_uint64, C.c_float, dp]
    L.vegas_flow_sample.argtypes = [vp, vp, i64, vp, vp]
    _lib = L
    return L


def _check(status, where):
    if status != OK:
        raise VegasError(status, where)


def make_config(process, ndim, nbins, seed=1, alpha=1.5, params=(), precision=FP64,
                waves_per_block=0, max_blocks=0):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    cfg = Config(process, ndim, nbins, precision, seed, alpha,
                 p.ctypes.data_as(C.POINTER(C.c_double)) if p.size else None, p.size,
                 waves_per_block, max_blocks)
    return cfg, p


def workspace_size(process, ndim, nbins, max_events, params=(), precision=FP64) -> int:
    L = load()
    cfg, _keep = make_config(process, ndim, nbins, params=params, precision=precision)
    b = C.c_size_t()
    _check(L.vegas_workspace_size(C.byref(cfg), max_events, C.byref(b)), "vegas_workspace_size")
    return b.value


class Integrator:
    """One VEGAS handle on the current torch device and stream.

    The device workspace is a torch uint8 tensor owned by this object; the
    stream is torch.cuda.current_stream() unless one is given.
    """

    def __init__(self, process, ndim, nbins, seed=1, alpha=1.5, params=(), precision=FP64,
                 max_events=1_000_000, waves_per_block=0, max_blocks=0, stream=None):
        import torch
        L = load()
        self._L = L
        self.ndim, self.nbins, self.process = ndim, nbins, process
        cfg, self._params = make_config(process, ndim, nbins, seed, alpha, params, precision,
                                        waves_per_block, max_blocks)
        nbytes = C.c_size_t()
        _check(L.vegas_workspace_size(C.byref(cfg), max_events, C.byref(nbytes)),
               "vegas_workspace_size")
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(L.vegas_init(C.byref(cfg), max_events, C.c_void_p(aligned), nbytes.value,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h)), "vegas_init")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.vegas_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, n, sync=True):
        if not sync:
            _check(self._L.vegas_iterate(self._h, n, None), "vegas_iterate")
            return None
        r = IterResult()
        _check(self._L.vegas_iterate(self._h, n, C.byref(r)), "vegas_iterate")
        return {"I": r.integral, "var": r.variance, "n_events": r.n_events,
                "n_nonzero": r.n_nonzero, "n_nonfinite": r.n_nonfinite, "iteration": r.iteration,
                "fold": r.fold}

    def iterate_flow(self, flow, n):
        """One iteration with the learned proposal `flow` (grid frozen)."""
        r = IterResult()
        _check(self._L.vegas_iterate_flow(self._h, flow._f, n, C.byref(r)), "vegas_iterate_flow")
        return {"I": r.integral, "var": r.variance, "n_events": r.n_events,
                "n_nonzero": r.n_nonzero, "n_nonfinite": r.n_nonfinite, "iteration": r.iteration,
                "fold": r.fold}

    def export(self, first, n):
        """Training data of the last (VEGAS) iteration: y [n,8] float32 and w [n] float64
        CUDA tensors."""
        import torch
        y = torch.empty(n, 8, dtype=torch.float32, device="cuda")
        w = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(self._L.vegas_export(self._h, first, n, C.c_void_p(y.data_ptr()), C.c_void_p(w.data_ptr())),
               "vegas_export")
        return y, w

    def refine(self):
        _check(self._L.vegas_refine(self._h), "vegas_refine")

    def run_schedule(self, n_events, refine=True):
        """Iterations of n_events[j] events (and a refinement after each): the first call
        records the launches as a HIP graph, a repeat from the same state replays it."""
        arr = (C.c_int64 * len(n_events))(*[int(n) for n in n_events])
        _check(self._L.vegas_run_schedule(self._h, arr, len(n_events), 1 if refine else 0),
               "vegas_run_schedule")

    def result(self, first=0):
        """Combined estimate over iterations first .. last (first > 0 drops warm-up iterations)."""
        I, e, c = C.c_double(), C.c_double(), C.c_double()
        n = C.c_int32()
        _check(self._L.vegas_result_from(self._h, first, C.byref(I), C.byref(e), C.byref(c), C.byref(n)),
               "vegas_result_from")
        return {"I": I.value, "sigma": e.value, "chi2_dof": c.value, "n_iter": n.value}

    def set_strata(self, m):
        """m strata per axis (0: off): iterations then use m^ndim floor(n / m^ndim) events."""
        _check(self._L.vegas_set_strata(self._h, m), "vegas_set_strata")
        self._strata_H = m ** self.ndim if m > 0 else 0

    def set_strata_beta(self, beta):
        """beta > 0: adaptive allocation n_h ~ sigma_h^beta over the hypercubes."""
        _check(self._L.vegas_set_strata_beta(self._h, beta), "vegas_set_strata_beta")

    def strata_counts(self):
        self._strata_H = getattr(self, "_strata_H", 0)
        c = np.zeros(self._strata_H, dtype=np.int32)
        _check(self._L.vegas_get_strata_counts(self._h, c.ctypes.data), "vegas_get_strata_counts")
        return c

    def set_observable(self, nbins, lo=0.0, hi=1.0, first=0):
        """Histogram the process's observable in nbins uniform bins on [lo, hi)
        (plus under- and overflow); iterations numbered >= first are combined."""
        _check(self._L.vegas_set_observable(self._h, nbins, lo, hi, first), "vegas_set_observable")
        self.nobs = nbins

    def get_observable(self):
        """(last, last_err, comb, comb_err), each of nbins + 2 (under- and overflow at the ends)."""
        k = getattr(self, "nobs", 0) + 2
        a = [np.zeros(k) for _ in range(4)]
        _check(self._L.vegas_get_observable(self._h, *[x.ctypes.data for x in a]), "vegas_get_observable")
        return tuple(a)

    def get_grid(self):
        e = np.zeros((self.ndim, self.nbins + 1))
        _check(self._L.vegas_get_grid(self._h, e.ctypes.data), "vegas_get_grid")
        return e

    def set_grid(self, edges):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64))
        _check(self._L.vegas_set_grid(self._h, e.ctypes.data), "vegas_set_grid")

    def get_hist(self):
        d = np.zeros((self.ndim, self.nbins))
        s = np.zeros(2)
        _check(self._L.vegas_get_hist(self._h, d.ctypes.data, s.ctypes.data), "vegas_get_hist")
        return d, s

    def get_weights(self, first, n, with_bins=True):
        w = np.zeros(n)
        b = np.zeros((n, self.ndim), dtype=np.uint8) if with_bins else None
        _check(self._L.vegas_get_weights(self._h, first, n, w.ctypes.data,
                                         b.ctypes.data if with_bins else None),
               "vegas_get_weights")
        return (w, b) if with_bins else w

    def get_state(self) -> bytes:
        n = C.c_size_t()
        _check(self._L.vegas_get_state(self._h, None, C.byref(n)), "vegas_get_state")
        buf = C.create_string_buffer(n.value)
        _check(self._L.vegas_get_state(self._h, buf, C.byref(n)), "vegas_get_state")
        return buf.raw[:n.value]

    def set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self._L.vegas_set_state(self._h, buf, len(blob)), "vegas_set_state")

    STAGES = ("event", "fold", "finalize", "refine")

    def set_timing(self, enable=True, stages=None):
        """Kernel timing with HIP events on the handle's stream: all stages, or only
        the named ones (a subset of STAGES); enable=False turns it off."""
        mask = 0
        if enable:
            names = self.STAGES if stages is None else stages
            for nm in names:
                mask |= 1 << self.STAGES.index(nm)
        _check(self._L.vegas_set_timing(self._h, mask), "vegas_set_timing")

    def stage_times(self, reset=False):
        """Summed kernel milliseconds and launch counts per stage since the last reset."""
        ms = np.zeros(4)
        n = np.zeros(4, dtype=np.int64)
        _check(self._L.vegas_stage_times(self._h, ms.ctypes.data, n.ctypes.data, 1 if reset else 0),
               "vegas_stage_times")
        names = ("event", "fold", "finalize", "refine")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(names)}

    def last_launch(self):
        """Launch shape of the last iteration: event blocks, threads per block, folded
        partial rows, int64 columns per row."""
        info = np.zeros(4, dtype=np.int64)
        _check(self._L.vegas_last_launch(self._h, info.ctypes.data), "vegas_last_launch")
        return {"event_blocks": int(info[0]), "threads": int(info[1]), "fold_rows": int(info[2]),
                "fold_cols": int(info[3])}

    def grad(self, theta, n_events, iteration):
        """sigma[B] and dsigma/dtheta[B,5] (Drell-Yan only) for theta[B,5] at the current
        grid; theta, sigma and dsigma are float64 CUDA tensors on this handle's stream."""
        import torch
        theta = theta.detach().to(device="cuda", dtype=torch.float64).contiguous()
        B = theta.shape[0]
        sigma = torch.empty(B, dtype=torch.float64, device="cuda")
        dsigma = torch.empty(B, 5, dtype=torch.float64, device="cuda")
        _check(self._L.vegas_grad(self._h, C.c_void_p(theta.data_ptr()), B, n_events, iteration,
                                  C.c_void_p(sigma.data_ptr()), C.c_void_p(dsigma.data_ptr())),
               "vegas_grad")
        return sigma, dsigma

    def grad_noalloc(self, theta, sigma, dsigma, n_events, iteration):
        """vegas_grad_noalloc: the same as grad into caller-allocated float64 CUDA tensors
        sigma[B] and dsigma[B,5] (theta[B,5] float64, contiguous, on the device), with the
        library's static scratch instead of any device allocation."""
        B = theta.shape[0]
        _check(self._L.vegas_grad_noalloc(self._h, C.c_void_p(theta.data_ptr()), B, n_events, iteration,
                                          C.c_void_p(sigma.data_ptr()), C.c_void_p(dsigma.data_ptr())),
               "vegas_grad_noalloc")

    def set_launch(self, waves_per_block, max_blocks=0):
        _check(self._L.vegas_set_launch(self._h, waves_per_block, max_blocks), "vegas_set_launch")


def _sigma_function():
    import torch

    class VegasSigma(torch.autograd.Function):
        """sigma(theta) of the Drell-Yan estimator at a fixed grid and random stream;
        backward returns grad_sigma[:, None] * dsigma/dtheta from the adjoint kernel."""

        @staticmethod
        def forward(ctx, theta, integrator, n_events, iteration):
            sigma, dsigma = integrator.grad(theta, n_events, iteration)
            ctx.save_for_backward(dsigma)
            ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
            return sigma.to(device=theta.device, dtype=theta.dtype)

        @staticmethod
        def backward(ctx, grad_sigma):
            (dsigma,) = ctx.saved_tensors
            g = grad_sigma.to(device=dsigma.device, dtype=dsigma.dtype)[:, None] * dsigma
            return g.to(device=ctx.theta_device, dtype=ctx.theta_dtype), None, None, None

    return VegasSigma


def vegas_sigma(theta, integrator, n_events, iteration):
    """Differentiable sigma(theta) for theta[B,5] (torch float64, requires_grad allowed)."""
    global VegasSigma
    if VegasSigma is None:
        VegasSigma = _sigma_function()
    return VegasSigma.apply(theta, integrator, n_events, iteration)


VegasSigma = None
