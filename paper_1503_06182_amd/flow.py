"""Learned proposal: ctypes binding of the flow functions of include/vegas.h and
the training driver.

The flow (six rational-quadratic spline coupling layers on the unit cube
[0,1]^8 that the VEGAS grid map is applied to) is trained on the GPU by the
library's own forward and backward kernels on the weighted events of a VEGAS
iteration, with loss L = -sum w log q / sum w.  A flow iteration weighs each
event by f J / q, an unbiased estimate of the same integral for any parameters,
so the flow can only change the variance; the fallback rule keeps plain VEGAS
when the flow does not lower the cost of a given error.
"""
from __future__ import annotations

import ctypes as C
import time

from .vegas import IterResult, _check, load  # noqa: F401  (IterResult re-exported for callers)

NPARAMS = 248424
NDIM = 8


class Flow:
    """One flow handle on the current device.  Tensors in and out are CUDA tensors
    (y float32 [B,8], w float64 [B], log q float32 [B], parameters float32 [NPARAMS])."""

    def __init__(self, max_batch=4096, max_sample=0, seed=1, stream=None):
        import torch
        L = load()
        self._L = L
        self.max_batch, self.max_sample = max_batch, max_sample
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        f = C.c_void_p()
        _check(L.vegas_flow_create(max_batch, max_sample, seed, C.c_void_p(self.stream.cuda_stream), C.byref(f)),
               "vegas_flow_create")
        self._f = f
        self.steps = 0

    def close(self):
        if getattr(self, "_f", None) is not None and self._f.value:
            self._L.vegas_flow_destroy(self._f)
            self._f = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import torch
        out = torch.empty(NPARAMS, dtype=torch.float32, device="cuda")
        _check(self._L.vegas_flow_get_params(self._f, C.c_void_p(out.data_ptr())), "vegas_flow_get_params")
        self.stream.synchronize()
        return out

    def set_params(self, theta):
        import torch
        t = theta.detach().to(device="cuda", dtype=torch.float32).contiguous()
        assert t.numel() == NPARAMS
        _check(self._L.vegas_flow_set_params(self._f, C.c_void_p(t.data_ptr())), "vegas_flow_set_params")
        self.stream.synchronize()
        self.steps = 0

    def density(self, y):
        import torch
        y = y.detach().to(device="cuda", dtype=torch.float32).contiguous()
        out = torch.empty(y.shape[0], dtype=torch.float32, device="cuda")
        _check(self._L.vegas_flow_density(self._f, C.c_void_p(y.data_ptr()), y.shape[0],
                                          C.c_void_p(out.data_ptr())), "vegas_flow_density")
        self.stream.synchronize()
        return out

    def loss_grad(self, y, w):
        import torch
        y = y.detach().to(device="cuda", dtype=torch.float32).contiguous()
        w = w.detach().to(device="cuda", dtype=torch.float64).contiguous()
        g = torch.empty(NPARAMS, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        _check(self._L.vegas_flow_loss_grad(self._f, C.c_void_p(y.data_ptr()), C.c_void_p(w.data_ptr()),
                                            y.shape[0], C.c_void_p(g.data_ptr()), C.byref(loss)),
               "vegas_flow_loss_grad")
        return loss.value, g

    def train_step(self, y, w, batch, lr=1e-3, with_loss=False):
        """One Adam step on the next batch of the data set (y, w); y, w stay resident."""
        loss = C.c_double()
        _check(self._L.vegas_flow_train_step(self._f, C.c_void_p(y.data_ptr()), C.c_void_p(w.data_ptr()),
                                             y.shape[0], batch, self.steps, lr,
                                             C.byref(loss) if with_loss else None),
               "vegas_flow_train_step")
        self.steps += 1
        return loss.value if with_loss else None

    def sample(self, z):
        """y = F^{-1}(z) and log q(y)."""
        import torch
        z = z.detach().to(device="cuda", dtype=torch.float32).contiguous()
        y = torch.empty_like(z)
        lq = torch.empty(z.shape[0], dtype=torch.float32, device="cuda")
        _check(self._L.vegas_flow_sample(self._f, C.c_void_p(z.data_ptr()), z.shape[0], C.c_void_p(y.data_ptr()),
                                         C.c_void_p(lq.data_ptr())), "vegas_flow_sample")
        self.stream.synchronize()
        return y, lq


def train(flow, y, w, epochs=20, batch=4096, lr=1e-3, log_every=0):
    """Adam over `epochs` passes of the data set (y [N,8] float32, w [N] float64, CUDA).
    Returns the losses of the steps at which the loss was read (every log_every steps
    and the last one)."""
    n = y.shape[0]
    steps = epochs * ((n + batch - 1) // batch)
    losses = []
    for s in range(steps):
        want = (log_every and s % log_every == 0) or s == steps - 1
        loss = flow.train_step(y, w, batch, lr, with_loss=want)
        if want:
            losses.append((s, loss))
    return losses


def _timed(fn, stream):
    stream.synchronize()
    t0 = time.perf_counter()
    r = fn()
    stream.synchronize()
    return r, time.perf_counter() - t0


def relative_cost(r, seconds):
    """Seconds to reach relative error 1 with this proposal: per-event relative variance
    (N var / I^2) times seconds per event (var is the variance of the iteration mean)."""
    n = r["n_events"]
    if r["I"] == 0:
        return float("inf")
    return (n * r["var"] / r["I"] ** 2) * (seconds / n)


def choose_proposal(integrator, flow, n_pilot):
    """Fallback rule: one pilot iteration with each proposal (both are unbiased and
    enter the combined result); use the flow only if its per-event relative variance
    times its cost per event is lower than plain VEGAS's.  The grid is not refined."""
    rv, tv = _timed(lambda: integrator.iterate(n_pilot), integrator.stream)
    rf, tf = _timed(lambda: integrator.iterate_flow(flow, n_pilot), integrator.stream)
    cv, cf = relative_cost(rv, tv), relative_cost(rf, tf)
    return {"use_flow": cf < cv, "vegas": rv, "flow": rf, "vegas_s": tv, "flow_s": tf,
            "vegas_cost": cv, "flow_cost": cf}
