"""CPU oracle of the learned proposal -- TEST INFRASTRUCTURE ONLY.

A coupling-layer rational-quadratic spline flow on the VEGAS y-space [0,1]^8,
in plain float64 PyTorch on the CPU (gradients by torch.autograd).  Loaded only
by tests/ and the benchmark's CPU leg; it shares no code with the HIP kernels.

Definitions (the build's reading of the learned-proposal extension; the paper
itself describes VEGAS only, Sec. 2.1):
* six coupling layers; layer l leaves its conditioning coordinates C_l unchanged
  and maps each of the four others, d in X_l, by a monotone rational-quadratic
  spline s on [0,1] with 16 bins (Durkan et al., Neural Spline Flows, 2019)
  whose parameters come from an MLP of the conditioning coordinates;
* the density direction y -> z applies layers 1..6 with the forward spline and
  log q(y) = sum over layers and transformed coordinates of log s'(v); the base
  density is uniform on [0,1]^8;  sampling z -> y applies the inverse splines in
  reverse order;
* MLP 4 -> 128 -> 128 -> 188 with ReLU; the 188 outputs are, per transformed
  coordinate in increasing order, 16 width logits, 16 height logits and 15
  interior derivative pre-activations;
* bin widths w = eps + (1 - 16 eps) softmax, heights likewise, interior
  derivatives eps + softplus(raw + c) with c chosen so raw = 0 gives 1, the two
  boundary derivatives fixed at 1, eps = 1e-3;
* loss for VEGAS-weighted events (y_i, w_i): L = -sum w_i log q(y_i) / sum w_i.

Flat parameter vector (the interface with the library): for each layer l:
W1 [4][128] (input-major), b1 [128], W2 [128][128], b2 [128], W3 [128][188], b3 [188].
"""
from __future__ import annotations

import math

import torch

NDIM = 8
NB = 16
NPAR = 3 * NB - 1          # 47 per transformed coordinate
HID = 128
NOUT = 4 * NPAR            # 188
NLAYER = 6
EPS = 1e-3
DSHIFT = math.log(math.expm1(1.0 - EPS))
# transformed coordinates of each layer (the conditioning set is the complement)
TRANSFORMED = [(4, 5, 6, 7), (0, 1, 2, 3), (1, 3, 5, 7), (0, 2, 4, 6), (2, 3, 6, 7), (0, 1, 4, 5)]
LAYER_SIZE = 4 * HID + HID + HID * HID + HID + HID * NOUT + NOUT   # 41404
NPARAMS = NLAYER * LAYER_SIZE                                          # 248424


def conditioning(l):
    return tuple(d for d in range(NDIM) if d not in TRANSFORMED[l])


def unpack(theta, l):
    """Views (W1, b1, W2, b2, W3, b3) of layer l in the flat vector."""
    o = l * LAYER_SIZE
    out = []
    for shape in ((4, HID), (HID,), (HID, HID), (HID,), (HID, NOUT), (NOUT,)):
        n = math.prod(shape)
        out.append(theta[o:o + n].view(*shape))
        o += n
    return out


def init_params(seed=0, dtype=torch.float64):
    """He-uniform hidden layers; the output layer zero, so the flow starts as the
    identity (q = 1: the plain VEGAS proposal)."""
    g = torch.Generator().manual_seed(seed)
    theta = torch.zeros(NPARAMS, dtype=dtype)
    for l in range(NLAYER):
        W1, b1, W2, b2, W3, b3 = unpack(theta, l)
        W1.copy_((torch.rand(4, HID, generator=g, dtype=dtype) * 2 - 1) * math.sqrt(6 / 4))
        W2.copy_((torch.rand(HID, HID, generator=g, dtype=dtype) * 2 - 1) * math.sqrt(6 / HID))
    return theta


def bf16(x):
    """Round to bfloat16 (through binary32, round to nearest even), back to float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def half(x):
    """Round to binary16 (round to nearest even), back to float64."""
    return x.to(torch.float16).to(torch.float64)


def mlp(cond, theta, l, bf16_emulation=False):
    """Spline parameters of layer l.  bf16_emulation rounds as the library's
    matrix-core path does: the operands of the two 128-wide products (h1, W2, h2,
    W3) to bfloat16 and the resulting spline parameters to binary16; the first
    layer (4 inputs) and the biases stay unrounded."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, l)
    r = bf16 if bf16_emulation else (lambda t: t)
    h1 = torch.relu(cond @ W1 + b1)
    h2 = torch.relu(r(h1) @ r(W2) + b2)
    out = r(h2) @ r(W3) + b3
    return half(out) if bf16_emulation else out


def spline_knots(raw):
    """raw [..., 47] -> knot abscissae xk [..., 17], ordinates yk [..., 17], derivatives dk [..., 17]."""
    w = EPS + (1 - NB * EPS) * torch.softmax(raw[..., :NB], dim=-1)
    h = EPS + (1 - NB * EPS) * torch.softmax(raw[..., NB:2 * NB], dim=-1)
    dint = EPS + torch.nn.functional.softplus(raw[..., 2 * NB:] + DSHIFT)
    zeros = torch.zeros(raw.shape[:-1] + (1,), dtype=raw.dtype)
    ones = torch.ones(raw.shape[:-1] + (1,), dtype=raw.dtype)
    xk = torch.cat([zeros, torch.cumsum(w, -1)], -1)
    yk = torch.cat([zeros, torch.cumsum(h, -1)], -1)
    xk = torch.cat([xk[..., :-1], ones], -1)
    yk = torch.cat([yk[..., :-1], ones], -1)
    dk = torch.cat([ones, dint, ones], -1)
    return xk, yk, dk


def _gather(t, k):
    return torch.gather(t, -1, k.unsqueeze(-1)).squeeze(-1)


def rqs_forward(x, raw):
    """y = s(x) and log s'(x) for x in [0,1]."""
    xk, yk, dk = spline_knots(raw)
    k = torch.clamp(torch.searchsorted(xk[..., 1:-1].contiguous(), x.unsqueeze(-1)).squeeze(-1), 0, NB - 1)
    x0, x1 = _gather(xk, k), _gather(xk, k + 1)
    y0, y1 = _gather(yk, k), _gather(yk, k + 1)
    d0, d1 = _gather(dk, k), _gather(dk, k + 1)
    w, h = x1 - x0, y1 - y0
    s = h / w
    xi = (x - x0) / w
    t = xi * (1 - xi)
    den = s + (d1 + d0 - 2 * s) * t
    y = y0 + h * (s * xi * xi + d0 * t) / den
    dy = s * s * (d1 * xi * xi + 2 * s * t + d0 * (1 - xi) ** 2) / (den * den)
    return y, torch.log(dy)


def rqs_inverse(y, raw):
    """x = s^{-1}(y) and log s'(x) (of the forward map) for y in [0,1]."""
    xk, yk, dk = spline_knots(raw)
    k = torch.clamp(torch.searchsorted(yk[..., 1:-1].contiguous(), y.unsqueeze(-1)).squeeze(-1), 0, NB - 1)
    x0, x1 = _gather(xk, k), _gather(xk, k + 1)
    y0, y1 = _gather(yk, k), _gather(yk, k + 1)
    d0, d1 = _gather(dk, k), _gather(dk, k + 1)
    w, h = x1 - x0, y1 - y0
    s = h / w
    dy = y - y0
    a = h * (s - d0) + dy * (d1 + d0 - 2 * s)
    b = h * d0 - dy * (d1 + d0 - 2 * s)
    c = -s * dy
    xi = 2 * c / (-b - torch.sqrt(b * b - 4 * a * c))
    x = x0 + xi * w
    t = xi * (1 - xi)
    den = s + (d1 + d0 - 2 * s) * t
    dydx = s * s * (d1 * xi * xi + 2 * s * t + d0 * (1 - xi) ** 2) / (den * den)
    return x, torch.log(dydx)


def log_density(y, theta, bf16_emulation=False):
    """log q(y) for y [N, 8] (density direction y -> z); also returns z."""
    v = y.clone()
    logq = torch.zeros(y.shape[0], dtype=y.dtype)
    for l in range(NLAYER):
        C, X = list(conditioning(l)), list(TRANSFORMED[l])
        raw = mlp(v[:, C], theta, l, bf16_emulation).view(-1, 4, NPAR)
        out, ld = rqs_forward(v[:, X], raw)
        v = v.clone()
        v[:, X] = out
        logq = logq + ld.sum(-1)
    return logq, v


def sample(z, theta, bf16_emulation=False):
    """y = F^{-1}(z) for z [N, 8] and log q(y)."""
    v = z.clone()
    logq = torch.zeros(z.shape[0], dtype=z.dtype)
    for l in reversed(range(NLAYER)):
        C, X = list(conditioning(l)), list(TRANSFORMED[l])
        raw = mlp(v[:, C], theta, l, bf16_emulation).view(-1, 4, NPAR)
        out, ld = rqs_inverse(v[:, X], raw)
        v = v.clone()
        v[:, X] = out
        logq = logq + ld.sum(-1)
    return v, logq


def loss(y, w, theta, bf16_emulation=False):
    logq, _ = log_density(y, theta, bf16_emulation)
    return -(w * logq).sum() / w.sum()


def loss_and_grad(y, w, theta, bf16_emulation=False):
    t = theta.clone().requires_grad_(True)
    L = loss(y, w, t, bf16_emulation)
    (g,) = torch.autograd.grad(L, t)
    return L.detach(), g
