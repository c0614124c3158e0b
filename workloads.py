"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the benchmark.

This module holds inputs only: process identifiers, dimensions, bin counts,
seeds, schedules and the physics parameter vectors.  It contains none of the
method's arithmetic and imports neither the oracle nor the HIP library.

Parameter-vector layout (physics processes), index: meaning [default]
    0 alpha_em [1/128]          1 sin^2 theta_W [1 - M_W^2/M_Z^2]
    2 M_Z [91.1876]             3 Gamma_Z [2.4952]
    4 M_W [80.4]                5 Gamma_W [2.1]
    6 sqrt(S) hadronic, or sqrt(shat) for the partonic processes
    7 PDF A [1]   8 PDF a [-0.5]   9 PDF b [3]
   10 lower mass of the Breit-Wigner window   11 upper mass (<= 0: sqrt S)
      (hadronic W+W-: the window of sqrt(shat) instead)
   12 lepton pT cut [20]        13 lepton |eta| cut [2.5]
   14 V_ud [1]                  15 (hbar c)^2 [0.3893794e9 pb GeV^2]
Test integrands: GAUSS params = (mu, sigma); GENZ params = (family, a[ndim], w[ndim]).
"""
from __future__ import annotations

import numpy as np

GAUSS, GENZ, EEMUMU, DY_Z, W_PLUS, WW_4L, WW_HAD = range(7)
NDIM = {EEMUMU: 2, DY_Z: 3, W_PLUS: 4, WW_4L: 8, WW_HAD: 10}

MZ, GZ, MW, GW = 91.1876, 2.4952, 80.4, 2.1
SW2_ONSHELL = 1.0 - (MW / MZ) ** 2


def phys_params(sqrts=13000.0, mlo=0.0, mhi=0.0, ptmin=0.0, etamax=1.0e300, **over):
    p = np.array([1.0 / 128.0, SW2_ONSHELL, MZ, GZ, MW, GW, sqrts, 1.0, -0.5, 3.0,
                  mlo, mhi, ptmin, etamax, 1.0, 0.3893794e9], dtype=np.float64)
    names = ["alpha", "sw2", "mz", "gz", "mw", "gw", "sqrts", "A", "a", "b", "mlo", "mhi",
             "ptmin", "etamax", "vud", "conv"]
    for k, v in over.items():
        p[names.index(k)] = v
    return p


def config(name: str) -> dict:
    """The named workloads.  'dy_z' .. 'ww_4l' are the measured configurations."""
    if name == "dy_z":  # q qbar -> Z/photon -> e+e-, 13 TeV, 81 < m_ll < 101, 3 dims
        return dict(process=DY_Z, ndim=3, nbins=50, seed=1, alpha=1.5,
                    params=phys_params(13000.0, mlo=81.0, mhi=101.0),
                    n_iter=5, n_events=10_000)
    if name == "w_plus":  # pp -> W+ -> e+ nu, BW mapping, pT > 20, |eta| < 2.5, 4 dims
        return dict(process=W_PLUS, ndim=4, nbins=100, seed=1, alpha=1.5,
                    params=phys_params(13000.0, mlo=40.0, mhi=0.0, ptmin=20.0, etamax=2.5),
                    n_iter=10, n_events=1_000_000)
    if name == "ww_4l":  # q qbar -> W+W- -> e+ nu mu- nubar at sqrt(shat) = 500 GeV, 8 dims
        return dict(process=WW_4L, ndim=8, nbins=100, seed=1, alpha=1.5,
                    params=phys_params(500.0),
                    n_iter=10, n_events=10_000_000)
    if name == "ww_4l_paper":  # the W+W- integrand on the two-stage schedule of the timing
        # runs in Sec. 3.2: 4 x 1,000 then 10 x 10,000 events, the first stage dropped
        c = config("ww_4l")
        c.update(schedule=[1000] * 4 + [10_000] * 10, discard_first=4,
                 n_iter=14, n_events=10_000)
        return c
    if name == "ww_had":  # pp -> W+W- -> e+ nu mu- nubar at 13 TeV, 150 GeV < sqrt(shat), 10 dims
        return dict(process=WW_HAD, ndim=10, nbins=100, seed=1, alpha=1.5,
                    params=phys_params(13000.0, mlo=150.0),
                    n_iter=10, n_events=10_000_000)
    if name == "eemumu":
        return dict(process=EEMUMU, ndim=2, nbins=50, seed=1, alpha=1.5,
                    params=phys_params(91.0), n_iter=5, n_events=100_000)
    if name == "gauss4":
        return dict(process=GAUSS, ndim=4, nbins=50, seed=7, alpha=1.5,
                    params=np.array([0.5, 0.1]), n_iter=8, n_events=20_000)
    raise KeyError(name)


def genz_params(family: int, ndim: int, seed: int = 3, difficulty: float = 5.0):
    """Random Genz parameters: a_i positive with sum a_i = difficulty, w_i uniform in (0,1)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.1, 1.0, ndim)
    a *= difficulty / a.sum()
    w = rng.uniform(0.05, 0.95, ndim)
    return np.concatenate([[float(family)], a, w])


def adjoint_points(B: int = 64, seed: int = 2):
    """B parameter points theta = nominal * (1 + 0.05 v), v uniform in [-1,1]^5,
    theta = (M_Z, Gamma_Z, sin^2 theta_W, pdf a, pdf b)."""
    nominal = np.array([MZ, GZ, SW2_ONSHELL, -0.5, 3.0])
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, (B, 5))
    return nominal * (1.0 + 0.05 * v)
