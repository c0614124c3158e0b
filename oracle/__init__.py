"""CPU oracle for the per-event VEGAS iteration -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path
(``paper_1503_06182_amd``) never does, and this package never imports it.

The C source (``vegas_oracle.c``) is a plain serial FP64 implementation with
long-double sums; this module only loads it with ctypes and marshals arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "vegas_oracle.c")

GAUSS, GENZ, EEMUMU, DY_Z, W_PLUS, WW_4L = range(6)

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-Wall", "-o", LIB_PATH, SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.ora_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.ora_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_int, _dp]
        L.ora_ndim.argtypes = [C.c_int, C.c_int]
        L.ora_integrand.argtypes = [C.c_int, C.c_int, _dp, C.c_int, _dp]
        L.ora_integrand.restype = C.c_double
        L.ora_me_dy.argtypes = [_dp, C.c_double, C.c_double, C.c_int]
        L.ora_me_dy.restype = C.c_double
        L.ora_sigmahat_dy.argtypes = [_dp, C.c_double, C.c_int]
        L.ora_sigmahat_dy.restype = C.c_double
        L.ora_me_eemumu_dirac.argtypes = [_dp, C.c_double, C.c_double, C.c_double]
        L.ora_me_eemumu_dirac.restype = C.c_double
        L.ora_spinor_check.argtypes = [_dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ora_ww_me2.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_int, C.c_int]
        L.ora_ww_me2.restype = C.c_double
        L.ora_ww_onshell_me2.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_int,
                                         C.c_int, C.c_int, C.c_int, C.c_int]
        L.ora_ww_onshell_me2.restype = C.c_double
        L.ora_ww_momenta.argtypes = [_dp, _dp, _dp, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ora_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_double, _dp, C.c_int]
        L.ora_create.restype = C.c_void_p
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_iterate.argtypes = [C.c_void_p, C.c_int64, _dp]
        L.ora_iterate_threads.argtypes = [C.c_void_p, C.c_int64, C.c_int, _dp]
        L.ora_refine.argtypes = [C.c_void_p]
        L.ora_result.argtypes = [C.c_void_p, _dp]
        L.ora_result_from.argtypes = [C.c_void_p, C.c_int, _dp]
        L.ora_get_grid.argtypes = [C.c_void_p, _dp]
        L.ora_set_grid.argtypes = [C.c_void_p, _dp]
        L.ora_get_hist.argtypes = [C.c_void_p, _dp, _dp]
        L.ora_set_iteration.argtypes = [C.c_void_p, C.c_uint32]
        L.ora_get_iteration.argtypes = [C.c_void_p]
        L.ora_get_iteration.restype = C.c_uint32
        L.ora_observable.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.ora_observable.restype = C.c_double
        L.ora_set_observable.argtypes = [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_int]
        L.ora_get_observable.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.ora_set_strata.argtypes = [C.c_void_p, C.c_int]
        L.ora_strata_cubes.argtypes = [C.c_void_p]
        L.ora_strata_cubes.restype = C.c_int64
        L.ora_strata_npc.argtypes = [C.c_void_p]
        L.ora_strata_npc.restype = C.c_int64
        _i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        L.ora_set_strata_beta.argtypes = [C.c_void_p, C.c_double]
        L.ora_get_strata_counts.argtypes = [C.c_void_p, _i64p]
        L.ora_inject_strata_counts.argtypes = [C.c_void_p, _i64p]
        L.ora_strata_next_counts.argtypes = [C.c_void_p, C.c_int64, _i64p]
        L.ora_event_weights.argtypes = [C.c_void_p, C.c_uint32, C.c_int64, C.c_int64, _dp, _u8p]
        L.ora_grid_map.argtypes = [C.c_void_p, _dp, _dp, C.POINTER(C.c_double),
                                   np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")]
        L.ora_refine_grid.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp]
        L.ora_refine_weights.argtypes = [C.c_int, C.c_double, _dp, _dp]
        L.ora_dy_grad.argtypes = [C.c_void_p, C.c_uint32, C.c_int64, _dp,
                                  C.POINTER(C.c_double), _dp]
        L.ora_dy_weight_theta.argtypes = [C.c_void_p, C.c_uint32, C.c_int64, _dp]
        L.ora_dy_weight_theta.restype = C.c_double
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


def uniforms(seed: int, it: int, event: int, ndim: int) -> np.ndarray:
    u = np.zeros(ndim)
    lib().ora_uniforms(seed, it, event, ndim, u)
    return u


def ndim_of(process: int, ndim: int = 0) -> int:
    return lib().ora_ndim(process, ndim)


def integrand(process: int, params, x) -> float:
    p = _f64(params)
    x = _f64(x)
    return lib().ora_integrand(process, len(x), p, len(p), x)


def observable(process: int, params, x) -> float:
    x = _f64(x)
    p = _f64(params) if len(params) else np.zeros(1)
    return lib().ora_observable(process, len(x), p, x)


def me_dy(params, shat, c, flavour):
    return lib().ora_me_dy(_f64(params), shat, c, flavour)


def sigmahat_dy(params, shat, flavour):
    return lib().ora_sigmahat_dy(_f64(params), shat, flavour)


def me_eemumu_dirac(params, s, c, phi):
    return lib().ora_me_eemumu_dirac(_f64(params), s, c, phi)


def spinor_check(p):
    a, b = C.c_double(), C.c_double()
    lib().ora_spinor_check(_f64(p), C.byref(a), C.byref(b))
    return a.value, b.value


def ww_momenta(params, x):
    mom = np.zeros((6, 4))
    m2p, m2m, jac = C.c_double(), C.c_double(), C.c_double()
    lib().ora_ww_momenta(_f64(params), _f64(x), mom, C.byref(m2p), C.byref(m2m), C.byref(jac))
    return mom, m2p.value, m2m.value, jac.value


def ww_me2(params, mom, m2p, m2m, flavour, helicity):
    return lib().ora_ww_me2(_f64(params), _f64(mom), m2p, m2m, flavour, helicity)


def ww_onshell_me2(params, shat, cth, phi, flavour, helicity, pol_p, pol_m, sign_t=0):
    return lib().ora_ww_onshell_me2(_f64(params), shat, cth, phi, flavour, helicity,
                                    pol_p, pol_m, sign_t)


def refine_weights(nbins, alpha, d):
    m = np.zeros(nbins)
    ok = lib().ora_refine_weights(nbins, alpha, _f64(d), m)
    return m if ok else None


def refine_grid(ndim, nbins, alpha, d, edges):
    e = _f64(edges).copy()
    lib().ora_refine_grid(ndim, nbins, alpha, _f64(d), e)
    return e


class Vegas:
    """The oracle's VEGAS state machine (serial, FP64)."""

    def __init__(self, process, ndim=0, nbins=50, seed=1, alpha=1.5, params=()):
        self.params = _f64(params) if len(params) else np.zeros(1)
        self.ndim = ndim_of(process, ndim)
        self.nbins = nbins
        self._h = lib().ora_create(process, ndim, nbins, seed, alpha, self.params,
                                   len(params))
        if not self._h:
            raise ValueError("invalid oracle configuration")
        self.process = process

    def __del__(self):
        if getattr(self, "_h", None):
            lib().ora_destroy(self._h)
            self._h = None

    def iterate(self, n):
        out = np.zeros(4)
        if lib().ora_iterate(self._h, n, out) != 0:
            raise ValueError("oracle iterate failed")
        H = lib().ora_strata_cubes(self._h)
        used = H * lib().ora_strata_npc(self._h) if H > 0 and not getattr(self, "_adaptive", False) else n
        return {"I": out[0], "var": out[1], "n_nonzero": int(out[2]), "n_nonfinite": int(out[3]),
                "n_events": int(used)}

    def iterate_threads(self, n, nthreads):
        """The same iteration over nthreads threads with fixed chunks and the partials
        added in chunk order (the all-core CPU baseline; plain importance sampling)."""
        out = np.zeros(4)
        if lib().ora_iterate_threads(self._h, n, nthreads, out) != 0:
            raise ValueError("oracle iterate_threads failed")
        return {"I": out[0], "var": out[1], "n_nonzero": int(out[2]), "n_nonfinite": int(out[3]),
                "n_events": int(n)}

    def refine(self):
        if lib().ora_refine(self._h) != 0:
            raise RuntimeError("refine before iterate")

    def result(self, first=0):
        out = np.zeros(4)
        if lib().ora_result_from(self._h, first, out) != 0:
            raise ValueError("no iteration, or first out of range")
        return {"I": out[0], "sigma": out[1], "chi2_dof": out[2], "n_iter": int(out[3])}

    def set_strata(self, m):
        """m strata per axis (0: off); an iteration of n events uses m^D floor(n / m^D)."""
        if lib().ora_set_strata(self._h, m) != 0:
            raise ValueError("invalid strata count")

    def set_strata_beta(self, beta):
        if lib().ora_set_strata_beta(self._h, beta) != 0:
            raise ValueError("invalid beta")
        self._adaptive = beta > 0

    def strata_counts(self):
        H = lib().ora_strata_cubes(self._h)
        c = np.zeros(max(H, 0), dtype=np.int64)
        if lib().ora_get_strata_counts(self._h, c) != 0:
            raise RuntimeError("no stratified iteration yet")
        return c

    def strata_next_counts(self, n):
        H = lib().ora_strata_cubes(self._h)
        c = np.zeros(max(H, 0), dtype=np.int64)
        if lib().ora_strata_next_counts(self._h, n, c) != 0:
            raise ValueError("needs adaptive strata and n >= 2H")
        return c

    def inject_strata_counts(self, counts):
        if lib().ora_inject_strata_counts(self._h, np.ascontiguousarray(counts, dtype=np.int64)) != 0:
            raise ValueError("counts need adaptive strata")

    @property
    def strata_npc(self):
        return lib().ora_strata_npc(self._h)

    def set_observable(self, nbins, lo=0.0, hi=1.0, first=0):
        if lib().ora_set_observable(self._h, nbins, lo, hi, first) != 0:
            raise ValueError("invalid observable binning")
        self.nobs = nbins

    def get_observable(self):
        """(last, last_err, comb, comb_err), each of nbins + 2 (under- and overflow
        at the ends)."""
        k = getattr(self, "nobs", 0) + 2
        a = [np.zeros(k) for _ in range(4)]
        if lib().ora_get_observable(self._h, *a) != 0:
            raise RuntimeError("observable off, or no iteration yet")
        return tuple(a)

    def get_grid(self):
        e = np.zeros((self.ndim, self.nbins + 1))
        lib().ora_get_grid(self._h, e)
        return e

    def set_grid(self, e):
        lib().ora_set_grid(self._h, _f64(e).reshape(-1))

    def get_hist(self):
        d = np.zeros((self.ndim, self.nbins))
        sums = np.zeros(2)
        lib().ora_get_hist(self._h, d, sums)
        return d, sums

    @property
    def iteration(self):
        return lib().ora_get_iteration(self._h)

    @iteration.setter
    def iteration(self, it):
        lib().ora_set_iteration(self._h, it)

    def event_weights(self, it, first, n):
        w = np.zeros(n)
        b = np.zeros((n, self.ndim), dtype=np.uint8)
        lib().ora_event_weights(self._h, it, first, n, w, b)
        return w, b

    def grid_map(self, u):
        x = np.zeros(self.ndim)
        b = np.zeros(self.ndim, dtype=np.int32)
        J = C.c_double()
        lib().ora_grid_map(self._h, _f64(u), x, C.byref(J), b)
        return x, J.value, b

    def dy_grad(self, it, n, theta):
        sig = C.c_double()
        ds = np.zeros(5)
        if lib().ora_dy_grad(self._h, it, n, _f64(theta), C.byref(sig), ds) != 0:
            raise ValueError("dy_grad needs the Drell-Yan process")
        return sig.value, ds

    def dy_weight_theta(self, it, event, theta):
        return lib().ora_dy_weight_theta(self._h, it, event, _f64(theta))
