"""FP64 CPU oracle for exact KDE bandwidth-selection sums.

TEST INFRASTRUCTURE ONLY.  This package is the checker that the GPU library is
compared against.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import it; the library itself never loads it and has no CPU
fallback.  It shares no code with the GPU path: the arithmetic lives in
``kde_oracle.c`` (plain C, FP64), which cites the paper's equations
(Andrzejewski, Gramacki, Gramacki, arXiv 1505.01998, Section 4.4); this module
only compiles it with gcc and marshals numpy arrays through ctypes.

Inputs stored as float32 are upcast exactly to float64 before the call, so
the oracle sees the same sample values the GPU path does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kde_oracle.c")
_LIB = os.path.join(_HERE, "libkde_oracle.so")

OK, INVAL, DEGENERATE, NOMEM = 0, 1, 2, 3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile kde_oracle.c into libkde_oracle.so (gcc -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _PluginInfo(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_double),
        ("h_rot", ctypes.c_double),
        ("stages", ctypes.c_int),
        ("g", ctypes.c_double * 3),
        ("psi", ctypes.c_double * 3),
        ("kappa", ctypes.c_double * 3),
        ("h", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    D = ctypes.c_double
    PD = ctypes.POINTER(ctypes.c_double)
    PI = ctypes.POINTER(ctypes.c_int)
    L = ctypes.c_long
    I = ctypes.c_int
    lib.orc_num_threads.restype = I
    lib.orc_set_threads.argtypes = [I]
    lib.orc_validate.argtypes = [PD, L]
    lib.orc_moments.argtypes = [PD, L, PD, PD]
    lib.orc_rot.argtypes = [PD, L, PD, PD]
    lib.orc_hermite_e.argtypes = [I, D]
    lib.orc_hermite_e.restype = D
    lib.orc_kernel_deriv.argtypes = [I, D]
    lib.orc_kernel_deriv.restype = D
    lib.orc_pair_sum_kr.argtypes = [PD, L, I, D, PD, PD]
    lib.orc_psi.argtypes = [PD, L, I, D, PD, PD, PD, PD]
    lib.orc_psi_ns.argtypes = [I, D]
    lib.orc_psi_ns.restype = D
    lib.orc_pilot.argtypes = [I, D, L, PD]
    lib.orc_plugin.argtypes = [PD, L, I, ctypes.POINTER(_PluginInfo)]
    lib.orc_default_grid.argtypes = [PD, L, I, PD]
    lib.orc_lscv_curve.argtypes = [PD, L, PD, I, PD, PD, PD, PD]
    lib.orc_lscv_block_sums.argtypes = [PD, L, L, L, L, L, PD, I, PD, PD]
    lib.orc_argmin.argtypes = [PD, I, PI, PI, PD]
    lib.orc_lscv.argtypes = [PD, L, PD, I, PD, PI, PI]
    lib.orc_lscv_min.argtypes = [PD, L, D, D, D, I, PD, PD, PI, PD, PD]
    lib.orc_density.argtypes = [PD, L, D, PD, I, PD]
    lib.orc_lscv_md_curve.argtypes = [PD, L, I, PD, I, PD, PD, PD, PD]
    lib.orc_lscv_H.argtypes = [PD, L, I, PD, PD]
    lib.orc_lscv_H_min.argtypes = [PD, L, I, D, D, I, PD, PD, PI]
    lib.orc_range_aggregates.argtypes = [PD, L, D, PD, PD, I, PD, PD]
    _lib = lib
    return lib


def _col(x) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x), dtype=np.float64)
    if a.ndim != 1:
        raise ValueError("sample column must be one-dimensional")
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(st: int, what: str):
    if st != OK:
        raise OracleError(st, what)


def num_threads() -> int:
    return _load().orc_num_threads()


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


def moments(x):
    """(mean, variance with n-1 denominator) -- eq. (PLUGIN-VarianceEstimator)."""
    a = _col(x)
    m, v = ctypes.c_double(), ctypes.c_double()
    _check(_load().orc_moments(_p(a), a.size, ctypes.byref(m), ctypes.byref(v)), "moments")
    return m.value, v.value


def bw_rot(x):
    """(sigma_hat, h_rot) -- normal-reference rule, eq. (LSCV-H-start) with d = 1."""
    a = _col(x)
    s, h = ctypes.c_double(), ctypes.c_double()
    _check(_load().orc_rot(_p(a), a.size, ctypes.byref(s), ctypes.byref(h)), "rot")
    return s.value, h.value


def hermite_e(r: int, u: float) -> float:
    return _load().orc_hermite_e(int(r), float(u))


def kernel_deriv(r: int, u: float) -> float:
    """K^(r)(u) = He_r(u) phi(u)."""
    return _load().orc_kernel_deriv(int(r), float(u))


def pair_sum_kr(x, r: int, g: float):
    """(sum_{i<j} K^(r)((x_i-x_j)/g), sum_{i<j} |K^(r)(...)|)."""
    a = _col(x)
    s, t = ctypes.c_double(), ctypes.c_double()
    _check(_load().orc_pair_sum_kr(_p(a), a.size, int(r), float(g), ctypes.byref(s), ctypes.byref(t)),
           "pair_sum_kr")
    return s.value, t.value


def psi(x, r: int, g: float):
    """(psi_r(g), kappa, pair_sum, pair_abs_sum) -- eq. (PLUGIN-Psi6Estimate)/(PLUGIN-Psi4Estimate)."""
    a = _col(x)
    out = [ctypes.c_double() for _ in range(4)]
    _check(_load().orc_psi(_p(a), a.size, int(r), float(g), *[ctypes.byref(o) for o in out]), "psi")
    return tuple(o.value for o in out)


def psi_ns(r: int, sigma: float) -> float:
    """Normal-scale psi_r; r = 8 is eq. (PLUGIN-Psi8Estimate)."""
    return _load().orc_psi_ns(int(r), float(sigma))


def pilot(r: int, psi_next: float, n: int) -> float:
    """AMSE pilot g for psi_r given psi_{r+2} -- eq. (PLUGIN-g1)/(PLUGIN-g2)."""
    g = ctypes.c_double()
    _check(_load().orc_pilot(int(r), float(psi_next), int(n), ctypes.byref(g)), "pilot")
    return g.value


@dataclass
class PluginInfo:
    sigma: float
    h_rot: float
    stages: int
    g: tuple
    psi: tuple
    kappa: tuple
    h: float


def bw_plugin(x, stages: int = 2) -> PluginInfo:
    """Direct plug-in selector, Section 4.4.1 (stages = 2 as printed, 3 adds a pairwise psi_8)."""
    a = _col(x)
    info = _PluginInfo()
    _check(_load().orc_plugin(_p(a), a.size, int(stages), ctypes.byref(info)), "plugin")
    return PluginInfo(info.sigma, info.h_rot, info.stages, tuple(info.g), tuple(info.psi),
                      tuple(info.kappa), info.h)


def default_grid(x, n_h: int = 150) -> np.ndarray:
    """Linear grid over sigma * [h0/4, 4 h0], eq. (LSCV-Zh0)."""
    a = _col(x)
    m = n_h if n_h > 0 else 150
    out = np.empty(m, dtype=np.float64)
    _check(_load().orc_default_grid(_p(a), a.size, int(n_h), _p(out)), "default_grid")
    return out


@dataclass
class LscvCurve:
    g: np.ndarray
    gscale: np.ndarray
    s1: np.ndarray  # sum_{i<j} exp(-D^2 / (4 h^2))
    s2: np.ndarray  # sum_{i<j} exp(-D^2 / (2 h^2))


def lscv_curve(x, grid) -> LscvCurve:
    """g(h) over a grid -- eq. (LSCV-gh) in data units, plus gscale and the raw pair sums."""
    a = _col(x)
    gr = _col(grid)
    m = gr.size
    g, gs, s1, s2 = (np.empty(m, dtype=np.float64) for _ in range(4))
    _check(_load().orc_lscv_curve(_p(a), a.size, _p(gr), m, _p(g), _p(gs), _p(s1), _p(s2)), "lscv_curve")
    return LscvCurve(g, gs, s1, s2)


def lscv_block_sums(x, i0: int, i1: int, j0: int, j1: int, grid):
    """(s1, s2) over the triangle block i in [i0, i1), j in [j0, j1), j > i."""
    a = _col(x)
    gr = _col(grid)
    s1 = np.empty(gr.size, np.float64)
    s2 = np.empty(gr.size, np.float64)
    _check(_load().orc_lscv_block_sums(_p(a), a.size, int(i0), int(i1), int(j0), int(j1), _p(gr), gr.size,
                                       _p(s1), _p(s2)), "lscv_block_sums")
    return s1, s2


def argmin(g):
    """(k, at_edge, margin) -- eq. (LSCV-finalH) on a grid, ties to the lowest index."""
    a = _col(g)
    k, e, mg = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(_load().orc_argmin(_p(a), a.size, ctypes.byref(k), ctypes.byref(e), ctypes.byref(mg)), "argmin")
    return k.value, bool(e.value), mg.value


def bw_lscv(x, grid):
    """(h, k, at_edge) -- the grid point minimising g(h)."""
    a = _col(x)
    gr = _col(grid)
    h, k, e = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
    _check(_load().orc_lscv(_p(a), a.size, _p(gr), gr.size, ctypes.byref(h), ctypes.byref(k), ctypes.byref(e)),
           "lscv")
    return h.value, k.value, bool(e.value)


def lscv_min(x, lo: float, hi: float, tol: float = 1e-4, points: int = 16):
    """(h, g, steps, (a, b)) -- LSCV bandwidth by the log-spaced k-section search
    over [lo, hi] (Section 4.4.2's alternative to the brute-force grid)."""
    a = _col(x)
    h, g, a0, b0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = ctypes.c_int()
    _check(_load().orc_lscv_min(_p(a), a.size, float(lo), float(hi), float(tol), int(points), ctypes.byref(h),
                                ctypes.byref(g), ctypes.byref(st), ctypes.byref(a0), ctypes.byref(b0)), "lscv_min")
    return h.value, g.value, st.value, (a0.value, b0.value)


def density(x, h: float, points) -> np.ndarray:
    """Density estimate at the points, eq. (kde-def), Gaussian kernel."""
    a = _col(x)
    p = _col(points)
    out = np.empty(p.size, np.float64)
    _check(_load().orc_density(_p(a), a.size, float(h), _p(p), p.size, _p(out)), "density")
    return out


def range_aggregates(x, h: float, lo, hi):
    """(count, sum) over the ranges [lo[k], hi[k]]: n times the integrals of f
    and x f over the range, eq. (count) and eq. (sum)."""
    a = _col(x)
    l = _col(lo)
    u = _col(hi)
    cnt = np.empty(l.size, np.float64)
    sm = np.empty(l.size, np.float64)
    _check(_load().orc_range_aggregates(_p(a), a.size, float(h), _p(l), _p(u), l.size, _p(cnt), _p(sm)),
           "range_aggregates")
    return cnt, sm


def lscv_md_curve(x, grid) -> LscvCurve:
    """LSCV_h for d-dimensional samples (rows of x, n x d), sphered by the
    sample covariance: eq. (LSCV-gh) with S(v) of eq. (LSCV_MOD-Pv)."""
    a = np.ascontiguousarray(np.asarray(x, np.float64))
    if a.ndim == 1:
        a = a[:, None]
    n, d = a.shape
    gr = _col(grid)
    m = gr.size
    g, gs, s1, s2 = (np.empty(m, dtype=np.float64) for _ in range(4))
    _check(_load().orc_lscv_md_curve(_p(a.ravel()), n, d, _p(gr), m, _p(g), _p(gs), _p(s1), _p(s2)), "lscv_md_curve")
    return LscvCurve(g, gs, s1, s2)


def lscv_H(x, H) -> float:
    """LSCV_H objective g(H), eq. (LSCV_MULTI-gh), at a bandwidth matrix H."""
    a = np.ascontiguousarray(np.asarray(x, np.float64))
    if a.ndim == 1:
        a = a[:, None]
    n, d = a.shape
    Hm = np.ascontiguousarray(np.asarray(H, np.float64).reshape(d, d))
    g = ctypes.c_double()
    _check(_load().orc_lscv_H(_p(a.ravel()), n, d, _p(Hm.ravel()), ctypes.byref(g)), "lscv_H")
    return g.value


def lscv_H_min(x, ftol: float = 1e-10, xtol: float = 1e-6, max_evals: int = 2000):
    """(H, g, evaluations) -- Nelder-Mead over the Cholesky parametrisation of H."""
    a = np.ascontiguousarray(np.asarray(x, np.float64))
    if a.ndim == 1:
        a = a[:, None]
    n, d = a.shape
    H = np.empty(d * d, np.float64)
    g = ctypes.c_double()
    ev = ctypes.c_int()
    _check(_load().orc_lscv_H_min(_p(a.ravel()), n, d, float(ftol), float(xtol), int(max_evals), _p(H),
                                  ctypes.byref(g), ctypes.byref(ev)), "lscv_H_min")
    return H.reshape(d, d), g.value, ev.value
