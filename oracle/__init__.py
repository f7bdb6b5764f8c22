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
    lib.orc_density_H.argtypes = [PD, L, I, PD, PD, I, PD]
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


def density_H(x, H, points) -> np.ndarray:
    """Density estimate with bandwidth matrix H at points (m x d), eq. (kde-def-H)."""
    a = np.ascontiguousarray(np.asarray(x, np.float64))
    if a.ndim == 1:
        a = a[:, None]
    n, d = a.shape
    Hm = np.ascontiguousarray(np.asarray(H, np.float64).reshape(d, d))
    p = np.ascontiguousarray(np.asarray(points, np.float64).reshape(-1, d))
    out = np.empty(p.shape[0], np.float64)
    _check(_load().orc_density_H(_p(a.ravel()), n, d, _p(Hm.ravel()), _p(p.ravel()), p.shape[0], _p(out)),
           "density_H")
    return out


def range_aggregates_2d(x, H, boxes):
    """COUNT, SUM of the first and SUM of the second coordinate over boxes
    [a, b] x [c, d] (rows of ``boxes``: a, b, c, d), eq. (count-sum-2D) with
    the density estimate of eq. (kde-def-H), d = 2.

    Per sample the kernel is a bivariate normal with mean X_i and covariance
    H.  In its standardised coordinates U (first) and V (second), corr rho,
    V given U = z is normal with mean rho z and deviation s = sqrt(1 - rho^2),
    so over the standardised box [al1, be1] x [al2, be2]
      P     = int_al1^be1 phi(z) B(z) dz,   B(z) = Phi(b'(z)) - Phi(a'(z)),
      E[U]  = int_al1^be1 z phi(z) B(z) dz,
      E[V]  = int_al1^be1 phi(z) (rho z B(z) + s (phi(a'(z)) - phi(b'(z)))) dz,
    a'(z) = (al2 - rho z)/s, b'(z) = (be2 - rho z)/s, each integral taken by
    adaptive quadrature (scipy's quad, relative tolerance 1e-12, absolute
    1e-15 of the kernel's unit mass) with break points at 0 and where B
    changes.  COUNT = sum_i P_i, SUM_x = sum_i (x_i P_i +
    sqrt(H11) E[U]_i), SUM_y = sum_i (y_i P_i + sqrt(H22) E[V]_i).  Pure
    Python per sample: for small n only."""
    import warnings

    from scipy import integrate
    from scipy.special import ndtr

    a = np.asarray(x, np.float64)
    if a.ndim != 2 or a.shape[1] != 2 or a.shape[0] < 1 or not np.all(np.isfinite(a)):
        raise OracleError(INVAL, "range_aggregates_2d")
    Hm = np.asarray(H, np.float64).reshape(2, 2)
    s1, s2 = np.sqrt(Hm[0, 0]), np.sqrt(Hm[1, 1])
    if not (Hm[0, 0] > 0 and Hm[1, 1] > 0) or not np.all(np.isfinite(Hm)):
        raise OracleError(DEGENERATE, "range_aggregates_2d")
    rho = Hm[1, 0] / (s1 * s2)
    if not (abs(rho) < 1.0 - 1e-12):
        raise OracleError(DEGENERATE, "range_aggregates_2d")
    s = np.sqrt((1.0 - rho) * (1.0 + rho))
    bx = np.asarray(boxes, np.float64).reshape(-1, 4)
    if np.any(np.isnan(bx)) or np.any(bx[:, 0] > bx[:, 1]) or np.any(bx[:, 2] > bx[:, 3]):
        raise OracleError(INVAL, "range_aggregates_2d")
    phi = lambda z: np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)  # noqa: E731
    cnt, sx, sy = (np.zeros(bx.shape[0]) for _ in range(3))
    for k, (lo1, hi1, lo2, hi2) in enumerate(bx):
        if lo1 == hi1 or lo2 == hi2:
            continue
        for xi, yi in a:
            al1, be1 = (lo1 - xi) / s1, (hi1 - xi) / s1
            al2, be2 = (lo2 - yi) / s2, (hi2 - yi) / s2
            z0, z1 = max(al1, -40.0), min(be1, 40.0)
            if not z1 > z0:
                continue

            def B(z):
                return ndtr((be2 - rho * z) / s) - ndtr((al2 - rho * z) / s)

            def C(z):
                ap, bp = (al2 - rho * z) / s, (be2 - rho * z) / s
                pa = 0.0 if np.isinf(ap) else phi(ap)
                pb = 0.0 if np.isinf(bp) else phi(bp)
                return rho * z * B(z) + s * (pa - pb)

            pts = []
            if rho != 0.0:
                w = s / abs(rho)
                for c in (al2 / rho, be2 / rho):
                    if np.isfinite(c):
                        pts += [c + f * w for f in (-30, -10, -3, -1, 0, 1, 3, 10, 30)]
            pts = sorted(p for p in pts + [0.0] if z0 < p < z1)
            kw = dict(epsabs=1e-15, epsrel=1e-12, limit=400)
            if pts:
                kw["points"] = pts
            with warnings.catch_warnings():
                # integrals that vanish (E[U] over the whole line) cannot meet a
                # relative tolerance; the absolute one still holds
                warnings.simplefilter("ignore", integrate.IntegrationWarning)
                P = integrate.quad(lambda z: phi(z) * B(z), z0, z1, **kw)[0]
                EU = integrate.quad(lambda z: z * phi(z) * B(z), z0, z1, **kw)[0]
                EV = integrate.quad(lambda z: phi(z) * C(z), z0, z1, **kw)[0]
            cnt[k] += P
            sx[k] += xi * P + s1 * EU
            sy[k] += yi * P + s2 * EV
    return cnt, sx, sy
