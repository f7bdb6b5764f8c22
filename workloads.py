"""Seeded synthetic sample columns and bandwidth grids.

This module only draws numbers: it holds none of the bandwidth-selection
arithmetic, and both the GPU path's tests/benchmark and the CPU oracle's
checks take their inputs from it, so the two sides always see identical bytes.

The paper times its selectors on unspecified "random" data (Section 7.2); the
workloads below stand in for that with named distributions, sizes and grids.
Every draw uses numpy's PCG64 generator from a fixed seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FAMILIES = ("uniform", "normal", "gamma", "bimodal", "mixture", "lognormal")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def draw(family: str, n: int, seed: int, dtype=np.float32) -> np.ndarray:
    """n samples of a named family, stored as `dtype`.

    uniform   U(0, 1)
    normal    N(0, 1)
    gamma     Gamma(shape 2, scale 1)
    bimodal   0.3 N(-3, 1) + 0.7 N(2, 0.5^2)
    mixture   0.5 N(-2, 0.5^2) + 0.5 N(1, 1)
    lognormal exp(N(0, 1))
    Mixtures draw the component indicator first, then both normal arrays.
    """
    rng = _rng(seed)
    if family == "uniform":
        x = rng.random(n)
    elif family == "normal":
        x = rng.standard_normal(n)
    elif family == "gamma":
        x = rng.gamma(2.0, 1.0, n)
    elif family == "bimodal":
        comp = rng.random(n) < 0.3
        a = rng.normal(-3.0, 1.0, n)
        b = rng.normal(2.0, 0.5, n)
        x = np.where(comp, a, b)
    elif family == "mixture":
        comp = rng.random(n) < 0.5
        a = rng.normal(-2.0, 0.5, n)
        b = rng.normal(1.0, 1.0, n)
        x = np.where(comp, a, b)
    elif family == "lognormal":
        x = rng.lognormal(0.0, 1.0, n)
    else:
        raise ValueError(f"unknown family {family!r}")
    return np.ascontiguousarray(x.astype(dtype))


@dataclass
class Workload:
    name: str
    family: str
    n: int
    seed: int
    dtype: type
    grid: np.ndarray
    stages: int
    note: str = ""
    extra: dict = field(default_factory=dict)

    def column(self) -> np.ndarray:
        return draw(self.family, self.n, self.seed, self.dtype)


def workload(name: str) -> Workload:
    """The single-column workloads.

    plain-1k      n = 1,000 float64 N(0,1); LSCV over 100 log-spaced h in [0.01, 1];
                  two-stage plug-in.
    mixture-100k  n = 100,000 float32 0.5 N(-2,0.5^2) + 0.5 N(1,1); LSCV over 256
                  log-spaced h in [0.005, 2]; three-stage plug-in.
    lognormal-1m  n = 1,000,000 float32 lognormal(0,1); LSCV over 512 log-spaced h
                  in [0.00225, 0.58]; three-stage plug-in.  The range spans
                  [h_ref/64, 4 h_ref] for h_ref = 0.1444, the normal-reference
                  bandwidth of the lognormal(0,1) law's own standard deviation
                  (2.1612) at this n, rounded outwards.
    """
    if name == "plain-1k":
        return Workload(name, "normal", 1000, 1998001, np.float64, np.geomspace(0.01, 1.0, 100), 2)
    if name == "mixture-100k":
        return Workload(name, "mixture", 100_000, 1998002, np.float32, np.geomspace(0.005, 2.0, 256), 3)
    if name == "lognormal-1m":
        return Workload(name, "lognormal", 1_000_000, 1998003, np.float32, np.geomspace(0.00225, 0.58, 512), 3)
    raise ValueError(f"unknown workload {name!r}")


WORKLOADS = ("plain-1k", "mixture-100k", "lognormal-1m")

BATCH_FAMILIES = ("uniform", "normal", "gamma", "bimodal")


@dataclass
class ColumnSpec:
    family: str
    n: int
    seed: int

    def column(self, dtype=np.float32) -> np.ndarray:
        return draw(self.family, self.n, self.seed, dtype)


def batch_columns(count: int = 512, seed: int = 1998004, n_lo: float = 1e3, n_hi: float = 2e5):
    """Uneven columns for the batched workload: n = round(exp(U(ln n_lo, ln n_hi))),
    family uniform over uniform(0,1), N(0,1), Gamma(2,1), 0.3N(-3,1)+0.7N(2,0.5^2);
    each column draws from its own child of SeedSequence(seed)."""
    rng = _rng(seed)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count))).astype(np.int64)
    fam = rng.integers(0, len(BATCH_FAMILIES), count)
    kids = np.random.SeedSequence(seed).spawn(count)
    return [ColumnSpec(BATCH_FAMILIES[int(f)], int(n), int(k.generate_state(1)[0])) for n, f, k in zip(ns, fam, kids)]


@dataclass
class Arrival:
    t: float
    spec: ColumnSpec


def served_stream(count: int | None = None, seed: int = 1998005, rate: float = 200.0, duration: float = 60.0,
                  n_lo: float = 2e3, n_hi: float = 2e6):
    """The served workload: Poisson arrivals at `rate` per second over
    `duration` seconds, n log-uniform in [n_lo, n_hi], family uniform over the
    four batch families; each request draws from its own child seed.  The
    whole stream is drawn first, so the first `count` requests (all when
    None) are the same prefix whatever count is asked for."""
    rng = _rng(seed)
    m = int(rate * duration + 10.0 * np.sqrt(rate * duration) + 10)
    t = np.cumsum(rng.exponential(1.0 / rate, m))
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), m))).astype(np.int64)
    fam = rng.integers(0, len(BATCH_FAMILIES), m)
    total = int(np.searchsorted(t, duration, side="right"))
    count = total if count is None else min(int(count), total)
    kids = np.random.SeedSequence(seed).spawn(count)
    return [Arrival(float(t[k]), ColumnSpec(BATCH_FAMILIES[int(fam[k])], int(ns[k]), int(kids[k].generate_state(1)[0])))
            for k in range(count)]


# Batched and served requests: plug-in with three stages and LSCV over 128
# points log-spaced over h_rot * [1/64, 4] (the optimum of skewed and
# multimodal columns lies well below h_rot).
BATCH_GRID = ("log_rot", 1.0 / 64.0, 4.0, 128)
BATCH_STAGES = 3


def draw_matrix(n: int, d: int, seed: int, dtype=np.float32) -> np.ndarray:
    """n x d samples, row-major: a two-component Gaussian mixture with
    correlated coordinates (35% of the samples in a tighter component shifted
    by 3 in every coordinate), the 2-D/d-D stand-in for the multivariate
    selectors and consumers."""
    rng = _rng(seed)
    A = rng.standard_normal((d, d)) + 2 * np.eye(d)
    comp = rng.random(n) < 0.35
    z = rng.standard_normal((n, d)) @ A.T
    z[comp] = 0.4 * z[comp] + 3.0
    return np.ascontiguousarray(z.astype(dtype))
