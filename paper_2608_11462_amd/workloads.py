"""Seeded synthetic inputs for the polyharmonic-spline workloads.

This module only draws points, right-hand sides and targets; it contains none
of the interpolation method's arithmetic.  Both the CPU oracle tests and the
HIP path take their inputs from here, so that the two sides see identical data.

Every generator uses ``numpy.random.Generator(PCG64(seed))``.

Workloads (sizes and distributions follow the paper's setting of scattered 2D
data interpolated by thin-plate and higher-order splines, Sec. 3):

* ``small_tps``   n=2000 uniform in [0,1]^2, k=2, linear block,
                  f = sin(4x)cos(3y) + 0.5x^2, 500 uniform targets.
* ``odd_clustered`` n=100000, 70% uniform + 30% from 10 Gaussian clusters
                  (sigma 0.02), k=3, quadratic block, f = 5 Gaussian bumps plus a
                  linear trend, 50000 uniform targets.
* ``large_tps``   n=2^20 uniform, k=2, linear block, f = a 16-mode random
                  Fourier field with integer wave vectors of norm <= 8.
* ``batched``     many problems of log-uniform size, mixed geometry and order.
* ``stream``      a Poisson stream of solve+evaluate requests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- geometry

def uniform_points(rng: np.random.Generator, n: int) -> np.ndarray:
    """n i.i.d. points uniform in [0,1]^2, shape (n, 2), float64."""
    return rng.random((n, 2))


def clustered_points(rng: np.random.Generator, n: int, frac_clustered: float = 0.3,
                     n_clusters: int = 10, sigma: float = 0.02) -> np.ndarray:
    """Mixture: (1-frac) uniform in [0,1]^2 plus frac split evenly over
    isotropic Gaussian clusters N(c_i, sigma^2 I) with centres c_i ~ U[0,1]^2.
    Cluster points are not clipped, so a few may fall outside the unit square."""
    n_cl = int(round(frac_clustered * n))
    n_uni = n - n_cl
    pts_u = rng.random((n_uni, 2))
    centres = rng.random((n_clusters, 2))
    per = np.full(n_clusters, n_cl // n_clusters, dtype=np.int64)
    per[: n_cl - per.sum()] += 1
    chunks = [pts_u]
    for c, m in zip(centres, per):
        chunks.append(c + sigma * rng.standard_normal((int(m), 2)))
    return np.concatenate(chunks, axis=0)


# ---------------------------------------------------------------- fields

def f_small(xy: np.ndarray) -> np.ndarray:
    """sin(4x)cos(3y) + 0.5 x^2."""
    x, y = xy[:, 0], xy[:, 1]
    return np.sin(4.0 * x) * np.cos(3.0 * y) + 0.5 * x * x


@dataclass
class BumpField:
    """sum_i a_i exp(-|x-b_i|^2/(2 s_i^2)) + e0 + e1 x + e2 y."""
    a: np.ndarray
    b: np.ndarray
    s: np.ndarray
    e: np.ndarray

    def __call__(self, xy: np.ndarray) -> np.ndarray:
        out = self.e[0] + self.e[1] * xy[:, 0] + self.e[2] * xy[:, 1]
        for ai, bi, si in zip(self.a, self.b, self.s):
            d2 = (xy[:, 0] - bi[0]) ** 2 + (xy[:, 1] - bi[1]) ** 2
            out = out + ai * np.exp(-d2 / (2.0 * si * si))
        return out


def bump_field(rng: np.random.Generator, n_bumps: int = 5) -> BumpField:
    a = rng.standard_normal(n_bumps)
    b = rng.random((n_bumps, 2))
    s = rng.uniform(0.05, 0.2, n_bumps)
    e = rng.standard_normal(3)
    return BumpField(a, b, s, e)


@dataclass
class FourierField:
    """sum_m a_m cos(2 pi kappa_m . x + phase_m)."""
    kappa: np.ndarray  # (M, 2) integer wave vectors
    a: np.ndarray
    phase: np.ndarray

    def __call__(self, xy: np.ndarray) -> np.ndarray:
        arg = 2.0 * math.pi * (xy @ self.kappa.T.astype(np.float64)) + self.phase
        return np.cos(arg) @ self.a


def fourier_field(rng: np.random.Generator, n_modes: int = 16, kmax: int = 8) -> FourierField:
    cand = [(i, j) for i in range(-kmax, kmax + 1) for j in range(-kmax, kmax + 1)
            if (i, j) != (0, 0) and i * i + j * j <= kmax * kmax]
    cand = np.array(cand, dtype=np.int64)
    idx = rng.choice(len(cand), size=n_modes, replace=False)
    kappa = cand[idx]
    a = rng.standard_normal(n_modes)
    phase = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    return FourierField(kappa, a, phase)


def f_interp(xy: np.ndarray) -> np.ndarray:
    """The accuracy-study test function of Sec. 3.2 (eq. f_interp)."""
    x1, x2 = xy[:, 0], xy[:, 1]
    return (np.cos(30.0 * x1 + 0.8) * np.sin(30.0 * x2 - 2.1)
            + 5.0 * np.exp(-5.0 * np.sqrt((x1 - 0.25) ** 2 + (x2 - 0.75) ** 2)))


def sobol_points(log2_n: int) -> np.ndarray:
    """The first 2^log2_n points of the (unscrambled) two-dimensional Sobol
    sequence on [0, 1)^2, the node sets of the accuracy experiments of Sec. 3.2
    and 3.3.  Deterministic; shape (2^log2_n, 2)."""
    from scipy.stats import qmc
    return qmc.Sobol(d=2, scramble=False).random_base2(log2_n)


def regrid_targets(g: int = 100) -> np.ndarray:
    """The regular g x g grid on [0, 1]^2 (both ends included) at which the
    interpolants of Sec. 3.2 and 3.3 are evaluated; shape (g*g, 2)."""
    t = np.linspace(0.0, 1.0, g)
    gx, gy = np.meshgrid(t, t, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel()], axis=1)


def f_franke(xy: np.ndarray) -> np.ndarray:
    """The four-term Franke function with the weights, centres and diagonal
    metrics printed in Sec. 3.3."""
    w = (0.75, 0.75, 0.50, -0.20)
    c = ((2.0, 2.0), (-1.0, -1.0), (7.0, 3.0), (4.0, 7.0))
    lam = ((0.25, 0.25), (1.0 / 49.0, 1.0 / 10.0), (0.25, 0.25), (1.0, 1.0))
    out = np.zeros(len(xy))
    for wj, cj, lj in zip(w, c, lam):
        u = 9.0 * xy[:, 0] - cj[0]
        v = 9.0 * xy[:, 1] - cj[1]
        out += wj * np.exp(-(lj[0] * u * u + lj[1] * v * v))
    return out


# ---------------------------------------------------------------- problems

@dataclass
class Problem:
    name: str
    xy: np.ndarray            # (n, 2) float64, user coordinates
    f: np.ndarray             # (n,) or (n, nrhs) float64
    k: int
    degree: int               # total degree of the polynomial block; -1 = minimal for k
    targets: np.ndarray       # (m, 2)
    precond: dict = field(default_factory=dict)  # m, nu, range, range_units

    @property
    def n(self) -> int:
        return self.xy.shape[0]


def small_tps(seed: int = 1, n: int = 2000, n_targets: int = 500) -> Problem:
    rng = rng_for(seed)
    xy = uniform_points(rng, n)
    tg = uniform_points(rng_for(seed + 10), n_targets)
    return Problem("small_tps", xy, f_small(xy), 2, 1, tg,
                   dict(m=20, nu=1.5, range=0.1, range_units="user"))


def odd_clustered(seed: int = 2, n: int = 100000, n_targets: int = 50000) -> Problem:
    rng = rng_for(seed)
    xy = clustered_points(rng, n)
    fld = bump_field(rng)
    tg = uniform_points(rng, n_targets)
    return Problem("odd_clustered", xy, fld(xy), 3, 2, tg,
                   dict(m=50, nu=1.5, range=1.0 / 3.0, range_units="normalized"))


def large_tps(seed: int = 3, n: int = 1 << 20, n_targets: int = 10000) -> Problem:
    rng = rng_for(seed)
    xy = uniform_points(rng, n)
    fld = fourier_field(rng)
    tg = uniform_points(rng, n_targets)
    return Problem("large_tps", xy, fld(xy), 2, 1, tg,
                   dict(m=30, nu=1.0, range=1.0 / 0.35, range_units="normalized"))


def batched(seed: int = 4, n_problems: int = 256, n_lo: int = 1000, n_hi: int = 200000,
            nrhs: int = 4) -> list[Problem]:
    rng = rng_for(seed)
    out = []
    for i in range(n_problems):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        clustered = rng.random() < 0.5
        xy = clustered_points(rng, n) if clustered else uniform_points(rng, n)
        k = int(rng.integers(1, 5))
        f = np.stack([fourier_field(rng)(xy) for _ in range(nrhs)], axis=1)
        m = int(rng.integers(20, 41))
        out.append(Problem(f"batch{i}", xy, f, k, -1, np.zeros((0, 2)),
                           dict(m=m, nu=k / 2.0, range=0.0, range_units="normalized")))
    return out


@dataclass
class Request:
    t_arrival: float
    problem: Problem


def stream(seed: int = 5, n_requests: int = 512, rate: float = 10.0, n_lo: int = 1000,
           n_hi: int = 1000000, n_targets: int = 10000) -> list[Request]:
    """Poisson arrivals at `rate` per second; problem sizes log-uniform."""
    rng = rng_for(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        clustered = rng.random() < 0.5
        xy = clustered_points(rng, n) if clustered else uniform_points(rng, n)
        k = int(rng.choice([2, 3]))
        f = fourier_field(rng)(xy)
        tg = uniform_points(rng, n_targets)
        out.append(Request(t, Problem(f"req{i}", xy, f, k, -1, tg,
                                      dict(m=30 if k == 2 else 50, nu=k / 2.0, range=0.0,
                                           range_units="normalized"))))
    return out


def sample_rows(seed: int, n: int, count: int) -> np.ndarray:
    """Sorted distinct row indices for sampled direct-summation checks."""
    rng = rng_for(seed)
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False))
