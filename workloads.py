"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no part of the method's arithmetic: it only draws points,
feature windows, hyper-parameters, right-hand sides and Rademacher probes.
Every stream is numpy's counter-based Philox generator with a stated seed.

The five workloads follow the shapes of the paper's experiments (bandwidth 32,
additive windows of dimension at most three, a few windows, many probe
vectors) sized up to a single MI355X; the paper's own data sets are not used.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

GAUSS = 0
MATERN12 = 1
MATERN32 = 2
MQ = 3
IMQ = 4
SINC = 5


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def rademacher(n: int, k: int, seed: int) -> np.ndarray:
    """n x k matrix of independent +-1 entries with probability 1/2 each."""
    bits = rng(seed).integers(0, 2, size=(n, k), dtype=np.int8)
    return (2.0 * bits - 1.0).astype(np.float64)


@dataclass
class Workload:
    name: str
    X: np.ndarray                 # n x p, float64
    windows: List[List[int]]      # disjoint feature windows, 0-based
    ktype: List[int]              # per window GAUSS / MATERN12
    ell: List[float]              # per window, caller units
    sigma_f: float
    sigma_eps: float
    N: List[int]                  # per window bandwidth
    m: int                        # window cutoff
    V: np.ndarray                 # n x nrhs right-hand sides
    scale_mode: int = 0           # 0 = auto, 1 = none (points already in the box)
    prec: str = "f32"
    y: np.ndarray = None          # regression targets (differentiation workload)
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def nrhs(self):
        return self.V.shape[1]


def c1(seed=11):
    """n = 2000 uniform in [-1/4, 1/4)^3, one 3-D Gaussian window, ell = 0.1,
    N = 32, m = 4, one N(0,1) vector, FP64."""
    X = rng(seed).uniform(-0.25, 0.25, size=(2000, 3))
    V = rng(seed + 1).standard_normal((2000, 1))
    return Workload("C1 n=2000 p=3 1x3D gauss N=32 m=4 f64", X, [[0, 1, 2]], [GAUSS], [0.1],
                    1.0, 0.0, [32], 4, V, scale_mode=1, prec="f64")


def c2(seed=21, n=100_000):
    """n = 100,000, p = 9 standard normal features, three 3-D Gaussian windows,
    ell = 0.5 (caller units), sigma_f = 1, sigma_eps = 0.1, N = 32, m = 4, one vector."""
    X = rng(seed).standard_normal((n, 9))
    V = rng(seed + 1).standard_normal((n, 1))
    return Workload(f"C2 n={n} p=9 3x3D gauss N=32 m=4 1rhs", X, [[0, 1, 2], [3, 4, 5], [6, 7, 8]],
                    [GAUSS] * 3, [0.5] * 3, 1.0, 0.1, [32] * 3, 4, V)


def c3(seed=31, n=500_000, nrhs=32):
    """n = 500,000, p = 12 standard normal features, windows of sizes 3,3,2,2,1,1,
    Matern-1/2, ell = 1.0, N = 32 for d = 3 and 64 for d <= 2, m = 4,
    32 Rademacher probes."""
    X = rng(seed).standard_normal((n, 12))
    wins = [[0, 1, 2], [3, 4, 5], [6, 7], [8, 9], [10], [11]]
    Ns = [32 if len(w) == 3 else 64 for w in wins]
    V = rademacher(n, nrhs, seed + 1)
    return Workload(f"C3 n={n} p=12 windows 3,3,2,2,1,1 matern N=32/64 m=4 {nrhs}rhs", X, wins,
                    [MATERN12] * 6, [1.0] * 6, 1.0, 0.1, Ns, 4, V)


def c4(seed=41, n=200_000, nprobe=16):
    """n = 200,000, p = 8 uniform features in [0,1), windows 3,3,2, Gaussian,
    y = sum_w sin(2 pi sum_{f in w} x_f) + N(0, 0.1^2), theta = (1.0, 0.2, 0.1),
    N = 32, m = 4; right-hand sides [y | 16 Rademacher probes]."""
    X = rng(seed).uniform(0.0, 1.0, size=(n, 8))
    wins = [[0, 1, 2], [3, 4, 5], [6, 7]]
    y = sum(np.sin(2 * np.pi * X[:, w].sum(axis=1)) for w in wins)
    y = y + 0.1 * rng(seed + 1).standard_normal(n)
    Z = rademacher(n, nprobe, seed + 2)
    V = np.concatenate([y[:, None], Z], axis=1)
    return Workload(f"C4 n={n} p=8 windows 3,3,2 gauss N=32 m=4 y+{nprobe} probes", X, wins,
                    [GAUSS] * 3, [0.2] * 3, 1.0, 0.1, [32] * 3, 4, V, y=y)


def c5(seed=51, n=2_000_000, nrhs=16):
    """n = 2,000,000, p = 20 standard normal features, six 3-D windows and one
    2-D window, kernels G,M,G,M,G,M (3-D) and G (2-D), ell = 1.0, N = 64, m = 6,
    16 N(0,1) vectors."""
    X = rng(seed).standard_normal((n, 20))
    wins = [[3 * i, 3 * i + 1, 3 * i + 2] for i in range(6)] + [[18, 19]]
    kt = [GAUSS, MATERN12] * 3 + [GAUSS]
    V = rng(seed + 1).standard_normal((n, nrhs))
    return Workload(f"C5 n={n} p=20 6x3D+1x2D mixed N=64 m=6 {nrhs}rhs", X, wins, kt, [1.0] * 7,
                    1.0, 0.1, [64] * 7, 6, V)


def cube6(seed=100, n=3000, ktype=MATERN12, ell=2.0, N=32, m=6):
    """The synthetic set of the preconditioned-iteration study (Sec. 5.1): n
    points uniform in a 6-D hypercube of side n^(1/3), two 3-D windows,
    sigma_f^2 = 1/P, sigma_eps^2 = 0.01, right-hand side uniform in
    [-0.5, 0.5]."""
    g = rng(seed)
    X = g.uniform(0.0, n ** (1.0 / 3.0), size=(n, 6))
    V = g.uniform(-0.5, 0.5, size=(n, 1))
    return Workload(f"cube6 n={n} 2x3D kernel={ktype} ell={ell}", X, [[0, 1, 2], [3, 4, 5]], [ktype] * 2,
                    [ell] * 2, float(np.sqrt(0.5)), 0.1, [N] * 2, m, V)


def unit6(seed=101, n=3000, ktype=GAUSS, ell=0.5, N=32, m=4):
    """The synthetic regression set of the estimator-variance study (Sec. 5.1):
    n points uniform in [0, 1]^6, y_i = sin(2 pi x_i)^T exp(x_i) + ||x_i||^2
    + N(0, 0.01) noise, two 3-D windows."""
    g = rng(seed)
    X = g.uniform(0.0, 1.0, size=(n, 6))
    y = np.sum(np.sin(2.0 * np.pi * X) * np.exp(X), axis=1) + np.sum(X * X, axis=1) + 0.1 * g.standard_normal(n)
    return Workload(f"unit6 n={n} 2x3D kernel={ktype}", X, [[0, 1, 2], [3, 4, 5]], [ktype] * 2, [ell] * 2,
                    1.0, 0.1, [N] * 2, m, y[:, None], y=y)


def small(seed, n, dims, ktypes, ell, N, m, nrhs, sigma_f=1.0, sigma_eps=0.1, dist="normal",
          scale_mode=0, prec="f32"):
    """Generic small case: windows of the given dimensions over consecutive features."""
    p = int(sum(dims))
    g = rng(seed)
    if dist == "normal":
        X = g.standard_normal((n, p))
    elif dist == "box":
        X = g.uniform(-0.25, 0.25, size=(n, p))
    elif dist == "cluster":
        centers = g.uniform(-3, 3, size=(4, p))
        X = centers[g.integers(0, 4, size=n)] + 0.05 * g.standard_normal((n, p))
    else:
        X = g.uniform(0.0, 1.0, size=(n, p))
    wins, f = [], 0
    for d in dims:
        wins.append(list(range(f, f + d)))
        f += d
    P = len(dims)
    kt = ktypes if isinstance(ktypes, (list, tuple)) else [ktypes] * P
    el = ell if isinstance(ell, (list, tuple)) else [ell] * P
    Ns = N if isinstance(N, (list, tuple)) else [N] * P
    V = rng(seed + 1).standard_normal((n, nrhs))
    return Workload(f"small n={n} dims={dims}", X, wins, list(kt), list(el), sigma_f, sigma_eps,
                    list(Ns), m, V, scale_mode=scale_mode, prec=prec)


CONFIGS = {"C1": c1, "C2": c2, "C3": c3, "C4": c4, "C5": c5}
