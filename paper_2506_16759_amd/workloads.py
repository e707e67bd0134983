"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the oracle.

This module holds no arithmetic of the construction method: it only draws point
clouds, low-rank factors and problem lists from NumPy's seeded generators, with
the shapes and distributions of the paper's workloads (uniform point clouds in
the unit square/cube, Sec. V-A; a Gaussian low-rank update, Sec. V-A last
paragraph).

Points are returned structure-of-arrays: a C-contiguous float64 array of shape
(dim, n), row ``a`` holding coordinate ``a`` of every point in input order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def uniform_points(n: int, dim: int, seed: int) -> np.ndarray:
    """n points uniform in [0,1)^dim drawn as ``default_rng(seed).random((n, dim))``."""
    if n < 0 or dim not in (1, 2, 3):
        raise ValueError("n >= 0 and dim in {1,2,3} required")
    rng = np.random.default_rng(seed)
    pts = rng.random((n, dim))
    return np.ascontiguousarray(pts.T)


def gaussian_factors(n: int, r: int, seed: int):
    """U, V of shape (n, r), i.i.d. N(0,1)/sqrt(n); U drawn first, then V."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((n, r)) / math.sqrt(n)
    v = rng.standard_normal((n, r)) / math.sqrt(n)
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


def gaussian_vectors(n: int, k: int, seed: int) -> np.ndarray:
    """Test vectors for matvec/error checks: (n, k) i.i.d. N(0,1), column-major friendly."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, k)))


@dataclass
class Workload:
    """One build problem: points plus kernel and construction parameters."""
    name: str
    n: int
    dim: int
    point_seed: int
    kernel: str = "exp"          # "exp": exp(-r/l); "gauss": exp(-r^2/(2 l^2))
    length: float = 0.2
    leaf_size: int = 64
    eta: float = 0.7
    tol: float = 1e-6
    d0: int = 32
    d_inc: int = 16
    omega_seed: int = 1000
    extra: dict = field(default_factory=dict)

    def points(self) -> np.ndarray:
        return uniform_points(self.n, self.dim, self.point_seed)


# Exponential covariance in the unit square, 4096 points (small parity case).
SMALL_2D = Workload("exp2d_n4096", n=4096, dim=2, point_seed=0, kernel="exp",
                    length=0.1, leaf_size=64, eta=0.7, tol=1e-6, omega_seed=1000)

# Exponential covariance (length 0.2) in the unit cube, 131072 points: the
# timed workload.
CUBE_131K = Workload("exp3d_n131072", n=131072, dim=3, point_seed=1, kernel="exp",
                     length=0.2, leaf_size=64, eta=0.7, tol=1e-6, omega_seed=1001)


def batch_problems(count: int = 64, seed: int = 4):
    """List of independent covariance problems for the batched build.

    N log-uniform in [2048, 65536], dim in {2,3}, kernel exp or gauss, length
    uniform in [0.05, 0.3]; points of problem i from seed 100+i.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(2048), math.log(65536)))))
        dim = int(rng.integers(2, 4))
        kern = "exp" if rng.integers(0, 2) == 0 else "gauss"
        length = float(rng.uniform(0.05, 0.3))
        out.append(Workload(f"batch{i}", n=n, dim=dim, point_seed=100 + i, kernel=kern,
                            length=length, leaf_size=64, eta=0.7, tol=1e-6,
                            omega_seed=2000 + i))
    return out


@dataclass
class UpdateWorkload:
    """Low-rank update of an H^2 matrix: A = H + U V^T, with H the H^2
    matrix of ``base`` and U, V = gaussian_factors(n, rank, factor_seed).
    Omega of the update is keyed by ``omega_seed`` (Omega' by omega_seed + 1)."""
    name: str
    base: Workload
    rank: int = 64
    factor_seed: int = 3
    omega_seed: int = 1002
    tol: float = 1e-6
    d0: int = 32
    d_inc: int = 16
    d_max: int = 256
    oversample: int = 5   # flat spectra of the update's block rows need a sampling margin

    @property
    def n(self) -> int:
        return self.base.n

    def factors(self):
        return gaussian_factors(self.base.n, self.rank, self.factor_seed)


def cube_update(n: int) -> UpdateWorkload:
    """The update workload on n uniform points in the unit cube (points seed 2):
    H built like the timed workload (exp(-r/0.2), leaf 64, eta 0.7, tol 1e-6),
    rank-64 Gaussian update."""
    base = Workload(f"exp3d_n{n}_seed2", n=n, dim=3, point_seed=2, kernel="exp", length=0.2, leaf_size=64,
                    eta=0.7, tol=1e-6, omega_seed=1001)
    return UpdateWorkload(f"update_exp3d_n{n}_r64", base=base)
