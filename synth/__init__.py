"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module only draws random numbers and lists workload parameters. It holds
none of the method's arithmetic: no Legendre polynomials, no quadrature, no
transforms. Each consumer (the oracle, or the GPU package) evaluates the
coefficient families at its own quadrature nodes with its own code.

Coefficient family (the workloads of the solver's benchmark configurations):
    a(x) = 2 + sum_{j_1..j_d <= J} c_{j_1..j_d} L_{j_1}(x_1) ... L_{j_d}(x_d)
    c_{j_1..j_d} = 0.3 * 2^-(j_1+...+j_d) * U(-1, 1)
    b(x) = 1 + x_1^2 + ... + x_d^2
    u*(x) = prod_i sin(pi x_i) exp(x_i)      (manufactured solution)
The array returned by `coefficient_draws` is indexed c[j_x, j_y(, j_z)], i.e.
axis 0 is the degree in x. Every node-space array used in this project is laid
out with x fastest: numpy shape (q,)*d indexed [..., i_y, i_x].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Config", "WORKLOADS", "coefficient_draws", "random_vector", "random_nodal",
    "serving_requests",
]


@dataclass(frozen=True)
class Config:
    """One solver workload: dimension, degree, truncation, family, tolerance."""
    name: str
    d: int
    N: int
    T: int
    J: int
    seed: int
    tol: float
    mixed: bool = False
    inner: tuple = field(default=())

    @property
    def n1(self) -> int:
        return self.N - 1

    @property
    def n(self) -> int:
        return (self.N - 1) ** self.d


WORKLOADS = {
    "2d_N32_T4": Config("2d_N32_T4", d=2, N=32, T=4, J=6, seed=0, tol=1e-10),
    "2d_N1024_T8": Config("2d_N1024_T8", d=2, N=1024, T=8, J=12, seed=1, tol=1e-10),
    "3d_N128_T6": Config("3d_N128_T6", d=3, N=128, T=6, J=6, seed=2, tol=1e-10),
    "3d_N256_T6_mixed": Config("3d_N256_T6_mixed", d=3, N=256, T=6, J=6, seed=3, tol=1e-10,
              mixed=True, inner=("bf16", "f32")),
}


def coefficient_draws(d: int, J: int, seed: int) -> np.ndarray:
    """c[j_x, j_y(, j_z)] = 0.3 * 2^-(sum j) * U(-1,1), drawn in C order."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(J + 1,) * d)
    deg = np.zeros((J + 1,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = J + 1
        deg = deg + np.arange(J + 1).reshape(shape)
    return 0.3 * np.power(2.0, -deg) * u


def random_vector(n: int, seed: int) -> np.ndarray:
    """uniform(0,1) coefficient vector of length n (matvec inputs)."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=n)


def random_nodal(d: int, q: int, seed: int, lo: float, hi: float) -> np.ndarray:
    """uniform(lo,hi) values on a q^d node grid, shape (q,)*d, x fastest."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(q,) * d)


def serving_requests(count: int = 4096, seed: int = 4):
    """The serving mix: 70% 2D with N log-uniform in [64,1024], 30% 3D with N
    log-uniform in [32,192]; T in {4,6,8}; tol in {1e-8,1e-10,1e-12}; request i
    uses coefficient seed 1000+i. Returns a list of dicts (no arrival times:
    the rate is chosen by the caller)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if rng.uniform() < 0.7:
            d = 2
            N = int(round(math.exp(rng.uniform(math.log(64), math.log(1024)))))
        else:
            d = 3
            N = int(round(math.exp(rng.uniform(math.log(32), math.log(192)))))
        T = int(rng.choice([4, 6, 8]))
        tol = float(rng.choice([1e-8, 1e-10, 1e-12]))
        out.append(dict(id=i, d=d, N=N, T=T, J=6, tol=tol, seed=1000 + i))
    return out
