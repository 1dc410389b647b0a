"""The benchmark coefficient family and manufactured data at the oracle's nodes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

a(x) = 2 + sum_j c_j prod_i L_{j_i}(x_i), b(x) = 1 + sum_i x_i^2, and the
right-hand side f = -div(a grad u*) + b u* of the manufactured solution
u*(x) = prod_i g(x_i), g(s) = sin(pi s) e^s:
    g'  = (pi cos(pi s) + sin(pi s)) e^s
    g'' = ((1 - pi^2) sin(pi s) + 2 pi cos(pi s)) e^s
    f   = -a lap(u*) - grad(a).grad(u*) + b u*,
with grad(a) from the derivative recurrence of Sec. 2.1.
Arrays are laid out x fastest (last axis).
"""
from __future__ import annotations

import numpy as np

from . import legendre as lg


def _grid(xs, d):
    # returns list of coordinate arrays X[i] with shape (q,)*d, X[0] = x (last axis)
    mesh = np.meshgrid(*([xs] * d), indexing="ij")   # mesh[k] varies along axis k
    return [mesh[d - 1 - i] for i in range(d)]


def coefficient_a(c: np.ndarray, xs) -> np.ndarray:
    return 2.0 + lg.legendre_series_eval(c, [xs] * c.ndim)


def coefficient_b(d: int, xs) -> np.ndarray:
    X = _grid(xs, d)
    return 1.0 + sum(Xi ** 2 for Xi in X)


def g(s):
    return np.sin(np.pi * s) * np.exp(s)


def dg(s):
    return (np.pi * np.cos(np.pi * s) + np.sin(np.pi * s)) * np.exp(s)


def d2g(s):
    return ((1 - np.pi ** 2) * np.sin(np.pi * s) + 2 * np.pi * np.cos(np.pi * s)) * np.exp(s)


def u_star(d: int, xs) -> np.ndarray:
    X = _grid(xs, d)
    out = np.ones_like(X[0])
    for Xi in X:
        out = out * g(Xi)
    return out


def rhs_f(c: np.ndarray, xs) -> np.ndarray:
    d = c.ndim
    X = _grid(xs, d)
    a = coefficient_a(c, xs)
    b = coefficient_b(d, xs)
    G = [g(Xi) for Xi in X]
    u = np.ones_like(X[0])
    for Gi in G:
        u = u * Gi
    lap = np.zeros_like(u)
    grad_dot = np.zeros_like(u)
    for i in range(d):
        other = np.ones_like(u)
        for j in range(d):
            if j != i:
                other = other * G[j]
        lap += d2g(X[i]) * other
        du_i = dg(X[i]) * other
        da_i = lg.legendre_series_grad_eval(c, [xs] * d, i)
        grad_dot += da_i * du_i
    return -a * lap - grad_dot + b * u


def paper_example(case: str, d: int, xs):
    """(a, b) of the paper's variable-coefficient examples (Sec. 5.2):
    Example 1 (d = 1), 2 (d = 2) and 3 (d = 3); case "a": a = (2|x|^2 + 1)^4,
    b = cos(sum_i x_i); case "b": a = exp(2 sum_i x_i), b = 0."""
    X = _grid(xs, d)
    s = sum(X)
    if case == "a":
        a = (2.0 * sum(Xi ** 2 for Xi in X) + 1.0) ** 4
        b = np.cos(s)
    elif case == "b":
        a = np.exp(2.0 * s)
        b = np.zeros_like(s)
    else:
        raise ValueError(case)
    return a, b


def example4(d: int, xs):
    """(a_dir, b) of the anisotropic Example 4 (Sec. 5.2): a_1 = exp(2x),
    a_2 = cos(y), a_3 = cos(z) (d = 3), b = 0; each field on the full grid."""
    X = _grid(xs, d)
    a_dir = [np.exp(2.0 * X[0])] + [np.cos(X[j]) for j in range(1, d)]
    return a_dir, np.zeros_like(X[0])
