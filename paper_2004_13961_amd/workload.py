"""Nodal input data for the solver's benchmark workloads (GPU side).

Evaluates the coefficient family at the library's own Legendre-Gauss nodes
with numpy.polynomial.legendre (grid evaluation and series derivative):
    a = 2 + sum_j c_j prod_i L_{j_i}(x_i),  b = 1 + |x|^2,
    f = -a lap(u*) - grad(a).grad(u*) + b u*,  u* = prod_i sin(pi x_i) e^{x_i}.
The random coefficients c come from the shared seeded generator (synth).
Arrays are returned x fastest: numpy shape (q,)*d indexed [..., i_y, i_x].
"""
from __future__ import annotations

import numpy as np
import numpy.polynomial.legendre as npleg

import synth
from .lgpcg import gauss_legendre


def _grid_eval(c: np.ndarray, xs: np.ndarray) -> np.ndarray:
    d = c.ndim
    if d == 2:
        v = npleg.leggrid2d(xs, xs, c)          # [ix, iy]
    else:
        v = npleg.leggrid3d(xs, xs, xs, c)      # [ix, iy, iz]
    return np.ascontiguousarray(np.transpose(v, tuple(range(d - 1, -1, -1))))


def _axis_coords(xs, d):
    # X[i] has shape (q,)*d and varies with direction i (i = 0: x, the last axis)
    out = []
    for i in range(d):
        shape = [1] * d
        shape[d - 1 - i] = len(xs)
        out.append(np.broadcast_to(xs.reshape(shape), (len(xs),) * d))
    return out


def family_nodal(d: int, N: int, J: int, seed: int, with_rhs: bool = True):
    """(a, b, f, u*) at the (N+1)^d library nodes for the benchmark family."""
    xs, _ = gauss_legendre(N)
    c = synth.coefficient_draws(d, J, seed)
    a = 2.0 + _grid_eval(c, xs)
    X = _axis_coords(xs, d)
    b = 1.0 + sum(Xi * Xi for Xi in X)
    if not with_rhs:
        return a, b, None, None
    g = [np.sin(np.pi * Xi) * np.exp(Xi) for Xi in X]
    g1 = [(np.pi * np.cos(np.pi * Xi) + np.sin(np.pi * Xi)) * np.exp(Xi) for Xi in X]
    g2 = [((1 - np.pi ** 2) * np.sin(np.pi * Xi) + 2 * np.pi * np.cos(np.pi * Xi)) * np.exp(Xi) for Xi in X]
    u = np.ones((N + 1,) * d)
    for gi in g:
        u = u * gi
    lap = np.zeros_like(u)
    gdot = np.zeros_like(u)
    for i in range(d):
        other = np.ones_like(u)
        for j in range(d):
            if j != i:
                other = other * g[j]
        lap += g2[i] * other
        da = _grid_eval(npleg.legder(c, axis=i), xs)
        gdot += da * g1[i] * other
    f = -a * lap - gdot + b * u
    return a, b, f, u


def paper_example_nodal(case: str, d: int, N: int):
    """(a, b, f) at the library nodes for the variable-coefficient examples of
    the paper's iteration tables (Sec. 5.2; Examples 1, 2, 3 in 1D, 2D, 3D):
    case "a": a = (2|x|^2 + 1)^4, b = cos(sum_i x_i); case "b": a =
    exp(2 sum_i x_i), b = 0. The paper does not state f; f = 1 here."""
    xs, _ = gauss_legendre(N)
    X = _axis_coords(xs, d)
    s = sum(X)
    if case == "a":
        a = (2.0 * sum(Xi * Xi for Xi in X) + 1.0) ** 4
        b = np.cos(s)
    elif case == "b":
        a = np.exp(2.0 * s)
        b = np.zeros((N + 1,) * d)
    else:
        raise ValueError(case)
    return np.ascontiguousarray(a), np.ascontiguousarray(b), np.ones((N + 1,) * d)


def paper_example4_nodal(d: int, N: int):
    """(a_dir, b, f) at the library nodes for the anisotropic Example 4
    (Sec. 5.2): a_1 = exp(2x), a_2 = cos(y), a_3 = cos(z) (d = 3), b = 0,
    f = 1 (not stated in the paper). a_dir holds the d fields one after the
    other, each on the full grid, x fastest."""
    xs, _ = gauss_legendre(N)
    X = _axis_coords(xs, d)
    fields = [np.exp(2.0 * X[0])] + [np.cos(X[j]) for j in range(1, d)]
    a_dir = np.concatenate([np.ascontiguousarray(f).reshape(-1) for f in fields])
    return a_dir, np.zeros((N + 1,) * d), np.ones((N + 1,) * d)
