"""Legendre polynomials, Gauss nodes and discrete Legendre transforms.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper Sec. 2.1: three-term recurrence, orthogonality, derivative recurrence
(eq. difRecerrence), endpoint values (eq. symproperty).
Paper Sec. 2.2: BDLT (eq. BDLT) and FDLT (eq. FDLT) at the N+1 Legendre-Gauss
nodes, the roots of L_{N+1}.
"""
from __future__ import annotations

import math

import numpy as np


def legendre_table(nmax: int, x) -> np.ndarray:
    """P[n, i] = L_n(x_i) for n = 0..nmax, by the three-term recurrence
    (n+1) L_{n+1} = (2n+1) x L_n - n L_{n-1}, L_0 = 1, L_1 = x  (Sec. 2.1)."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((nmax + 1,) + x.shape)
    P[0] = 1.0
    if nmax >= 1:
        P[1] = x
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
    return P


def legendre_deriv_table(nmax: int, x) -> np.ndarray:
    """dP[n, i] = L'_n(x_i), from the derivative recurrence of Sec. 2.1,
    (2n+1) L_n = L'_{n+1} - L'_{n-1}, with L'_0 = 0 and L'_1 = 1."""
    P = legendre_table(nmax, x)
    dP = np.zeros_like(P)
    if nmax >= 1:
        dP[1] = 1.0
    for n in range(1, nmax):
        dP[n + 1] = dP[n - 1] + (2 * n + 1) * P[n]
    return dP


def _legendre_pair(m: int, x):
    """(L_{m-1}(x), L_m(x)) by the three-term recurrence, in the dtype of x."""
    p0 = np.ones_like(x)
    p1 = x.copy()
    for k in range(1, m):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p0, p1


def gauss_legendre(N: int):
    """Nodes x_0 < ... < x_N (roots of L_{N+1}, Sec. 2.2) and weights.

    Newton's method on the recurrence from the classical initial guess
    x ~ cos(pi (i + 3/4) / (N + 3/2)) (Tricomi's asymptotic first term),
    weights w_i = 2 / ((1 - x_i^2) L'_{N+1}(x_i)^2).

    The iteration and the weight formula run in extended precision
    (numpy longdouble) and are rounded to FP64 at the end: a node off by one
    FP64 unit near an end of the interval moves its weight by about
    2 x / (1 - x^2) units, i.e. up to ~2 q^2 * 1e-16 relative (2e-10 at
    q = 1025), which the operator then carries.
    """
    m = N + 1
    i = np.arange(m)
    x = np.cos(np.pi * (i + 0.75) / (m + 0.5)).astype(np.longdouble)
    eps = np.finfo(np.longdouble).eps
    for _ in range(100):
        pm1, pm = _legendre_pair(m, x)
        # L'_m from (1 - x^2) L'_m = m (L_{m-1} - x L_m)
        dp = m * (pm1 - x * pm) / (1 - x * x)
        dx = pm / dp
        x = x - dx
        if np.max(np.abs(dx)) < 4 * eps:
            break
    pm1, pm = _legendre_pair(m, x)
    dp = m * (pm1 - x * pm) / (1 - x * x)
    w = 2 / ((1 - x * x) * dp * dp)
    order = np.argsort(x)
    return x[order].astype(np.float64), w[order].astype(np.float64)


def bdlt(c: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Backward DLT (eq. BDLT): f_k = sum_n c_n L_n(x_k); P[n, k] = L_n(x_k).
    Applied along axis 0 of c."""
    return np.tensordot(P.T, c, axes=(1, 0))


def fdlt(f: np.ndarray, P: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Forward DLT (eq. FDLT): c_n = (2n+1)/2 sum_k w_k f_k L_n(x_k).
    Applied along axis 0 of f."""
    n = np.arange(P.shape[0])
    s = (2 * n + 1) / 2.0
    c = np.tensordot(P * w[None, :], f, axes=(1, 0))
    return c * s.reshape((-1,) + (1,) * (f.ndim - 1))


def apply_along(mat: np.ndarray, arr: np.ndarray, axis: int) -> np.ndarray:
    """out[..., i, ...] = sum_k mat[i, k] arr[..., k, ...] along `axis`."""
    out = np.tensordot(mat, arr, axes=(1, axis))
    return np.moveaxis(out, 0, axis)


def tensor_fdlt(f: np.ndarray, P: np.ndarray, w: np.ndarray) -> np.ndarray:
    """d-dimensional FDLT of node values f (x fastest: last axis is x).
    Result c[..., n_y, n_x] with the same axis order."""
    n = np.arange(P.shape[0])
    F = (P * w[None, :]) * ((2 * n + 1) / 2.0)[:, None]
    out = f
    for ax in range(f.ndim):
        out = apply_along(F, out, ax)
    return out


def tensor_bdlt(c: np.ndarray, P: np.ndarray) -> np.ndarray:
    """d-dimensional BDLT of Legendre coefficients (same axis convention)."""
    out = c
    for ax in range(c.ndim):
        out = apply_along(P.T, out, ax)
    return out


def legendre_series_eval(coef: np.ndarray, xs) -> np.ndarray:
    """Evaluate sum c[j_x, j_y, ...] L_{j_x}(x) L_{j_y}(y) ... on the tensor
    grid xs (one 1D node array per direction); result laid out x fastest,
    i.e. shape (len(xs[d-1]), ..., len(xs[0]))."""
    d = coef.ndim
    out = coef
    # contract degree axis 0 (x) ... ; build result with axes reversed
    for ax in range(d):
        P = legendre_table(coef.shape[ax] - 1, xs[ax])  # [deg, node]
        out = np.tensordot(out, P, axes=([0], [0]))      # consumes leading axis, appends node axis
    # now axes are (x_node, y_node, ...) -> reverse to (..., y, x)
    return np.transpose(out, tuple(range(d - 1, -1, -1)))


def legendre_series_grad_eval(coef: np.ndarray, xs, direction: int) -> np.ndarray:
    """Partial derivative along `direction` (0 = x) of the series above,
    using L'_n from the derivative recurrence."""
    d = coef.ndim
    out = coef
    for ax in range(d):
        if ax == direction:
            P = legendre_deriv_table(coef.shape[ax] - 1, xs[ax])
        else:
            P = legendre_table(coef.shape[ax] - 1, xs[ax])
        out = np.tensordot(out, P, axes=([0], [0]))
    return np.transpose(out, tuple(range(d - 1, -1, -1)))


def gauss_points_needed(deg: int) -> int:
    """Number of Gauss points that integrate degree `deg` exactly."""
    return int(math.ceil((deg + 1) / 2.0))
