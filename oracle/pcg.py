"""PCG (Alg. 1) and unpreconditioned CG.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The textbook preconditioned conjugate gradient method for a symmetric
positive definite K with preconditioner M (Alg. 1 of the paper): the search
direction is the preconditioned residual made K-conjugate to the previous
direction, and the iteration stops once the recursive residual's 2-norm
falls to eps times that of F, or after k_max iterations.
Readings: x_0 = 0 unless given; k_max defaults to 2000; the test is on the
recursive residual r.
"""
from __future__ import annotations

import numpy as np


def pcg(matvec, precond, F, eps, kmax=2000, x0=None):
    F = np.asarray(F, dtype=np.float64)
    x = np.zeros_like(F) if x0 is None else np.array(x0, dtype=np.float64)
    r = F - matvec(x)
    normF = np.sqrt(F @ F)
    k = 0
    rho = 0.0
    p = None
    hist = [np.sqrt(r @ r) / normF]
    while np.sqrt(r @ r) > eps * normF and k < kmax:
        z = precond(r)
        k += 1
        if k == 1:
            p = z.copy()
            rho = r @ z
        else:
            rho_old = rho
            rho = r @ z
            beta = rho / rho_old
            p = z + beta * p
        w = matvec(p)
        alpha = rho / (p @ w)
        x = x + alpha * p
        r = r - alpha * w
        hist.append(np.sqrt(r @ r) / normF)
    return x, k, hist


def cg(matvec, F, eps, kmax=2000, x0=None):
    """Alg. 1 with M = I (z = r)."""
    return pcg(matvec, lambda r: r.copy(), F, eps, kmax, x0)
