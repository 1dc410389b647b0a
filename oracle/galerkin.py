"""Legendre-Galerkin discretisation: basis, operator K = A + B, load vector.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 3: compact basis phi_k = L_k - L_{k+2}, k = 0..N-2; tensor basis with x
fastest (the unknown ordering printed for d = 2, 3); system (A + B) u = F.
Sec. 4.3: the matrix-vector product is taken with the interpolation operator
I_N on the (N+1)^d Legendre-Gauss grid, i.e. (I_N(a grad u), grad v) and
(I_N(b u), v). Since I_N g times a test function has degree <= 2N+1 per
direction this is exactly (N+1)-point Gauss quadrature of the bilinear form
(the "G-NI" operator). That operator is what the oracle calls K.

Array conventions: a coefficient vector of length (N-1)^d is reshaped to
(n1,)*d with x on the LAST axis; node arrays are (q,)*d with x last.

The diffusion coefficient is either one field a (the isotropic problem of
Sec. 3) or a list of d fields [a_1, ..., a_d] (a_1 for x), the diagonal
anisotropic form -sum_j (a_j u_{x_j})_{x_j} + b u of Example 4 (Sec. 5.2);
the bilinear form then weights the j-th gradient component by a_j.

Three independent routes to K u are given:
  dense_operator          K assembled entry by entry from node sums (tiny N)
  matvec_sumfact          one 1D table per direction applied along each axis
  matvec_legendre_route   the paper's four steps with its printed step-4
                          recombination formulas (Sec. 4.3, d = 1, 2, 3)
"""
from __future__ import annotations

import numpy as np

from . import legendre as lg


class Basis:
    """Node and table data for degree N: q = N+1 Gauss nodes x, weights w,
    Phi[m, k] = phi_k(x_m), D[m, k] = phi_k'(x_m) = -(2k+3) L_{k+1}(x_m)
    (derivative relation of Sec. 2.1, as used in the proof of the
    bandwidth proposition), P[n, m] = L_n(x_m) for n = 0..N."""

    def __init__(self, N: int):
        if N < 2:
            raise ValueError("N must be >= 2")
        self.N = N
        self.n1 = N - 1
        self.q = N + 1
        self.x, self.w = lg.gauss_legendre(N)
        self.P = lg.legendre_table(N + 1, self.x)          # L_0..L_{N+1}
        k = np.arange(self.n1)
        self.Phi = (self.P[k] - self.P[k + 2]).T            # [m, k]
        self.D = (-(2 * k + 3)[:, None] * self.P[k + 1]).T  # [m, k]
        self.PN = self.P[: N + 1]                           # L_0..L_N at nodes


def _kron_all(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def node_weights(basis: Basis, d: int) -> np.ndarray:
    """Tensor Gauss weights W[..., n_y, n_x] = prod_i w_{n_i}."""
    W = basis.w
    for _ in range(d - 1):
        W = np.multiply.outer(basis.w, W)
    return W


def a_by_direction(a_nodes, d: int):
    """[a_1, ..., a_d] (direction 0 = x): the list itself for the anisotropic
    form, d references to the one field otherwise."""
    if isinstance(a_nodes, (list, tuple)):
        assert len(a_nodes) == d
        return [np.asarray(a, dtype=np.float64) for a in a_nodes]
    return [np.asarray(a_nodes, dtype=np.float64)] * d


def dense_operator(d: int, N: int, a_nodes, b_nodes) -> np.ndarray:
    """K_ij = sum_nodes W [a grad psi_i . grad psi_j + b psi_i psi_j]  (G-NI).

    Built with Kronecker products in the ordering (..., y, x): the basis
    matrix is kron(Phi_z, Phi_y, Phi_x) and the d-th gradient component swaps
    that direction's Phi for D. For tiny N only (dense n x n)."""
    B = Basis(N)
    W = node_weights(B, d).reshape(-1)
    a_dir = [a.reshape(-1) * W for a in a_by_direction(a_nodes, d)]
    b = np.asarray(b_nodes, dtype=np.float64).reshape(-1) * W
    Psi = _kron_all([B.Phi] * d)
    K = Psi.T @ (b[:, None] * Psi)
    for i in range(d):                      # i = 0 is x = last kron factor
        mats = [B.Phi] * d
        mats[d - 1 - i] = B.D
        G = _kron_all(mats)
        K += G.T @ (a_dir[i][:, None] * G)
    return K


def matvec_sumfact(d: int, N: int, a_nodes, b_nodes, u, basis: Basis = None):
    """y = K u by sum factorisation: values and gradient of u_N at the nodes
    (BDLT composed with the basis change), pointwise W*a, W*b, then the
    transposed tables (FDLT composed with the step-4 recombination)."""
    B = basis if basis is not None else Basis(N)
    n1 = B.n1
    U = np.asarray(u, dtype=np.float64).reshape((n1,) * d)
    W = node_weights(B, d)
    wa = [W * a.reshape((B.q,) * d) for a in a_by_direction(a_nodes, d)]
    wb = W * np.asarray(b_nodes).reshape((B.q,) * d)

    def fwd(deriv_axis):
        out = U
        for ax in range(d):
            # axis ax of the array is direction d-1-ax (x is last)
            direction = d - 1 - ax
            T = B.D if direction == deriv_axis else B.Phi
            out = lg.apply_along(T, out, ax)
        return out

    def bwd(g, deriv_axis):
        out = g
        for ax in range(d):
            direction = d - 1 - ax
            T = B.D if direction == deriv_axis else B.Phi
            out = lg.apply_along(T.T, out, ax)
        return out

    y = bwd(wb * fwd(None), None)
    for i in range(d):
        y = y + bwd(wa[i] * fwd(i), i)
    return y.reshape(-1)


def matvec_sumfact_ext(d: int, N: int, a_nodes, b_nodes, u, basis: Basis = None):
    """matvec_sumfact in extended precision (numpy longdouble, 64-bit
    mantissa): the same nodes, weights and coefficient values (FP64 inputs,
    widened), the tables phi_k, phi_k' rebuilt by the recurrence in extended
    precision, the same steps. A reference for large N, where the FP64
    product itself drifts by ~N^2 * 1e-16 relative (the derivative tables
    grow like k). Slow: minutes at N = 1024 in 2D."""
    B = basis if basis is not None else Basis(N)
    LD = np.longdouble
    x = B.x.astype(LD)
    m = N + 2
    P = np.zeros((m + 1, B.q), dtype=LD)
    P[0] = 1
    P[1] = x
    for n in range(1, m):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
    k = np.arange(B.n1)
    Phi = (P[k] - P[k + 2]).T
    Dt = (-(2 * k + 3)[:, None].astype(LD) * P[k + 1]).T
    w = B.w.astype(LD)
    W = w
    for _ in range(d - 1):
        W = np.multiply.outer(w, W)
    U = np.asarray(u, dtype=np.float64).astype(LD).reshape((B.n1,) * d)
    wa = [W * a.astype(LD).reshape((B.q,) * d) for a in a_by_direction(a_nodes, d)]
    wb = W * np.asarray(b_nodes, dtype=np.float64).astype(LD).reshape((B.q,) * d)

    def along(T, arr, ax):
        return np.moveaxis(np.tensordot(T, arr, axes=(1, ax)), 0, ax)

    def fwd(deriv_axis):
        out = U
        for ax in range(d):
            out = along(Dt if d - 1 - ax == deriv_axis else Phi, out, ax)
        return out

    def bwd(g, deriv_axis):
        out = g
        for ax in range(d):
            out = along((Dt if d - 1 - ax == deriv_axis else Phi).T, out, ax)
        return out

    y = bwd(wb * fwd(None), None)
    for i in range(d):
        y = y + bwd(wa[i] * fwd(i), i)
    return y.reshape(-1).astype(np.float64)


def load_vector(d: int, N: int, f_nodes, basis: Basis = None) -> np.ndarray:
    """F_k = (I_N f, psi_k) = sum_nodes W f psi_k (reading: the same
    (N+1)-point rule as the operator; the paper leaves the rule open)."""
    B = basis if basis is not None else Basis(N)
    g = node_weights(B, d) * np.asarray(f_nodes).reshape((B.q,) * d)
    out = g
    for ax in range(d):
        out = lg.apply_along(B.Phi.T, out, ax)
    return out.reshape(-1)


# --------------------------------------------------------------------------
# The paper's four-step route (Sec. 4.3) with the printed step-4 formulas.
# --------------------------------------------------------------------------

def _phi_to_legendre(uh: np.ndarray, axis: int, N: int) -> np.ndarray:
    """Step 1 (values): sum_k u_k phi_k = sum_n u~_n L_n with
    u~_n = u_n - u_{n-2}, n = 0..N (phi_k = L_k - L_{k+2})."""
    uh = np.moveaxis(uh, axis, 0)
    out = np.zeros((N + 1,) + uh.shape[1:])
    out[: N - 1] += uh
    out[2: N + 1] -= uh
    return np.moveaxis(out, 0, axis)


def _dphi_to_legendre(uh: np.ndarray, axis: int, N: int) -> np.ndarray:
    """Step 1 (derivative), via eq. difRecerrence: sum_k u_k phi_k' =
    sum_k u_k (-(2k+3)) L_{k+1}, i.e. u~'_{k+1} = -(2k+3) u_k."""
    uh = np.moveaxis(uh, axis, 0)
    k = np.arange(N - 1).reshape((-1,) + (1,) * (uh.ndim - 1))
    out = np.zeros((N + 1,) + uh.shape[1:])
    out[1:N] = -(2 * k + 3) * uh
    return np.moveaxis(out, 0, axis)


def matvec_legendre_route(d: int, N: int, a_nodes, b_nodes, u) -> np.ndarray:
    """(A + B) u by steps 1-4 of Sec. 4.3 for d = 1, 2, 3.

    Index convention of the printed formulas: u_{k j l} multiplies
    phi_k(x) phi_j(y) phi_l(z); here arrays are stored (l, j, k) (x last), so
    the formulas below address them as arr[l, j, k]."""
    B = Basis(N)
    n1 = N - 1
    q = N + 1
    P = B.PN
    U = np.asarray(u, dtype=np.float64).reshape((n1,) * d)
    a = np.asarray(a_nodes).reshape((q,) * d)
    b = np.asarray(b_nodes).reshape((q,) * d)

    def to_nodes(c):
        return lg.tensor_bdlt(c, P)          # step 2 (BDLT)

    def coeffs(v):
        return lg.tensor_fdlt(v, P, B.w)     # step 3 (FDLT)

    # Step 1 for each field, axes ordered (..., y, x): axis of x is d-1.
    def conv(deriv_dir):
        c = U
        for ax in range(d):
            direction = d - 1 - ax
            if direction == deriv_dir:
                c = _dphi_to_legendre(c, ax, N)
            else:
                c = _phi_to_legendre(c, ax, N)
        return c

    alpha = coeffs(b * to_nodes(conv(None)))
    betas = [coeffs(a * to_nodes(conv(i))) for i in range(d)]

    if d == 1:
        j = np.arange(n1)
        bx = betas[0]
        Au = -2.0 * bx[j + 1]
        Bu = 2 * alpha[j] / (2 * j + 1) - 2 * alpha[j + 2] / (2 * j + 5)
        return Au + Bu

    if d == 2:
        # arrays are [j (y), k (x)]
        k = np.arange(n1)[None, :]
        j = np.arange(n1)[:, None]
        K_, J_ = np.arange(n1), np.arange(n1)
        bx, by = betas[0], betas[1]
        sl = np.ix_
        Au = (4.0 / (2 * j + 5) * bx[sl(J_ + 2, K_ + 1)]
              - 4.0 / (2 * j + 1) * bx[sl(J_, K_ + 1)]
              + 4.0 / (2 * k + 5) * by[sl(J_ + 1, K_ + 2)]
              - 4.0 / (2 * k + 1) * by[sl(J_ + 1, K_)])
        Bu = (4 * alpha[sl(J_, K_)] / ((2 * k + 1) * (2 * j + 1))
              - 4 * alpha[sl(J_ + 2, K_)] / ((2 * k + 1) * (2 * j + 5))
              - 4 * alpha[sl(J_, K_ + 2)] / ((2 * k + 5) * (2 * j + 1))
              + 4 * alpha[sl(J_ + 2, K_ + 2)] / ((2 * k + 5) * (2 * j + 5)))
        return (Au + Bu).reshape(-1)

    # d == 3: arrays are [l (z), j (y), k (x)]
    r = np.arange(n1)
    k = r[None, None, :]
    j = r[None, :, None]
    l = r[:, None, None]
    sl = np.ix_
    bx, by, bz = betas
    Au = (-8.0 / ((2 * j + 1) * (2 * l + 1)) * bx[sl(r, r, r + 1)]
          + 8.0 / ((2 * j + 5) * (2 * l + 1)) * bx[sl(r, r + 2, r + 1)]
          + 8.0 / ((2 * j + 1) * (2 * l + 5)) * bx[sl(r + 2, r, r + 1)]
          - 8.0 / ((2 * j + 5) * (2 * l + 5)) * bx[sl(r + 2, r + 2, r + 1)]
          - 8.0 / ((2 * k + 1) * (2 * l + 1)) * by[sl(r, r + 1, r)]
          + 8.0 / ((2 * k + 5) * (2 * l + 1)) * by[sl(r, r + 1, r + 2)]
          + 8.0 / ((2 * k + 1) * (2 * l + 5)) * by[sl(r + 2, r + 1, r)]
          - 8.0 / ((2 * k + 5) * (2 * l + 5)) * by[sl(r + 2, r + 1, r + 2)]
          - 8.0 / ((2 * k + 1) * (2 * j + 1)) * bz[sl(r + 1, r, r)]
          + 8.0 / ((2 * k + 5) * (2 * j + 1)) * bz[sl(r + 1, r, r + 2)]
          + 8.0 / ((2 * k + 1) * (2 * j + 5)) * bz[sl(r + 1, r + 2, r)]
          - 8.0 / ((2 * k + 5) * (2 * j + 5)) * bz[sl(r + 1, r + 2, r + 2)])
    Bu = (-8 * alpha[sl(r + 2, r, r)] / ((2 * k + 1) * (2 * j + 1) * (2 * l + 5))
          + 8 * alpha[sl(r, r, r)] / ((2 * k + 1) * (2 * j + 1) * (2 * l + 1))
          - 8 * alpha[sl(r, r + 2, r)] / ((2 * k + 1) * (2 * j + 5) * (2 * l + 1))
          + 8 * alpha[sl(r + 2, r + 2, r)] / ((2 * k + 1) * (2 * j + 5) * (2 * l + 5))
          - 8 * alpha[sl(r, r, r + 2)] / ((2 * k + 5) * (2 * j + 1) * (2 * l + 1))
          + 8 * alpha[sl(r, r + 2, r + 2)] / ((2 * k + 5) * (2 * j + 5) * (2 * l + 1))
          + 8 * alpha[sl(r + 2, r, r + 2)] / ((2 * k + 5) * (2 * j + 1) * (2 * l + 5))
          - 8 * alpha[sl(r + 2, r + 2, r + 2)] / ((2 * k + 5) * (2 * j + 5) * (2 * l + 5)))
    return (Au + Bu).reshape(-1)


def constant_coefficient_factors(N: int):
    """Closed forms for a constant coefficient (exact and G-NI coincide):
    S_kj = (phi_j', phi_k') = (4k+6) delta_kj and the mass matrix
    M_kk = 2/(2k+1) + 2/(2k+5), M_{k,k+2} = M_{k+2,k} = -2/(2k+5),
    from the orthogonality relation of Sec. 2.1 and phi_k' = -(2k+3)L_{k+1}."""
    n1 = N - 1
    k = np.arange(n1)
    S = np.diag(4.0 * k + 6.0)
    M = np.diag(2.0 / (2 * k + 1) + 2.0 / (2 * k + 5))
    off = -2.0 / (2 * k[:-2] + 5)
    M[k[:-2], k[:-2] + 2] = off
    M[k[:-2] + 2, k[:-2]] = off
    return S, M
