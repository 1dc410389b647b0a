"""Preconditioner M built from truncated Legendre series of the coefficients.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Sec. 4.1: a and b are replaced by Legendre series p_T with indices <= T in
each direction (eqs. 1DM/2DM/3DM). Sec. 4.2 writes M in 2D as a sum of
Kronecker products of 1D factors
    S^(t)_{im} = (L_t phi_i', phi_m'),   M^(t)_{im} = (L_t phi_i, phi_m),
weighted by the series coefficients; the same form is used for 3D and for the
b part. The integrals are exact (Lemma LegProduct, Sec. 2.1).

Readings of the paper used here (where it is silent):
  * the truncated coefficients are the discrete Legendre coefficients (FDLT)
    of the nodal coefficient values on the problem's (N+1)^d grid, kept for
    indices <= T in every direction (a tensor box);
  * NZ(M) is the union of the structural supports of the Kronecker terms
    whose series coefficient is not negligible (|c| > 1e-13 * max|c|):
    per direction S^(t) reaches |delta| <= t and M^(t) reaches |delta| <= t+2.
    Entries inside that union are kept even when they happen to be zero.

The anisotropic form of Example 4 (Sec. 5.2) has one diffusion field per
direction: there `ahat` is a list [a_1 series, ..., a_d series], each with
its own truncation t_{1j}, and the term with S^(t) in direction j carries
the series of a_j. A single array means the same series in every direction.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np

from . import legendre as lg
from .galerkin import Basis

NEGLIGIBLE = 1e-13


# ---------------------------------------------------------------- p_T ------
def truncated_coefficients(nodal: np.ndarray, basis: Basis, T: int) -> np.ndarray:
    """Legendre coefficients of the nodal field (FDLT on the grid), indices
    <= T per direction. Axis order as the nodes (x last)."""
    c = lg.tensor_fdlt(np.asarray(nodal, dtype=np.float64), basis.PN, basis.w)
    sl = tuple(slice(0, T + 1) for _ in range(c.ndim))
    return c[sl].copy()


def _a_list(ahat, d: int):
    return list(ahat) if isinstance(ahat, (list, tuple)) else [ahat] * d


def series_dir(a_dir, b_nodes, basis: Basis, Ta_dir, Tb: int):
    """Anisotropic form: ([a_1 series <= Ta_dir[0]], ..., b series <= Tb),
    with the same negligible-term rule as series_pair over all d+1 series."""
    ahs = [truncated_coefficients(a, basis, t) for a, t in zip(a_dir, Ta_dir)]
    bh = truncated_coefficients(b_nodes, basis, Tb)
    mx = max(max(np.max(np.abs(ah)) for ah in ahs), np.max(np.abs(bh)))
    for ah in ahs:
        ah[np.abs(ah) <= NEGLIGIBLE * mx] = 0.0
    bh[np.abs(bh) <= NEGLIGIBLE * mx] = 0.0
    return ahs, bh


def series_pair(a_nodes, b_nodes, basis: Basis, Ta: int, Tb: int):
    """(a_T, b_T): truncated coefficients of a (indices <= Ta) and b (<= Tb),
    with every coefficient of magnitude <= 1e-13 * (largest magnitude over
    both series) set to zero (reading: such terms are rounding residue of
    the transform, e.g. of a polynomial b, and are not part of p_T)."""
    ah = truncated_coefficients(a_nodes, basis, Ta)
    bh = truncated_coefficients(b_nodes, basis, Tb)
    mx = max(np.max(np.abs(ah)), np.max(np.abs(bh)))
    ah[np.abs(ah) <= NEGLIGIBLE * mx] = 0.0
    bh[np.abs(bh) <= NEGLIGIBLE * mx] = 0.0
    return ah, bh


# ------------------------------------------------ triple products ----------
@lru_cache(maxsize=None)
def _logC(r: int) -> float:
    """log C_r, C_r = 1*3*...*(2r-1) / (r! 2^r) (Lemma LegProduct)."""
    return math.fsum(math.log1p(-1.0 / (2 * i)) for i in range(1, r + 1))


def triple(t: int, m: int, n: int) -> float:
    """int_{-1}^{1} L_t L_m L_n dx from the product formula (Lemma LegProduct):
    L_m L_n = sum_s (m+n+1/2-2s)/(m+n+1/2-s) C_s C_{m-s} C_{n-s}/C_{m+n-s}
    L_{m+n-2s}, then orthogonality picks the term with m+n-2s = t, times
    2/(2t+1)."""
    if t < 0 or m < 0 or n < 0:
        return 0.0
    if (t + m + n) % 2 or t > m + n or t < abs(m - n):
        return 0.0
    s = (m + n - t) // 2
    ratio = (m + n + 0.5 - 2 * s) / (m + n + 0.5 - s)
    logc = _logC(s) + _logC(m - s) + _logC(n - s) - _logC(m + n - s)
    return ratio * math.exp(logc) * 2.0 / (2 * t + 1)


def triple_exact(t: int, m: int, n: int) -> Fraction:
    """The same integral in exact rational arithmetic (for pins)."""
    if (t + m + n) % 2 or t > m + n or t < abs(m - n) or min(t, m, n) < 0:
        return Fraction(0)

    def C(r):
        num = 1
        for i in range(1, r + 1):
            num *= 2 * i - 1
        return Fraction(num, math.factorial(r) * 2 ** r)

    s = (m + n - t) // 2
    ratio = Fraction(2 * (m + n) + 1 - 4 * s, 2 * (m + n) + 1 - 2 * s)
    return ratio * C(s) * C(m - s) * C(n - s) / C(m + n - s) * Fraction(2, 2 * t + 1)


def triple_quadrature(t: int, m: int, n: int) -> float:
    """The same integral by an over-integrating Gauss rule (cross-check)."""
    npts = lg.gauss_points_needed(t + m + n) + 1
    x, w = lg.gauss_legendre(npts - 1)
    P = lg.legendre_table(max(t, m, n), x)
    return float(np.sum(w * P[t] * P[m] * P[n]))


def S_entry(t: int, i: int, m: int) -> float:
    """S^(t)_{im} = (L_t phi_i', phi_m') = (2i+3)(2m+3) int L_t L_{i+1} L_{m+1}."""
    return (2 * i + 3) * (2 * m + 3) * triple(t, i + 1, m + 1)


def M_entry(t: int, i: int, m: int) -> float:
    """M^(t)_{im} = (L_t (L_i - L_{i+2}), L_m - L_{m+2})."""
    return (triple(t, i, m) - triple(t, i, m + 2)
            - triple(t, i + 2, m) + triple(t, i + 2, m + 2))


def band_factors(n1: int, T: int):
    """Dense 1D factors S[t], Mm[t] (n1 x n1) for t = 0..T. Only entries with
    |i - m| <= t + 2 can be nonzero (bandwidth proposition), so only those
    are evaluated."""
    S = np.zeros((T + 1, n1, n1))
    Mm = np.zeros((T + 1, n1, n1))
    for t in range(T + 1):
        for i in range(n1):
            for m in range(max(0, i - t - 2), min(n1, i + t + 3)):
                S[t, i, m] = S_entry(t, i, m)
                Mm[t, i, m] = M_entry(t, i, m)
    return S, Mm


# ---------------------------------------------------------- pattern --------
def _support(c: np.ndarray):
    if c is None or c.size == 0:
        return []
    return [idx for idx in np.ndindex(*c.shape) if c[idx] != 0.0]


def stencil_offsets(ahat: np.ndarray, bhat: np.ndarray):
    """NZ(M) as a set of offsets (dx, dy[, dz]) (reading: structural union).

    ahat/bhat (from series_pair, negligible terms already zero) are
    indexed [..., t_y, t_x] (x last); the diagonal is always included. For an a-term with
    degrees (t_x, t_y, ...) the direction carrying S^(t) reaches |d| <= t and
    the others (carrying M^(t)) reach |d| <= t+2; a b-term reaches t+2 in all
    directions. Returned sorted in column order (lexicographic on
    (dz, dy, dx)), which equals column order for every in-grid pair."""
    d = bhat.ndim if bhat is not None else _a_list(ahat, 1)[0].ndim
    a_dir = _a_list(ahat, d)
    offs = set([tuple([0] * d)])

    def add_box(reach):
        rng = [range(-r, r + 1) for r in reach]
        for pt in np.ndindex(*[len(r) for r in rng]):
            offs.add(tuple(rng[k][pt[k]] for k in range(d)))

    for s_dir in range(d):                 # the direction carrying S^(t)
        for idx in _support(a_dir[s_dir]):
            deg = idx[::-1]                # (t_x, t_y, ...)
            reach = [deg[k] + 2 for k in range(d)]
            reach[s_dir] = deg[s_dir]
            add_box(reach)
    if bhat is not None:
        for idx in _support(bhat):
            deg = idx[::-1]
            add_box([deg[k] + 2 for k in range(d)])
    return sorted(offs, key=lambda o: tuple(reversed(o)))


# --------------------------------------------------------- assembly --------
def _kron_all(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


def dense_M(d: int, n1: int, ahat: np.ndarray, bhat: np.ndarray) -> np.ndarray:
    """M = sum_t a_t [sum over directions of (S^(t_dir) in that direction,
    M^(t) in the others)] + sum_t b_t (M^(t) in all directions), as the
    Kronecker sum of Sec. 4.2 (kron order z, y, x). Dense; tiny n only."""
    a_dir = _a_list(ahat, d)
    T = max(max(ah.shape[0] for ah in a_dir), bhat.shape[0] if bhat is not None else 0) - 1
    S, Mm = band_factors(n1, T)
    n = n1 ** d
    M = np.zeros((n, n))
    for s_pos in range(d):
        # kron position s_pos (order z, y, x) is direction d-1-s_pos
        ah = a_dir[d - 1 - s_pos]
        for idx in np.ndindex(*ah.shape):
            c = ah[idx]
            if c == 0.0:
                continue
            # idx = (t_z, t_y, t_x) ~ kron factor order
            mats = [S[idx[k]] if k == s_pos else Mm[idx[k]] for k in range(d)]
            M += c * _kron_all(mats)
    if bhat is not None:
        for idx in np.ndindex(*bhat.shape):
            c = bhat[idx]
            if c == 0.0:
                continue
            M += c * _kron_all([Mm[idx[k]] for k in range(d)])
    return M


def M_row_entries(d: int, n1: int, ahat, bhat, row_idx, offsets,
                  S=None, Mm=None, return_abs: bool = False):
    """Entries M(row, row+delta) for the listed offsets (0 outside the grid),
    computed term by term from the 1D factors (for sampled-row checks).
    With return_abs, also the sums of the magnitudes of the terms and of the
    1D factor products alone (the scales of the rounding in any evaluation
    of the entry, and of its sensitivity to the series coefficients)."""
    T = max(ahat.shape[0], bhat.shape[0]) - 1
    if S is None:
        S, Mm = band_factors(n1, T)
    # row coordinates (ix, iy, iz)
    coords = []
    r = row_idx
    for _ in range(d):
        coords.append(r % n1)
        r //= n1
    out = np.zeros(len(offsets))
    mag = np.zeros(len(offsets))
    pmag = np.zeros(len(offsets))
    for oi, off in enumerate(offsets):
        col = [coords[k] + off[k] for k in range(d)]
        if any(c < 0 or c >= n1 for c in col):
            continue
        val = 0.0
        for idx in np.ndindex(*ahat.shape):
            deg = idx[::-1]           # (t_x, t_y, ...)
            for s_dir in range(d):
                prod = ahat[idx]
                for k in range(d):
                    F = S if k == s_dir else Mm
                    prod *= F[deg[k], coords[k], col[k]]
                val += prod
                mag[oi] += abs(prod)
                if ahat[idx] != 0.0:
                    pmag[oi] += abs(prod / ahat[idx])
        for idx in np.ndindex(*bhat.shape):
            deg = idx[::-1]
            prod = bhat[idx]
            for k in range(d):
                prod *= Mm[deg[k], coords[k], col[k]]
            val += prod
            mag[oi] += abs(prod)
            if bhat[idx] != 0.0:
                pmag[oi] += abs(prod / bhat[idx])
        out[oi] = val
    return (out, mag, pmag) if return_abs else out


def M_rows_entries(d: int, n1: int, ahat, bhat, rows, offsets, S=None, Mm=None):
    """M_row_entries for many rows at once: the same term-by-term sums of
    Kronecker products of the 1D factors (Sec. 4.2), each term evaluated for
    all (row, offset) pairs as one array. Returns (entries, magnitudes,
    factor magnitudes), each of shape (len(rows), len(offsets))."""
    T = max(ahat.shape[0], bhat.shape[0]) - 1
    if S is None:
        S, Mm = band_factors(n1, T)
    rows = np.asarray(rows, dtype=np.int64)
    offs = np.asarray(offsets, dtype=np.int64).reshape(len(offsets), -1)[:, :d]
    coords = np.stack([(rows // n1 ** k) % n1 for k in range(d)], axis=1)      # (R, d)
    col = coords[:, None, :] + offs[None, :, :]                                   # (R, K, d)
    inside = np.all((col >= 0) & (col < n1), axis=2)
    colc = np.clip(col, 0, n1 - 1)
    out = np.zeros(inside.shape)
    mag = np.zeros(inside.shape)
    pmag = np.zeros(inside.shape)

    def factor(F, t, k):
        return F[t, coords[:, k][:, None], colc[:, :, k]]

    def add(c, mats):
        prod = np.ones(inside.shape)
        for m in mats:
            prod = prod * m
        out[...] += c * prod
        mag[...] += np.abs(c * prod)
        if c != 0.0:
            pmag[...] += np.abs(prod)

    for idx in np.ndindex(*ahat.shape):
        c = ahat[idx]
        if c == 0.0:
            continue
        deg = idx[::-1]
        for s_dir in range(d):
            add(c, [factor(S if k == s_dir else Mm, deg[k], k) for k in range(d)])
    for idx in np.ndindex(*bhat.shape):
        c = bhat[idx]
        if c == 0.0:
            continue
        deg = idx[::-1]
        add(c, [factor(Mm, deg[k], k) for k in range(d)])
    out[~inside] = 0.0
    mag[~inside] = 0.0
    pmag[~inside] = 0.0
    return out, mag, pmag


def pattern_mask(d: int, n1: int, offsets) -> np.ndarray:
    """Dense boolean NZ pattern for tiny n from the offset set."""
    n = n1 ** d
    mask = np.zeros((n, n), dtype=bool)
    for row in range(n):
        coords = []
        r = row
        for _ in range(d):
            coords.append(r % n1)
            r //= n1
        for off in offsets:
            col = [coords[k] + off[k] for k in range(d)]
            if any(c < 0 or c >= n1 for c in col):
                continue
            ci = 0
            for k in reversed(range(d)):
                ci = ci * n1 + col[k]
            mask[row, ci] = True
    return mask


def _diag_of(F: np.ndarray, delta: int) -> np.ndarray:
    """v[i] = F[i, i + delta] (0 where i + delta leaves 0..n1-1)."""
    n1 = F.shape[0]
    v = np.zeros(n1)
    lo, hi = max(0, -delta), min(n1, n1 - delta)
    idx = np.arange(lo, hi)
    v[idx] = F[idx, idx + delta]
    return v


def stencil_rows(d: int, n1: int, ahat: np.ndarray, bhat: np.ndarray, offsets,
                 S=None, Mm=None, nplanes: int = None) -> np.ndarray:
    """H[row, o] = M(row, row + offsets[o]) for every row, from the Kronecker
    form (each term separable, so each offset is a tensor product of 1D
    diagonals contracted with the coefficient array). d = 1, 2, 3. For d = 3,
    `nplanes` keeps the rows of the first nplanes z-planes only (a prefix of
    the rows, for timing a bounded sample)."""
    a_dir = _a_list(ahat, d)
    Tb = bhat.shape[0] - 1
    T = max(max(ah.shape[0] - 1 for ah in a_dir), Tb)
    if S is None:
        S, Mm = band_factors(n1, T)
    nz = n1 if (d != 3 or nplanes is None) else min(nplanes, n1)
    n = n1 ** (d - 1) * nz if d == 3 else n1 ** d
    H = np.zeros((n, len(offsets)))
    Ad = []                                # per direction, padded to T
    for ah in a_dir:
        A = np.zeros((T + 1,) * d)
        A[tuple(slice(0, ah.shape[0]) for _ in range(d))] = ah
        Ad.append(A)
    Bc = np.zeros((T + 1,) * d)
    Bc[tuple(slice(0, Tb + 1) for _ in range(d))] = bhat
    for o, off in enumerate(offsets):
        Sd = [np.stack([_diag_of(S[t], off[k]) for t in range(T + 1)]) for k in range(d)]
        Md = [np.stack([_diag_of(Mm[t], off[k]) for t in range(T + 1)]) for k in range(d)]
        if d == 3:
            Sd[2], Md[2] = Sd[2][:, :nz], Md[2][:, :nz]
        def term(C, Fz, Fy, Fx):
            # sum_{r,s,t} C[r,s,t] Fz[r,z] Fy[s,y] Fx[t,x], one direction at a time
            if d == 2:
                tmp = np.tensordot(C, Fy, axes=(0, 0))          # [t, y]
                return np.tensordot(tmp, Fx, axes=(0, 0))        # [y, x]
            tmp = np.tensordot(C, Fz, axes=(0, 0))               # [s, t, z]
            tmp = np.tensordot(tmp, Fy, axes=(0, 0))             # [t, z, y]
            return np.tensordot(tmp, Fx, axes=(0, 0))            # [z, y, x]

        if d == 1:
            # sum_t a_t S^(t) + b_t M^(t) along the one direction
            val = np.tensordot(Ad[0], Sd[0], axes=(0, 0)) + np.tensordot(Bc, Md[0], axes=(0, 0))
        elif d == 2:
            # coefficient index [s (y), t (x)]; S in x carries a_1, S in y a_2
            val = (term(Ad[0], None, Md[1], Sd[0]) + term(Ad[1], None, Sd[1], Md[0])
                   + term(Bc, None, Md[1], Md[0]))
        else:
            val = (term(Ad[0], Md[2], Md[1], Sd[0]) + term(Ad[1], Md[2], Sd[1], Md[0])
                   + term(Ad[2], Sd[2], Md[1], Md[0]) + term(Bc, Md[2], Md[1], Md[0]))
        H[:, o] = val.reshape(-1)
    return H


# --------------------------------------------------------------- PCG-I -----
def constant_coefficients(a_nodes, b_nodes, basis: Basis):
    """(c_a, c_b): the series of a and b truncated at T = 0 (Sec. 4.1), the
    preconditioner of the comparison method PCG-I (Sec. 5.2)."""
    if isinstance(a_nodes, (list, tuple)):
        # anisotropic form: one constant per direction
        ahs, bh = series_dir(a_nodes, b_nodes, basis, [0] * len(a_nodes), 0)
        return [float(ah.reshape(-1)[0]) for ah in ahs], float(bh.reshape(-1)[0])
    ah, bh = series_pair(a_nodes, b_nodes, basis, 0, 0)
    return float(ah.reshape(-1)[0]), float(bh.reshape(-1)[0])


def constant_operator_dense(d: int, N: int, ca: float, cb: float) -> np.ndarray:
    """K0 = c_a sum_dir (S in that direction, M elsewhere) + c_b (M x ... x M)
    from the closed-form 1D stiffness and mass of the compact basis."""
    from .galerkin import constant_coefficient_factors
    S1, M1 = constant_coefficient_factors(N)
    cs = _a_list(ca, d)
    K = cb * _kron_all([M1] * d)
    for i in range(d):
        mats = [M1] * d
        mats[i] = S1                       # kron position i = direction d-1-i
        K = K + cs[d - 1 - i] * _kron_all(mats)
    return K


def constant_solve(d: int, N: int, ca: float, cb: float, r) -> np.ndarray:
    """z = K0^{-1} r through the generalized eigenvectors of (M, S) in 1D
    (scipy's symmetric-definite eigensolver): E^T S E = I, E^T M E = diag(lam),
    so K0 is diagonal in the tensor basis E x ... x E."""
    import scipy.linalg as sla
    from .galerkin import constant_coefficient_factors
    S1, M1 = constant_coefficient_factors(N)
    lam, E = sla.eigh(M1, S1)
    n1 = N - 1
    R = np.asarray(r, dtype=np.float64).reshape((n1,) * d)
    V = R
    for ax in range(d):
        V = lg.apply_along(E.T, V, ax)
    grids = np.meshgrid(*([lam] * d), indexing="ij")
    prod = np.ones_like(grids[0])
    for g in grids:
        prod = prod * g
    cs = _a_list(ca, d)
    den = cb * prod
    for i in range(d):                     # S along axis i = direction d-1-i
        term = np.ones_like(grids[0])
        for k in range(d):
            if k != i:
                term = term * grids[k]
        den = den + cs[d - 1 - i] * term
    V = V / den
    for ax in range(d):
        V = lg.apply_along(E, V, ax)
    return V.reshape(-1)


def constant_apply(d: int, N: int, ca: float, cb: float, z) -> np.ndarray:
    """K0 z from the 1D factors (one direction at a time)."""
    from .galerkin import constant_coefficient_factors
    S1, M1 = constant_coefficient_factors(N)
    n1 = N - 1
    Z = np.asarray(z, dtype=np.float64).reshape((n1,) * d)

    def chain(mats):
        out = Z
        for ax in range(d):
            out = lg.apply_along(mats[ax], out, ax)
        return out

    cs = _a_list(ca, d)
    y = cb * chain([M1] * d)
    for i in range(d):
        mats = [M1] * d
        mats[i] = S1                       # axis i = direction d-1-i
        y = y + cs[d - 1 - i] * chain(mats)
    return y.reshape(-1)
