"""Pins for the preconditioner (Sec. 4.1-4.2) and ILU(0) (Alg. 2-4).

Independent references: numpy's Legendre product (legmul) and over-integrated
Gauss quadrature for the triple products of Lemma LegProduct; the bandwidth
proposition; the ILU(0) defining property (LU)_ij = m_ij on NZ(M); exact LU
when the pattern is full; the symmetric identity U = diag(U) L^T."""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import synth
from oracle import galerkin as gk
from oracle import ilu
from oracle import pcg as opcg
from oracle import precond as pc
from oracle import workload as wl


@pytest.mark.parametrize("t,m,n", [(0, 0, 0), (2, 1, 3), (3, 4, 5), (6, 10, 12),
                                   (8, 300, 305), (5, 1000, 1003), (7, 40, 33)])
def test_triple_product_vs_numpy_legmul(t, m, n):
    cm = np.zeros(m + 1)
    cm[m] = 1
    cn = np.zeros(n + 1)
    cn[n] = 1
    prod = npleg.legmul(cm, cn)
    ref = prod[t] * 2.0 / (2 * t + 1) if t < len(prod) else 0.0
    got = pc.triple(t, m, n)
    assert abs(got - ref) <= 1e-13 * max(abs(ref), 1e-300) + 1e-300
    if m + n < 60:
        assert abs(float(pc.triple_exact(t, m, n)) - got) <= 1e-14 * max(abs(got), 1e-300)
        assert abs(pc.triple_quadrature(t, m, n) - got) <= 1e-13


def test_bandwidth_proposition_1d():
    """Bandwidths of M_1 = sum beta_t S^(t) and M_2 = sum alpha_t M^(t) for
    even/odd coefficient series (Proposition, with t_2 in the odd-alpha case)."""
    n1 = 30
    rng = np.random.default_rng(0)
    S, Mm = pc.band_factors(n1, 7)

    def bw(A):
        i, j = np.nonzero(np.abs(A) > 1e-14 * np.max(np.abs(A)))
        return 2 * np.max(np.abs(i - j)) + 1

    for t1 in range(2, 8):
        for parity in (0, 1):          # 0: even function, 1: odd function
            ts = [t for t in range(t1 + 1) if t % 2 == parity]
            M1 = sum(rng.uniform(0.5, 1) * S[t] for t in ts)
            M2 = sum(rng.uniform(0.5, 1) * Mm[t] for t in ts)
            even_t = (t1 % 2 == 0)
            if parity == 1:   # odd
                q1 = 2 * t1 - 1 if even_t else 2 * t1 + 1
                q2 = 2 * t1 + 3 if even_t else 2 * t1 + 5
            else:
                q1 = 2 * t1 + 1 if even_t else 2 * t1 - 1
                q2 = 2 * t1 + 5 if even_t else 2 * t1 + 3
            assert bw(M1) == q1
            assert bw(M2) == q2


def _config_problem(d, N, T, J=6, seed=0):
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, J, seed)
    a = wl.coefficient_a(c, B.x)
    b = wl.coefficient_b(d, B.x)
    ah, bh = pc.series_pair(a, b, B, T, T)
    return B, a, b, ah, bh


@pytest.mark.parametrize("d,N,T", [(1, 30, 4), (1, 12, 8), (2, 12, 4), (2, 20, 8), (3, 6, 2)])
def test_M_spd_symmetric_and_pattern(d, N, T):
    B, a, b, ah, bh = _config_problem(d, N, T)
    M = pc.dense_M(d, N - 1, ah, bh)
    assert np.max(np.abs(M - M.T)) < 1e-13 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(M).min() > 0
    offs = pc.stencil_offsets(ah, bh)
    mask = pc.pattern_mask(d, N - 1, offs)
    assert np.array_equal(mask, M != 0.0)
    # separable stencil assembly agrees with the dense Kronecker form
    H = pc.stencil_rows(d, N - 1, ah, bh, offs)
    H2 = ilu.stencil_rows_from_dense(M, d, N - 1, offs)
    assert np.max(np.abs(H - H2)) < 1e-13 * np.max(np.abs(M))


@pytest.mark.parametrize("d,N,T", [(2, 12, 4), (3, 6, 2)])
def test_M_row_entries_match_dense(d, N, T):
    """The term-by-term row entries (used by the full-size sampled checks)
    equal the dense Kronecker-form M, out-of-grid columns included as 0."""
    B, a, b, ah, bh = _config_problem(d, N, T)
    M = pc.dense_M(d, N - 1, ah, bh)
    offs = pc.stencil_offsets(ah, bh)
    H2 = ilu.stencil_rows_from_dense(M, d, N - 1, offs)
    n = (N - 1) ** d
    for row in (0, n // 3, n // 2 + 1, n - 1):
        e = pc.M_row_entries(d, N - 1, ah, bh, row, offs)
        assert np.max(np.abs(e - H2[row])) < 1e-13 * np.max(np.abs(M))


@pytest.mark.parametrize("d,N", [(2, 9), (2, 14), (3, 6)])
def test_constant_preconditioner(d, N):
    """PCG-I's preconditioner (Sec. 5.2): the closed-form Kronecker K0 equals
    the assembled operator for constant coefficients, and the
    diagonalisation solve equals a dense solve."""
    ca, cb = 1.7, 0.4
    q = N + 1
    K0 = pc.constant_operator_dense(d, N, ca, cb)
    Kd = gk.dense_operator(d, N, np.full((q,) * d, ca), np.full((q,) * d, cb))
    assert np.max(np.abs(K0 - Kd)) < 1e-13 * np.max(np.abs(Kd))
    r = np.random.default_rng(N).uniform(-1, 1, (N - 1) ** d)
    z = pc.constant_solve(d, N, ca, cb, r)
    zd = np.linalg.solve(K0, r)
    assert np.linalg.norm(z - zd) < 1e-12 * np.linalg.norm(zd)
    assert np.linalg.norm(pc.constant_apply(d, N, ca, cb, z) - K0 @ z) < 1e-13 * np.linalg.norm(K0 @ z)
    # the constants of PCG-I are the T = 0 series: the weighted means
    B, a, b, ah, bh = _config_problem(d, N, 0)
    ca2, cb2 = pc.constant_coefficients(a, b, B)
    W = gk.node_weights(B, d)
    assert abs(ca2 - np.sum(W * a) / 2 ** d) < 1e-14 * abs(ca2)
    assert abs(cb2 - np.sum(W * b) / 2 ** d) < 1e-14 * abs(cb2)


def test_config_pattern_is_box_minus_corners():
    for (d, N, T, J) in [(2, 40, 4, 6), (2, 40, 8, 12), (3, 20, 6, 6)]:
        B, a, b, ah, bh = _config_problem(d, N, T, J=J)
        offs = set(pc.stencil_offsets(ah, bh))
        h = T + 2
        box = set()
        for o in np.ndindex(*([2 * h + 1] * d)):
            dd = tuple(v - h for v in o)
            if not all(abs(v) > T for v in dd):
                box.add(dd)
        assert offs == box
    # counts per interior row quoted for the configurations
    assert len(box) == 4849


@pytest.mark.parametrize("d,N,T", [(2, 10, 4), (2, 14, 3), (3, 6, 2)])
def test_ilu0_defining_property(d, N, T):
    B, a, b, ah, bh = _config_problem(d, N, T)
    M = pc.dense_M(d, N - 1, ah, bh)
    nz = M != 0.0
    L, U = ilu.ilu0_dense(M, nz)
    LU = L @ U
    assert np.max(np.abs((LU - M)[nz])) < 1e-12 * np.max(np.abs(M))
    # nnz(L) + nnz(U) = nnz(M) + n (unit diagonal of L counted)
    n = M.shape[0]
    assert np.count_nonzero(L) + np.count_nonzero(U) <= nz.sum() + n
    # symmetric M, symmetric pattern: U = diag(U) L^T
    Dg = np.diag(U)
    assert np.max(np.abs(U - Dg[:, None] * L.T)) < 1e-12 * np.max(np.abs(U))
    assert Dg.min() > 0
    # stencil (plain C) form gives the same factors and the same solves
    offs = pc.stencil_offsets(ah, bh)
    H = pc.stencil_rows(d, N - 1, ah, bh, offs)
    st = ilu.StencilILU(d, N - 1, offs, H).factor()
    Hd = ilu.stencil_rows_from_dense(np.tril(L, -1) + U, d, N - 1, offs)
    assert np.max(np.abs(st.H - Hd)) < 1e-12 * np.max(np.abs(M))
    r = np.random.default_rng(0).uniform(0, 1, n)
    y = ilu.forward_dense(L, r)
    assert np.linalg.norm(L @ y - r) < 1e-12 * np.linalg.norm(r)
    z = ilu.backward_dense(U, y)
    assert np.linalg.norm(U @ z - y) < 1e-12 * np.linalg.norm(y)
    assert np.linalg.norm(st.apply(r) - z) < 1e-12 * np.linalg.norm(z)


def test_full_pattern_gives_exact_lu():
    """3D, N = 5 (4^3 unknowns), T = 3: the pattern keeps every offset with
    |d_k| <= 5 unless all three exceed 3; in-grid offsets have |d_k| <= 3, so
    the pattern is full and ILU(0) is the exact LU."""
    d, N, T = 3, 5, 3
    B, a, b, ah, bh = _config_problem(d, N, T)
    M = pc.dense_M(d, N - 1, ah, bh)
    offs = pc.stencil_offsets(ah, bh)
    mask = pc.pattern_mask(d, N - 1, offs)
    assert mask.all()
    L, U = ilu.ilu0_dense(M, mask)
    assert np.max(np.abs(L @ U - M)) < 1e-12 * np.max(np.abs(M))
    r = np.random.default_rng(2).uniform(0, 1, M.shape[0])
    z = ilu.backward_dense(U, ilu.forward_dense(L, r))
    assert np.linalg.norm(z - np.linalg.solve(M, r)) < 1e-11 * np.linalg.norm(z)


def test_1d_ilu0_is_banded_lu():
    """In 1D M is banded and ILU(0) on its band has no dropped fill, so the
    one-step method solves M z = r exactly."""
    N, T = 40, 4
    B = gk.Basis(N)
    a = 2 + np.cos(B.x)
    b = 1 + B.x ** 2
    ah, bh = pc.series_pair(a, b, B, T, T)
    M = pc.dense_M(1, N - 1, ah, bh)
    L, U = ilu.ilu0_dense(M, M != 0)
    r = np.random.default_rng(1).uniform(0, 1, N - 1)
    z = ilu.backward_dense(U, ilu.forward_dense(L, r))
    assert np.linalg.norm(M @ z - r) < 1e-12 * np.linalg.norm(r)


def test_pcg_ilu_2d_N32_T4_full():
    """2D, N = 32, T = 4: PCG with the ILU(0) one-step
    preconditioner reaches 1e-10 and agrees with the dense solve."""
    cfg = synth.WORKLOADS["2d_N32_T4"]
    B, a, b, ah, bh = _config_problem(2, cfg.N, cfg.T, J=cfg.J, seed=cfg.seed)
    c = synth.coefficient_draws(2, cfg.J, cfg.seed)
    F = gk.load_vector(2, cfg.N, wl.rhs_f(c, B.x), B)
    offs = pc.stencil_offsets(ah, bh)
    st = ilu.StencilILU(2, cfg.n1, offs, pc.stencil_rows(2, cfg.n1, ah, bh, offs)).factor()
    mv = lambda v: gk.matvec_sumfact(2, cfg.N, a, b, v, B)
    x, k, hist = opcg.pcg(mv, st.apply, F, cfg.tol)
    assert np.linalg.norm(F - mv(x)) <= 1.01 * cfg.tol * np.linalg.norm(F)
    K = gk.dense_operator(2, cfg.N, a, b)
    xd = np.linalg.solve(K, F)
    assert np.linalg.norm(x - xd) < 1e-8 * np.linalg.norm(xd)
    assert 2 <= k <= 10
    xc, kc, _ = opcg.cg(mv, F, cfg.tol)
    assert kc > 10 * k


def test_paper_iteration_counts_soft(golden_dir):
    """Example 2(a) (Sec. 5.2): beta = (2x^2+2y^2+1)^4, alpha = cos(x+y),
    t1 = 6, t2 = 3, N = 40: the paper prints 6 PCG-II iterations. With f
    unstated (here f = 1) only the order of magnitude is checked."""
    N = 40
    B = gk.Basis(N)
    X, Y = np.meshgrid(B.x, B.x, indexing="xy")
    a = (2 * X ** 2 + 2 * Y ** 2 + 1) ** 4
    b = np.cos(X + Y)
    ah, bh = pc.series_pair(a, b, B, 6, 3)
    offs = pc.stencil_offsets(ah, bh)
    st = ilu.StencilILU(2, N - 1, offs, pc.stencil_rows(2, N - 1, ah, bh, offs)).factor()
    F = gk.load_vector(2, N, np.ones((N + 1, N + 1)), B)
    mv = lambda v: gk.matvec_sumfact(2, N, a, b, v, B)
    x, k, _ = opcg.pcg(mv, st.apply, F, 1e-12)
    assert 3 <= k <= 20


def test_1d_constant_preconditioner_is_t0_band_factor():
    """In 1D, K0 = c_a S + c_b M (Sec. 5.2) is banded and equals the T = 0
    truncation (the degree-0 Legendre coefficient is the mean), and ILU(0)
    on its full band is exact: the stencil ILU and the diagonalisation solve
    are two independent routes to the same K0^{-1} r."""
    N = 90
    B = gk.Basis(N)
    rng = np.random.default_rng(5)
    a = 1.0 + rng.random(N + 1)
    b = rng.random(N + 1)
    ca, cb = pc.constant_coefficients(a, b, B)
    ah, bh = pc.series_pair(a, b, B, 0, 0)
    assert abs(ah[0] - ca) <= 1e-14 * ca and abs(bh[0] - cb) <= 1e-14 * cb
    offs = pc.stencil_offsets(ah, bh)
    assert offs == [(-2,), (-1,), (0,), (1,), (2,)]
    st = ilu.StencilILU(1, N - 1, offs, pc.stencil_rows(1, N - 1, ah, bh, offs)).factor()
    r = rng.standard_normal(N - 1)
    z1 = st.apply(r)
    z2 = pc.constant_solve(1, N, ca, cb, r)
    assert np.linalg.norm(z1 - z2) <= 1e-11 * np.linalg.norm(z2)
    assert np.linalg.norm(pc.constant_apply(1, N, ca, cb, z1) - r) <= 1e-12 * np.linalg.norm(r)


@pytest.mark.parametrize("d,N,T,seed", [(2, 20, 4, 0), (3, 11, 3, 2), (3, 9, 6, 1)])
def test_many_rows_entries_match_row_by_row(d, N, T, seed):
    """The many-rows form of M's entries equals the row-by-row form (same
    terms, another multiplication order) on sampled rows, inside and at the
    grid's faces."""
    import synth
    from oracle import galerkin as gk
    from oracle import precond as pc
    from oracle import workload as owl
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, 6, seed)
    ah, bh = pc.series_pair(owl.coefficient_a(c, B.x), owl.coefficient_b(d, B.x), B, T, T)
    offs = pc.stencil_offsets(ah, bh)
    S, Mm = pc.band_factors(N - 1, T)
    n = (N - 1) ** d
    rows = [0, 1, n - 1, n // 2, n // 3, N - 2]
    out, mag, pmag = pc.M_rows_entries(d, N - 1, ah, bh, rows, offs, S, Mm)
    for t, r in enumerate(rows):
        o1, m1, p1 = pc.M_row_entries(d, N - 1, ah, bh, r, offs, S, Mm, return_abs=True)
        scale = max(np.max(m1), 1e-300)
        assert np.max(np.abs(out[t] - o1)) <= 1e-14 * scale
        assert np.max(np.abs(mag[t] - m1)) <= 1e-14 * scale
        assert np.max(np.abs(pmag[t] - p1)) <= 1e-14 * max(np.max(p1), 1e-300)


def test_stencil_rows_plane_prefix():
    """The first z-planes of the stencil rows equal the prefix of the full
    array, and the oracle's ILU(0) of that prefix equals the prefix of the
    full factorisation (rows only read earlier rows)."""
    import synth
    from oracle import galerkin as gk
    from oracle import ilu as oilu
    from oracle import precond as pc
    from oracle import workload as owl
    d, N, T = 3, 9, 3
    n1 = N - 1
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, 6, 4)
    ah, bh = pc.series_pair(owl.coefficient_a(c, B.x), owl.coefficient_b(d, B.x), B, T, T)
    offs = pc.stencil_offsets(ah, bh)
    H = pc.stencil_rows(d, n1, ah, bh, offs)
    Hp = pc.stencil_rows(d, n1, ah, bh, offs, nplanes=3)
    assert Hp.shape == (3 * n1 * n1, len(offs))
    assert np.array_equal(Hp, H[: 3 * n1 * n1])
    full = oilu.StencilILU(d, n1, offs, H).factor()
    part = oilu.StencilILU(d, n1, offs, Hp).factor(nrows=3 * n1 * n1)
    assert np.array_equal(part.H, full.H[: 3 * n1 * n1])


def test_forward_prefix_matches_full():
    """Alg. 3 over a prefix of the rows gives the prefix of the full result."""
    import synth
    from oracle import galerkin as gk
    from oracle import ilu as oilu
    from oracle import precond as pc
    from oracle import workload as owl
    d, N, T = 3, 9, 3
    n1 = N - 1
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, 6, 4)
    ah, bh = pc.series_pair(owl.coefficient_a(c, B.x), owl.coefficient_b(d, B.x), B, T, T)
    offs = pc.stencil_offsets(ah, bh)
    st = oilu.StencilILU(d, n1, offs, pc.stencil_rows(d, n1, ah, bh, offs)).factor()
    r = synth.random_vector(n1 ** d, 5)
    y, yp = st.forward(r), st.forward_prefix(r, 100)
    assert np.array_equal(y[:100], yp[:100]) and not np.any(yp[100:])
