"""Oracle pins for the diagonal anisotropic form of Example 4 (Sec. 5.2):
-sum_j (a_j u_{x_j})_{x_j} + b u, one diffusion field per direction.

Each pin uses fields that differ between directions, so a field applied to
the wrong direction (a transposed operand) fails it:
  * the dense node-sum assembly and the sum-factorised product agree;
  * with every a_j a polynomial of degree <= 3 and b of degree <= 1 per
    direction, Gauss quadrature on N+1 nodes is exact for the bilinear
    form, and the Legendre series are exact once T >= 3, so M (Sec. 4.2,
    exact triple products) equals the operator K itself;
  * the separable stencil rows equal the rows of the dense Kronecker M;
  * with constant fields a_j = c_j the closed-form K0 equals K, and the
    diagonalisation solve inverts it.
"""
import numpy as np
import pytest

from oracle import galerkin as gk
from oracle import ilu
from oracle import pcg as opcg
from oracle import precond as pc
from oracle import workload as owl


def _grid(xs, d):
    mesh = np.meshgrid(*([xs] * d), indexing="ij")
    return [mesh[d - 1 - i] for i in range(d)]        # X[0] = x (last axis)


def _poly_fields(d, N, seed):
    rng = np.random.default_rng(seed)
    B = gk.Basis(N)
    X = _grid(B.x, d)
    a_dir = []
    for j in range(d):
        c = rng.uniform(-0.3, 0.3, 4)
        # a_j: a cubic in its own variable and a linear term in the next one
        a_dir.append(2.0 + j + sum(c[k] * X[j] ** k for k in range(1, 4)) + 0.2 * X[(j + 1) % d])
    b = 1.0 + 0.3 * X[0] - 0.2 * X[d - 1]
    return B, a_dir, b


@pytest.mark.parametrize("d,N", [(2, 7), (2, 11), (3, 5)])
def test_two_product_routes_agree(d, N):
    B, a_dir, b = _poly_fields(d, N, 10 + N)
    rng = np.random.default_rng(N)
    a_dir = [a * (1.0 + 0.1 * rng.random(a.shape)) for a in a_dir]   # not separable any more
    u = rng.uniform(-1, 1, (N - 1) ** d)
    K = gk.dense_operator(d, N, a_dir, b)
    y = gk.matvec_sumfact(d, N, a_dir, b, u, B)
    assert np.linalg.norm(K @ u - y) <= 1e-13 * np.linalg.norm(y)
    assert np.max(np.abs(K - K.T)) <= 1e-13 * np.max(np.abs(K))
    # swapping the fields changes the operator (the pins below can see a swap)
    Ks = gk.dense_operator(d, N, a_dir[::-1], b)
    assert np.max(np.abs(K - Ks)) > 1e-3 * np.max(np.abs(K))


@pytest.mark.parametrize("d,N", [(2, 8), (2, 12), (3, 6)])
def test_full_series_M_equals_K_for_polynomial_fields(d, N):
    B, a_dir, b = _poly_fields(d, N, N)
    ahs, bh = pc.series_dir(a_dir, b, B, [4] * d, 4)
    M = pc.dense_M(d, N - 1, ahs, bh)
    K = gk.dense_operator(d, N, a_dir, b)
    assert np.max(np.abs(M - K)) <= 1e-12 * np.max(np.abs(K))
    offs = pc.stencil_offsets(ahs, bh)
    mask = pc.pattern_mask(d, N - 1, offs)
    assert np.all(mask[M != 0.0])
    H = pc.stencil_rows(d, N - 1, ahs, bh, offs)
    H2 = ilu.stencil_rows_from_dense(M, d, N - 1, offs)
    assert np.max(np.abs(H - H2)) <= 1e-13 * np.max(np.abs(M))


@pytest.mark.parametrize("d,N,Ta", [(2, 14, (4, 2)), (2, 14, (1, 5)), (3, 7, (3, 1, 2))])
def test_per_direction_truncation(d, N, Ta):
    """Different truncations per direction: rows against the dense Kronecker
    M, and M's pattern inside NZ(M); a field's reach follows its own t_1j."""
    B, a_dir, b = _poly_fields(d, N, 3 * N)
    rng = np.random.default_rng(N)
    a_dir = [a * np.exp(0.2 * rng.random(a.shape)) for a in a_dir]
    ahs, bh = pc.series_dir(a_dir, b, B, list(Ta), 1)
    for ah, t in zip(ahs, Ta):
        assert ah.shape == (t + 1,) * d
    M = pc.dense_M(d, N - 1, ahs, bh)
    assert np.linalg.eigvalsh(M).min() > 0
    offs = pc.stencil_offsets(ahs, bh)
    mask = pc.pattern_mask(d, N - 1, offs)
    assert np.array_equal(mask, M != 0.0)
    H = pc.stencil_rows(d, N - 1, ahs, bh, offs)
    H2 = ilu.stencil_rows_from_dense(M, d, N - 1, offs)
    assert np.max(np.abs(H - H2)) <= 1e-13 * np.max(np.abs(M))


@pytest.mark.parametrize("d,N", [(2, 9), (3, 6)])
def test_constant_anisotropic_k0(d, N):
    cs = [1.7, 0.6, 2.3][:d]
    cb = 0.4
    q = N + 1
    K0 = pc.constant_operator_dense(d, N, cs, cb)
    Kd = gk.dense_operator(d, N, [np.full((q,) * d, c) for c in cs], np.full((q,) * d, cb))
    assert np.max(np.abs(K0 - Kd)) <= 1e-13 * np.max(np.abs(Kd))
    r = np.random.default_rng(N).uniform(-1, 1, (N - 1) ** d)
    z = pc.constant_solve(d, N, cs, cb, r)
    assert np.linalg.norm(K0 @ z - r) <= 1e-12 * np.linalg.norm(r)
    assert np.linalg.norm(pc.constant_apply(d, N, cs, cb, z) - K0 @ z) <= 1e-13 * np.linalg.norm(K0 @ z)
    B = gk.Basis(N)
    a_dir = [np.full((q,) * d, c) for c in cs]
    cs2, cb2 = pc.constant_coefficients(a_dir, np.full((q,) * d, cb), B)
    assert np.allclose(cs2, cs, rtol=1e-14) and abs(cb2 - cb) <= 1e-14


def test_example4a_soft(golden_dir):
    """Example 4(a), N = 40: the paper prints 86 (PCG-I), 10 (t11 = 4,
    t12 = 3) and 8 (t11 = 5, t12 = 3); f is not stated (f = 1 here), so the
    counts are checked to within a factor 3."""
    N = 40
    B = gk.Basis(N)
    a_dir, b = owl.example4(2, B.x)
    F = gk.load_vector(2, N, np.ones((N + 1, N + 1)), B)
    mv = lambda v: gk.matvec_sumfact(2, N, a_dir, b, v, B)
    cs, cb = pc.constant_coefficients(a_dir, b, B)
    k1 = opcg.pcg(mv, lambda r: pc.constant_solve(2, N, cs, cb, r), F, 1e-12, kmax=4000)[1]
    ks = []
    for Ta in ((4, 3), (5, 3)):
        ahs, bh = pc.series_dir(a_dir, b, B, list(Ta), 0)
        offs = pc.stencil_offsets(ahs, bh)
        st = ilu.StencilILU(2, N - 1, offs, pc.stencil_rows(2, N - 1, ahs, bh, offs)).factor()
        ks.append(opcg.pcg(mv, st.apply, F, 1e-12, kmax=4000)[1])
    print("Example 4(a) N=40: PCG-I %d, PCG-II %s" % (k1, ks))
    assert 86 / 3 <= k1 <= 86 * 3
    assert 10 / 3 <= ks[0] <= 30 and 8 / 3 <= ks[1] <= 24
