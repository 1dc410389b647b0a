"""Pins for the operator K = A + B and the load vector (paper Sec. 3, 4.3).

Independent references: the constant-coefficient closed forms (stiffness
diag(4k+6), pentadiagonal mass) that follow from Sec. 2.1; three separately
written routes to K u (dense node sums, sum factorisation, the paper's
printed step-4 formulas); exact integrals of low-degree data; the
manufactured solution's spectral convergence."""
import numpy as np
import pytest

import synth
from oracle import galerkin as gk
from oracle import legendre as lg
from oracle import pcg as opcg
from oracle import precond as pc
from oracle import workload as wl


def _kron(mats):
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(out, m)
    return out


@pytest.mark.parametrize("d,N", [(1, 12), (2, 9), (3, 6)])
def test_constant_coefficients_closed_form(d, N):
    ca, cb = 2.7, 0.4
    S, M = gk.constant_coefficient_factors(N)
    Kc = cb * _kron([M] * d)
    for i in range(d):
        mats = [M] * d
        mats[d - 1 - i] = S
        Kc = Kc + ca * _kron(mats)
    q = N + 1
    a = ca * np.ones((q,) * d)
    b = cb * np.ones((q,) * d)
    K = gk.dense_operator(d, N, a, b)
    scale = np.max(np.abs(Kc))
    assert np.max(np.abs(K - Kc)) < 1e-13 * scale
    u = np.random.default_rng(d).uniform(0, 1, (N - 1) ** d)
    for y in (gk.matvec_sumfact(d, N, a, b, u), gk.matvec_legendre_route(d, N, a, b, u)):
        assert np.linalg.norm(y - Kc @ u) < 1e-13 * np.linalg.norm(Kc @ u)


@pytest.mark.parametrize("d,N", [(1, 3), (1, 20), (2, 3), (2, 8), (2, 13), (3, 3), (3, 7)])
def test_three_matvec_routes_agree(d, N):
    q = N + 1
    rng = np.random.default_rng(10 * d + N)
    a = 1.0 + rng.uniform(0, 1, (q,) * d)
    b = rng.uniform(0, 1, (q,) * d)
    u = rng.uniform(0, 1, (N - 1) ** d)
    K = gk.dense_operator(d, N, a, b)
    y0 = K @ u
    y1 = gk.matvec_sumfact(d, N, a, b, u)
    y2 = gk.matvec_legendre_route(d, N, a, b, u)
    nrm = np.linalg.norm(y0)
    assert np.linalg.norm(y1 - y0) < 1e-13 * nrm
    assert np.linalg.norm(y2 - y0) < 1e-13 * nrm
    # symmetric positive definite
    assert np.max(np.abs(K - K.T)) < 1e-13 * np.max(np.abs(K))
    assert np.linalg.eigvalsh(K).min() > 0


@pytest.mark.parametrize("d,N", [(2, 8), (2, 40), (3, 7)])
def test_extended_matvec_matches_dense_and_fp64(d, N):
    """The extended-precision product (the reference at the benchmark sizes)
    agrees with the dense node-sum operator and with the FP64 product."""
    q = N + 1
    rng = np.random.default_rng(7 * d + N)
    a = 1.0 + rng.uniform(0, 1, (q,) * d)
    b = rng.uniform(0, 1, (q,) * d)
    u = rng.uniform(-1, 1, (N - 1) ** d)
    ye = gk.matvec_sumfact_ext(d, N, a, b, u)
    y0 = gk.dense_operator(d, N, a, b) @ u
    y1 = gk.matvec_sumfact(d, N, a, b, u)
    nrm = np.linalg.norm(y0)
    assert np.linalg.norm(ye - y0) < 1e-13 * nrm
    assert np.linalg.norm(ye - y1) < 1e-14 * nrm


def test_matvec_symmetry_large():
    d, N = 2, 48
    q = N + 1
    rng = np.random.default_rng(3)
    a = 1.0 + rng.uniform(0, 1, (q, q))
    b = rng.uniform(0, 1, (q, q))
    u = rng.uniform(-1, 1, (N - 1) ** 2)
    v = rng.uniform(-1, 1, (N - 1) ** 2)
    Ku = gk.matvec_sumfact(d, N, a, b, u)
    Kv = gk.matvec_sumfact(d, N, a, b, v)
    assert abs(v @ Ku - u @ Kv) < 1e-12 * abs(v @ Ku)
    assert u @ Ku > 0


def test_polynomial_coefficients_exact_galerkin_equals_M():
    """When a and b have degree <= 1 per direction, (N+1)-point Gauss
    integrates the bilinear form exactly (degree <= 2N+1 per direction,
    including the mass-type direction of each gradient term), and p_T = a, b
    for T >= 1, so
    the quadrature operator K equals the preconditioner M assembled from the
    product formula (two independent routes to the same matrix)."""
    d, N, T = 2, 7, 4
    B = gk.Basis(N)
    rng = np.random.default_rng(5)
    ca = rng.uniform(-0.2, 0.2, (2, 2))
    ca[0, 0] = 3.0
    cb = rng.uniform(0.0, 0.2, (2, 2))
    cb[0, 0] = 1.0
    a = lg.legendre_series_eval(ca, [B.x, B.x])
    b = lg.legendre_series_eval(cb, [B.x, B.x])
    K = gk.dense_operator(d, N, a, b)
    ah, bh = pc.series_pair(a, b, B, T, T)
    M = pc.dense_M(d, N - 1, ah, bh)
    assert np.max(np.abs(K - M)) < 1e-12 * np.max(np.abs(K))


def test_load_vector_exact():
    """f = 1: F_{kj} = int phi_k int phi_j = 4 delta_k0 delta_j0
    (int L_k = 2 delta_k0)."""
    N = 10
    F = gk.load_vector(2, N, np.ones((N + 1, N + 1)))
    ref = np.zeros((N - 1) ** 2)
    ref[0] = 4.0
    assert np.max(np.abs(F - ref)) < 1e-14


def _solve_config(N, J=6, seed=0, T=4, tol=1e-12):
    B = gk.Basis(N)
    c = synth.coefficient_draws(2, J, seed)
    a = wl.coefficient_a(c, B.x)
    b = wl.coefficient_b(2, B.x)
    f = wl.rhs_f(c, B.x)
    F = gk.load_vector(2, N, f, B)
    K = gk.dense_operator(2, N, a, b)
    x = np.linalg.solve(K, F)
    vals = B.Phi @ x.reshape(N - 1, N - 1) @ B.Phi.T
    return np.max(np.abs(vals - wl.u_star(2, B.x)))


def test_manufactured_solution_spectral_convergence():
    errs = [_solve_config(N) for N in (8, 12, 16, 24)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e-5
    assert errs[3] < 1e-10


def test_mutations_are_caught():
    """A sign flip or an index shift in the printed step-4 formula makes the
    Legendre route disagree with the dense operator (the pins above would
    fail): checks that those pins are sensitive."""
    d, N = 2, 6
    q = N + 1
    rng = np.random.default_rng(1)
    a = 1.0 + rng.uniform(0, 1, (q, q))
    b = rng.uniform(0, 1, (q, q))
    u = rng.uniform(0, 1, (N - 1) ** 2)
    y0 = gk.dense_operator(d, N, a, b) @ u
    good = gk.matvec_legendre_route(d, N, a, b, u)
    assert np.linalg.norm(good - y0) < 1e-13 * np.linalg.norm(y0)
    orig = gk._dphi_to_legendre
    try:
        gk._dphi_to_legendre = lambda uh, axis, N_: orig(uh, axis, N_) * 1.01
        bad = gk.matvec_legendre_route(d, N, a, b, u)
    finally:
        gk._dphi_to_legendre = orig
    assert np.linalg.norm(bad - y0) > 1e-4 * np.linalg.norm(y0)


def test_pcg_matches_dense_solve_2d_N32_family():
    cfg = synth.WORKLOADS["2d_N32_T4"]
    N = 16
    B = gk.Basis(N)
    c = synth.coefficient_draws(2, cfg.J, cfg.seed)
    a = wl.coefficient_a(c, B.x)
    b = wl.coefficient_b(2, B.x)
    F = gk.load_vector(2, N, wl.rhs_f(c, B.x), B)
    K = gk.dense_operator(2, N, a, b)
    xd = np.linalg.solve(K, F)
    x, k, hist = opcg.cg(lambda v: K @ v, F, 1e-12)
    assert np.linalg.norm(F - K @ x) <= 1.01e-12 * np.linalg.norm(F)
    assert np.linalg.norm(x - xd) < 1e-9 * np.linalg.norm(xd)
