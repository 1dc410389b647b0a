"""Pins for oracle/legendre.py and the basis tables (paper Sec. 2, Sec. 3).

Independent references: textbook closed forms of small Gauss rules
(tests/golden), exact polynomial moments, numpy.polynomial.legendre (a
separate implementation of the same special functions)."""
import math
import os

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

from oracle import legendre as lg
from oracle.galerkin import Basis


def test_gauss_closed_forms(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "gauss_nodes_closed_form.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            N, i, xe, we = line.split()
            env = {"sqrt": math.sqrt}
            rows.append((int(N), int(i), eval(xe, env), eval(we, env)))
    for N, i, xv, wv in rows:
        x, w = lg.gauss_legendre(N)
        assert abs(x[i] - xv) < 1e-15
        assert abs(w[i] - wv) < 1e-15


@pytest.mark.parametrize("N", [2, 5, 16, 31, 64, 127, 255, 1024])
def test_gauss_rule_properties(N):
    x, w = lg.gauss_legendre(N)
    assert np.all(np.diff(x) > 0)
    assert abs(w.sum() - 2.0) < 1e-13
    # roots of L_{N+1}: the residual is at rounding level relative to the
    # slope there, i.e. the node sits within ~1 ulp of the root
    P = lg.legendre_table(N + 1, x)
    dP = lg.legendre_deriv_table(N + 1, x)
    assert np.max(np.abs(P[N + 1] / dP[N + 1])) < 4e-16
    # exact for every monomial of degree <= 2N+1 (checked up to 40)
    for k in range(0, min(2 * N + 1, 40) + 1):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * x ** k) - exact) < 1e-13


@pytest.mark.parametrize("N", [3, 10, 50, 100])
def test_gauss_vs_numpy(N):
    x, w = lg.gauss_legendre(N)
    xr, wr = npleg.leggauss(N + 1)
    assert np.max(np.abs(x - xr)) < 1e-14
    assert np.max(np.abs(w - wr)) < 1e-14


def test_legendre_table_vs_numpy_and_endpoints():
    x = np.linspace(-1, 1, 37)
    P = lg.legendre_table(30, x)
    for n in range(31):
        c = np.zeros(n + 1)
        c[n] = 1.0
        assert np.max(np.abs(P[n] - npleg.legval(x, c))) < 1e-13
        # symmetry property: L_n(+-1) = (+-1)^n
        assert P[n][0] == pytest.approx((-1.0) ** n, abs=1e-14)
        assert P[n][-1] == pytest.approx(1.0, abs=1e-14)


def test_derivative_recurrence_vs_numpy():
    x = np.linspace(-0.99, 0.99, 29)
    dP = lg.legendre_deriv_table(25, x)
    for n in range(26):
        c = np.zeros(n + 1)
        c[n] = 1.0
        ref = npleg.legval(x, npleg.legder(c))
        assert np.max(np.abs(dP[n] - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("N", [4, 17, 64])
def test_discrete_orthogonality_and_dlt_roundtrip(N):
    x, w = lg.gauss_legendre(N)
    P = lg.legendre_table(N, x)
    G = (P * w) @ P.T
    ref = np.diag(2.0 / (2 * np.arange(N + 1) + 1))
    assert np.max(np.abs(G - ref)) < 1e-13
    c = np.random.default_rng(N).standard_normal(N + 1)
    assert np.max(np.abs(lg.fdlt(lg.bdlt(c, P), P, w) - c)) < 1e-12
    c2 = np.random.default_rng(N + 1).standard_normal((N + 1, N + 1))
    back = lg.tensor_fdlt(lg.tensor_bdlt(c2, P), P, w)
    assert np.max(np.abs(back - c2)) < 1e-12


@pytest.mark.parametrize("N", [4, 9, 33])
def test_basis_tables(N):
    B = Basis(N)
    ends = np.array([-1.0, 1.0])
    Pe = lg.legendre_table(N + 1, ends)
    k = np.arange(N - 1)
    # phi_k(+-1) = 0 (Sec. 3)
    assert np.max(np.abs(Pe[k] - Pe[k + 2])) < 1e-14
    # D = phi_k' from numpy's derivative of L_k - L_{k+2}
    for kk in range(N - 1):
        c = np.zeros(kk + 3)
        c[kk] = 1.0
        c[kk + 2] = -1.0
        ref = npleg.legval(B.x, npleg.legder(c))
        assert np.max(np.abs(B.D[:, kk] - ref)) < 1e-11 * (2 * kk + 3)
        ref0 = npleg.legval(B.x, c)
        assert np.max(np.abs(B.Phi[:, kk] - ref0)) < 1e-13
