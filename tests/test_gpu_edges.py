"""Degenerate and boundary cases of the GPU path against the oracle: one
unknown (N = 2), patterns wider than the grid (T > N), the constant
truncation T = 0, a zero right-hand side, and Ta != Tb.

Tolerances as in test_gpu_parity: products relative 1e-12, factors and
substitutions relative 1e-12, solutions by the oracle's own residual.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import galerkin as gk
from oracle import ilu as oilu
from oracle import precond as pc
from tests.checks import assert_entrywise, matvec_magnitude

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _inputs(d, N, seed):
    q = N + 1
    return synth.random_nodal(d, q, seed, 1.0, 2.0), synth.random_nodal(d, q, seed + 1, 0.0, 1.0)


@pytest.mark.parametrize("d,N,Ta,Tb", [(2, 2, 4, 4), (3, 2, 2, 2), (2, 5, 8, 8), (2, 12, 0, 0), (3, 4, 0, 0),
                                       (2, 20, 6, 2), (3, 6, 1, 3)])
def test_edge_factor_sweeps_and_solve(d, N, Ta, Tb):
    from paper_2004_13961_amd.solver import Factor, Problem, pcg_solve
    print("case edge d=%d N=%d Ta=%d Tb=%d" % (d, N, Ta, Tb), flush=True)
    a, b = _inputs(d, N, 40 + 3 * N + d)
    n = (N - 1) ** d
    B = gk.Basis(N)
    P = Problem(d, N, _dev(a), _dev(b))
    # product
    u = synth.random_vector(n, 9)
    ref = gk.matvec_sumfact(d, N, a, b, u, B)
    assert_entrywise(_host(P.matvec(_dev(u))), ref, 1e-12, matvec_magnitude(d, N, a, b, u, B), "matvec")
    # factor against the oracle's stencil ILU(0)
    ah, bh = pc.series_pair(a, b, B, Ta, Tb)
    offs = pc.stencil_offsets(ah, bh)
    st = oilu.StencilILU(d, N - 1, offs, pc.stencil_rows(d, N - 1, ah, bh, offs)).factor()
    M = Factor(P, Ta, Tb)
    desc = M.describe()
    assert [tuple(o[:d]) for o in desc["offsets"]] == [tuple(o) for o in offs]
    nlo = desc["n_lower"]
    Lo, Do = st.H[:, :nlo], st.H[:, nlo]
    assert np.max(np.abs(_host(desc["L"]) - Lo)) <= 1e-12 * max(1.0, np.max(np.abs(Lo)))
    assert np.max(np.abs(_host(desc["D"]) - Do)) <= 1e-12 * np.max(np.abs(Do))
    r = synth.random_vector(n, 10)
    assert_entrywise(_host(M.forward(_dev(r))), st.forward(r), 1e-12, label="forward")
    assert_entrywise(_host(M.backward(_dev(r))), st.backward(r), 1e-12, label="backward")
    assert_entrywise(_host(M.apply(_dev(r))), st.apply(r), 1e-12, label="apply")
    # solve
    F = _dev(synth.random_vector(n, 11))
    x, info = pcg_solve(P, M, F, rtol=1e-10)
    xg = _host(x)
    Fh = _host(F)
    assert np.linalg.norm(Fh - gk.matvec_sumfact(d, N, a, b, xg, B)) <= 1.5e-10 * np.linalg.norm(Fh)
    if n == 1:
        # one unknown: K is 1x1 and M is exactly K up to the truncation
        assert info["iters"] <= 2


def test_zero_rhs_gives_zero():
    from paper_2004_13961_amd.solver import Factor, Problem, pcg_solve
    a, b = _inputs(2, 16, 3)
    P = Problem(2, 16, _dev(a), _dev(b))
    M = Factor(P, 4)
    F = torch.zeros(15 * 15, dtype=torch.float64, device="cuda")
    x = torch.full_like(F, 7.0)
    x, info = pcg_solve(P, M, F, x=x, rtol=1e-10)
    assert info["status"] == "LGP_OK"
    assert info["iters"] == 0
    assert np.all(_host(x) == 0.0)


def test_initial_guess_is_used():
    """Starting from the solution itself, PCG stops at once (true residual
    already below the tolerance)."""
    from paper_2004_13961_amd.solver import Factor, Problem, pcg_solve
    a, b = _inputs(2, 24, 5)
    P = Problem(2, 24, _dev(a), _dev(b))
    M = Factor(P, 4)
    F = _dev(synth.random_vector(23 * 23, 6))
    x, info = pcg_solve(P, M, F, rtol=1e-11)
    x2, info2 = pcg_solve(P, M, F, x=x.clone(), rtol=1e-10)
    assert info2["iters"] == 0
    assert info2["relres_true"] <= 1e-10
