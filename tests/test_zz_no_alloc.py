"""lgp_pcg_solve_noalloc (the solve whose workspace is the library's own
device array) against lgp_pcg_solve with a caller workspace, through the C
ABI: two calls in a row, the second on a smaller problem, each compared
with the ordinary entry point (same kernels, same reduction order, so the
solutions agree bit for bit); and a problem whose workspace exceeds the
array is refused with LGP_E_NOMEM."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import galerkin as gk
from oracle import workload as owl

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def _solve_noalloc(P, M, F, rtol, inner):
    from paper_2004_13961_amd import lgpcg
    from paper_2004_13961_amd.solver import _ptr, _stream
    L = lgpcg.lib()
    x = torch.zeros_like(F)
    o = lgpcg.SolveOpts(rtol, 2000, lgpcg.DTYPES[inner], 0.0, 60, 4)
    info = lgpcg.SolveInfo()
    st = L.lgp_pcg_solve_noalloc(P.handle, M.handle, _ptr(F), _ptr(x), ctypes.byref(o), _stream(),
                                 ctypes.byref(info))
    torch.cuda.synchronize()
    return st, x, info


def _case(d, N, T, seed):
    from paper_2004_13961_amd.solver import Factor, Problem
    from paper_2004_13961_amd.workload import family_nodal
    a, b, f, _ = family_nodal(d, N, 6, seed)
    P = Problem(d, N, _dev(a), _dev(b))
    F = P.load_vector(_dev(f))
    return P, F, Factor(P, T, store="f32")


def test_noalloc_matches_workspace_solve():
    from paper_2004_13961_amd import lgpcg
    from paper_2004_13961_amd.solver import pcg_solve
    assert lgpcg.lib().lgp_pcg_solve_noalloc_max_bytes() == 64 << 20
    for (d, N, T, seed, inner) in [(2, 64, 6, 0, "f64"), (2, 33, 4, 1, "f64"), (2, 40, 4, 2, "f32"),
                                   (3, 10, 4, 3, "f64")]:
        print("case noalloc d=%d N=%d T=%d %s" % (d, N, T, inner), flush=True)
        P, F, M = _case(d, N, T, seed)
        x_ref, info_ref = pcg_solve(P, M, F, rtol=1e-10, inner=inner)
        st, x, info = _solve_noalloc(P, M, F, 1e-10, inner)
        assert st == 0, lgpcg.STATUS.get(st)
        assert info.iters == info_ref["iters"] and info.outer == info_ref["outer"]
        assert info.relres_true <= 1e-10
        assert torch.equal(x, x_ref)
        # the oracle's own residual of the result
        B = gk.Basis(N)
        c = synth.coefficient_draws(d, 6, seed)
        a_o, b_o = owl.coefficient_a(c, B.x), owl.coefficient_b(d, B.x)
        F_o = gk.load_vector(d, N, owl.rhs_f(c, B.x), B)
        xg = x.cpu().numpy()
        assert np.linalg.norm(F_o - gk.matvec_sumfact(d, N, a_o, b_o, xg, B)) <= 1.5e-10 * np.linalg.norm(F_o)


def test_noalloc_refuses_oversized_workspace():
    from paper_2004_13961_amd import lgpcg
    from paper_2004_13961_amd.solver import Factor, Problem
    N = 1500   # 2.24e6 unknowns: 72 MB of FP64 workspace
    q = N + 1
    a = synth.random_nodal(2, q, 5, 1.0, 2.0)
    b = synth.random_nodal(2, q, 6, 0.0, 1.0)
    P = Problem(2, N, _dev(a), _dev(b))
    M = Factor(P, 0)
    F = torch.ones(P.n, dtype=torch.float64, device="cuda")
    assert lgpcg.lib().lgp_solve_workspace_bytes(P.handle, 0) > (64 << 20)
    st, x, info = _solve_noalloc(P, M, F, 1e-10, "f64")
    assert lgpcg.STATUS[st] == "LGP_E_NOMEM"
