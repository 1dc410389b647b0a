"""Fast discrete Legendre transforms (lgp_dlt_lines) and the product through
them (lgp_matvec_fast) against the oracle.

The transforms are compared with the oracle's BDLT and FDLT sums of Sec. 2.2
(dense sums over its own table of L_n at its own Gauss nodes), entry by entry
against each entry's term magnitude (sum of |c_n L_n(x_k)|, resp. (2n+1)/2
sum of |w_k f_k L_n(x_k)|): the expansion is cut where its error bound is
1e-16, and its FFT sums round at about eps log2(L) of the sum of the
expansion's terms, which exceed the terms |c_n L_n(x_k)| by up to the ratio
of C_n / sqrt(2 sin theta) to |L_n(cos theta)|, about sqrt(n); so the bound is
max(1e-13, 4 eps sqrt(N+1) log2(L)), 3.1e-13 at N = 1023. Sizes with N >= 64 use the expansion (lgp_dlt_blocks > 0), the
smaller ones the recurrence alone. The product is compared with the oracle's
sum-factorised product entry by entry within 1e-12 of each entry's term
magnitude, as the dense product is.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import galerkin as gk
from oracle import legendre as lg
from oracle import workload as owl
from tests.checks import assert_entrywise, matvec_magnitude

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _problem(d, N, seed=5):
    from paper_2004_13961_amd.solver import Problem
    from paper_2004_13961_amd.workload import family_nodal, paper_example_nodal
    if d == 1:   # the transforms do not read the coefficients; Example 1(a)'s are positive at every N
        a, b, _ = paper_example_nodal("a", 1, N)
    else:
        a, b, _, _ = family_nodal(d, N, 6, seed, with_rhs=False)
    return Problem(d, N, _dev(a), _dev(b))


def _dlt_tol(N):
    L = 1
    while L < 2 * (N + 1):
        L *= 2
    return max(1e-13, 4 * np.finfo(float).eps * np.sqrt(N + 1) * np.log2(L))


@pytest.mark.parametrize("N", [3, 17, 63, 64, 100, 255, 400, 1023, 1024, 2047])
def test_dlt_lines_vs_oracle(N):
    from paper_2004_13961_amd.solver import FastTransforms
    print("case dlt N=%d" % N, flush=True)
    P = _problem(1, N)
    T = FastTransforms(P)
    print("blocks %d" % T.blocks(), flush=True)
    if N >= 100:
        assert T.blocks() > 0
    if N < 64:
        assert T.blocks() == 0
    x, w = lg.gauss_legendre(N)
    Ptab = lg.legendre_table(N, x)           # [n, k] = L_n(x_k)
    rng = np.random.default_rng(N)
    count = 3
    c = rng.standard_normal((count, N + 1))
    c[1] /= (1.0 + np.arange(N + 1)) ** 2    # a decaying spectrum
    f = _host(T.lines(_dev(c).reshape(count, N + 1)))
    f = f.reshape(count, N + 1)
    for i in range(count):
        ref = lg.bdlt(c[i], Ptab)
        mag = np.abs(Ptab).T @ np.abs(c[i])
        worst = assert_entrywise(f[i], ref, _dlt_tol(N), mag, "BDLT N=%d row %d" % (N, i))
        print("BDLT row %d worst %.2e of term magnitude" % (i, worst), flush=True)
    v = rng.standard_normal((count, N + 1))
    cf = _host(T.lines(_dev(v).reshape(count, N + 1), forward=True)).reshape(count, N + 1)
    s = (2 * np.arange(N + 1) + 1) / 2.0
    for i in range(count):
        ref = lg.fdlt(v[i], Ptab, w)
        mag = s * (np.abs(Ptab) @ (w * np.abs(v[i])))
        worst = assert_entrywise(cf[i], ref, _dlt_tol(N), mag, "FDLT N=%d row %d" % (N, i))
        print("FDLT row %d worst %.2e of term magnitude" % (i, worst), flush=True)


@pytest.mark.parametrize("d,N", [(1, 200), (1, 1023), (2, 33), (2, 100), (2, 130), (3, 12), (3, 70)])
def test_matvec_fast_vs_oracle(d, N):
    """Sec. 4.3 steps 1-4 through the fast transforms, against the oracle's
    sum-factorised product and the library's dense product."""
    from paper_2004_13961_amd.solver import FastTransforms
    print("case matvec_fast d=%d N=%d" % (d, N), flush=True)
    P = _problem(d, N, seed=N)
    T = FastTransforms(P)
    B = gk.Basis(N)
    if d == 1:
        a_o, b_o = owl.paper_example("a", 1, B.x)
    else:
        c = synth.coefficient_draws(d, 6, N)
        a_o = owl.coefficient_a(c, B.x)
        b_o = owl.coefficient_b(d, B.x)
    u = synth.random_vector((N - 1) ** d, 31)
    y = _host(T.matvec(_dev(u)))
    ref = gk.matvec_sumfact(d, N, a_o, b_o, u, B)
    mag = matvec_magnitude(d, N, a_o, b_o, u, B)
    worst = assert_entrywise(y, ref, 1e-12, mag, "fast product")
    yd = _host(P.matvec(_dev(u)))
    print("blocks %d, worst %.2e of term magnitude, max |fast - dense| / max|dense| %.2e" % (
        T.blocks(), worst, np.max(np.abs(y - yd)) / np.max(np.abs(yd))), flush=True)


def test_matvec_fast_anisotropic():
    """Example 4's per-direction coefficients (lgp_build_problem_diag)."""
    from paper_2004_13961_amd.solver import FastTransforms, Problem
    from paper_2004_13961_amd.workload import paper_example4_nodal
    d, N = 2, 90
    a_g, b_g, _ = paper_example4_nodal(d, N)
    P = Problem(d, N, _dev(a_g), _dev(b_g))
    T = FastTransforms(P)
    B = gk.Basis(N)
    a_dir, b = owl.example4(d, B.x)
    u = synth.random_vector((N - 1) ** d, 33)
    y = _host(T.matvec(_dev(u)))
    ref = gk.matvec_sumfact(d, N, list(a_dir), b, u, B)
    mag = matvec_magnitude(d, N, list(a_dir), b, u, B)
    assert_entrywise(y, ref, 1e-12, mag, "fast product, anisotropic")


def test_dlt_unsupported_size():
    """N + 1 > 2048: no plan (size query 0, create refused)."""
    import ctypes
    from paper_2004_13961_amd import lgpcg
    P = _problem(1, 2048)
    L = lgpcg.lib()
    assert L.lgp_dlt_bytes(P.handle) == 0
    buf = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = L.lgp_dlt_create(P.handle, ctypes.c_void_p(buf.data_ptr()), buf.numel(), None, ctypes.byref(h))
    assert lgpcg.STATUS[st] == "LGP_E_UNSUPPORTED"
