"""GPU path (C ABI) against the oracle, element by element, at sizes the
oracle finishes in seconds (several 64x64 tiles, ragged tails).

Tolerances: matvec relative 1e-12 in FP64 (2-norm, as the solver's
matvec target); factors, sweeps relative 1e-12; solutions by the oracle's
own FP64 true residual <= tol.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import galerkin as gk
from oracle import ilu as oilu
from oracle import pcg as opcg
from oracle import precond as pc
from oracle import workload as owl
from tests.checks import assert_entrywise, load_magnitude, matvec_magnitude

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _random_problem(d, N, seed):
    q = N + 1
    a = synth.random_nodal(d, q, seed, 1.0, 2.0)
    b = synth.random_nodal(d, q, seed + 1, 0.0, 1.0)
    return a, b


MATVEC_CASES = [(2, 3), (2, 4), (2, 17), (2, 32), (2, 33), (2, 64), (2, 100), (2, 130),
                (3, 3), (3, 5), (3, 8), (3, 12), (3, 17), (3, 24)]


@pytest.mark.parametrize("d,N", MATVEC_CASES)
def test_matvec_f64(d, N):
    from paper_2004_13961_amd.solver import Problem
    print("case matvec d=%d N=%d" % (d, N), flush=True)
    a, b = _random_problem(d, N, 10 * N + d)
    u = synth.random_vector((N - 1) ** d, 100 + N)
    ref = gk.matvec_sumfact(d, N, a, b, u)
    P = Problem(d, N, _dev(a).reshape(-1), _dev(b).reshape(-1))
    y = _host(P.matvec(_dev(u)))
    assert_entrywise(y, ref, 1e-12, matvec_magnitude(d, N, a, b, u), "matvec")


@pytest.mark.parametrize("d,N,prec,tol", [(2, 40, "f32", 2e-6), (2, 40, "bf16", 3e-2),
                                          (3, 12, "f32", 2e-6), (3, 12, "bf16", 3e-2)])
def test_matvec_low_precision(d, N, prec, tol):
    from paper_2004_13961_amd.solver import Problem
    print("case matvec %s d=%d N=%d" % (prec, d, N), flush=True)
    a, b = _random_problem(d, N, 7)
    u = synth.random_vector((N - 1) ** d, 8)
    ref = gk.matvec_sumfact(d, N, a, b, u)
    P = Problem(d, N, _dev(a).reshape(-1), _dev(b).reshape(-1))
    y = _host(P.matvec(torch.from_numpy(u.astype(np.float32)).cuda(), prec=prec)).astype(np.float64)
    assert_entrywise(y, ref, tol, matvec_magnitude(d, N, a, b, u), "matvec " + prec)


@pytest.mark.parametrize("d,N", [(2, 9), (2, 40), (3, 7), (3, 16)])
def test_load_vector(d, N):
    from paper_2004_13961_amd.solver import Problem
    a, b = _random_problem(d, N, 3)
    f = synth.random_nodal(d, N + 1, 4, -1.0, 1.0)
    ref = gk.load_vector(d, N, f)
    P = Problem(d, N, _dev(a).reshape(-1), _dev(b).reshape(-1))
    F = _host(P.load_vector(_dev(f).reshape(-1)))
    assert_entrywise(F, ref, 1e-13, load_magnitude(d, N, f), "load vector")


def _oracle_factor(d, N, a, b, Ta, Tb):
    B = gk.Basis(N)
    ah, bh = pc.series_pair(a, b, B, Ta, Tb)
    offs = pc.stencil_offsets(ah, bh)
    H = pc.stencil_rows(d, N - 1, ah, bh, offs)
    st = oilu.StencilILU(d, N - 1, offs, H).factor()
    return st, offs


# 3D: N = 7, 10, 12 are narrower than twice the stencil's reach (generic
# kernel); N = 14 and 18 take the chunked kernel, with a part-filled last
# chunk on every line (13 = 8 + 5 and 17 = 2 x 8 + 1 rows)
FACTOR_CASES = [(2, 12, 4, 4, 0), (2, 33, 4, 4, 0), (2, 40, 8, 8, 1), (2, 50, 6, 3, 2),
                (3, 7, 2, 2, 0), (3, 10, 4, 4, 1), (3, 12, 6, 6, 2), (3, 14, 2, 2, 1), (3, 18, 6, 6, 2)]


# the ILU(0) kernel variants: 2 (dataflow, the default where it applies) and
# 1 (generic; the only one for the 3D stencils, whose hundreds of lower
# offsets exceed what the dataflow kernel holds)
KERNEL_CASES = [(2, 40, 8, 8, 1, k) for k in (2, 1)] + [(2, 50, 6, 3, 2, 2), (2, 33, 4, 4, 0, 1)]


@pytest.mark.parametrize("d,N,Ta,Tb,seed,kernel", [c + (0,) for c in FACTOR_CASES] + KERNEL_CASES)
def test_factor_and_sweeps(d, N, Ta, Tb, seed, kernel, monkeypatch):
    """Benchmark-family coefficients (evaluated independently on each side):
    same pattern, L and pivots to 1e-12, both sweeps to 1e-12."""
    from paper_2004_13961_amd.solver import Problem, Factor
    from paper_2004_13961_amd.workload import family_nodal
    print("case factor d=%d N=%d Ta=%d Tb=%d kernel=%d" % (d, N, Ta, Tb, kernel), flush=True)
    monkeypatch.setenv("LGP_FACTOR_KERNEL", str(kernel))
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, 6, seed)
    a_o = owl.coefficient_a(c, B.x)
    b_o = owl.coefficient_b(d, B.x)
    st, offs = _oracle_factor(d, N, a_o, b_o, Ta, Tb)
    a_g, b_g, _, _ = family_nodal(d, N, 6, seed, with_rhs=False)
    P = Problem(d, N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    Fc = Factor(P, Ta, Tb)
    desc = Fc.describe()
    print("factor kernel %d" % desc["factor_kernel"], flush=True)
    if kernel:
        assert desc["factor_kernel"] == kernel
    elif d == 3:   # the chunked kernel wherever the grid is wider than twice the reach in x and y
        reach = max(max(abs(o[0]), abs(o[1])) for o in offs)
        assert desc["factor_kernel"] == (3 if N - 1 > 2 * reach else 1)
    assert [tuple(o[:d]) for o in desc["offsets"]] == [tuple(o) for o in offs]
    nlo = desc["n_lower"]
    Lg = _host(desc["L"])
    Dg = _host(desc["D"])
    Lo = st.H[:, :nlo]
    Do = st.H[:, nlo]
    assert np.max(np.abs(Lg - Lo)) <= 1e-12 * max(1.0, np.max(np.abs(Lo)))
    assert np.max(np.abs(Dg - Do)) <= 1e-12 * np.max(np.abs(Do))
    assert np.max(np.abs(_host(desc["invD"]) * Do - 1.0)) <= 1e-12
    r = synth.random_vector((N - 1) ** d, 5)
    y_ref = st.forward(r)
    y = _host(Fc.forward(_dev(r)))
    assert_entrywise(y, y_ref, 1e-12, label="forward")
    z_ref = st.backward(r)
    z = _host(Fc.backward(_dev(r)))
    assert_entrywise(z, z_ref, 1e-12, label="backward")
    zz = _host(Fc.apply(_dev(r)))
    assert_entrywise(zz, st.apply(r), 1e-12, label="apply")


def _config_oracle(cfg, N=None):
    N = cfg.N if N is None else N
    B = gk.Basis(N)
    c = synth.coefficient_draws(cfg.d, cfg.J, cfg.seed)
    a = owl.coefficient_a(c, B.x)
    b = owl.coefficient_b(cfg.d, B.x)
    f = owl.rhs_f(c, B.x)
    F = gk.load_vector(cfg.d, N, f, B)
    return B, a, b, F


def test_pcg_2d_N32_T4_vs_oracle():
    """2D, N = 32, T = 4, tol 1e-10 (the small benchmark configuration)."""
    from paper_2004_13961_amd.solver import Problem, Factor, pcg_solve
    from paper_2004_13961_amd.workload import family_nodal
    cfg = synth.WORKLOADS["2d_N32_T4"]
    B, a_o, b_o, F_o = _config_oracle(cfg)
    st, _ = _oracle_factor(2, cfg.N, a_o, b_o, cfg.T, cfg.T)
    mv = lambda v: gk.matvec_sumfact(2, cfg.N, a_o, b_o, v, B)
    x_o, k_o, _ = opcg.pcg(mv, st.apply, F_o, cfg.tol)
    a_g, b_g, f_g, _ = family_nodal(2, cfg.N, cfg.J, cfg.seed)
    P = Problem(2, cfg.N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    Fg = P.load_vector(_dev(f_g).reshape(-1))
    assert_entrywise(_host(Fg), F_o, 1e-13, label="load vector")
    M = Factor(P, cfg.T)
    x, info = pcg_solve(P, M, Fg, rtol=cfg.tol)
    xg = _host(x)
    assert info["relres_true"] <= cfg.tol
    assert abs(info["iters"] - k_o) <= 1
    res = np.linalg.norm(F_o - mv(xg)) / np.linalg.norm(F_o)
    assert res <= cfg.tol * 1.5
    assert np.linalg.norm(xg - x_o) <= 1e-8 * np.linalg.norm(x_o)


@pytest.mark.parametrize("inner", ["f32", "bf16"])
def test_pcg_mixed_2d_N32_T4(inner):
    from paper_2004_13961_amd.solver import Problem, Factor, pcg_solve
    from paper_2004_13961_amd.workload import family_nodal
    cfg = synth.WORKLOADS["2d_N32_T4"]
    B, a_o, b_o, F_o = _config_oracle(cfg)
    a_g, b_g, f_g, _ = family_nodal(2, cfg.N, cfg.J, cfg.seed)
    P = Problem(2, cfg.N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    Fg = P.load_vector(_dev(f_g).reshape(-1))
    M = Factor(P, cfg.T, store="f32")
    x, info = pcg_solve(P, M, Fg, rtol=cfg.tol, inner=inner)
    xg = _host(x)
    mv = lambda v: gk.matvec_sumfact(2, cfg.N, a_o, b_o, v, B)
    res = np.linalg.norm(F_o - mv(xg)) / np.linalg.norm(F_o)
    assert info["relres_true"] <= cfg.tol
    assert res <= cfg.tol * 1.5
    xd = np.linalg.solve(gk.dense_operator(2, cfg.N, a_o, b_o), F_o)
    print("mixed %s: outer %d, inner iters %d, err vs FP64 oracle %.2e" % (
        inner, info["outer"], info["iters"], np.linalg.norm(xg - xd) / np.linalg.norm(xd)))


@pytest.mark.parametrize("d,N,T", [(3, 12, 6), (3, 16, 4), (2, 96, 8)])
def test_pcg_other_shapes(d, N, T):
    from paper_2004_13961_amd.solver import Problem, Factor, pcg_solve
    from paper_2004_13961_amd.workload import family_nodal
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, 6, 2)
    a_o = owl.coefficient_a(c, B.x)
    b_o = owl.coefficient_b(d, B.x)
    F_o = gk.load_vector(d, N, owl.rhs_f(c, B.x), B)
    a_g, b_g, f_g, _ = family_nodal(d, N, 6, 2)
    P = Problem(d, N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    Fg = P.load_vector(_dev(f_g).reshape(-1))
    M = Factor(P, T)
    x, info = pcg_solve(P, M, Fg, rtol=1e-10)
    xg = _host(x)
    res = np.linalg.norm(F_o - gk.matvec_sumfact(d, N, a_o, b_o, xg, B)) / np.linalg.norm(F_o)
    assert res <= 1.5e-10
    assert info["iters"] < 40


def test_error_paths():
    from paper_2004_13961_amd.lgpcg import LgpError
    from paper_2004_13961_amd.solver import Problem, Factor, pcg_solve
    N = 10
    a, b = _random_problem(2, N, 1)
    bad = a.copy()
    bad[3, 4] = -1.0
    with pytest.raises(LgpError) as e:
        Problem(2, N, _dev(bad).reshape(-1), _dev(b).reshape(-1))
    assert e.value.status == 3
    # b may dip below zero as far as the coercivity bound -(d pi^2/4) min a
    Problem(2, N, _dev(a).reshape(-1), _dev(np.full_like(b, -0.5)).reshape(-1))
    with pytest.raises(LgpError) as e:
        Problem(2, N, _dev(a).reshape(-1), _dev(np.full_like(b, -10.0)).reshape(-1))
    assert e.value.status == 3
    P = Problem(2, N, _dev(a).reshape(-1), _dev(b).reshape(-1))
    M = Factor(P, 2)
    F = _dev(synth.random_vector((N - 1) ** 2, 3))
    x, info = pcg_solve(P, M, F, rtol=1e-14, max_iter=1, raise_on_error=False)
    assert info["status"] == "LGP_E_NOCONV"


@pytest.mark.parametrize("N,T,lo,hi", [(40, 10, 257, 512), (48, 14, 513, 10 ** 6)])
def test_wide_2d_stencils(N, T, lo, hi):
    """2D truncations T = 10 and T = 14 on fields of full degree: 304 and 536
    lower offsets, beyond the two-lines-per-wave substitution (<= 256), so
    the banded substitution (<= 512) and the line-per-workgroup one run;
    factor (generic kernel) and both substitutions entry by entry against
    the oracle's Alg. 2-4."""
    from paper_2004_13961_amd.solver import Factor, Problem
    print("case wide 2D N=%d T=%d" % (N, T), flush=True)
    a, b = _random_problem(2, N, 60 + T)
    st, offs = _oracle_factor(2, N, a, b, T, T)
    P = Problem(2, N, _dev(a).reshape(-1), _dev(b).reshape(-1))
    M = Factor(P, T)
    desc = M.describe()
    nlo = desc["n_lower"]
    assert lo <= nlo <= hi, nlo
    assert [tuple(o[:2]) for o in desc["offsets"]] == [tuple(o) for o in offs]
    Lo, Do = st.H[:, :nlo], st.H[:, nlo]
    assert np.max(np.abs(_host(desc["L"]) - Lo)) <= 1e-12 * max(1.0, np.max(np.abs(Lo)))
    assert np.max(np.abs(_host(desc["D"]) - Do)) <= 1e-12 * np.max(np.abs(Do))
    r = synth.random_vector((N - 1) ** 2, 61 + T)
    assert_entrywise(_host(M.forward(_dev(r))), st.forward(r), 1e-12, label="forward")
    assert_entrywise(_host(M.backward(_dev(r))), st.backward(r), 1e-12, label="backward")
    assert_entrywise(_host(M.apply(_dev(r))), st.apply(r), 1e-12, label="apply")


@pytest.mark.parametrize("inner", ["f32", "bf16"])
def test_pcg_mixed_3d_N16_T4(inner):
    """3D mixed precision: FP32 / BF16 inner PCG (FP32 factor copy) inside
    FP64 refinement. Judged by the oracle's own FP64 true residual; the error
    against the oracle's FP64 PCG solution is printed per result."""
    from paper_2004_13961_amd.solver import Problem, Factor, pcg_solve
    from paper_2004_13961_amd.workload import family_nodal
    d, N, T, seed, tol = 3, 16, 4, 2, 1e-10
    print("case mixed 3D N=%d T=%d inner=%s" % (N, T, inner), flush=True)
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, 6, seed)
    a_o, b_o = owl.coefficient_a(c, B.x), owl.coefficient_b(d, B.x)
    F_o = gk.load_vector(d, N, owl.rhs_f(c, B.x), B)
    mv = lambda v: gk.matvec_sumfact(d, N, a_o, b_o, v, B)
    st, _ = _oracle_factor(d, N, a_o, b_o, T, T)
    x_o, _, _ = opcg.pcg(mv, st.apply, F_o, 1e-13)
    a_g, b_g, f_g, _ = family_nodal(d, N, 6, seed)
    P = Problem(d, N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    Fg = P.load_vector(_dev(f_g).reshape(-1))
    M = Factor(P, T, store="f32")
    x, info = pcg_solve(P, M, Fg, rtol=tol, inner=inner)
    xg = _host(x)
    res = np.linalg.norm(F_o - mv(xg)) / np.linalg.norm(F_o)
    print("mixed 3D %s: outer %d, inner iters %d, oracle relres %.2e, err vs FP64 oracle %.2e" % (
        inner, info["outer"], info["iters"], res, np.linalg.norm(xg - x_o) / np.linalg.norm(x_o)))
    assert info["relres_true"] <= tol
    assert res <= 1.5 * tol


@pytest.mark.parametrize("where,value", [("F", np.nan), ("F", np.inf), ("x0", np.nan)])
def test_non_finite_inputs_rejected(where, value):
    """A NaN or an infinity in F or in the initial guess is rejected with
    LGP_E_ARG before any iteration (the stop rule could never be met)."""
    from paper_2004_13961_amd.solver import Problem, Factor, pcg_solve
    N = 10
    a, b = _random_problem(2, N, 1)
    P = Problem(2, N, _dev(a).reshape(-1), _dev(b).reshape(-1))
    M = Factor(P, 2)
    F = synth.random_vector((N - 1) ** 2, 3)
    x0 = np.zeros_like(F)
    (F if where == "F" else x0)[7] = value
    x, info = pcg_solve(P, M, _dev(F), x=_dev(x0), rtol=1e-10, raise_on_error=False)
    assert info["status"] == "LGP_E_ARG", info


@pytest.mark.parametrize("ring_planes", [0, 12, 10])
def test_3d_factor_window(ring_planes, monkeypatch):
    """3D factor through an FP64 window of recent rows: with the window cut
    down to 12 and 10 of the 15 z-planes (LGP_RING_PLANES) the factorisation
    runs as 2 and 6 launches that reuse the window's slots; L, D and both
    substitutions still match the oracle's Alg. 2-4 entry by entry."""
    from paper_2004_13961_amd.solver import Factor, Problem
    from paper_2004_13961_amd.workload import family_nodal
    d, N, T, seed = 3, 16, 4, 3
    print("case 3d window N=%d T=%d ring_planes=%d" % (N, T, ring_planes), flush=True)
    if ring_planes:
        monkeypatch.setenv("LGP_RING_PLANES", str(ring_planes))
    B = gk.Basis(N)
    c = synth.coefficient_draws(d, 6, seed)
    a_o, b_o = owl.coefficient_a(c, B.x), owl.coefficient_b(d, B.x)
    st, offs = _oracle_factor(d, N, a_o, b_o, T, T)
    a_g, b_g, _, _ = family_nodal(d, N, 6, seed, with_rhs=False)
    P = Problem(d, N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    M = Factor(P, T, store="f32")
    desc = M.describe()
    assert desc["layout"] == 1 and desc["factor_kernel"] == 3
    nlo = desc["n_lower"]
    Lo, Do = st.H[:, :nlo], st.H[:, nlo]
    assert np.max(np.abs(_host(desc["L"]) - Lo)) <= 1e-12 * max(1.0, np.max(np.abs(Lo)))
    assert np.max(np.abs(_host(desc["D"]) - Do)) <= 1e-12 * np.max(np.abs(Do))
    r = synth.random_vector((N - 1) ** d, 77)
    assert_entrywise(_host(M.forward(_dev(r))), st.forward(r), 1e-12, label="forward")
    assert_entrywise(_host(M.backward(_dev(r))), st.backward(r), 1e-12, label="backward")


def test_3d_fp32_only_factor():
    """store = FP32 only (d = 3): the mixed solves give bit for bit what the
    FP64+FP32 factor gives (same FP64 factorisation, same FP32 rounding of
    it), and an FP64 solve with it is refused (LGP_E_UNSUPPORTED)."""
    from paper_2004_13961_amd.solver import Factor, Problem, pcg_solve
    from paper_2004_13961_amd.workload import family_nodal
    d, N, T, seed = 3, 14, 4, 2
    a_g, b_g, f_g, _ = family_nodal(d, N, 6, seed)
    P = Problem(d, N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    Fg = P.load_vector(_dev(f_g).reshape(-1))
    M_both = Factor(P, T, store="f32")
    M_only = Factor(P, T, store="f32only")
    assert M_only.describe()["L"] is None
    assert M_only.buf.numel() < M_both.buf.numel()
    for inner in ("f32", "bf16"):
        x1, i1 = pcg_solve(P, M_both, Fg, rtol=1e-10, inner=inner)
        x2, i2 = pcg_solve(P, M_only, Fg, rtol=1e-10, inner=inner)
        assert i1["iters"] == i2["iters"] and i1["outer"] == i2["outer"]
        assert torch.equal(x1, x2)
        assert i2["relres_true"] <= 1e-10
    x, info = pcg_solve(P, M_only, Fg, rtol=1e-10, raise_on_error=False)
    assert info["status"] == "LGP_E_UNSUPPORTED"


@pytest.mark.parametrize("d,N,T,ring_planes", [(3, 16, 4, 10), (3, 18, 6, 0), (2, 40, 8, 0)])
def test_factor_bitwise_repeatable(d, N, T, ring_planes, monkeypatch):
    """The factorisation gives the same bits on every run: a step whose
    neighbour row is not yet written is formed again with the operations of
    the first attempt, in the same order, so which steps waited (a matter of
    timing) does not show in L or D (3D through six window launches, 3D with
    4-row chunks, 2D)."""
    from paper_2004_13961_amd.solver import Factor, Problem
    from paper_2004_13961_amd.workload import family_nodal
    print("case repeatable d=%d N=%d T=%d ring_planes=%d" % (d, N, T, ring_planes), flush=True)
    if ring_planes:
        monkeypatch.setenv("LGP_RING_PLANES", str(ring_planes))
    a_g, b_g, _, _ = family_nodal(d, N, 6, 4, with_rhs=False)
    P = Problem(d, N, _dev(a_g).reshape(-1), _dev(b_g).reshape(-1))
    runs = []
    for rep in range(3):
        M = Factor(P, T, T)
        desc = M.describe()
        runs.append((desc["L"].clone(), desc["D"].clone(), desc["factor_kernel"]))
        del M, desc
    torch.cuda.synchronize()
    assert runs[0][2] == (3 if d == 3 else 2)
    for L, D, _ in runs[1:]:
        assert torch.equal(L, runs[0][0]) and torch.equal(D, runs[0][1])
