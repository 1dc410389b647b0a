"""Python objects over the C ABI: Problem, Factor and pcg_solve.

Device buffers are torch uint8 tensors sized by the library's queries; the
stream is torch's current stream. Tensors passed in must be contiguous CUDA
tensors of the documented dtype and length.
"""
from __future__ import annotations

import ctypes

import torch

from . import lgpcg
from .lgpcg import DTYPES, check, lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, numel: int, name: str):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == numel):
        raise ValueError("%s must be a contiguous CUDA %s tensor with %d elements" % (name, dtype, numel))


class Problem:
    """The operator K = A + B for nodal coefficients a, b on the (N+1)^d
    Legendre-Gauss grid (x fastest). a_nodes holds one field ((N+1)^d values)
    or, for the anisotropic form of Example 4, d fields one after the other
    (a_1 for x first)."""

    def __init__(self, d: int, N: int, a_nodes: torch.Tensor, b_nodes: torch.Tensor):
        L = lib()
        self.d, self.N = d, N
        self.n1, self.q = N - 1, N + 1
        self.n = self.n1 ** d
        self.nq = self.q ** d
        self.aniso = a_nodes.numel() == d * self.nq and d > 1
        _need(a_nodes, torch.float64, d * self.nq if self.aniso else self.nq, "a_nodes")
        _need(b_nodes, torch.float64, self.nq, "b_nodes")
        nbytes = L.lgp_problem_bytes(d, N)
        if nbytes == 0:
            raise lgpcg.LgpError(1, "lgp_problem_bytes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        build = L.lgp_build_problem_diag if self.aniso else L.lgp_build_problem
        check(build(d, N, _ptr(a_nodes), _ptr(b_nodes), _ptr(self.buf), nbytes, _stream(), ctypes.byref(h)),
              "lgp_build_problem")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lgpcg._lib is not None:
            lgpcg._lib.lgp_destroy_problem(h)
            self.handle = None

    def matvec(self, u: torch.Tensor, y: torch.Tensor = None, prec: str = "f64") -> torch.Tensor:
        dt = torch.float64 if prec == "f64" else torch.float32
        _need(u, dt, self.n, "u")
        if y is None:
            y = torch.empty_like(u)
        _need(y, dt, self.n, "y")
        check(lib().lgp_matvec(self.handle, _ptr(u), _ptr(y), DTYPES[prec], _stream()), "lgp_matvec")
        return y

    def load_vector(self, f_nodes: torch.Tensor, F: torch.Tensor = None) -> torch.Tensor:
        _need(f_nodes, torch.float64, self.nq, "f_nodes")
        if F is None:
            F = torch.empty(self.n, dtype=torch.float64, device="cuda")
        check(lib().lgp_load_vector(self.handle, _ptr(f_nodes), _ptr(F), _stream()), "lgp_load_vector")
        return F


class Factor:
    """ILU(0) factors of the preconditioner M (truncations Ta for a, Tb for b;
    Ta may be a sequence of d per-direction truncations t_1j, Example 4)."""

    def __init__(self, problem: Problem, Ta, Tb: int = None, store: str = "f64"):
        L = lib()
        if isinstance(Ta, (list, tuple)):
            if Tb is None:
                raise ValueError("Tb is required with per-direction Ta")
            Tdir = (ctypes.c_int * 3)(*(list(Ta) + [0] * (3 - len(Ta))))
        else:
            Tb = Ta if Tb is None else Tb
            Tdir = (ctypes.c_int * 3)(Ta, Ta, Ta)
        self.problem = problem
        self.Ta, self.Tb = Ta, Tb
        nbytes = L.lgp_factor_bytes_dir(problem.handle, Tdir, Tb, DTYPES[store])
        if nbytes == 0:
            raise lgpcg.LgpError(1, "lgp_factor_bytes_dir")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        check(L.lgp_factor_M_dir(problem.handle, Tdir, Tb, DTYPES[store], _ptr(self.buf), nbytes, _stream(),
                                 ctypes.byref(h)), "lgp_factor_M_dir")
        self.handle = h

    @classmethod
    def constant(cls, problem: Problem):
        """The constant-coefficient preconditioner of PCG-I (a, b replaced by
        their means), inverted exactly; apply() and pcg_solve() accept it."""
        L = lib()
        self = cls.__new__(cls)
        self.problem = problem
        self.Ta = self.Tb = 0
        nbytes = L.lgp_factor_const_bytes(problem.handle)
        if nbytes == 0:
            raise lgpcg.LgpError(1, "lgp_factor_const_bytes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        check(L.lgp_factor_const(problem.handle, _ptr(self.buf), nbytes, _stream(), ctypes.byref(h)),
              "lgp_factor_const")
        self.handle = h
        return self

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lgpcg._lib is not None:
            lgpcg._lib.lgp_destroy_factor(h)
            self.handle = None

    def _vec(self, v, name):
        _need(v, torch.float64, self.problem.n, name)

    def apply(self, r: torch.Tensor, z: torch.Tensor = None) -> torch.Tensor:
        self._vec(r, "r")
        z = torch.empty_like(r) if z is None else z
        check(lib().lgp_precond_apply(self.handle, _ptr(r), _ptr(z), _stream()), "lgp_precond_apply")
        return z

    def forward(self, r: torch.Tensor, y: torch.Tensor = None) -> torch.Tensor:
        self._vec(r, "r")
        y = torch.empty_like(r) if y is None else y
        check(lib().lgp_ilu_forward(self.handle, _ptr(r), _ptr(y), _stream()), "lgp_ilu_forward")
        return y

    def backward(self, y: torch.Tensor, z: torch.Tensor = None) -> torch.Tensor:
        self._vec(y, "y")
        z = torch.empty_like(y) if z is None else z
        check(lib().lgp_ilu_backward(self.handle, _ptr(y), _ptr(z), _stream()), "lgp_ilu_backward")
        return z

    def forward32(self, r: torch.Tensor, y: torch.Tensor = None) -> torch.Tensor:
        """y = L^{-1} r in FP32 on the factor's FP32 copy."""
        _need(r, torch.float32, self.problem.n, "r")
        y = torch.empty_like(r) if y is None else y
        check(lib().lgp_ilu_forward_f32(self.handle, _ptr(r), _ptr(y), _stream()), "lgp_ilu_forward_f32")
        return y

    def backward32(self, y: torch.Tensor, z: torch.Tensor = None) -> torch.Tensor:
        """z = U^{-1} y in FP32 on the factor's FP32 copy."""
        _need(y, torch.float32, self.problem.n, "y")
        z = torch.empty_like(y) if z is None else z
        check(lib().lgp_ilu_backward_f32(self.handle, _ptr(y), _ptr(z), _stream()), "lgp_ilu_backward_f32")
        return z

    def describe(self):
        """Pattern (offsets, n_lower) and views of the factor storage."""
        dsc = lgpcg.FactorDesc()
        check(lib().lgp_factor_describe(self.handle, ctypes.byref(dsc)), "lgp_factor_describe")
        offs = [(dsc.offsets[3 * k], dsc.offsets[3 * k + 1], dsc.offsets[3 * k + 2]) for k in range(dsc.noff)]
        n, nlo, ld = dsc.n, dsc.n_lower, dsc.ld
        base = self.buf.data_ptr()
        Dv = self.buf[dsc.D - base: dsc.D - base + n * 8].view(torch.float64)
        iv = self.buf[dsc.invD - base: dsc.invD - base + n * 8].view(torch.float64)
        if dsc.layout == 1:
            # offset-major: L[k * ld + i] = L(i, i + offset_k); an (n, n_lower) strided view
            Lv = None
            if dsc.L:
                Lv = self.buf[dsc.L - base: dsc.L - base + nlo * ld * 8].view(torch.float64).view(nlo, ld)[:, :n].t()
        else:
            rows = self.buf[dsc.L - base: dsc.L - base + n * ld * 8].view(torch.float64).view(n, ld)
            Lv = rows[:, :nlo]
        return dict(offsets=offs, n_lower=nlo, ld=ld, L=Lv, invD=iv, D=Dv,
                    levels=dsc.levels, n=n, factor_kernel_ms=dsc.factor_kernel_ms,
                    factor_kernel=dsc.factor_kernel, layout=dsc.layout,
                    factor_launches=dsc.factor_launches, factor_waits=dsc.factor_waits)


def pcg_solve(problem: Problem, factor: Factor, F: torch.Tensor, x: torch.Tensor = None, rtol: float = 1e-10,
              max_iter: int = 2000, inner: str = "f64", inner_rtol: float = 0.0, max_outer: int = 60,
              check_every: int = 4, ws: torch.Tensor = None, raise_on_error: bool = True):
    """Solve K x = F by PCG (Alg. 1) with the one-step ILU(0) preconditioner.
    Returns (x, info dict). `x` is used as the initial guess (zeros if None)."""
    L = lib()
    _need(F, torch.float64, problem.n, "F")
    if x is None:
        x = torch.zeros_like(F)
    _need(x, torch.float64, problem.n, "x")
    nbytes = L.lgp_solve_workspace_bytes(problem.handle, DTYPES[inner])
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    o = lgpcg.SolveOpts(rtol, max_iter, DTYPES[inner], inner_rtol, max_outer, check_every)
    info = lgpcg.SolveInfo()
    st = L.lgp_pcg_solve(problem.handle, factor.handle, _ptr(F), _ptr(x), ctypes.byref(o), _ptr(ws),
                         ws.numel(), _stream(), ctypes.byref(info))
    out = dict(iters=info.iters, outer=info.outer, relres_true=info.relres_true,
               relres_recursive=info.relres_recursive, status=lgpcg.STATUS.get(st, st))
    if st != 0 and raise_on_error:
        raise lgpcg.LgpError(st, "lgp_pcg_solve")
    return x, out


class Batch:
    """Same-shape requests solved together (lgp_batch_*): add() admits a
    request into a free slot, step(k) runs k PCG iterations of every running
    request (one launch per kernel for all of them, the iteration replayed
    as a HIP graph), info() reads a slot's result, remove() frees it. Work
    runs on the batch's own stream (a graph cannot be captured on the null
    stream), which waits for the caller's stream at every add."""

    def __init__(self, shape: Problem, slots: int, stream: torch.cuda.Stream = None):
        L = lib()
        self.shape = shape
        self.slots = slots
        self.stream = stream if stream is not None else torch.cuda.Stream()
        nbytes = L.lgp_batch_workspace_bytes(shape.handle, slots)
        if nbytes == 0:
            raise lgpcg.LgpError(1, "lgp_batch_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        check(L.lgp_batch_create(shape.handle, slots, _ptr(self.ws), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "lgp_batch_create")
        self.handle = h
        self.keep = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lgpcg._lib is not None:
            lgpcg._lib.lgp_batch_destroy(h)
            self.handle = None

    def add(self, problem: Problem, factor: Factor, F: torch.Tensor, x: torch.Tensor = None,
            rtol: float = 1e-10, max_iter: int = 2000, check: bool = True):
        _need(F, torch.float64, problem.n, "F")
        if x is None:
            x = torch.zeros_like(F)
        _need(x, torch.float64, problem.n, "x")
        self.stream.wait_stream(torch.cuda.current_stream())
        o = lgpcg.SolveOpts(rtol, max_iter, lgpcg.LGP_F64, 0.0, 60, 4)
        slot = ctypes.c_int(-1)
        st = lib().lgp_batch_add(self.handle, problem.handle, factor.handle, _ptr(F), _ptr(x), ctypes.byref(o),
                                 ctypes.byref(slot))
        if check:
            lgpcg.check(st, "lgp_batch_add")
        elif st != 0:
            return None, x, lgpcg.STATUS.get(st, st)
        self.keep[slot.value] = (problem, factor, F, x)
        return slot.value, x, "LGP_OK"

    def step(self, iters: int = 4) -> int:
        running = ctypes.c_int(0)
        lgpcg.check(lib().lgp_batch_step(self.handle, iters, ctypes.byref(running)), "lgp_batch_step")
        return running.value

    def info(self, slot: int):
        inf = lgpcg.SolveInfo()
        fin = ctypes.c_int(0)
        lgpcg.check(lib().lgp_batch_info(self.handle, slot, ctypes.byref(inf), ctypes.byref(fin)), "lgp_batch_info")
        return dict(iters=inf.iters, outer=inf.outer, relres_true=inf.relres_true,
                    relres_recursive=inf.relres_recursive, status=lgpcg.STATUS.get(inf.status, inf.status)), bool(fin.value)

    def remove(self, slot: int):
        lgpcg.check(lib().lgp_batch_remove(self.handle, slot), "lgp_batch_remove")
        self.keep.pop(slot, None)


def pcg_solve_batched(problems, factors, Fs, xs=None, rtol: float = 1e-10, max_iter: int = 2000,
                      check_every: int = 4, stream: torch.cuda.Stream = None):
    """lgp_pcg_solve_batched: solve count same-shape requests together.
    Returns (xs, infos)."""
    L = lib()
    count = len(problems)
    if xs is None:
        xs = [torch.zeros_like(F) for F in Fs]
    for P, F, x in zip(problems, Fs, xs):
        _need(F, torch.float64, P.n, "F")
        _need(x, torch.float64, P.n, "x")
    stream = stream if stream is not None else torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    nbytes = L.lgp_batch_workspace_bytes(problems[0].handle, count)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    vp = ctypes.c_void_p
    arr = lambda vals: (vp * count)(*vals)
    o = lgpcg.SolveOpts(rtol, max_iter, lgpcg.LGP_F64, 0.0, 60, check_every)
    infos = (lgpcg.SolveInfo * count)()
    st = L.lgp_pcg_solve_batched(count, arr([P.handle.value for P in problems]),
                                 arr([M.handle.value for M in factors]), arr([F.data_ptr() for F in Fs]),
                                 arr([x.data_ptr() for x in xs]), ctypes.byref(o), _ptr(ws), nbytes,
                                 vp(stream.cuda_stream), infos)
    out = [dict(iters=i.iters, outer=i.outer, relres_true=i.relres_true, relres_recursive=i.relres_recursive,
                status=lgpcg.STATUS.get(i.status, i.status)) for i in infos]
    if st != 0:
        raise lgpcg.LgpError(st, "lgp_pcg_solve_batched")
    torch.cuda.current_stream().wait_stream(stream)
    return xs, out


class FastTransforms:
    """Fast discrete Legendre transforms at a problem's nodes and the product
    of Sec. 4.3 through them (lgp_dlt_*). The problem must outlive it."""

    def __init__(self, problem: Problem):
        L = lib()
        self.problem = problem
        nbytes = L.lgp_dlt_bytes(problem.handle)
        if nbytes == 0:
            raise lgpcg.LgpError(8, "lgp_dlt_bytes")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        check(L.lgp_dlt_create(problem.handle, _ptr(self.buf), nbytes, _stream(), ctypes.byref(h)), "lgp_dlt_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lgpcg._lib is not None:
            lgpcg._lib.lgp_dlt_destroy(h)
            self.handle = None

    def blocks(self) -> int:
        return lib().lgp_dlt_blocks(self.handle)

    def lines(self, v: torch.Tensor, forward: bool = False, out: torch.Tensor = None) -> torch.Tensor:
        """BDLT (forward=False) or FDLT of each row of v (count x (N+1))."""
        q = self.problem.q
        count = v.numel() // q
        _need(v, torch.float64, count * q, "v")
        if out is None:
            out = torch.empty_like(v)
        _need(out, torch.float64, count * q, "out")
        check(lib().lgp_dlt_lines(self.handle, 1 if forward else 0, count, _ptr(v), _ptr(out), _stream()),
              "lgp_dlt_lines")
        return out

    def matvec(self, u: torch.Tensor, y: torch.Tensor = None) -> torch.Tensor:
        n = self.problem.n
        _need(u, torch.float64, n, "u")
        if y is None:
            y = torch.empty_like(u)
        check(lib().lgp_matvec_fast(self.handle, _ptr(u), _ptr(y), _stream()), "lgp_matvec_fast")
        return y
