"""ILU(0) and the one-step preconditioner application (Sec. 4.2, Alg. 2-4).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The one-step method solves M z = r approximately by z = U^{-1} L^{-1} r with
the ILU(0) factors (reading: one step from z_0 = 0; M itself is never
applied). Alg. 2 overwrites H(i,j) by L(i,j) for i > j and by U(i,j)
otherwise; only pairs in NZ(M) are touched. Alg. 4 is read with the inner
loop over j = i+1..n.

Dense forms (tiny n) take a boolean NZ mask; the stencil forms call the plain
C file oracle/c/ilu_stencil.c through ctypes (built by build_c()).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "c", "ilu_stencil.c")
_CLIB = os.path.join(_HERE, "c", "libilu_stencil.so")


# ------------------------------------------------------------ dense --------
def ilu0_dense(M: np.ndarray, nz: np.ndarray):
    """Alg. 2 on a dense copy. Returns (L unit lower, U upper)."""
    H = np.array(M, dtype=np.float64, copy=True)
    n = H.shape[0]
    for i in range(1, n):
        for k in range(i):
            if not nz[i, k]:
                continue
            H[i, k] = H[i, k] / H[k, k]
            js = np.nonzero(nz[i, k + 1:])[0] + k + 1
            H[i, js] -= H[i, k] * H[k, js]
    L = np.tril(H, -1) + np.eye(n)
    U = np.triu(H)
    # entries outside NZ were never touched; they keep M's values, which are
    # zero there by definition of NZ
    L[~nz & ~np.eye(n, dtype=bool)] = 0.0
    U[~nz] = 0.0
    return L, U


def forward_dense(L: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Alg. 3: y(1) = r(1); y(i) = r(i) - sum_{j<i} L(i,j) y(j)."""
    n = len(r)
    y = np.zeros(n)
    y[0] = r[0]
    for i in range(1, n):
        y[i] = r[i] - L[i, :i] @ y[:i]
    return y


def backward_dense(U: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Alg. 4: z(n) = y(n)/U(n,n); z(i) = (y(i) - sum_{j>i} U(i,j) z(j))/U(i,i)."""
    n = len(y)
    z = np.zeros(n)
    z[n - 1] = y[n - 1] / U[n - 1, n - 1]
    for i in range(n - 2, -1, -1):
        z[i] = (y[i] - U[i, i + 1:] @ z[i + 1:]) / U[i, i]
    return z


# ---------------------------------------------------------- stencil --------
def build_c(force: bool = False) -> str:
    """Compile oracle/c/ilu_stencil.c with gcc into a shared object."""
    if force or not os.path.exists(_CLIB) or \
            os.path.getmtime(_CLIB) < os.path.getmtime(_CSRC):
        tmp = _CLIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC",
                               _CSRC, "-o", tmp])
        os.replace(tmp, _CLIB)
    return _CLIB


_lib = None


def _clib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_c())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        _lib.ilu0_stencil.restype = ctypes.c_int64
        _lib.ilu0_stencil.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, ctypes.c_int64]
        for f in (_lib.forward_stencil, _lib.backward_stencil):
            f.restype = None
            f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, dp]
        _lib.forward_stencil_rows.restype = None
        _lib.forward_stencil_rows.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, dp,
                                              ctypes.c_int64]
    return _lib


def _offs_array(offsets):
    arr = np.zeros((len(offsets), 3), dtype=np.int32)
    for i, o in enumerate(offsets):
        arr[i, : len(o)] = o
    return np.ascontiguousarray(arr)


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


class StencilILU:
    """ILU(0) of a matrix stored as rows over a fixed offset list.

    H has shape (n, noff): H[row, o] = M(row, row + offsets[o]). After
    factor(), H holds L (strict lower offsets) and U (diagonal and upper)."""

    def __init__(self, d: int, n1: int, offsets, H: np.ndarray):
        self.d, self.n1 = d, n1
        self.offsets = list(offsets)
        self.off = _offs_array(self.offsets)
        self.H = np.ascontiguousarray(H, dtype=np.float64)
        self.diag = self.offsets.index(tuple([0] * d))

    def factor(self, nrows: int = -1):
        """Alg. 2 over all rows, or over the first `nrows` rows only (a prefix
        is the same computation as in the full factorisation; used to time a
        bounded sample)."""
        rc = _clib().ilu0_stencil(self.d, self.n1, len(self.offsets),
                                  _p(self.off, ctypes.c_int), _p(self.H, ctypes.c_double), nrows)
        if rc != 0:
            raise ZeroDivisionError("zero pivot in ILU(0) at row %d" % (rc - 1))
        return self

    def forward(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        y = np.zeros_like(r)
        _clib().forward_stencil(self.d, self.n1, len(self.offsets),
                                _p(self.off, ctypes.c_int), _p(self.H, ctypes.c_double),
                                _p(r, ctypes.c_double), _p(y, ctypes.c_double))
        return y

    def forward_prefix(self, r, nrows: int):
        """Alg. 3 over the first `nrows` rows only (rows read earlier rows
        only; used to time a bounded sample on a prefix of the rows)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        y = np.zeros_like(r)
        _clib().forward_stencil_rows(self.d, self.n1, len(self.offsets),
                                     _p(self.off, ctypes.c_int), _p(self.H, ctypes.c_double),
                                     _p(r, ctypes.c_double), _p(y, ctypes.c_double), nrows)
        return y

    def backward(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        z = np.zeros_like(y)
        _clib().backward_stencil(self.d, self.n1, len(self.offsets),
                                 _p(self.off, ctypes.c_int), _p(self.H, ctypes.c_double),
                                 _p(y, ctypes.c_double), _p(z, ctypes.c_double))
        return z

    def apply(self, r):
        """One-step method: z = U^{-1} L^{-1} r."""
        return self.backward(self.forward(r))


def stencil_rows_from_dense(M: np.ndarray, d: int, n1: int, offsets) -> np.ndarray:
    """H[row, o] = M(row, row + offset) (0 where the column leaves the grid)."""
    n = n1 ** d
    H = np.zeros((n, len(offsets)))
    for row in range(n):
        c = [(row // n1 ** k) % n1 for k in range(d)]
        for o, off in enumerate(offsets):
            col = [c[k] + off[k] for k in range(d)]
            if any(v < 0 or v >= n1 for v in col):
                continue
            ci = sum(col[k] * n1 ** k for k in range(d))
            H[row, o] = M[row, ci]
    return H
