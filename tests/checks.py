"""Entry-by-entry comparison of GPU results with the oracle.

Every entry i must satisfy |got_i - ref_i| <= rtol * s_i, where s_i is the
magnitude of the terms that make up entry i when it is known (products and
load vectors: the same sum-factorised expansion with every table, field and
input replaced by its absolute value, the standard bound of a rounded sum),
else the largest reference entry. The 2-norm of the difference is checked as
well, against the 2-norm of the same scale.
"""
import copy

import numpy as np

from oracle import galerkin as gk


def _abs_basis(B):
    Ba = copy.copy(B)
    Ba.Phi = np.abs(B.Phi)
    Ba.D = np.abs(B.D)
    return Ba


def matvec_magnitude(d, N, a, b, u, basis=None):
    """Entry i: the sum of the absolute values of the terms of (K u)_i in the
    sum-factorised expansion."""
    B = basis if basis is not None else gk.Basis(N)
    aa = [np.abs(x) for x in a] if isinstance(a, (list, tuple)) else np.abs(a)
    return gk.matvec_sumfact(d, N, aa, np.abs(b), np.abs(u), _abs_basis(B))


def load_magnitude(d, N, f, basis=None):
    """Entry k: sum over the nodes of |W f psi_k|."""
    B = basis if basis is not None else gk.Basis(N)
    return gk.load_vector(d, N, np.abs(f), _abs_basis(B))


def assert_entrywise(got, ref, rtol, scale=None, label=""):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    assert got.shape == ref.shape, (label, got.shape, ref.shape)
    if ref.size == 0:
        return 0.0
    if scale is None:
        s = np.full(ref.shape, max(np.max(np.abs(ref)), np.finfo(float).tiny))
    else:
        s = np.maximum(np.abs(np.asarray(scale, dtype=np.float64).reshape(-1)), np.finfo(float).tiny)
    err = np.abs(got - ref)
    ratio = err / s
    i = int(np.argmax(ratio))
    worst = float(ratio[i])
    assert np.all(np.isfinite(got)), "%s: non-finite entries" % label
    assert worst <= rtol, "%s: entry %d off by %.3e (scale %.3e, ratio %.2e > %.1e)" % (
        label, i, err[i], s[i], worst, rtol)
    assert np.linalg.norm(got - ref) <= rtol * np.linalg.norm(s), "%s: 2-norm" % label
    return worst
