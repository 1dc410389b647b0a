"""The C-ABI library loads on the CPU and exports every symbol of
include/lgpcg.h; host-only entry points behave (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import legendre as olg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "lgpcg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(lgp_[A-Za-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_header_function():
    from paper_2004_13961_amd import lgpcg
    L = lgpcg.lib()
    names = _header_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(lgpcg.EXPORTS)


def test_gauss_nodes_match_oracle():
    from paper_2004_13961_amd import lgpcg
    for N in (1, 2, 7, 32, 127, 255, 1024):
        x, w = lgpcg.gauss_legendre(N)
        xo, wo = olg.gauss_legendre(N)
        assert np.max(np.abs(x - xo)) < 2e-16 * 4
        assert np.max(np.abs(w - wo)) < 1e-15 * max(1.0, np.max(wo)) * 4


def test_size_queries_and_argument_errors():
    from paper_2004_13961_amd import lgpcg
    L = lgpcg.lib()
    assert L.lgp_problem_bytes(2, 32) > 0
    assert L.lgp_problem_bytes(3, 16) > 0
    assert L.lgp_problem_bytes(1, 32) > 0
    assert L.lgp_problem_bytes(1, 10240) > 0
    assert L.lgp_problem_bytes(0, 32) == 0
    assert L.lgp_problem_bytes(4, 8) == 0
    assert L.lgp_problem_bytes(2, 1) == 0
    assert L.lgp_problem_bytes(2, 4097) == 0
    assert L.lgp_problem_bytes(1, 65537) == 0
    assert L.lgp_factor_bytes(None, 4, 4, 0) == 0
    h = ctypes.c_void_p()
    assert L.lgp_build_problem(4, 10, None, None, None, 0, None, ctypes.byref(h)) == 1
    assert L.lgp_status_str(3) == b"coefficient violates a > 0 at a node, or b below the coercivity bound"
    assert L.lgp_version() >= 100
