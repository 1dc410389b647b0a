"""Writes matvec_ext_2d_N1024.txt: sampled entries of K u for the 2D,
N = 1024 benchmark problem (coefficients of the benchmark family, seed 1,
J = 12; u = synth.random_vector(n, 79)), computed by the oracle's
extended-precision sum factorisation. Calls only the oracle and the shared
seeded input generators. Takes a few minutes:

    python tests/golden/make_matvec_ext.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import galerkin as gk  # noqa: E402
from oracle import workload as owl  # noqa: E402

N, J, SEED, USEED, SAMPLES = 1024, 12, 1, 79, 4096


def main():
    B = gk.Basis(N)
    c = synth.coefficient_draws(2, J, SEED)
    a, b = owl.coefficient_a(c, B.x), owl.coefficient_b(2, B.x)
    n = (N - 1) ** 2
    u = synth.random_vector(n, USEED)
    y = gk.matvec_sumfact_ext(2, N, a, b, u, B)
    y64 = gk.matvec_sumfact(2, N, a, b, u, B)
    rows = np.unique(np.concatenate([[0, n - 1, N - 2, n - (N - 1), n // 2],
                                     np.random.default_rng(SEED).integers(0, n, SAMPLES)]))
    path = os.path.join(HERE, "matvec_ext_2d_N1024.txt")
    with open(path, "w") as fh:
        fh.write("# K u at sampled rows, 2D N=%d, benchmark family J=%d seed=%d, u = synth.random_vector(n, %d)\n"
                 % (N, J, SEED, USEED))
        fh.write("# oracle.galerkin.matvec_sumfact_ext (extended precision), written by make_matvec_ext.py\n")
        fh.write("# norm2 %.17e\n# norminf %.17e\n# fp64_oracle_rel_err_norm2 %.3e\n"
                 % (np.linalg.norm(y), np.max(np.abs(y)), np.linalg.norm(y64 - y) / np.linalg.norm(y)))
        for r in rows:
            fh.write("%d %.17e\n" % (r, y[r]))
    print("wrote", path, len(rows), "rows")


if __name__ == "__main__":
    main()
