"""Oracle for the preconditioned Legendre-Galerkin PCG solver (arXiv 2004.13961).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, FP64 CPU statement of
what the solver computes, written from the paper so that a reader can check it
against the text by eye. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it. The GPU library never calls it,
links it or shares code with it.

Modules
    legendre   Legendre recurrence, derivative relation, Gauss nodes, DLTs (Sec. 2)
    galerkin   compact basis, G-NI operator (dense / sum-factorised / the
               paper's four-step Legendre route), load vector (Sec. 3, 4.3)
    precond    truncated Legendre series p_T, 1D band factors, stencil pattern,
               preconditioner M (Sec. 4.1, Sec. 4.2 Kronecker form)
    ilu        ILU(0), forward and backward substitution (Alg. 2-4), dense
               and stencil (plain C, oracle/c/ilu_stencil.c) forms
    pcg        PCG (Alg. 1) and plain CG
    workload   evaluation of the benchmark coefficient family and the
               manufactured right-hand side at the oracle's own nodes

Pinned by tests/test_oracle_*.py. Functions without such a pin say so in
their docstring ("parity unpinned").
"""
