"""Plain FP64 CPU oracle of Nystrom-preconditioned image reconstruction.

TEST INFRASTRUCTURE ONLY.  This package is what the HIP implementation is
checked against; it is imported only by the test suite, by the smoke check of
the build entry point and by the CPU-baseline leg of the benchmark.  It shares
no code with the HIP path: operators are written as their plain definitions,
the randomized Nystrom approximation follows Alg. 1 step by step with library
Cholesky / triangular solve / SVD, the preconditioner is eq. (11) written out,
and the solvers follow Alg. 3, the dual of eqs. (21)-(29) and Thm. 1.

Modules: operators (A, A^T, W, W^T, L, L^T), nystrom (Alg. 1, P, P^{-1},
power method), prox (weighted proximal maps), solver (problems, WAPG, cost).
Every function here is pinned by `-m "not gpu"` tests to closed forms,
invariants or brute force; none is marked "parity unpinned".
"""
from . import operators, nystrom, prox, solver  # noqa: F401
