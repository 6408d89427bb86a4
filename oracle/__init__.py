"""Plain FP64 CPU oracle of the low-rank DST Poisson solver with Cross-DEIM.

TEST INFRASTRUCTURE ONLY. Only the test-suite (tests/), the smoke entry point and
the benchmark's CPU-baseline leg may import, call or run anything in this package.
The GPU library never calls it, shares no code, headers, tables or helpers with it,
and this package imports nothing from the GPU library.

Contents (each function names the passage of the paper it follows):
    crossdeim.eigenvalues      Section 3, eigenpairs of T
    crossdeim.dst1             Section 3 / 3.2, orthonormal DST-I, DST(DST(I)) = I
    crossdeim.spectral_factors Section 3.2, F^ = DST(U_F) S_F DST(V_F)^T
    crossdeim.columns / rows   Section 3.1 eq. g_for_p, fibers of W^
    crossdeim.scross           Algorithm 1 (stabilized cross approximation)
    crossdeim.leverage_scores  Algorithm 3 (statistical leverage scores)
    crossdeim.select           Algorithm 4, index-set update (deterministic reading)
    crossdeim.solve            Algorithm 4 (Cross-DEIM) inside the Section 3.2 solver
    crossdeim.lr_norm          Frobenius norm of a sum of factored terms (stopping test)
    dense.dense_solve          Section 3.1 full-rank DST solver (small n only)
    dense.laplacian_apply      Section 3, eq. matrix_poisson, T W + W T^T
"""
from . import crossdeim, dense  # noqa: F401
