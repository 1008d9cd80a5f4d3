"""CPU oracle for the pressure-Poisson solve.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use this package to check the GPU library; the library itself never
imports it, and this package never imports the library.

Contents
--------
direct      FP64 O(N*M) direct sum of Appendix A, eq. greenSum (C + OpenMP).
closed      closed-form and quadrature solutions used to pin the direct sum.
tree_ref    plain reference quadtree: Morton keys, stable target sort, cell
            ranges and the dual-tree interaction lists (bit-exact reference).
fmm_ref     plain FP64 expansion operators (P2M, M2M, M2L, L2L, L2P) and a slow
            FMM built from them, for per-pass checks.
"""
