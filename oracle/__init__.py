"""Plain, slow, serial FP64 CPU oracle for the KLE-CGC hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.

It shares no code with the GPU path.  Every array is FP64 (complex128 where
the method is complex), every solve is a direct library solve (banded
Cholesky / banded or sparse LU), the discrete Fourier transform over slices is
a dense matrix product, and every function follows one passage of the paper
(arXiv 2510.26180), cited in its docstring.

Modules
  field     closed-form KL of the exponential covariance (input field)
  operator  finite-difference diffusion operator with face coefficients
  prop      fine propagator F, coarse propagator G, serial fine reference
  cgc       alpha-circulant all-at-once system and its diagonalised solve
  parareal  Algorithm 1 (sequential CGC) and Algorithms 2/3 (parallel CGC)
  snapshot  KL expansion of solution snapshots (Section 2.1)
  gpc       Hermite gPC basis and least-squares fit (Section 2.2)
  theory    scalar model problem: stability functions and contraction factors
  mlp       learned initial guess (MLP) forward/backward/Adam in FP64
  guess     random initial guess (counter-based SplitMix64), continuity defect and the
            learned-guess / gPC fallback rule

Parity status: every function is pinned by a closed form, an invariant or a
brute-force computation in tests/test_oracle_*.py.  Where the paper is silent
the reading taken is listed in the module docstring.
"""
