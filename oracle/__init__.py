"""Plain FP64 CPU oracle for the stochastic-Galerkin (SG) KKT solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code with the HIP library (no kernels,
headers, tables or constant generators); the only inputs both sides see come
from the seeded generators in ``sg_inputs``.

Every function cites the passage of Li, Onwunta & Sousedik, "Stochastic
Galerkin method and hierarchical preconditioning for PDE-constrained
optimization" (arXiv 2512.23804) that it follows.  Arithmetic is float64
throughout; the method's exact answer (the solution of the discrete KKT system,
Section 2.1 eq. (stoch-system) and Section 3 eq. (KKT:stoch-time-dependent)) is
computed by sparse direct factorisation.

Modules
  basis     multi-index set and Legendre triple products   (Section 2.1)
  fem       Q1 assembly on the unit square                  (Section 2.1, eq. gPC-A)
  kkt       SG matrices, KKT systems, right-hand sides      (Section 2.1, Section 3)
  precond   Chebyshev mass solve, geometric multigrid, hGS, block preconditioner
            (Section 2.2-2.3, Algorithm 1, Algorithm 5, Section 3.1)
  fgmres    restarted flexible GMRES                         (Section 5)
"""
