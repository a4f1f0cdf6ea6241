"""Plain FP64 CPU oracle of the Closest Point Method multigrid solver (Chen & Macdonald).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The GPU library never calls it and
shares no code with it; the only common module is ``workloads`` (seeded problem
descriptions, no arithmetic of the method).

Layout (each function cites the passage of the paper it follows):

* ``geometry``  closest-point functions of circle / sphere / torus (Sec. 2.1)
* ``band``      computational band, interpolation stencils, operators E, L, N and the
                closest-point restriction / prolongation matrices (Sec. 3.1, Sec. 4.3)
* ``vcycle``    Ruuth-Merriman Jacobi smoothing, residual, V-cycle (Algorithm 4.1),
                coarsest direct solve, solve loop
* ``direct``    assembled matrix A = cI - M of eq. (3.3) and sparse direct solves
* ``mixed``     FP32-inner / FP64-outer iterative refinement of the same V-cycle
* ``standard``  the V-cycle with standard relaxation: Jacobi on A, residual f - A(E u) (Sec. 4.5)
* ``varcoef``   variable diffusion coefficients: flux-form L~ and its V-cycle
* ``mlp``       reference forward / backward of the learned local smoother network
* ``errors``    error evaluation on the surface by cubic interpolation (Sec. 3.4)

Parity status: every function is pinned by a test against values the paper prints
(Table 3.1, Table 4.1), closed forms, invariants or brute force, except the per-cycle
V-cycle iterates (the paper's convergence plots carry no numbers), which are pinned
only through their fixed point (brute-force sparse solve) and the h-independence of
the contraction factor; the learned-smoother training outcome is "parity unpinned".
"""
