"""CPU FP64 oracle for the high-order continuous-FE multigrid of Sundar, Stadler and Biros,
"Comparison of Multigrid Algorithms for High-order Continuous Finite Element Discretizations".

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or execute this
package: only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the GPU library (no kernels, headers, tables or helpers); the two meet
only at the seeded input descriptions in ``paper_1402_5938_amd.inputs`` (which hold no
arithmetic of the method) and at plain arrays handed to both.

What it computes, in the paper's own approach (§2.3: a prototype built on sparse assembled
operators), written plainly and without blocking, fusion or reordering:

* ``gll``        GLL nodes/weights, Lagrange derivative and interpolation matrices (§1, §2.3, Fig. 1)
* ``fields``     the domain maps Phi and coefficient families mu (§2.3, §4.1)
* ``fem``        mesh, isoparametric geometry at the GLL quadrature points, the assembled
                 Galerkin stiffness a(phi_i, phi_j) in the factored sparse form B^T G B and as
                 an explicit CSR matrix, its diagonal, the lumped mass and the load vector
                 (§2.1, §2.3)
* ``transfer``   prolongation P_ij = phi_j^{k-1}(p_i) by direct evaluation, restriction P^T
                 (§2.2, Eq. (Pstencil))
* ``relax``      multicolor SSOR, l1-Jacobi and element block-Jacobi smoothers (§3.2, §4.3,
                 §4.4.3) on the assembled interior matrix
* ``mg``         Jacobi and Chebyshev-Jacobi smoothers, the Lanczos/Arnoldi lambda_max
                 estimate, the h-/p-hierarchy, the V-cycle, multigrid as solver and the
                 multigrid-preconditioned CG of Algorithm 1 (§3, §4.2-§4.3)
* ``splitmix``   the SplitMix64 counter-based generator (Steele, Lea and Flood 2014) used for
                 the Lanczos start vector on both sides

Every function is pinned by the ``-m "not gpu"`` tests against closed forms, printed values of
the paper, exactness properties, invariants and dense brute force; none is "parity unpinned".
"""
