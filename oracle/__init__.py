"""Plain FP64 CPU oracle for the eigCG hot path (TEST INFRASTRUCTURE ONLY).

This package is the correctness reference for the HIP library.  It is slow on
purpose: every function follows the paper's definitions or algorithm boxes in
their own order, in complex128 NumPy, with no blocking, fusion or reordering.

Only the test-suite, the package's smoke check and the benchmark's
``cpu_baseline`` leg may import it.  The product path never calls it and
shares no code with it; the only common module is ``synthetic`` (seeded input
generation, which contains none of the method's arithmetic).

Paper: A. Stathopoulos and K. Orginos, "Computing and deflating eigenvalues
while solving multiple right hand side linear systems with an application to
Quantum Chromodynamics" (arXiv:0707.0131).

Modules:

* ``dirac``        - Wilson-Dirac operator M, its adjoint and A = M^H M
                     (Section 1; operator written out in the module).
* ``cg``           - CG, left box of Figure 3.1 (P = I, or an SPD
                     preconditioner given as P^{-1}).
* ``eigcg``        - eigCG(nev, m), right box of Figure 3.1, also in the
                     preconditioned form of Section 3 (V = P^{-1} R).
* ``initcg``       - init-CG Galerkin guess, eq. (2.1), and the restarted
                     init-CG of Section 5.3.
* ``incremental``  - Incremental eigCG outer loop (Section 4 algorithm box).
* ``dense``        - dense matrices of the operator for tiny lattices.
* ``schur``        - odd-even (Schur complement) preconditioned operator on
                     the even sites, with the maps to and from the full
                     system (the operator of the paper's lattice runs).
* ``bicgstab``     - BiCGSTAB on gamma5 M (or M) with a deflated initial
                     guess from the bank (Section 1's use of the eigCG
                     vectors for a nonsymmetric solver).
* ``spectral``     - the bank used as a spectral preconditioner (Section
                     2.1's alternative to init-CG; Section 4's example).
* ``restart_model`` - a dynamic init-CG restart threshold from the bank's
                     Ritz values and residual norms (the open choice at the
                     end of Section 5.3), as a stated cost model.

Parity status: every function here is pinned by a test under ``tests/``
(closed forms, invariants, dense linear algebra or brute force); nothing is
"parity unpinned".
"""

from . import dirac, cg, eigcg, initcg, incremental, dense, schur, bicgstab, spectral  # noqa: F401
