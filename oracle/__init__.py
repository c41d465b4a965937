"""Plain, slow FP64 CPU oracle for sgn(gamma5 Dw(mu)) x.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP library; both sides
draw their seeded inputs from ``latgen`` alone.

Contents, each following the paper (Bloch & Heybrock, "A nested Krylov
subspace method for the overlap operator", PoS LATTICE2009):

* ``wilson``   -- gamma5*Dw(mu) with the Hasenfratz-Karsch chemical potential
                  (Sec. 1, the operator in Eq. (1)); explicit-loop and
                  vectorised versions, dense assembly.
* ``dense``    -- the exact sign through the spectral definition, Eq. (2),
                  with sgn(z) = sgn(Re z) for complex eigenvalues (Sec. 1);
                  an independent Schur route for cross-checks.
* ``krylov``   -- Hermitian Lanczos and two-sided (biorthogonal) Lanczos
                  (Sec. 2), building V_k and the tridiagonal Ritz matrix H_k.
* ``rh``       -- the Roberts-Higham iteration, Eq. (4).
* ``nested``   -- the non-nested approximation, Eq. (3) with Eq. (4), and the
                  nested approximation, Eq. (5), with the preconditioning step
                  H_k -> H_k + H_k^{-1} of Eq. (6); the convergence estimate.
* ``deflation``-- exact treatment of m critical eigenvalues (Sec. 2): the
                  exact part R_m sgn(Lambda_m) L_m^dag x plus the Krylov
                  approximation on the projected source; dense critical
                  eigenpairs for small lattices.
* ``overlap``  -- Dov(mu) = 1 + gamma5 sgn(gamma5 Dw(mu)) (Eq. (1)), its
                  adjoint, and CG on the normal equations (CGNR) to solve
                  Dov y = b.
* ``freefield``-- closed form of the free-field (U = 1) operator in momentum
                  space, an exact reference at any volume.

Pins: every function is checked by ``tests/test_oracle_*.py`` against
something other than itself (closed forms, library routines taking a
different route, algebraic identities, brute force on tiny lattices).
``nested.convergence_estimate`` (the paper defines no estimator) is pinned at
mu = 0, where the outer basis is orthonormal, between the true errors against
the exact sign; on the two-sided coefficients (mu != 0) it is a heuristic.
"""
