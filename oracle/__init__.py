"""Plain FP64 CPU oracle for ADMM on the homogeneous self-dual embedding.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or call anything in this package.
The GPU library shares no code with it: the two meet only in the seeded
draws of ``datagen``.

Modules (each function cites the passage of the paper it follows):

* ``cones``     -- projections onto the zero, nonnegative, second-order, PSD
                   (scaled svec) and exponential cones and their duals
                   (Sect. 6.1 cone list; Moreau decomposition, Sect. 3.2).
* ``scaling``   -- data equilibration D, E, sigma, rho (Sect. 5).
* ``linsys``    -- the subspace projection (I+Q)^{-1} w by block elimination
                   and Sherman-Morrison-Woodbury (Sect. 4.1), with an exact
                   (dense Cholesky) and an indirect (CG) mode.
* ``admm``      -- the iteration (e-SCS) with over-relaxation and
                   approximate projection (Sect. 3.2-3.3), termination
                   (Sect. 3.5, scaled form Sect. 5), outputs and
                   certificates (Sect. 2.3), warm start (Sect. 4.2), and the
                   five-sequence ADMM (e-SCS-naive) used as a cross-check.
* ``instances`` -- the random feasible program of Sect. 6 (random cone
                   programs) built from a ``datagen`` draw, plus infeasible
                   and unbounded constructions.
* ``mlp``       -- NumPy reference of the warm-start network (forward,
                   backward, Adam).
"""
