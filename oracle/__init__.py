"""Plain FP64 CPU oracle for the implicit reaction-diffusion step solved by G-prox PDHG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the tests,
the smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
code with the GPU path: no kernels, no helpers, no tables, no constants.

What it computes follows Liu, Liu, Osher and Li, "A first-order computational
algorithm for reaction-diffusion type equations via primal-dual hybrid gradient
method" (arXiv 2305.03945):

* ``grid``       -- the discrete Laplacians of Sec. 2.1 (periodic) and Remark 1
                    (Neumann), the 13-point biharmonic ``Lap Lap`` of Sec. 3.2, and
                    the 7-point Laplacian of 3-D grids.
* ``spectral``   -- Laplacian eigenvalues and the preconditioner solve ``G^-1 w``
                    by FFT (periodic) or DCT-II (Neumann) in 2-D and 3-D, Sec. 2.1
                    ("Choosing the matrix G", "Application of FFT") and Remark 1.
* ``equations``  -- ``F(U)`` and ``grad F(U)^T P`` for Allen-Cahn (eq. 12),
                    Cahn-Hilliard (eq. 29), the Schnakenberg system (Sec. 3.4.1),
                    the functionalized Cahn-Hilliard equation of Sec. 3.3 and the
                    linear heat / biharmonic steps.
* ``adaptive``   -- the step-size rule of Sec. 2.2 and a trajectory advanced with it.
* ``pdhg``       -- Algorithm 1: the G-prox linearized PDHG time step.
* ``newton``     -- the plain definition of the step's result: the root of
                    ``F(U) = 0`` by damped Newton with a direct Jacobian solve.
* ``prox``       -- the pointwise implicit reaction step (proximal map of the
                    reaction potential), a predictor for ``U_0`` (Sec. 2.1,
                    "Initial guess").
* ``theory``     -- Theorem 1 / Appendix A spectral radius and Remark 2 closed forms.
* ``invariants`` -- discrete energy (eq. 27), mass, maximum principle.

Every function is FP64 and written for readability, not speed.
"""
