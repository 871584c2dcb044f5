"""CPU oracle for the space-time KKT solve -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 reference implementation of what the GPU library computes,
written from the paper (Deng, Cai, Zou, "Two-level space-time domain
decomposition methods for unsteady inverse problems", arXiv:1508.06103):

* ``fem``      -- 1-D/3-D Q1 finite-element matrices and the time matrices
                  (Section 3.1, Appendix A element matrices A, B, E, L, K, D).
* ``kkt``      -- the fully discretised KKT system F_h U = b as a sum of
                  Kronecker products, its right-hand side, a level-by-level
                  application and principal submatrices on space-time boxes
                  (Section 3.2 ordering, Appendix A block structure).
* ``ras``      -- space-time partition/overlap and one-level restricted additive
                  Schwarz with 3x3 point-block ILU(0) subdomain solves
                  (Section 3.2, one-level preconditioner; Section 4 settings).
* ``krylov``   -- right-preconditioned restarted GMRES / flexible GMRES
                  (Section 3.2, Section 4 solver settings).
* ``twolevel`` -- nested coarse space-time mesh, linear interpolation and the
                  multiplicative two-level preconditioner (Section 3.2).
* ``reduced``  -- forward/adjoint time marching, the discrete objective J_h and
                  a reduced-space CG solve (used only to pin the KKT system).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU product path never does.
Where the paper is silent or garbled, each module states the reading it takes.
"""
