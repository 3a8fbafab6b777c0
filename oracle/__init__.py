"""CPU oracle for the hp space-time multigrid of Margenberg, Bause and Munch,
"An hp Multigrid Approach for Tensor-Product Space-Time Finite Element
Discretizations of the Stokes Equations" (arXiv 2502.09159).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
restatement of what the method computes.  It exists to check the HIP library;
only the test-suite, the smoke entry point and the CPU-baseline leg of the
benchmark may import it.  The product path never does, and it shares no code,
tables or constants with the HIP library: both sides only receive the same
seeded input arrays.

Modules (each function cites the passage of the paper it follows):

* ``elements``  - Gauss/Gauss-Lobatto/Radau rules, Lagrange and Legendre bases,
                  temporal matrices K, M, C (Sec. 3.1, Eq. (GF), (BasYk), (DefKMC)).
* ``mesh``      - structured quad/hex meshes, optional vertex deformation.
* ``assembly``  - element and global matrices M_h, A_h, B_h, M_h^p (Eq. (DefMAB)).
* ``spacetime`` - the slab operator of Eq. (GloSys), literal CSR and factored.
* ``hierarchy`` - level lists (Alg. 2, Alg. 3, App. C) and smoother sizes.
* ``transfer``  - canonical h/p prolongation and restriction (App. A).
* ``vanka``     - the cell Vanka smoother, Eq. (vanka0)/(vanka).
* ``coarse``    - bordered direct solve on the coarsest level.
* ``mg``        - the hp V-cycle, Alg. 1 with Alg. 4-7.
* ``fgmres``    - flexible GMRES (right preconditioned, CGS2).
* ``errors``    - space-time error norms for manufactured solutions.
* ``learned``   - the small convolutional correction network (forward and
                  backward), written independently of the GPU kernels.
"""
