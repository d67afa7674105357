"""CPU FP64 oracle for the symmetric near-field Schur-complement preconditioner.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow, obviously correct
reference that the GPU library is checked against. Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does, and it shares no code with the HIP library.

Stages (each module cites the passage of the paper it follows):

* ``kernel``    scalar Helmholtz Green's function entries (Eq. 5-6 kernel)
* ``tree``      octree decomposition to leaf size (Sec. 2)
* ``partition`` near / far block partition (Eq. 8, Sec. 2, Fig. 1)
* ``aca``       ACA with partial pivoting and SVD re-compression (Eq. 9-10)
* ``hmatrix``   near assembly, far compression and the matvec (Eq. 11)
* ``ordering``  near-field block ordering (Algorithm 1; CM / RCM)
* ``symbolic``  filled pattern of the scaling coefficients (Sec. 3.3)
* ``schur``     symmetric Schur elimination, fill-in compression and the
                preconditioner apply (Eq. 12-24, Sec. 3.2, Sec. 3.4)
* ``gmres``     right-preconditioned GMRES(m) (Eq. 2, Sec. 5)
* ``pipeline``  end to end: h_build, precond_setup, solve

Parity status of each function is stated in its module; functions without a
pin say "parity unpinned".
"""
from . import kernel, tree, partition, aca, hmatrix, ordering, symbolic, schur, gmres, pipeline  # noqa: F401
