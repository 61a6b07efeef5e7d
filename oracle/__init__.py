"""CPU FP64 oracle for randomized (augmented) block-CG.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code with the GPU library (no kernels, headers,
helpers, tables or constant generators); the two meet only through the seeded
inputs of the ``synth`` package and through their outputs.

Every routine is plain NumPy/SciPy in float64, written for readability, not
speed, and cites the passage of the paper (arXiv 2501.18717, "Preconditioning
without a preconditioner using randomized block Krylov subspace methods") it
follows.

Modules
-------
block_cg    block Krylov definitions, block-Lanczos with full
            reorthogonalisation, block-CG for one or many shifts, block-Lanczos
            square root (Sec. 1.1, Sec. 3, Sec. 3.2 eq. bcg_alg, Sec. 5 def.
            blansq).
krylov      single-vector CG, Nystrom approximation, deflation preconditioner
            and preconditioned CG by their optimality definitions (Sec. 2).
quadrature  conformal-map quadrature for the square-root integral (Sec. 1
            eq. sqrt_rational) and the elliptic-integral facts used in the
            proof of Thm. lansq.
truth       dense direct references (Cholesky, eigendecomposition, SVD).

Parity status: every function is pinned by a CPU test except where its
docstring says "parity unpinned".
"""
from . import block_cg, krylov, quadrature, truth  # noqa: F401
