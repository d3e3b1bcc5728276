"""CPU FP64 oracle for randomized Nystrom PCG (Frangella, Tropp & Udell).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The library under
``paper_2110_02820_amd`` never imports it and shares no code with it.

Everything here is plain NumPy/SciPy in float64, written from the paper's
definitions and algorithms in their order and notation, with no blocking,
fusion or reordering beyond what a definition states (the RBF operator is
evaluated in row blocks only so that it fits in memory; each block is the
textbook formula).

Pinned parts (tests/test_oracle_*.py):
  operators        -- against scipy.spatial.distance / explicit products
  XtDXOp           -- row-by-row sum of d_i x_i x_i^T, d = 1 reduces to XtXOp,
                      one-hot d gives the rank-one x_k x_k^T
  nystrom          -- Lemma (Nystrom properties), closed form of eq. (nys-unstable),
                      exact recovery for rank(A) <= l
  precond          -- P P^{-1} = I, spectrum of P^{-1}, Woodbury identity
  pcg              -- dense Cholesky solve (LAPACK), scipy.sparse.linalg.cg iterates,
                      iteration counts for rank(A) < l and rank(A) = l,
                      CG iteration bound with the exact condition number
  power            -- power estimate against the exact spectral norm of E
  adaptive         -- the base algorithm when no doubling is allowed, the closed
                      form of the Nystrom approximation on the concatenated test
                      matrix, the first doubling stage whose exact ||E|| meets the
                      tolerance, the l_max cap, Strategy 2's stopping stage, and
                      the theorem's bound on the final sketch size (frequency
                      over seeds)
  columns          -- the column Nystrom formula A(:,S) A(S,S)^{-1} A(S,:), exact
                      recovery of a rank-r matrix from r independent columns,
                      interpolation of A on the sampled rows and columns
  sketch_solve     -- a dense solve of the proxy system (LAPACK), the exact
                      solution when rank(A) <= l, the theorem's bound on the
                      expected relative error (mean over seeds)
  block_pcg        -- scipy cg iterates for one column, the Galerkin property of
                      block CG on the block Krylov space (explicit projection),
                      termination near ceil(n / s) steps (dimension of the block
                      Krylov space), a LAPACK solve
  grad             -- central finite differences of dense solves and a closed form
  philox           -- Random123 known-answer vectors
Parity unpinned: none of the functions above is unpinned; the mixed-precision
forms have no oracle of their own (they are judged by this FP64 oracle's true
residual).
"""
from .operators import DenseOp, XtXOp, XtDXOp, RBFOp, rbf_kernel_block  # noqa: F401
from .nystrom import orthonormalize, matlab_eps, randomized_nystrom, nystrom_factor  # noqa: F401
from .precond import precond_inv_apply, precond_matrix, precond_inv_matrix  # noqa: F401
from .pcg import nystrom_pcg, true_relres, dense_solve  # noqa: F401
from .power import rand_pow_err_est  # noqa: F401
from .adaptive import ada_rand_nystrom, effective_dimension  # noqa: F401
from .columns import column_nystrom, selection_matrix  # noqa: F401
from .sketch_solve import nystrom_sketch_solve  # noqa: F401
from .block_pcg import block_nystrom_pcg  # noqa: F401
from .grad import adjoint_gradients, validation_loss, validation_loss_grads  # noqa: F401
from .philox import philox4x32_10, gaussian_philox  # noqa: F401
