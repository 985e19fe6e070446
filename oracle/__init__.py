"""FP64 CPU oracle for the mu-mode product and the Tucker operator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and its
Python binding) imports, links or calls this package; only the test suite, the
smoke check and the CPU-baseline leg of the benchmark do. It shares no code with
the GPU path: the two sides meet only in the seeded input generators of
``kp_workloads``, which hold none of the method's arithmetic.

Everything here is plain numpy / scipy in float64, written for a reader who
checks it against the paper by eye (Caliari, Cassini, Zivcovich, "A mu-mode BLAS
approach for multidimensional tensor-structured problems"):

* ``tucker``   -- vec, mu-matricization, mu-mode product, Tucker operator,
                  element-wise nested-sum formula, Kronecker product and sum.
* ``factors``  -- the one-dimensional factors of the paper's applications:
                  the exponential of the Dirichlet finite-difference Laplacian
                  (closed form), barycentric Lagrange matrices on Chebyshev
                  nodes, the 5-D Runge function.
* ``semilinear`` -- the semilinear diffusion-reaction experiment: tridiagonal
                  inverses (ADI factors), preconditioned conjugate gradients on
                  the Kronecker-sum matrix, backward-forward Euler steps.
* ``complex_tucker`` -- the Tucker operator over C and its conjugate-transpose
                  form (spectral transforms).
* ``grad``     -- the gradient of a scalar loss through the Tucker operator
                  and a central finite-difference checker.

Pins (what each function is checked against, other than itself) are listed
per function and exercised by the CPU test suite. Parity status:
every function here is pinned; none is "parity unpinned".
"""
from .tucker import (vec, unvec, mumat, mump, tucker, nested, tucker_entry,
                     kron, kronsum, kronsumv)
from .factors import (fd_laplacian_dirichlet, expm_fd_laplacian_dirichlet,
                      dst1_eigenpairs, chebyshev_nodes, chebyshev_weights,
                      lagrange_matrix, runge)
from .grad import tucker_vjp, factor_gradient_column, central_fd_directional
from .complex_tucker import zmump, ztucker, cttucker, dft_matrix
from .semilinear import (tridiag, tridiag_inverse, pcg, semilinear_grid, semilinear_u0,
                         semilinear_laplacian_u0, semilinear_phi, semilinear_rhs,
                         semilinear_factors, semilinear_imex)

__all__ = [
    "vec", "unvec", "mumat", "mump", "tucker", "nested", "tucker_entry",
    "kron", "kronsum", "kronsumv",
    "fd_laplacian_dirichlet", "expm_fd_laplacian_dirichlet", "dst1_eigenpairs",
    "chebyshev_nodes", "chebyshev_weights", "lagrange_matrix", "runge",
    "tucker_vjp", "factor_gradient_column", "central_fd_directional",
    "zmump", "ztucker", "cttucker", "dft_matrix",
    "tridiag", "tridiag_inverse", "pcg", "semilinear_grid", "semilinear_u0",
    "semilinear_laplacian_u0", "semilinear_phi", "semilinear_rhs", "semilinear_factors",
    "semilinear_imex",
]
