"""MI355X (gfx950) mu-mode product and Tucker operator.

Caliari, Cassini, Zivcovich, "A mu-mode BLAS approach for multidimensional
tensor-structured problems": S = T x_mu L and S = T x_1 L_1 ... x_d L_d, in
hand-written HIP kernels behind the C-ABI of include/kp.h (libkp.so), with a
thin torch binding (ops) that only marshals arguments.
"""
from .ops import (mump, tucker, tucker_with_cache, tucker_backward,  # noqa: F401
                  tucker_autograd, TuckerFunction, expm, BatchedTucker, force_tile, kronsum,
                  tridiag_inverse, pcg_kronsum, semilinear_imex, tucker_complex,
                  tucker_noalloc)
from . import tune  # noqa: F401,E402

__all__ = ["mump", "tucker", "tucker_with_cache", "tucker_backward", "tucker_autograd",
           "TuckerFunction", "expm", "BatchedTucker", "force_tile", "kronsum",
           "tridiag_inverse", "pcg_kronsum", "semilinear_imex", "tucker_complex",
           "tucker_noalloc", "tune"]
