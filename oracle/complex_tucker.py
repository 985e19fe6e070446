"""The Tucker operator over the complex field and its conjugate-transpose
form, in complex128.

Test infrastructure only (see the package docstring).

The paper states the mu-mode product and the Tucker operator for complex
tensors and matrices (Sec. 2), and evaluates pseudospectral decompositions
at their own quadrature grid with the conjugate-transposed basis matrices,
C x_1 Psi_1^* ... x_d Psi_d^* (Sec. 3, the remark on direct and inverse
spectral transforms). Pins: element-wise nested sums on tiny tensors, the
Kronecker form, numpy's FFT for Fourier matrices (a different algorithm),
the adjoint identity between the two forms, and the real case.
"""
from __future__ import annotations

import numpy as np


def _c128(x):
    return np.asarray(x, dtype=np.complex128)


def zmump(T, L, mu):
    """S = T x_mu L for complex T and L (L is n x m_mu, mu 1-based): every
    mu-fiber of T is multiplied by L (S^(mu) = L T^(mu))."""
    T = _c128(T)
    L = _c128(L)
    X = np.moveaxis(T, mu - 1, 0)
    shape = X.shape
    Y = L @ X.reshape(shape[0], -1)
    return np.moveaxis(Y.reshape((L.shape[0],) + shape[1:]), 0, mu - 1)


def ztucker(T, Ls):
    """T x_1 L_1 x_2 ... x_d L_d in definition order; None is the identity."""
    S = _c128(T)
    for mu, L in enumerate(Ls, start=1):
        if L is not None:
            S = zmump(S, L, mu)
    return S


def cttucker(T, Ls):
    """T x_1 L_1^* x_2 ... x_d L_d^*, with ^* the conjugate transpose."""
    return ztucker(T, [None if L is None else _c128(L).conj().T for L in Ls])


def dft_matrix(n):
    """The Fourier matrix F[j, k] = exp(-2 pi i j k / n)."""
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)
