"""Gradient of a scalar loss through the Tucker operator, in float64.

Test infrastructure only (see the package docstring).

The paper does not treat derivatives; they follow from its Lemma relating the
Tucker operator to the Kronecker product (Sec. 2) and the Kronecker transpose
rule (Appendix A, property 5). With S = T x_1 L_1 ... x_d L_d and a cotangent
G = dloss/dS:

* vec(S) = (L_d (x) ... (x) L_1) vec(T), so dloss/dvec(T) is
  (L_d^T (x) ... (x) L_1^T) vec(G), i.e. dT = G x_1 L_1^T ... x_d L_d^T.
* By order independence S = Z_mu x_mu L_mu with Z_mu = T multiplied by every
  factor except L_mu; then S^(mu) = L_mu Z_mu^(mu) and
  dL_mu = G^(mu) (Z_mu^(mu))^T.

Pins: the Kronecker matrix (tiny sizes) for dT, central finite differences for
both, and the adjoint identity <G, dS> = <dT, dT_dir> + sum <dL, dL_dir>.
"""
from __future__ import annotations

import numpy as np

from .tucker import mumat, mump, tucker


def tucker_vjp(T, Ls, G):
    """Return (dT, [dL_1, ..., dL_d]) for S = tucker(T, Ls) and cotangent G."""
    T = np.asarray(T, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    d = T.ndim
    dT = tucker(G, [np.asarray(L, float).T for L in Ls])
    dLs = []
    for mu in range(1, d + 1):
        Z = T
        for nu in range(1, d + 1):
            if nu != mu:
                Z = mump(Z, Ls[nu - 1], nu)
        dLs.append(mumat(G, mu) @ mumat(Z, mu).T)
    return dT, dLs


def factor_gradient_column(T, Ls, G, mu, j):
    """Column j (0-based) of dL_mu for S = tucker(T, Ls) and cotangent G.

    With Z_mu = T multiplied by every factor except L_mu, dL_mu = G^(mu)
    (Z_mu^(mu))^T, so its column j only involves the mu-fibers' entry j of
    Z_mu, i.e. the slice of T at j_mu = j multiplied by the other factors
    (each mu-mode product acts on the other modes only, Sec. 2). Cost: about
    1/m_mu of a full Tucker operator; used to sample gradients of tensors too
    large for :func:`tucker_vjp`. Pinned against central differences and
    against :func:`tucker_vjp`."""
    T = np.asarray(T, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    d = T.ndim
    Z = np.take(T, [j], axis=mu - 1)
    for nu in range(1, d + 1):
        if nu != mu:
            Z = mump(Z, Ls[nu - 1], nu)
    return (mumat(G, mu) @ mumat(Z, mu).T)[:, 0]


def central_fd_directional(f, x, v, h):
    """(f(x + h v) - f(x - h v)) / (2h): the central difference of the scalar
    function f at x along direction v."""
    return (f(x + h * v) - f(x - h * v)) / (2.0 * h)
