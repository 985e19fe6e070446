"""One-dimensional factors used by the paper's applications, in float64.

Test infrastructure only (see the package docstring).

* The exponential of the second-order finite-difference Laplacian with
  homogeneous Dirichlet conditions, the 1-D building block of the exponential
  of a Kronecker sum (Sec. 3.3). It is given in closed form through the
  eigenpairs of tridiag(1, -2, 1), whose eigenvectors are the discrete sine
  basis (DST-I). Pins: scipy's general-purpose matrix exponential, and the
  exact action on eigenvectors.
* Barycentric Lagrange interpolation matrices on Chebyshev nodes (Sec. 4.3,
  multivariate interpolation). Pins: partition of unity, exact reproduction
  of polynomials of degree < m, and the relative errors the paper prints for
  its 5-D Runge example.
"""
from __future__ import annotations

import numpy as np


def fd_laplacian_dirichlet(n, h):
    """tridiag(1, -2, 1) / h^2 of size n: the centred second difference on n
    interior points with homogeneous Dirichlet ends."""
    A = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    return A / (h * h)


def dst1_eigenpairs(n, h):
    """Eigenpairs of tridiag(1, -2, 1)/h^2 (size n).

    Eigenvector k (k = 1..n) has entries q_jk = sqrt(2/(n+1)) sin(j k pi/(n+1))
    and eigenvalue -(4/h^2) sin^2(k pi / (2(n+1))). The eigenvector matrix Q is
    symmetric and orthogonal. Returns (lam, Q) with Q[:, k-1] the k-th vector.
    """
    j = np.arange(1, n + 1)
    Q = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))
    lam = -(4.0 / (h * h)) * np.sin(j * np.pi / (2.0 * (n + 1))) ** 2
    return lam, Q


def expm_fd_laplacian_dirichlet(n, h, tau):
    """exp(tau * tridiag(1,-2,1)/h^2) = Q diag(exp(tau*lam)) Q^T, from the
    eigenpairs of :func:`dst1_eigenpairs`."""
    lam, Q = dst1_eigenpairs(n, h)
    return (Q * np.exp(tau * lam)) @ Q.T


def chebyshev_nodes(m):
    """Chebyshev nodes xi_k = cos((2k-1) pi / (2m)), k = 1..m (Sec. 4.3)."""
    k = np.arange(1, m + 1)
    return np.cos((2 * k - 1) * np.pi / (2.0 * m))


def chebyshev_weights(m):
    """Barycentric weights of the Chebyshev nodes, up to a common factor that
    cancels in the second barycentric form: w_k = (-1)^(k+1) sin((2k-1) pi/(2m))
    (Sec. 4.3)."""
    k = np.arange(1, m + 1)
    return (-1.0) ** (k + 1) * np.sin((2 * k - 1) * np.pi / (2.0 * m))


def lagrange_matrix(m, x, nodes=None, weights=None):
    """Matrix of Lagrange basis values, entry (l, i) = L_i(x_l), with L_i the
    degree-(m-1) Lagrange polynomial on ``nodes`` written in the second
    barycentric form (Sec. 4.3):

        L_i(x) = (w_i / (x - xi_i)) / sum_k (w_k / (x - xi_k)).

    Defaults: Chebyshev nodes and their weights. Where an evaluation point
    coincides with a node the formula is 0/0; the Lagrange property gives the
    value there: row l is the unit vector of that node.
    """
    xi = chebyshev_nodes(m) if nodes is None else np.asarray(nodes, float)
    w = chebyshev_weights(m) if weights is None else np.asarray(weights, float)
    x = np.asarray(x, dtype=np.float64)
    L = np.empty((x.size, xi.size))
    for l, xl in enumerate(x):
        diff = xl - xi
        hit = np.flatnonzero(diff == 0.0)
        if hit.size:
            L[l] = 0.0
            L[l, hit[0]] = 1.0
            continue
        t = w / diff
        L[l] = t / t.sum()
    return L


def runge(*xs):
    """d-variate Runge function 1 / (1 + 16 sum_mu x_mu^2) (Sec. 4.3) on the
    Cartesian grid spanned by the 1-D point sets ``xs`` (ndgrid order: the
    first set varies along the first axis)."""
    acc = np.asarray(xs[0], float) ** 2
    for x in xs[1:]:
        acc = np.add.outer(acc, np.asarray(x, float) ** 2)
    acc *= 16.0
    acc += 1.0
    return np.reciprocal(acc, out=acc)
