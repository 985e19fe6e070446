"""The semilinear diffusion-reaction experiment: backward-forward Euler in
time, a preconditioned conjugate gradient solve per step on the Kronecker-sum
matrix, an ADI-type Kronecker-product preconditioner (Sec. 3.4 and Sec. 4.5),
in float64.

Test infrastructure only (see the package docstring).

* ``tridiag_inverse`` -- the inverse of a tridiagonal matrix, assembled dense
  and inverted by LAPACK. Pins: the closed form of (I - tau A)^{-1} for the
  Dirichlet second difference A through its sine eigenbasis; P P^{-1} = I for
  general diagonally dominant tridiagonals.
* ``pcg``             -- the textbook preconditioned conjugate gradient method
  (Hestenes and Stiefel; Saad, Iterative Methods for Sparse Linear Systems,
  Algorithm 9.1) with the relative-residual stopping test ||r|| <= tol ||b||.
  Pins: the dense solution of the assembled system; one iteration with the
  exact inverse as preconditioner; termination within the number of distinct
  eigenvalues on a diagonal Kronecker sum.
* ``semilinear_*``    -- the experiment: u_t = Laplacian(u) + 1/(1 + u^2) + Phi
  on [0,1]^d with homogeneous Dirichlet ends and exact solution
  u = e^t u0, u0 = prod_mu x_mu (1 - x_mu). Pins: the grid function e^t u0
  solves the semi-discrete system exactly (the second difference is exact on
  quadratics); the final relative error and the average iteration counts the
  paper prints for n = (40, 44, 48), tau = 0.01, t* = 1.

Readings where the paper is silent: the grid holds the n_mu interior points
x_i = i h_mu, h_mu = 1/(n_mu + 1); the stopping tolerance is 1e-5 (relative
residual), the value with which this oracle reproduces the printed average
of two preconditioned iterations per step; every solve starts from the
previous step's solution.
"""
from __future__ import annotations

import numpy as np

from .tucker import kronsumv, tucker


def tridiag(lower, diag, upper):
    """Dense tridiagonal matrix: P[i, i-1] = lower[i] (i >= 1), P[i, i] =
    diag[i], P[i, i+1] = upper[i] (i <= n-2); lower[0] and upper[n-1] are
    not used."""
    diag = np.asarray(diag, dtype=np.float64)
    n = diag.shape[0]
    P = np.diag(diag)
    if n > 1:
        P += np.diag(np.asarray(lower, dtype=np.float64)[1:], k=-1)
        P += np.diag(np.asarray(upper, dtype=np.float64)[:n - 1], k=1)
    return P


def tridiag_inverse(lower, diag, upper):
    """P^{-1} for the tridiagonal P of :func:`tridiag` (the ADI factor
    inverses (I - tau A_mu)^{-1} of Sec. 3.4), by LAPACK on the dense matrix."""
    return np.linalg.inv(tridiag(lower, diag, upper))


def pcg(apply_A, b, x0, apply_Minv=None, tol=1e-5, maxit=1000):
    """Preconditioned conjugate gradients for A x = b, A symmetric positive
    definite, preconditioner action z = Minv(r) (identity if None).

    From x0: r = b - A x0. Stop when ||r|| <= tol ||b|| (also before the
    first iteration). Each iteration: z = Minv(r); rho = <r, z>;
    p = z (first iteration) or z + (rho / rho_prev) p; q = A p;
    alpha = rho / <p, q>; x += alpha p; r -= alpha q.
    Returns (x, iterations, ||r|| / ||b||)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_A(x)
    nb = np.sqrt(np.sum(b * b))
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0
    res = np.sqrt(np.sum(r * r)) / nb
    it = 0
    p = None
    rho_prev = None
    while res > tol and it < maxit:
        z = r if apply_Minv is None else apply_Minv(r)
        rho = np.sum(r * z)
        p = z.copy() if p is None else z + (rho / rho_prev) * p
        q = apply_A(p)
        alpha = rho / np.sum(p * q)
        x = x + alpha * p
        r = r - alpha * q
        rho_prev = rho
        it += 1
        res = np.sqrt(np.sum(r * r)) / nb
    return x, it, res


def semilinear_grid(n):
    """Interior points x_i = i h, i = 1..n, h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    return np.arange(1, n + 1) * h, h


def semilinear_u0(xs):
    """u0 = prod_mu x_mu (1 - x_mu) on the tensor grid (axis mu-1 = x_mu)."""
    q = np.ones(())
    for x in xs:
        q = np.multiply.outer(q, x * (1.0 - x))
    return q


def semilinear_laplacian_u0(xs):
    """The exact Laplacian of u0: sum over mu of -2 prod_{nu != mu} q_nu."""
    d = len(xs)
    out = 0.0
    for mu in range(d):
        term = np.ones(())
        for nu, x in enumerate(xs):
            term = np.multiply.outer(term, np.full_like(x, -2.0) if nu == mu else x * (1.0 - x))
        out = out + term
    return out


def semilinear_phi(t, xs):
    """Phi(t, x) = e^t u0 - e^t Laplacian(u0) - 1/(1 + e^{2t} u0^2): the source
    that makes e^t u0 the exact solution."""
    u0 = semilinear_u0(xs)
    return np.exp(t) * (u0 - semilinear_laplacian_u0(xs)) - 1.0 / (1.0 + np.exp(2 * t) * u0 ** 2)


def semilinear_rhs(u, t, tau, xs):
    """Right-hand side of one backward-forward Euler step:
    b = u + tau (1/(1 + u^2) + Phi(t, x))."""
    return u + tau * (1.0 / (1.0 + u * u) + semilinear_phi(t, xs))


def semilinear_factors(ns, tau):
    """(As, Ms, Pinvs): the second differences A_mu, the Kronecker-sum terms
    M_mu = I/d - tau A_mu (M = M_d (+) ... (+) M_1 = I - tau (A_d (+) ... (+)
    A_1)) and the ADI factor inverses (I - tau A_mu)^{-1} (Sec. 3.4)."""
    d = len(ns)
    As, Ms, Pinvs = [], [], []
    for n in ns:
        _, h = semilinear_grid(n)
        A = (-2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)) / (h * h)
        As.append(A)
        Ms.append(np.eye(n) / d - tau * A)
        off = np.full(n, -tau / (h * h))
        Pinvs.append(tridiag_inverse(off, np.full(n, 1.0 + 2.0 * tau / (h * h)), off))
    return As, Ms, Pinvs


def semilinear_imex(ns, tau=0.01, steps=100, tol=1e-5, maxit=1000, precondition=True,
                    u=None, t0=0.0):
    """Run `steps` backward-forward Euler steps M u_{k+1} = u_k + tau f(t_k, u_k)
    from u (default u0) at t0, each solved by :func:`pcg` from u_k with the
    Kronecker-sum action of M (Sec. 2) and, if `precondition`, the inverse
    ADI preconditioner V x_1 P_1^{-1} ... x_d P_d^{-1} (Sec. 3.4).
    Returns (u, iterations per step)."""
    xs = [semilinear_grid(n)[0] for n in ns]
    _, Ms, Pinvs = semilinear_factors(ns, tau)
    u = semilinear_u0(xs) if u is None else np.array(u, dtype=np.float64, copy=True)
    A = lambda v: kronsumv(v, Ms)
    Minv = (lambda v: tucker(v, Pinvs)) if precondition else None
    its = []
    for k in range(steps):
        b = semilinear_rhs(u, t0 + k * tau, tau, xs)
        u, it, _ = pcg(A, b, u, Minv, tol, maxit)
        its.append(it)
    return u, its
