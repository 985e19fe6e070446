"""Seeded synthetic inputs for the Tucker-operator workloads.

This module is the only code shared by the GPU path's tests and benchmark and
by the oracle's tests. It draws random numbers and assembles input matrices; it
performs none of the mu-mode / Tucker arithmetic. Everything is generated in
float64 with ``numpy.random.default_rng(seed)``; a consumer casts to its
working precision and (for comparisons) promotes the cast values back to
float64, so input rounding never counts as a kernel error.

Draw order is fixed: the tensor first, then L_1, ..., L_d (for the batched
workload the table of mode sizes is drawn before everything else).

Workloads (the paper draws its test data as standard normal values, Sec. 1
Table 1 and Sec. 4.1; its applications supply structured factors):

* ``small2d``   d=2, 50 x 50 tensor and factors, the 2-D form L1 T L2^T
                (Sec. 1, Table 1 at n=50).
* ``cube200``   d=3, all sizes 200, square standard-normal factors (between
                the n=196 and n=256 points of the paper's d=3 timing sweep).
* ``heat128``   d=3, n=128 per mode; A_mu = tridiag(1,-2,1)/h^2 with h=1/129
                (Dirichlet), tau = 1e-3; tensor standard normal (Sec. 3.3).
* ``interp6d``  d=6, 16^6 standard-normal tensor; factors 24x16 barycentric
                Lagrange matrices from 16 Chebyshev nodes to 24 uniform
                points of [-1, 1] (Sec. 4.3 shape, with d=6).
* ``batch64``   64 tensors of order 4, each mode size uniform in [16, 64],
                square factors with entries N(0,1)/sqrt(n_mu).
* ``runge5d``   d=5 Runge function on m^5 Chebyshev nodes, Lagrange matrices
                to 35 equispaced points (Sec. 4.3, m = 5..45).
* ``codeval``   standard-normal cubes of the paper's timing sweep, d=3
                n = 144..324 and d=6 n = 12..18 (use ``cube(seed, n, d)``).
* ``semilinear`` the semilinear diffusion-reaction experiment (Sec. 4.5):
                grids of n = (40, 44, 48) interior points, the diagonals of
                each second difference, the initial value
                prod_mu x_mu (1 - x_mu), tau = 0.01, 100 steps to t = 1.
"""
from __future__ import annotations

import numpy as np

SEED = 0


def _normal(rng, shape):
    return rng.standard_normal(size=shape)


def small2d(seed=SEED, n=50):
    rng = np.random.default_rng(seed)
    T = _normal(rng, (n, n))
    Ls = [_normal(rng, (n, n)) for _ in range(2)]
    return T, Ls


def cube(seed=SEED, n=200, d=3):
    rng = np.random.default_rng(seed)
    T = _normal(rng, (n,) * d)
    Ls = [_normal(rng, (n, n)) for _ in range(d)]
    return T, Ls


def cube200(seed=SEED):
    return cube(seed, 200, 3)


def random_problem(seed, m_dims, n_dims, scale_by_cols=False):
    """Standard-normal tensor of sizes ``m_dims`` and factors of shapes
    (n_mu, m_mu); with ``scale_by_cols`` the factors are divided by
    sqrt(n_mu) (the batched workload's scaling)."""
    rng = np.random.default_rng(seed)
    T = _normal(rng, tuple(m_dims))
    Ls = []
    for n, m in zip(n_dims, m_dims):
        L = _normal(rng, (n, m))
        if scale_by_cols:
            L = L / np.sqrt(n)
        Ls.append(L)
    return T, Ls


def heat_matrix(n=128):
    """tridiag(1, -2, 1) / h^2 with h = 1/(n+1): the Dirichlet second
    difference on n interior points of [0, 1]."""
    h = 1.0 / (n + 1)
    A = -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)
    return A / (h * h)


def second_difference_diagonals(n):
    """(lower, diag, upper, h) of tridiag(1, -2, 1)/h^2 on n interior points,
    h = 1/(n+1) (lower[0] and upper[n-1] are padding)."""
    h = 1.0 / (n + 1)
    off = np.full(n, 1.0 / (h * h))
    return off, np.full(n, -2.0 / (h * h)), off.copy(), h


def semilinear(ns=(40, 44, 48), tau=0.01, steps=100):
    """Returns (u0, [(lower, diag, upper, h) per axis], tau, steps): the
    initial value prod_mu x_mu (1 - x_mu) on the interior grid x = i h,
    i = 1..n_mu (axis mu-1 = x_mu), and each axis's second difference."""
    diags = [second_difference_diagonals(n) for n in ns]
    u0 = np.ones(())
    for n, (_, _, _, h) in zip(ns, diags):
        x = np.arange(1, n + 1) * h
        u0 = np.multiply.outer(u0, x * (1.0 - x))
    return u0, diags, tau, steps


def spd_matrices(seed, ns, shift=1.0):
    """Symmetric positive definite matrices B B^T / n + shift I, B standard
    normal n x n, one per size in ns (drawn in order)."""
    rng = np.random.default_rng(seed)
    out = []
    for n in ns:
        B = _normal(rng, (n, n))
        out.append(B @ B.T / n + shift * np.eye(n))
    return out


def heat128(seed=SEED, n=128, d=3, tau=1e-3):
    """Returns (V, [A_1..A_d], tau)."""
    rng = np.random.default_rng(seed)
    V = _normal(rng, (n,) * d)
    As = [heat_matrix(n) for _ in range(d)]
    return V, As, tau


def lagrange_chebyshev_to_uniform(m=16, n=24):
    """Entry (l, i): the i-th Lagrange basis polynomial on the m Chebyshev
    nodes cos((2i-1)pi/(2m)) evaluated at the l-th of n equispaced points of
    [-1, 1] (endpoints included), by the second barycentric form with weights
    (-1)^(i+1) sin((2i-1)pi/(2m)). No evaluation point coincides with a node
    for the sizes used here; a coincidence yields the node's unit row."""
    i = np.arange(1, m + 1)
    xi = np.cos((2 * i - 1) * np.pi / (2.0 * m))
    w = (-1.0) ** (i + 1) * np.sin((2 * i - 1) * np.pi / (2.0 * m))
    x = np.linspace(-1.0, 1.0, n)
    L = np.zeros((n, m))
    for l in range(n):
        diff = x[l] - xi
        exact = np.flatnonzero(diff == 0.0)
        if exact.size:
            L[l, exact[0]] = 1.0
        else:
            r = w / diff
            L[l] = r / r.sum()
    return L


def runge5d(m, n=35, d=5):
    """(F, [L] * d, x): the d-variate Runge function 1/(1 + 16 sum_mu x_mu^2)
    sampled on the m^d grid of Chebyshev nodes (axis mu-1 = x_mu), the n x m
    Lagrange matrix from those nodes to the n equispaced points x of [-1, 1],
    and x (Sec. 4.3, the 5-D interpolation example)."""
    i = np.arange(1, m + 1)
    xi = np.cos((2 * i - 1) * np.pi / (2.0 * m))
    acc = xi ** 2
    for _ in range(d - 1):
        acc = np.add.outer(acc, xi ** 2)
    acc *= 16.0
    acc += 1.0
    F = np.reciprocal(acc, out=acc)
    L = lagrange_chebyshev_to_uniform(m, n)
    return F, [L.copy() for _ in range(d)], np.linspace(-1.0, 1.0, n)


def fourier_matrix(n):
    """The n x n Fourier matrix exp(-2 pi i j k / n) (complex128), the basis
    matrix of a discrete Fourier transform along one direction."""
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def complex_problem(seed, m_dims, n_dims, conj=False):
    """Complex standard-normal T (real and imaginary parts N(0,1)) and
    factors, n_mu x m_mu (m_mu x n_mu if conj); drawn T first."""
    rng = np.random.default_rng(seed)
    T = _normal(rng, tuple(m_dims)) + 1j * _normal(rng, tuple(m_dims))
    Ls = []
    for n, m in zip(n_dims, m_dims):
        shape = (m, n) if conj else (n, m)
        Ls.append(_normal(rng, shape) + 1j * _normal(rng, shape))
    return T, Ls


def codeval_shapes():
    """The shapes of the paper's timing sweep of the Tucker operator: d = 3
    with n in {144, 196, 256, 324} and d = 6 with n in {12, 14, 16, 18}
    (square factors)."""
    return [(3, n) for n in (144, 196, 256, 324)] + [(6, n) for n in (12, 14, 16, 18)]


def interp6d(seed=SEED, m=16, n=24, d=6):
    rng = np.random.default_rng(seed)
    T = _normal(rng, (m,) * d)
    L = lagrange_chebyshev_to_uniform(m, n)
    return T, [L.copy() for _ in range(d)]


def batch_sizes(seed=SEED, count=64, d=4, lo=16, hi=64):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(count, d))


def batch64(seed=SEED, count=64, d=4, lo=16, hi=64):
    """Returns (sizes, [(T_k, [L_k1..L_kd]) for k in range(count)]).

    One generator serves the whole batch: sizes first, then per tensor its
    tensor followed by its d factors."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=(count, d))
    items = []
    for k in range(count):
        dims = tuple(int(s) for s in sizes[k])
        T = _normal(rng, dims)
        Ls = [_normal(rng, (s, s)) / np.sqrt(s) for s in dims]
        items.append((T, Ls))
    return sizes, items


WORKLOADS = {
    "small2d": dict(d=2, m=(50, 50), n=(50, 50)),
    "cube200": dict(d=3, m=(200,) * 3, n=(200,) * 3),
    "heat128": dict(d=3, m=(128,) * 3, n=(128,) * 3, tau=1e-3, h=1.0 / 129),
    "interp6d": dict(d=6, m=(16,) * 6, n=(24,) * 6),
    "batch64": dict(count=64, d=4, lo=16, hi=64),
}


def tucker_flops(m_dims, n_dims, order=None):
    """Algorithmic flop count of the Tucker operator applied mode by mode in
    ``order`` (default 1..d): each mu-mode product costs 2 * n_mu times the
    number of entries of its input (one multiply-add per term). This is
    bookkeeping for throughput figures, not part of the method."""
    d = len(m_dims)
    cur = list(m_dims)
    total = 0
    for mu in (order or range(1, d + 1)):
        entries = int(np.prod(cur, dtype=np.int64))
        total += 2 * int(n_dims[mu - 1]) * entries
        cur[mu - 1] = n_dims[mu - 1]
    return total
