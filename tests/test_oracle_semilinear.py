"""Pins of the semilinear-experiment oracle (tridiagonal inverses, PCG, the
backward-forward Euler run) against closed forms, library solvers and the
figures the paper prints (Sec. 4.5, Table of the semilinear results)."""
import numpy as np
import pytest
import scipy.linalg

import oracle


def _sine_inverse(n, tau):
    """(I - tau A)^{-1} for A = tridiag(1,-2,1)/h^2, h = 1/(n+1), written from
    the sine eigenbasis: eigenvectors sqrt(2/(n+1)) sin(j k pi/(n+1)),
    eigenvalues -(4/h^2) sin^2(k pi/(2(n+1)))."""
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    Q = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))
    lam = -(4.0 / h ** 2) * np.sin(j * np.pi / (2.0 * (n + 1))) ** 2
    return (Q / (1.0 - tau * lam)) @ Q.T


@pytest.mark.parametrize("n,tau", [(1, 0.01), (5, 0.3), (48, 0.01), (97, 1e-3)])
def test_adi_inverse_matches_sine_closed_form(n, tau):
    h = 1.0 / (n + 1)
    off = np.full(n, -tau / h ** 2)
    got = oracle.tridiag_inverse(off, np.full(n, 1 + 2 * tau / h ** 2), off)
    ref = _sine_inverse(n, tau)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [2, 7, 64])
def test_tridiag_inverse_general_against_banded_solver(n):
    rng = np.random.default_rng(n)
    lo, up = rng.standard_normal(n), rng.standard_normal(n)
    dg = 3.0 + rng.random(n)                      # diagonally dominant
    got = oracle.tridiag_inverse(lo, dg, up)
    ab = np.zeros((3, n))                         # LAPACK band storage
    ab[0, 1:] = up[:n - 1]
    ab[1] = dg
    ab[2, :n - 1] = lo[1:]
    ref = scipy.linalg.solve_banded((1, 1), ab, np.eye(n))
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)) * n


def _spd(rng, n):
    B = rng.standard_normal((n, n))
    return B @ B.T / n + np.eye(n)


def test_pcg_matches_dense_solve():
    rng = np.random.default_rng(3)
    As = [_spd(rng, k) for k in (3, 4, 5)]
    b = rng.standard_normal((3, 4, 5))
    x, it, res = oracle.pcg(lambda v: oracle.kronsumv(v, As), b, np.zeros_like(b), tol=1e-13)
    K = np.zeros((60, 60))                        # the Kronecker sum, assembled by columns
    for c in range(60):
        e = np.zeros(60)
        e[c] = 1.0
        K[:, c] = oracle.vec(oracle.kronsumv(oracle.unvec(e, (3, 4, 5)), As))
    ref = oracle.unvec(np.linalg.solve(K, oracle.vec(b)), (3, 4, 5))
    assert res <= 1e-13 and it <= 60
    assert np.max(np.abs(x - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_pcg_with_exact_inverse_takes_one_iteration():
    rng = np.random.default_rng(4)
    A = _spd(rng, 12)
    Ainv = np.linalg.inv(A)
    b = rng.standard_normal(12)
    x, it, res = oracle.pcg(lambda v: A @ v, b, np.zeros(12), lambda r: Ainv @ r, tol=1e-12)
    assert it == 1 and res <= 1e-12


def test_cg_terminates_within_distinct_eigenvalues():
    # diagonal Kronecker sum with eigenvalues a_i + b_j + c_k: 4 distinct values
    As = [np.diag([1.0, 2.0]), np.diag([1.0, 2.0]), np.diag([1.0, 1.0, 2.0])]
    b = np.random.default_rng(5).standard_normal((2, 2, 3))
    x, it, res = oracle.pcg(lambda v: oracle.kronsumv(v, As), b, np.zeros_like(b), tol=1e-12)
    assert it <= 4 and res <= 1e-12


def test_pcg_zero_rhs_and_converged_start():
    A = lambda v: 2.0 * v
    x, it, res = oracle.pcg(A, np.zeros(5), np.ones(5))
    assert it == 0 and np.all(x == 0)
    b = np.arange(1.0, 6.0)
    x, it, res = oracle.pcg(A, b, b / 2)
    assert it == 0 and res == 0.0


def _second_difference(n):
    h = 1.0 / (n + 1)
    return (np.diag(np.full(n, -2.0)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) / h ** 2


def test_second_difference_is_exact_on_u0():
    ns = (6, 7, 9)
    xs = [oracle.semilinear_grid(n)[0] for n in ns]
    u0 = oracle.semilinear_u0(xs)
    # u0 closed form on the grid, and its Laplacian -2 (q2 q3 + q1 q3 + q1 q2)
    X = np.meshgrid(*xs, indexing="ij")
    q = [x * (1 - x) for x in X]
    assert np.allclose(u0, q[0] * q[1] * q[2], rtol=1e-15, atol=0)
    lap = oracle.kronsumv(u0, [_second_difference(n) for n in ns])
    ref = -2 * (q[1] * q[2] + q[0] * q[2] + q[0] * q[1])
    assert np.max(np.abs(lap - ref)) <= 1e-12
    assert np.max(np.abs(oracle.semilinear_laplacian_u0(xs) - ref)) <= 1e-15


@pytest.mark.parametrize("t", [0.0, 0.37, 1.0])
def test_exact_solution_solves_semidiscrete_system(t):
    ns = (5, 6, 8)
    xs = [oracle.semilinear_grid(n)[0] for n in ns]
    u = np.exp(t) * oracle.semilinear_u0(xs)
    # u' = e^t u0 must equal Laplacian_h u + 1/(1+u^2) + Phi(t)
    rhs = oracle.kronsumv(u, [_second_difference(n) for n in ns]) + 1 / (1 + u * u) \
        + oracle.semilinear_phi(t, xs)
    assert np.max(np.abs(rhs - u)) <= 1e-12


def test_imex_step_against_direct_solve():
    ns, tau = (5, 6, 7), 0.05
    xs = [oracle.semilinear_grid(n)[0] for n in ns]
    u0 = oracle.semilinear_u0(xs)
    u1, its = oracle.semilinear_imex(ns, tau=tau, steps=1, tol=1e-14)
    # backward-forward Euler written as one dense solve with the assembled
    # M = I - tau (A_3 (+) A_2 (+) A_1) (column-major vec)
    A = [_second_difference(n) for n in ns]
    I = [np.eye(n) for n in ns]
    K = (np.kron(I[2], np.kron(I[1], A[0])) + np.kron(I[2], np.kron(A[1], I[0]))
         + np.kron(A[2], np.kron(I[1], I[0])))
    M = np.eye(K.shape[0]) - tau * K
    b = u0 + tau * (1 / (1 + u0 ** 2) + oracle.semilinear_phi(0.0, xs))
    ref = np.linalg.solve(M, b.reshape(-1, order="F")).reshape(ns, order="F")
    assert np.max(np.abs(u1 - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_semilinear_experiment_matches_printed_results():
    """n = (40, 44, 48), tau = 0.01, t* = 1: final relative max-norm error
    9.7e-3 for every solver, about 2 PCG iterations per step with the ADI
    preconditioner and about 30 CG iterations without it."""
    ns, tau, steps = (40, 44, 48), 0.01, 100
    xs = [oracle.semilinear_grid(n)[0] for n in ns]
    exact = np.exp(1.0) * oracle.semilinear_u0(xs)
    for pre in (True, False):
        u, its = oracle.semilinear_imex(ns, tau=tau, steps=steps, precondition=pre)
        err = np.max(np.abs(u - exact)) / np.max(np.abs(exact))
        assert 9.65e-3 <= err <= 9.8e-3, err
        if pre:
            assert round(np.mean(its)) == 2, np.mean(its)
        else:
            assert 25 <= np.mean(its) <= 40, np.mean(its)
