"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the literal
element-wise formula, the Kronecker-product form of the Lemma in Sec. 2, the
index formula of vec (Appendix A), textbook matrix products, exact special
cases (identity and permutation factors, eigenvectors), scipy's matrix
exponential, and the relative errors the paper prints for its 5-D
interpolation example (Sec. 4.3). A plausible slip in the oracle -- a dropped
term, a wrong index or sign, a transposed factor, a reversed Kronecker order --
fails at least one of them.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.linalg

import oracle
import kp_workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_problem(rng, m, n):
    T = rng.standard_normal(m)
    Ls = [rng.standard_normal((nn, mm)) for nn, mm in zip(n, m)]
    return T, Ls


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ---------------------------------------------------------------------------
# vec and matricization (Appendix A; Sec. 2 definitions)
# ---------------------------------------------------------------------------

def test_vec_follows_index_formula():
    rng = np.random.default_rng(1)
    m = (3, 4, 2, 5)
    T = rng.standard_normal(m)
    v = oracle.vec(T)
    for j in itertools.product(*[range(1, mm + 1) for mm in m]):
        lin = j[0]
        stride = 1
        for mu in range(1, len(m)):
            stride *= m[mu - 1]
            lin += (j[mu] - 1) * stride
        assert v[lin - 1] == T[tuple(jj - 1 for jj in j)]
    assert np.array_equal(oracle.unvec(v, m), T)


def test_mumat_columns_are_fibers_in_column_major_order():
    rng = np.random.default_rng(2)
    m = (3, 4, 5)
    T = rng.standard_normal(m)
    for mu in (1, 2, 3):
        M = oracle.mumat(T, mu)
        rest = [k for k in range(3) if k != mu - 1]
        assert M.shape == (m[mu - 1], m[rest[0]] * m[rest[1]])
        col = 0
        # remaining indices in column-major order: the first one runs fastest
        for b in range(m[rest[1]]):
            for a in range(m[rest[0]]):
                idx = [0, 0, 0]
                idx[rest[0]], idx[rest[1]] = a, b
                fiber = [T[tuple(idx[:mu - 1] + [j] + idx[mu:])]
                         for j in range(m[mu - 1])]
                assert np.array_equal(M[:, col], fiber)
                col += 1


def test_mump_is_matrix_vector_per_fiber():
    # Sec. 2: each mu-fiber of S is L times the matching mu-fiber of T.
    rng = np.random.default_rng(3)
    m = (3, 4, 5)
    T = rng.standard_normal(m)
    for mu in (1, 2, 3):
        L = rng.standard_normal((6, m[mu - 1]))
        S = oracle.mump(T, L, mu)
        assert S.shape == tuple(6 if k == mu - 1 else m[k] for k in range(3))
        others = [range(m[k]) for k in range(3) if k != mu - 1]
        for fix in itertools.product(*others):
            sl_T = list(fix)
            sl_T.insert(mu - 1, slice(None))
            fT = T[tuple(sl_T)]
            fS = S[tuple(sl_T)]
            expect = np.array([sum(L[i, j] * fT[j] for j in range(m[mu - 1]))
                               for i in range(6)])
            np.testing.assert_allclose(fS, expect, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------------------
# Tucker operator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_tucker_matches_elementwise_nested_sums(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(1, 5))
    m = tuple(int(x) for x in rng.integers(1, 5 if d < 4 else 4, size=d))
    n = tuple(int(x) for x in rng.integers(1, 5 if d < 4 else 4, size=d))
    T, Ls = rand_problem(rng, m, n)
    S = oracle.tucker(T, Ls)
    assert S.shape == n
    assert rel(S, oracle.nested(T, Ls)) < 1e-13


def test_tucker_entry_matches_full_tucker():
    rng = np.random.default_rng(4)
    m, n = (4, 3, 5, 2), (3, 6, 2, 4)
    T, Ls = rand_problem(rng, m, n)
    S = oracle.tucker(T, Ls)
    for idx in itertools.product(*[range(k) for k in n]):
        assert abs(oracle.tucker_entry(T, Ls, idx) - S[idx]) < 1e-13 * np.abs(S).max()


@pytest.mark.parametrize("m,n", [((3, 4, 2), (2, 5, 3)), ((2, 3, 2, 3), (3, 2, 2, 2)),
                                 ((5,), (3,)), ((2, 2, 2, 2, 2), (3, 1, 2, 2, 3))])
def test_kronecker_lemma(m, n):
    # vec(S) = (L_d (x) ... (x) L_1) vec(T), with numpy's own kron.
    rng = np.random.default_rng(5)
    T, Ls = rand_problem(rng, m, n)
    K = np.ones((1, 1))
    for L in Ls:
        K = np.kron(L, K)
    v = oracle.vec(oracle.tucker(T, Ls))
    assert rel(v, K @ oracle.vec(T)) < 1e-13
    assert rel(oracle.kron(Ls), K) == 0.0


def test_row_major_reading_reverses_kronecker_order():
    # For row-major data (last index fastest) the same operator is
    # (L_1 (x) ... (x) L_d) acting on the row-major stacking.
    rng = np.random.default_rng(6)
    m, n = (3, 2, 4), (2, 3, 3)
    T, Ls = rand_problem(rng, m, n)
    K = np.kron(np.kron(Ls[0], Ls[1]), Ls[2])
    S = oracle.tucker(T, Ls)
    assert rel(S.reshape(-1, order="C"), K @ T.reshape(-1, order="C")) < 1e-13


@pytest.mark.parametrize("d", [3, 4])
def test_order_invariance(d):
    rng = np.random.default_rng(7 + d)
    m = tuple(int(x) for x in rng.integers(2, 6, size=d))
    n = tuple(int(x) for x in rng.integers(2, 6, size=d))
    T, Ls = rand_problem(rng, m, n)
    ref = oracle.tucker(T, Ls)
    for perm in itertools.permutations(range(1, d + 1)):
        assert rel(oracle.tucker(T, Ls, order=perm), ref) < 1e-13


def test_identity_factors_are_exact():
    rng = np.random.default_rng(8)
    T = rng.standard_normal((3, 4, 5))
    assert np.array_equal(oracle.tucker(T, [None, None, None]), T)
    assert np.array_equal(oracle.tucker(T, [np.eye(3), np.eye(4), np.eye(5)]), T)
    L2 = rng.standard_normal((6, 4))
    assert np.array_equal(oracle.tucker(T, [None, L2, None]),
                          oracle.mump(T, L2, 2))


def test_permutation_factors_permute_exactly():
    rng = np.random.default_rng(9)
    m = (4, 3, 5)
    T = rng.standard_normal(m)
    perms = [rng.permutation(k) for k in m]
    Ls = [np.eye(k)[p] for k, p in zip(m, perms)]   # (L x)_i = x_{p(i)}
    S = oracle.tucker(T, Ls)
    assert np.array_equal(S, T[np.ix_(*perms)])


def test_two_dimensional_matrix_form():
    # Sec. 1: s = L1 T L2^T, two textbook matrix products.
    T, Ls = kp_workloads.small2d(seed=0, n=50)
    S = oracle.tucker(T, Ls)
    ref = np.einsum("ia,ab,jb->ij", Ls[0], T, Ls[1])
    assert rel(S, ref) < 1e-13
    assert rel(oracle.mump(T, Ls[0], 1), Ls[0] @ T) < 1e-14
    assert rel(oracle.mump(T, Ls[1], 2), T @ Ls[1].T) < 1e-14


def test_meshgrid_ordering_swaps_first_two_factors():
    # Sec. 4: swapping L1 and L2 on meshgrid-ordered data gives the
    # (2,1,3)-permutation of S.
    rng = np.random.default_rng(10)
    m, n = (3, 4, 5), (2, 6, 3)
    T, Ls = rand_problem(rng, m, n)
    S = oracle.tucker(T, Ls)
    Tm = np.transpose(T, (1, 0, 2))
    Sm = oracle.tucker(Tm, [Ls[1], Ls[0], Ls[2]])
    assert rel(Sm, np.transpose(S, (1, 0, 2))) < 1e-13


def test_kronecker_sum_action():
    # Sec. 2: (L_d (+) ... (+) L_1) vec(V) = vec(sum_mu V x_mu L_mu).
    rng = np.random.default_rng(11)
    m = (3, 4, 2)
    V = rng.standard_normal(m)
    Ls = [rng.standard_normal((k, k)) for k in m]
    # Kronecker sum from its definition, built independently here
    I = [np.eye(k) for k in m]
    K = (np.kron(np.kron(I[2], I[1]), Ls[0]) + np.kron(np.kron(I[2], Ls[1]), I[0])
         + np.kron(np.kron(Ls[2], I[1]), I[0]))
    assert rel(oracle.kronsum(Ls), K) < 1e-15
    assert rel(oracle.vec(oracle.kronsumv(V, Ls)), K @ oracle.vec(V)) < 1e-13


def test_exponential_of_kronecker_sum_full_matrix():
    # Sec. 3.3: exp(tau (A_d (+) ... (+) A_1)) vec(V) = vec(V x_mu exp(tau A_mu)).
    rng = np.random.default_rng(12)
    m = (4, 3, 5)
    V = rng.standard_normal(m)
    As = [oracle.fd_laplacian_dirichlet(k, 1.0 / (k + 1)) for k in m]
    As[1] = As[1] + 0.3 * rng.standard_normal((3, 3))   # non-symmetric too
    tau = 0.01
    big = scipy.linalg.expm(tau * oracle.kronsum(As))
    Es = [scipy.linalg.expm(tau * A) for A in As]
    assert rel(oracle.vec(oracle.tucker(V, Es)), big @ oracle.vec(V)) < 1e-12


# ---------------------------------------------------------------------------
# 1-D factors
# ---------------------------------------------------------------------------

def test_dst_eigenpairs_satisfy_eigen_equation():
    n, h = 128, 1.0 / 129
    lam, Q = oracle.dst1_eigenpairs(n, h)
    A = oracle.fd_laplacian_dirichlet(n, h)
    assert rel(A @ Q, Q * lam) < 1e-13
    assert np.abs(Q @ Q.T - np.eye(n)).max() < 1e-13


@pytest.mark.parametrize("n,tau", [(5, 0.05), (128, 1e-3)])
def test_closed_form_exponential_matches_scipy(n, tau):
    h = 1.0 / (n + 1)
    E = oracle.expm_fd_laplacian_dirichlet(n, h, tau)
    ref = scipy.linalg.expm(tau * oracle.fd_laplacian_dirichlet(n, h))
    assert rel(E, ref) < 1e-13


def test_heat_eigentensor_at_full_size():
    # V = q_a (x) q_b (x) q_c is an eigentensor: the Tucker operator with the
    # factors exp(tau A) multiplies it by exp(tau (lam_a + lam_b + lam_c)).
    n, tau = 128, 1e-3
    h = 1.0 / (n + 1)
    lam, Q = oracle.dst1_eigenpairs(n, h)
    E = oracle.expm_fd_laplacian_dirichlet(n, h, tau)
    a, b, c = 0, 5, 12     # modest decay: the result stays far above rounding
    V = np.einsum("i,j,k->ijk", Q[:, a], Q[:, b], Q[:, c])
    S = oracle.tucker(V, [E, E, E])
    assert rel(S, np.exp(tau * (lam[a] + lam[b] + lam[c])) * V) < 1e-12


def test_workload_heat_matrix_is_the_dirichlet_laplacian():
    A = kp_workloads.heat_matrix(128)
    assert np.array_equal(A, oracle.fd_laplacian_dirichlet(128, 1.0 / 129))


def test_chebyshev_weights_are_barycentric_weights():
    # Up to one common factor, w_k = 1 / prod_{j != k} (xi_k - xi_j).
    for m in (3, 8, 16):
        xi = oracle.chebyshev_nodes(m)
        w_def = np.array([1.0 / np.prod([xi[k] - xi[j] for j in range(m) if j != k])
                          for k in range(m)])
        ratio = oracle.chebyshev_weights(m) / w_def
        assert np.abs(ratio / ratio[0] - 1).max() < 1e-10


def test_lagrange_matrix_properties():
    m, n = 16, 24
    x = np.linspace(-1, 1, n)
    L = oracle.lagrange_matrix(m, x)
    np.testing.assert_allclose(L.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    # Lagrange property at the nodes (each node hits the 0/0 branch)
    xi = oracle.chebyshev_nodes(m)
    assert np.array_equal(oracle.lagrange_matrix(m, xi), np.eye(m))
    # exact reproduction of polynomials of degree < m (power basis test)
    for deg in range(m):
        p_nodes = xi ** deg
        np.testing.assert_allclose(L @ p_nodes, x ** deg, rtol=0, atol=1e-12)
    # the workload generator builds the same matrix
    assert rel(kp_workloads.lagrange_chebyshev_to_uniform(m, n), L) < 1e-15


def test_polynomial_reproduction_in_six_dimensions():
    # Interpolation of a separable polynomial of degree <= 15 per variable is
    # exact; the Tucker operator reproduces it on the evaluation grid.
    m, n, d = 4, 5, 6
    x = np.linspace(-1, 1, n)
    xi = oracle.chebyshev_nodes(m)
    L = oracle.lagrange_matrix(m, x)
    rng = np.random.default_rng(13)
    coefs = rng.standard_normal((d, m))
    ps_nodes = [np.polyval(c, xi) for c in coefs]
    ps_x = [np.polyval(c, x) for c in coefs]
    T = ps_nodes[0]
    P = ps_x[0]
    for k in range(1, d):
        T = np.multiply.outer(T, ps_nodes[k])
        P = np.multiply.outer(P, ps_x[k])
    S = oracle.tucker(T, [L] * d)
    assert rel(S, P) < 1e-12


def _runge_interp_error(m, n=35):
    x = np.linspace(-1, 1, n)
    xi = oracle.chebyshev_nodes(m)
    L = oracle.lagrange_matrix(m, x)
    F = oracle.runge(*([xi] * 5))
    P = oracle.tucker(F, [L] * 5)
    f = oracle.runge(*([x] * 5))
    return np.abs(P - f).max() / np.abs(f).max()


def _golden_cases():
    with open(os.path.join(GOLDEN, "lagrange_runge5d.json")) as fh:
        g = json.load(fh)
    return list(zip(g["m"], g["relative_error_printed"]))


@pytest.mark.parametrize("m,printed", [
    pytest.param(mm, e, marks=[pytest.mark.slow] if mm >= 35 else [])
    for mm, e in _golden_cases()])
def test_runge_interpolation_errors_match_paper(m, printed):
    # Sec. 4.3 figure: relative errors printed with 3 significant digits.
    err = _runge_interp_error(m)
    assert float(f"{err:.3g}") == pytest.approx(printed, rel=1e-9), err


def test_runge_decay_line():
    # The dashed line of the same figure: c K^-m with K = 1/4 + sqrt(17/16).
    K = 0.25 + np.sqrt(17.0 / 16.0)
    c = 0.27607 * K ** 5
    assert c * K ** -45 == pytest.approx(1.387e-5, rel=2e-3)


# ---------------------------------------------------------------------------
# gradient
# ---------------------------------------------------------------------------

def test_dT_is_transpose_kronecker_action():
    rng = np.random.default_rng(14)
    m, n = (3, 2, 4), (2, 4, 3)
    T, Ls = rand_problem(rng, m, n)
    G = rng.standard_normal(n)
    dT, _ = oracle.tucker_vjp(T, Ls, G)
    K = np.ones((1, 1))
    for L in Ls:
        K = np.kron(L, K)
    assert rel(oracle.vec(dT), K.T @ oracle.vec(G)) < 1e-13


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(15)
    m, n = (3, 4, 2), (4, 2, 3)
    T, Ls = rand_problem(rng, m, n)
    G = rng.standard_normal(n)
    dT, dLs = oracle.tucker_vjp(T, Ls, G)

    def loss_T(t):
        return float(np.sum(G * oracle.tucker(t, Ls)))

    for _ in range(4):
        V = rng.standard_normal(m)
        fd = oracle.central_fd_directional(loss_T, T, V, 1e-5)
        assert fd == pytest.approx(np.sum(dT * V), rel=1e-8)
    for mu in range(3):
        def loss_L(Lm, mu=mu):
            L2 = list(Ls)
            L2[mu] = Lm
            return float(np.sum(G * oracle.tucker(T, L2)))
        # every entry by central differences
        for i in range(Ls[mu].shape[0]):
            for j in range(Ls[mu].shape[1]):
                E = np.zeros_like(Ls[mu])
                E[i, j] = 1.0
                fd = oracle.central_fd_directional(loss_L, Ls[mu], E, 1e-5)
                assert fd == pytest.approx(dLs[mu][i, j], rel=1e-7, abs=1e-9)


def test_gradient_q_p_form_agrees():
    # dL_mu also equals Q_mu^(mu) P_{mu-1}^(mu)^T with forward partials P and
    # reverse partials Q (the form the GPU backward sweep uses).
    rng = np.random.default_rng(16)
    m, n = (3, 4, 5, 2), (2, 3, 4, 5)
    T, Ls = rand_problem(rng, m, n)
    G = rng.standard_normal(n)
    _, dLs = oracle.tucker_vjp(T, Ls, G)
    d = 4
    P = [T]
    for k in range(1, d):
        P.append(oracle.mump(P[-1], Ls[k - 1], k))
    Q = G
    for mu in range(d, 0, -1):
        dL = oracle.mumat(Q, mu) @ oracle.mumat(P[mu - 1], mu).T
        assert rel(dL, dLs[mu - 1]) < 1e-13
        Q = oracle.mump(Q, Ls[mu - 1].T, mu)


def test_factor_gradient_column_matches_central_differences():
    # every entry of the sampled column by central differences of the loss
    # <G, tucker(T, Ls)> in the one factor entry, and the column against the
    # full gradient
    rng = np.random.default_rng(17)
    m, n = (3, 4, 2, 3), (2, 3, 4, 2)
    T, Ls = rand_problem(rng, m, n)
    G = rng.standard_normal(n)
    _, dLs = oracle.tucker_vjp(T, Ls, G)
    for mu in range(1, 5):
        for j in range(m[mu - 1]):
            col = oracle.factor_gradient_column(T, Ls, G, mu, j)
            assert rel(col, dLs[mu - 1][:, j]) < 1e-13

            def loss(Lm, mu=mu):
                L2 = list(Ls)
                L2[mu - 1] = Lm
                return float(np.sum(G * oracle.nested(T, L2)))
            for i in range(n[mu - 1]):
                E = np.zeros_like(Ls[mu - 1])
                E[i, j] = 1.0
                fd = oracle.central_fd_directional(loss, Ls[mu - 1], E, 1e-5)
                assert fd == pytest.approx(col[i], rel=1e-7, abs=1e-9)
