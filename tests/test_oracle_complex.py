"""Pins of the complex Tucker oracle: nested sums, the Kronecker form,
numpy's FFT, the adjoint identity and the real case (Sec. 2 over C; Sec. 3,
the conjugate-transpose form for spectral transforms)."""
import itertools

import numpy as np
import pytest

import oracle


def _crandn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_ztucker_matches_nested_sums():
    rng = np.random.default_rng(1)
    m, n = (3, 2, 4), (2, 3, 3)
    T = _crandn(rng, m)
    Ls = [_crandn(rng, (n[k], m[k])) for k in range(3)]
    S = oracle.ztucker(T, Ls)
    for i in itertools.product(*[range(v) for v in n]):
        ref = 0j
        for j in itertools.product(*[range(v) for v in m]):
            ref += T[j] * Ls[0][i[0], j[0]] * Ls[1][i[1], j[1]] * Ls[2][i[2], j[2]]
        assert abs(S[i] - ref) <= 1e-13 * (1 + abs(ref))


def test_ztucker_kronecker_form():
    rng = np.random.default_rng(2)
    m, n = (3, 4, 2), (4, 2, 3)
    T = _crandn(rng, m)
    Ls = [_crandn(rng, (n[k], m[k])) for k in range(3)]
    K = np.kron(Ls[2], np.kron(Ls[1], Ls[0]))      # L_3 (x) L_2 (x) L_1
    ref = K @ T.reshape(-1, order="F")
    got = oracle.ztucker(T, Ls).reshape(-1, order="F")
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", [(8,), (5, 6), (4, 7, 9)])
def test_fourier_matrices_give_the_fft(shape):
    rng = np.random.default_rng(3)
    T = _crandn(rng, shape)
    Fs = [oracle.dft_matrix(n) for n in shape]
    got = oracle.ztucker(T, Fs)
    ref = np.fft.fftn(T)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # conjugate-transposed Fourier matrices: the unnormalised inverse
    back = oracle.cttucker(got, Fs)
    assert np.max(np.abs(back / T.size - T)) <= 1e-12 * np.max(np.abs(T))


def test_cttucker_is_the_adjoint():
    rng = np.random.default_rng(4)
    m, n = (3, 5, 2), (4, 2, 6)
    T = _crandn(rng, m)
    G = _crandn(rng, n)
    Ls = [_crandn(rng, (n[k], m[k])) for k in range(3)]
    lhs = np.vdot(G, oracle.ztucker(T, Ls))           # <G, K T>
    rhs = np.vdot(oracle.cttucker(G, Ls), T)          # <K^* G, T>
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_real_case_and_identity():
    rng = np.random.default_rng(5)
    T = rng.standard_normal((4, 3, 5))
    Ls = [rng.standard_normal((2, 4)), None, rng.standard_normal((3, 5))]
    got = oracle.ztucker(T, Ls)
    assert np.max(np.abs(got.imag)) == 0.0
    assert np.allclose(got.real, oracle.tucker(T, Ls), rtol=1e-14, atol=1e-14)
    assert np.array_equal(oracle.ztucker(T + 0j, [None] * 3), T + 0j)
