"""Tensor primitives of Sec. 2 and Appendix A, in float64 numpy.

Test infrastructure only (see the package docstring).

Conventions
-----------
A tensor ``T`` of order d with sizes m_1 x ... x m_d is a numpy array of shape
``(m_1, ..., m_d)``; the paper's element t_{j_1...j_d} (1-based indices) sits
at ``T[j_1-1, ..., j_d-1]``. How numpy lays it out in memory is irrelevant
here: every memory order that matters (vec, matricization) is spelled out.
Modes ``mu`` are 1-based, as in the paper. A factor list ``Ls`` holds one
matrix per mode, ``Ls[mu-1]`` of shape (n_mu, m_mu); an entry ``None`` stands
for the identity matrix, which is the identity element of the mu-mode product
(Sec. 2, discussion of the Kronecker-sum action).
"""
from __future__ import annotations

import itertools

import numpy as np


def _as64(x):
    return np.asarray(x, dtype=np.float64)


def vec(T):
    """Stack a tensor into a vector (Appendix A, definition of vec).

    Entry (j_1, ..., j_d) goes to linear position
    j_1 + sum_{mu>=2} (j_mu - 1) * prod_{k<mu} m_k (1-based), i.e. the first
    index runs fastest: column-major order.
    """
    return np.reshape(_as64(T), -1, order="F")


def unvec(v, dims):
    """Inverse of :func:`vec` for a tensor of sizes ``dims``."""
    return np.reshape(_as64(v), tuple(dims), order="F")


def mumat(T, mu):
    """mu-matricization T^(mu) (Sec. 2, Definition of the mu-matricization).

    The columns of T^(mu) are the mu-fibers of T. Columns are ordered as the
    paper's realization orders them: bring mode mu to the front (the other
    modes keep their relative order), then unfold column-major.
    """
    T = _as64(T)
    d = T.ndim
    if not 1 <= mu <= d:
        raise ValueError(f"mode {mu} out of range for an order-{d} tensor")
    X = np.moveaxis(T, mu - 1, 0)
    return np.reshape(X, (T.shape[mu - 1], -1), order="F")


def _unmumat(M, mu, dims):
    """Fold a matrix with rows along mode mu back into a tensor of sizes dims."""
    rest = [dims[k] for k in range(len(dims)) if k != mu - 1]
    X = np.reshape(M, [dims[mu - 1]] + rest, order="F")
    return np.moveaxis(X, 0, mu - 1)


def mump(T, L, mu):
    """mu-mode product S = T x_mu L (Sec. 2, Definition of the mu-mode product).

    L has shape (n, m_mu); S has the sizes of T with m_mu replaced by n. It is
    computed through its defining matrix identity S^(mu) = L T^(mu): one
    matrix product of L with the mu-matricization, then folding back.
    ``L=None`` is the identity and returns a copy of T.
    """
    T = _as64(T)
    if L is None:
        return T.copy()
    L = _as64(L)
    if L.ndim != 2 or L.shape[1] != T.shape[mu - 1]:
        raise ValueError(
            f"factor of shape {L.shape} does not act on mode {mu} of size "
            f"{T.shape[mu - 1]}")
    dims = list(T.shape)
    dims[mu - 1] = L.shape[0]
    return _unmumat(L @ mumat(T, mu), mu, dims)


def tucker(T, Ls, order=None):
    """Tucker operator S = T x_1 L_1 x_2 ... x_d L_d (Sec. 2, Definition of the
    Tucker operator): d consecutive mu-mode products.

    ``order`` is an optional permutation of 1..d giving the sequence in which
    the products are applied; the default is the definition's order 1, 2, ...,
    d. The paper notes the result does not depend on the order (in exact
    arithmetic); the test suite checks that claim on this implementation.
    """
    S = _as64(T)
    d = S.ndim
    if len(Ls) != d:
        raise ValueError(f"need {d} factors, got {len(Ls)}")
    seq = list(range(1, d + 1)) if order is None else list(order)
    if sorted(seq) != list(range(1, d + 1)):
        raise ValueError(f"order {order} is not a permutation of 1..{d}")
    for mu in seq:
        S = mump(S, Ls[mu - 1], mu)
    return S


def nested(T, Ls):
    """Element-wise Tucker formula (Sec. 2, the nested-sum expression for
    s_{i_1...i_d}): s_i = sum over all j of t_j * prod_mu l^mu_{i_mu j_mu}.

    Literal loops over every output index and every input index. Cost is
    prod(n) * prod(m) * d, so use it only on tiny tensors.
    """
    T = _as64(T)
    d = T.ndim
    mats = [np.eye(T.shape[k]) if Ls[k] is None else _as64(Ls[k])
            for k in range(d)]
    out_dims = tuple(M.shape[0] for M in mats)
    S = np.zeros(out_dims)
    for i in itertools.product(*[range(n) for n in out_dims]):
        acc = 0.0
        for j in itertools.product(*[range(m) for m in T.shape]):
            p = T[j]
            for k in range(d):
                p *= mats[k][i[k], j[k]]
            acc += p
        S[i] = acc
    return S


def tucker_entry(T, Ls, idx):
    """One output element s_{i_1...i_d} of the Tucker operator.

    The nested sums of the element-wise formula (Sec. 2) are carried out from
    the innermost (over j_1) outwards, each sum being the contraction of one
    mode with row i_mu of L_mu. Used to sample outputs of tensors too large for
    the full oracle. ``idx`` holds 0-based output indices.
    """
    X = _as64(T)
    d = X.ndim
    for k in range(d):
        row = (np.eye(X.shape[0])[idx[k]] if Ls[k] is None
               else _as64(Ls[k])[idx[k]])
        X = np.tensordot(row, X, axes=([0], [0]))
    return float(X)


def kron(Ls):
    """The Kronecker product L_d (x) ... (x) L_1 (Appendix A; the order of the
    factors is the one of the Lemma relating the Tucker operator to the
    Kronecker product, Sec. 2). Dense: tiny sizes only."""
    K = np.ones((1, 1))
    for L in Ls:
        K = np.kron(_as64(L), K)
    return K


def kronsum(As):
    """The Kronecker sum A_d (+) ... (+) A_1 (Appendix A: for square A of size
    p and B of size q, A (+) B = A (x) I_q + I_p (x) B). Dense: tiny sizes."""
    K = _as64(As[0])
    for A in As[1:]:
        A = _as64(A)
        K = np.kron(A, np.eye(K.shape[0])) + np.kron(np.eye(A.shape[0]), K)
    return K


def kronsumv(V, Ls):
    """Action of the Kronecker sum of the L_mu on vec(V), in tensor form
    (Sec. 2, the Kronecker-sum action): the sum over mu of V x_mu L_mu.
    Returned as a tensor with the sizes of V."""
    V = _as64(V)
    S = np.zeros_like(V)
    for mu in range(1, V.ndim + 1):
        S += mump(V, Ls[mu - 1], mu)
    return S
