"""Kronecker-sum action kp_kronsum: S = sum_mu T x_mu A_mu against the
oracle's kronsumv, in every form, over layouts that take the k-loop tile and
the strip tile (accumulating products)."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, say, to_dev, unit_error

pytestmark = pytest.mark.gpu

FORMS = [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16x6")]
DT = {"f64": torch.float64, "f32": torch.float32}
CASES = [(7, 5), (19, 45, 13), (30, 3, 70, 2), (90, 130, 5)]


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


@pytest.mark.parametrize("dt,prec", FORMS)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_kronsum_matches_oracle(kp, dt, prec, case):
    m = CASES[case]
    rng = np.random.default_rng(7000 + case)
    T = rng.standard_normal(m)
    As = [rng.standard_normal((k, k)) for k in m]
    T64, A64 = cast64(T, DT[dt]), [cast64(A, DT[dt]) for A in As]
    say("kronsum", m, dt, prec)
    S = kp.kronsum(to_dev(T, DT[dt]), [to_dev(A, DT[dt]) for A in As], prec=prec)
    torch.cuda.synchronize()
    ref = oracle.kronsumv(T64, A64)
    # componentwise: each term within its mode's bound, plus d - 1 additions
    bound = np.zeros_like(ref)
    for mu in range(1, len(m) + 1):
        bound += unit_error(prec, DT[dt], m[mu - 1]) * oracle.mump(np.abs(T64), np.abs(A64[mu - 1]), mu)
    u = 2.0 ** -53 if dt == "f64" else 2.0 ** -24
    absum = sum(np.abs(oracle.mump(T64, A64[mu - 1], mu)) for mu in range(1, len(m) + 1))
    bound = 2 * (bound + len(m) * u * absum) + 1e-300
    assert np.all(np.abs(S.double().cpu().numpy() - ref) <= bound)


def test_kronsum_heat_laplacian(kp):
    """The paper's use: the finite-difference Laplacian of a 3-D grid as a
    Kronecker sum of tridiag(1, -2, 1)/h^2, applied to a smooth grid function
    (second differences of sin products are exact multiples of them)."""
    n = 40
    h = 1.0 / (n + 1)
    A = kp_workloads.heat_matrix(n)
    x = np.arange(1, n + 1) * h
    s = np.sin(np.pi * x)
    V = np.einsum("i,j,k->ijk", s, s, s)
    S = kp.kronsum(to_dev(V, torch.float64), [to_dev(A, torch.float64)] * 3)
    torch.cuda.synchronize()
    # eigenvector of each tridiagonal factor: eigenvalue -4/h^2 sin^2(pi h / 2)
    lam = -4.0 / h ** 2 * np.sin(np.pi * h / 2) ** 2
    assert np.max(np.abs(S.cpu().numpy() - 3 * lam * V)) <= 1e-9 * np.max(np.abs(3 * lam * V))


def test_kronsum_order_one_and_strided_factors(kp):
    rng = np.random.default_rng(71)
    v = rng.standard_normal(37)
    A = rng.standard_normal((37, 37))
    S = kp.kronsum(to_dev(v, torch.float64), [to_dev(A, torch.float64)])
    torch.cuda.synchronize()
    assert np.max(np.abs(S.cpu().numpy() - A @ v)) <= 1e-13 * np.max(np.abs(A @ v))
    # transposed views (non-unit column stride) give the transposed sum
    T = rng.standard_normal((6, 9, 5))
    As = [rng.standard_normal((k, k)) for k in (6, 9, 5)]
    S = kp.kronsum(to_dev(T, torch.float64), [to_dev(B, torch.float64).t() for B in As])
    torch.cuda.synchronize()
    ref = oracle.kronsumv(T, [B.T for B in As])
    assert np.max(np.abs(S.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
