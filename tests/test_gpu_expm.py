"""GPU FP64 matrix exponential (kp_expm_f64) and the exponential of a
Kronecker sum through the Tucker operator (Sec. 3.3), against the oracle."""
import numpy as np
import pytest
import scipy.linalg
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, rel_max, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


@pytest.mark.parametrize("n,scale", [(1, 0.5), (2, 3.0), (7, 0.01), (16, 1.0), (33, 20.0),
                                     (64, 0.2), (100, 60.0), (200, 5.0), (256, 2.0)])
def test_expm_matches_scipy(kp, n, scale):
    rng = np.random.default_rng(600 + n)
    A = rng.standard_normal((n, n)) * scale / np.sqrt(n)
    say("expm", n, scale)
    E = kp.expm(to_dev(A, torch.float64), tau=1.0)
    torch.cuda.synchronize()
    ref = scipy.linalg.expm(A)
    # both are backward-stable algorithms; the gap is bounded by the
    # conditioning of exp at A, small for these norms
    assert rel_max(E.cpu().numpy(), ref) < 1e-11


def test_expm_many_squarings(kp):
    # skew-symmetric, ||A||_1 in the thousands: s = ceil(log2(||A||_1 / theta_13))
    # exceeds the squaring launches, so the last squarings run in the final
    # launch; exp(A) is orthogonal, hence well conditioned
    rng = np.random.default_rng(650)
    n = 40
    G = rng.standard_normal((n, n))
    A = (G - G.T) * 100.0
    norm1 = np.abs(A).sum(axis=0).max()
    assert np.ceil(np.log2(norm1 / 5.371920351148152)) >= 10
    say("expm skew", n, norm1)
    E = kp.expm(to_dev(A, torch.float64), tau=1.0).cpu().numpy()
    assert rel_max(E, scipy.linalg.expm(A)) < 1e-9
    assert np.abs(E.T @ E - np.eye(n)).max() < 1e-9


def test_expm_zero_and_identity_exact(kp):
    say("expm special cases")
    Z = torch.zeros(9, 9, dtype=torch.float64, device="cuda")
    assert torch.equal(kp.expm(Z), torch.eye(9, dtype=torch.float64, device="cuda"))
    D = torch.diag(torch.tensor([0.0, 1.0, -2.0], dtype=torch.float64, device="cuda"))
    np.testing.assert_allclose(kp.expm(D).cpu().numpy(), np.diag(np.exp([0.0, 1.0, -2.0])),
                               rtol=1e-14, atol=1e-15)


def test_expm_heat_matrix_closed_form(kp):
    # heat128 factor: tau * tridiag(1,-2,1)/h^2, ||.||_1 = 66.6 (four squarings)
    n, tau = 128, 1e-3
    A = kp_workloads.heat_matrix(n)
    say("expm heat128")
    E = kp.expm(to_dev(A, torch.float64), tau=tau)
    torch.cuda.synchronize()
    ref = oracle.expm_fd_laplacian_dirichlet(n, 1.0 / (n + 1), tau)
    assert rel_max(E.cpu().numpy(), ref) < 1e-12


def test_expm_batched(kp):
    rng = np.random.default_rng(700)
    As = rng.standard_normal((3, 20, 20))
    say("expm batched")
    E = kp.expm(to_dev(As, torch.float64), tau=0.3)
    torch.cuda.synchronize()
    for k in range(3):
        assert rel_max(E[k].cpu().numpy(), scipy.linalg.expm(0.3 * As[k])) < 1e-12


def test_exp_kronecker_sum_full_matrix_tiny(kp):
    # exp(tau (A_3 (+) A_2 (+) A_1)) vec(V) = vec(V x_mu exp(tau A_mu)), with the
    # full-matrix exponential of the assembled Kronecker sum.
    rng = np.random.default_rng(710)
    m = (4, 5, 3)
    V = rng.standard_normal(m)
    As = [kp_workloads.heat_matrix(k) for k in m]
    As[1] = As[1] + rng.standard_normal((5, 5))
    tau = 0.01
    say("exp of Kronecker sum, tiny, GPU expm + GPU Tucker")
    Es = [kp.expm(to_dev(A, torch.float64), tau=tau) for A in As]
    S = kp.tucker(to_dev(V, torch.float64), Es)
    torch.cuda.synchronize()
    big = scipy.linalg.expm(tau * oracle.kronsum(As))
    assert rel_max(oracle.vec(S.cpu().numpy()), big @ oracle.vec(V)) < 1e-12


@pytest.mark.parametrize("dt,prec", [("f64", "native"), ("f32", "native"),
                                     ("f32", "bf16x3"), ("f32", "bf16x6")])
def test_heat128_pipeline(kp, dt, prec):
    # Full size: GPU FP64 expm factors, Tucker in each form, vs the oracle.
    V, As, tau = kp_workloads.heat128(seed=0)
    tdt = torch.float64 if dt == "f64" else torch.float32
    say("heat128 pipeline", dt, prec)
    Ad = to_dev(np.stack(As), torch.float64)
    Es = kp.expm(Ad, tau=tau)
    Ls = [Es[k].to(tdt).contiguous() for k in range(3)]
    S = kp.tucker(to_dev(V, tdt), Ls, prec=prec)
    torch.cuda.synchronize()
    Eref = oracle.expm_fd_laplacian_dirichlet(128, 1.0 / 129, tau)
    V64 = cast64(V, tdt)
    # the oracle uses the GPU-cast factors for the low-precision forms so that
    # only the contraction's error is measured; FP64 uses the exact factors
    L64 = [Eref] * 3 if dt == "f64" else [Ls[k].double().cpu().numpy() for k in range(3)]
    ref = oracle.tucker(V64, L64)
    got = S.double().cpu().numpy()
    err = rel_max(got, ref)
    say("rel err", err)
    if dt == "f64":
        # the FP64 target; the GPU factors themselves differ from the closed
        # form by about 1e-14
        assert err < 1e-13
    else:
        bound = chain_bound(V64, L64, prec, tdt)
        assert np.all(np.abs(got - ref) <= bound)
        if prec in ("native", "bf16x6"):
            assert err < 1e-6


def test_heat128_eigentensor(kp):
    # V = q_a (x) q_b (x) q_c maps to exp(tau(lam_a + lam_b + lam_c)) V exactly.
    n, tau = 128, 1e-3
    h = 1.0 / (n + 1)
    lam, Q = oracle.dst1_eigenpairs(n, h)
    a, b, c = 0, 5, 12
    V = np.einsum("i,j,k->ijk", Q[:, a], Q[:, b], Q[:, c])
    say("heat128 eigentensor")
    E = kp.expm(to_dev(kp_workloads.heat_matrix(n), torch.float64), tau=tau)
    S = kp.tucker(to_dev(V, torch.float64), [E, E, E])
    torch.cuda.synchronize()
    assert rel_max(S.cpu().numpy(), np.exp(tau * (lam[a] + lam[b] + lam[c])) * V) < 1e-12
