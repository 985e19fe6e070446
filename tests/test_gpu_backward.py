"""GPU parity of the Tucker operator's backward (kp_tucker_backward and the
torch.autograd.Function) against the FP64 oracle and finite differences."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import U32, U64, cast64, rel_max, say, to_dev, unit_error

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32}
FORMS = [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16x6")]
CASES = [
    ((7, 5), (4, 9)),
    ((5, 6, 7), (8, 3, 6)),
    ((3, 1, 4, 9), (2, 5, 4, 3)),
    ((40, 33, 3), (17, 70, 5)),
    ((4, 4, 4, 4, 4, 4), (6, 6, 6, 6, 6, 6)),
    # tens of thousands of fibers per factor gradient: several chunks per workgroup
    ((60, 50, 40, 30), (20, 64, 33, 9)),
    # inner strides that are multiples of 4 (16-byte fiber groups) with a
    # ragged last chunk
    ((36, 12, 20), (8, 16, 24)),
]


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


def grad_bounds(T, Ls, G, prec, dt):
    """Componentwise error bounds for dT and dL_mu: the absolute-value form of
    the same computation times the summed per-stage error coefficients."""
    d = T.ndim
    aT, aG = np.abs(T), np.abs(G)
    aL = [np.abs(L) for L in Ls]
    dT_abs, dL_abs = oracle.tucker_vjp(aT, aL, aG)
    m = T.shape
    n = tuple(L.shape[0] for L in Ls)
    coef_dT = sum(unit_error(prec, DT[dt], n[k]) for k in range(d))
    coef_dL = []
    for mu in range(d):
        fibers = int(np.prod([n[k] for k in range(mu)] + [m[k] for k in range(mu + 1, d)]))
        c = sum(unit_error(prec, DT[dt], m[k]) for k in range(mu))            # P chain
        c += sum(unit_error(prec, DT[dt], n[k]) for k in range(mu + 1, d))   # Q chain
        u = U64 if dt == "f64" else U32
        c += (fibers + 2) * u                                                 # gram sum
        coef_dL.append(c)
    return 2 * coef_dT * dT_abs + 1e-300, [2 * c * a + 1e-300 for c, a in zip(coef_dL, dL_abs)]


@pytest.mark.parametrize("cache", [True, False])
@pytest.mark.parametrize("dt,prec", FORMS)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_backward_matches_oracle(kp, dt, prec, case, cache):
    m, n = CASES[case]
    T, Ls = kp_workloads.random_problem(4000 + case, m, n)
    G = np.random.default_rng(5000 + case).standard_normal(n)
    say("backward", m, n, dt, prec, "cache" if cache else "recompute")
    Td, Gd = to_dev(T, DT[dt]), to_dev(G, DT[dt])
    Lds = [to_dev(L, DT[dt]) for L in Ls]
    cbuf = kp.tucker_with_cache(Td, Lds, prec)[1] if cache else None
    dT, dLs = kp.tucker_backward(Gd, Td, Lds, prec, cbuf)
    torch.cuda.synchronize()
    T64, G64 = cast64(T, DT[dt]), cast64(G, DT[dt])
    L64 = [cast64(L, DT[dt]) for L in Ls]
    rT, rL = oracle.tucker_vjp(T64, L64, G64)
    bT, bL = grad_bounds(T64, L64, G64, prec, dt)
    got = dT.double().cpu().numpy()
    assert np.all(np.abs(got - rT) <= bT), float(np.max(np.abs(got - rT) / bT))
    for k in range(len(m)):
        g = dLs[k].double().cpu().numpy()
        assert np.all(np.abs(g - rL[k]) <= bL[k]), (k, float(np.max(np.abs(g - rL[k]) / bL[k])))


def test_backward_partial_outputs(kp):
    m, n = (6, 7, 8), (5, 4, 9)
    T, Ls = kp_workloads.random_problem(4100, m, n)
    G = np.random.default_rng(4101).standard_normal(n)
    Td, Gd = to_dev(T, torch.float64), to_dev(G, torch.float64)
    Lds = [to_dev(L, torch.float64) for L in Ls]
    rT, rL = oracle.tucker_vjp(T, Ls, G)
    for need_dT, need_dL in [(False, [True, False, False]), (False, [False, False, True]),
                             (True, [False, False, False]), (False, [False, True, True])]:
        say("backward partial", need_dT, need_dL)
        dT, dLs = kp.tucker_backward(Gd, Td, Lds, need_dT=need_dT, need_dL=need_dL)
        torch.cuda.synchronize()
        assert (dT is None) == (not need_dT)
        if need_dT:
            assert rel_max(dT.cpu().numpy(), rT) < 1e-13
        for k in range(3):
            assert (dLs[k] is None) == (not need_dL[k])
            if need_dL[k]:
                assert rel_max(dLs[k].cpu().numpy(), rL[k]) < 1e-13


def test_backward_central_differences_fp64(kp):
    # The loss <W, tucker(T, Ls)> evaluated by the GPU forward in FP64.
    m, n = (5, 6, 4), (3, 7, 5)
    T, Ls = kp_workloads.random_problem(4200, m, n)
    rng = np.random.default_rng(4201)
    W = rng.standard_normal(n)
    Wd = to_dev(W, torch.float64)
    Lds = [to_dev(L, torch.float64) for L in Ls]

    def loss(Tv, Lv):
        return float((kp.tucker(Tv, Lv) * Wd).sum())

    say("backward central differences")
    dT, dLs = kp.tucker_backward(Wd, to_dev(T, torch.float64), Lds)
    torch.cuda.synchronize()
    h = 1e-6
    for _ in range(3):
        V = to_dev(rng.standard_normal(m), torch.float64)
        Td = to_dev(T, torch.float64)
        fd = (loss(Td + h * V, Lds) - loss(Td - h * V, Lds)) / (2 * h)
        assert fd == pytest.approx(float((dT * V).sum()), rel=1e-5)
    for k in range(3):
        E = to_dev(rng.standard_normal(Ls[k].shape), torch.float64)
        Lp = list(Lds)
        Lm = list(Lds)
        Lp[k] = Lds[k] + h * E
        Lm[k] = Lds[k] - h * E
        Td = to_dev(T, torch.float64)
        fd = (loss(Td, Lp) - loss(Td, Lm)) / (2 * h)
        assert fd == pytest.approx(float((dLs[k] * E).sum()), rel=1e-5)


@pytest.mark.parametrize("cache", [True, False])
def test_autograd_function(kp, cache):
    m, n = (6, 5, 7), (4, 8, 3)
    T, Ls = kp_workloads.random_problem(4300, m, n)
    W = np.random.default_rng(4301).standard_normal(n)
    Td = to_dev(T, torch.float64).requires_grad_(True)
    Lds = [to_dev(L, torch.float64).requires_grad_(True) for L in Ls]
    say("autograd function", cache)
    S = kp.tucker_autograd(Td, Lds, cache_partials=cache)
    loss = (S * to_dev(W, torch.float64)).sum()
    grads = torch.autograd.grad(loss, [Td] + Lds)
    torch.cuda.synchronize()
    rT, rL = oracle.tucker_vjp(T, Ls, W)
    assert rel_max(grads[0].cpu().numpy(), rT) < 1e-13
    for k in range(3):
        assert rel_max(grads[k + 1].cpu().numpy(), rL[k]) < 1e-13
    # only some inputs need gradients
    Td2 = to_dev(T, torch.float64)
    S2 = kp.tucker_autograd(Td2, Lds, cache_partials=cache)
    g2 = torch.autograd.grad((S2 * to_dev(W, torch.float64)).sum(), [Lds[1]])
    assert rel_max(g2[0].cpu().numpy(), rL[1]) < 1e-13


def _rank1_closed_forms(T, Ls, ws):
    """For the cotangent W = w_1 (x) ... (x) w_d the gradients have closed
    forms: dT = (L_1^T w_1) (x) ... (x) (L_d^T w_d), and
    dL_mu = w_mu (x) c_mu with c_mu = T contracted over every mode nu != mu
    with u_nu = L_nu^T w_nu (from dL_mu = G^(mu) Z_mu^(mu)^T)."""
    us = [L.T @ w for L, w in zip(Ls, ws)]
    d = T.ndim
    dLs = []
    for mu in range(d):
        X = T
        # contract the modes after mu first (keeps axis numbering simple)
        for nu in range(d - 1, mu, -1):
            X = np.tensordot(X, us[nu], axes=([nu], [0]))
        for nu in range(mu):
            X = np.tensordot(us[nu], X, axes=([0], [0]))
        dLs.append(np.outer(ws[mu], X))
    return us, dLs


@pytest.mark.parametrize("prec", ["native", "bf16x6", "bf16x3"])
def test_interp6d_backward_full_size_rank1_cotangent(kp, prec):
    # d = 6, T 16^6 FP32, Lagrange factors 24 x 16: full size, forward cache.
    T, Ls = kp_workloads.interp6d(seed=0)
    rng = np.random.default_rng(4400)
    ws = [rng.standard_normal(24) for _ in range(6)]
    say("interp6d backward full size", prec)
    Td = to_dev(T, torch.float32)
    Lds = [to_dev(L, torch.float32) for L in Ls]
    S, cache = kp.tucker_with_cache(Td, Lds, prec)
    W = torch.tensor(ws[0], dtype=torch.float32, device="cuda")
    for w in ws[1:]:
        W = torch.multiply(W.unsqueeze(-1), torch.tensor(w, dtype=torch.float32, device="cuda"))
    del S
    dT, dLs = kp.tucker_backward(W.contiguous(), Td, Lds, prec, cache)
    torch.cuda.synchronize()
    del cache, W
    T64 = cast64(T, torch.float32)
    L64 = [cast64(L, torch.float32) for L in Ls]
    w64 = [cast64(w, torch.float32) for w in ws]
    us, rL = _rank1_closed_forms(T64, L64, w64)
    rT = us[0]
    for u in us[1:]:
        rT = np.multiply.outer(rT, u)
    # componentwise bounds from the absolute-value form of the same sums
    aus, aL = _rank1_closed_forms(np.abs(T64), [np.abs(L) for L in L64], [np.abs(w) for w in w64])
    aT = aus[0]
    for u in aus[1:]:
        aT = np.multiply.outer(aT, u)
    m, n = (16,) * 6, (24,) * 6
    coef_T = sum(unit_error(prec, torch.float32, n[k]) for k in range(6))
    got = dT.double().cpu().numpy()
    say("dT rel err", rel_max(got, rT))
    assert np.all(np.abs(got - rT) <= 2 * coef_T * aT + 1e-300)
    for k in range(6):
        fibers = 24 ** k * 16 ** (5 - k)
        coef = (sum(unit_error(prec, torch.float32, m[j]) for j in range(k))
                + sum(unit_error(prec, torch.float32, n[j]) for j in range(k + 1, 6))
                + (fibers + 2) * U32)
        g = dLs[k].double().cpu().numpy()
        say("dL", k, "rel err", rel_max(g, rL[k]))
        assert np.all(np.abs(g - rL[k]) <= 2 * coef * aL[k] + 1e-300), k


# ---------------------------------------------------------------------------
# Directional central differences at the full interp6d size (d = 6, T 16^6,
# 24 x 16 Lagrange factors) with a general cotangent G (24^6, standard
# normal): the loss f(T, L) = <G, tucker(T, L)> is evaluated by the FP64
# oracle at theta +- h v for 16 random directions v, and compared with the
# directional derivative <dT, v_T> + sum_mu <dL_mu, v_mu> of the GPU gradient.
# Each block of v is scaled to the norm of its parameter block (every block
# then contributes to the derivative on the same scale), so |v| = |theta| and
# the step h = 1e-4 |theta| / |v| is 1e-4. f is a polynomial of degree 7 along
# v, so the central difference's truncation error is about 35 h^2 relative.
# ---------------------------------------------------------------------------
FD_DIRECTIONS = 16
FD_STEP = 1e-4


def _fd_direction(k, T64, L64):
    rng = np.random.default_rng(4600 + k)
    VT = rng.standard_normal(T64.shape)
    VT *= np.linalg.norm(T64) / np.linalg.norm(VT)
    VL = []
    for L in L64:
        V = rng.standard_normal(L.shape)
        VL.append(V * (np.linalg.norm(L) / np.linalg.norm(V)))
    return VT, VL


@pytest.fixture(scope="module")
def interp6d_fd():
    T, Ls = kp_workloads.interp6d(seed=0)
    T64 = cast64(T, torch.float32)
    L64 = [cast64(L, torch.float32) for L in Ls]
    G = np.random.default_rng(4500).standard_normal((24,) * 6).astype(np.float32)
    Gf = np.asfortranarray(G.astype(np.float64))

    def loss(Tx, Lx):
        S = oracle.tucker(Tx, Lx)
        return float(np.dot(Gf.reshape(-1, order="F"), S.reshape(-1, order="F")))

    say("interp6d directional FD: oracle evaluations")
    fd = []
    for k in range(FD_DIRECTIONS):
        VT, VL = _fd_direction(k, T64, L64)
        h = FD_STEP
        fp = loss(T64 + h * VT, [L + h * V for L, V in zip(L64, VL)])
        fm = loss(T64 - h * VT, [L - h * V for L, V in zip(L64, VL)])
        fd.append((fp - fm) / (2 * h))
        say("direction", k, "done")
    del Gf
    return T, Ls, G, T64, L64, fd


# 32 FP64 oracle evaluations of a 24^6 output (a few seconds each on the
# host) run in the module fixture: the limit covers that CPU work.
#
# The directional derivative is a sum of one term per parameter block,
# <dT, v_T> + sum_mu <dL_mu, v_mu>, and for a random direction these terms
# cancel (direction 13: terms of up to 1.8e4 summing to 2.6e3). The FP64
# gradient is held to 1e-5 of |FD| itself. An FP32 gradient carries FP32
# rounding in every block term (the factor gradients are sums of 16^5 * 24
# products), so its difference from the FD is measured against the size of
# the terms, sum_b |<grad_b, v_b>|, at the same 1e-5; its distance to |FD|
# is reported beside it.
@pytest.mark.timeout(600)
@pytest.mark.parametrize("dt,prec", [("f64", "native"), ("f32", "native"), ("f32", "bf16x6")])
def test_interp6d_backward_directional_fd(kp, interp6d_fd, dt, prec):
    T, Ls, G, T64, L64, fd = interp6d_fd
    tdt = torch.float64 if dt == "f64" else torch.float32
    say("interp6d backward vs directional FD", dt, prec)
    # T64, L64 hold the FP32-rounded inputs (exact in either dtype)
    Td = to_dev(T64, tdt)
    Lds = [to_dev(L, tdt) for L in L64]
    dT, dLs = kp.tucker_backward(to_dev(G, tdt), Td, Lds, prec)
    torch.cuda.synchronize()
    gT = dT.double().cpu().numpy()
    gL = [x.double().cpu().numpy() for x in dLs]
    del dT, dLs, Td
    worst = worst_fd = 0.0
    for k in range(FD_DIRECTIONS):
        VT, VL = _fd_direction(k, T64, L64)
        terms = [float(np.vdot(gT, VT))] + [float(np.vdot(g, V)) for g, V in zip(gL, VL)]
        dd = sum(terms)
        rel_fd = abs(dd - fd[k]) / abs(fd[k])
        rel = rel_fd if dt == "f64" else abs(dd - fd[k]) / sum(abs(x) for x in terms)
        worst, worst_fd = max(worst, rel), max(worst_fd, rel_fd)
        assert rel <= 1e-5, (k, dd, fd[k], rel, rel_fd)
    say("worst relative difference", worst, "(to |FD|:", worst_fd, ")")


@pytest.mark.timeout(600)
def test_interp6d_backward_general_cotangent_vs_oracle(kp, interp6d_fd):
    # The FP32 gradient against the oracle's analytic gradient at full size,
    # max-norm relative <= 1e-6 (the FP32 target).
    T, Ls, G, T64, L64, _ = interp6d_fd
    say("interp6d backward, general cotangent, vs oracle")
    Td = to_dev(T, torch.float32)
    Lds = [to_dev(L, torch.float32) for L in Ls]
    dT, dLs = kp.tucker_backward(to_dev(G, torch.float32), Td, Lds)
    torch.cuda.synchronize()
    rT, rL = oracle.tucker_vjp(T64, L64, G.astype(np.float64))
    err = rel_max(dT.double().cpu().numpy(), rT)
    say("dT rel err", err)
    assert err <= 1e-6
    for k in range(6):
        e = rel_max(dLs[k].double().cpu().numpy(), rL[k])
        say("dL", k, "rel err", e)
        assert e <= 1e-6, k
