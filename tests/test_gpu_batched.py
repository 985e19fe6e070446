"""Batched Tucker operator (one persistent launch per dependency level,
kp_tucker_batched): parity with the single-problem path and the FP64 oracle,
gradients and graph capture."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, rel_max, say, to_dev, unit_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


def mixed_problems(seed, count, dt, square=False):
    rng = np.random.default_rng(seed)
    probs = []
    for k in range(count):
        d = int(rng.integers(1, 5))
        m = tuple(int(x) for x in rng.integers(1, 40, size=d))
        n = m if square else tuple(int(x) for x in rng.integers(1, 40, size=d))
        T, Ls = kp_workloads.random_problem(seed * 100 + k, m, n)
        probs.append((T, Ls))
    Td = [to_dev(T, dt) for T, _ in probs]
    Ld = [[to_dev(L, dt) for L in Ls] for _, Ls in probs]
    return probs, Td, Ld


@pytest.mark.parametrize("prec", ["native", "bf16x3", "bf16x6"])
def test_batched_forward_equals_single_path(kp, prec):
    # square factors: kp_tucker applies the modes in definition order too, and
    # the FP32 default tiles are in the executor, so FP32 results match bitwise
    probs, Td, Ld = mixed_problems(11, 12, torch.float32, square=True)
    say("batched forward vs single", prec)
    bt = kp.BatchedTucker(Td, Ld, prec=prec)
    S = bt.run()
    torch.cuda.synchronize()
    for k in range(len(probs)):
        ref = kp.tucker(Td[k], Ld[k], prec=prec)
        torch.cuda.synchronize()
        if prec == "native":
            assert torch.equal(S[k], ref), k
        T64, L64 = cast64(probs[k][0], torch.float32), [cast64(L, torch.float32)
                                                       for L in probs[k][1]]
        got = S[k].double().cpu().numpy()
        assert np.all(np.abs(got - oracle.tucker(T64, L64)) <=
                      chain_bound(T64, L64, prec, torch.float32)), k


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_batched_forward_backward_mixed(kp, dt):
    probs, Td, Ld = mixed_problems(12, 10, dt)
    rng = np.random.default_rng(13)
    Gs = [rng.standard_normal(tuple(L.shape[0] for L in Ls)) for _, Ls in probs]
    Gd = [to_dev(G, dt) for G in Gs]
    say("batched fwd+bwd mixed", dt)
    bt = kp.BatchedTucker(Td, Ld, Gs=Gd)
    bt.run()
    torch.cuda.synchronize()
    tol = 1e-12 if dt == torch.float64 else 2e-5
    for k, (T, Ls) in enumerate(probs):
        T64, L64, G64 = cast64(T, dt), [cast64(L, dt) for L in Ls], cast64(Gs[k], dt)
        assert rel_max(bt.S[k].double().cpu().numpy(), oracle.tucker(T64, L64)) < tol, k
        rT, rL = oracle.tucker_vjp(T64, L64, G64)
        assert rel_max(bt.dT[k].double().cpu().numpy(), rT) < tol, k
        for j in range(len(Ls)):
            assert rel_max(bt.dL[k][j].double().cpu().numpy(), rL[j]) < 10 * tol, (k, j)


def test_batched_partial_gradients(kp):
    probs, Td, Ld = mixed_problems(14, 5, torch.float64)
    rng = np.random.default_rng(15)
    Gs = [to_dev(rng.standard_normal(tuple(L.shape[0] for L in Ls)), torch.float64)
          for _, Ls in probs]
    say("batched, dL only")
    bt = kp.BatchedTucker(Td, Ld, Gs=Gs, need_dT=False)
    bt.run()
    torch.cuda.synchronize()
    assert bt.dT is None
    for k, (T, Ls) in enumerate(probs):
        _, rL = oracle.tucker_vjp(T, Ls, Gs[k].cpu().numpy())
        for j in range(len(Ls)):
            assert rel_max(bt.dL[k][j].cpu().numpy(), rL[j]) < 1e-12


def entry_bound(T64, L64, idx, prec, dtype):
    """Componentwise a-priori bound of one output entry (gpu_util.chain_bound
    for a single entry, through oracle.tucker_entry on absolute values)."""
    coef = sum(unit_error(prec, dtype, T64.shape[k]) for k in range(T64.ndim))
    return 2.0 * coef * oracle.tucker_entry(np.abs(T64), [np.abs(L) for L in L64], idx) + 1e-300


# Max-norm relative tolerance of a factor-gradient column (an FP32 sum over
# all fibers of products of two chains computed in the form): FP32 and BF16x6
# carry about FP32 rounding, BF16x3 about 2^-16 per operand.
DL_TOL = {"native": 2e-5, "bf16x6": 2e-5, "bf16x3": 3e-4}


@pytest.mark.parametrize("prec", ["native", "bf16x3", "bf16x6"])
def test_batch64_forward_backward(kp, prec):
    # Every problem of the batch against the FP64 oracle: problems 0, 8, ...,
    # 56 in full (S, dT and every dL_mu), the others by sampled entries of S
    # and dT (componentwise bound) and one sampled column of every dL_mu.
    sizes, items = kp_workloads.batch64(seed=0)
    Td = [to_dev(T, torch.float32) for T, _ in items]
    Ld = [[to_dev(L, torch.float32) for L in Ls] for _, Ls in items]
    rng = np.random.default_rng(16)
    Gs = [rng.standard_normal(tuple(int(s) for s in sizes[k])) for k in range(len(items))]
    Gd = [to_dev(G, torch.float32) for G in Gs]
    say("batch64 forward+backward", prec)
    bt = kp.BatchedTucker(Td, Ld, prec=prec, Gs=Gd)
    bt.run()
    torch.cuda.synchronize()
    pick = np.random.default_rng(19)
    for k in range(len(items)):
        T64 = cast64(items[k][0], torch.float32)
        L64 = [cast64(L, torch.float32) for L in items[k][1]]
        G64 = cast64(Gs[k], torch.float32)
        Lt64 = [L.T for L in L64]
        S = bt.S[k].double().cpu().numpy()
        dT = bt.dT[k].double().cpu().numpy()
        dL = [x.double().cpu().numpy() for x in bt.dL[k]]
        if k % 8 == 0:
            assert np.all(np.abs(S - oracle.tucker(T64, L64)) <=
                          chain_bound(T64, L64, prec, torch.float32)), k
            rT, rL = oracle.tucker_vjp(T64, L64, G64)
            assert np.all(np.abs(dT - rT) <= chain_bound(G64, Lt64, prec, torch.float32)), k
            for j in range(4):
                assert rel_max(dL[j], rL[j]) < DL_TOL[prec], (k, j)
            continue
        for _ in range(4):
            i = tuple(int(pick.integers(0, s)) for s in S.shape)
            ref = oracle.tucker_entry(T64, L64, i)
            assert abs(S[i] - ref) <= entry_bound(T64, L64, i, prec, torch.float32), (k, i)
            j = tuple(int(pick.integers(0, s)) for s in dT.shape)
            ref = oracle.tucker_entry(G64, Lt64, j)
            assert abs(dT[j] - ref) <= entry_bound(G64, Lt64, j, prec, torch.float32), (k, j)
        for mu in range(1, 5):
            col = int(pick.integers(0, T64.shape[mu - 1]))
            ref = oracle.factor_gradient_column(T64, L64, G64, mu, col)
            assert rel_max(dL[mu - 1][:, col], ref) < DL_TOL[prec], (k, mu, col)


def test_batched_graph_capture_replays(kp):
    # square factors: the single-problem path takes the same order and tiles,
    # so every replay must reproduce its results bitwise
    probs, Td, Ld = mixed_problems(17, 8, torch.float32, square=True)
    rng = np.random.default_rng(18)
    Gd = [to_dev(rng.standard_normal(tuple(L.shape[0] for L in Ls)), torch.float32)
          for _, Ls in probs]
    bt = kp.BatchedTucker(Td, Ld, Gs=Gd)
    bt.run()  # warm up outside the capture
    torch.cuda.synchronize()
    say("batched graph capture")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        # change the inputs in place (eager work between replays)
        for k in range(len(Td)):
            Td[k].copy_(torch.randn_like(Td[k]))
            Gd[k].copy_(torch.randn_like(Gd[k]))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(len(Td)):
            ref = kp.tucker(Td[k], Ld[k])
            dT, dLs = kp.tucker_backward(Gd[k], Td[k], Ld[k])
            torch.cuda.synchronize()
            assert torch.equal(bt.S[k], ref), (rep, k)
            assert rel_max(bt.dT[k].double().cpu().numpy(), dT.double().cpu().numpy()) < 1e-5
            for j in range(len(dLs)):
                assert rel_max(bt.dL[k][j].double().cpu().numpy(),
                               dLs[j].double().cpu().numpy()) < 1e-4
