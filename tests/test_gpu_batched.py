"""Batched Tucker operator (one persistent launch per dependency level,
kp_tucker_batched): parity with the single-problem path and the FP64 oracle,
gradients and graph capture."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, rel_max, say, to_dev

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


@pytest.mark.parametrize("prec", ["native", "bf16x3"])
def test_batch64_forward_backward(kp, prec):
    sizes, items = kp_workloads.batch64(seed=0)
    Td = [to_dev(T, torch.float32) for T, _ in items]
    Ld = [[to_dev(L, torch.float32) for L in Ls] for _, Ls in items]
    rng = np.random.default_rng(16)
    Gd = [torch.randn(tuple(int(s) for s in sizes[k]), generator=None, dtype=torch.float32,
                      device="cuda") for k in range(len(items))]
    say("batch64 forward+backward", prec)
    bt = kp.BatchedTucker(Td, Ld, prec=prec, Gs=Gd)
    bt.run()
    torch.cuda.synchronize()
    for k in range(0, 64, 9):
        ref = kp.tucker(Td[k], Ld[k], prec=prec)
        dT, dLs = kp.tucker_backward(Gd[k], Td[k], Ld[k], prec)
        torch.cuda.synchronize()
        if prec == "native":
            assert torch.equal(bt.S[k], ref), k
        assert rel_max(bt.S[k].double().cpu().numpy(), ref.double().cpu().numpy()) < 1e-5
        assert rel_max(bt.dT[k].double().cpu().numpy(), dT.double().cpu().numpy()) < 1e-4
        for j in range(4):
            assert rel_max(bt.dL[k][j].double().cpu().numpy(),
                           dLs[j].double().cpu().numpy()) < 1e-4, (k, j)
    # one problem fully against the FP64 oracle
    k = 5
    T64 = cast64(items[k][0], torch.float32)
    L64 = [cast64(L, torch.float32) for L in items[k][1]]
    G64 = Gd[k].double().cpu().numpy()
    rT, rL = oracle.tucker_vjp(T64, L64, G64)
    tol = 3e-4 if prec == "bf16x3" else 2e-5
    assert rel_max(bt.dT[k].double().cpu().numpy(), rT) < tol
    for j in range(4):
        assert rel_max(bt.dL[k][j].double().cpu().numpy(), rL[j]) < 10 * tol


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
