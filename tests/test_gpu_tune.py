"""Tile autotuning on the GPU: the tuner records tiles that the calls then
use, results stay within the oracle bounds, and the batched executor built
after throughput tuning still matches the single-problem path bitwise."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, rel_max, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture()
def kp():
    import paper_2112_11238_amd as kp
    from paper_2112_11238_amd import tune
    tune.clear()
    yield kp
    tune.clear()


@pytest.mark.parametrize("dt,prec", [(torch.float64, "native"), (torch.float32, "native"),
                                     (torch.float32, "bf16x3")])
def test_autotune_then_tucker(kp, dt, prec):
    from paper_2112_11238_amd import tune
    T, Ls = kp_workloads.random_problem(41, (48, 40, 56), (36, 72, 20))
    Td, Ld = to_dev(T, dt), [to_dev(L, dt) for L in Ls]
    say("autotune", dt, prec)
    rec = tune.autotune(Td, Ld, prec=prec, backward=True, reps=3)
    assert len(rec) >= 3
    form = tune.form_code(dt, prec)
    names = set(tune.variants(form))
    for r in rec:
        assert r["tile"] in names and r["seconds"] > 0
        assert tune.lookup(form, r["Il"], r["m"], r["n"], r["Ir"]) == (True, r["tile"])
    # the calls now report (and use) the tuned tiles
    for p in tune.products(Td, Ld, prec) + tune.products(Td, Ld, prec, "backward"):
        assert tune.lookup(form, p["Il"], p["m"], p["n"], p["Ir"])[0]
    S = kp.tucker(Td, Ld, prec=prec)
    torch.cuda.synchronize()
    T64, L64 = cast64(T, dt), [cast64(L, dt) for L in Ls]
    ref = oracle.tucker(T64, L64)
    assert np.all(np.abs(S.double().cpu().numpy() - ref) <= chain_bound(T64, L64, prec, dt))
    G = np.random.default_rng(42).standard_normal(S.shape)
    dT, dLs = kp.tucker_backward(to_dev(G, dt), Td, Ld, prec)
    torch.cuda.synchronize()
    rT, rL = oracle.tucker_vjp(T64, L64, cast64(G, dt))
    tol = {torch.float64: 1e-12, torch.float32: 2e-5}[dt] * (20 if prec != "native" else 1)
    assert rel_max(dT.double().cpu().numpy(), rT) < tol
    for j in range(3):
        assert rel_max(dLs[j].double().cpu().numpy(), rL[j]) < 10 * tol


def test_tune_view_picks_its_fastest(kp):
    from paper_2112_11238_amd import tune
    best, sec, times = tune.tune_view(torch.float32, "native", 1, 64, 64, 4096, reps=3)
    assert best == min(times, key=times.get) and sec == times[best]
    assert set(times) == set(tune.variants("f32", m=64))
    bbest, _, btimes = tune.tune_view(torch.float32, "native", 64, 64, 64, 64,
                                      objective="throughput", reps=2, fill_fibers=1 << 18)
    assert set(btimes) == set(tune.variants("f32", batch=True, m=64))
    assert tune.lookup("f32", 64, 64, 64, 64)[1][:3] == bbest[:3]


def test_batched_after_throughput_tuning(kp):
    from paper_2112_11238_amd import tune
    rng = np.random.default_rng(43)
    probs = []
    for k in range(6):
        d = int(rng.integers(2, 5))
        m = tuple(int(x) for x in rng.integers(8, 40, size=d))
        probs.append(kp_workloads.random_problem(4300 + k, m, m))
    Td = [to_dev(T, torch.float32) for T, _ in probs]
    Ld = [[to_dev(L, torch.float32) for L in Ls] for _, Ls in probs]
    Gd = [torch.randn(T.shape, dtype=torch.float32, device="cuda") for T in Td]
    say("autotune_batch")
    rec = tune.autotune_batch(Td, Ld, backward=True, reps=2, fill_fibers=1 << 17)
    assert rec
    bt = kp.BatchedTucker(Td, Ld, Gs=Gd)
    bt.run()
    torch.cuda.synchronize()
    for k in range(len(Td)):
        ref = kp.tucker(Td[k], Ld[k])
        dT, dLs = kp.tucker_backward(Gd[k], Td[k], Ld[k])
        torch.cuda.synchronize()
        # same order (square factors) and, through the table, the same tiles
        assert torch.equal(bt.S[k], ref), k
        assert rel_max(bt.dT[k].double().cpu().numpy(), dT.double().cpu().numpy()) < 1e-5
        for j in range(len(dLs)):
            assert rel_max(bt.dL[k][j].double().cpu().numpy(),
                           dLs[j].double().cpu().numpy()) < 1e-4
