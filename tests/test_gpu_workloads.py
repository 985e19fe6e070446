"""Full-size parity of the Tucker operator on every workload, in the launch
configuration the benchmark times (default tiles, kp_tucker)."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, rel_max, say, to_dev, unit_error

pytestmark = pytest.mark.gpu

FORMS = [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16x6")]
DT = {"f64": torch.float64, "f32": torch.float32}
# precision targets of the method's forms (max-norm relative error)
TARGET = {("f64", "native"): 1e-13, ("f32", "native"): 1e-6, ("f32", "bf16x6"): 1e-6}


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


def run(kp, T, Ls, dt, prec):
    S = kp.tucker(to_dev(T, DT[dt]), [to_dev(L, DT[dt]) for L in Ls], prec=prec)
    torch.cuda.synchronize()
    return S


@pytest.mark.parametrize("dt,prec", FORMS)
def test_small2d(kp, dt, prec):
    T, Ls = kp_workloads.small2d()
    say("small2d", dt, prec)
    got = run(kp, T, Ls, dt, prec).double().cpu().numpy()
    T64, L64 = cast64(T, DT[dt]), [cast64(L, DT[dt]) for L in Ls]
    ref = oracle.tucker(T64, L64)
    assert np.all(np.abs(got - ref) <= chain_bound(T64, L64, prec, DT[dt]))
    if (dt, prec) in TARGET:
        assert rel_max(got, ref) <= TARGET[(dt, prec)]


@pytest.mark.parametrize("dt,prec", FORMS)
def test_cube200_full(kp, dt, prec):
    T, Ls = kp_workloads.cube200()
    say("cube200", dt, prec)
    got = run(kp, T, Ls, dt, prec).double().cpu().numpy()
    T64, L64 = cast64(T, DT[dt]), [cast64(L, DT[dt]) for L in Ls]
    ref = oracle.tucker(T64, L64)
    err = rel_max(got, ref)
    say("rel err", err)
    assert np.all(np.abs(got - ref) <= chain_bound(T64, L64, prec, DT[dt]))
    if (dt, prec) in TARGET:
        assert err <= TARGET[(dt, prec)]


@pytest.mark.parametrize("prec", ["native", "bf16x3", "bf16x6"])
def test_interp6d_sampled_entries(kp, prec):
    T, Ls = kp_workloads.interp6d()
    say("interp6d sampled", prec)
    S = run(kp, T, Ls, "f32", prec)
    T64 = cast64(T, torch.float32)
    L64 = [cast64(L, torch.float32) for L in Ls]
    rng = np.random.default_rng(77)
    idx = [tuple(int(v) for v in rng.integers(0, 24, size=6)) for _ in range(120)]
    idx += [(0,) * 6, (23,) * 6, (0, 23, 0, 23, 0, 23)]
    Sc = S.cpu()
    absT = np.abs(T64)
    absL = [np.abs(L) for L in L64]
    coef = 2 * 6 * {"native": 18 * 2.0 ** -24, "bf16x3": 3 * 2.0 ** -16 + 18 * 2.0 ** -24,
                    "bf16x6": 6 * 2.0 ** -24 + 18 * 2.0 ** -24}[prec]
    for i in idx:
        ref = oracle.tucker_entry(T64, L64, i)
        bound = coef * oracle.tucker_entry(absT, absL, i)
        assert abs(float(Sc[i]) - ref) <= bound, i


@pytest.mark.parametrize("prec", ["native", "bf16x6"])
def test_interp6d_polynomial_reproduction_full(kp, prec):
    # T samples a separable polynomial of degree <= 15 per variable at the 16
    # Chebyshev nodes; the Lagrange factors reproduce it exactly on the 24
    # uniform points, so S equals the polynomial on the full 24^6 grid.
    _, Ls = kp_workloads.interp6d()
    xi = oracle.chebyshev_nodes(16)
    x = np.linspace(-1, 1, 24)
    rng = np.random.default_rng(78)
    coefs = rng.standard_normal((6, 16)) / np.arange(1, 17)
    fn = [np.polyval(c, xi) for c in coefs]
    fx = [np.polyval(c, x) for c in coefs]
    T = fn[0]
    for k in range(1, 6):
        T = np.multiply.outer(T, fn[k])
    say("interp6d polynomial reproduction", prec)
    S = run(kp, T, Ls, "f32", prec)
    P = torch.tensor(fx[0], dtype=torch.float64, device="cuda")
    for k in range(1, 6):
        P = torch.multiply(P.unsqueeze(-1), torch.tensor(fx[k], dtype=torch.float64,
                                                           device="cuda"))
    err = float((S.double() - P).abs().max() / P.abs().max())
    say("rel err", err)
    # FP32 inputs and factors: relative error of a few units of 2^-24 per mode
    assert err < 2e-5


@pytest.mark.parametrize("prec", ["native", "bf16x3", "bf16x6"])
def test_batch64_each_tensor(kp, prec):
    sizes, items = kp_workloads.batch64()
    say("batch64 per tensor", prec)
    for k, (T, Ls) in enumerate(items):
        got = run(kp, T, Ls, "f32", prec).double().cpu().numpy()
        T64, L64 = cast64(T, torch.float32), [cast64(L, torch.float32) for L in Ls]
        if k % 8 == 0:
            ref = oracle.tucker(T64, L64)
            assert np.all(np.abs(got - ref) <= chain_bound(T64, L64, prec, torch.float32)), k
        else:
            coef = 2 * sum(unit_error(prec, torch.float32, int(s)) for s in sizes[k])
            for i in [tuple(int(s) // 2 for s in sizes[k]), tuple(int(s) - 1 for s in sizes[k])]:
                ref = oracle.tucker_entry(T64, L64, i)
                bnd = coef * oracle.tucker_entry(np.abs(T64), [np.abs(L) for L in L64], i)
                assert abs(got[i] - ref) <= bnd, (k, i)


@pytest.mark.parametrize("dt,prec", [("f64", "native"), ("f32", "bf16x3")])
def test_cube200_graph_replay(kp, dt, prec):
    """kp_tucker captured into a HIP graph (the benchmark's timed step):
    every replay, with eager library calls on other data and host
    synchronisations between replays, equals the eager result bitwise."""
    T, Ls = kp_workloads.cube200()
    Td = to_dev(T, DT[dt])
    Lds = [to_dev(L, DT[dt]) for L in Ls]
    want = kp.tucker(Td, Lds, prec=prec)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        kp.tucker(Td, Lds, prec=prec)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        Sg = kp.tucker(Td, Lds, prec=prec)
    T2, L2 = kp_workloads.random_problem(11, (30, 40, 50), (20, 35, 45))
    for r in range(3):
        say("graph replay", dt, prec, r)
        Sg.fill_(float("nan"))
        g.replay()
        other = kp.tucker(to_dev(T2, DT[dt]), [to_dev(L, DT[dt]) for L in L2], prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Sg, want), r
        assert torch.isfinite(other).all()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
def test_presplit_planes_bitwise(kp, prec):
    """BF16 products on wide tiles (n > 176) read factor planes split once
    per kp_tucker call. The same call with a workspace that holds only the
    intermediates (each tile then splits its rows itself) and the chain of
    kp_mump calls in kp_tucker's order must agree with it bit for bit, and
    all of them with the FP64 oracle within the split form's bound.
    Ragged sizes: rows past n in the last tile and a k tail in the last step."""
    import ctypes
    from paper_2112_11238_amd import ops
    rng = np.random.default_rng(29)
    tshape = (181, 200, 197)                 # torch order (mode d first)
    nrows = (204, 185, 200)                  # factor rows, torch order
    T = rng.standard_normal(tshape)
    Ls = [rng.standard_normal((nrows[j], tshape[j])) / np.sqrt(tshape[j]) for j in range(3)]
    Td = to_dev(T, torch.float32)
    Ld = [to_dev(L, torch.float32) for L in Ls]
    say("presplit planes", prec)
    S_full = kp.tucker(Td, Ld, prec=prec)

    # kp_tucker with a workspace that holds only the intermediates
    lb = ops.lib()
    td = ops._tdesc(ops._canon(Td), True)
    arr = ops._mlist([ops._mdesc(L) for L in Ld][::-1])
    p = ops._prec(prec)
    full = lb.kp_tucker_workspace(ctypes.byref(td), arr, p)
    S_inreg = torch.empty_like(S_full)
    sd = ops._tdesc(S_inreg, True)
    order = (ctypes.c_int * 8)()
    cnt = ctypes.c_int()
    assert lb.kp_tucker_order(ctypes.byref(td), arr, order, ctypes.byref(cnt)) == 0
    # intermediates only: the largest intermediate, twice (column-major dims)
    dims = list(tshape[::-1])
    nrev = list(nrows[::-1])
    big = 0
    for s in range(cnt.value - 1):
        k = order[s] - 1
        dims[k] = nrev[k]
        big = max(big, int(np.prod(dims)) * 4)
    inter = 2 * ((big + 255) // 256 * 256)
    assert inter < full                       # the planes take room of their own
    ws = torch.empty(inter, dtype=torch.uint8, device=Td.device)
    st = lb.kp_tucker(ctypes.byref(td), arr, ctypes.byref(sd), p, ws.data_ptr(), inter,
                      None, 0, ops._stream())
    assert st == 0
    # the same products one by one (torch mode index = d - column-major mode)
    X = Td
    for s in range(cnt.value):
        mu_cm = order[s]
        X = kp.mump(X, Ld[3 - mu_cm], 4 - mu_cm, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(S_full, S_inreg)
    assert torch.equal(S_full, X)
    T64, L64 = cast64(T, torch.float32), [cast64(L, torch.float32) for L in Ls]
    ref = oracle.tucker(T64, L64)
    assert np.all(np.abs(S_full.double().cpu().numpy() - ref)
                  <= chain_bound(T64, L64, prec, torch.float32))
