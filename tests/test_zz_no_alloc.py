"""kp_tucker_noalloc (intermediates in the library's fixed device buffer)
against kp_tucker (caller workspace) through the C-ABI: the same kernels in
the same order, so the results must be bitwise equal; both are also held to
the oracle's componentwise bound. Two calls in a row per case, the second on
a smaller problem, so the second call runs on a buffer that still holds the
first call's intermediates."""
import ctypes

import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, say, to_dev

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32}
# (dtype, prec, first problem (m, n), second (smaller) problem (m, n))
CASES = [
    ("f64", "native", ((200, 200, 200), (200, 200, 200)), ((37, 50, 23), (41, 17, 29))),
    ("f32", "bf16x6", ((64, 48, 80, 40), (72, 56, 40, 64)), ((9, 30, 17, 5), (12, 19, 33, 7))),
    ("f32", "native", ((16,) * 5, (24,) * 5), ((5, 7, 6), (8, 3, 9))),
    # wide tiles (n > 176) reading factor planes split into the scratch
    ("f32", "bf16x3", ((181, 200, 40), (204, 185, 30)), ((9, 30, 17), (12, 19, 33))),
]


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


def noalloc_call(kp, Td, Lds, prec):
    """kp_tucker_noalloc through the C-ABI on a preallocated output."""
    from paper_2112_11238_amd import _lib, ops
    d = Td.dim()
    shape = [Lds[k].shape[0] for k in range(d)]
    out = torch.empty(shape, dtype=Td.dtype, device=Td.device)
    mds = [ops._mdesc(L) for L in Lds][::-1]
    td, sd = ops._tdesc(Td, True), ops._tdesc(out, True)
    st = _lib.load().kp_tucker_noalloc(ctypes.byref(td), ops._mlist(mds), ctypes.byref(sd),
                                       ops._prec(prec), ops._stream())
    assert st == 0, _lib.STATUS.get(st, st)
    return out


@pytest.mark.parametrize("dt,prec,first,second", CASES)
def test_noalloc_matches_workspace_path(kp, dt, prec, first, second):
    from paper_2112_11238_amd import _lib
    assert _lib.load().kp_noalloc_scratch_bytes() == 128 << 20
    for seed, (m, n) in enumerate((first, second)):
        say("noalloc", dt, prec, m, "->", n)
        T, Ls = kp_workloads.random_problem(100 + seed, m, n)
        Td = to_dev(T, DT[dt])
        Lds = [to_dev(L, DT[dt]) for L in Ls]
        got = noalloc_call(kp, Td, Lds, prec)
        want = kp.tucker(Td, Lds, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(got, want), "noalloc result differs from kp_tucker's"
        T64, L64 = cast64(T, DT[dt]), [cast64(L, DT[dt]) for L in Ls]
        ref = oracle.tucker(T64, L64)
        g = got.double().cpu().numpy()
        assert np.all(np.abs(g - ref) <= chain_bound(T64, L64, prec, DT[dt]))


def test_noalloc_binding_with_out(kp):
    """The ops wrapper with a caller-provided output (no allocation at all)."""
    T, Ls = kp_workloads.random_problem(7, (30, 20, 10), (10, 25, 12))
    Td = to_dev(T, torch.float64)
    Lds = [to_dev(L, torch.float64) for L in Ls]
    out = torch.full((10, 25, 12), float("nan"), dtype=torch.float64, device="cuda")
    r = kp.tucker_noalloc(Td, Lds, out=out)
    want = kp.tucker(Td, Lds)
    torch.cuda.synchronize()
    assert r is out and torch.equal(out, want)
