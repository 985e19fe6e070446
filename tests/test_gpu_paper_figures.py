"""The paper's figures on the device: the 5-D Runge interpolation errors
(Sec. 4.3) and the shapes of its Tucker timing sweep (Sec. 4.1), each checked
against the oracle (full tensors where it is quick, sampled entries at the
largest sizes) and against the values the paper prints."""
import json
import os

import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import chain_bound, say, to_dev, unit_error

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "lagrange_runge5d.json")


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


def _golden():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    return list(zip(g["m"], g["relative_error_printed"]))


@pytest.mark.parametrize("m,printed", _golden())
def test_runge5d_errors_match_printed(kp, m, printed):
    F, Ls, x = kp_workloads.runge5d(m)
    say("runge5d", m)
    S = kp.tucker(to_dev(F, torch.float64), [to_dev(L, torch.float64) for L in Ls])
    torch.cuda.synchronize()
    got = S.cpu().numpy()
    f = oracle.runge(*([x] * 5))
    err = np.abs(got - f).max() / np.abs(f).max()
    say("rel err", err)
    assert float(f"{err:.3g}") == pytest.approx(printed, rel=1e-9), err
    if m <= 25:
        ref = oracle.tucker(F, Ls)
        assert np.all(np.abs(got - ref) <= chain_bound(F, Ls, "native", torch.float64))
    else:
        rng = np.random.default_rng(m)
        idx = [tuple(int(v) for v in rng.integers(0, 35, size=5)) for _ in range(6)]
        idx += [(0,) * 5, (34,) * 5, (17,) * 5]
        absL = [np.abs(L) for L in Ls]
        coef = 2 * 5 * unit_error("native", torch.float64, m)
        for i in idx:
            ref = oracle.tucker_entry(F, Ls, i)
            assert abs(got[i] - ref) <= coef * oracle.tucker_entry(np.abs(F), absL, i), i


@pytest.mark.parametrize("d,n", kp_workloads.codeval_shapes())
@pytest.mark.parametrize("dt,prec", [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"),
                                     ("f32", "bf16x6")])
def test_codeval_shapes_sampled(kp, d, n, dt, prec):
    T, Ls = kp_workloads.cube(seed=n, n=n, d=d)
    tdt = torch.float64 if dt == "f64" else torch.float32
    say("codeval", d, n, dt, prec)
    S = kp.tucker(to_dev(T, tdt), [to_dev(L, tdt) for L in Ls], prec=prec)
    torch.cuda.synchronize()
    Sc = S.double().cpu().numpy()
    T64 = torch.as_tensor(T).to(tdt).double().numpy()
    L64 = [torch.as_tensor(L).to(tdt).double().numpy() for L in Ls]
    rng = np.random.default_rng(1000 * d + n)
    idx = [tuple(int(v) for v in rng.integers(0, n, size=d)) for _ in range(24)]
    idx += [(0,) * d, (n - 1,) * d]
    absT, absL = np.abs(T64), [np.abs(L) for L in L64]
    coef = 2 * d * unit_error(prec, tdt, n)
    for i in idx:
        ref = oracle.tucker_entry(T64, L64, i)
        assert abs(Sc[i] - ref) <= coef * oracle.tucker_entry(absT, absL, i), i
