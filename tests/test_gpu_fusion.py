"""Fused pairs of consecutive modes (KP_OPT_FUSE): the fused Tucker operator
equals the mode-by-mode one bitwise (same sums, same rounding of the
intermediate) and the FP64 oracle within the chain bound."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, say, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    # torch shapes m, n; at least one pair of consecutive short modes (m <= 16,
    # n <= 32) applied back to back: strided pairs (I_l > 1) and, where the
    # two leading modes go last, the lead-layout pair (I_l = 1)
    ((6, 7, 16, 16, 16), (6, 7, 24, 24, 24)),
    ((5, 9, 13, 11, 7), (6, 10, 15, 14, 9)),
    ((3, 16, 16, 16, 16), (3, 24, 24, 24, 24)),
    ((40, 2, 3, 33), (41, 3, 4, 34)),
    ((30, 3, 5, 7), (31, 4, 6, 9)),
    # lead-layout pairs: 16-byte loads and stores (m1, n1 multiples of 4) ...
    ((3, 20, 9, 12), (3, 7, 9, 12)),
    ((50, 16, 16), (20, 32, 24)),
    # ... element loads and stores, three fibers (not a multiple of a workgroup)
    ((30, 6, 13), (11, 6, 13)),
    ((5, 4, 7), (3, 5, 9)),
]
LEAD_CASES = [0, 2, 5, 6, 7, 8]  # cases whose chain has the lead-layout pair


@pytest.fixture()
def kp():
    import paper_2112_11238_amd as kp
    from paper_2112_11238_amd import _lib
    lib = _lib.load()
    yield kp
    lib.kp_set_option(_lib.KP_OPT_FUSE, 1)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_split_forms_against_oracle(kp, case, prec):
    """The BF16 split forms fuse pairs too: the fused chain within the form's
    componentwise bound of the oracle, and within twice that bound of the
    unfused chain (the fused pass takes the 16-long bf16 MFMA where the
    unfused kernels zero-pad a 32-long one: equal up to rounding)."""
    from paper_2112_11238_amd import _lib, tune
    lib = _lib.load()
    m, n = CASES[case]
    T, Ls = kp_workloads.random_problem(6100 + case, m, n)
    Td = to_dev(T, torch.float32)
    Ld = [to_dev(L, torch.float32) for L in Ls]
    launches = tune.products(Td, Ld, prec, which="launches")
    assert any(p["kind"] == 2 for p in launches), launches
    say("fusion", prec, m, n, [p["kind"] for p in launches])
    S_f = kp.tucker(Td, Ld, prec=prec)
    torch.cuda.synchronize()
    assert lib.kp_set_option(_lib.KP_OPT_FUSE, 0) == 0
    S_u = kp.tucker(Td, Ld, prec=prec)
    torch.cuda.synchronize()
    T64, L64 = cast64(T, torch.float32), [cast64(L, torch.float32) for L in Ls]
    ref = oracle.tucker(T64, L64)
    bound = chain_bound(T64, L64, prec, torch.float32)
    got_f = S_f.double().cpu().numpy()
    assert np.all(np.abs(got_f - ref) <= bound)
    assert np.all(np.abs(got_f - S_u.double().cpu().numpy()) <= 2 * bound)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_equals_unfused_and_oracle(kp, case):
    from paper_2112_11238_amd import _lib, tune
    lib = _lib.load()
    m, n = CASES[case]
    T, Ls = kp_workloads.random_problem(6000 + case, m, n)
    Td = to_dev(T, torch.float32)
    Ld = [to_dev(L, torch.float32) for L in Ls]
    if case == 1:   # a factor given as a transposed (non-contiguous) view
        Ld[3] = Ld[3].t().contiguous().t()
    launches = tune.products(Td, Ld, which="launches")
    assert any(p["kind"] == 2 for p in launches), launches
    if case in LEAD_CASES:
        assert any(p["kind"] == 2 and p["Il"] == 1 for p in launches), launches
    say("fusion", m, n, [(p["kind"], p["Il"]) for p in launches])
    S_f = kp.tucker(Td, Ld)
    torch.cuda.synchronize()
    assert lib.kp_set_option(_lib.KP_OPT_FUSE, 0) == 0
    assert all(p["kind"] != 2 for p in tune.products(Td, Ld, which="launches"))
    S_u = kp.tucker(Td, Ld)
    torch.cuda.synchronize()
    assert torch.equal(S_f, S_u)
    T64, L64 = cast64(T, torch.float32), [cast64(L, torch.float32) for L in Ls]
    ref = oracle.tucker(T64, L64)
    assert np.all(np.abs(S_f.double().cpu().numpy() - ref) <= chain_bound(T64, L64, "native",
                                                                         torch.float32))


def test_fused_interp6d_full_size(kp):
    """The 16^6 -> 24^6 interpolation: three fused passes, the last (writing
    the 24^6 result) on the lead layout; result equal to the unfused chain."""
    from paper_2112_11238_amd import _lib, tune
    lib = _lib.load()
    T, Ls = kp_workloads.interp6d(seed=0)
    Td = to_dev(T, torch.float32)
    Ld = [to_dev(L, torch.float32) for L in Ls]
    launches = tune.products(Td, Ld, which="launches")
    say("fusion interp6d", [(p["kind"], p["Il"]) for p in launches])
    assert [p["kind"] for p in launches] == [2, 2, 2] and launches[-1]["Il"] == 1
    S_f = kp.tucker(Td, Ld)
    torch.cuda.synchronize()
    lib.kp_set_option(_lib.KP_OPT_FUSE, 0)
    S_u = kp.tucker(Td, Ld)
    torch.cuda.synchronize()
    assert torch.equal(S_f, S_u)


@pytest.mark.parametrize("m,n", [((16, 16, 16, 16), (24, 24, 24, 24)),
                                 ((10, 12, 13), (12, 20, 28)),
                                 ((4, 4, 4, 4, 4), (6, 6, 6, 6, 6))])
def test_fused_backward_step(kp, m, n):
    """FP32 backward: on short modes with I_l a multiple of 4 the factor
    gradient and the next cotangent come from one pass over Q_mu. The
    cotangent sweep (dT) equals the unfused one bitwise (same products, same
    order); dL differs from it only in how the fiber sum is split, and both
    meet the oracle within the chain bound."""
    from paper_2112_11238_amd import _lib
    from test_gpu_backward import grad_bounds
    lib = _lib.load()
    T, Ls = kp_workloads.random_problem(6200 + len(m), m, n)
    G = np.random.default_rng(6300 + len(m)).standard_normal(n)
    Td, Gd = to_dev(T, torch.float32), to_dev(G, torch.float32)
    Ld = [to_dev(L, torch.float32) for L in Ls]
    say("fused backward", m, n)
    dT_f, dL_f = kp.tucker_backward(Gd, Td, Ld)
    torch.cuda.synchronize()
    assert lib.kp_set_option(_lib.KP_OPT_FUSE, 0) == 0
    dT_u, dL_u = kp.tucker_backward(Gd, Td, Ld)
    torch.cuda.synchronize()
    assert torch.equal(dT_f, dT_u)
    T64, G64 = cast64(T, torch.float32), cast64(G, torch.float32)
    L64 = [cast64(L, torch.float32) for L in Ls]
    rT, rL = oracle.tucker_vjp(T64, L64, G64)
    bT, bL = grad_bounds(T64, L64, G64, "native", "f32")
    assert np.all(np.abs(dT_f.double().cpu().numpy() - rT) <= bT)
    for k in range(len(m)):
        for got in (dL_f[k], dL_u[k]):
            g = got.double().cpu().numpy()
            assert np.all(np.abs(g - rL[k]) <= bL[k]), (k, float(np.max(np.abs(g - rL[k]) / bL[k])))


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("m,n", [((16, 16, 16, 16), (24, 24, 24, 24)),
                                 ((10, 12, 13), (12, 20, 28))])
def test_fused_backward_step_split_forms(kp, m, n, prec):
    """The fused backward step in the BF16 split forms: the product takes the
    16-long bf16 MFMA where the unfused kernels zero-pad a 32-long one, so dT
    agrees with the unfused sweep to rounding; both sweeps and every factor
    gradient meet the oracle within the form's chain bound."""
    from paper_2112_11238_amd import _lib
    from test_gpu_backward import grad_bounds
    lib = _lib.load()
    T, Ls = kp_workloads.random_problem(6400 + len(m), m, n)
    G = np.random.default_rng(6500 + len(m)).standard_normal(n)
    Td, Gd = to_dev(T, torch.float32), to_dev(G, torch.float32)
    Ld = [to_dev(L, torch.float32) for L in Ls]
    say("fused backward", prec, m, n)
    dT_f, dL_f = kp.tucker_backward(Gd, Td, Ld, prec)
    torch.cuda.synchronize()
    assert lib.kp_set_option(_lib.KP_OPT_FUSE, 0) == 0
    dT_u, dL_u = kp.tucker_backward(Gd, Td, Ld, prec)
    torch.cuda.synchronize()
    T64, G64 = cast64(T, torch.float32), cast64(G, torch.float32)
    L64 = [cast64(L, torch.float32) for L in Ls]
    rT, rL = oracle.tucker_vjp(T64, L64, G64)
    bT, bL = grad_bounds(T64, L64, G64, prec, "f32")
    for got in (dT_f, dT_u):
        assert np.all(np.abs(got.double().cpu().numpy() - rT) <= bT)
    for k in range(len(m)):
        for got in (dL_f[k], dL_u[k]):
            g = got.double().cpu().numpy()
            assert np.all(np.abs(g - rL[k]) <= bL[k]), (k, float(np.max(np.abs(g - rL[k]) / bL[k])))
