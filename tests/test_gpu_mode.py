"""GPU parity of the mu-mode product and the Tucker operator against the FP64
oracle, element by element, through the C-ABI (libkp.so)."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import cast64, chain_bound, rel_max, say, to_dev

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32}
FORMS = [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16x6")]


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


def run_mump(kp, T, L, mu, dt, prec):
    Td, Ld = to_dev(T, DT[dt]), to_dev(L, DT[dt])
    S = kp.mump(Td, Ld, mu, prec=prec)
    torch.cuda.synchronize()
    return S.double().cpu().numpy(), cast64(T, DT[dt]), cast64(L, DT[dt])


# shapes spanning several tiles, ragged tails, size-1 modes, primes, n > 256
MUMP_CASES = [
    ((37,), (53,)),
    ((50, 50), (50, 50)),
    ((1, 7), (3, 1)),
    ((70, 33), (65, 17)),
    ((5, 66, 3), (17, 9, 2)),
    ((20, 31, 17), (33, 20, 5)),
    ((3, 1, 4, 9), (2, 5, 4, 3)),
    ((9, 130, 7), (300, 211, 40)),
    ((64, 16, 5), (24, 200, 129)),
]


@pytest.mark.parametrize("dt,prec", FORMS)
@pytest.mark.parametrize("case", range(len(MUMP_CASES)))
def test_mump_matches_oracle(kp, dt, prec, case):
    m, n = MUMP_CASES[case]
    d = len(m)
    for mu in range(1, d + 1):
        T, Ls = kp_workloads.random_problem(1000 + case, m, n)
        L = Ls[mu - 1]
        say("mump", m, n, "mu", mu, dt, prec)
        S, T64, L64 = run_mump(kp, T, L, mu, dt, prec)
        ref = oracle.mump(T64, L64, mu)
        factors = [None] * d
        factors[mu - 1] = L64
        bound = chain_bound(T64, factors, prec, DT[dt])
        assert S.shape == ref.shape
        assert np.all(np.abs(S - ref) <= bound), (mu, float(np.max(np.abs(S - ref) / bound)))


@pytest.mark.parametrize("dt,prec", FORMS)
def test_mump_accumulate(kp, dt, prec):
    m, n = (6, 40, 11), (6, 30, 11)
    T, Ls = kp_workloads.random_problem(7, m, n)
    rng = np.random.default_rng(8)
    S0 = rng.standard_normal(n)
    say("mump accumulate", dt, prec)
    out = to_dev(S0, DT[dt])
    kp.mump(to_dev(T, DT[dt]), to_dev(Ls[1], DT[dt]), 2, prec=prec, out=out, accumulate=True)
    torch.cuda.synchronize()
    ref = cast64(S0, DT[dt]) + oracle.mump(cast64(T, DT[dt]), cast64(Ls[1], DT[dt]), 2)
    tol = 1e-13 if dt == "f64" else 1e-4
    assert rel_max(out.double().cpu().numpy(), ref) < tol


# Views whose default tile comes from the size rules (inner layout over more
# than 64K fibers, short contractions): torch shape (Ir, m, Il), factor
# (n, m), mode 2; with the tile kind the default must pick (0 k-loop,
# 1 strip) and a view a strip covers that stays on it (lead layout)
RULE_CASES = [
    ("f32", (3000, 24, 24), 40, 0),     # FP32 16 < m, 16 < n <= 64: k-loop
    ("f32", (1500, 45, 45), 35, 0),     # FP32 m = 45 (the Runge modes)
    ("f64", (4000, 18, 18), 18, 0),     # FP64 16 < m <= 24: 8-wide chunks
    ("f64", (3000, 28, 28), 28, 0),     # FP64 24 < m <= 32
    ("f32", (37500, 14, 14), 14, 1),    # FP32 m < 16 over >= 512K fibers: strip
    ("f32", (13824, 24, 16), 16, 1),    # FP32 n <= 16: the strip stays
    ("f64", (50000, 18, 1), 18, 1),     # lead layout: the strip stays
]


@pytest.mark.parametrize("case", range(len(RULE_CASES)))
def test_mump_default_tile_rules(kp, case):
    dt, shape, n, kind = RULE_CASES[case]
    Ir, m, Il = shape
    rng = np.random.default_rng(300 + case)
    T = rng.standard_normal(shape)
    L = rng.standard_normal((n, m))
    form = "f64" if dt == "f64" else "f32"
    assert kp.tune.lookup(form, Il, m, n, Ir)[1][5] == kind
    say("mump default rule", dt, shape, n, "kind", kind)
    S, T64, L64 = run_mump(kp, T, L, 2, dt, "native")
    ref = oracle.mump(T64, L64, 2)
    factors = [None, L64, None]
    bound = chain_bound(T64, factors, "native", DT[dt])
    assert np.all(np.abs(S - ref) <= bound), float(np.max(np.abs(S - ref) / bound))


# Tensors past 2 GiB: each launch addresses its operands with 32-bit byte
# offsets, so the product is split along the outer index b into pieces below
# 2^31 bytes. torch shape (Ir, m, Il), factor (n, m), mode 2, and the first
# b of the second piece: floor((2^31 - 1) / (Il * max(m, n) * bytes)).
BIG_CASES = [
    ("f64", (1500, 200, 1000), 150),      # inner, k-loop tile
    ("f64", (1_500_000, 200, 1), 150),    # lead, k-loop tile
    ("f64", (8_000_000, 40, 1), 40),      # lead, 48-long strip
    ("f32", (3000, 200, 1000), 100),      # inner, FP32 k-loop tile
]


@pytest.mark.parametrize("case", range(len(BIG_CASES)))
def test_mump_beyond_2gib_sampled(kp, case):
    from gpu_util import unit_error
    dt, (Ir, m, Il), n = BIG_CASES[case]
    es = 8 if dt == "f64" else 4
    assert Ir * m * Il * es > 2 ** 31
    per = (2 ** 31 - 1) // (Il * max(m, n) * es)
    assert 0 < per < Ir
    say("mump beyond 2 GiB", dt, (Ir, m, Il), n, "piece", per)
    g = torch.Generator(device="cuda").manual_seed(500 + case)
    X = torch.randn((Ir, m, Il), dtype=DT[dt], device="cuda", generator=g)
    L = torch.randn((n, m), dtype=DT[dt], device="cuda", generator=g)
    Y = kp.mump(X, L, 2)
    torch.cuda.synchronize()
    rng = np.random.default_rng(600 + case)
    bs = np.unique(np.concatenate([[0, per - 1, per, per + 1, Ir - 1],
                                   rng.integers(0, Ir, 40)]))
    As = np.unique(np.concatenate([[0, Il - 1], rng.integers(0, Il, 8)]))
    bi = torch.as_tensor(bs, device="cuda")
    ai = torch.as_tensor(As, device="cuda")
    xs = X[bi][:, :, ai].double().cpu().numpy()      # (nb, m, na)
    ys = Y[bi][:, :, ai].double().cpu().numpy()      # (nb, n, na)
    L64 = L.double().cpu().numpy()
    ref = np.einsum("ij,bja->bia", L64, xs)
    bound = 2 * unit_error("native", DT[dt], m) * np.einsum("ij,bja->bia", np.abs(L64),
                                                               np.abs(xs)) + 1e-300
    assert np.all(np.abs(ys - ref) <= bound), float(np.max(np.abs(ys - ref) / bound))
    del X, Y
    torch.cuda.empty_cache()


def test_mump_empty_contraction_gives_zeros(kp):
    # m_mu = 0: every output entry is an empty sum.
    T = np.zeros((3, 0, 4))
    L = np.zeros((5, 0))
    say("mump empty contraction")
    S = kp.mump(to_dev(T, torch.float64), to_dev(L, torch.float64), 2)
    torch.cuda.synchronize()
    assert S.shape == (3, 5, 4)
    assert torch.count_nonzero(S).item() == 0


def test_mump_empty_output(kp):
    T = np.zeros((3, 5, 0))
    L = np.ones((4, 5))
    say("mump empty output")
    S = kp.mump(to_dev(T, torch.float32), to_dev(L, torch.float32), 2)
    torch.cuda.synchronize()
    assert S.shape == (3, 4, 0)


def test_mump_strided_factor(kp):
    # L given as a transposed view (column strides), as the backward uses it.
    T, Ls = kp_workloads.random_problem(9, (12, 33, 7), (12, 21, 7))
    Lt = to_dev(Ls[1].T.copy(), torch.float64).t()   # (21, 33) with strides (1, 21)
    say("mump strided factor")
    S = kp.mump(to_dev(T, torch.float64), Lt, 2)
    torch.cuda.synchronize()
    assert rel_max(S.cpu().numpy(), oracle.mump(T, Ls[1], 2)) < 1e-13


# every compiled tile variant, both layouts
TILES = {
    "native64": [(1, 4, 16, 1), (2, 2, 16, 2), (4, 1, 16, 2), (7, 1, 16, 2), (8, 1, 16, 2),
                 (13, 1, 16, 2), (7, 1, 8, 2), (7, 1, 8, 3), (4, 1, 8, 3), (8, 1, 8, 3),
                 (2, 2, 8, 3), (13, 1, 8, 2), (7, 1, 16, 2, 2), (7, 1, 8, 2, 2), (4, 1, 16, 2, 2)],
    "native32": [(1, 4, 16, 2), (2, 4, 16, 2), (2, 2, 16, 2), (4, 2, 16, 2), (4, 1, 16, 2),
                 (8, 1, 16, 2), (7, 2, 16, 2), (13, 1, 16, 2), (4, 1, 16, 2, 2), (7, 1, 16, 2, 2),
                 (8, 1, 16, 2, 2)],
    "bf16x3": [(1, 4, 32, 2), (2, 4, 32, 2), (2, 2, 32, 2), (4, 2, 32, 2), (4, 1, 32, 2),
               (8, 1, 32, 2), (7, 1, 32, 2), (1, 2, 32, 2), (2, 1, 32, 2), (4, 1, 32, 2, 2),
               (2, 4, 32, 2, 2, 3), (4, 2, 32, 2, 2, 3), (4, 4, 32, 1, 2, 3)],
    "bf16x6": [(1, 4, 32, 2), (2, 4, 32, 2), (2, 2, 32, 2), (4, 2, 32, 2), (4, 1, 32, 2),
               (8, 1, 32, 2), (1, 2, 32, 2), (2, 1, 32, 2), (4, 1, 32, 2, 2),
               (2, 4, 32, 2, 2, 3), (4, 2, 32, 2, 2, 3), (4, 4, 32, 1, 2, 3)],
}


@pytest.mark.parametrize("dt,prec", FORMS)
@pytest.mark.parametrize("shape", ["ragged", "aligned", "quad"])
def test_every_tile_variant(kp, dt, prec, shape):
    # ragged: m not a multiple of the load group (element-wise loads);
    # aligned: contiguous factors with m a multiple of 8 and 16-byte rows, so
    # the 16-byte group loads run (with a k tail of whole groups);
    # quad: m a multiple of 4 but not of 8, so the BF16 forms' 8-element
    # groups straddle k = m and their second 16-byte piece reads as zero
    key = prec if prec != "native" else ("native64" if dt == "f64" else "native32")
    m = {"ragged": (19, 45, 13), "aligned": (24, 40, 16), "quad": (20, 44, 12)}[shape]
    n = (7, 70, 29)
    T, Ls = kp_workloads.random_problem(11, m, n)
    T64 = cast64(T, DT[dt])
    try:
        for tile in TILES[key]:
            kp.force_tile(*tile)
            for mu in (1, 2, 3):
                L64 = cast64(Ls[mu - 1], DT[dt])
                say("tile", tile, dt, prec, "mu", mu)
                S = kp.mump(to_dev(T, DT[dt]), to_dev(Ls[mu - 1], DT[dt]), mu, prec=prec)
                torch.cuda.synchronize()
                ref = oracle.mump(T64, L64, mu)
                f = [None] * 3
                f[mu - 1] = L64
                bound = chain_bound(T64, f, prec, DT[dt])
                assert np.all(np.abs(S.double().cpu().numpy() - ref) <= bound), (tile, mu)
    finally:
        kp.force_tile(0)


def strip_cases(kp_len):
    """(torch shape, mode, layout) cases for a strip of padded length kp_len:
    the lead layout with m = kp_len (16-byte loads), with a k tail and with a
    tail of whole 16-byte pieces (m = kp_len - 4), the
    innermost-strided layout and a middle mode; enough fibers that every
    workgroup streams several tiles."""
    m = kp_len
    return [((150001, m), 2, "lead"), ((150001, m - 3), 2, "lead tail"),
            ((150001, m - 4), 2, "lead 16-byte tail"),
            ((m - 1, 300, 500), 1, "inner"), ((40, m, 3750), 2, "middle")]


@pytest.mark.parametrize("dt,prec", FORMS)
def test_every_strip_variant(kp, dt, prec):
    from paper_2112_11238_amd import tune
    form = tune.form_code(DT[dt], prec)
    strips = [v for v in tune.variants(form) if v[5] == 1]
    assert strips
    rng = np.random.default_rng(77)
    try:
        for tile in strips:
            nb, fb, klen = tile[0], tile[1], tile[2]
            n = 16 * nb * 2 + 5            # three n blocks, the last one ragged
            for shape, mu, what in strip_cases(klen):
                T = rng.standard_normal(shape)
                Lm = rng.standard_normal((n, shape[mu - 1]))
                T64, L64 = cast64(T, DT[dt]), cast64(Lm, DT[dt])
                say("strip", tile, dt, prec, shape, mu, what)
                kp.force_tile(*tile)
                S = kp.mump(to_dev(T, DT[dt]), to_dev(Lm, DT[dt]), mu, prec=prec)
                torch.cuda.synchronize()
                kp.force_tile(0)
                ref = oracle.mump(T64, L64, mu)
                f = [None] * len(shape)
                f[mu - 1] = L64
                bound = chain_bound(T64, f, prec, DT[dt])
                assert np.all(np.abs(S.double().cpu().numpy() - ref) <= bound), (tile, what)
    finally:
        kp.force_tile(0)


TUCKER_CASES = [
    ((50, 50), (50, 50)),
    ((4, 5, 6), (7, 3, 9)),
    ((17, 1, 33, 2), (5, 4, 40, 3)),
    ((6, 5, 4, 3, 2), (2, 3, 4, 5, 6)),
    ((4, 4, 4, 4, 4, 4), (6, 6, 6, 6, 6, 6)),
]


@pytest.mark.parametrize("dt,prec", FORMS)
@pytest.mark.parametrize("case", range(len(TUCKER_CASES)))
def test_tucker_matches_oracle(kp, dt, prec, case):
    m, n = TUCKER_CASES[case]
    T, Ls = kp_workloads.random_problem(2000 + case, m, n)
    say("tucker", m, n, dt, prec)
    S = kp.tucker(to_dev(T, DT[dt]), [to_dev(L, DT[dt]) for L in Ls], prec=prec)
    torch.cuda.synchronize()
    T64 = cast64(T, DT[dt])
    L64 = [cast64(L, DT[dt]) for L in Ls]
    ref = oracle.tucker(T64, L64)
    bound = chain_bound(T64, L64, prec, DT[dt])
    got = S.double().cpu().numpy()
    assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))


def test_tucker_identity_factors(kp):
    T, Ls = kp_workloads.random_problem(3000, (5, 6, 7), (5, 8, 7))
    say("tucker identity factors")
    Td = to_dev(T, torch.float64)
    S = kp.tucker(Td, [None, to_dev(Ls[1], torch.float64), None])
    torch.cuda.synchronize()
    assert rel_max(S.cpu().numpy(), oracle.mump(T, Ls[1], 2)) < 1e-13
    S2 = kp.tucker(Td, [None, None, None])
    torch.cuda.synchronize()
    assert torch.equal(S2, Td)
