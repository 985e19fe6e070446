"""Host-side checks of the tile table and the tuning helpers (no kernel is
launched): validation, lookup, listing, the product views a call reports,
and that the batched planner takes its tiles from the table."""
import ctypes
import itertools
import json

import numpy as np
import pytest
import torch

from test_abi_host import matrix, mlist, no_device, tensor
from test_batch_plan_host import make_items, plan, Alloc


@pytest.fixture(scope="module")
def L():
    from paper_2112_11238_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def lib(L):
    return L.load()


@pytest.fixture()
def tune(lib):
    from paper_2112_11238_amd import tune as t
    t.clear()
    yield t
    t.clear()


def entry(L, form, Il, m, n, Ir, tile):
    e = L.KpTuneEntry()
    e.form, e.Il, e.m, e.n, e.Ir = form, Il, m, n, Ir
    t = tuple(tile) + (0,) * (6 - len(tile))
    e.nb, e.fb, e.bk, e.occ, e.pf, e.kind = t
    return e


def test_variant_lists(lib, tune):
    for form in (0, 1, 3, 6):
        mode = tune.variants(form)
        assert len(mode) >= 10
        assert len(set(mode)) == len(mode)
        bk = 16 if form in (0, 1) else 32
        assert any(v[2] == bk for v in mode)
        # every tile of the batched executor has a standalone kernel with the
        # same (nb, fb, bk): the throughput tuner times it there
        for v in tune.variants(form, batch=True):
            assert v[3:5] == (0, 0)
            assert any(w[:3] == v[:3] and w[5] == v[5] for w in mode), (form, v)
        # strip tiles (kind 1): occ = pf = 0, bk the padded contraction length
        strips = [v for v in mode if v[5] == 1]
        assert strips and all(v[3:5] == (0, 0) and v[2] in (16, 32, 48, 64) for v in strips)
        assert any(v[2] == 48 for v in strips) == (form == 0)      # FP64 only
        assert all(v[5] != 1 or v[2] >= 40 for v in tune.variants(form, m=40))
        # wide tiles (kind 3): the BF16 split forms only, 32-wide k steps
        wide = [v for v in mode if v[5] == 3]
        assert (len(wide) > 0) == (form in (3, 6)) and all(v[2] == 32 and v[4] == 2 for v in wide)
        assert len(tune.variants(form, m=200)) == len(mode) - len(strips)
    assert lib.kp_tile_variants(2, 0, None, 0) == -9
    assert lib.kp_tile_variants(0, 2, None, 0) == -9
    assert lib.kp_tile_variants(0, 0, None, 5) == -1


def test_set_lookup_list_clear(lib, L, tune):
    assert lib.kp_tune_set(None) == -1
    assert lib.kp_tune_set(ctypes.byref(entry(L, 2, 1, 8, 8, 8, (4, 1, 16, 0, 0)))) == -9
    assert lib.kp_tune_set(ctypes.byref(entry(L, 0, 0, 8, 8, 8, (4, 1, 16, 0, 0)))) == -9
    assert lib.kp_tune_set(ctypes.byref(entry(L, 0, 1, 8, 8, 8, (5, 1, 16, 0, 0)))) == -9
    assert lib.kp_tune_set(ctypes.byref(entry(L, 0, 1, 8, 8, 8, (4, 1, 16, 0, 3)))) == -9
    assert lib.kp_tune_set(ctypes.byref(entry(L, 1, 1, 40, 8, 8, (2, 2, 32, 0, 0, 1)))) == -9
    assert lib.kp_tune_set(ctypes.byref(entry(L, 1, 1, 8, 8, 8, (2, 2, 32, 0, 0, 2)))) == -9
    assert lib.kp_tune_count() == 0
    # short contractions default to a strip tile covering m; on small
    # problems with fewer rows per workgroup, so the workgroups fill the chip
    tuned, tile = tune.lookup("f32", 1, 24, 40, 630000)
    assert not tuned and tile[5] == 1 and tile[2] >= 24 and 16 * tile[0] >= 32
    tuned, tile = tune.lookup("f32", 7, 24, 40, 9)
    assert not tuned and tile[5] == 1 and tile[2] >= 24 and tile[0] == 1
    # the inner layout over many fibers takes the k-loop tile for 16 < m
    # (FP32) and 16 < m <= 32 (FP64) when 16 < n <= 64, with 8-wide chunks
    # for FP64 m <= 24
    assert tune.lookup("f32", 24, 24, 16, 13824)[1][5] == 1
    assert tune.lookup("f32", 7, 24, 40, 90000) == (False, (4, 1, 16, 2, 1, 0))
    assert tune.lookup("f32", 45, 45, 35, 45 ** 3) == (False, (4, 1, 16, 2, 1, 0))
    assert tune.lookup("f64", 18, 18, 18, 18 ** 4) == (False, (2, 2, 8, 3, 1, 0))
    assert tune.lookup("f64", 28, 28, 28, 28 ** 3) == (False, (2, 2, 16, 2, 1, 0))
    assert tune.lookup("f64", 1, 18, 18, 18 ** 5)[1][5] == 1        # lead: a strip
    assert tune.lookup("f64", 18, 18, 18, 100)[1][5] == 1           # small: a strip
    # FP32 m < 16 over many fibers: the 16-long strip
    assert tune.lookup("f32", 14, 14, 14, 14 ** 4) == (False, (1, 2, 16, 0, 0, 1))
    assert tune.lookup("f32", 14, 14, 14, 14 ** 3)[1][5] == 0
    assert tune.lookup("f32", 16, 16, 16, 16 ** 4)[1][5] == 0
    tune.set_tile("f32", 7, 24, 40, 9, (1, 2, 32, 0, 0, 1))
    assert tune.lookup("f32", 7, 24, 40, 9) == (True, (1, 2, 32, 0, 0, 1))
    tune.clear()
    # default first
    tuned, tile = tune.lookup("f64", 40, 200, 200, 200)
    assert not tuned and tile[:3] == (7, 1, 8)
    # long FP64 contractions keep two chunks of loads in flight
    assert tune.lookup("f64", 1, 324, 324, 324 * 324) == (False, (7, 1, 8, 2, 2, 0))
    # FP64 with 32 < m <= 64: a strip on the lead layout, the k-loop tile inside
    assert tune.lookup("f64", 1, 45, 35, 10 ** 6) == (False, (4, 1, 48, 0, 0, 1))
    assert tune.lookup("f64", 1, 60, 64, 10 ** 6) == (False, (4, 1, 64, 0, 0, 1))
    assert tune.lookup("f64", 35, 45, 35, 10000)[1][5] == 0
    assert tune.lookup("f64", 35, 45, 35, 1000)[1][5] == 1          # small: a strip
    # small k-loop problems (64 < n <= 184) take smaller tiles
    assert tune.lookup("f64", 1, 128, 128, 128 * 128)[1][:3] == (4, 1, 16)
    assert tune.lookup("f64", 1, 200, 200, 200 * 200)[1][:3] == (7, 1, 8)
    # n > 184: shorter tiles where 7-block tiles would leave the last one
    # mostly empty (16-row blocks: 15, 16, 22, 24 for n = 240, 256, 352, 384)
    for n in (240, 256, 352, 384):
        assert tune.lookup("f64", n, n, n, n)[1] == (4, 1, 16, 2, 2, 0)
        assert tune.lookup("f32", n, n, n, n)[1] == (8, 1, 16, 2, 2, 0)
    for n in (200, 272, 288, 320, 324):
        assert tune.lookup("f64", n, n, n, n)[1][0] == 7
        assert tune.lookup("f32", n, n, n, n)[1][0] == 7
    tune.set_tile("f64", 40, 200, 200, 200, (4, 1, 16))
    tuned, tile = tune.lookup("f64", 40, 200, 200, 200)
    assert tuned and tile[:3] == (4, 1, 16) and tile[3] > 0 and tile[4:] == (1, 0)  # resolved
    tune.set_tile("f64", 40, 200, 200, 200, (7, 1, 8, 2, 2))     # replace
    assert tune.lookup("f64", 40, 200, 200, 200) == (True, (7, 1, 8, 2, 2, 0))
    assert tune.lookup("f32", 40, 200, 200, 200)[0] is False      # the form is in the key
    # a view without an entry takes its shape class's: same form, layout, m
    # and n, fiber count within a factor of two, the nearest in ratio
    assert tune.lookup("f64", 41, 200, 200, 200) == (True, (7, 1, 8, 2, 2, 0))
    assert tune.lookup("f64", 40, 200, 200, 399) == (True, (7, 1, 8, 2, 2, 0))
    assert tune.lookup("f64", 40, 200, 200, 401)[0] is False      # 2.005 x the fibers
    assert tune.lookup("f64", 40, 200, 200, 99)[0] is False
    assert tune.lookup("f64", 1, 200, 200, 8000)[0] is False      # lead layout: own class
    assert tune.lookup("f64", 40, 200, 208, 200)[0] is False      # n is in the class
    tune.set_tile("f64", 40, 200, 200, 300, (4, 1, 16))
    assert tune.lookup("f64", 40, 200, 200, 260)[1][:3] == (4, 1, 16)   # 1.15 x vs 1.3 x
    assert tune.lookup("f64", 40, 200, 200, 240)[1][:3] == (7, 1, 8)    # 1.2 x vs 1.25 x
    tune.set_tile("f64", 40, 200, 200, 300, (7, 1, 8, 2, 2))     # back to one class tile
    assert lib.kp_tune_count() == 2
    tune.clear()
    tune.set_tile("f64", 40, 200, 200, 200, (7, 1, 8, 2, 2))
    tune.set_tile("bf16x3", 1, 30, 20, 1000, (2, 2, 32))
    ents = tune.entries()
    assert len(ents) == 2 == lib.kp_tune_count()
    assert [e["form"] for e in ents] == [0, 3]                    # key order
    assert lib.kp_tune_list(None, 0) == 2
    tune.clear()
    assert lib.kp_tune_count() == 0 and tune.entries() == []


def test_save_load_round_trip(tune, tmp_path):
    tune.set_tile("f32", 1, 64, 48, 4096, (4, 1, 16))
    tune.set_tile("f64", 16, 20, 30, 7, (2, 2, 16))
    before = tune.entries()
    path = tmp_path / "table.json"
    tune.save(str(path))
    rec = json.loads(path.read_text())
    assert rec["entries"] == before
    assert rec["variants"] == tune.variants_signature() and "arch" in rec
    tune.clear()
    assert tune.load(str(path)) == 2
    assert tune.entries() == before
    # a table tuned for other compiled tiles, another device or another
    # library version is refused unless forced
    for key, value in (("variants", "0" * 16), ("arch", "gfx000"), ("kp_version", 1)):
        bad = dict(rec, **{key: value})
        if key == "arch" and tune.device_arch() is None:
            continue                       # no device here: nothing to compare with
        p2 = tmp_path / f"bad_{key}.json"
        p2.write_text(json.dumps(bad))
        tune.clear()
        with pytest.raises(ValueError):
            tune.load(str(p2))
        assert tune.entries() == []
        assert tune.load(str(p2), force=True) == 2
    tune.clear()


def views(m, n, order, backward=False):
    """The 3-index views of a chain in column-major (canonical) mode order."""
    d = len(m)
    cur = list(m)
    out = []
    if backward:
        cur = list(n)
        for k in reversed(range(d)):
            Il, Ir = int(np.prod(cur[:k])), int(np.prod(cur[k + 1:]))
            out.append((Il, n[k], m[k], Ir))
            cur[k] = m[k]
        return out
    for k in order:
        Il, Ir = int(np.prod(cur[:k])), int(np.prod(cur[k + 1:]))
        out.append((Il, m[k], n[k], Ir))
        cur[k] = n[k]
    return out


@pytest.mark.parametrize("seed", range(4))
def test_products_report_the_chain_views(lib, L, tune, seed):
    rng = np.random.default_rng(70 + seed)
    d = int(rng.integers(1, 6))
    tm = [int(x) for x in rng.integers(1, 12, size=d)]   # torch shape
    tn = [int(x) for x in rng.integers(1, 12, size=d)]
    T = torch.zeros(tm, dtype=torch.float64)             # pointers are not read
    Ls = [torch.zeros((tn[k], tm[k]), dtype=torch.float64) for k in range(d)]
    m, n = tm[::-1], tn[::-1]                              # canonical order
    got = [(p["Il"], p["m"], p["n"], p["Ir"]) for p in tune.products(T, Ls)]
    Td = tensor(L, m)
    arr = mlist(L, [matrix(L, n[k], m[k]) for k in range(d)])
    order = (ctypes.c_int * 8)()
    cnt = ctypes.c_int()
    assert lib.kp_tucker_order(ctypes.byref(Td), arr, order, ctypes.byref(cnt)) == 0
    planned = [order[k] - 1 for k in range(cnt.value)]
    assert got == views(m, n, planned)
    got1 = [(p["Il"], p["m"], p["n"], p["Ir"]) for p in tune.products(T, Ls, which="forward_cached")]
    assert got1 == views(m, n, list(range(d)))
    got2 = [(p["Il"], p["m"], p["n"], p["Ir"]) for p in tune.products(T, Ls, which="backward")]
    assert got2 == views(m, n, None, backward=True)
    # the reported tile follows the table
    p0 = tune.products(T, Ls)[0]
    tune.set_tile("f64", p0["Il"], p0["m"], p0["n"], p0["Ir"], (2, 2, 16))
    q0 = tune.products(T, Ls)[0]
    assert (q0["nb"], q0["fb"], q0["bk"], q0["kind"]) == (2, 2, 16, 0)
    with pytest.raises(Exception):
        tune.products(T, Ls, which="nope")


@no_device
def test_batch_plan_takes_tiles_from_the_table(lib, L, tune):
    shapes = [((20, 30, 40), (24, 16, 40)), ((33, 17), (50, 9))]
    alloc = Alloc()
    items = make_items(L, shapes, 1, True, alloc)
    _, st0, _, _ = plan(lib, L, items, len(shapes), 0)
    allv = tune.variants("f32", batch=True)
    tiles = [v for v in allv if v[5] == 0]     # stage kind 0 indexes these
    strips = [v for v in allv if v[5] == 1]    # stage kind 3 indexes these
    modes = [s for s in st0 if s.kind in (0, 3)]
    assert modes and any(s.kind == 3 for s in modes)   # short contractions stream
    # move every mode stage to another executor tile: strips to k-loop tiles
    # and the other way round where the strip covers m
    for s in modes:
        a = s.m
        if s.kind == 3:
            new = tiles[(s.variant // 2) % len(tiles)]
        else:
            new = next((v for v in strips if v[2] >= a.m), tiles[(s.variant // 2 + 1) % len(tiles)])
        tune.set_tile("f32", a.Il, a.m, a.n, a.Ir, new)
    _, st1, _, _ = plan(lib, L, items, len(shapes), 0)
    m1 = [s for s in st1 if s.kind in (0, 3)]
    assert len(m1) == len(modes)
    for s in m1:
        a = s.m
        _, tile = tune.lookup("f32", a.Il, a.m, a.n, a.Ir)
        got = (tiles if s.kind == 0 else strips)[s.variant // 2]
        assert got[:3] == tile[:3] and got[5] == tile[5]
        assert (s.variant & 1) == (1 if a.Il > 1 else 0)


def test_fusion_option_and_reported_launches(lib, L, tune):
    assert lib.kp_get_option(L.KP_OPT_FUSE) == 1
    assert lib.kp_set_option(L.KP_OPT_FUSE, 2) == -9
    assert lib.kp_set_option(99, 0) == -9 and lib.kp_get_option(99) == -9
    # canonical dims (16, 16, 16, 7, 6): the square modes go first (fewer
    # flops), then mode 2, and the two leading modes last (same flops as any
    # order of modes 0, 1, 2; FP32 data whose leading modes fit a pair):
    # (3, 4) is a strided pair (I_l > 1, m <= 16, n <= 32), mode 2 runs
    # alone, (0, 1) is the lead-layout pair (I_l = 1)
    T = torch.zeros((6, 7, 16, 16, 16), dtype=torch.float32)
    Ls = [torch.zeros((6, 6)), torch.zeros((7, 7))] + [torch.zeros((24, 16))] * 3
    try:
        got = tune.products(T, Ls, which="launches")
        assert [p["kind"] for p in got] == [2, 0, 2]   # FP32 m = 16 alone: k-loop tile
        assert [(p["Il"], p["m"], p["n"]) for p in got] == [(4096, 7, 7), (256, 16, 24),
                                                              (1, 16, 24)]
        assert lib.kp_set_option(L.KP_OPT_FUSE, 0) == 0
        assert all(p["kind"] != 2 for p in tune.products(T, Ls, which="launches"))
        assert len(tune.products(T, Ls, which="launches")) == 5
        # six 16 -> 24 modes (the interpolation shape): the leading modes go
        # last, and the chain is three fused pairs, the last one on the lead
        # layout
        assert lib.kp_set_option(L.KP_OPT_FUSE, 1) == 0
        T6 = torch.zeros((16,) * 6, dtype=torch.float32)
        got6 = tune.products(T6, [torch.zeros((24, 16))] * 6, which="launches")
        assert [p["kind"] == 2 for p in got6] == [True, True, True]
        assert [(p["Il"], p["m"], p["n"]) for p in got6] == \
            [(16 * 16, 16, 24), (16 * 16 * 24 * 24, 16, 24), (1, 16, 24)]
        # unfused, the same order: six launches, the leading modes last
        assert lib.kp_set_option(L.KP_OPT_FUSE, 0) == 0
        got6u = tune.products(T6, [torch.zeros((24, 16))] * 6, which="launches")
        assert [p["Il"] for p in got6u] == [256, 256 * 24, 256 * 576, 256 * 576 * 24, 1, 24]
        assert lib.kp_set_option(L.KP_OPT_FUSE, 1) == 0
        # FP64 keeps the minimum-flop order with its definition-order ties
        order = (ctypes.c_int * 8)()
        cnt = ctypes.c_int()
        T6d = tensor(L, [16] * 6, dtype=0)
        arr = mlist(L, [matrix(L, 24, 16, dtype=0) for _ in range(6)])
        assert lib.kp_tucker_order(ctypes.byref(T6d), arr, order, ctypes.byref(cnt)) == 0
        assert [order[k] for k in range(cnt.value)] == [1, 2, 3, 4, 5, 6]
        T6f = tensor(L, [16] * 6, dtype=1)
        arr = mlist(L, [matrix(L, 24, 16, dtype=1) for _ in range(6)])
        assert lib.kp_tucker_order(ctypes.byref(T6f), arr, order, ctypes.byref(cnt)) == 0
        assert [order[k] for k in range(cnt.value)] == [3, 4, 5, 6, 1, 2]
        # FP64 is never fused; the split forms are, like FP32
        T64 = T.double()
        L64 = [x.double() for x in Ls]
        assert all(p["kind"] != 2 for p in tune.products(T64, L64, which="launches"))
        for prec in ("bf16x3", "bf16x6"):
            assert [p["kind"] == 2 for p in tune.products(T, Ls, prec, which="launches")] == \
                [True, False, True]
    finally:
        lib.kp_set_option(L.KP_OPT_FUSE, 1)
