"""Host-side checks of the batched executor's plan (kp_batch_plan), without a
GPU: the plan is parsed and checked for dependency order, task numbering and
buffer bounds before any kernel could run it. Fake device addresses are used,
so these tests only run where no GPU is visible."""
import ctypes

import numpy as np
import pytest

from test_abi_host import matrix, no_device, tensor

FAKE_WS = 0x7000_0000_0000


class ModeArgsC(ctypes.Structure):
    _fields_ = [("X", ctypes.c_uint64), ("Y", ctypes.c_uint64), ("L", ctypes.c_uint64),
                ("Il", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("Ir", ctypes.c_int64), ("rs", ctypes.c_int64), ("cs", ctypes.c_int64),
                ("accumulate", ctypes.c_int32), ("pad", ctypes.c_int32)]


class GramArgsC(ctypes.Structure):
    _fields_ = [("Q", ctypes.c_uint64), ("P", ctypes.c_uint64), ("part", ctypes.c_uint64),
                ("Il", ctypes.c_int64), ("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("Ir", ctypes.c_int64), ("chunks", ctypes.c_int64),
                ("per_split", ctypes.c_int64), ("achunks", ctypes.c_int64)]


class StageC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("variant", ctypes.c_int32), ("tx", ctypes.c_int32),
                ("ty", ctypes.c_int32), ("tz", ctypes.c_int32), ("dep0", ctypes.c_int32),
                ("dep1", ctypes.c_int32), ("problem", ctypes.c_int32), ("begin", ctypes.c_int64),
                ("m", ModeArgsC), ("g", GramArgsC), ("splits", ctypes.c_int64),
                ("dL", ctypes.c_uint64), ("rs", ctypes.c_int64), ("cs", ctypes.c_int64),
                ("ntiles", ctypes.c_int64)]


class GroupC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("s_begin", ctypes.c_int32), ("s_end", ctypes.c_int32),
                ("level", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_begin", ctypes.c_int64), ("t_end", ctypes.c_int64)]


class HeaderC(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint64), ("nstages", ctypes.c_int32),
                ("form", ctypes.c_int32), ("ntasks", ctypes.c_int64),
                ("nlevels", ctypes.c_int32), ("ngroups", ctypes.c_int32),
                ("ws_base", ctypes.c_uint64), ("ws_bytes", ctypes.c_uint64)]


@pytest.fixture(scope="module")
def L():
    from paper_2112_11238_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def lib(L):
    return L.load()


class Alloc:
    """Hands out disjoint fake device ranges and remembers them."""

    def __init__(self):
        self.next = 0x1000_0000
        self.ranges = {}

    def get(self, nbytes, name):
        a = self.next
        self.next += (nbytes + 4095) // 4096 * 4096 + 4096
        self.ranges[name] = (a, nbytes)
        return a


def make_items(L, shapes, dtype, backward, alloc):
    es = 8 if dtype == 0 else 4
    items = (L.KpBatchItem * len(shapes))()
    for k, (m, n) in enumerate(shapes):
        d = len(m)
        it = items[k]
        it.T = tensor(L, list(m)[::-1], dtype, alloc.get(int(np.prod(m)) * es, f"T{k}"))
        it.S = tensor(L, list(n)[::-1], dtype, alloc.get(int(np.prod(n)) * es, f"S{k}"))
        for j in range(d):  # canonical order is reversed
            mm, nn = m[d - 1 - j], n[d - 1 - j]
            it.L[j] = matrix(L, nn, mm, dtype, alloc.get(nn * mm * es, f"L{k}_{j}"))
        if backward:
            it.G = tensor(L, list(n)[::-1], dtype, alloc.get(int(np.prod(n)) * es, f"G{k}"))
            it.dT = tensor(L, list(m)[::-1], dtype, alloc.get(int(np.prod(m)) * es, f"dT{k}"))
            for j in range(d):
                mm, nn = m[d - 1 - j], n[d - 1 - j]
                it.dL[j] = matrix(L, nn, mm, dtype, alloc.get(nn * mm * es, f"dL{k}_{j}"))
    return items


def plan(lib, L, items, count, prec):
    ws_bytes = lib.kp_batch_workspace(count, items, prec)
    pb = lib.kp_batch_plan_bytes(count, items, prec)
    assert ws_bytes > 0 and pb > 0
    buf = (ctypes.c_char * pb)()
    assert lib.kp_batch_plan(count, items, prec, FAKE_WS, ws_bytes, buf, pb) == 0
    raw = bytes(buf)
    h = HeaderC.from_buffer_copy(raw[:ctypes.sizeof(HeaderC)])
    o = ctypes.sizeof(HeaderC)
    st = (StageC * h.nstages).from_buffer_copy(raw[o:o + h.nstages * ctypes.sizeof(StageC)])
    o += h.nstages * ctypes.sizeof(StageC)
    lb = list((ctypes.c_int64 * (h.nlevels + 1)).from_buffer_copy(raw[o:o + 8 * (h.nlevels + 1)]))
    o += 8 * (h.nlevels + 1)
    gr = list((GroupC * h.ngroups).from_buffer_copy(raw[o:o + h.ngroups * ctypes.sizeof(GroupC)]))
    assert o + h.ngroups * ctypes.sizeof(GroupC) == len(raw)
    plan.groups = gr
    return h, list(st), ws_bytes, lb


def within(addr, nbytes, ranges):
    for a, n in ranges:
        if a <= addr and addr + nbytes <= a + n:
            return True
    return False


@no_device
@pytest.mark.parametrize("dtype,prec,backward", [(1, 0, False), (1, 0, True), (0, 0, True),
                                                 (1, 3, True), (1, 6, False)])
def test_plan_is_ordered_and_in_bounds(lib, L, dtype, prec, backward):
    rng = np.random.default_rng(5 + dtype + prec)
    shapes = []
    for _ in range(9):
        d = int(rng.integers(1, 5))
        m = tuple(int(x) for x in rng.integers(1, 40, size=d))
        n = tuple(int(x) for x in rng.integers(1, 40, size=d))
        shapes.append((m, n))
    alloc = Alloc()
    items = make_items(L, shapes, dtype, backward, alloc)
    h, st, ws_bytes, lb = plan(lib, L, items, len(shapes), prec)
    assert h.ws_base == FAKE_WS
    es = 8 if dtype == 0 else 4
    # task numbering; levels are consecutive task ranges
    task = 0
    for i, s in enumerate(st):
        assert s.begin == task
        task += s.tx * s.ty * s.tz
        assert s.tx >= 1 and s.ty >= 1 and s.tz >= 1
    assert task == h.ntasks
    assert lb[0] == 0 and lb[-1] == h.ntasks and all(a <= b for a, b in zip(lb, lb[1:]))

    def level_of(i):
        b = st[i].begin
        return max(lv for lv in range(h.nlevels) if lb[lv] <= b)

    # every dependency sits in a strictly lower level (an earlier launch)
    for i, s in enumerate(st):
        for dep in (s.dep0, s.dep1):
            if dep >= 0:
                assert dep < i and level_of(dep) < level_of(i)
    # launch groups: consecutive, covering every stage and task once, one
    # task type and one level each, levels ascending
    gr = plan.groups
    assert gr[0].s_begin == 0 and gr[-1].s_end == len(st)
    assert gr[0].t_begin == 0 and gr[-1].t_end == h.ntasks
    for a, b in zip(gr, gr[1:]):
        assert a.s_end == b.s_begin and a.t_end == b.t_begin and a.level <= b.level
    for g in gr:
        assert g.s_begin < g.s_end
        assert g.t_begin == st[g.s_begin].begin
        for i in range(g.s_begin, g.s_end):
            assert (st[i].kind, st[i].variant) == (g.kind, g.variant)
            assert level_of(i) == g.level
    ws = (FAKE_WS, ws_bytes)
    user = list(alloc.ranges.values())
    # every access inside the user buffers or the workspace; outputs distinct
    writes = []
    for s in st:
        if s.kind in (0, 3):
            mm = s.m
            F = mm.Il * mm.Ir
            assert within(mm.X, F * mm.m * es, user + [ws])
            assert within(mm.Y, F * mm.n * es, user + [ws])
            span = ((mm.n - 1) * mm.rs + (mm.m - 1) * mm.cs + 1) * es
            assert within(mm.L, span, user)
            writes.append((mm.Y, F * mm.n * es))
            if s.kind == 3:       # strip: every fiber tile of every n block once
                assert s.ntiles >= 1 and 1 <= s.tx <= s.ntiles
        elif s.kind == 4:
            g = s.g
            F = g.Il * g.Ir
            assert within(g.Q, F * g.n * es, user + [ws])
            assert within(g.P, F * g.m * es, user + [ws])
            assert s.tx == s.splits and s.ty == s.tz == 1 and 1 <= s.splits <= s.ntiles
            assert g.n <= 64 and g.m <= 64
            assert within(g.part, s.splits * g.n * g.m * es, [ws])
            writes.append((g.part, s.splits * g.n * g.m * es))
        elif s.kind == 1:
            g = s.g
            F = g.Il * g.Ir
            assert within(g.Q, F * g.n * es, user + [ws])
            assert within(g.P, F * g.m * es, user + [ws])
            assert within(g.part, s.tz * g.n * g.m * es, [ws])
            assert g.chunks <= s.tz * g.per_split
            writes.append((g.part, s.tz * g.n * g.m * es))
        else:
            assert s.kind == 2
            assert s.tx == (s.g.n * s.g.m + 15) // 16
            assert within(s.dL, s.g.n * s.g.m * es, user)
            writes.append((s.dL, s.g.n * s.g.m * es))
    writes.sort()
    for (a0, n0), (a1, _) in zip(writes, writes[1:]):
        assert a0 + n0 <= a1, "two stages write overlapping memory"


@no_device
def test_plan_rejects_bad_items(lib, L):
    alloc = Alloc()
    items = make_items(L, [((3, 4), (5, 6))], 1, False, alloc)
    bad = make_items(L, [((3, 4), (5, 6))], 1, False, alloc)
    bad[0].L[0].cols = 9
    assert lib.kp_batch_workspace(1, bad, 0) == 0
    buf = (ctypes.c_char * 10)()
    ws = lib.kp_batch_workspace(1, items, 0)
    assert lib.kp_batch_plan(1, items, 0, FAKE_WS, ws, buf, 10) == -7   # plan buffer too small
    pb = lib.kp_batch_plan_bytes(1, items, 0)
    big = (ctypes.c_char * pb)()
    assert lib.kp_batch_plan(1, items, 0, FAKE_WS, ws - 1, big, pb) == -7
    assert lib.kp_batch_plan(1, items, 6, FAKE_WS, ws, big, pb) == 0   # FP32 + BF16x6 ok
    items64 = make_items(L, [((3, 4), (5, 6))], 0, False, alloc)
    assert lib.kp_batch_workspace(1, items64, 3) == 0                   # BF16 needs FP32
    neg = make_items(L, [((3, 4), (5, 6))], 1, False, alloc)
    neg[0].L[1].cs = -1                                                 # negative stride
    assert lib.kp_batch_workspace(1, neg, 0) == 0
    assert lib.kp_batch_plan(1, neg, 0, FAKE_WS, ws, big, pb) == -9
    assert lib.kp_batch_info(big, None, None, None) == 0
    assert lib.kp_batch_info(buf, None, None, None) == -9   # not a plan
