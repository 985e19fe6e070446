"""Tile autotuning for the mu-mode product kernels.

Each mu-mode product takes its tile from the library's tile table, keyed by
the arithmetic form and the product's exact 3-index view (I_l, m, n, I_r),
or failing that by its shape class (same form, layout, m and n, fiber count
within a factor of two), before the built-in defaults (include/kp.h,
kp_tune_*). This module fills that table: it asks the library which products
a call launches (kp_tucker_products), times every compiled tile variant on
each of them with HIP events, and records the fastest. Tables are saved to
and loaded from JSON together with the device architecture, library version
and compiled-tile signature they were tuned for; loading checks them.

Two timing objectives:

* ``latency`` (single Tucker calls): the product is timed at its own size,
  so a tile that leaves the GPU half empty loses.
* ``throughput`` (the batched executor, where one launch runs the tiles of
  many problems at once): the view is enlarged along I_r until it spans at
  least ``fill_fibers`` fibers and the time per original view is compared;
  only tiles the executor compiles are candidates.
"""
from __future__ import annotations

import ctypes
import json

import torch

from . import _lib
from .ops import _canon, _mdesc, _mlist, _prec, _tdesc, check, force_tile, lib, mump

FORMS = {"f64": 0, "f32": 1, "bf16x3": 3, "bf16x6": 6}
FORM_NAMES = {v: k for k, v in FORMS.items()}
_FIELDS = ("form", "Il", "m", "n", "Ir", "nb", "fb", "bk", "occ", "pf", "kind")


def form_code(dtype, prec="native"):
    """Form of a call: FP64/FP32 data with the native precision, or a BF16 split."""
    p = _prec(prec)
    if p == _lib.KP_PREC_NATIVE:
        if dtype == torch.float64:
            return FORMS["f64"]
        if dtype == torch.float32:
            return FORMS["f32"]
        raise TypeError(f"unsupported dtype {dtype}")
    if dtype != torch.float32:
        raise TypeError("the BF16 split forms take float32 data")
    return p


def _entry_dict(e):
    return {k: int(getattr(e, k)) for k in _FIELDS}


def variants(form, batch=False, m=None):
    """Compiled tiles (nb, fb, bk, occ, pf, kind) of a form: the standalone
    kernels, or the batched executor's. With `m`, only the tiles that can run
    a contraction of that length (strip tiles need m <= bk)."""
    form = FORMS.get(form, form)
    n = lib().kp_tile_variants(form, int(bool(batch)), None, 0)
    check(min(n, 0), "kp_tile_variants")
    buf = (ctypes.c_int32 * (6 * max(n, 1)))()
    lib().kp_tile_variants(form, int(bool(batch)), buf, n)
    out = [tuple(buf[6 * i:6 * i + 6]) for i in range(n)]
    if m is not None:
        out = [v for v in out if v[5] != 1 or m <= v[2]]
    return out


def entries():
    """The table, as a list of dicts (form, Il, m, n, Ir, nb, fb, bk, occ, pf)."""
    n = lib().kp_tune_count()
    buf = (_lib.KpTuneEntry * max(n, 1))()
    n = lib().kp_tune_list(buf, n)
    return [_entry_dict(buf[i]) for i in range(n)]


def clear():
    check(lib().kp_tune_clear(), "kp_tune_clear")


def set_tile(form, Il, m, n, Ir, tile):
    """Record `tile` = (nb, fb, bk[, occ, pf, kind]) for one product view."""
    t = tuple(tile) + (0,) * (6 - len(tile))
    e = _lib.KpTuneEntry()
    e.form = FORMS.get(form, form)
    e.Il, e.m, e.n, e.Ir = Il, m, n, Ir
    e.nb, e.fb, e.bk, e.occ, e.pf, e.kind = t
    check(lib().kp_tune_set(ctypes.byref(e)), "kp_tune_set")


def lookup(form, Il, m, n, Ir):
    """(tuned, tile): the tile this view gets now, and whether it is from the table."""
    e = _lib.KpTuneEntry()
    st = lib().kp_tune_lookup(FORMS.get(form, form), Il, m, n, Ir, ctypes.byref(e))
    check(min(st, 0), "kp_tune_lookup")
    return bool(st), (e.nb, e.fb, e.bk, e.occ, e.pf, e.kind)


def device_arch():
    """Architecture name of the current device (e.g. 'gfx950'), or None."""
    try:
        if torch.cuda.is_available():
            return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(
                ":")[0]
    except Exception:  # pragma: no cover
        pass
    return None


def variants_signature():
    """Digest of every compiled tile (standalone and batched, every form): a
    saved table is only meaningful for the library build it was tuned on."""
    import hashlib
    h = hashlib.sha256()
    for form in sorted(FORMS.values()):
        for batch in (False, True):
            h.update(repr((form, batch, variants(form, batch=batch))).encode())
    return h.hexdigest()[:16]


def save(path):
    """Write the table with what it was tuned for: the device architecture,
    the library version and the compiled-tile signature."""
    with open(path, "w") as fh:
        json.dump({"kp_version": lib().kp_version(), "arch": device_arch(),
                   "variants": variants_signature(), "entries": entries()}, fh, indent=1)


def load(path, force=False):
    """Add the entries of a saved table; returns how many were loaded.
    Refuses (ValueError) a table tuned for another library version, another
    device architecture or other compiled tiles, unless ``force``."""
    with open(path) as fh:
        rec = json.load(fh)
    if not force:
        if rec.get("kp_version") != lib().kp_version():
            raise ValueError(f"table tuned for library version {rec.get('kp_version')}")
        arch = device_arch()
        if rec.get("arch") is not None and arch is not None and rec["arch"] != arch:
            raise ValueError(f"table tuned on {rec['arch']}, this device is {arch}")
        if rec.get("variants") is not None and rec["variants"] != variants_signature():
            raise ValueError("table tuned for a library build with other compiled tiles")
    for e in rec["entries"]:
        set_tile(e["form"], e["Il"], e["m"], e["n"], e["Ir"],
                 (e["nb"], e["fb"], e["bk"], e["occ"], e["pf"], e.get("kind", 0)))
    return len(rec["entries"])


WHICH = {"forward": 0, "forward_cached": 1, "backward": 2, "launches": 3}


def products(T, Ls, prec="native", which="forward"):
    """The mu-mode products a call launches, in launch order, each a dict with
    its view and current tile. which: "forward" (kp_tucker), "forward_cached"
    (kp_tucker with a cache / the backward's recomputed partials, and the
    batched executor's forward), "backward" (the cotangent sweep), "launches"
    (kp_tucker's launches: a fused pair of modes is one entry of kind 2)."""
    Tc = _canon(T)
    td = _tdesc(Tc, True)
    arr = _mlist([None if L is None else _mdesc(L) for L in Ls][::-1])
    p = _prec(prec)
    w = WHICH[which]
    n = lib().kp_tucker_products(ctypes.byref(td), arr, p, w, None, 0)
    check(min(n, 0), "kp_tucker_products")
    buf = (_lib.KpTuneEntry * max(n, 1))()
    lib().kp_tucker_products(ctypes.byref(td), arr, p, w, buf, n)
    return [_entry_dict(buf[i]) for i in range(n)]


def _time_view(dtype, prec, Il, m, n, Ir, tile, reps):
    """Average seconds per launch of one product on an (Il, m, Ir) view with
    `tile` forced; the torch tensor (Ir, m, Il) is that view's mode 2."""
    X = torch.randn((Ir, m, Il), dtype=dtype, device="cuda")
    L = torch.randn((n, m), dtype=dtype, device="cuda")
    Y = torch.empty((Ir, n, Il), dtype=dtype, device="cuda")
    force_tile(*tile)
    try:
        for _ in range(2):
            mump(X, L, 2, prec=prec, out=Y)
        best = None
        for _ in range(2):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                mump(X, L, 2, prec=prec, out=Y)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / reps
            best = t if best is None else min(best, t)
    finally:
        force_tile(0)
    return best


def tune_view(dtype, prec, Il, m, n, Ir, objective="latency", reps=10, fill_fibers=1 << 20,
              max_bytes=1 << 30):
    """Time every candidate tile on one view; record and return the fastest
    as (tile, seconds per original view, {tile: seconds})."""
    form = form_code(dtype, prec)
    batch = objective == "throughput"
    cands = variants(form, batch=batch, m=m)
    rep_Ir, scale = Ir, 1
    if batch:
        es = torch.empty((), dtype=dtype).element_size()
        per = Il * Ir
        want = max(1, -(-fill_fibers // per))
        cap = max(1, max_bytes // max(1, per * max(m, n) * es))
        scale = min(want, cap)
        rep_Ir = Ir * scale
    times = {}
    for c in cands:
        times[c] = _time_view(dtype, prec, Il, m, n, rep_Ir, c, reps) / scale
    best = min(times, key=times.get)
    set_tile(form, Il, m, n, Ir, best)
    return best, times[best], times


def autotune(T, Ls, prec="native", backward=False, reps=10):
    """Tune every product a Tucker call (and, with ``backward``, its gradient)
    launches on these shapes at their own size; returns the recorded entries."""
    whichs = ["forward"] + (["forward_cached", "backward"] if backward else [])
    return _tune_keys([(T, Ls)], prec, whichs, "latency", reps)


def autotune_batch(Ts, Ls, prec="native", backward=False, reps=5, fill_fibers=1 << 20):
    """Tune the products the batched executor runs for these problems (forward
    in definition order, and the cotangent sweep with ``backward``) for
    throughput over the executor's tiles. Build the BatchedTucker after this:
    its plan takes the tiles when it is constructed."""
    whichs = ["forward_cached"] + (["backward"] if backward else [])
    return _tune_keys(list(zip(Ts, Ls)), prec, whichs, "throughput", reps, fill_fibers)


def _tune_keys(problems, prec, whichs, objective, reps, fill_fibers=1 << 20):
    seen = {}
    for T, L in problems:
        for w in whichs:
            for p in products(T, L, prec, w):
                key = (p["form"], p["Il"], p["m"], p["n"], p["Ir"])
                if key not in seen:
                    seen[key] = T.dtype
    out = []
    for (form, Il, m, n, Ir), dtype in seen.items():
        tile, sec, _ = tune_view(dtype, prec, Il, m, n, Ir, objective, reps, fill_fibers)
        out.append({"form": form, "Il": Il, "m": m, "n": n, "Ir": Ir, "tile": tile,
                    "seconds": sec})
    return out
