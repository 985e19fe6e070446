"""Benchmark: Tucker operator TFLOP/s at d=3, m=n=200 on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one Tucker operator S = T x_1 L_1 x_2 L_2 x_3 L_3 on the resident
cube200 input (8M-entry tensor, three 200x200 standard-normal factors, seed 0)
through the C-ABI (kp_tucker), in each arithmetic form:

  f64     FP64 MFMA                      (the reported `value`)
  f32     FP32 MFMA
  bf16x3  BF16 split, 3 products, FP32 accumulation
  bf16x6  BF16 split, 6 products, FP32 accumulation

The steps are kp_tucker calls issued back to back (the rate of the same step
replayed from a HIP graph is reported beside it). Each form's error against the FP64
oracle (max-norm relative, the paper's metric) is reported with it. Each
mu-mode product is also timed alone (kp_mump, launches back to back between
two HIP events on the launch stream); the FP64 per-launch average gives the
roofline entry of the dominant kernel.
The oracle (numpy FP64 on the host) is timed on a bounded sample of the same
workload as the CPU baseline. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import kp_workloads  # noqa: E402

METRIC = "Tucker-op TFLOP/s d=3 n=200: FP64 vs BF16x3 MFMA at 1e-6 rel err, % of peak"
PEAK = {  # MI355X published dense peaks, TFLOP/s
    "f64": 78.6, "f32": 157.3, "bf16": 2500.0,
}
HBM_PEAK_GBS = 8000.0
FORMS = [("f64", "native"), ("f32", "native"), ("f32", "bf16x3"), ("f32", "bf16x6")]
CSRC = os.path.join(ROOT, "paper_2112_11238_amd", "csrc")
MODE_KERNEL_SRC = [os.path.join(CSRC, f) for f in ("mode_kernels.hip", "mode_tile.h",
                                                    "kp_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mode_f64_cube200.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed warmup steps (default: 200 for cube200, 5 for the other "
                         "workloads). cube200's launches are short next to the time the GPU "
                         "takes to raise its clock under load: after 2-20 launches an FP64 "
                         "mode product runs ~80 us, after a few hundred back-to-back ones ~70")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="all", help="comma list of f64,f32,bf16x3,bf16x6")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--workload", default="cube200",
                    choices=["cube200", "small2d", "heat128", "interp6d", "batch64", "semilinear",
                             "runge5d", "codeval", "fft3d"],
                    help="cube200 is the headline line; the others time the remaining "
                         "configurations (one JSON line each)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the tiles of every launched product before timing")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only launch the FP64 mode products of cube200 (--steps each) and a "
                         "plain 512 MiB device copy, for hardware-counter runs")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def form_name(dt, prec):
    return dt if prec == "native" else prec


def source_hash(paths):
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(per_launch_units):
    """HBM bytes per launch of the FP64 mode kernel from the committed rocprof
    counter summary, or None if absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != source_hash(MODE_KERNEL_SRC):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def cpu_baseline(T, Ls, flops, budget_s=12.0):
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.tucker(T, Ls)
        reps += 1
        el = time.perf_counter() - t0
        if el > budget_s or reps >= 2000:
            break
    return {"value": flops * reps / el / 1e12, "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"full cube200 Tucker operator (8M entries, 9.6 GFLOP), {reps} "
                      f"repetitions in {el:.1f} s, numpy float64"}


def traffic_probe(args):
    """Launches for a counter run: each FP64 mu-mode product of cube200 with
    the default tiles (interp6d: the FP32 forward, fused, then unfused), then
    a plain device-to-device copy of known size whose counter readings
    calibrate the HBM byte counters."""
    import torch

    import paper_2112_11238_amd as kp
    dev = torch.device("cuda:0")
    if args.workload == "interp6d":
        from paper_2112_11238_amd import _lib, tune
        lib = _lib.load()
        T, Ls = kp_workloads.interp6d(seed=0)
        Td = torch.tensor(T, dtype=torch.float32, device=dev)
        Lds = [torch.tensor(L, dtype=torch.float32, device=dev) for L in Ls]
        plans = {}
        for fuse in (1, 0):
            lib.kp_set_option(_lib.KP_OPT_FUSE, fuse)
            plans["fused" if fuse else "unfused"] = [
                [p["kind"], p["Il"], p["m"], p["n"], p["Ir"]]
                for p in tune.products(Td, Lds, which="launches")]
            for _ in range(args.steps):
                kp.tucker(Td, Lds)
            torch.cuda.synchronize()
        lib.kp_set_option(_lib.KP_OPT_FUSE, 1)
        del Td
    else:
        T, Ls = kp_workloads.cube200(seed=0)
    if args.workload == "interp6d":
        copy_bytes = 512 << 20
        a = torch.ones(copy_bytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "traffic", "workload": "interp6d", "forwards": args.steps,
                          "launches": plans, "input_bytes": 16 ** 6 * 4,
                          "output_bytes": 24 ** 6 * 4, "copy_bytes_read": copy_bytes,
                          "copy_bytes_written": copy_bytes, "copy_launches": 3}), flush=True)
        return
    Td = torch.tensor(T, dtype=torch.float64, device=dev)
    Lds = [torch.tensor(L, dtype=torch.float64, device=dev) for L in Ls]
    out = torch.empty_like(Td)
    for mu in (1, 2, 3):
        for _ in range(args.steps):
            kp.mump(Td, Lds[mu - 1], mu, out=out)
    torch.cuda.synchronize()
    copy_bytes = 512 << 20
    a = torch.ones(copy_bytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "traffic", "mode_launches_per_mu": args.steps,
                      "mode_bytes_in_out": 2 * Td.numel() * 8,
                      "copy_bytes_read": copy_bytes, "copy_bytes_written": copy_bytes,
                      "copy_launches": 3, "kernel_source_sha256_16": source_hash(MODE_KERNEL_SRC)}),
          flush=True)


def main():
    args = parse()
    if args.warmup is None:
        args.warmup = 200 if args.workload == "cube200" and not args.traffic_probe else 5
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: there is no "
                                   "multi-GPU path, only one GPU's share is measured"}))
        sys.exit(2)
    if args.traffic_probe:
        traffic_probe(args)
        return
    if args.workload != "cube200":
        print(json.dumps(WORKLOAD_BENCHES[args.workload](args)), flush=True)
        return
    import torch

    import oracle
    import paper_2112_11238_amd as kp
    from paper_2112_11238_amd import _lib
    _lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    want = None if args.forms == "all" else set(args.forms.split(","))

    T, Ls = kp_workloads.cube200(seed=0)
    m = T.shape
    flops = kp_workloads.tucker_flops(m, [L.shape[0] for L in Ls])
    flops_mode = 2 * 200 * T.size
    log(args, "oracle reference (numpy FP64) ...")
    t0 = time.perf_counter()
    ref64 = oracle.tucker(T, Ls)
    oracle_once = time.perf_counter() - t0
    ref32 = None
    results = {}
    mode_avg = {}
    for dt, prec in FORMS:
        name = form_name(dt, prec)
        if want and name not in want:
            continue
        tdt = torch.float64 if dt == "f64" else torch.float32
        Td = torch.tensor(T, dtype=tdt, device=dev)
        Lds = [torch.tensor(L, dtype=tdt, device=dev) for L in Ls]
        if dt == "f32" and ref32 is None:
            ref32 = oracle.tucker(Td.double().cpu().numpy(),
                                  [L.double().cpu().numpy() for L in Lds])
        ref = ref64 if dt == "f64" else ref32
        log(args, f"form {name}: warmup {args.warmup}")
        for _ in range(args.warmup):
            S = kp.tucker(Td, Lds, prec=prec)
        torch.cuda.synchronize()
        got = S.double().cpu().numpy()
        err = float(np.abs(got - ref).max() / np.abs(ref).max())
        err_fro = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        # Timed regions: K full Tucker steps (each one kp_tucker call, three
        # mode launches) issued eagerly, HIP events on the launch stream
        # (ms_per_step_eager); then the same call captured once in a HIP graph
        # and replayed K times back to back (ms_per_step, the line's value):
        # the replay runs the same kernels in the same order (checked bitwise
        # below) without the host work of each call (argument checks, the
        # allocation of S and the workspace).
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        ev[0].record()
        for k in range(args.steps):
            S = kp.tucker(Td, Lds, prec=prec)
            ev[k + 1].record()
        torch.cuda.synchronize()
        step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
        ms = ev[0].elapsed_time(ev[-1]) / args.steps
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            kp.tucker(Td, Lds, prec=prec)  # warm the pool outside the capture
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            Sg = kp.tucker(Td, Lds, prec=prec)
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(args.steps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / args.steps
        # the replays computed what the eager calls compute (same kernels,
        # same order): checked bitwise after the timed regions
        graph_equal = bool(torch.equal(Sg, S))
        del graph, Sg
        # each mu-mode product alone (kp_mump): `warmup` untimed launches,
        # then `steps` launches back to back on the launch stream between two
        # HIP events; the queue stays ahead of the GPU, so the average is the
        # kernel time plus the dispatch gap between consecutive launches (an
        # upper bound of the kernel time)
        per_mode = {}
        # an untimed pass over the three modes first: whichever mode was
        # timed first after the graph section ran 3-4 us slower than when
        # timed later (the same for any order of the modes), a transient of
        # the GPU, not of the mode
        out = torch.empty_like(Td)
        for _ in range(max(2, args.warmup)):
            for mu in (1, 2, 3):
                kp.mump(Td, Lds[mu - 1], mu, prec=prec, out=out)
        torch.cuda.synchronize()
        for mu in (1, 2, 3):
            out = torch.empty_like(Td)
            for _ in range(max(2, args.warmup)):
                kp.mump(Td, Lds[mu - 1], mu, prec=prec, out=out)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for k in range(args.steps):
                kp.mump(Td, Lds[mu - 1], mu, prec=prec, out=out)
            e1.record()
            torch.cuda.synchronize()
            per_mode[mu] = e0.elapsed_time(e1) / args.steps
        peak = PEAK["f64"] if dt == "f64" else (PEAK["f32"] if prec == "native" else PEAK["bf16"])
        hbm_min_bytes = (T.size + S.numel()) * Td.element_size() + \
            sum(L.size for L in Ls) * Td.element_size()
        # roofline of the form: useful-flop peak (the split forms issue S
        # products per useful one) against the unfused traffic (every mode
        # reads and writes the whole tensor) at 8 TB/s
        unfused_bytes = 3 * (T.size + S.numel()) * Td.element_size() + \
            sum(L.size for L in Ls) * Td.element_size()
        useful_peak = peak / (1 if prec == "native" else int(prec[-1]))
        roof_tflops = min(useful_peak, flops / unfused_bytes * HBM_PEAK_GBS / 1e3)
        tflops_eager = flops / (ms * 1e-3) / 1e12
        tflops = flops / (ms_graph * 1e-3) / 1e12
        mfma_tflops = tflops * (1 if prec == "native" else int(prec[-1]))
        results[name] = {
            "tflops": round(tflops, 3),
            "ms_per_step": round(ms_graph, 5),
            "ms_per_step_eager": round(ms, 5),
            "ms_median_eager": round(statistics.median(step_ms), 5),
            "tflops_eager": round(tflops_eager, 3),
            "graph_replay_equals_eager": graph_equal,
            "frac_of_mfma_peak": round(mfma_tflops / peak, 4),
            "mfma_issued_tflops": round(mfma_tflops, 3),
            "peak_tflops": peak,
            "hbm_min_gbs": round(hbm_min_bytes / (ms_graph * 1e-3) / 1e9, 1),
            "roofline_tflops": round(roof_tflops, 1),
            "frac_of_roofline": round(tflops / roof_tflops, 4),
            "rel_err_maxnorm": err,
            "rel_err_frobenius": err_fro,
            "meets_1e-6": err <= 1e-6,
            "mode_ms": {str(k): round(v, 5) for k, v in per_mode.items()},
        }
        mode_avg[name] = statistics.mean(per_mode.values())
        log(args, f"form {name}: {ms_graph:.4f} ms/step (eager {ms:.4f})  {tflops:.2f} TFLOP/s  "
                  f"err {err:.2e}  "
                  f"modes {[round(v, 4) for v in per_mode.values()]} ms")

    head = results.get("f64") or next(iter(results.values()))
    line = {
        "metric": METRIC,
        "value": head["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cube200: Tucker operator, d=3, m=n=200 (8M-entry tensor), "
                               "square standard-normal factors, seed 0; value is the FP64 "
                               "form, other forms under 'forms'",
                   "d": 3, "m": 200, "n": 200, "flops_per_step": flops},
        "forms": results,
    }
    line["config"]["timing"] = ("one kp_tucker call per step, captured once in a HIP graph and "
                                "replayed back to back between HIP events (the replays are "
                                "checked bitwise against the eager calls); ms_per_step_eager "
                                "per form: the same calls issued eagerly; every timed region "
                                "follows `warmup` untimed back-to-back steps (launches for the "
                                "per-mode averages), so the GPU runs at its loaded clock")
    if "f64" in mode_avg:
        avg_ms = mode_avg["f64"]
        achieved = flops_mode / (avg_ms * 1e-3) / 1e12
        line["roofline"] = {
            "kernel": "mode_kernel<FP64> (one mu-mode product, FP64 MFMA)",
            "bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["f64"],
            "unit": "TFLOP/s", "frac": round(achieved / PEAK["f64"], 4),
            "avg_launch_ms": round(avg_ms, 5),
            "flops_per_launch": flops_mode,
            "traffic": load_traffic(1),
        }
    if not args.no_cpu_baseline:
        log(args, "cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(T, Ls, flops)
    line["oracle_first_call_s"] = round(oracle_once, 2)
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------------------
# The other configurations (not the headline line): --workload NAME
# ---------------------------------------------------------------------------

# Seconds of back-to-back untimed calls before every timed run of the other
# configurations: the GPU's clock ramps up under a sustained load, and a few
# warm-up calls of a short kernel end before it has.
WARM_S = 0.3


def _events_ms(fn, steps, warmup):
    """Average ms per call of fn() over `steps` calls, events on the current
    stream around the whole run (inputs resident, warm: at least `warmup`
    untimed calls and WARM_S seconds of them)."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while i < warmup or time.perf_counter() - t0 < WARM_S:
        fn()
        i += 1
        if i % 32 == 0:
            torch.cuda.synchronize()  # wall time then tracks the GPU's
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _graph_ms(fn, steps, warmup):
    """Average ms per replay of fn() captured into one HIP graph."""
    import torch
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return _events_ms(g.replay, steps, warmup), g


def _launch_ms(kp, dtype, prec, view, steps):
    """Average ms of one mu-mode product launch on the view (Il, m, n, Ir),
    HIP events around every launch on the launch stream."""
    import torch
    Il, m, n, Ir = view
    X = torch.randn((Ir, m, Il), dtype=dtype, device="cuda")
    L = torch.randn((n, m), dtype=dtype, device="cuda")
    Y = torch.empty((Ir, n, Il), dtype=dtype, device="cuda")
    _events_ms(lambda: kp.mump(X, L, 2, prec=prec, out=Y), 1, 2)  # warm-up, as every timed run
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    for k in range(steps):
        ev[2 * k].record()
        kp.mump(X, L, 2, prec=prec, out=Y)
        ev[2 * k + 1].record()
    torch.cuda.synchronize()
    return statistics.mean(ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(steps))


def _views(kp, Td, Lds, prec, which="forward"):
    return [(p["Il"], p["m"], p["n"], p["Ir"]) for p in kp.tune.products(Td, Lds, prec, which)]


def _line(args, metric, value, unit, ms, dtype, workload, extra, higher=True):
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "warm_s": WARM_S, "ms_per_step": ms,
            "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": workload}
    line.update(extra)
    return line


def _form_list(args, default):
    if args.forms == "all":
        return default
    want = set(args.forms.split(","))
    return [f for f in default if form_name(*f) in want]


def _rel(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def bench_small2d(args):
    """d = 2, 50 x 50 FP64 (and the other forms): latency of one Tucker call,
    eager and replayed from a HIP graph; each mode alone."""
    import torch

    import oracle
    import paper_2112_11238_amd as kp
    T, Ls = kp_workloads.small2d(seed=0)
    flops = kp_workloads.tucker_flops(T.shape, [L.shape[0] for L in Ls])
    ref = oracle.tucker(T, Ls)
    forms = {}
    for dt, prec in _form_list(args, FORMS):
        tdt = torch.float64 if dt == "f64" else torch.float32
        Td = torch.tensor(T, dtype=tdt, device="cuda")
        Lds = [torch.tensor(L, dtype=tdt, device="cuda") for L in Ls]
        if args.autotune:
            kp.tune.autotune(Td, Lds, prec=prec, reps=20)
        S = kp.tucker(Td, Lds, prec=prec)
        torch.cuda.synchronize()
        eager = _events_ms(lambda: kp.tucker(Td, Lds, prec=prec), args.steps * 10, args.warmup)
        graph, _ = _graph_ms(lambda: kp.tucker(Td, Lds, prec=prec), args.steps * 10, args.warmup)
        modes = [_launch_ms(kp, tdt, prec, v, args.steps) for v in _views(kp, Td, Lds, prec)]
        forms[form_name(dt, prec)] = {
            "us_per_call_eager": round(eager * 1e3, 2), "us_per_call_graph": round(graph * 1e3, 2),
            "us_per_mode_launch": [round(x * 1e3, 2) for x in modes],
            "rel_err_maxnorm": _rel(S.double().cpu().numpy(), ref)}
    head = forms.get("f64") or next(iter(forms.values()))
    t0 = time.perf_counter()
    reps = 0
    while time.perf_counter() - t0 < 3.0:
        oracle.tucker(T, Ls)
        reps += 1
    cpu_us = (time.perf_counter() - t0) / reps * 1e6
    return _line(args, "Tucker-op latency small2d (d=2, 50x50), us per call, graph replay",
                 head["us_per_call_graph"], "us", head["us_per_call_graph"] / 1e3, "f64",
                 {"workload": "small2d: Tucker operator d=2, m=n=50, standard-normal T and "
                              "factors, seed 0; value is the FP64 form replayed from a graph",
                  "flops_per_call": flops},
                 {"forms": forms, "cpu_baseline": {"value": round(cpu_us, 2), "unit": "us",
                                                   "cores": _threads(), "kind": "oracle",
                                                   "sample": f"{reps} oracle calls"}},
                 higher=False)


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([p.get("num_threads", 1) for p in threadpool_info()] or [1]))
    except Exception:  # pragma: no cover
        return os.cpu_count()


def bench_heat128(args):
    """d = 3, n = 128: E_mu = exp(tau A_mu) built in FP64 on the device, then
    S = V x_1 E_1 x_2 E_2 x_3 E_3 in every form."""
    import torch

    import oracle
    import paper_2112_11238_amd as kp
    V, As, tau = kp_workloads.heat128(seed=0)
    n = V.shape[0]
    h = 1.0 / (n + 1)
    A = torch.tensor(np.stack(As), dtype=torch.float64, device="cuda")
    expm_ms = _events_ms(lambda: kp.expm(A, tau), args.steps, args.warmup)
    E = kp.expm(A, tau)
    torch.cuda.synchronize()
    Eref = oracle.expm_fd_laplacian_dirichlet(n, h, tau)
    expm_err = max(_rel(E[k].cpu().numpy(), Eref) for k in range(3))
    Es = [E[k].contiguous() for k in range(3)]
    ref = oracle.tucker(V, [Eref] * 3)
    flops = kp_workloads.tucker_flops(V.shape, [n] * 3)
    forms = {}
    for dt, prec in _form_list(args, FORMS):
        tdt = torch.float64 if dt == "f64" else torch.float32
        Vd = torch.tensor(V, dtype=tdt, device="cuda")
        Ed = [x.to(tdt) for x in Es]
        if args.autotune:
            kp.tune.autotune(Vd, Ed, prec=prec, reps=10)
        S = kp.tucker(Vd, Ed, prec=prec)
        torch.cuda.synchronize()
        ms = _events_ms(lambda: kp.tucker(Vd, Ed, prec=prec), args.steps, args.warmup)
        modes = [_launch_ms(kp, tdt, prec, v, args.steps) for v in _views(kp, Vd, Ed, prec)]
        forms[form_name(dt, prec)] = {
            "tflops": round(flops / (ms * 1e-3) / 1e12, 3), "ms_per_step": round(ms, 5),
            "mode_ms": [round(x, 5) for x in modes],
            "rel_err_maxnorm": _rel(S.double().cpu().numpy(), ref)}
    head = forms.get("f64") or next(iter(forms.values()))
    return _line(args, "Tucker-op TFLOP/s heat128 (d=3, n=128, exp(tau A) factors)",
                 head["tflops"], "TFLOP/s", head["ms_per_step"], "f64",
                 {"workload": "heat128: V ~ N(0,1) 128^3 seed 0, A = tridiag(1,-2,1)/h^2, "
                              "h = 1/129, tau = 1e-3, E = exp(tau A) built in FP64 on the "
                              "device; value is the FP64 form", "flops_per_step": flops},
                 {"forms": forms, "expm": {"ms_three_factors": round(expm_ms, 4),
                                           "rel_err_vs_dst_closed_form": expm_err}})


def bench_interp6d(args):
    """d = 6, 16^6 -> 24^6 Lagrange interpolation in FP32 (and the BF16
    splits): forward, and forward + backward (dT and every dL)."""
    import torch

    import paper_2112_11238_amd as kp
    T, Ls = kp_workloads.interp6d(seed=0)
    m, n = list(T.shape), [L.shape[0] for L in Ls]
    fwd_flops = kp_workloads.tucker_flops(m, n)
    # backward: the cotangent sweep (mode d down to 1, L^T) and one gram per mode
    bwd_flops = kp_workloads.tucker_flops(n[::-1], m[::-1])
    for mu in range(6):
        bwd_flops += 2 * n[mu] * m[mu] * int(np.prod(n[:mu])) * int(np.prod(m[mu + 1:]))
    forms = {}
    roof = None
    for dt, prec in _form_list(args, FORMS[1:]):
        Td = torch.tensor(T, dtype=torch.float32, device="cuda")
        Lds = [torch.tensor(L, dtype=torch.float32, device="cuda") for L in Ls]
        G = torch.randn(n, dtype=torch.float32, device="cuda")
        if args.autotune:
            kp.tune.autotune(Td, Lds, prec=prec, backward=True, reps=5)
        fwd = _events_ms(lambda: kp.tucker(Td, Lds, prec=prec), args.steps, args.warmup)

        def step():
            S, cache = kp.tucker_with_cache(Td, Lds, prec=prec)
            kp.tucker_backward(G, Td, Lds, prec, cache=cache)
        both = _events_ms(step, args.steps, args.warmup)
        views = _views(kp, Td, Lds, prec)
        launch = [_launch_ms(kp, torch.float32, prec, v, args.steps) for v in views]
        min_bytes = (int(np.prod(m)) + int(np.prod(n))) * 4
        unfused = sum((Il * mm * Ir + Il * nn * Ir) * 4 for Il, mm, nn, Ir in views)
        forms[form_name(dt, prec)] = {
            "fwd_ms": round(fwd, 4), "fwd_tflops": round(fwd_flops / (fwd * 1e-3) / 1e12, 3),
            "fwd_min_bytes_gbs": round(min_bytes / (fwd * 1e-3) / 1e9, 1),
            "fwd_unfused_bytes_gbs": round(unfused / (fwd * 1e-3) / 1e9, 1),
            "fwd_bwd_ms": round(both, 4),
            "fwd_bwd_tflops": round((fwd_flops + bwd_flops) / (both * 1e-3) / 1e12, 3),
            "launch_ms": [round(x, 4) for x in launch]}
        if roof is None:
            k = int(np.argmax(launch))
            Il, mm, nn, Ir = views[k]
            byts = (Il * mm * Ir + Il * nn * Ir) * 4 + nn * mm * 4
            gbs = byts / (launch[k] * 1e-3) / 1e9
            roof = {"kernel": f"mode_kernel<{form_name(dt, prec)}> largest forward launch "
                              f"(Il={Il}, m={mm}, n={nn}, Ir={Ir})",
                    "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "avg_launch_ms": round(launch[k], 4), "bytes_per_launch": byts,
                    "traffic": None}
    head = forms.get("f32") or next(iter(forms.values()))
    return _line(args, "Tucker-op TFLOP/s interp6d (d=6, 16^6 -> 24^6, FP32), forward + backward",
                 head["fwd_bwd_tflops"], "TFLOP/s", head["fwd_bwd_ms"], "f32",
                 {"workload": "interp6d: T ~ N(0,1) 16^6 seed 0, six 24x16 Lagrange factors "
                              "(Chebyshev nodes to 24 equispaced points); value is FP32 "
                              "forward + backward (forward with cache, dT and all dL)",
                  "fwd_flops": fwd_flops, "bwd_flops": bwd_flops},
                 {"forms": forms, "roofline": roof})


def bench_batch64(args):
    """64 independent d = 4 problems (sizes in [16, 64]), forward + backward
    in one batched executor run, replayed from a HIP graph."""
    import torch

    import paper_2112_11238_amd as kp
    sizes, items = kp_workloads.batch64(seed=0)
    fwd = bwd = 0
    for k in range(len(items)):
        m = [int(x) for x in sizes[k]]
        fwd += kp_workloads.tucker_flops(m, m)
        bwd += kp_workloads.tucker_flops(m[::-1], m[::-1])
        for mu in range(4):
            bwd += 2 * m[mu] * m[mu] * int(np.prod(m)) // m[mu]
    forms = {}
    for prec in ("native", "bf16x3", "bf16x6"):
        name = form_name("f32", prec)
        if args.forms != "all" and name not in args.forms.split(","):
            continue
        Td = [torch.tensor(T, dtype=torch.float32, device="cuda") for T, _ in items]
        Ld = [[torch.tensor(L, dtype=torch.float32, device="cuda") for L in Ls] for _, Ls in items]
        Gd = [torch.randn(T.shape, dtype=torch.float32, device="cuda") for T in Td]
        rec = {}
        for tuned in ([False, True] if args.autotune else [False]):
            if tuned:
                kp.tune.autotune_batch(Td, Ld, prec=prec, backward=True, reps=3)
            bt_f = kp.BatchedTucker(Td, Ld, prec=prec)
            bt_b = kp.BatchedTucker(Td, Ld, prec=prec, Gs=Gd)
            f_ms, _ = _graph_ms(bt_f.run, args.steps, args.warmup)
            b_ms, _ = _graph_ms(bt_b.run, args.steps, args.warmup)
            rec["tuned" if tuned else "default"] = {
                "fwd_ms": round(f_ms, 4), "fwd_tflops": round(fwd / (f_ms * 1e-3) / 1e12, 3),
                "fwd_bwd_ms": round(b_ms, 4),
                "fwd_bwd_tflops": round((fwd + bwd) / (b_ms * 1e-3) / 1e12, 3),
                "levels": bt_b.nlevels, "tasks": int(bt_b.ntasks)}
            kp.tune.clear()
        forms[name] = rec
    head = forms.get("f32") or next(iter(forms.values()))
    best = max(head.values(), key=lambda r: r["fwd_bwd_tflops"])
    return _line(args, "Batched Tucker-op TFLOP/s batch64 (64 x d=4, sizes 16..64, FP32), "
                       "forward + backward, graph replay",
                 best["fwd_bwd_tflops"], "TFLOP/s", best["fwd_bwd_ms"], "f32",
                 {"workload": "batch64: 64 tensors of order 4, sizes from seed 0 in [16, 64], "
                              "L ~ N(0,1)/sqrt(n); forward + backward (dT and all dL) in one "
                              "batched executor run replayed from a HIP graph",
                  "fwd_flops": fwd, "bwd_flops": bwd},
                 {"forms": forms})


def bench_runge5d(args):
    """The 5-D Runge interpolation at the paper's largest size: F on 45^5
    Chebyshev nodes (1.48 GB in FP64) to 35^5 equispaced points, in FP64 and
    the FP32 forms; error against the exact function values."""
    import torch

    import oracle
    import paper_2112_11238_amd as kp
    m, n, d = 45, 35, 5
    F, Ls, x = kp_workloads.runge5d(m, n, d)
    flops = kp_workloads.tucker_flops([m] * d, [n] * d)
    f = oracle.runge(*([x] * d))
    fmax = float(np.abs(f).max())
    forms = {}
    roof = None
    for dt, prec in _form_list(args, FORMS):
        tdt = torch.float64 if dt == "f64" else torch.float32
        Fd = torch.tensor(F, dtype=tdt, device="cuda")
        Ld = [torch.tensor(L, dtype=tdt, device="cuda") for L in Ls]
        S = kp.tucker(Fd, Ld, prec=prec)
        torch.cuda.synchronize()
        err = float(np.abs(S.double().cpu().numpy() - f).max() / fmax)
        del S
        ms = _events_ms(lambda: kp.tucker(Fd, Ld, prec=prec), args.steps, args.warmup)
        views = _views(kp, Fd, Ld, prec)
        es = 8 if dt == "f64" else 4
        modes = []
        for Il, mm, nn, Ir in views:
            lms = _launch_ms(kp, tdt, prec, (Il, mm, nn, Ir), args.steps)
            byts = (Il * mm * Ir + Il * nn * Ir) * es
            modes.append({"view": [Il, mm, nn, Ir], "ms": round(lms, 5),
                          "gbs": round(byts / (lms * 1e-3) / 1e9, 1)})
        forms[form_name(dt, prec)] = {
            "ms_per_step": round(ms, 5), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
            "rel_err_vs_runge_maxnorm": err, "modes": modes}
        if dt == "f64" and prec == "native":
            # the first (largest) product: 1.48 GB in, 1.15 GB out, 4.9 flop/B
            g = modes[0]["gbs"]
            roof = {"bound": "hbm", "achieved": g, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(g / HBM_PEAK_GBS, 4), "traffic": None}
        del Fd
        torch.cuda.empty_cache()
    head = forms.get("f64") or next(iter(forms.values()))
    extra = {"forms": forms, "paper_printed_rel_err_m45": 1.39e-5}
    if roof:
        extra["roofline"] = roof
    if not args.no_cpu_baseline:
        Fs, Lss, _ = kp_workloads.runge5d(35, n, d)
        t0 = time.perf_counter()
        oracle.tucker(Fs, Lss)
        sec = time.perf_counter() - t0
        sflops = kp_workloads.tucker_flops([35] * d, [n] * d)
        extra["cpu_baseline"] = {"value": round(sflops / sec / 1e12, 6), "unit": "TFLOP/s",
                                 "cores": _threads(), "kind": "oracle",
                                 "sample": f"one oracle Tucker call at m=35 ({sec:.1f} s)"}
    return _line(args, "Tucker-op TFLOP/s runge5d (d=5, 45^5 Chebyshev -> 35^5 uniform, FP64)",
                 head["tflops"], "TFLOP/s", head["ms_per_step"], "f64",
                 {"workload": "runge5d: Runge function 1/(1+16|x|^2) on 45^5 Chebyshev nodes, "
                              "barycentric Lagrange factors to 35 equispaced points of [-1,1] "
                              "per direction; value is the FP64 form", "flops_per_step": flops},
                 extra)


def bench_codeval(args):
    """The paper's Tucker timing sweep shapes: d = 3 with n in {144, 196,
    256, 324} and d = 6 with n in {12, 14, 16, 18}, square standard-normal
    factors, in every form."""
    import torch

    import oracle
    import paper_2112_11238_amd as kp
    shapes = {}
    for d, n in kp_workloads.codeval_shapes():
        T, Ls = kp_workloads.cube(seed=n, n=n, d=d)
        flops = kp_workloads.tucker_flops([n] * d, [n] * d)
        rec = {}
        for dt, prec in _form_list(args, FORMS):
            tdt = torch.float64 if dt == "f64" else torch.float32
            Td = torch.tensor(T, dtype=tdt, device="cuda")
            Ld = [torch.tensor(L, dtype=tdt, device="cuda") for L in Ls]
            ms = _events_ms(lambda: kp.tucker(Td, Ld, prec=prec), args.steps, args.warmup)
            tf = flops / (ms * 1e-3) / 1e12
            peak = PEAK["f64"] if dt == "f64" else (PEAK["f32"] if prec == "native"
                                                    else PEAK["bf16"])
            rec[form_name(dt, prec)] = {"ms": round(ms, 5), "tflops": round(tf, 3),
                                        "frac_of_form_peak": round(tf / peak, 4)}
        shapes[f"d{d}_n{n}"] = {"flops": flops, "forms": rec}
    head = shapes["d3_n324"]["forms"].get("f64") or next(iter(shapes["d3_n324"]["forms"].values()))
    extra = {"shapes": shapes, "paper_context": {"d3_gflops_cpu": [106, 127],
                                                 "d6_gflops_cpu": [11, 14],
                                                 "hardware": "the paper's CPU"}}
    if not args.no_cpu_baseline:
        T, Ls = kp_workloads.cube(seed=196, n=196, d=3)
        t0 = time.perf_counter()
        oracle.tucker(T, Ls)
        sec = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": round(kp_workloads.tucker_flops([196] * 3, [196] * 3)
                                                / sec / 1e12, 6), "unit": "TFLOP/s",
                                 "cores": _threads(), "kind": "oracle",
                                 "sample": f"one oracle Tucker call at d=3 n=196 ({sec:.2f} s)"}
    return _line(args, "Tucker-op TFLOP/s codeval sweep (d=3 n=144..324, d=6 n=12..18), "
                       "value at d=3 n=324 FP64",
                 head["tflops"], "TFLOP/s", head["ms"], "f64",
                 {"workload": "codeval: standard-normal cubes and square factors, seed = n, "
                              "d=3 n in {144,196,256,324}, d=6 n in {12,14,16,18}"}, extra)


def bench_fft3d(args):
    """A 3-D discrete Fourier transform of a complex 200^3 tensor as a
    complex Tucker operator with Fourier matrices, and its inverse through
    the conjugate-transpose form, in complex128 and complex64 (and the BF16
    splits on complex64). Real flops: 8 n m per complex output of each mode."""
    import torch

    import paper_2112_11238_amd as kp
    n = 200
    rng = np.random.default_rng(0)
    T = rng.standard_normal((n,) * 3) + 1j * rng.standard_normal((n,) * 3)
    F = kp_workloads.fourier_matrix(n)
    ref = np.fft.fftn(T)
    rmax = float(np.abs(ref).max())
    flops = 3 * 8 * n ** 4
    forms = {}
    for name, cdt, prec in [("c128", torch.complex128, "native"), ("c64", torch.complex64, "native"),
                            ("c64_bf16x3", torch.complex64, "bf16x3"),
                            ("c64_bf16x6", torch.complex64, "bf16x6")]:
        if args.forms != "all" and name.split("_")[-1] not in args.forms.split(",") and \
                name not in args.forms.split(","):
            continue
        Td = torch.tensor(T, dtype=cdt, device="cuda")
        Fd = [torch.tensor(F, dtype=cdt, device="cuda")] * 3
        S = kp.tucker_complex(Td, Fd, prec=prec)
        back = kp.tucker_complex(S, Fd, conj=True, prec=prec)
        torch.cuda.synchronize()
        err = float(np.abs(S.to(torch.complex128).cpu().numpy() - ref).max() / rmax)
        inv = float(np.abs(back.to(torch.complex128).cpu().numpy() / T.size - T).max()
                    / np.abs(T).max())
        ms = _events_ms(lambda: kp.tucker_complex(Td, Fd, prec=prec), args.steps, args.warmup)
        ims = _events_ms(lambda: kp.tucker_complex(S, Fd, conj=True, prec=prec), args.steps,
                         args.warmup)
        forms[name] = {"ms_forward": round(ms, 4), "tflops": round(flops / (ms * 1e-3) / 1e12, 3),
                       "ms_inverse": round(ims, 4), "rel_err_vs_numpy_fft": err,
                       "inverse_rel_err": inv}
        del Td, S, back
        torch.cuda.empty_cache()
    head = forms.get("c128") or next(iter(forms.values()))
    extra = {"forms": forms}
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        reps = 0
        while reps < 3 or time.perf_counter() - t0 < 5.0:
            oracle.ztucker(T, [F] * 3)
            reps += 1
        sec = (time.perf_counter() - t0) / reps
        extra["cpu_baseline"] = {"value": round(flops / sec / 1e12, 6),
                                 "unit": "TFLOP/s", "cores": _threads(), "kind": "oracle",
                                 "sample": f"{reps} oracle complex Tucker calls on the same "
                                           f"input ({sec:.3f} s each)"}
    return _line(args, "complex Tucker-op TFLOP/s fft3d (d=3, n=200, Fourier factors, complex128)",
                 head["tflops"], "TFLOP/s", head["ms_forward"], "c128",
                 {"workload": "fft3d: complex 200^3 tensor, real and imaginary parts N(0,1) "
                              "seed 0, Fourier matrices per mode; forward transform timed, the "
                              "inverse through the conjugate-transpose form",
                  "flops_per_step": flops}, extra)


def bench_semilinear(args):
    """The semilinear experiment (n = (40, 44, 48), tau = 0.01, 100 steps to
    t = 1): ADI factor inverses built on the device, one PCG solve per step
    on the Kronecker-sum matrix; also plain CG. Each timed run starts from u0."""
    import torch

    import oracle
    import paper_2112_11238_amd as kp
    u0, diags, tau, nsteps = kp_workloads.semilinear()
    ns = u0.shape
    N = int(np.prod(ns))
    dev = [[torch.tensor(dd[j], dtype=torch.float64, device="cuda") for dd in diags]
           for j in range(3)]
    hs = [dd[3] for dd in diags]
    xs = [oracle.semilinear_grid(n)[0] for n in ns]
    exact = np.exp(1.0) * oracle.semilinear_u0(xs)
    runs = max(1, min(args.steps, 5))
    tuned = None
    if args.autotune:
        # the preconditioner and Kronecker-sum products share their views
        Ud = torch.tensor(u0, dtype=torch.float64, device="cuda")
        sq = [torch.randn((n, n), dtype=torch.float64, device="cuda") for n in ns]
        tuned = kp.tune.autotune(Ud, sq, reps=20)
    out = {}
    finals = {}
    for pre in (True, False):
        U = torch.tensor(u0, dtype=torch.float64, device="cuda")
        kp.semilinear_imex(U, *dev, hs, tau, nsteps, precondition=pre)   # warm-up
        torch.cuda.synchronize()
        times = []
        for _ in range(runs):
            U.copy_(torch.tensor(u0, dtype=torch.float64, device="cuda"))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = kp.semilinear_imex(U, *dev, hs, tau, nsteps, precondition=pre)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
        ms = statistics.median(times)
        u = U.cpu().numpy()
        finals[pre] = u
        total_its = int(sum(its))
        out["pcg" if pre else "cg"] = {
            "ms_per_run": round(ms, 3), "avg_iterations": round(total_its / nsteps, 3),
            "us_per_iteration": round(ms * 1e3 / max(total_its + nsteps, 1), 2),
            "rel_err_vs_exact_maxnorm": float(np.abs(u - exact).max() / np.abs(exact).max())}
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        ref, rits = oracle.semilinear_imex(ns, tau=tau, steps=nsteps)
        cpu_ms = (time.perf_counter() - t0) * 1e3
        out["pcg"]["rel_diff_vs_oracle"] = _rel(finals[True], ref)
        cpu = {"value": round(cpu_ms, 1), "unit": "ms", "cores": _threads(), "kind": "oracle",
               "sample": "one whole oracle run (100 PCG steps)"}
    head = out["pcg"]
    # per PCG iteration the vectors of length N cross memory about 30 times
    # (3 preconditioner products and 3 Kronecker-sum products, each reading
    # and writing N; the accumulating products read N more; dot products and
    # updates): 30 N doubles; the run is launch- and sync-latency bound
    it_bytes = 30 * N * 8
    achieved = it_bytes / (head["us_per_iteration"] * 1e-6) / 1e9
    extra = {"solvers": out, "paper_context": {"pcg_tensor_s": 0.5, "cg_tensor_s": 2.2,
                                               "avg_iterations_pcg": 2, "avg_iterations_cg": 30,
                                               "rel_err": 9.7e-3, "hardware": "the paper's CPU"},
             "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                          "traffic": None}}
    if cpu:
        extra["cpu_baseline"] = cpu
    if tuned is not None:
        extra["tuned_tiles"] = tuned
    return _line(args, "semilinear experiment wall time (n=(40,44,48), tau=0.01, 100 "
                       "backward-forward Euler steps, ADI-preconditioned CG)",
                 head["ms_per_run"], "ms", head["ms_per_run"], "f64",
                 {"workload": "semilinear: u_t = Laplacian u + 1/(1+u^2) + Phi on [0,1]^3, "
                              "Dirichlet, n = (40, 44, 48) interior points, tau = 0.01, t* = 1, "
                              "u0 = prod x(1-x), PCG tol 1e-5; value is ms per whole run",
                  "elements": N}, extra, higher=False)


WORKLOAD_BENCHES = {"small2d": bench_small2d, "heat128": bench_heat128,
                    "interp6d": bench_interp6d, "batch64": bench_batch64,
                    "semilinear": bench_semilinear, "runge5d": bench_runge5d,
                    "codeval": bench_codeval, "fft3d": bench_fft3d}


if __name__ == "__main__":
    main()
