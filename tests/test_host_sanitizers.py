"""The host side of the library (argument validation, the mode-order
planner, workspace and cache layouts, the batch plan, the tile table) under
AddressSanitizer and UndefinedBehaviorSanitizer: the host-only test suites
run in a child process against a build whose host code is instrumented
(paper_2112_11238_amd.build.build_hostsan), with the clang ASan runtime
preloaded. Any sanitizer report fails the child (halt_on_error)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_SUITES = ["tests/test_abi_host.py", "tests/test_batch_plan_host.py",
               "tests/test_tune_host.py"]


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


@pytest.mark.skipif(_gpu_visible(), reason="the host suites use fake device addresses")
@pytest.mark.timeout(900)
def test_host_code_under_asan_and_ubsan():
    from paper_2112_11238_amd import build
    if not shutil.which("hipcc") and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc missing")
    rt = build.asan_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime missing")
    lib = build.build_hostsan()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "KP_LIBRARY": lib,
    })
    probe = subprocess.run(
        [sys.executable, "-c",
         "from paper_2112_11238_amd import _lib; import ctypes; l = _lib.load(); "
         "print(l._name); print(hasattr(l, '__asan_init'))"],
        cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-2000:]
    name, has_asan = probe.stdout.split()[-2:]
    assert name == lib and has_asan == "True", probe.stdout
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"]
                       + HOST_SUITES, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in r.stdout
