import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line(
        "markers", "slow: CPU test that takes more than a few seconds")


def pytest_collection_modifyitems(config, items):
    # GPU tests need a visible device; skip them cleanly elsewhere.
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def pytest_runtest_setup(item):
    # Multi-GB CPU cases (e.g. the m=35, 45 interpolation errors) run only on
    # request, to keep the default CPU suite within a few minutes.
    if "slow" in item.keywords and os.environ.get("KP_RUN_SLOW") != "1":
        pytest.skip("slow CPU case; set KP_RUN_SLOW=1 to run it")
