import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# The library keeps autotuned schedules in a cache file; the tests use one of
# their own (a fresh temporary file per session) so that a user's cache never
# changes which schedule a test's plan starts on.
if "QFT_SCHEDULE_CACHE" not in os.environ:
    import tempfile
    os.environ["QFT_SCHEDULE_CACHE"] = os.path.join(
        tempfile.mkdtemp(prefix="qft_sched_"), "schedules.json")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests are collected everywhere; without a GPU they are skipped
    # unless explicitly selected with -m gpu (then they must run, and fail
    # loudly if the device or the library is missing).
    markexpr = config.getoption("-m") or ""
    if "gpu" in markexpr and "not gpu" not in markexpr:
        return
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
