import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def pytest_collection_modifyitems(config, items):
    # GPU tests cannot run without a device; skip them (with the reason) rather
    # than erroring when someone runs the whole suite on a CPU-only host.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


def pytest_sessionstart(session):
    # name the HIP / HSA runtime files this process maps (GPU runs only), so a
    # failure report shows which runtime the library and torch resolved to
    try:
        import torch
        if not torch.cuda.is_available():
            return
        import paper_0710_2442_amd  # noqa: F401  (loads libwd.so)
        with open("/proc/self/maps") as f:
            libs = sorted({l.split()[-1] for l in f if ("amdhip" in l or "hsa-runtime" in l or "libwd" in l)})
        print("\n[runtime libraries]", *libs, sep="\n  ", flush=True)
    except Exception as e:  # pragma: no cover
        print("[runtime libraries] unavailable:", e, flush=True)
