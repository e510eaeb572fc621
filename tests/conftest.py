import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

# Under pytest-xdist every worker runs the OpenMP oracle.  A full thread team per worker
# oversubscribes the cores, and the teams' spinning barriers then slow the long oracle runs
# by an order of magnitude.  Each worker gets its share of the cores instead; this must be
# set before the oracle library (and its OpenMP runtime) is loaded.
_WORKERS = int(os.environ.get("PYTEST_XDIST_WORKER_COUNT", "0") or 0)
if _WORKERS > 1:
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // _WORKERS))
    os.environ.setdefault("OMP_WAIT_POLICY", "passive")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: longer CPU test")


_GPU = None


def gpu_available() -> bool:
    global _GPU
    if _GPU is None:
        try:
            import torch
            _GPU = torch.cuda.device_count() > 0
        except Exception:
            _GPU = False
    return _GPU


def pytest_collection_modifyitems(config, items):
    import pytest
    if gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


def pytest_runtest_setup(item):
    # name the case before any GPU work starts, so a failing run still says which one
    if "gpu" in item.keywords:
        print(f"\n[gpu-test] {item.nodeid}", flush=True)
