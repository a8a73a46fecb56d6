import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

# Under pytest-xdist every worker would start one OpenMP thread (the oracle) and one
# intra-op thread (torch) per core; share the cores out instead, before either
# runtime starts in this worker.
_workers = os.environ.get("PYTEST_XDIST_WORKER_COUNT")
if _workers:
    _per = str(max(1, (os.cpu_count() or 1) // max(1, int(_workers))))
    os.environ["OMP_NUM_THREADS"] = _per
    os.environ["MKL_NUM_THREADS"] = _per


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_collection_modifyitems(config, items):
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
