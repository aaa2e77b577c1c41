import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_collection_modifyitems(config, items):
    # GPU tests cannot run without a device; mark them skipped here rather than fail.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture
def measured(request):
    """Record a measured value (an error, an iteration count) of a test: when
    WCMG_MEASURED names a file, one JSON line per value is appended to it."""
    import json

    path = os.environ.get("WCMG_MEASURED")

    def record(name, value):
        if path:
            with open(path, "a") as f:
                f.write(json.dumps({"test": request.node.nodeid, "name": name, "value": value}) + "\n")

    return record
