import gc
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(autouse=True)
def _release_device_memory(request):
    """After a GPU test, drop what still references its solvers (pytest keeps
    the last failure's traceback, and with it the test's locals) and give the
    cached device memory back, so one test's tens of gigabytes of recorded
    paths do not starve the next."""
    yield
    if request.node.get_closest_marker("gpu") is None:
        return
    sys.last_type = sys.last_value = sys.last_traceback = None
    gc.collect()
    import torch
    if torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
